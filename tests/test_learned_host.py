"""Host logic of the learned form on a batch: the search rounds of
BatchedLearnedAADescent (Armijo trials on the theta window, the pbar_theta
check, the plain window's trials, the plain pbar, restarts) take, instance by
instance, the decisions of LearnedAADescent.  The device calls are replaced
by CPU stand-ins shared by both drivers (a separable misfit with a known
gradient, a mixing rule with a chosen overshoot per iteration, a network
that rescales the gradient), so the drivers' own sequencing is what is
compared; the GPU tests compare the real kernels the same way."""
import numpy as np
import pytest
import torch

from paper_2008_11778_amd import batched as batched_mod
from paper_2008_11778_amd import inversion as inversion_mod
from paper_2008_11778_amd import learned as learned_mod


class Misfit:
    """J(m) = sum(w (m - t)^2 / 2 + c (m - t)^4 / 4) in FP64 over an image."""

    def __init__(self, shape, seed):
        r = np.random.default_rng(seed)
        self.shape = shape
        self.w = r.uniform(0.5, 2.0, shape)
        self.c = r.uniform(0.0, 0.3, shape)
        self.t = r.uniform(1.0, 2.0, shape)

    def J(self, m):
        e = m.double().numpy().reshape(self.shape) - self.t
        return float(np.sum(0.5 * self.w * e * e + 0.25 * self.c * e ** 4))

    def grad(self, m):
        e = m.double().numpy().reshape(self.shape) - self.t
        return torch.from_numpy((self.w * e + self.c * e ** 3).astype(np.float32))


class MixState:
    """One Anderson window stand-in: pbar = p - eta g; ptilde = pbar +
    f_k (pbar - p) with f_k from a per-window schedule over the steps since
    the last reset; mk counts them."""

    def __init__(self, schedule):
        self.schedule = schedule
        self.k = 0
        self.mk = torch.zeros(1, dtype=torch.int32)

    def step(self, p, g, eta, pbar, ptilde):
        eta = float(np.float32(eta))
        pbar.copy_(p - eta * g)
        f = self.schedule[self.k % len(self.schedule)]
        ptilde.copy_(pbar + f * (pbar - p))
        self.k += 1
        self.mk.fill_(min(self.k, 10))

    resets = 0

    def reset(self):
        self.k = 0
        self.mk.zero_()
        MixState.resets += 1


SCHEDULES = {}  # (instance, window) -> schedule, set per test case


class FakeAA:
    """Stand-in for the single-instance Anderson state (LearnedAADescent
    creates the theta window, then the plain one; AADescent one plain)."""
    made = []
    order = ("theta", "plain")

    def __init__(self, n, M, cond_max=1e5, stream=None, solver="gram"):
        inst, which = FakeAA.made[0], FakeAA.order[len(FakeAA.made) - 1]
        FakeAA.made.append(which)
        self.s = MixState(SCHEDULES[(inst, which)])
        self.mk = self.s.mk

    def step(self, p, g, eta, pbar, ptilde):
        self.s.step(p, g, eta, pbar, ptilde)

    def reset(self):
        self.s.reset()

    def close(self):
        pass


class FakeBatchAA:
    """Stand-in for the batched Anderson state: the plain window is created
    first (by the base class), then the theta window."""
    made = 0

    def __init__(self, ns, M, cond_max=1e5, stream=None):
        which = ("plain", "theta")[FakeBatchAA.made]
        FakeBatchAA.made += 1
        self.st = [MixState(SCHEDULES[(i, which)]) for i in range(len(ns))]

    def step(self, ps, gs, etas, pbars, ptildes, active=None):
        for i, s in enumerate(self.st):
            if active is None or active[i]:
                s.step(ps[i], gs[i], etas[i], pbars[i], ptildes[i])

    def reset(self, which=None):
        for i, s in enumerate(self.st):
            if which is None or which[i]:
                s.reset()

    def close(self):
        pass


class FakeReducer:
    def __init__(self, stream=None, device=None):
        pass

    def dot_diff(self, g, a, b, out=None):
        v = torch.tensor([float(np.dot(g.double().numpy().ravel(), (a.double() - b.double()).numpy().ravel()))],
                         dtype=torch.float64)
        if out is not None:
            out.copy_(v)
            return out
        return v


class FakeCNN:
    """d = (1 + 0.5 tanh(m - 1.5)) g: a positive rescaling of the gradient."""

    def __init__(self, nz, nx, max_batch, weights, stream=None):
        self.nz, self.nx = nz, nx

    def forward(self, g, m, z=None, d=None):
        d.copy_((1.0 + 0.5 * torch.tanh(m - 1.5)) * g)
        return None, d

    def close(self):
        pass


def fake_blend(lam, p_tilde, p_bar, out=None, stream=None):
    out.copy_(lam * p_tilde + (1.0 - lam) * p_bar)
    return out


def fake_floor(x, floor, stream=None):
    return x.clamp_(min=floor)


class Problem:
    """The single driver's problem: gradient and kept misfit runs."""

    def __init__(self, f, floor):
        self.f, self.floor = f, floor
        self.n_adj = self.n_fwd = 0

    def gradient(self, p, g):
        self.n_adj += 1
        g.copy_(self.f.grad(p).view(-1))
        return self.f.J(p)

    def misfit_keep(self, p):
        self.n_fwd += 1
        return self.f.J(p)


class Batch:
    """The batch: per instance the model buffer, the gradient of its kept
    forward run and that run's misfit."""

    def __init__(self, fs, floors):
        self.fs, self.N, self.floors = fs, len(fs), floors
        self.device, self.stream = torch.device("cpu"), None
        self.m = [torch.zeros(f.shape, dtype=torch.float32) for f in fs]
        self.grad = [torch.zeros(f.shape, dtype=torch.float32) for f in fs]
        self.kept = [None] * self.N
        self.J = [float("nan")] * self.N
        self.active = np.ones(self.N, bool)

    def set_active(self, mask):
        self.active = np.asarray(mask).astype(bool)

    def forward(self, keep_ckpt=True):
        for i in range(self.N):
            if self.active[i]:
                self.kept[i] = self.m[i].clone()
                self.J[i] = self.fs[i].J(self.kept[i])

    def backward(self):
        for i in range(self.N):
            if self.active[i]:
                self.grad[i].copy_(self.fs[i].grad(self.kept[i]))

    def misfits(self):
        return list(self.J)


@pytest.fixture
def fakes(monkeypatch):
    for mod in (learned_mod, batched_mod):
        monkeypatch.setattr(mod, "Reducer", FakeReducer)
        monkeypatch.setattr(mod, "blend", fake_blend)
        monkeypatch.setattr(mod, "floor_", fake_floor)
    monkeypatch.setattr(learned_mod, "AA", FakeAA)
    monkeypatch.setattr(inversion_mod, "AA", FakeAA)
    monkeypatch.setattr(inversion_mod, "Reducer", FakeReducer)
    monkeypatch.setattr(inversion_mod, "blend", fake_blend)
    monkeypatch.setattr(inversion_mod, "floor_", fake_floor)
    monkeypatch.setattr(learned_mod, "BatchAA", FakeBatchAA)
    monkeypatch.setattr(batched_mod, "BatchAA", FakeBatchAA)
    monkeypatch.setattr(learned_mod, "CNN", FakeCNN)


# eta and eta_theta as multiples of 1 / max(w): the theta step overshoots
# (pbar_theta raises J) from about 2 on; the schedules pick the overshoot of
# ptilde over pbar per step
CASES = [
    dict(eta=0.4, eta_theta=0.8, theta=(0.0, 0.5, 3.0), plain=(0.0, 1.0)),
    dict(eta=0.6, eta_theta=2.6, theta=(0.5, 40.0), plain=(0.2, 100.0, 0.0)),
    dict(eta=1.9, eta_theta=3.5, theta=(60.0,), plain=(100.0, 0.5, 200.0)),
    dict(eta=0.9, eta_theta=1.4, theta=(9.0, 0.0, 2.0, 30.0), plain=(0.0,)),
    dict(eta=0.3, eta_theta=5.0, theta=(0.0,), plain=(80.0,)),
]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_batched_search_rounds_take_the_single_decisions(fakes, seed):
    shapes = [(6, 9), (4, 4), (7, 5), (5, 8), (3, 11)]
    fs = [Misfit(sh, 100 * seed + i) for i, sh in enumerate(shapes)]
    floors = [0.9, 0.5, 1.2, 0.0, 1.05]
    p0 = [torch.from_numpy(f.t + np.random.default_rng(7 + i + seed).uniform(-1.5, 1.5, f.shape)).float()
          for i, f in enumerate(fs)]
    etas = [c["eta"] / f.w.max() for c, f in zip(CASES, fs)]
    eta_thetas = [c["eta_theta"] / f.w.max() for c, f in zip(CASES, fs)]
    for i, c in enumerate(CASES):
        SCHEDULES[(i, "theta")], SCHEDULES[(i, "plain")] = c["theta"], c["plain"]
    iters = 8

    singles = []
    MixState.resets = 0
    FakeAA.order = ("theta", "plain")
    for i, f in enumerate(fs):
        FakeAA.made = [i]
        prob = Problem(f, floors[i])
        run = learned_mod.LearnedAADescent(prob, p0[i].clone(), FakeCNN(*f.shape, 1, None), M=10,
                                           eta=etas[i], eta_theta=eta_thetas[i])
        run.first()
        its, lams, fbs = [run.p.clone()], [], []
        for _ in range(iters):
            log = run.iterate()
            its.append(run.p.clone())
            lams.append(log.lam)
            fbs.append(log.fallback)
        singles.append(dict(its=its, lams=lams, fbs=fbs, n_fallback=run.n_fallback, J_end=f.J(run.p)))

    FakeBatchAA.made = 0
    b = Batch(fs, floors)
    br = learned_mod.BatchedLearnedAADescent(b, [x.clone() for x in p0], None, M=10, etas=etas,
                                             eta_thetas=eta_thetas)
    br.first()
    its, lams, fbs = [[x.clone() for x in br.p]], [], []
    for _ in range(iters):
        _, lam, fb = br.iterate()
        its.append([x.clone() for x in br.p])
        lams.append(lam)
        fbs.append(fb)
    J_end = br.current_misfits()

    outcomes = set()
    for i, s in enumerate(singles):
        for k in range(iters + 1):
            assert torch.equal(its[k][i], s["its"][k]), (seed, i, k)
        assert [lams[k][i] for k in range(iters)] == s["lams"], (seed, i)
        assert [fbs[k][i] for k in range(iters)] == s["fbs"], (seed, i)
        assert br.n_fallback[i] == s["n_fallback"]
        assert J_end[i] == s["J_end"]
        assert all(float(x.min()) >= np.float32(floors[i]) for x in s["its"][1:])  # p_1, ... in the domain
        for lam, fb in zip(s["lams"], s["fbs"]):
            outcomes.add(("plain" if fb else "theta", lam > 0))
    assert MixState.resets > 0  # windows restarted after fallbacks that decreased J
    # every way out of the search is taken somewhere: a theta trial, pbar_theta,
    # a plain trial, the plain pbar
    assert outcomes == {("theta", True), ("theta", False), ("plain", True), ("plain", False)}, outcomes


@pytest.mark.parametrize("seed", [0, 1])
def test_batched_plain_search_rounds_take_the_single_decisions(fakes, seed):
    """The same for plain Algorithm 2: BatchedAADescent against AADescent
    (trials, the fallback to pbar, the restart after a fallback that
    decreased J)."""
    shapes = [(6, 9), (4, 4), (7, 5), (5, 8), (3, 11)]
    fs = [Misfit(sh, 50 + 100 * seed + i) for i, sh in enumerate(shapes)]
    floors = [0.9, 0.5, 1.2, 0.0, 1.05]
    p0 = [torch.from_numpy(f.t + np.random.default_rng(3 + i + seed).uniform(-1.5, 1.5, f.shape)).float()
          for i, f in enumerate(fs)]
    etas = [c["eta"] / f.w.max() for c, f in zip(CASES, fs)]
    for i, c in enumerate(CASES):
        SCHEDULES[(i, "plain")] = c["theta"]  # the overshooting schedules
    iters = 8
    singles = []
    MixState.resets = 0
    FakeAA.order = ("plain",)
    for i, f in enumerate(fs):
        FakeAA.made = [i]
        prob = Problem(f, floors[i])
        run = inversion_mod.AADescent(prob, p0[i].clone().reshape(-1), etas[i], M=10)
        run.first()
        its, lams = [run.p.clone()], []
        for _ in range(iters):
            lams.append(run.iterate().lam)
            its.append(run.p.clone())
        singles.append(dict(its=its, lams=lams, J_end=f.J(run.p)))
    FakeBatchAA.made = 0
    br = batched_mod.BatchedAADescent(Batch(fs, floors), [x.clone() for x in p0], M=10, etas=etas)
    br.first()
    its, lams = [[x.clone() for x in br.p]], []
    for _ in range(iters):
        lams.append(br.iterate()[1])
        its.append([x.clone() for x in br.p])
    J_end = br.current_misfits()
    taken = set()
    for i, s in enumerate(singles):
        for k in range(iters + 1):
            assert torch.equal(its[k][i].view(-1), s["its"][k].view(-1)), (seed, i, k)
        assert [lams[k][i] for k in range(iters)] == s["lams"], (seed, i)
        assert J_end[i] == s["J_end"]
        taken.update(s["lams"])
    assert 0.0 in taken and 1.0 in taken and len(taken) >= 3, taken
    assert MixState.resets > 0
