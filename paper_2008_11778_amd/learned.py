"""Anderson acceleration of a learned descent map, its training data and its
training loop.

The map keeps the structure of the Method section: G_theta(p) = p - eta_theta
d_theta(p), with d_theta = softplus(z) * g and z the network's output on
[g / rms(g), (m - mean m) / std m] (so G_theta has the fixed points of G in
eq. GD).  Algorithm 2 runs unchanged on G_theta (its history holds d_theta
instead of g).  Fallback: when the line search accepts no lambda in
{1, 1/2, 1/4, 1/8} and J(pbar_theta) >= J(p_k) as well, the iteration is redone
with plain Anderson acceleration on G, whose history is fed with (p_k, g_k) at
every iteration so that it is ready when needed.  A window whose search fell
back to its plain descent step restarts (is cleared) at the next iteration
when that step decreased J, as in plain Algorithm 2.

Training pairs (g_k, p_k, s_k = p_{k+1} - p_k) come from plain Anderson runs
(all instances of a batch advanced together by BatchedAADescent) and from
L-BFGS runs; the network learns the direction of the step those optimisers
took, up to scale.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np
import torch

from ._lib import AA, CNN, Batch, BatchAA, Context, Reducer, axpy, blend, floor_
from .batched import BatchedAADescent
from .inversion import ARMIJO_C1, LAMBDAS, FWIProblem, IterLog, step_size


SHIPPED_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_mi355x.npy")


def shipped_weights():
    """(weights, provenance) of the network trained at the stated recipe that
    ships with the package (a training run of the learned workload)."""
    w = np.load(SHIPPED_WEIGHTS).astype(np.float32)
    with open(os.path.splitext(SHIPPED_WEIGHTS)[0] + ".json") as f:
        return w, json.load(f)


@dataclasses.dataclass
class LearnedLog(IterLog):
    fallback: bool = False
    # |eta_theta d_theta - eta g| / |eta g| at p_k: how far the learned map's
    # step departs from the plain descent step (None unless tracked)
    step_rel_err: float | None = None


class LearnedAADescent:
    """Algorithm 2 on G_theta with the plain-AA fallback (one problem)."""

    def __init__(self, problem, p0: torch.Tensor, net: CNN, M: int = 10, eta: float | None = None,
                 eta_theta: float | None = None, cond_max: float = 1e5, lambdas=LAMBDAS, c1: float = ARMIJO_C1,
                 eta_frac: float = 0.02, restart: bool = True, track_step_error: bool = False,
                 floor="problem"):
        self.problem, self.net, self.M = problem, net, M
        # pbar and ptilde of both windows are kept at or above the floor (the
        # model's stable domain); by default the problem's own
        self.floor = getattr(problem, "floor", None) if floor == "problem" else floor
        self.restart = restart
        self.track_step_error = track_step_error
        # which window's search fell back to its plain step in the last
        # iteration; the window restarts if that step decreased J
        self.fb_theta = self.fb_plain = False
        self.J_prev = None
        self.eta, self.eta_theta, self.eta_frac = eta, eta_theta, eta_frac
        self.lambdas, self.c1 = lambdas, c1
        self.shape = tuple(p0.shape)
        if len(self.shape) != 2 or (net.nz, net.nx) != self.shape:
            raise ValueError("the model must be an [nz][nx] image of the network's size")
        n = p0.numel()
        self.aa_theta = AA(n, M, cond_max)
        self.aa_plain = AA(n, M, cond_max)
        self.red = Reducer()
        self.p = p0.detach().clone().reshape(-1)
        self.g = torch.empty_like(self.p)
        self.d = torch.empty_like(self.p)
        self.pbar, self.ptilde = torch.empty_like(self.p), torch.empty_like(self.p)
        self.pbar_plain, self.ptilde_plain = torch.empty_like(self.p), torch.empty_like(self.p)
        self.trials = [torch.empty_like(self.p) for _ in range(2)]
        self.k = 0
        self.n_fallback = 0
        self.t0 = time.perf_counter()

    def _img(self, x):
        return x.view(1, *self.shape)

    def _direction(self):
        self.net.forward(self._img(self.g), self._img(self.p), z=False, d=self._img(self.d))

    def _maps(self):
        self.aa_theta.step(self.p, self.d, self.eta_theta, self.pbar, self.ptilde)
        self.aa_plain.step(self.p, self.g, self.eta, self.pbar_plain, self.ptilde_plain)
        if self.floor is not None:
            for x in (self.pbar, self.ptilde, self.pbar_plain, self.ptilde_plain):
                floor_(x, self.floor)

    def _search(self, ptilde, J):
        """Backtracking search of Algorithm 2 (Step 4) between ptilde and the
        matching pbar; returns (lambda, accepted buffer) or (0, None)."""
        pbar = self.pbar if ptilde is self.ptilde else self.pbar_plain
        for i, lam in enumerate(self.lambdas):
            trial = self.trials[i % 2]
            blend(lam, ptilde, pbar, trial)
            Jt = self.problem.misfit_keep(trial)
            slope = float(self.red.dot_diff(self.g, trial, self.p).item())
            if Jt <= J + self.c1 * slope:
                self.trials[i % 2] = torch.empty_like(self.p)
                return lam, trial
        return 0.0, None

    def _step_error(self):
        """|eta_theta d - eta g| / |eta g| from three FP64 dot products."""
        if not self.track_step_error:
            return None
        dd = float(self.red.dot(self.d, self.d).item())
        dg = float(self.red.dot(self.d, self.g).item())
        gg = float(self.red.dot(self.g, self.g).item())
        a, b = self.eta_theta, self.eta
        num = max(a * a * dd - 2.0 * a * b * dg + b * b * gg, 0.0)
        return float(np.sqrt(num) / (b * np.sqrt(gg))) if gg > 0 else None

    def _log(self, J, lam, fallback, err=None):
        return LearnedLog(self.k, J, lam, int(self.aa_theta.mk.item()), self.problem.n_adj, self.problem.n_fwd,
                          time.perf_counter() - self.t0, fallback, err)

    def first(self) -> LearnedLog:
        J = self.problem.gradient(self.p, self.g)
        self.J_prev = J
        self._direction()
        if self.eta is None:
            self.eta = step_size(self.p, self.g, self.eta_frac)
        if self.eta_theta is None:
            self.eta_theta = step_size(self.p, self.d, self.eta_frac)
        self._maps()
        self.p = self.pbar
        self.pbar = torch.empty_like(self.p)
        return self._log(J, 0.0, False)

    def iterate(self) -> LearnedLog:
        self.k += 1
        J = self.problem.gradient(self.p, self.g)
        if self.restart and J < self.J_prev:
            if self.fb_theta:
                self.aa_theta.reset()
            if self.fb_plain:
                self.aa_plain.reset()
        self.J_prev = J
        self._direction()
        err = self._step_error()
        self._maps()
        lam, p_next = self._search(self.ptilde, J)
        fallback = False
        self.fb_theta = self.fb_plain = False
        if p_next is None:
            self.fb_theta = True
            if self.problem.misfit_keep(self.pbar) < J:
                p_next = self.pbar
                self.pbar = torch.empty_like(self.p)
            else:
                fallback = True
                self.n_fallback += 1
                lam, p_next = self._search(self.ptilde_plain, J)
                if p_next is None:
                    self.fb_plain = True
                    p_next = self.pbar_plain
                    self.pbar_plain = torch.empty_like(self.p)
        self.p = p_next
        return self._log(J, lam, fallback, err)

    def close(self):
        for a in (self.aa_theta, self.aa_plain):
            a.close()


class BatchedLearnedAADescent(BatchedAADescent):
    """The learned form on many uneven instances at once: every instance runs
    its own Algorithm 2 on G_theta with the plain-AA fallback (its own eta,
    eta_theta, both Anderson windows, restarts and search), while all
    instances share every wave-equation launch of a Batch, one Anderson
    launch sequence per window and map for the whole batch, and one network
    per grid shape.

    A search round runs one masked batched forward for the instances still
    searching, each at its next trial: lambda in {1, 1/2, 1/4, 1/8} between
    ptilde_theta and pbar_theta (Armijo), then pbar_theta itself (accepted
    if it decreases J), then the plain window's lambdas (Armijo), then the
    plain pbar.  Instance by instance this is LearnedAADescent on a separate
    context: the same kernels in the same arithmetic order, so the same
    iterates."""

    def __init__(self, batch: Batch, p0, weights, M: int = 10, etas=None, eta_thetas=None,
                 eta_frac: float = 0.02, cond_max: float = 1e5, lambdas=LAMBDAS, c1: float = ARMIJO_C1,
                 restart: bool = True, project: bool = True):
        if M < 1:
            raise ValueError("the learned form needs an Anderson window (M >= 1)")
        super().__init__(batch, p0, M, etas=etas, eta_frac=eta_frac, cond_max=cond_max, lambdas=lambdas,
                         c1=c1, restart=restart, project=project)
        s = batch.stream
        self.shapes = [tuple(batch.m[i].shape) for i in range(self.N)]
        self.eta_thetas = None if eta_thetas is None else [float(e) for e in eta_thetas]
        # self.aa (the base class's window) is the plain window on G; the
        # theta window holds d_theta
        self.aa_theta = BatchAA([x.numel() for x in self.p], M, cond_max, stream=s)
        self.nets = {sh: CNN(sh[0], sh[1], 1, weights, stream=s) for sh in sorted(set(self.shapes))}
        with torch.cuda.stream(s):
            self.d = [torch.empty_like(x) for x in self.p]
            self.pbar_plain = [torch.empty_like(x) for x in self.p]
            self.ptilde_plain = [torch.empty_like(x) for x in self.p]
        self.fb_theta = [False] * self.N
        self.fb_plain = [False] * self.N
        self.n_fallback = [0] * self.N

    def _directions(self):
        for i in range(self.N):
            sh = self.shapes[i]
            self.nets[sh].forward(self._g(i).view(1, *sh), self.p[i].view(1, *sh), z=False,
                                  d=self.d[i].view(1, *sh))

    def _maps(self):
        self.aa_theta.step(self.p, self.d, self.eta_thetas, self.pbar, self.ptilde)
        self.aa.step(self.p, [self._g(i) for i in range(self.N)], self.etas, self.pbar_plain, self.ptilde_plain)
        if self.floors is not None:
            s = self.b.stream
            for i in range(self.N):
                for x in (self.pbar, self.ptilde, self.pbar_plain, self.ptilde_plain):
                    floor_(x[i], self.floors[i], stream=s)

    def first(self):
        """g_0 and d_theta at p_0 for every instance, then p_1 = G_theta(p_0)."""
        J = self._gradients()
        self.J_prev = np.array(J, np.float64)
        self._directions()
        with torch.cuda.stream(self.b.stream):
            if self.etas is None:
                self.etas = [step_size(self.p[i], self._g(i), self.eta_frac) for i in range(self.N)]
            if self.eta_thetas is None:
                self.eta_thetas = [step_size(self.p[i], self.d[i], self.eta_frac) for i in range(self.N)]
        self._maps()
        with torch.cuda.stream(self.b.stream):
            self.p = [x.clone() for x in self.pbar]
        self.kept_ok = [False] * self.N
        return J

    def _trial(self, i, stage):
        """Write instance i's trial of this search stage into its model
        buffer; returns the acceptance rule ("armijo" or "decrease")."""
        L = len(self.lambdas)
        s = self.b.stream
        if stage < L:
            blend(self.lambdas[stage], self.ptilde[i], self.pbar[i], self._m(i), stream=s)
            return "armijo"
        if stage == L:
            blend(1.0, self.pbar[i], self.pbar[i], self._m(i), stream=s)
            return "decrease"
        blend(self.lambdas[stage - L - 1], self.ptilde_plain[i], self.pbar_plain[i], self._m(i), stream=s)
        return "armijo"

    def iterate(self):
        """One iteration k >= 1 for every instance.

        Returns (J(p_k), lambdas, fallbacks): lambda is 0 where the
        instance took pbar_theta or the plain pbar; fallback marks the
        instances that redid the iteration with plain AA."""
        s = self.b.stream
        L = len(self.lambdas)
        self.k += 1
        J = self._gradients()
        if self.restart:
            th = [self.fb_theta[i] and J[i] < self.J_prev[i] for i in range(self.N)]
            pl = [self.fb_plain[i] and J[i] < self.J_prev[i] for i in range(self.N)]
            if any(th):
                self.aa_theta.reset(th)
            if any(pl):
                self.aa.reset(pl)
        self.J_prev = np.array(J, np.float64)
        self._directions()
        self._maps()
        stage = [0] * self.N
        pending = [True] * self.N
        lam = [0.0] * self.N
        fallback = [False] * self.N
        new_p = [None] * self.N
        self.fb_theta = [False] * self.N
        self.fb_plain = [False] * self.N
        while any(pending):
            idx = [i for i in range(self.N) if pending[i]]
            rule = {i: self._trial(i, stage[i]) for i in idx}
            Jt = self._forward(pending)
            for i in idx:
                if rule[i] == "armijo":
                    self.red.dot_diff(self._g(i), self._m(i), self.p[i], out=self.slope[i:i + 1])
            with torch.cuda.stream(s):
                slope = self.slope.cpu().numpy()
            for i in idx:
                st = stage[i]
                ok = Jt[i] <= J[i] + self.c1 * slope[i] if rule[i] == "armijo" else Jt[i] < J[i]
                if ok:
                    with torch.cuda.stream(s):
                        new_p[i] = self._m(i).clone()
                    lam[i] = self.lambdas[st] if st < L else (0.0 if st == L else self.lambdas[st - L - 1])
                    pending[i] = False
                    self.fb_theta[i] = st >= L
                    continue
                if st == L:
                    # pbar_theta does not decrease J either: redo with plain AA
                    fallback[i] = True
                    self.n_fallback[i] += 1
                stage[i] = st + 1
                if stage[i] == 2 * L + 1:
                    # no plain trial accepted: the plain descent step
                    self.fb_theta[i] = self.fb_plain[i] = True
                    with torch.cuda.stream(s):
                        new_p[i] = self.pbar_plain[i].clone()
                    self.kept_ok[i] = False
                    pending[i] = False
        self.fell_back = [self.fb_theta[i] or self.fb_plain[i] for i in range(self.N)]
        self.b.set_active(np.ones(self.N, np.uint8))
        self.p = new_p
        return J, lam, fallback

    def close(self):
        super().close()
        if self.aa_theta is not None:
            self.aa_theta.close()
            self.aa_theta = None
        for net in self.nets.values():
            net.close()
        self.nets = {}


def init_weights(seed: int):
    """He-normal weights per layer ([C_out][C_in][3][3]); the last layer is
    scaled by 0.1 so that softplus(z) starts near ln 2 (d close to g)."""
    from ._lib import CNN_SHAPES
    rng = np.random.default_rng(seed)
    ws = []
    for i, shp in enumerate(CNN_SHAPES):
        w = rng.standard_normal(shp) * np.sqrt(2.0 / (shp[1] * 9))
        ws.append(w * (0.1 if i == len(CNN_SHAPES) - 1 else 1.0))
    return ws


# ---------------------------------------------------------------------------
# training data
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Pairs:
    g: torch.Tensor   # [N][nz][nx] gradients g_k
    m: torch.Tensor   # [N][nz][nx] models p_k
    s: torch.Tensor   # [N][nz][nx] steps p_{k+1} - p_k
    source: list      # "aa" or "lbfgs" per pair

    def __len__(self):
        return self.g.shape[0]


def _observed(geoms, m_trues):
    """Observed data of each instance: the HIP forward model on the true model."""
    out = []
    for geom, mt in zip(geoms, m_trues):
        with Context(geom) as ctx:
            out.append(ctx.forward_model(torch.from_numpy(np.ascontiguousarray(mt)).cuda()).clone())
    torch.cuda.synchronize()
    return out


def aa_pairs(cases, M: int = 10, iters: int = 8, ckpt_every: int = 50):
    """Pairs from plain Anderson runs on a batch of instances of one size.
    cases: list of (geometry, m_true, m0) on the same grid."""
    geoms = [c[0] for c in cases]
    d_obs = _observed(geoms, [c[1] for c in cases])
    gs, ms, ss = [], [], []
    with Batch(geoms, d_obs, ckpt_every=ckpt_every, use_graphs=True) as b:
        from .batched import BatchedAADescent
        run = BatchedAADescent(b, [torch.from_numpy(c[2]).cuda() for c in cases], M=M)
        run.first()
        for _ in range(iters):
            with torch.cuda.stream(b.stream):
                pk = [x.clone() for x in run.p]
            run.iterate()
            with torch.cuda.stream(b.stream):
                for i in range(b.N):
                    gs.append(b.grad[i].clone())
                    ms.append(pk[i])
                    ss.append(axpy(-1.0, pk[i], run.p[i].clone()))  # p_{k+1} - p_k
        run.close()
        b.stream.synchronize()
    shape = cases[0][2].shape
    st = lambda xs: torch.stack([x.view(shape) for x in xs])
    return Pairs(st(gs), st(ms), st(ss), ["aa"] * len(gs))


def lbfgs_pairs(cases, M: int = 10, iters: int = 6, ckpt_every: int = 50, progress=None):
    """Pairs from L-BFGS(M) runs (one context per instance); progress(i), if
    given, is called after instance i."""
    from .comparators import LBFGS
    gs, ms, ss = [], [], []
    shape = cases[0][2].shape
    for ci, (geom, mt, m0) in enumerate(cases):
        with Context(geom, ckpt_every=ckpt_every) as ctx:
            d_obs = ctx.forward_model(torch.from_numpy(np.ascontiguousarray(mt)).cuda()).clone()
            prob = FWIProblem(ctx, d_obs)
            run = LBFGS(prob, torch.from_numpy(m0).cuda(), M)
            for _ in range(iters):
                pk, gk = run.p.clone(), run.g.clone()
                run.iterate()
                gs.append(gk.view(shape))
                ms.append(pk.view(shape))
                ss.append(axpy(-1.0, pk, run.p.clone()).view(shape))  # p_{k+1} - p_k
        if progress:
            progress(ci)
    return Pairs(torch.stack(gs), torch.stack(ms), torch.stack(ss), ["lbfgs"] * len(gs))


def drop_degenerate(p: Pairs):
    """The pairs that carry a direction: a step of zero (a line search that
    did not move) or a zero gradient makes the scale-free target or input
    0/0, and a non-finite entry poisons every later Adam step; those pairs
    are removed.  Squared norms come from the library's FP64 dot product.
    Returns (pairs kept, number dropped)."""
    red = Reducer()
    n = len(p)
    sq = torch.empty(3, n, dtype=torch.float64, device=p.g.device)
    for i in range(n):
        for k, x in enumerate((p.g[i], p.m[i], p.s[i])):
            red.dot(x, x, sq[k, i:i + 1])
    sq = sq.cpu().numpy()
    keep = np.flatnonzero(np.isfinite(sq).all(axis=0) & (sq[0] > 0) & (sq[2] > 0))
    if len(keep) == n:
        return p, 0
    idx = torch.from_numpy(keep).to(p.g.device)
    return Pairs(p.g.index_select(0, idx), p.m.index_select(0, idx), p.s.index_select(0, idx),
                 [p.source[i] for i in keep]), n - len(keep)


def merge(*ps: Pairs) -> Pairs:
    return Pairs(torch.cat([p.g for p in ps]), torch.cat([p.m for p in ps]), torch.cat([p.s for p in ps]),
                 sum((p.source for p in ps), []))


def flip_x(p: Pairs) -> Pairs:
    """The pairs mirrored along x (augmentation: the layered family and the
    evenly spread shots look alike under the mirror, the network does not)."""
    return Pairs(torch.flip(p.g, dims=[2]).contiguous(), torch.flip(p.m, dims=[2]).contiguous(),
                 torch.flip(p.s, dims=[2]).contiguous(), [f"{x}-flip" for x in p.source])


def train(net: CNN, pairs: Pairs, epochs: int = 20, batch: int = 8, lr: float = 1e-3, seed: int = 5006):
    """Adam over shuffled mini-batches; returns the mean loss of each epoch."""
    rng = np.random.default_rng(seed)
    n = len(pairs)
    hist = []
    for _ in range(epochs):
        order = rng.permutation(n)
        losses = []
        for i in range(0, n - batch + 1, batch):
            idx = torch.from_numpy(order[i:i + batch]).to(pairs.g.device)
            gb = pairs.g.index_select(0, idx).contiguous()
            mb = pairs.m.index_select(0, idx).contiguous()
            sb = pairs.s.index_select(0, idx).contiguous()
            losses.append(net.train_step(gb, mb, sb, lr).clone())
        hist.append(float(torch.cat(losses).mean().item()))
    return hist
