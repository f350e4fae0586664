"""The full-size workloads in the launch shapes the bench uses (the shipped
autotuned shapes, checkpoints every 50 steps), checked against the FP64
oracle over the whole 4000-step record:

* the 768 x 256, 64-shot forward: traces of two sampled shots over all 4000
  steps against the oracle's run of those shots alone (shots do not
  interact), with the error of the first 500, 1000, 2000 and 4000 samples
  printed (FP32 error growth with the record length);
* a two-shot context on the same grid, in the same launch shapes: the
  gradient element by element against the oracle's two-shot gradient, with
  observed data from the oracle's forward run of the true model;
* the 1024 x 384, 96-shot forward: one sampled shot over all 4000 steps;
* the gradient against a central difference of J along a random smooth
  perturbation, and the Born dot-product test, on all 64 shots.

The oracle runs (about a minute of CPU per job) start in threads when the
module's first test asks for them, so they overlap with the GPU work.
"""
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth
from oracle import fd

pytestmark = pytest.mark.gpu

SHOTS = (0, 37)      # sampled shots of the 64-shot case
LARGE_SHOT = 50      # sampled shot of the 96-shot case
GROWTH = (500, 1000, 2000, 4000)


class _OracleRuns:
    """FP64 oracle results for the sampled shots, computed in worker threads
    (NumPy releases the interpreter lock inside its array loops)."""

    def __init__(self):
        g, m_true, m0 = synth.config2()
        self.g, self.m_true, self.m0 = g, m_true, m0
        g5, _, m05 = synth.config5()
        self.g5, self.m05 = g5, m05
        self.pool = ThreadPoolExecutor(len(SHOTS) * 2 + 1)
        # observed data of the sampled shots: the oracle's forward run of the
        # true model, rounded to FP32 as both sides receive it
        self.obs = {s: self.pool.submit(self._fwd, g, m_true, s) for s in SHOTS}
        # forward runs at the start model keeping q^n for the adjoint
        self.fwd = {s: self.pool.submit(self._fwd_keep, g, m0, s) for s in SHOTS}
        self.large = self.pool.submit(self._fwd, g5, m05, LARGE_SHOT)
        self._grad = None
        self._lock = threading.Lock()

    @staticmethod
    def _fwd(g, m, s):
        return fd.forward_shot(g.subset_shots([s]), m, 0)[0]

    @staticmethod
    def _fwd_keep(g, m, s):
        d, qs, _ = fd.forward_shot(g.subset_shots([s]), m, 0, keep_q=True)
        return d, qs

    def traces(self, s):
        return self.fwd[s].result()[0]

    def d_obs(self, s):
        return self.obs[s].result().astype(np.float32)

    def gradient(self):
        """(J, dJ/dm) of the two sampled shots (after the sponge fold)."""
        with self._lock:
            if self._grad is None:
                def adj(s):
                    d, qs = self.fwd[s].result()
                    r = d - self.d_obs(s).astype(np.float64)
                    gp = fd.adjoint_shot(self.g.subset_shots([s]), self.m0, 0, r, qs)
                    return 0.5 * float(np.sum(r * r)), gp
                parts = list(self.pool.map(adj, SHOTS))
                J = sum(p[0] for p in parts)
                g_pad = sum(p[1] for p in parts)
                self._grad = (J, fd.fold(g_pad, self.g.nz, self.g.nx, self.g.nb))
                for s in SHOTS:  # free the q^n lists (7.6 GB per shot)
                    self.fwd[s] = _Done(self.fwd[s].result()[0], None)
            return self._grad

    def close(self):
        self.pool.shutdown(wait=True)


class _Done:
    def __init__(self, d, qs):
        self._v = (d, qs)

    def result(self):
        return self._v


@pytest.fixture(scope="module")
def oracle_runs():
    runs = _OracleRuns()
    yield runs
    runs.close()


@pytest.fixture(scope="module")
def c2():
    import torch
    from paper_2008_11778_amd import Context, autotune
    g, m_true, m0 = synth.config2()
    ctx = Context(g, ckpt_every=50)
    m0t = torch.from_numpy(m0).cuda()
    shapes = autotune.tune(g, m0t)
    autotune.apply(ctx, shapes)
    yield g, m_true, m0, ctx, shapes
    ctx.close()


def _growth(got, ref):
    out = {}
    for n in GROWTH:
        n = min(n, ref.shape[0])
        out[n] = float(np.linalg.norm(got[:n] - ref[:n]) / np.linalg.norm(ref[:n]))
    return out


def test_sampled_shot_traces_full_record(oracle_runs, c2):
    """Both sampled shots of the 64-shot forward over all 4000 steps within
    1e-4 relative L2 (each gather, and the two together)."""
    import torch
    g, _, m0, ctx, shapes = c2
    print("launch shapes:", shapes, "modes (bit mask):", ctx.time_blocking())
    d = ctx.forward_model(torch.from_numpy(m0).cuda()).cpu().numpy()
    got_all, ref_all = [], []
    for s in SHOTS:
        ref = oracle_runs.traces(s)
        got = d[s]
        assert got.shape == ref.shape == (4000, g.nrec)
        gr = _growth(got, ref)
        print(f"shot {s}: rel L2 by record length " + ", ".join(f"nt={n}: {e:.2e}" for n, e in gr.items()))
        assert gr[4000] <= 1e-4, (s, gr)
        got_all.append(got)
        ref_all.append(ref)
    err = float(np.linalg.norm(np.stack(got_all) - np.stack(ref_all)) / np.linalg.norm(np.stack(ref_all)))
    print(f"both shots: rel L2 {err:.2e}")
    assert err <= 1e-4


def test_two_shot_gradient_matches_oracle(oracle_runs, c2):
    """A context of the two sampled shots in the bench's launch shapes with
    checkpoints every 50 steps: misfit within 1e-3 and the gradient element
    by element within 1e-3 relative L2 of the oracle's."""
    import torch
    from paper_2008_11778_amd import Context, autotune
    g, _, m0, _, shapes = c2
    g2 = g.subset_shots(list(SHOTS))
    d_obs = np.stack([oracle_runs.d_obs(s) for s in SHOTS])
    with Context(g2, ckpt_every=50) as ctx2:
        autotune.apply(ctx2, shapes)
        print("modes (bit mask):", ctx2.time_blocking(), "rows:", [ctx2.get_tile(k) for k in range(4)])
        grad, J = ctx2.adjoint_gradient(torch.from_numpy(m0).cuda(), torch.from_numpy(d_obs).cuda())
        grad = grad.cpu().numpy().astype(np.float64)
        J = float(J.item())
    J_ref, g_ref = oracle_runs.gradient()
    eJ = abs(J - J_ref) / abs(J_ref)
    eg = float(np.linalg.norm(grad - g_ref) / np.linalg.norm(g_ref))
    # the largest pointwise deviation, relative to the gradient's peak
    emax = float(np.abs(grad - g_ref).max() / np.abs(g_ref).max())
    print(f"J {J:.9e} oracle {J_ref:.9e} (rel {eJ:.2e}); gradient rel L2 {eg:.2e}, max abs / peak {emax:.2e}")
    assert grad.shape == g_ref.shape == (g.nz, g.nx)
    assert eJ <= 1e-3
    assert eg <= 1e-3


def test_large_grid_sampled_shot_full_record(oracle_runs):
    """The 1024 x 384, 96-shot forward in its shipped launch shapes: one
    sampled shot over all 4000 steps within 1e-4."""
    import torch
    from paper_2008_11778_amd import Context, autotune
    g, m0 = oracle_runs.g5, oracle_runs.m05
    with Context(g, ckpt_every=50) as ctx:
        m = torch.from_numpy(m0).cuda()
        autotune.apply(ctx, autotune.tune(g, m))
        print("modes (bit mask):", ctx.time_blocking(), "rows:", [ctx.get_tile(k) for k in range(4)])
        got = ctx.forward_model(m)[LARGE_SHOT].cpu().numpy()
    ref = oracle_runs.large.result()
    gr = _growth(got, ref)
    print(f"shot {LARGE_SHOT}: rel L2 by record length " + ", ".join(f"nt={n}: {e:.2e}" for n, e in gr.items()))
    assert gr[4000] <= 1e-4


def test_gradient_directional_derivative(c2):
    import torch
    g, m_true, m0, ctx, _ = c2
    d_obs = ctx.forward_model(torch.from_numpy(m_true).cuda()).clone()
    r = np.random.default_rng(17)
    dm = synth.smooth(r.standard_normal(m0.shape), 6.0)
    dm = (dm / np.abs(dm).max() * 0.002 * np.abs(m0).max()).astype(np.float32)
    m = torch.from_numpy(m0).cuda()
    grad, J = ctx.adjoint_gradient(m, d_obs)
    slope = float((grad.double() * torch.from_numpy(dm).cuda().double()).sum())
    Jp = ctx.adjoint_gradient(m + torch.from_numpy(dm).cuda(), d_obs)[1].item()
    Jm = ctx.adjoint_gradient(m - torch.from_numpy(dm).cuda(), d_obs)[1].item()
    fd_slope = (Jp - Jm) / 2.0
    print(f"J {J.item():.6e} slope {slope:.6e} central difference {fd_slope:.6e}")
    assert abs(fd_slope - slope) <= 1e-2 * abs(slope)


def test_born_dot_product(c2):
    import torch
    g, _, m0, ctx, _ = c2
    r = np.random.default_rng(18)
    x = torch.from_numpy((synth.smooth(r.standard_normal(m0.shape), 2.0) * 1e-9).astype(np.float32)).cuda()
    y = torch.from_numpy(r.standard_normal((g.nshots, g.nt, g.nrec)).astype(np.float32)).cuda()
    m = torch.from_numpy(m0).cuda()
    lx = ctx.born(m, x)
    lty = ctx.born_adjoint(m, y)
    a = float((lx.double() * y.double()).sum())
    b = float((x.double() * lty.double()).sum())
    print(f"<Lx, y> {a:.9e} <x, L^T y> {b:.9e}")
    assert abs(a - b) <= 1e-4 * abs(a)
