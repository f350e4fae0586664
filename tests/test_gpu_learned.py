"""Algorithm 2 on the learned map G_theta and its plain-AA fallback.

* With the last layer zero, z = 0 and d = ln(2) g, so AA on G_theta follows
  plain AA on G (up to FP32 rounding of eta_theta d versus eta g).
* A step size far beyond stability makes every learned trial and pbar_theta
  worse than p_k on a diagonal quadratic; every iteration then falls back,
  and the iterates are those of plain Algorithm 2 from the same history.
* Training pairs from the batched AA runs chain p_{k+1} = p_k + s_k and
  pair each p_k with the gradient computed at it."""
import numpy as np
import pytest

import synth
from oracle import fd

pytestmark = pytest.mark.gpu


def zero_gate_weights(seed=3):
    from paper_2008_11778_amd.learned import init_weights
    ws = init_weights(seed)
    ws[3] = np.zeros_like(ws[3])
    return ws


class Quadratic:
    """J(p) = 1/2 sum w (p - t)^2 with torch ops (test scaffolding only)."""

    def __init__(self, w, t):
        self.w, self.t = w, t
        self.n_fwd = self.n_adj = 0

    def misfit_keep(self, p):
        self.n_fwd += 1
        return float((0.5 * self.w.double() * (p.double() - self.t.double()) ** 2).sum().item())

    def gradient(self, p, g):
        self.n_adj += 1
        g.copy_(self.w * (p - self.t))
        return self.misfit_keep(p)


def test_zero_gate_follows_plain_aa():
    import torch
    from paper_2008_11778_amd import CNN, Context
    from paper_2008_11778_amd.inversion import AADescent, FWIProblem
    from paper_2008_11778_amd.learned import LearnedAADescent
    g, m = synth.small_case(nz=30, nx=44, nb=10, nt=220, nshots=3, nrec=11, instance=21)
    r = np.random.default_rng(21)
    mt = (m.astype(np.float64) * (1 + 0.03 * r.standard_normal(m.shape))).astype(np.float32)
    d_obs = fd.forward_model(g, mt).astype(np.float32)
    with Context(g, ckpt_every=30) as ctx, CNN(g.nz, g.nx, 1, zero_gate_weights()) as net:
        dd = torch.from_numpy(d_obs).cuda()
        plain = AADescent(FWIProblem(ctx, dd), torch.from_numpy(m).cuda(), None, M=3)
        learned = LearnedAADescent(FWIProblem(ctx, dd), torch.from_numpy(m).cuda(), net, M=3)
        plain.first()
        learned.first()
        assert abs(learned.eta_theta * np.log(2.0) / plain.eta - 1) < 1e-5
        for k in range(4):
            a, b = plain.iterate(), learned.iterate()
            assert a.lam == b.lam and not b.fallback, k
            assert abs(a.J - b.J) <= 1e-4 * a.J, k
            pa, pb = plain.p.cpu().numpy(), learned.p.cpu().numpy()
            assert np.linalg.norm(pa - pb) <= 1e-5 * np.linalg.norm(pa), k
        plain.close()
        learned.close()


def test_fallback_reproduces_plain_algorithm2():
    import torch
    from paper_2008_11778_amd import CNN
    from paper_2008_11778_amd.inversion import AADescent
    from paper_2008_11778_amd.learned import LearnedAADescent
    nz, nx = 20, 50
    r = np.random.default_rng(4)
    w = torch.from_numpy(r.uniform(0.5, 1.0, nz * nx).astype(np.float32)).cuda()
    t = torch.from_numpy(r.standard_normal(nz * nx).astype(np.float32)).cuda()
    p0 = torch.from_numpy((1.0 + 0.1 * r.standard_normal((nz, nx))).astype(np.float32)).cuda()
    eta = 0.5
    with CNN(nz, nx, 1, zero_gate_weights()) as net:
        # eta_theta * ln 2 * w is 170 to 350: G_theta amplifies every error
        # mode, beyond what extrapolation over two history columns can undo
        learned = LearnedAADescent(Quadratic(w, t), p0, net, M=2, eta=eta, eta_theta=500.0)
        learned.first()
        plain = AADescent(Quadratic(w, t), p0, eta, M=2)
        plain.first()
        # the same p_1 = G(p_0) and the same (p_0, g_0) history on both sides
        learned.p = plain.p.clone()
        for k in range(5):
            b = learned.iterate()
            a = plain.iterate()
            assert b.fallback and b.lam == a.lam, k
            assert torch.equal(learned.p, plain.p), k
        assert learned.n_fallback == 5
        plain.close()
        learned.close()


def test_aa_pairs_chain_and_gradients():
    import torch
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.learned import aa_pairs
    cases = []
    for i in range(2):
        g, m = synth.small_case(nz=24, nx=40, nb=8, nt=160, nshots=2, nrec=9, instance=30 + i)
        r = np.random.default_rng(30 + i)
        mt = (m.astype(np.float64) * (1 + 0.03 * r.standard_normal(m.shape))).astype(np.float32)
        cases.append((g, mt, m))
    pairs = aa_pairs(cases, M=3, iters=3, ckpt_every=20)
    assert len(pairs) == 6 and pairs.g.shape == (6, 24, 40)
    for i in range(2):
        idx = [k * 2 + i for k in range(3)]
        for a, b in zip(idx[:-1], idx[1:]):
            np.testing.assert_allclose((pairs.m[a] + pairs.s[a]).cpu().numpy(), pairs.m[b].cpu().numpy(),
                                       rtol=1e-6, atol=0)
    # the gradient paired with p_k is the gradient at p_k
    g0, mt0, _ = cases[0]
    with Context(g0, ckpt_every=20) as ctx:
        d_obs = ctx.forward_model(torch.from_numpy(mt0).cuda())
        grad, _ = ctx.adjoint_gradient(pairs.m[2].contiguous(), d_obs)
        assert torch.equal(grad.view(24, 40), pairs.g[2])
