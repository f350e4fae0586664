"""Options of the Anderson step against the oracle.

* The rank-updated QR solver of the least squares (Algorithm 2, Step 2)
  against the oracle's definition of gamma (SVD least squares in FP64 of the
  same FP32 gradients): the step, the window drops (full ring and condition
  guard), and its accuracy on an ill-conditioned window, where the FP64
  normal equations lose about cond^2 * eps and the QR update cond * eps.
* Damping beta and a weighted l2 norm, on both solvers."""
import numpy as np
import pytest

from oracle import aa as oaa

pytestmark = pytest.mark.gpu


def T(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_qr_step_matches_oracle_through_ring_drops():
    from paper_2008_11778_amd import AA
    r = np.random.default_rng(8)
    n, M, eta = 5000, 3, 0.37
    ref = oaa.AAHistory(M, cond_max=1e5)
    aa = AA(n, M, cond_max=1e5, solver="qr")
    p = r.standard_normal(n).astype(np.float32)
    for k in range(9):  # the ring of M + 1 = 4 fills at k = 3 and then drops one per step
        g = (r.standard_normal(n) + 0.3 * k).astype(np.float32)
        pb, pt = aa.step(T(p), T(g), eta)
        pbr, ptr_, gam, mk = ref.step(p, g, eta)
        assert int(aa.mk.item()) == mk
        assert rel(pb.cpu().numpy(), pbr) <= 1e-6
        assert rel(pt.cpu().numpy(), ptr_) <= 1e-5, (k, rel(pt.cpu().numpy(), ptr_))
        if mk:
            np.testing.assert_allclose(aa.gamma.cpu().numpy()[:mk], gam, rtol=1e-9, atol=1e-12)
        p = ptr_.astype(np.float32)
    aa.close()


def test_qr_condition_guard_matches_oracle():
    from paper_2008_11778_amd import AA
    r = np.random.default_rng(9)
    n, M = 3000, 5
    base = r.standard_normal(n)
    ref = oaa.AAHistory(M, cond_max=1e5)
    aa = AA(n, M, cond_max=1e5, solver="qr")
    p = np.zeros(n, np.float32)
    for k in range(6):
        g = (base * (1 + k) + (1e-7 if k % 2 else 1e-2) * r.standard_normal(n)).astype(np.float32)
        _, pt = aa.step(T(p), T(g), 0.1)
        _, ptr_, _, mk = ref.step(p, g, 0.1)
        assert int(aa.mk.item()) == mk, (k, int(aa.mk.item()), mk)
        assert rel(pt.cpu().numpy(), ptr_) <= 1e-4, (k, rel(pt.cpu().numpy(), ptr_))
        p = (p + 0.01).astype(np.float32)
    aa.close()


def ill_conditioned_gradients(n=20000, sig=(1.0, 1e-1, 1e-3, 2e-5), seed=3):
    """g_0 = 0 and g_{i+1} = g_i + a_i with a = U diag(sig) V^T (cond 5e4),
    small enough values that FP32 rounding stays far below sig_min."""
    r = np.random.default_rng(seed)
    U, _ = np.linalg.qr(r.standard_normal((n, len(sig))))
    V, _ = np.linalg.qr(r.standard_normal((len(sig), len(sig))))
    A = U @ np.diag(sig) @ V.T
    gs = [np.zeros(n)]
    for i in range(len(sig)):
        gs.append(gs[-1] + A[:, i])
    return [g.astype(np.float32) for g in gs], r.standard_normal(n).astype(np.float32)


def test_qr_is_accurate_on_an_ill_conditioned_window():
    from paper_2008_11778_amd import AA
    gs, p = ill_conditioned_gradients()
    n, M = p.size, 4
    errs = {}
    for solver in ("gram", "qr"):
        ref = oaa.AAHistory(M, cond_max=1e5)
        aa = AA(n, M, cond_max=1e5, solver=solver)
        for g in gs:
            aa.step(T(p), T(g), 0.05)
            _, _, gam, mk = ref.step(p, g, 0.05)
        assert int(aa.mk.item()) == mk == 4
        got = aa.gamma.cpu().numpy()[:mk]
        errs[solver] = float(np.abs(got - gam).max() / np.abs(gam).max())
        aa.close()
    print("gamma error vs FP64 SVD least squares:", errs)
    assert errs["qr"] <= 1e-9
    assert errs["qr"] < errs["gram"]


@pytest.mark.parametrize("solver", ["gram", "qr"])
def test_damped_and_weighted_steps_match_oracle(solver):
    """Damping beta (eq. AAupdate0 in the gamma form) and a weighted l2
    least-squares norm, on both solvers, against the oracle step."""
    import torch
    from paper_2008_11778_amd import AA
    r = np.random.default_rng(12)
    n, M, eta, beta = 4000, 3, 0.21, 0.6
    w = r.uniform(0.2, 3.0, n).astype(np.float32)
    ref = oaa.AAHistory(M, cond_max=1e5, beta=beta, weights=w.astype(np.float64))
    aa = AA(n, M, cond_max=1e5, solver=solver)
    aa.set_damping(beta)
    wt = T(w)
    aa.set_weights(wt)
    p = r.standard_normal(n).astype(np.float32)
    for k in range(7):
        g = (r.standard_normal(n) + 0.2 * k).astype(np.float32)
        pb, pt = aa.step(T(p), T(g), eta)
        pbr, ptr_, gam, mk = ref.step(p, g, eta)
        assert int(aa.mk.item()) == mk
        assert rel(pb.cpu().numpy(), pbr) <= 1e-6
        assert rel(pt.cpu().numpy(), ptr_) <= 1e-5, (k, rel(pt.cpu().numpy(), ptr_))
        if mk:
            np.testing.assert_allclose(aa.gamma.cpu().numpy()[:mk], gam, rtol=1e-6, atol=1e-9)
        p = ptr_.astype(np.float32)
    torch.cuda.synchronize()
    aa.close()
