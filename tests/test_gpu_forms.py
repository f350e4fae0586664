"""GPU tests of the autograd form and the comparators (GMRES(M) on the LSRTM
normal equations, L-BFGS, Algorithm 2 on LSRTM) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import aa as oaa
from oracle import fd, krylov

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def T(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


@pytest.fixture(scope="module")
def fwi_small():
    g, m = synth.small_case(nz=40, nx=70, nb=10, nt=260, nshots=3, nrec=14, f0=18.0, instance=4)
    r = np.random.default_rng(21)
    m_true = (m.astype(np.float64) * (1 + 0.03 * r.standard_normal(m.shape))).astype(np.float32)
    d_obs = fd.forward_model(g, m_true).astype(np.float32)
    return g, m, d_obs


@pytest.fixture(scope="module")
def lsrtm_small():
    g, _ = synth.small_case(nz=40, nx=70, nb=10, nt=260, nshots=3, nrec=14, f0=18.0, instance=5)
    v0 = synth.lsrtm_background(40, 70, 1800.0, 2600.0)
    m0 = synth.to_m(v0)
    dm = np.zeros_like(m0, dtype=np.float64)
    dm[15, 10:60] = 0.05 * m0[15, 10:60]
    dm[28, 5:50] = -0.04 * m0[28, 5:50]
    dm = dm.astype(np.float32)
    g = g.replace(vref=float(v0.max()))
    d_r = fd.born(g, m0, dm).astype(np.float32)
    return g, m0, dm, d_r


def test_autograd_gradient(fwi_small):
    import torch
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.autograd import seismic_forward
    g, m, d_obs = fwi_small
    J_ref, g_ref = fd.adjoint_gradient(g, m, d_obs)
    with Context(g, ckpt_every=23) as ctx:
        mt = T(m).requires_grad_(True)
        d = seismic_forward(mt, ctx)
        loss = 0.5 * ((d - T(d_obs)) ** 2).sum()
        loss.backward()
        grad_ag = mt.grad.cpu().numpy()
        grad_c, J = ctx.adjoint_gradient(T(m), T(d_obs))
        grad_c = grad_c.cpu().numpy()
    assert rel(grad_ag, g_ref) <= 1e-3, rel(grad_ag, g_ref)
    np.testing.assert_allclose(grad_ag, grad_c, rtol=1e-5, atol=1e-6 * np.abs(grad_c).max())


def test_autograd_finite_difference(fwi_small):
    """Central difference of J along dm (FP32 forward, FP64 misfit sum)."""
    import torch
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.autograd import seismic_forward
    g, m, d_obs = fwi_small
    dm = (0.01 * m * np.random.default_rng(22).standard_normal(m.shape)).astype(np.float32)
    with Context(g) as ctx:
        mt = T(m).requires_grad_(True)
        d = seismic_forward(mt, ctx)
        (0.5 * ((d - T(d_obs)) ** 2).sum()).backward()
        slope = float((mt.grad.double() * T(dm).double()).sum())

        def J(mm):
            dd = ctx.forward_model(T(mm))
            return 0.5 * float(((dd.double() - T(d_obs).double()) ** 2).sum())

        fdv = (J(m + dm) - J(m - dm)) / 2.0
    assert abs(fdv - slope) / abs(slope) < 5e-3, (fdv, slope)


def test_autograd_recomputes_after_foreign_forward(fwi_small):
    import torch
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.autograd import seismic_forward
    g, m, d_obs = fwi_small
    with Context(g) as ctx:
        mt = T(m).requires_grad_(True)
        d = seismic_forward(mt, ctx)
        ctx.forward_model(T(m * 1.05), keep_ckpt=True)  # another run replaces the checkpoints
        (0.5 * ((d - T(d_obs)) ** 2).sum()).backward()
        g_after = mt.grad.cpu().numpy()
        g_clean = ctx.adjoint_gradient(T(m), T(d_obs))[0].cpu().numpy()
    np.testing.assert_allclose(g_after, g_clean, rtol=1e-5, atol=1e-6 * np.abs(g_clean).max())


def test_born_adjoint_reuses_background_run(lsrtm_small):
    from paper_2008_11778_amd import Context
    g, m0, dm, d_r = lsrtm_small
    y = np.random.default_rng(23).standard_normal(d_r.shape).astype(np.float32)
    ref = fd.born_adjoint(g, m0, y)
    with Context(g) as ctx:
        a = ctx.born_adjoint(T(m0), T(y)).cpu().numpy()
        ctx.born(T(m0), T(dm))
        b = ctx.born_adjoint(T(m0), T(y)).cpu().numpy()  # reuses the kept m0 run
        ctx.born_adjoint(T(m0 * 1.1), T(y))             # different background
        c = ctx.born_adjoint(T(m0), T(y)).cpu().numpy()
    assert rel(a, ref) <= 1e-3
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_gmres_lsrtm_matches_oracle(lsrtm_small):
    import torch
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.comparators import gmres_restarted
    from paper_2008_11778_amd.inversion import LSRTMProblem
    g, m0, dm, d_r = lsrtm_small
    rtm_ref = fd.born_adjoint(g, m0, d_r).ravel()
    LtL = lambda x: fd.born_adjoint(g, m0, fd.born(g, m0, x.reshape(m0.shape))).ravel()
    ref = krylov.gmres_restarted(LtL, rtm_ref, np.zeros(m0.size), 3, 6)
    with Context(g) as ctx:
        prob = LSRTMProblem(ctx, T(m0), T(d_r))
        b = ctx.born_adjoint(T(m0), T(d_r)).reshape(-1)
        xs = gmres_restarted(lambda x, out: prob.normal_op(x.view(m0.shape), out.view(m0.shape)),
                             b, torch.zeros_like(b), 3, 6)
    for k, (a, r_) in enumerate(zip(xs, ref)):
        print(f"gmres iterate {k}: rel {rel(a.cpu().numpy(), r_):.2e}")
        assert rel(a.cpu().numpy(), r_) <= 2e-3, (k, rel(a.cpu().numpy(), r_))


def test_aa_lsrtm_matches_oracle(lsrtm_small):
    import torch
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.inversion import LSRTMProblem, aa_descent
    g, m0, dm, d_r = lsrtm_small
    shape = m0.shape

    def grad_fn(x):
        res = fd.born(g, m0, x.reshape(shape)) - d_r
        return 0.5 * float(np.sum(res * res)), fd.born_adjoint(g, m0, res).ravel()

    def mis_fn(x):
        res = fd.born(g, m0, x.reshape(shape)) - d_r
        return 0.5 * float(np.sum(res * res))

    J0, g0 = grad_fn(np.zeros(m0.size))
    eta = float(0.3 * np.abs(dm).max() / np.abs(g0).max())
    ref = oaa.alg2(grad_fn, mis_fn, np.zeros(m0.size), eta, 3, 4)
    with Context(g) as ctx:
        prob = LSRTMProblem(ctx, T(m0), T(d_r))
        its, hist, _ = aa_descent(prob, torch.zeros(shape, device="cuda:0"), eta, M=3, iters=4)
    assert [h.lam for h in hist[1:]] == ref["lambdas"]
    for k, (a, r_) in enumerate(zip(its, ref["iterates"])):
        if k == 0:
            continue
        assert rel(a.cpu().numpy(), r_) <= 2e-3, (k, rel(a.cpu().numpy(), r_))


def test_two_loop_matches_oracle():
    import torch
    from paper_2008_11778_amd.comparators import two_loop
    r = np.random.default_rng(24)
    n, k = 4000, 4
    A = r.standard_normal((n, 8)) / np.sqrt(n)
    S = [r.standard_normal(n).astype(np.float32) for _ in range(k)]
    Y = [(s + A @ (A.T @ s)).astype(np.float32) for s in S]
    gv = r.standard_normal(n).astype(np.float32)
    ref = krylov.two_loop(gv.astype(np.float64), [s.astype(np.float64) for s in S], [y.astype(np.float64) for y in Y])
    out = two_loop(T(gv), [T(s) for s in S], [T(y) for y in Y]).cpu().numpy()
    assert rel(out, ref) <= 1e-5


def _check_strong_wolfe(st, c1=1e-4):
    """The strong-Wolfe conditions on an accepted step (Nocedal and Wright,
    eq. 3.7): sufficient decrease J(p + a d) <= J(p) + c1 a g.d and the
    curvature bound |g(p + a d).d| <= c2 |g.d|, with g.d < 0.  Several points
    can satisfy them, so this checks validity, not the point chosen."""
    assert st["d0"] < 0.0, st
    assert st["alpha"] > 0.0, st
    assert st["J"] <= st["J0"] + c1 * st["alpha"] * st["d0"], st
    assert abs(st["slope"]) <= st["c2"] * abs(st["d0"]), st


def test_lbfgs_fwi_steps_satisfy_strong_wolfe(fwi_small):
    """L-BFGS (M = 5) on a small FWI problem: every accepted step satisfies
    both strong-Wolfe conditions (c1 = 1e-4, c2 = 0.9), checked from the
    misfits and directional derivatives the HIP path computed, and J falls."""
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.comparators import LBFGS
    from paper_2008_11778_amd.inversion import FWIProblem
    g, m, d_obs = fwi_small
    with Context(g) as ctx:
        prob = FWIProblem(ctx, T(d_obs))
        opt = LBFGS(prob, T(m), M=5)
        Js = [opt.J]
        for _ in range(4):
            Js.append(opt.iterate())
            print(opt.last_step)
            _check_strong_wolfe(opt.last_step)
    assert all(b < a for a, b in zip(Js, Js[1:])), Js


def test_ncg_matches_oracle_iterates(fwi_small):
    """Polak-Ribiere+ CG on the HIP path against the oracle's, from the same
    start and the same first step: same line-search outcome, iterates within
    the gradient tolerance; every accepted step satisfies the strong-Wolfe
    conditions (c1 = 1e-4, c2 = 0.1) on the HIP path's own values."""
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.comparators import NCG
    from paper_2008_11778_amd.inversion import FWIProblem
    g, m, d_obs = fwi_small
    shape = m.shape
    with Context(g) as ctx:
        prob = FWIProblem(ctx, T(d_obs))
        opt = NCG(prob, T(m))
        a1 = opt.a_init * float(np.linalg.norm(fd.adjoint_gradient(g, m, d_obs)[1]))
        its = [opt.p.cpu().numpy()]
        Js = [opt.J]
        steps = []
        for _ in range(2):
            Js.append(opt.iterate())
            its.append(opt.p.cpu().numpy())
            steps.append(opt.last_step)
    ref = krylov.ncg(lambda p: fd.adjoint_gradient(g, p.reshape(shape), d_obs), m.ravel(), 2, a1=a1)
    assert all(b < a for a, b in zip(Js, Js[1:])), Js
    for st in steps:
        _check_strong_wolfe(st)
    for k, (a, b) in enumerate(zip(its, ref)):
        assert rel(a, b) <= 1e-3, (k, rel(a, b))


def test_laplacian_filter_matches_oracle():
    from paper_2008_11778_amd._lib import laplacian_filter
    r = np.random.default_rng(44)
    img = r.standard_normal((37, 53)).astype(np.float32)
    out = laplacian_filter(T(img), 12.5).cpu().numpy()
    assert rel(out, fd.rtm_filter(img, 12.5)) <= 1e-6


def test_filtered_rtm_and_scaled_start_match_oracle(lsrtm_small):
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.inversion import LSRTMProblem
    g, m0, dm, d_r = lsrtm_small
    x_ref, a_ref = fd.scaled_rtm_start(g, m0, d_r)
    f_ref = fd.rtm_filter(fd.born_adjoint(g, m0, d_r), g.h)
    with Context(g) as ctx:
        prob = LSRTMProblem(ctx, T(m0), T(d_r))
        f = prob.filtered_rtm(g.h).cpu().numpy()
        x0, alpha = prob.scaled_start(g.h)
        x0 = x0.cpu().numpy()
    assert rel(f, f_ref) <= 1e-3
    assert abs(alpha - a_ref) / abs(a_ref) <= 1e-3
    assert rel(x0, x_ref) <= 1e-3


def test_autograd_problem_matches_c_abi_problem(fwi_small):
    """The autograd form of J and its gradient (torch.autograd over the same
    forward, the library's residual kernel and the same adjoint) hands the
    adjoint the same FP32 residual as the C-ABI problem: identical gradients,
    identical J, and the same Algorithm 2 iterates over a few iterations."""
    import torch
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd.inversion import AADescent, AutogradFWIProblem, FWIProblem
    g, m, d_obs = fwi_small
    with Context(g, ckpt_every=32) as ctx:
        do = T(d_obs)
        mt = T(m).reshape(-1)
        g1, g2 = torch.empty_like(mt), torch.empty_like(mt)
        J1 = FWIProblem(ctx, do).gradient(mt, g1)
        J2 = AutogradFWIProblem(ctx, do).gradient(mt, g2)
        assert torch.equal(g1, g2)
        assert J1 == J2
        ps = []
        for prob in (FWIProblem(ctx, do), AutogradFWIProblem(ctx, do)):
            run = AADescent(prob, T(m), None, M=5)
            run.first()
            lams = [run.iterate().lam for _ in range(3)]
            ps.append((run.p.clone(), lams))
            run.close()
    assert ps[0][1] == ps[1][1]
    assert float(torch.linalg.norm(ps[0][0] - ps[1][0]) / torch.linalg.norm(ps[0][0])) <= 1e-6
