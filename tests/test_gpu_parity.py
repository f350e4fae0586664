"""GPU (FP32 HIP path, through the C ABI) versus the FP64 oracle on identical
seeded FP32 inputs.

Tolerances (relative L2): seismograms and Born data 1e-4, gradients and
Born-adjoint images 1e-3, the Anderson candidate p_tilde 1e-5.
"""
import numpy as np
import pytest

import synth
from oracle import aa as oaa
from oracle import fd

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda", 0)


def T(torch, dev, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype or np.float32)).to(dev)


@pytest.fixture(scope="module")
def c1():
    g, m_true, m0 = synth.config1()
    d_obs = fd.forward_model(g, m_true).astype(np.float32)
    return g, m_true, m0, d_obs


@pytest.fixture(scope="module")
def c1_oracle(c1):
    g, m_true, m0, d_obs = c1
    d0 = fd.forward_model(g, m0)
    J, grad = fd.adjoint_gradient(g, m0, d_obs)
    return d0, J, grad


def ragged_case(nshots=3, nt=300):
    """Grid spanning several 64-column tiles and z-strips, with ragged tails,
    receivers in two rows (one duplicated node) and a source in the sponge
    neighbourhood."""
    g, m = synth.small_case(nz=70, nx=150, nb=10, nt=nt, nshots=nshots, nrec=12, f0=20.0, instance=3)
    r = np.random.default_rng(11)
    rec_iz = np.tile(np.array([2] * 6 + [40] * 6, np.int32), (nshots, 1))
    rec_ix = np.tile(np.array([0, 31, 63, 64, 100, 149, 5, 5, 77, 120, 140, 149], np.int32), (nshots, 1))
    g = g.replace(rec_iz=rec_iz, rec_ix=rec_ix, src_iz=np.array([0, 35, 69][:nshots], np.int32),
                  src_ix=np.array([0, 75, 149][:nshots], np.int32))
    return g, m


def test_forward_parity_config1(torch_dev, c1, c1_oracle):
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m_true, m0, d_obs = c1
    d0, _, _ = c1_oracle
    with Context(g) as ctx:
        d = ctx.forward_model(T(torch, dev, m0)).cpu().numpy()
    print(f"config1: seismogram rel L2 {rel(d, d0):.2e}")
    assert rel(d, d0) <= 1e-4, rel(d, d0)
    for s in range(g.nshots):
        assert rel(d[s], d0[s]) <= 1e-4, (s, rel(d[s], d0[s]))


def test_gradient_parity_config1(torch_dev, c1, c1_oracle):
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m_true, m0, d_obs = c1
    _, J_ref, g_ref = c1_oracle
    with Context(g) as ctx:
        grad, J = ctx.adjoint_gradient(T(torch, dev, m0), T(torch, dev, d_obs))
        grad = grad.cpu().numpy()
        J = float(J.item())
    print(f"config1: J rel {abs(J - J_ref) / J_ref:.2e}, gradient rel L2 {rel(grad, g_ref):.2e}")
    # J = 1/2 |r|^2 amplifies the seismogram error by |d|/|r|: misfits take 1e-3
    assert abs(J - J_ref) / J_ref <= 1e-3, (J, J_ref)
    assert rel(grad, g_ref) <= 1e-3, rel(grad, g_ref)


def test_ragged_grid_forward_and_gradient(torch_dev):
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m = ragged_case()
    m_true = (m.astype(np.float64) * (1 + 0.02 * np.random.default_rng(5).standard_normal(m.shape))).astype(np.float32)
    d_obs = fd.forward_model(g, m_true).astype(np.float32)
    d_ref = fd.forward_model(g, m)
    J_ref, g_ref = fd.adjoint_gradient(g, m, d_obs)
    for rows in (0, 16, 37, 64):
        with Context(g, ckpt_every=37) as ctx:
            ctx.set_tile(rows)
            d = ctx.forward_model(T(torch, dev, m)).cpu().numpy()
            grad, J = ctx.adjoint_gradient(T(torch, dev, m), T(torch, dev, d_obs))
            grad = grad.cpu().numpy()
        print(f"ragged rows={rows}: d {rel(d, d_ref):.2e} grad {rel(grad, g_ref):.2e}")
        assert rel(d, d_ref) <= 1e-4, (rows, rel(d, d_ref))
        assert rel(grad, g_ref) <= 1e-3, (rows, rel(grad, g_ref))
        assert abs(float(J.item()) - J_ref) / J_ref <= 1e-3


def test_single_cell_interior_and_one_step(torch_dev):
    """Degenerate sizes: a 1x1 interior, one time step, one receiver."""
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g = synth.make_geometry(1, 1, 10.0, 1, 1e-3, 1, nb=4, vref=2000.0, src_depth=0, rec_depth=0)
    g = g.replace(wavelet=np.array([1.0], np.float32))
    m = np.full((1, 1), 1 / 2000.0 ** 2, np.float32)
    d_ref = fd.forward_model(g, m)
    with Context(g) as ctx:
        d = ctx.forward_model(T(torch, dev, m)).cpu().numpy()
    assert rel(d, d_ref) <= 1e-6


def test_checkpointed_gradient_is_bitwise_store_all(torch_dev):
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m = ragged_case(nshots=2, nt=200)
    d_obs = np.zeros((g.nshots, g.nt, g.nrec), np.float32)
    outs = []
    for k in (1, 7, 50, 200):
        with Context(g, ckpt_every=k) as ctx:
            grad, J = ctx.adjoint_gradient(T(torch, dev, m), T(torch, dev, d_obs))
            outs.append((grad.cpu().numpy(), float(J.item())))
    for gk, Jk in outs[1:]:
        assert np.array_equal(gk, outs[0][0])
        assert Jk == outs[0][1]


def test_repeatable_bitwise(torch_dev, c1):
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m_true, m0, d_obs = c1
    with Context(g) as ctx:
        a = ctx.adjoint_gradient(T(torch, dev, m0), T(torch, dev, d_obs))[0].cpu().numpy()
        b = ctx.adjoint_gradient(T(torch, dev, m0), T(torch, dev, d_obs))[0].cpu().numpy()
    assert np.array_equal(a, b)


def test_born_and_adjoint_parity(torch_dev):
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m = ragged_case(nshots=2, nt=250)
    r = np.random.default_rng(6)
    dm = (0.05 * m * r.standard_normal(m.shape)).astype(np.float32)
    y = r.standard_normal((g.nshots, g.nt, g.nrec)).astype(np.float32)
    dB_ref = fd.born(g, m, dm)
    img_ref = fd.born_adjoint(g, m, y)
    with Context(g) as ctx:
        dB = ctx.born(T(torch, dev, m), T(torch, dev, dm)).cpu().numpy()
        img = ctx.born_adjoint(T(torch, dev, m), T(torch, dev, y)).cpu().numpy()
    assert rel(dB, dB_ref) <= 1e-4, rel(dB, dB_ref)
    assert rel(img, img_ref) <= 1e-3, rel(img, img_ref)


def test_velocities_above_the_bound(torch_dev):
    """Cells faster than the geometry's velocity bound (m below 1/vmax_bound^2;
    a patch crossing a 64-column tile edge, a cell at three times the bound in
    the first row, one in the last column): the scheme runs them at the bound,
    so seismograms, gradient, Born data and the Born-adjoint image match the
    oracle's clamped map, the data stay finite, and gradient and image are
    exactly zero at the clamped cells, in the one- and two-step launch modes."""
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m = ragged_case(nshots=2, nt=250)
    floor = fd.model_floor(g)
    bad = m.copy()
    bad[30:33, 62:66] = np.float32(floor / 1.5 ** 2)
    bad[0, 20] = np.float32(floor / 9.0)
    bad[50, 149] = np.float32(floor / 2.0)
    _, mask = fd.effective_model(g, bad)
    assert mask.sum() == bad.size - 14
    r = np.random.default_rng(12)
    d_obs = fd.forward_model(g, m * (1 + 0.02 * r.standard_normal(m.shape))).astype(np.float32)
    d_ref = fd.forward_model(g, bad)
    J_ref, g_ref = fd.adjoint_gradient(g, bad, d_obs)
    dm = (0.05 * m * r.standard_normal(m.shape)).astype(np.float32)
    y = r.standard_normal((g.nshots, g.nt, g.nrec)).astype(np.float32)
    dB_ref = fd.born(g, bad, dm)
    img_ref = fd.born_adjoint(g, bad, y)
    for tb in (False, True):
        with Context(g, ckpt_every=40) as ctx:
            ctx.set_time_blocking(tb)
            d = ctx.forward_model(T(torch, dev, bad)).cpu().numpy()
            grad, J = ctx.adjoint_gradient(T(torch, dev, bad), T(torch, dev, d_obs))
            grad = grad.cpu().numpy()
            dB = ctx.born(T(torch, dev, bad), T(torch, dev, dm)).cpu().numpy()
            img = ctx.born_adjoint(T(torch, dev, bad), T(torch, dev, y)).cpu().numpy()
        assert np.isfinite(d).all()
        assert rel(d, d_ref) <= 1e-4, (tb, rel(d, d_ref))
        assert rel(grad, g_ref) <= 1e-3, (tb, rel(grad, g_ref))
        assert abs(float(J.item()) - J_ref) / J_ref <= 1e-3
        assert np.all(grad[mask == 0] == 0.0) and np.all(img[mask == 0] == 0.0)
        assert rel(dB, dB_ref) <= 1e-4, (tb, rel(dB, dB_ref))
        assert rel(img, img_ref) <= 1e-3, (tb, rel(img, img_ref))


def test_fp32_dot_product_tests(torch_dev, c1):
    """<L dm, y> = <dm, L^T y> and <J'(m) dm, r> = <dm, J'(m)^T r> in FP32."""
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m_true, m0, _ = c1
    r = np.random.default_rng(7)
    dm = (0.05 * m0 * r.standard_normal(m0.shape)).astype(np.float32)
    y = r.standard_normal((g.nshots, g.nt, g.nrec)).astype(np.float32)
    with Context(g) as ctx:
        Ld = ctx.born(T(torch, dev, m0), T(torch, dev, dm)).double()
        LTy = ctx.born_adjoint(T(torch, dev, m0), T(torch, dev, y)).double()
        ctx.forward_model(T(torch, dev, m0), keep_ckpt=True)
        JTy = ctx.adjoint_from_residual(T(torch, dev, y)).double()
        lhs = float((Ld.cpu() * torch.from_numpy(y).double()).sum())
        rhs = float((torch.from_numpy(dm).double() * LTy.cpu()).sum())
        rhs2 = float((torch.from_numpy(dm).double() * JTy.cpu()).sum())
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)
    assert abs(rhs2 - rhs) <= 1e-6 * abs(rhs), (rhs2, rhs)


def test_reciprocity_gpu(torch_dev):
    torch, dev = torch_dev
    from paper_2008_11778_amd import Context
    g, m = synth.small_case(nz=60, nx=90, nb=12, nt=400, nshots=1, nrec=1, f0=15.0)
    a, b = (5, 10), (40, 70)
    ga = g.replace(src_iz=np.array([a[0]], np.int32), src_ix=np.array([a[1]], np.int32),
                   rec_iz=np.array([[b[0]]], np.int32), rec_ix=np.array([[b[1]]], np.int32))
    gb = g.replace(src_iz=np.array([b[0]], np.int32), src_ix=np.array([b[1]], np.int32),
                   rec_iz=np.array([[a[0]]], np.int32), rec_ix=np.array([[a[1]]], np.int32))
    with Context(ga) as ca, Context(gb) as cb:
        da = ca.forward_model(T(torch, dev, m)).cpu().numpy()
        db = cb.forward_model(T(torch, dev, m)).cpu().numpy()
    assert rel(da, db) <= 1e-5, rel(da, db)


def test_green_function_gpu(torch_dev):
    """FP32 trace against the analytic 2D Green's function (same bound as the oracle)."""
    torch, dev = torch_dev
    import math
    from paper_2008_11778_amd import Context
    h, dt, v, f0, T_, L = 10.0, 1e-3, 2000.0, 10.0, 0.6, 1600.0
    n = int(round(L / h)) + 1
    nt = int(round(T_ / dt))
    g = synth.make_geometry(n, n, h, nt, dt, 1, f0=f0, nb=20, vref=v)
    c, off = n // 2, 30
    g = g.replace(src_iz=np.array([c], np.int32), src_ix=np.array([c], np.int32),
                  rec_iz=np.array([[c]], np.int32), rec_ix=np.array([[c + off]], np.int32))
    m = np.full((n, n), 1.0 / v ** 2, np.float32)
    with Context(g) as ctx:
        d = ctx.forward_model(T(torch, dev, m)).cpu().numpy()[0, :, 0]
    t0 = 1.5 / f0
    w = lambda t: (1 - 2 * (math.pi * f0 * (t - t0)) ** 2) * math.exp(-(math.pi * f0 * (t - t0)) ** 2)
    ref = fd.green_2d_trace((np.arange(nt) + 1) * dt, off * h, v, w)
    assert rel(d, ref) < 1e-2, rel(d, ref)


def test_aa_step_parity(torch_dev):
    torch, dev = torch_dev
    from paper_2008_11778_amd import AA
    r = np.random.default_rng(8)
    n, M = 5000, 3
    eta = 0.37
    ref = oaa.AAHistory(M, cond_max=1e5)
    aa = AA(n, M, cond_max=1e5)
    p = r.standard_normal(n).astype(np.float32)
    for k in range(7):
        g = (r.standard_normal(n) + 0.3 * k).astype(np.float32)
        pb, pt = aa.step(T(torch, dev, p), T(torch, dev, g), eta)
        pbr, ptr_, gam, mk = ref.step(p, g, eta)
        assert int(aa.mk.item()) == mk
        assert rel(pb.cpu().numpy(), pbr) <= 1e-6
        assert rel(pt.cpu().numpy(), ptr_) <= 1e-5, (k, rel(pt.cpu().numpy(), ptr_))
        if mk:
            np.testing.assert_allclose(aa.gamma.cpu().numpy()[:mk], gam, rtol=1e-6, atol=1e-9)
        p = ptr_.astype(np.float32)
    aa.close()


def test_aa_condition_guard_matches_oracle(torch_dev):
    torch, dev = torch_dev
    from paper_2008_11778_amd import AA
    r = np.random.default_rng(9)
    n, M = 3000, 5
    base = r.standard_normal(n)
    ref = oaa.AAHistory(M, cond_max=1e5)
    aa = AA(n, M, cond_max=1e5)
    p = np.zeros(n, np.float32)
    for k in range(6):
        # nearly collinear gradient differences: the guard must drop columns
        g = (base * (1 + k) + (1e-7 if k % 2 else 1e-2) * r.standard_normal(n)).astype(np.float32)
        pb, pt = aa.step(T(torch, dev, p), T(torch, dev, g), 0.1)
        _, ptr_, _, mk = ref.step(p, g, 0.1)
        assert int(aa.mk.item()) == mk, (k, int(aa.mk.item()), mk)
        assert rel(pt.cpu().numpy(), ptr_) <= 1e-4, (k, rel(pt.cpu().numpy(), ptr_))
        p = (p + 0.01).astype(np.float32)
    aa.close()


def test_blend_and_dots(torch_dev):
    torch, dev = torch_dev
    from paper_2008_11778_amd import Reducer, blend
    r = np.random.default_rng(10)
    n = 100003
    a, b, c = (r.standard_normal(n).astype(np.float32) for _ in range(3))
    red = Reducer()
    out = blend(0.25, T(torch, dev, a), T(torch, dev, b)).cpu().numpy()
    np.testing.assert_allclose(out, 0.25 * a.astype(np.float64) + 0.75 * b, rtol=1e-6, atol=1e-7)
    d1 = float(red.dot(T(torch, dev, a), T(torch, dev, b)).item())
    d2 = float(red.dot_diff(T(torch, dev, a), T(torch, dev, b), T(torch, dev, c)).item())
    assert abs(d1 - float(np.dot(a.astype(np.float64), b))) <= 1e-12 * n
    assert abs(d2 - float(np.dot(a.astype(np.float64), b.astype(np.float64) - c))) <= 1e-12 * n


def test_invalid_arguments_raise(torch_dev):
    torch, dev = torch_dev
    from paper_2008_11778_amd import AafwiError, Context
    g, m = synth.small_case()
    with pytest.raises(AafwiError) as e:
        Context(g.replace(dt=0.01))  # CFL violation
    assert e.value.code == -2
    with Context(g) as ctx:
        with pytest.raises(AafwiError) as e:
            ctx.adjoint_from_residual(torch.zeros(ctx.data_shape, device=dev))
        assert e.value.code == -6
        with pytest.raises(ValueError):
            ctx.forward_model(torch.zeros(3, device=dev))
        bad = T(torch, dev, m).clone()
        bad[0, 0] = -1.0
        ctx.forward_model(bad)
        with pytest.raises(AafwiError) as e:
            ctx.sync()
        assert e.value.code == -5


def test_batched_aa_step_matches_oracle_and_single_steps(torch_dev):
    """The batched Anderson step over three instances of different sizes
    (n = 700, 5000, 12345; M = 4, two of the instances with nearly collinear
    gradients so that the condition guard drops columns): every instance's
    gamma, window size, p_bar and p_tilde against the oracle's AAHistory of
    that instance at the tolerances of the single step, and bitwise against
    separate single-instance steps; one instance is masked for one step
    (left untouched) and one is reset midway."""
    torch, dev = torch_dev
    from paper_2008_11778_amd import AA, BatchAA
    r = np.random.default_rng(12)
    ns, M, etas = [700, 5000, 12345], 4, [0.37, 0.1, 0.05]
    refs = [oaa.AAHistory(M, cond_max=1e5) for _ in ns]
    singles = [AA(n, M, cond_max=1e5) for n in ns]
    batch = BatchAA(ns, M, cond_max=1e5)
    base = [r.standard_normal(n) for n in ns]
    ps = [r.standard_normal(n).astype(np.float32) for n in ns]
    pb_b = [torch.empty(n, device=dev) for n in ns]
    pt_b = [torch.empty(n, device=dev) for n in ns]
    for k in range(8):
        gs = []
        for i, n in enumerate(ns):
            if i == 0:
                g = r.standard_normal(n) + 0.3 * k
            else:  # nearly collinear differences on the larger instances
                g = base[i] * (1 + k) + (1e-7 if (k + i) % 2 else 1e-2) * r.standard_normal(n)
            gs.append(g.astype(np.float32))
        active = [True, k != 3, True]
        if k == 5:
            batch.reset([False, False, True])
            singles[2].reset()
            refs[2].reset()
        pt_in = [T(torch, dev, p) for p in ps]
        gt_in = [T(torch, dev, g) for g in gs]
        batch.step(pt_in, gt_in, etas, pb_b, pt_b, active=active)
        gam_b, mk_b = batch.state()
        gam_b, mk_b = gam_b.cpu().numpy(), mk_b.cpu().numpy()
        for i in range(len(ns)):
            if not active[i]:
                continue
            pb_s, pt_s = singles[i].step(pt_in[i], gt_in[i], etas[i])
            pbr, ptr_, gam, mk = refs[i].step(ps[i], gs[i], etas[i])
            assert int(mk_b[i]) == mk == int(singles[i].mk.item()), (k, i)
            assert torch.equal(pb_b[i], pb_s) and torch.equal(pt_b[i], pt_s), (k, i)
            if mk:
                assert np.array_equal(gam_b[i, :mk], singles[i].gamma.cpu().numpy()[:mk]), (k, i)
            assert rel(pb_b[i].cpu().numpy(), pbr) <= 1e-6
            tol = 1e-5 if i == 0 else 1e-4
            assert rel(pt_b[i].cpu().numpy(), ptr_) <= tol, (k, i, rel(pt_b[i].cpu().numpy(), ptr_))
            ps[i] = (ptr_ if i == 0 else ps[i] + 0.01).astype(np.float32)
    batch.close()
    for a in singles:
        a.close()
