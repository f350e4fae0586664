"""Pins for the FP64 oracle of the discretised acoustic problem.

Each test ties the oracle to something other than itself: Taylor
conditions of the stencil, the exact discrete dispersion relation, the
analytic 2D Green's function, symmetry of the discrete operator
(reciprocity, dot-product tests), central finite differences, the Born
Taylor remainder and the conserved discrete energy.
"""
import math

import numpy as np

import synth
from oracle import fd


def _taylor_weights():
    """Weights c0..c4 of the centred second difference exact on polynomials of
    degree <= 9: sum over the stencil of c_j j^(2p) = (2p)! [p == 1]."""
    M = np.zeros((5, 5))
    rhs = np.zeros(5)
    for p in range(5):
        M[p, 0] = 1.0 if p == 0 else 0.0
        for j in range(1, 5):
            M[p, j] = 2.0 * float(j) ** (2 * p)
        rhs[p] = 2.0 if p == 1 else 0.0
    return np.linalg.solve(M, rhs)


def test_stencil_weights_are_the_8th_order_taylor_weights():
    np.testing.assert_allclose(fd.C8, _taylor_weights(), rtol=1e-13, atol=1e-15)
    # consistency: weights sum to zero and the Nyquist symbol is the known one
    w = _taylor_weights()
    assert abs(w[0] + 2 * w[1:].sum()) < 1e-14
    nyq = w[0] + 2 * sum(w[j] * math.cos(j * math.pi) for j in range(1, 5))
    assert abs(nyq - (-6.501587301587302)) < 1e-12


def test_sponge_profile_closed_form():
    xi = fd.sponge_xi(10, 4)
    np.testing.assert_allclose(xi[:4], [1.0, 0.75, 0.5, 0.25])
    np.testing.assert_allclose(xi[4:14], 0.0)
    np.testing.assert_allclose(xi[14:], [0.25, 0.5, 0.75, 1.0])
    g, _ = synth.small_case()
    A, B = fd.sponge(g)
    # interior is undamped; B = 2A - 1 everywhere
    nb = g.nb
    np.testing.assert_allclose(A[nb:-nb, nb:-nb], 1.0)
    np.testing.assert_allclose(B, 2 * A - 1, atol=1e-15)
    smax = 3 * g.vref * math.log(1 / g.refl) / (2 * nb * g.h)
    st = smax * 2.0 * g.dt / 2  # corner: xi_x = xi_z = 1
    assert abs(A[0, 0] - 1 / (1 + st)) < 1e-15


def test_fold_is_adjoint_of_pad():
    r = np.random.default_rng(0)
    m = r.standard_normal((7, 9))
    gp = r.standard_normal((7 + 6, 9 + 6))
    lhs = float(np.sum(fd.pad_model(m, 3) * gp))
    rhs = float(np.sum(m * fd.fold(gp, 7, 9, 3)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_discrete_dispersion_relation_periodic():
    """u^0 = phi, u^-1 = cos(w dt) phi on a periodic undamped grid stays
    cos(w n dt) phi, with 2(1 - cos w dt) = -(v dt/h)^2 [S(kx h) + S(kz h)]."""
    nz, nx, h, dt, v = 30, 40, 10.0, 1e-3, 2500.0
    g = synth.make_geometry(nz, nx, h, 60, dt, 1, nb=4, refl=1.0, vref=v)
    nzp, nxp = g.nz_p, g.nx_p
    kz, kx = 2 * math.pi * 3 / (nzp * h), 2 * math.pi * 5 / (nxp * h)
    zz = np.arange(nzp)[:, None] * h
    xx = np.arange(nxp)[None, :] * h
    phi = np.cos(kz * zz) * np.cos(kx * xx)
    w8 = _taylor_weights()
    S = lambda th: w8[0] + 2 * sum(w8[j] * math.cos(j * th) for j in range(1, 5))
    c = 1 + 0.5 * (v * dt / h) ** 2 * (S(kx * h) + S(kz * h))
    om = math.acos(c) / dt
    m = np.full((nz, nx), 1.0 / v ** 2)
    _, _, (u, _) = fd.forward_shot(g, m, 0, periodic=True, u_init=(phi, math.cos(om * dt) * phi),
                                   src_on=False)
    np.testing.assert_allclose(u, math.cos(om * g.nt * dt) * phi, atol=1e-11)


def _green_error(h, dt, r=300.0, v=2000.0, f0=10.0, T=0.6, L=1600.0):
    n = int(round(L / h)) + 1
    nt = int(round(T / dt))
    g = synth.make_geometry(n, n, h, nt, dt, 1, f0=f0, nb=20, vref=v)
    c = n // 2
    off = int(round(r / h))
    g = g.replace(src_iz=np.array([c], np.int32), src_ix=np.array([c], np.int32),
                  rec_iz=np.array([[c]], np.int32), rec_ix=np.array([[c + off]], np.int32))
    m = np.full((n, n), 1.0 / v ** 2)
    d = fd.forward_shot(g, m, 0)[0][:, 0]
    t0 = 1.5 / f0
    w = lambda t: (1 - 2 * (math.pi * f0 * (t - t0)) ** 2) * math.exp(-(math.pi * f0 * (t - t0)) ** 2)
    ref = fd.green_2d_trace((np.arange(nt) + 1) * dt, off * h, v, w)
    return np.linalg.norm(d - ref) / np.linalg.norm(ref)


def test_green_function_2d_homogeneous():
    e_fine = _green_error(10.0, 1e-3)
    e_coarse = _green_error(20.0, 2e-3)
    assert e_fine < 1e-2, e_fine
    assert e_fine < e_coarse, (e_fine, e_coarse)


def test_reciprocity():
    g, m = synth.small_case(nt=120)
    a, b = (3, 5), (15, 20)
    ga = g.replace(src_iz=np.array([a[0]], np.int32), src_ix=np.array([a[1]], np.int32),
                   rec_iz=np.array([[b[0]]], np.int32), rec_ix=np.array([[b[1]]], np.int32))
    gb = g.replace(src_iz=np.array([b[0]], np.int32), src_ix=np.array([b[1]], np.int32),
                   rec_iz=np.array([[a[0]]], np.int32), rec_ix=np.array([[a[1]]], np.int32))
    da = fd.forward_shot(ga, m, 0)[0]
    db = fd.forward_shot(gb, m, 0)[0]
    assert np.linalg.norm(da - db) <= 1e-12 * np.linalg.norm(da)


def test_dot_product_source_to_data():
    g, m = synth.small_case(nt=80)
    r = np.random.default_rng(1)
    src = r.standard_normal((g.nt, g.nz_p, g.nx_p))
    y = r.standard_normal((g.nt, g.nrec))
    lhs = float(np.sum(fd.source_to_data(g, m, src) * y))
    rhs = float(np.sum(src * fd.data_to_source(g, m, y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_dot_product_born():
    g, m = synth.small_case(nt=100)
    r = np.random.default_rng(2)
    dm = r.standard_normal(m.shape) * 0.05 * m
    y = r.standard_normal((g.nshots, g.nt, g.nrec))
    lhs = float(np.sum(fd.born(g, m, dm) * y))
    rhs = float(np.sum(dm * fd.born_adjoint(g, m, y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # L^T L is symmetric (it is the LSRTM normal operator)
    x1 = r.standard_normal(m.shape) * m
    x2 = r.standard_normal(m.shape) * m
    a = float(np.sum(fd.born_adjoint(g, m, fd.born(g, m, x1)) * x2))
    b = float(np.sum(x1 * fd.born_adjoint(g, m, fd.born(g, m, x2))))
    assert abs(a - b) <= 1e-11 * abs(a)


def test_gradient_matches_central_differences():
    g, m = synth.small_case(nt=150)
    m = m.astype(np.float64)
    r = np.random.default_rng(3)
    m_true = m * (1 + 0.03 * r.standard_normal(m.shape))
    d_obs = fd.forward_model(g, m_true)
    J, grad = fd.adjoint_gradient(g, m, d_obs)
    dm = r.standard_normal(m.shape) * m  # whole interior, edges included (exercises P^T)
    exact = float(np.sum(grad * dm))
    errs = []
    for eps in (1e-4, 1e-5):
        jp = fd.misfit(fd.forward_model(g, m + eps * dm), d_obs)
        jm = fd.misfit(fd.forward_model(g, m - eps * dm), d_obs)
        errs.append(abs((jp - jm) / (2 * eps) - exact) / abs(exact))
    assert errs[1] < 1e-7, errs
    assert errs[1] < errs[0] / 50, errs  # second order in eps


def test_born_is_the_jacobian():
    g, m = synth.small_case(nt=120)
    m = m.astype(np.float64)
    r = np.random.default_rng(4)
    dm = r.standard_normal(m.shape) * m
    F0 = fd.forward_model(g, m)
    Ld = fd.born(g, m, dm)
    rem = []
    for eps in (1e-2, 5e-3):
        rem.append(np.linalg.norm(fd.forward_model(g, m + eps * dm) - F0 - eps * Ld))
    ratio = rem[0] / rem[1]
    assert 3.6 < ratio < 4.4, ratio  # O(eps^2) remainder


def test_energy_conserved_without_sponge_and_source():
    g = synth.make_geometry(24, 30, 10.0, 200, 1e-3, 1, nb=4, refl=1.0, vref=2500.0)
    r = np.random.default_rng(5)
    v = 2000 + 500 * r.random((24, 30))
    m = 1.0 / v ** 2
    m_pad = fd.pad_model(m, g.nb)
    from scipy.ndimage import gaussian_filter
    u0 = gaussian_filter(r.standard_normal((g.nz_p, g.nx_p)), 2.0)
    um = gaussian_filter(r.standard_normal((g.nz_p, g.nx_p)), 2.0) * 0.1 + 0.9 * u0
    E0 = fd.energy(u0, um, m_pad, g.h, g.dt)
    u, up = u0, um
    for k in (50, 100, 150):
        gk = g.replace(nt=k)
        _, _, (u, up) = fd.forward_shot(gk, m, 0, u_init=(u0, um), src_on=False)
        assert abs(fd.energy(u, up, m_pad, g.h, g.dt) - E0) <= 1e-10 * abs(E0)


def test_energy_decays_with_sponge_after_source():
    g, m = synth.small_case(nt=400)
    m_pad = fd.pad_model(m, g.nb)
    es = []
    for k in (250, 300, 350, 400):
        _, _, (u, up) = fd.forward_shot(g.replace(nt=k), m, 0)
        es.append(fd.energy(u, up, m_pad, g.h, g.dt))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(es, es[1:])), es


def test_rtm_filter_is_exact_on_quadratics():
    """-Lap of x^2 + 3 z^2 is -8 away from the image edge (the 8th-order
    second differences are exact on polynomials of low degree)."""
    h = 12.5
    z = np.arange(30)[:, None] * h
    x = np.arange(40)[None, :] * h
    f = fd.rtm_filter(x * x + 3.0 * z * z, h)
    np.testing.assert_allclose(f[4:-4, 4:-4], -8.0, rtol=1e-9)
    # at the edge the zero extension shows: the first row differs
    assert abs(f[0, 20] + 8.0) > 1.0


def test_scaled_rtm_start_minimises_the_data_misfit():
    g, m = synth.small_case(nz=20, nx=26, nb=6, nt=120, nshots=2, nrec=8, instance=7)
    dm = np.zeros(m.shape)
    dm[10, 5:20] = 0.05 * m[10, 5:20]
    d_r = fd.born(g, m, dm)
    x0, alpha = fd.scaled_rtm_start(g, m, d_r)
    J = lambda a: float(np.sum((fd.born(g, m, x0 * (a / alpha)) - d_r) ** 2))
    assert alpha > 0 and J(alpha) < J(alpha * 1.01) and J(alpha) < J(alpha * 0.99)
    assert J(alpha) < float(np.sum(d_r ** 2))


def _above_bound_model(instance=0):
    """The small case with a few cells whose velocity exceeds the geometry's
    bound vmax_bound (m below the floor 1/vmax_bound^2): a 2x2 patch at 1.4
    times the bound, one edge cell at 3 times it."""
    g, m = synth.small_case(nt=120, instance=instance)
    m = m.astype(np.float64)
    floor = fd.model_floor(g)
    bad = m.copy()
    bad[8:10, 11:13] = floor / 1.4 ** 2
    bad[0, 5] = floor / 9.0
    return g, m, bad, floor


def test_model_floor_is_the_velocity_bound():
    g, _, bad, floor = _above_bound_model()
    assert floor == 1.0 / g.vmax_bound ** 2
    m_eff, mask = fd.effective_model(g, bad)
    assert np.array_equal(m_eff, np.maximum(bad, floor))
    assert mask.sum() == bad.size - 5 and mask[0, 5] == 0 and mask[8, 11] == 0


def test_velocities_above_the_bound_are_seen_at_the_bound():
    """The scheme runs on m_eff: data are bitwise those of the model clamped
    by hand, and stay bounded (the cell at three times the CFL velocity would
    otherwise grow without limit)."""
    g, m, bad, floor = _above_bound_model()
    d_bad = fd.forward_model(g, bad)
    assert np.array_equal(d_bad, fd.forward_model(g, np.maximum(bad, floor)))
    assert np.isfinite(d_bad).all()
    assert np.abs(d_bad).max() < 10.0 * np.abs(fd.forward_model(g, m)).max()


def test_gradient_is_zero_where_the_floor_is_taken_and_exact_elsewhere():
    """Central differences of J(m_eff(m)) along a direction that moves both
    clamped cells (which stay below the floor) and free cells match <g, dm>:
    a gradient without the mask would count the clamped cells, on which J
    does not depend."""
    g, m, bad, floor = _above_bound_model()
    r = np.random.default_rng(5)
    d_obs = fd.forward_model(g, m * (1 + 0.03 * r.standard_normal(m.shape)))
    J, grad = fd.adjoint_gradient(g, bad, d_obs)
    _, mask = fd.effective_model(g, bad)
    assert np.all(grad[mask == 0] == 0.0) and np.abs(grad[mask == 1]).max() > 0
    # just above the floor the same cells carry a gradient: the mask is what zeroes it
    _, grad_up = fd.adjoint_gradient(g, np.where(mask == 0, floor * 1.01, bad), d_obs)
    assert np.all(grad_up[mask == 0] != 0.0)
    dm = r.standard_normal(m.shape) * m
    exact = float(np.sum(grad * dm))
    errs = []
    for eps in (1e-4, 1e-5):
        # clamped cells sit at most at floor / 1.96; eps * |dm| keeps them below the floor
        jp = fd.misfit(fd.forward_model(g, bad + eps * dm), d_obs)
        jm = fd.misfit(fd.forward_model(g, bad - eps * dm), d_obs)
        errs.append(abs((jp - jm) / (2 * eps) - exact) / abs(exact))
    assert errs[1] < 1e-7, errs
    assert errs[1] < errs[0] / 50, errs


def test_born_linearises_the_clamped_map():
    """Born modelling at a background with clamped cells ignores dm there (J
    does not move with them), is the Jacobian of the clamped forward map, and
    its adjoint passes the dot test."""
    g, m, bad, floor = _above_bound_model(instance=1)
    _, mask = fd.effective_model(g, bad)
    r = np.random.default_rng(6)
    only_clamped = np.where(mask == 0, r.standard_normal(m.shape) * floor, 0.0)
    assert np.all(fd.born(g, bad, only_clamped) == 0.0)
    dm = r.standard_normal(m.shape) * m
    F0 = fd.forward_model(g, bad)
    Ld = fd.born(g, bad, dm)
    rem = [np.linalg.norm(fd.forward_model(g, bad + eps * dm * mask) - F0 - eps * Ld) for eps in (1e-2, 5e-3)]
    assert 3.6 < rem[0] / rem[1] < 4.4, rem
    y = r.standard_normal((g.nshots, g.nt, g.nrec))
    lhs = float(np.sum(Ld * y))
    rhs = float(np.sum(dm * fd.born_adjoint(g, bad, y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
