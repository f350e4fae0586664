"""Pins for the Anderson-acceleration, GMRES and L-BFGS oracle.

Identities from the paper's Sections "Anderson acceleration" and
"Discussions" and from the literature it cites: M = 0 is Picard; the
alpha and gamma forms agree; the least-squares optimality bound; AA on a
linear fixed-point map reproduces GMRES (x^AA_{k+1} = G(x^GMRES_k), Walker
and Ni 2011, Thm 2.2); the multi-secant form; finite termination; GMRES
equals the Krylov least-squares definition; the two-loop recursion equals
dense BFGS.
"""
import numpy as np

from oracle import aa, krylov


def _lin_problem(n=8, seed=0, cond=30.0):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    Amat = Q @ np.diag(np.linspace(1.0, np.sqrt(cond), n)) @ Q.T
    b = r.standard_normal(n)
    return Amat, b


def test_m0_is_picard():
    Amat, b = _lin_problem()
    eta = 0.02
    grad = lambda p: (0.5 * np.sum((Amat @ p - b) ** 2), Amat.T @ (Amat @ p - b))
    x0 = np.zeros(8)
    res = aa.alg2(grad, lambda p: grad(p)[0], x0, eta, M=0, iters=6, linesearch=False)
    pic = aa.picard(grad, x0, eta, 7)
    for a_, b_ in zip(res["iterates"], pic):
        np.testing.assert_allclose(a_, b_, rtol=0, atol=1e-15)


def test_alpha_and_gamma_forms_agree_and_optimality():
    r = np.random.default_rng(1)
    n, mk = 50, 4
    P = r.standard_normal((n, mk + 1))
    F = r.standard_normal((n, mk + 1))
    GP = P + F
    alpha = aa.alpha_weights(F)
    assert abs(alpha.sum() - 1) < 1e-13
    A = F[:, 1:] - F[:, :-1]
    gamma = aa.gamma_weights(A, F[:, -1])
    np.testing.assert_allclose(aa.gamma_to_alpha(gamma), alpha, rtol=1e-10, atol=1e-12)
    p_alpha = aa.alpha_update(P, GP, alpha, 1.0)
    dG = GP[:, 1:] - GP[:, :-1]
    p_gamma = GP[:, -1] - dG @ gamma
    np.testing.assert_allclose(p_gamma, p_alpha, rtol=1e-11, atol=1e-12)
    # ||F alpha|| <= ||f_k|| (Picard weights are feasible)
    assert np.linalg.norm(F @ alpha) <= np.linalg.norm(F[:, -1]) + 1e-14


def test_aa_reproduces_gmres_on_linear_problem():
    """Untruncated AA on G(x) = x - eta A^T(Ax - b): x^AA_{k+1} = G(x^GMRES_k) with
    GMRES on (eta A^T A) x = eta A^T b from the same start."""
    Amat, b = _lin_problem(n=12, seed=2, cond=50.0)
    eta = 0.5 / np.linalg.norm(Amat, 2) ** 2
    N = Amat.T @ Amat
    c = Amat.T @ b
    G = lambda x: x - eta * (N @ x - c)
    x0 = np.random.default_rng(3).standard_normal(12)
    grad = lambda p: (0.0, N @ p - c)
    res = aa.alg2(grad, None, x0, eta, M=50, iters=7, cond_max=np.inf, linesearch=False)
    xs = res["iterates"]
    for k in range(1, 8):
        xg = krylov.krylov_ls(eta * N, eta * c, x0, k)
        np.testing.assert_allclose(xs[k + 1], G(xg), rtol=0, atol=1e-9 * np.linalg.norm(xg))


def test_aa_matches_restarted_gmres_cycle_by_cycle():
    """AA restarted with the GMRES cycle: each cycle of length m from the cycle's
    start point gives G(GMRES iterate)."""
    Amat, b = _lin_problem(n=10, seed=4, cond=40.0)
    eta = 0.5 / np.linalg.norm(Amat, 2) ** 2
    N, c = Amat.T @ Amat, Amat.T @ b
    G = lambda x: x - eta * (N @ x - c)
    m = 3
    gm = krylov.gmres_restarted(lambda v: eta * (N @ v), eta * c, np.zeros(10), m, 6)
    start = np.zeros(10)
    grad = lambda p: (0.0, N @ p - c)
    for cyc in range(2):
        res = aa.alg2(grad, None, start, eta, M=m, iters=m - 1, cond_max=np.inf, linesearch=False)
        for k in range(1, m):
            np.testing.assert_allclose(res["iterates"][k + 1], G(gm[cyc * m + k - 1]),
                                       atol=1e-9 * np.linalg.norm(start + 1))
        start = gm[cyc * m + m - 1]


def test_multisecant_form():
    r = np.random.default_rng(5)
    n, mk = 9, 3
    ps = [r.standard_normal(n) for _ in range(mk + 1)]
    fs = [r.standard_normal(n) for _ in range(mk + 1)]
    P = np.stack([ps[i + 1] - ps[i] for i in range(mk)], axis=1)
    D = np.stack([fs[i + 1] - fs[i] for i in range(mk)], axis=1)
    S = aa.multisecant_matrix(P, D)
    np.testing.assert_allclose(S @ D, P, atol=1e-12)
    # S is the closest to -I: any other solution of S D = P is farther
    Z = r.standard_normal((n, n))
    S2 = S + Z - Z @ D @ np.linalg.solve(D.T @ D, D.T)
    np.testing.assert_allclose(S2 @ D, P, atol=1e-10)
    assert np.linalg.norm(S + np.eye(n)) <= np.linalg.norm(S2 + np.eye(n))
    # p_k - S f_k equals the gamma-form update
    gamma = aa.gamma_weights(D, fs[-1])
    dG = P + D
    np.testing.assert_allclose(ps[-1] - S @ fs[-1], ps[-1] + fs[-1] - dG @ gamma, atol=1e-11)


def test_finite_termination():
    n = 6
    Amat, b = _lin_problem(n=n, seed=6, cond=20.0)
    eta = 0.5 / np.linalg.norm(Amat, 2) ** 2
    N, c = Amat.T @ Amat, Amat.T @ b
    grad = lambda p: (0.0, N @ p - c)
    res = aa.alg2(grad, None, np.zeros(n), eta, M=50, iters=n, cond_max=np.inf, linesearch=False)
    xstar = np.linalg.solve(N, c)
    np.testing.assert_allclose(res["iterates"][n + 1], xstar, rtol=1e-7)


def test_condition_guard_drops_oldest():
    r = np.random.default_rng(7)
    n = 40
    h = aa.AAHistory(M=5, cond_max=1e5)
    base = r.standard_normal(n)
    p = np.zeros(n)
    # gradients whose differences are nearly collinear: cond(A) explodes
    for k in range(5):
        g = base * (1 + k) + 1e-9 * r.standard_normal(n)
        pbar, ptilde, gamma, mk = h.step(p + k, g, 0.1)
    assert mk < 4
    f = [-0.1 * g for g in h.g]
    if len(f) > 1:
        A = np.stack([f[i + 1] - f[i] for i in range(len(f) - 1)], axis=1)
        assert np.linalg.cond(A) <= 1e5


def test_gmres_equals_krylov_definition():
    Amat, b = _lin_problem(n=15, seed=8, cond=100.0)
    Amat = Amat + 0.3 * np.random.default_rng(9).standard_normal((15, 15))  # nonsymmetric
    x0 = np.random.default_rng(10).standard_normal(15)
    xs = krylov.gmres_cycle(lambda v: Amat @ v, b, x0, 6)
    for k, x in enumerate(xs, start=1):
        np.testing.assert_allclose(x, krylov.krylov_ls(Amat, b, x0, k), rtol=1e-9, atol=1e-10)
    # restart: the second cycle starts from the first cycle's last iterate
    xr = krylov.gmres_restarted(lambda v: Amat @ v, b, x0, 3, 6)
    np.testing.assert_allclose(xr[4], krylov.krylov_ls(Amat, b, xr[2], 2), rtol=1e-9, atol=1e-10)


def test_two_loop_equals_dense_bfgs():
    r = np.random.default_rng(11)
    n, k = 10, 4
    Amat, _ = _lin_problem(n=n, seed=12)
    S = [r.standard_normal(n) for _ in range(k)]
    Y = [Amat @ s for s in S]  # y^T s > 0
    g = r.standard_normal(n)
    g0 = float(np.dot(S[-1], Y[-1]) / np.dot(Y[-1], Y[-1]))
    H = krylov.dense_bfgs_inverse(S, Y, g0 * np.eye(n))
    np.testing.assert_allclose(krylov.two_loop(g, S, Y), H @ g, rtol=1e-11, atol=1e-12)
    # inverse secant condition for the newest pair
    np.testing.assert_allclose(H @ Y[-1], S[-1], rtol=1e-10, atol=1e-12)


def test_lbfgs_converges_on_quadratic_with_monotone_misfit():
    Amat, b = _lin_problem(n=20, seed=13, cond=100.0)
    fg = lambda p: (0.5 * np.sum((Amat @ p - b) ** 2), Amat.T @ (Amat @ p - b))
    xs = krylov.lbfgs(fg, np.zeros(20), M=5, iters=60)
    xstar = np.linalg.lstsq(Amat, b, rcond=None)[0]
    assert np.linalg.norm(xs[-1] - xstar) < 1e-5 * np.linalg.norm(xstar)
    Js = [fg(x)[0] for x in xs]
    assert all(b_ <= a_ + 1e-12 for a_, b_ in zip(Js, Js[1:]))


def test_ncg_with_exact_steps_is_linear_cg():
    """On an SPD quadratic with exact line searches, Polak-Ribiere nonlinear CG
    produces the iterates of linear CG (scipy.sparse.linalg.cg)."""
    from scipy.sparse.linalg import cg
    r = np.random.default_rng(31)
    n = 30
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1.0, 50.0, n)) @ Q.T
    b = r.standard_normal(n)
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)

    def exact(phi, dphi, f0, d0, a_init):
        # phi is quadratic in a: phi'(0) = d0, phi'(1) = dphi(1); exact minimiser
        return -d0 / (dphi(1.0) - d0)

    xs = krylov.ncg(fg, np.zeros(n), 8, line_search=exact)
    ref = []
    cg(A, b, x0=np.zeros(n), rtol=1e-30, maxiter=8, callback=lambda xk: ref.append(xk.copy()))
    for k in range(8):
        np.testing.assert_allclose(xs[k + 1], ref[k], rtol=1e-8, atol=1e-10)


def test_ncg_wolfe_converges_and_descends():
    r = np.random.default_rng(32)
    n = 25
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1.0, 20.0, n)) @ Q.T
    b = r.standard_normal(n)
    fg = lambda x: (0.5 * x @ A @ x - b @ x + 0.05 * np.sum(x ** 4), A @ x - b + 0.2 * x ** 3)
    xs = krylov.ncg(fg, np.zeros(n), 60)
    J = [fg(x)[0] for x in xs]
    assert all(b2 <= a2 + 1e-12 for a2, b2 in zip(J, J[1:]))
    assert np.linalg.norm(fg(xs[-1])[1]) < 1e-6


def test_damped_gamma_form_equals_alpha_form():
    """With damping beta the gamma-form step xbar + beta fbar equals
    Algorithm 1's (1 - beta) sum alpha p + beta sum alpha G(p) (eq. AAupdate0)
    for the alpha that gamma maps to."""
    r = np.random.default_rng(41)
    n, M, eta, beta = 12, 3, 0.3, 0.45
    hist = aa.AAHistory(M, cond_max=1e12, beta=beta)
    ps = [r.standard_normal(n) for _ in range(M + 1)]
    gs = [r.standard_normal(n) for _ in range(M + 1)]
    for p, g in zip(ps, gs):
        _, pt, gamma, mk = hist.step(p, g, eta)
    alpha = aa.gamma_to_alpha(gamma)
    P = np.stack(ps, axis=1)
    GP = np.stack([p - eta * g for p, g in zip(ps, gs)], axis=1)
    np.testing.assert_allclose(alpha, aa.alpha_weights(GP - P), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(pt, aa.alpha_update(P, GP, alpha, beta), rtol=1e-12, atol=1e-12)


def test_weighted_gamma_solves_weighted_normal_equations():
    r = np.random.default_rng(42)
    n, M, eta = 40, 3, 0.2
    w = r.uniform(0.2, 3.0, n)
    ps = [r.standard_normal(n) for _ in range(M + 1)]
    gs = [r.standard_normal(n) for _ in range(M + 1)]
    hw = aa.AAHistory(M, cond_max=1e12, weights=w)
    hc = aa.AAHistory(M, cond_max=1e12, weights=np.full(n, 7.0))
    h1 = aa.AAHistory(M, cond_max=1e12)
    for p, g in zip(ps, gs):
        _, _, gw, _ = hw.step(p, g, eta)
        _, _, gc, _ = hc.step(p, g, eta)
        _, _, g1, _ = h1.step(p, g, eta)
    A = np.stack([(-eta) * (gs[i + 1] - gs[i]) for i in range(M)], axis=1)
    f = -eta * gs[-1]
    ref = np.linalg.solve(A.T @ (w[:, None] * A), A.T @ (w * f))
    np.testing.assert_allclose(gw, ref, rtol=1e-10)
    np.testing.assert_allclose(gc, g1, rtol=1e-10)   # a constant weight changes nothing
    assert np.abs(gw - g1).max() > 1e-3               # a varying one does


def test_alg2_projects_onto_the_stable_domain():
    """With a floor (the smallest model value the scheme is stable for),
    Algorithm 2 keeps every iterate at or above it.  Hand-worked: on
    J(p) = 1/2 (p + 1)^2 with floor 0, steepest descent with eta = 1/2 from
    p = 2 (M = 0, no search) goes 2 -> 0.5 -> max(-0.25, 0) = 0 -> 0;
    without the floor it goes to -0.25.  With M = 2 and the search on
    J(p) = 1/2 |p - (-1, 3)|^2 the iterates stay at or above 0 and converge
    to the constrained minimiser (0, 3)."""
    from oracle.aa import alg2
    q = lambda p: (0.5 * float(np.sum((np.asarray(p) + 1.0) ** 2)), np.asarray(p) + 1.0)
    out = alg2(q, lambda p: q(p)[0], [2.0], 0.5, M=0, iters=3, linesearch=False, floor=0.0)
    assert [float(x[0]) for x in out["iterates"]] == [2.0, 0.5, 0.0, 0.0, 0.0]
    free = alg2(q, lambda p: q(p)[0], [2.0], 0.5, M=0, iters=1, linesearch=False)
    assert float(free["iterates"][-1][0]) == -0.25
    a = np.array([-1.0, 3.0])
    f = lambda p: (0.5 * float(np.sum((np.asarray(p) - a) ** 2)), np.asarray(p) - a)
    out = alg2(f, lambda p: f(p)[0], [2.0, 0.0], 0.5, M=2, iters=12, floor=0.0)
    assert all(np.all(x >= 0.0) for x in out["iterates"])
    assert np.allclose(out["iterates"][1], [0.5, 1.5])  # G(p_0) = (0.5, 1.5), already feasible
    assert np.allclose(out["iterates"][-1], [0.0, 3.0], atol=1e-8)
    free = alg2(f, lambda p: f(p)[0], [2.0, 0.0], 0.5, M=2, iters=12)
    assert min(float(x[0]) for x in free["iterates"]) < -0.5


def test_learned_alg2_projects_both_windows():
    """The learned form with a floor: with a direction that overshoots (d = 3 g)
    the learned window's steps would leave the domain; every accepted iterate
    stays at or above the floor and the run reaches the constrained
    minimiser of J(p) = 1/2 |p - (-1, 3)|^2."""
    from oracle.aa import learned_alg2
    a = np.array([-1.0, 3.0])
    f = lambda p: (0.5 * float(np.sum((np.asarray(p) - a) ** 2)), np.asarray(p) - a)
    out = learned_alg2(f, lambda p: f(p)[0], lambda g, p: 3.0 * g, [2.0, 0.0], 0.5, 0.5, M=2, iters=15,
                       floor=0.0)
    assert all(np.all(x >= 0.0) for x in out["iterates"])
    assert np.allclose(out["iterates"][-1], [0.0, 3.0], atol=1e-6)
