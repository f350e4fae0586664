"""Pins for the decisions the oracle takes in its line searches.

Algorithm 2, Step 4 (Section "Method"): lambda is backtracked over
{1, 1/2, 1/4, 1/8}; the first lambda whose blend
p(lambda) = lambda ptilde + (1 - lambda) pbar satisfies
J(p(lambda)) <= J(p_k) + c1 <g_k, p(lambda) - p_k> is taken, otherwise
lambda = 0 (pbar).  The cases below are worked by hand on a convex,
piecewise-quadratic J of one variable, so every expected number is exact in
binary floating point and every decision is fixed by the numbers written in
the docstrings, not by re-running the oracle's formula.

The comparators' strong-Wolfe search (Section "Discussions": L-BFGS and
nonlinear CG) is pinned by hand-worked bracketing/zoom sequences and by
checking both Wolfe conditions on every step that the L-BFGS and nCG
drivers accept.
"""
import numpy as np
import pytest

from oracle import aa, krylov


def _kinked(K, c=0.5):
    """J(p) = 1/2 + (p - 1) + (c/2)(p - 1)^2 for p > 1 and
    1/2 + (p - 1) + (K/2)(p - 1)^2 for p <= 1: C^1 and convex, with gradient
    1 + c (p - 1) on the right and 1 + K (p - 1) on the left.  Steepest
    descent from p > 1 sees only the gentle slope c, so the secant step of
    Anderson mixing lands far on the steep side."""
    def J(p):
        x = float(np.asarray(p).ravel()[0]) - 1.0
        k = c if x > 0 else K
        return 0.5 + x + 0.5 * k * x * x

    def grad(p):
        x = float(np.asarray(p).ravel()[0]) - 1.0
        k = c if x > 0 else K
        return J(p), np.array([1.0 + k * x])

    return J, grad


def _run(K, c1, iters=1, M=1, restart=True):
    J, grad = _kinked(K)
    calls = []

    def misfit(p):
        calls.append(float(np.asarray(p).ravel()[0]))
        return J(p)

    res = aa.alg2(grad, misfit, np.array([3.0]), 0.5, M=M, iters=iters, c1=c1, restart=restart)
    return res, calls


# Shared hand computation (eta = 1/2, p_0 = 3, c = 1/2):
#   g_0 = 1 + 0.5*2 = 2, p_1 = G(p_0) = 3 - 1 = 2, g_1 = 1.5, J(p_1) = 1.75
#   f_0 = -1, f_1 = -0.75, A_1 = f_1 - f_0 = 0.25, gamma = f_1 / A_1 = -3
#   G(p_0) = 2, G(p_1) = 1.25, dG = -0.75
#   ptilde = G(p_1) - dG gamma = 1.25 - 2.25 = -1, pbar = 1.25
#   p(lambda) = 1.25 - 2.25 lambda: 1 -> -1, 1/2 -> 0.125, 1/4 -> 0.6875,
#   1/8 -> 0.96875.


def test_step4_backtracks_to_a_quarter():
    """K = 8, c1 = 1e-4.
    J(-1) = 0.5 - 2 + 4*4 = 14.5 and J(0.125) = 0.5 - 0.875 + 4*0.765625 =
    2.6875 both exceed the bound 1.75 + 1e-4*1.5*(p - 2) (about 1.7497);
    J(0.6875) = 0.5 - 0.3125 + 4*0.09765625 = 0.578125 passes.
    A slip that compares against J(p_0) = 3.5 instead of J(p_1) would take
    lambda = 1/2 (2.6875 < 3.5); testing ptilde instead of p(lambda) would
    fail every trial (14.5) and fall back to lambda = 0."""
    res, calls = _run(K=8.0, c1=1e-4)
    assert res["lambdas"] == [0.25]
    np.testing.assert_allclose(calls, [-1.0, 0.125, 0.6875], rtol=1e-14)   # trial points, in order
    assert res["n_fwd"] == 3 and res["n_grad"] == 2
    assert res["misfits"] == [3.5, 1.75]
    np.testing.assert_allclose(res["gammas"][0], [-3.0], rtol=1e-14)
    assert res["iterates"][1][0] == 2.0
    np.testing.assert_allclose(res["iterates"][2], [0.6875], rtol=1e-14)


def test_step4_sign_of_the_sufficient_decrease_term():
    """K = 8 with a wide band, c1 = 1/2: the bound is 1.75 + 0.75 (p - 2).
    lambda = 1/2: bound 1.75 - 1.40625 = 0.34375 < J = 2.6875, rejected;
    lambda = 1/4: bound 1.75 - 0.984375 = 0.765625 >= J = 0.578125, taken.
    With the c1 term's sign flipped the bound at lambda = 1/2 would be
    3.15625 >= 2.6875 and lambda = 1/2 would be taken."""
    res, calls = _run(K=8.0, c1=0.5)
    assert res["lambdas"] == [0.25]
    np.testing.assert_allclose(calls, [-1.0, 0.125, 0.6875], rtol=1e-14)
    np.testing.assert_allclose(res["iterates"][2], [0.6875], rtol=1e-14)


def test_step4_falls_back_to_pbar_without_a_test():
    """K = 4096: every blend lands on the steep side and fails
    (J(0.96875) = 0.46875 + 2048/1024 = 2.46875 > 1.7497 is the smallest),
    so lambda = 0 and p_2 = pbar = 1.25, with four trial runs and no run at
    pbar itself."""
    res, calls = _run(K=4096.0, c1=1e-4)
    assert res["lambdas"] == [0.0]
    np.testing.assert_allclose(calls, [-1.0, 0.125, 0.6875, 0.96875], rtol=1e-14)
    assert res["n_fwd"] == 4
    np.testing.assert_allclose(res["iterates"][2], [1.25], rtol=1e-14)


def test_window_holds_the_accepted_iterate():
    """Second iteration of the K = 8 case with M = 1: the window is
    (p_1, p_2) = (2, 0.6875), the accepted blend, not ptilde or pbar.
    g_2 = 1 + 8*(-0.3125) = -1.5, f_2 = 0.75, f_1 = -0.75, A_2 = 1.5,
    gamma = 0.5; G(p_1) = 1.25, G(p_2) = 1.4375, dG = 0.1875,
    ptilde = 1.4375 - 0.09375 = 1.34375, pbar = 1.4375.
    J(p_2) = 0.578125 and every blend lies right of the kink with
    J >= 0.5 + 0.34375 + 0.25*0.3437^2 > 0.578, so lambda = 0 and
    p_3 = 1.4375."""
    res, calls = _run(K=8.0, c1=1e-4, iters=2)
    assert res["lambdas"] == [0.25, 0.0]
    np.testing.assert_allclose(res["gammas"][1], [0.5], rtol=1e-14)
    np.testing.assert_allclose(calls[3:], [1.34375, 1.390625, 1.4140625, 1.42578125], rtol=1e-14)
    np.testing.assert_allclose(res["iterates"][3], [1.4375], rtol=1e-14)
    np.testing.assert_allclose(res["misfits"][2], 0.578125, rtol=1e-14)


def test_window_length_is_min_of_M_and_k():
    """M_k = min(M, k): with M = 1 the second iteration uses one column
    (above); with M = 2 it uses both differences.  On the K = 8 case the
    window (p_0, p_1, p_2) gives A = [f_1 - f_0, f_2 - f_1] = [0.25, 1.5] in
    one dimension, a single row, so the minimum-norm gamma is
    f_2 [0.25, 1.5] / (0.25^2 + 1.5^2) = 0.75 [0.25, 1.5] / 2.3125."""
    res, _ = _run(K=8.0, c1=1e-4, iters=2, M=2)
    np.testing.assert_allclose(res["gammas"][1], 0.75 * np.array([0.25, 1.5]) / 2.3125, rtol=1e-14)


def test_restart_after_a_fallback_that_decreased_J():
    """K = 4096, three iterations.  Iteration 1 falls back to p_2 = pbar =
    1.25 (above).  At p_2: g_2 = 1 + 0.5*0.25 = 1.125 and J(p_2) = 0.5 +
    0.25 + 0.25*0.0625 = 0.765625 < J(p_1) = 1.75, so the fallback step
    decreased J and the window restarts from p_2: no difference column,
    gamma empty, ptilde = pbar = G(p_2) = 1.25 - 0.5625 = 0.6875, and all
    four trials sit at 0.6875, where J = 0.5 - 0.3125 + 2048*0.09765625 =
    200.1875 fails; p_3 = 0.6875.  At p_3: g_3 = 1 + 4096*(-0.3125) = -1279
    and J(p_3) = 200.1875 > J(p_2), so this fallback keeps the window
    (p_2, p_3): f_2 = -0.5625, f_3 = 639.5, A = 640.0625 and
    gamma = 639.5 / 640.0625.
    Without the restart, iteration 2 would use the window (p_1, p_2):
    A = -0.5625 + 0.75 = 0.1875, gamma = -3, ptilde = 0.6875 - (-0.5625)(-3)
    = -1, so its first trial would be at -1."""
    res, calls = _run(K=4096.0, c1=1e-4, iters=3)
    assert res["lambdas"] == [0.0, 0.0, res["lambdas"][2]]
    assert res["restarts"] == [2]
    assert res["gammas"][1].size == 0
    np.testing.assert_allclose(calls[4:8], [0.6875] * 4, rtol=1e-14)
    np.testing.assert_allclose(res["iterates"][3], [0.6875], rtol=1e-14)
    np.testing.assert_allclose(res["misfits"][2:4], [0.765625, 200.1875], rtol=1e-14)
    np.testing.assert_allclose(res["gammas"][2], [639.5 / 640.0625], rtol=1e-14)
    res0, calls0 = _run(K=4096.0, c1=1e-4, iters=2, restart=False)
    assert res0["restarts"] == []
    np.testing.assert_allclose(res0["gammas"][1], [-3.0], rtol=1e-14)
    assert calls0[4] == -1.0


def test_no_restart_without_a_fallback():
    """The K = 8 case accepts lambda = 1/4 in iteration 1 (no fallback), so
    iteration 2 keeps the window (p_1, p_2) whatever the misfits do:
    gamma = 0.5 as worked above."""
    res, _ = _run(K=8.0, c1=1e-4, iters=2)
    assert res["restarts"] == []
    np.testing.assert_allclose(res["gammas"][1], [0.5], rtol=1e-14)


# ----------------------------------------------------------------------------
# strong-Wolfe search
# ----------------------------------------------------------------------------

def _quad_phi(a0, shift):
    """phi(a) = (a - a0)^2 - shift, phi(0) = a0^2 - shift, phi'(a) = 2 (a - a0)."""
    return (lambda a: (a - a0) ** 2 - shift), (lambda a: 2.0 * (a - a0))


def test_strong_wolfe_accepts_first_trial_inside_the_interval():
    """phi(a) = (a - 2)^2 - 4: phi(0) = 0, phi'(0) = -4.  At a = 1:
    phi = -3 <= -4e-4 and |phi'| = 2 <= 0.9*4 = 3.6, so a = 1."""
    phi, dphi = _quad_phi(2.0, 4.0)
    assert krylov.strong_wolfe(phi, dphi, 0.0, -4.0) == 1.0


def test_strong_wolfe_zoom_sequence_c2_09():
    """phi(a) = (a - 0.1)^2 - 0.01: phi(0) = 0, phi'(0) = -0.2.
    The sufficient-decrease bound is c1 a phi'(0) = -2e-5 a.
    a = 1: phi = 0.8 > bound, zoom on [0, 1]; 0.5: 0.15 > bound, hi = 0.5;
    0.25: 0.0125 > bound, hi = 0.25; 0.125: -0.009375 passes, phi' = 0.05
    and 0.05 <= 0.9*0.2: a = 0.125."""
    phi, dphi = _quad_phi(0.1, 0.01)
    a = krylov.strong_wolfe(phi, dphi, 0.0, -0.2)
    assert a == 0.125


def test_strong_wolfe_zoom_sequence_c2_01():
    """The same phi with c2 = 0.1 (the nCG setting): at 0.125, |phi'| = 0.05 >
    0.02 and phi' (hi - lo) >= 0, so hi = 0, lo = 0.125; 0.0625: -0.00859375
    >= f_lo = -0.009375, hi = 0.0625; 0.09375: -0.0099609375 < f_lo, phi' =
    -0.0125 and 0.0125 <= 0.02: a = 0.09375."""
    phi, dphi = _quad_phi(0.1, 0.01)
    a = krylov.strong_wolfe(phi, dphi, 0.0, -0.2, c2=0.1)
    assert a == 0.09375


def test_strong_wolfe_expands_until_the_curvature_test_passes():
    """phi(a) = (a - 5)^2 - 25: phi'(0) = -10.  At a = 1, |phi'| = 8 <= 0.9*10,
    so c2 = 0.9 takes a = 1.  With c2 = 0.5: 8 > 5, a -> 2: |phi'| = 6 > 5,
    a -> 4: |phi'| = 2 passes (phi(4) = -24 <= bound): a = 4."""
    phi, dphi = _quad_phi(5.0, 25.0)
    assert krylov.strong_wolfe(phi, dphi, 0.0, -10.0) == 1.0
    assert krylov.strong_wolfe(phi, dphi, 0.0, -10.0, c2=0.5) == 4.0


def _recording(monkeypatch, c2_expected):
    """Wrap krylov.strong_wolfe so that every step it returns is checked for
    both strong-Wolfe conditions: phi(a) <= phi(0) + c1 a phi'(0) and
    |phi'(a)| <= c2 |phi'(0)|."""
    seen = []
    inner = krylov.strong_wolfe

    def wrapped(phi, dphi, f0, d0, a1=1.0, c1=1e-4, c2=0.9, **kw):
        assert c2 == c2_expected
        a = inner(phi, dphi, f0, d0, a1=a1, c1=c1, c2=c2, **kw)
        seen.append((phi(a), dphi(a), f0, d0, a, c1, c2))
        return a

    monkeypatch.setattr(krylov, "strong_wolfe", wrapped)
    return seen


def _assert_wolfe(seen):
    assert seen
    for fa, da, f0, d0, a, c1, c2 in seen:
        assert d0 < 0.0
        assert fa <= f0 + c1 * a * d0
        assert abs(da) <= c2 * abs(d0)


def _nonquadratic(n, seed, spread):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1.0, spread, n)) @ Q.T
    b = r.standard_normal(n)
    return lambda x: (0.5 * x @ A @ x - b @ x + 0.05 * np.sum(x ** 4), A @ x - b + 0.2 * x ** 3)


def test_lbfgs_steps_satisfy_strong_wolfe(monkeypatch):
    seen = _recording(monkeypatch, 0.9)
    fg = _nonquadratic(20, 51, 100.0)
    xs = krylov.lbfgs(fg, np.zeros(20), M=5, iters=25)
    assert len(seen) == 25
    _assert_wolfe(seen)
    assert np.linalg.norm(fg(xs[-1])[1]) < 1e-3 * np.linalg.norm(fg(xs[0])[1])


def test_ncg_steps_satisfy_strong_wolfe(monkeypatch):
    seen = _recording(monkeypatch, 0.1)
    fg = _nonquadratic(25, 52, 20.0)
    xs = krylov.ncg(fg, np.zeros(25), 25)
    assert len(seen) == 25
    _assert_wolfe(seen)
    assert np.linalg.norm(fg(xs[-1])[1]) < 1e-3 * np.linalg.norm(fg(xs[0])[1])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lbfgs_on_rosenbrock_steps_satisfy_strong_wolfe(monkeypatch, seed):
    """A non-convex test function: every accepted step still meets both
    conditions (the search's bracketing guarantees it where it terminates
    normally)."""
    seen = _recording(monkeypatch, 0.9)

    def fg(x):
        a, b = x[:-1], x[1:]
        J = float(np.sum(100.0 * (b - a * a) ** 2 + (1.0 - a) ** 2))
        g = np.zeros_like(x)
        g[:-1] += -400.0 * a * (b - a * a) - 2.0 * (1.0 - a)
        g[1:] += 200.0 * (b - a * a)
        return J, g

    x0 = np.random.default_rng(seed).uniform(-1.2, 1.2, 6)
    krylov.lbfgs(fg, x0, M=5, iters=20)
    _assert_wolfe(seen)
