"""Pins for the oracle's Algorithm 2 on the learned map (learned_alg2):

* a constant gate reduces it to plain Algorithm 2: with d = c g and
  eta_theta = eta / c, G_theta is G, so the iterates, misfits and lambdas
  are those of ``alg2`` (itself pinned by hand in test_oracle_linesearch);
* hand-worked one-dimensional cases of the two branches taken when the
  learned search fails: pbar_theta accepted because it decreases J, and the
  fallback to plain Anderson acceleration."""
import numpy as np

from oracle import aa, fd
import synth


def _quad():
    """J(p) = 1/2 sum p^2, g = p."""
    calls = []

    def grad(p):
        p = np.asarray(p, np.float64)
        return 0.5 * float(np.dot(p, p)), p.copy()

    def misfit(p):
        p = np.asarray(p, np.float64)
        calls.append(p.copy())
        return 0.5 * float(np.dot(p, p))

    return grad, misfit, calls


def test_constant_gate_reduces_to_plain_algorithm2():
    g, m = synth.small_case(nz=12, nx=14, nb=6, nt=90, nshots=1, nrec=6, f0=30.0)
    r = np.random.default_rng(5)
    mt = (m.astype(np.float64) * (1 + 0.04 * r.standard_normal(m.shape))).astype(np.float32)
    d_obs = fd.forward_model(g, mt).astype(np.float32)
    shape = m.shape
    grad_fn = lambda p: fd.adjoint_gradient(g, p.reshape(shape), d_obs)
    mis_fn = lambda p: fd.misfit(fd.forward_model(g, p.reshape(shape)), d_obs)
    _, g0 = grad_fn(m.ravel())
    eta = float(0.02 * np.abs(m).max() / np.abs(g0).max())
    c = np.log(2.0)
    ref = aa.alg2(grad_fn, mis_fn, m.ravel(), eta, 3, 3)
    got = aa.learned_alg2(grad_fn, mis_fn, lambda gg, p: c * gg, m.ravel(), eta, eta / c, 3, 3)
    assert got["lambdas"] == ref["lambdas"]
    assert got["fallbacks"] == [False] * 3
    for a, b in zip(got["iterates"], ref["iterates"]):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())
    np.testing.assert_allclose(got["misfits"], ref["misfits"], rtol=1e-12)


def test_fallback_to_plain_aa_hand_worked():
    """J = p^2 / 2 in one variable, eta = 1/2, d = 10 g, eta_theta = 1/2,
    M = 0 (no mixing), lambda in {1}.  G_theta(p) = -4 p, G(p) = p / 2.
    p_0 = 1, p_1 = G_theta(p_0) = -4 (J = 8).  Iteration 1: pbar_theta = 16,
    J = 128 fails the test and is not below 8, so the iteration falls back:
    pbar = -2, J = 2 <= 8 + 1e-4 (-4)(2), lambda = 1, p_2 = -2.
    Iteration 2 likewise: pbar_theta = 8 (J = 32), fallback, p_3 = -1.
    Three forward runs per iteration (learned trial, pbar_theta, plain
    trial)."""
    grad, misfit, calls = _quad()
    res = aa.learned_alg2(grad, misfit, lambda g, p: 10.0 * g, np.array([1.0]), 0.5, 0.5, 0, 2, lambdas=(1.0,))
    assert [float(x[0]) for x in res["iterates"]] == [1.0, -4.0, -2.0, -1.0]
    assert res["lambdas"] == [1.0, 1.0]
    assert res["fallbacks"] == [True, True]
    assert res["misfits"] == [0.5, 8.0, 2.0]
    assert [float(x[0]) for x in calls] == [16.0, 16.0, -2.0, 8.0, 8.0, -1.0]
    assert res["n_fwd"] == 6 and res["n_grad"] == 3


def test_pbar_theta_taken_when_it_decreases_J():
    """J = p^2 / 2, d = g, eta_theta = 1.9, M = 0, c1 = 0.9, lambda in {1}:
    G_theta(p) = -0.9 p.  p_1 = -0.9 (J = 0.405).  Iteration 1: the trial
    pbar_theta = 0.81 has J = 0.32805, above the bound
    0.405 + 0.9 (-0.9)(0.81 + 0.9) = -0.9801, so the search fails; but
    J(pbar_theta) < J(p_1), so p_2 = pbar_theta with lambda = 0 and no
    fallback; two forward runs."""
    grad, misfit, calls = _quad()
    res = aa.learned_alg2(grad, misfit, lambda g, p: g, np.array([1.0]), 0.5, 1.9, 0, 1, lambdas=(1.0,), c1=0.9)
    np.testing.assert_allclose([float(x[0]) for x in res["iterates"]], [1.0, -0.9, 0.81], rtol=1e-14)
    assert res["lambdas"] == [0.0]
    assert res["fallbacks"] == [False]
    np.testing.assert_allclose([float(x[0]) for x in calls], [0.81, 0.81], rtol=1e-14)
    assert res["n_fwd"] == 2
