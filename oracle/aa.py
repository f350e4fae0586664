"""FP64 oracle for Anderson acceleration (Section "Anderson acceleration" and
Section "Method").  TEST INFRASTRUCTURE ONLY.

* Algorithm 1, alpha form: min ||F_k alpha|| subject to sum(alpha) = 1
  (eq. AAopt), update with damping beta (eq. AAupdate0).
* gamma form: gamma = argmin ||A_k gamma - f_k|| with A_k the consecutive
  residual differences (eq. Ak, eq. AAopt2, eq. solveGamma) and, for
  beta = 1, p_{k+1} = G(p_k) - sum_i gamma_i [G(p_{i+1}) - G(p_i)]
  (eq. AA2_update).
* For steepest descent G(p) = p - eta grad J(p) (eq. GD) the residual is
  f_k = -eta grad J(p_k).
* Damping beta (eq. AAupdate0) in the gamma form: with xbar = p_k - sum_i
  gamma_i (p_{i+1} - p_i) and fbar = f_k - sum_i gamma_i (f_{i+1} - f_i)
  (that is, sum alpha_i p_i and sum alpha_i f_i), p_{k+1} = xbar + beta fbar.
* A weighted l2 norm in the least-squares problem (the norm is left open
  where eq. AAopt is stated): min ||W^(1/2) (A_k gamma - f_k)|| for positive
  per-entry weights w; the drop rule then uses cond_2(W^(1/2) A_k).
* Algorithm 2: pbar = G(p_k), ptilde from the gamma form, and the new
  iterate lambda ptilde + (1 - lambda) pbar with lambda from a backtracking
  test on J.

Readings taken where the paper leaves a choice (each listed in the design
notes): the least-squares solve here is numpy's SVD-based lstsq on A_k
itself; columns are dropped oldest first while cond_2(A_k) exceeds
``cond_max``; lambda is tried in {1, 1/2, 1/4, 1/8} with the Armijo test
J(p) <= J(p_k) + c1 <g_k, p - p_k>, falling back to lambda = 0 untested;
when such a fallback step then turns out to have decreased J, the window is
cleared and mixing restarts from it (a restart safeguard in the manner of
damped AA with restarts, Henderson and Varadhan 2019; the paper leaves the
fallback's effect on the window open).
"""
from __future__ import annotations

import numpy as np

COND_MAX = 1e5
LAMBDAS = (1.0, 0.5, 0.25, 0.125)
ARMIJO_C1 = 1e-4


# ----------------------------------------------------------------------------
# Algorithm 1 (generic fixed-point form)
# ----------------------------------------------------------------------------

def alpha_weights(F: np.ndarray) -> np.ndarray:
    """argmin ||F alpha||_2 subject to sum(alpha) = 1, via the KKT system."""
    k = F.shape[1]
    kkt = np.zeros((k + 1, k + 1))
    kkt[:k, :k] = 2.0 * F.T @ F
    kkt[:k, k] = 1.0
    kkt[k, :k] = 1.0
    rhs = np.zeros(k + 1)
    rhs[k] = 1.0
    sol = np.linalg.lstsq(kkt, rhs, rcond=None)[0]
    return sol[:k]


def alpha_update(P: np.ndarray, GP: np.ndarray, alpha: np.ndarray, beta: float = 1.0):
    """(1 - beta) sum alpha_i p_i + beta sum alpha_i G(p_i)."""
    return (1.0 - beta) * (P @ alpha) + beta * (GP @ alpha)


def gamma_weights(A: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Minimum-norm least-squares gamma = argmin ||A gamma - f||_2."""
    if A.shape[1] == 0:
        return np.zeros(0)
    return np.linalg.lstsq(A, f, rcond=None)[0]


def gamma_to_alpha(gamma: np.ndarray) -> np.ndarray:
    """The change of variables gamma_i = alpha_0 + ... + alpha_i, inverted."""
    mk = gamma.shape[0]
    alpha = np.zeros(mk + 1)
    prev = 0.0
    for i in range(mk):
        alpha[i] = gamma[i] - prev
        prev = gamma[i]
    alpha[mk] = 1.0 - prev
    return alpha


def anderson_alg1(G, p0, M, iters, beta=1.0):
    """Algorithm 1 with the alpha form; returns the iterate list p_0..p_iters."""
    ps = [np.asarray(p0, np.float64)]
    gs = [G(ps[0])]
    ps.append(gs[0].copy())
    for k in range(1, iters):
        gs.append(G(ps[k]))
        mk = min(M, k)
        P = np.stack(ps[k - mk:k + 1], axis=1)
        GP = np.stack(gs[k - mk:k + 1], axis=1)
        alpha = alpha_weights(GP - P)
        ps.append(alpha_update(P, GP, alpha, beta))
    return ps


# ----------------------------------------------------------------------------
# gamma form with an explicit history window (what the GPU step computes)
# ----------------------------------------------------------------------------

class AAHistory:
    """Window of the most recent accepted iterates p_i and gradients g_i.

    ``step`` appends (p_k, g_k) and returns pbar = G(p_k), ptilde
    (eq. AA2_update), gamma and M_k.  The window holds at most M+1 entries;
    while cond_2(A_k) > cond_max the oldest entry is dropped for good.
    """

    def __init__(self, M: int, cond_max: float = COND_MAX, beta: float = 1.0, weights=None):
        self.M = M
        self.cond_max = cond_max
        self.beta = float(beta)
        self.sw = None if weights is None else np.sqrt(np.asarray(weights, np.float64).ravel())
        self.p = []
        self.g = []

    def reset(self):
        self.p.clear()
        self.g.clear()

    def _matrices(self, eta):
        f = [-eta * g for g in self.g]
        Gp = [p + fi for p, fi in zip(self.p, f)]
        A = np.stack([f[i + 1] - f[i] for i in range(len(f) - 1)], axis=1) \
            if len(f) > 1 else np.zeros((f[0].size, 0))
        dG = np.stack([Gp[i + 1] - Gp[i] for i in range(len(Gp) - 1)], axis=1) \
            if len(Gp) > 1 else np.zeros((Gp[0].size, 0))
        return f, Gp, A, dG

    def step(self, p_k, g_k, eta):
        self.p.append(np.asarray(p_k, np.float64).ravel().copy())
        self.g.append(np.asarray(g_k, np.float64).ravel().copy())
        while len(self.p) > self.M + 1:
            self.p.pop(0)
            self.g.pop(0)
        eta = float(eta)
        while True:
            f, Gp, A, dG = self._matrices(eta)
            if A.shape[1] == 0:
                break
            Aw = A if self.sw is None else self.sw[:, None] * A
            sv = np.linalg.svd(Aw, compute_uv=False)
            cond = np.inf if sv[-1] <= 0.0 else sv[0] / sv[-1]
            if cond <= self.cond_max:
                break
            self.p.pop(0)
            self.g.pop(0)
        if self.sw is None:
            gamma = gamma_weights(A, f[-1])
        else:
            gamma = gamma_weights(self.sw[:, None] * A, self.sw * f[-1])
        pbar = Gp[-1]
        if self.beta == 1.0:
            ptilde = pbar - dG @ gamma if gamma.size else pbar.copy()
        else:
            dP = np.stack([self.p[i + 1] - self.p[i] for i in range(len(self.p) - 1)], axis=1) \
                if len(self.p) > 1 else np.zeros((pbar.size, 0))
            xbar = self.p[-1] - dP @ gamma if gamma.size else self.p[-1].copy()
            fbar = f[-1] - A @ gamma if gamma.size else f[-1].copy()
            ptilde = xbar + self.beta * fbar
        return pbar, ptilde, gamma, A.shape[1]


def multisecant_matrix(P: np.ndarray, D: np.ndarray) -> np.ndarray:
    """S = argmin ||S + I||_F subject to S D = P (eq. aaFnorm, eq. multisecant):
    S = -I + (P + D)(D^T D)^{-1} D^T."""
    n = P.shape[0]
    return -np.eye(n) + (P + D) @ np.linalg.solve(D.T @ D, D.T)


# ----------------------------------------------------------------------------
# Algorithm 2 driver
# ----------------------------------------------------------------------------

def project(p, floor):
    """Keep an iterate in the model's stable domain: max(p, floor) (no-op
    when floor is None)."""
    return p if floor is None else np.maximum(p, floor)


def alg2(grad_fn, misfit_fn, p0, eta, M, iters, cond_max=COND_MAX, lambdas=LAMBDAS,
         c1=ARMIJO_C1, linesearch=True, beta=1.0, weights=None, restart=True, floor=None):
    """Run Algorithm 2 for ``iters`` AA iterations after p_1 = G(p_0).

    grad_fn(p) -> (J, g); misfit_fn(p) -> J.  Returns a dict with the
    accepted iterates, misfits, chosen lambdas and evaluation counts.
    With ``restart``, when the search of iteration k fell back to
    lambda = 0 and that plain descent step decreased the misfit
    (J(p_{k+1}) < J(p_k), known from the gradient evaluation at p_{k+1}),
    the window is cleared before p_{k+1} enters it: Anderson mixing
    restarts from the descent step (M_k counts the iterations since the
    restart).  A descent step that did not decrease J keeps the window.
    With ``floor`` (the smallest model value the forward scheme is stable
    for), pbar = G(p_k) and ptilde are projected onto p >= floor before the
    search; every blend of the two is then in the domain too.
    """
    hist = AAHistory(M, cond_max, beta, weights)
    p = np.asarray(p0, np.float64).ravel().copy()
    J0, g0 = grad_fn(p)
    g0 = np.asarray(g0, np.float64).ravel()
    hist.step(p, g0, eta)
    iterates, misfits, lams, gammas = [p.copy()], [J0], [], []
    n_grad, n_fwd = 1, 0
    p = project(p - eta * g0, floor)
    iterates.append(p.copy())
    fell_back = False
    restarts = []  # iterations k whose window was cleared before p_k entered
    for _ in range(iters):
        J, g = grad_fn(p)
        g = np.asarray(g, np.float64).ravel()
        n_grad += 1
        if restart and fell_back and J < misfits[-1]:
            hist.reset()
            restarts.append(len(misfits))
        misfits.append(J)
        pbar, ptilde, gamma, mk = hist.step(p, g, eta)
        pbar, ptilde = project(pbar, floor), project(ptilde, floor)
        gammas.append(gamma)
        lam_acc = 0.0
        new = pbar
        if linesearch:
            for lam in lambdas:
                trial = lam * ptilde + (1.0 - lam) * pbar
                Jt = misfit_fn(trial)
                n_fwd += 1
                if Jt <= J + c1 * float(np.dot(g, trial - p)):
                    lam_acc, new = lam, trial
                    break
        else:
            lam_acc, new = 1.0, ptilde
        lams.append(lam_acc)
        fell_back = linesearch and lam_acc == 0.0
        p = new.copy()
        iterates.append(p.copy())
    return dict(iterates=iterates, misfits=misfits, lambdas=lams, gammas=gammas,
                n_grad=n_grad, n_fwd=n_fwd, restarts=restarts)


def learned_alg2(grad_fn, misfit_fn, dir_fn, p0, eta, eta_theta, M, iters, cond_max=COND_MAX,
                 lambdas=LAMBDAS, c1=ARMIJO_C1, restart=True, floor=None):
    """Algorithm 2 on the learned map G_theta(p) = p - eta_theta d(p), with
    d = dir_fn(g, p) the network's direction at p (its gradient g), and
    plain Anderson acceleration on G(p) = p - eta g as the fallback.

    Both windows are fed at every iteration: (p_k, d_k) for G_theta and
    (p_k, g_k) for G.  Step 4 backtracks over ``lambdas`` between
    ptilde_theta and pbar_theta with the sufficient-decrease test on the true
    gradient, J(p) <= J(p_k) + c1 <g_k, p - p_k>.  When no lambda passes,
    pbar_theta is taken if J(pbar_theta) < J(p_k) (one more forward run);
    otherwise the iteration is redone on the plain window (the fallback):
    the same backtracking between its ptilde and pbar, and its pbar if no
    lambda passes.  A window whose search ended on its pbar restarts at the
    next iteration if that iteration's J is below the previous one (as in
    ``alg2``).  With ``floor``, every pbar and ptilde is projected onto
    p >= floor (as in ``alg2``).  Returns the accepted iterates, misfits,
    directions d_k, lambdas, fallback flags and evaluation counts."""
    h_t = AAHistory(M, cond_max)
    h_p = AAHistory(M, cond_max)
    p = np.asarray(p0, np.float64).ravel().copy()
    J, g = grad_fn(p)
    g = np.asarray(g, np.float64).ravel()
    d = np.asarray(dir_fn(g, p), np.float64).ravel()
    iterates, misfits, dirs, lams, fallbacks = [p.copy()], [J], [d], [], []
    n_grad, n_fwd = 1, 0
    pbar_t = project(h_t.step(p, d, eta_theta)[0], floor)
    h_p.step(p, g, eta)
    p = pbar_t.copy()
    iterates.append(p.copy())
    fb_t = fb_p = False

    def search(ptilde, pbar, J, g, p):
        nonlocal n_fwd
        for lam in lambdas:
            trial = lam * ptilde + (1.0 - lam) * pbar
            n_fwd += 1
            if misfit_fn(trial) <= J + c1 * float(np.dot(g, trial - p)):
                return lam, trial
        return 0.0, None

    for _ in range(iters):
        J, g = grad_fn(p)
        g = np.asarray(g, np.float64).ravel()
        n_grad += 1
        if restart and J < misfits[-1]:
            if fb_t:
                h_t.reset()
            if fb_p:
                h_p.reset()
        misfits.append(J)
        d = np.asarray(dir_fn(g, p), np.float64).ravel()
        dirs.append(d)
        pbar_t, ptilde_t, _, _ = h_t.step(p, d, eta_theta)
        pbar_p, ptilde_p, _, _ = h_p.step(p, g, eta)
        pbar_t, ptilde_t = project(pbar_t, floor), project(ptilde_t, floor)
        pbar_p, ptilde_p = project(pbar_p, floor), project(ptilde_p, floor)
        fb_t = fb_p = False
        fell = False
        lam, new = search(ptilde_t, pbar_t, J, g, p)
        if new is None:
            fb_t = True
            n_fwd += 1
            if misfit_fn(pbar_t) < J:
                new = pbar_t
            else:
                fell = True
                lam, new = search(ptilde_p, pbar_p, J, g, p)
                if new is None:
                    fb_p = True
                    new = pbar_p
        lams.append(lam)
        fallbacks.append(fell)
        p = new.copy()
        iterates.append(p.copy())
    return dict(iterates=iterates, misfits=misfits, dirs=dirs, lambdas=lams, fallbacks=fallbacks,
                n_grad=n_grad, n_fwd=n_fwd)


def picard(grad_fn, p0, eta, iters):
    """Steepest descent with a fixed step = AA with M = 0."""
    p = np.asarray(p0, np.float64).ravel().copy()
    out = [p.copy()]
    for _ in range(iters):
        _, g = grad_fn(p)
        p = p - eta * np.asarray(g, np.float64).ravel()
        out.append(p.copy())
    return out
