"""FP64 oracle for the comparators of Section "Discussions": restarted
GMRES (eq. Krylov, eq. GMRES and the restart rule) and L-BFGS.
TEST INFRASTRUCTURE ONLY.

The paper's secant and L-BFGS update equations are garbled in the source
text; the reading taken is the textbook one: the inverse secant condition
B_k y_k = s_k with s_k = p_k - p_{k-1}, y_k = grad J(p_k) - grad J(p_{k-1}),
and p_{k+1} = p_k - alpha_k B_k grad J(p_k).
"""
from __future__ import annotations

import numpy as np


def gmres_cycle(apply_A, b, x0, m):
    """One GMRES cycle of at most m Arnoldi steps (modified Gram-Schmidt,
    Givens rotations).  Returns the iterates x_1..x_j after each inner step."""
    x0 = np.asarray(x0, np.float64)
    r0 = b - apply_A(x0)
    beta = np.linalg.norm(r0)
    if beta == 0.0:
        return [x0.copy()]
    V = [r0 / beta]
    H = np.zeros((m + 1, m))
    cs, sn = np.zeros(m), np.zeros(m)
    e1 = np.zeros(m + 1)
    e1[0] = beta
    out = []
    for j in range(m):
        w = apply_A(V[j])
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        rho = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
        H[j, j] = rho
        H[j + 1, j] = 0.0
        e1[j + 1] = -sn[j] * e1[j]
        e1[j] = cs[j] * e1[j]
        y = np.linalg.solve(np.triu(H[:j + 1, :j + 1]), e1[:j + 1])
        x = x0 + np.stack(V[:j + 1], axis=1) @ y
        out.append(x)
        hj = np.linalg.norm(w)
        if hj == 0.0:
            break
        V.append(w / hj)
    return out


def gmres_restarted(apply_A, b, x0, m, n_iter):
    """GMRES(m): restart from the last iterate every m inner steps; returns the
    n_iter iterates produced (one per operator application)."""
    xs = []
    x = np.asarray(x0, np.float64)
    while len(xs) < n_iter:
        cyc = gmres_cycle(apply_A, b, x, min(m, n_iter - len(xs)))
        xs.extend(cyc)
        x = cyc[-1]
        if len(cyc) < min(m, n_iter - len(xs) + len(cyc)):
            break
    return xs[:n_iter]


def krylov_ls(A, b, x0, k):
    """Definition of the k-th GMRES iterate: argmin over x0 + K_k(A, r0) of
    ||A x - b||_2, with an explicit (orthonormalised) Krylov basis."""
    r0 = b - A @ x0
    cols = [r0]
    for _ in range(k - 1):
        cols.append(A @ cols[-1])
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    y = np.linalg.lstsq(A @ Q, b - A @ x0, rcond=None)[0]
    return x0 + Q @ y


# ----------------------------------------------------------------------------
# L-BFGS
# ----------------------------------------------------------------------------

def two_loop(g, S, Y):
    """H_k g by the two-loop recursion with H0 = (s^T y / y^T y) I (newest pair)."""
    q = np.asarray(g, np.float64).copy()
    k = len(S)
    rho = [1.0 / float(np.dot(Y[i], S[i])) for i in range(k)]
    a = np.zeros(k)
    for i in range(k - 1, -1, -1):
        a[i] = rho[i] * np.dot(S[i], q)
        q = q - a[i] * Y[i]
    gamma0 = float(np.dot(S[-1], Y[-1]) / np.dot(Y[-1], Y[-1])) if k else 1.0
    r = gamma0 * q
    for i in range(k):
        bcoef = rho[i] * np.dot(Y[i], r)
        r = r + S[i] * (a[i] - bcoef)
    return r


def dense_bfgs_inverse(S, Y, H0):
    """BFGS inverse-Hessian updates H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T."""
    H = np.array(H0, np.float64)
    n = H.shape[0]
    for s, y in zip(S, Y):
        rho = 1.0 / float(np.dot(y, s))
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def _zoom(phi, dphi, a_lo, a_hi, f_lo, f0, d0, c1, c2, max_iter=20):
    for _ in range(max_iter):
        a = 0.5 * (a_lo + a_hi)
        fa = phi(a)
        if fa > f0 + c1 * a * d0 or fa >= f_lo:
            a_hi = a
        else:
            da = dphi(a)
            if abs(da) <= -c2 * d0:
                return a
            if da * (a_hi - a_lo) >= 0:
                a_hi = a_lo
            a_lo, f_lo = a, fa
    return a_lo


def strong_wolfe(phi, dphi, f0, d0, a1=1.0, c1=1e-4, c2=0.9, a_max=16.0, max_iter=10):
    """Line search for the strong Wolfe conditions (bracketing + bisection zoom)."""
    a_prev, f_prev = 0.0, f0
    a = a1
    for i in range(max_iter):
        fa = phi(a)
        if fa > f0 + c1 * a * d0 or (i > 0 and fa >= f_prev):
            return _zoom(phi, dphi, a_prev, a, f_prev, f0, d0, c1, c2)
        da = dphi(a)
        if abs(da) <= -c2 * d0:
            return a
        if da >= 0:
            return _zoom(phi, dphi, a, a_prev, fa, f0, d0, c1, c2)
        a_prev, f_prev = a, fa
        a = min(2.0 * a, a_max)
    return a


def lbfgs(fun_grad, p0, M, iters, a1=1.0):
    """L-BFGS with the two-loop recursion and a strong-Wolfe line search.
    fun_grad(p) -> (J, g).  Pairs with y^T s <= 1e-10 |s||y| are skipped."""
    p = np.asarray(p0, np.float64).ravel().copy()
    J, g = fun_grad(p)
    g = np.asarray(g, np.float64).ravel()
    S, Y = [], []
    out = [p.copy()]
    for _ in range(iters):
        d = -two_loop(g, S, Y) if S else -g * (a1 / max(np.linalg.norm(g), 1e-300))
        cache = {}

        def eval_at(a):
            if a not in cache:
                Ja, ga = fun_grad(p + a * d)
                cache[a] = (Ja, np.asarray(ga, np.float64).ravel())
            return cache[a]

        phi = lambda a: eval_at(a)[0]
        dphi = lambda a: float(np.dot(eval_at(a)[1], d))
        a = strong_wolfe(phi, dphi, J, float(np.dot(g, d)))
        Jn, gn = eval_at(a)
        s, y = a * d, gn - g
        if np.dot(y, s) > 1e-10 * np.linalg.norm(s) * np.linalg.norm(y):
            S.append(s)
            Y.append(y)
            if len(S) > M:
                S.pop(0)
                Y.pop(0)
        p, J, g = p + s, Jn, gn
        out.append(p.copy())
    return out


def ncg(fun_grad, p0, iters, a1=1.0, c2=0.1, line_search=None):
    """Nonlinear conjugate gradients, Polak-Ribiere+ (Nocedal & Wright,
    eq. 5.44-5.45): d_0 = -g_0, beta = max(0, g_{k+1}.(g_{k+1} - g_k) / g_k.g_k),
    d_{k+1} = -g_{k+1} + beta d_k, restarted with -g_{k+1} when that is not
    a descent direction.  Step lengths from a strong-Wolfe search
    (c1 = 1e-4, c2 = 0.1) started at a1 / |g_0| on the first iteration and at
    alpha_{k-1} g_{k-1}.d_{k-1} / g_k.d_k afterwards (N&W eq. 3.60).
    ``line_search(phi, dphi, f0, d0, a_init)`` replaces the search (tests)."""
    p = np.asarray(p0, np.float64).ravel().copy()
    J, g = fun_grad(p)
    g = np.asarray(g, np.float64).ravel()
    d = -g
    a_init = a1 / max(np.linalg.norm(g), 1e-300)
    out = [p.copy()]
    for _ in range(iters):
        cache = {}

        def eval_at(a):
            if a not in cache:
                Ja, ga = fun_grad(p + a * d)
                cache[a] = (Ja, np.asarray(ga, np.float64).ravel())
            return cache[a]

        phi = lambda a: eval_at(a)[0]
        dphi = lambda a: float(np.dot(eval_at(a)[1], d))
        d0 = float(np.dot(g, d))
        if line_search is None:
            a = strong_wolfe(phi, dphi, J, d0, a1=a_init, c2=c2)
        else:
            a = line_search(phi, dphi, J, d0, a_init)
        Jn, gn = eval_at(a)
        p = p + a * d
        beta = max(0.0, float(np.dot(gn, gn - g)) / float(np.dot(g, g)))
        dn = -gn + beta * d
        if float(np.dot(gn, dn)) >= 0.0:
            dn = -gn
        a_init = a * d0 / float(np.dot(gn, dn))
        J, g, d = Jn, gn, dn
        out.append(p.copy())
    return out
