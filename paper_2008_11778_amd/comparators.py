"""Comparator optimisers of the paper's Section "Discussions", on the HIP path.

* Restarted GMRES(M) for the LSRTM normal equations L^T L x = L^T d_r
  (eq. LSRTM2, eq. LSRTM3): Arnoldi with modified Gram-Schmidt, Givens
  rotations, restart from the last iterate every M steps (the restart rule
  of the GMRES subsection).  One L^T L product (a Born run and a Born-adjoint
  run) per inner step; dot products in FP64 on the device; the small
  Hessenberg least-squares problem on the host in FP64.
* L-BFGS with the two-loop recursion, H0 = (s^T y / y^T y) I from the newest
  pair, and a strong-Wolfe line search (bracketing and bisection zoom).  The
  paper's secant equation is garbled; the textbook inverse secant condition
  H_k y_k = s_k is used (p_{k+1} = p_k - alpha H_k grad J(p_k)).
* Steepest descent with a fixed step is ``inversion.aa_descent(..., M=0)``.

Every vector operation runs in libaafwi.so (blend, axpy, FP64 dots).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from ._lib import Reducer, axpy, blend, scale


def _copy(x, out):
    return blend(1.0, x, x, out)


def _scale_into(a, x, out):
    """out = a * x."""
    return scale(a, x, out)


def power_iteration(normal_op, n, device, iters=5, seed=0):
    """Largest eigenvalue estimate of an SPD operator by power iteration
    (Rayleigh quotient of the last iterate)."""
    red = Reducer()
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn(n, generator=g, dtype=torch.float32).to(device)
    w = torch.empty_like(v)
    rho = 0.0
    for _ in range(iters):
        nv = math.sqrt(float(red.dot(v, v).item()))
        _scale_into(1.0 / nv, v, v)
        normal_op(v, w)
        rho = float(red.dot(v, w).item())
        v, w = w, v
    return rho


def gmres_restarted(normal_op, b, x0, M, n_iter, callback=None):
    """GMRES(M) on A x = b with A = normal_op; returns the iterates after
    every inner step (n_iter of them; one operator application each)."""
    red = Reducer()
    n = b.numel()
    x = x0.clone().reshape(-1)
    b = b.reshape(-1)
    xs = []
    w = torch.empty_like(x)
    while len(xs) < n_iter:
        m = min(M, n_iter - len(xs))
        normal_op(x, w)
        r0 = torch.empty_like(x)
        blend(0.0, w, b, r0)          # r0 = b
        axpy(-1.0, w, r0)             # r0 = b - A x
        beta = math.sqrt(float(red.dot(r0, r0).item()))
        if beta == 0.0:
            xs.append(x.clone())
            break
        V = [_scale_into(1.0 / beta, r0, torch.empty_like(x))]
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        e = np.zeros(m + 1)
        e[0] = beta
        x_start = x.clone()
        done = False
        for j in range(m):
            normal_op(V[j], w)
            for i in range(j + 1):
                H[i, j] = float(red.dot(w, V[i]).item())
                axpy(-H[i, j], V[i], w)
            hj = math.sqrt(float(red.dot(w, w).item()))
            H[j + 1, j] = hj
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            e[j + 1] = -sn[j] * e[j]
            e[j] = cs[j] * e[j]
            y = np.linalg.solve(np.triu(H[:j + 1, :j + 1]), e[:j + 1])
            xj = x_start.clone()
            for i in range(j + 1):
                axpy(float(y[i]), V[i], xj)
            xs.append(xj)
            if callback:
                callback(len(xs), abs(e[j + 1]))
            if hj == 0.0:
                done = True
                break
            V.append(_scale_into(1.0 / hj, w, torch.empty_like(x)))
        x = xs[-1]
        if done:
            break
    return xs


# ----------------------------------------------------------------------------
# L-BFGS
# ----------------------------------------------------------------------------

def two_loop(g, S, Y, red=None):
    """H_k g by the two-loop recursion (device vectors, FP64 dots)."""
    red = red or Reducer()
    q = g.clone()
    k = len(S)
    rho = [1.0 / float(red.dot(Y[i], S[i]).item()) for i in range(k)]
    a = [0.0] * k
    for i in range(k - 1, -1, -1):
        a[i] = rho[i] * float(red.dot(S[i], q).item())
        axpy(-a[i], Y[i], q)
    gamma0 = float(red.dot(S[-1], Y[-1]).item() / red.dot(Y[-1], Y[-1]).item()) if k else 1.0
    r = _scale_into(gamma0, q, torch.empty_like(q))
    for i in range(k):
        bcoef = rho[i] * float(red.dot(Y[i], r).item())
        axpy(a[i] - bcoef, S[i], r)
    return r


def _zoom(phi, dphi, a_lo, a_hi, f_lo, f0, d0, c1, c2, max_iter=12):
    a = a_lo
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


def strong_wolfe(phi, dphi, f0, d0, a1=1.0, c1=1e-4, c2=0.9, a_max=16.0, max_iter=8):
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


class LBFGS:
    """L-BFGS(M) on a problem with ``gradient(p, g) -> J`` (flat device vectors).

    The first direction is scaled so its largest entry equals ``first_step``
    times the largest entry of p (the analogue of the fixed-step rule)."""

    def __init__(self, problem, p0, M, first_step=0.02):
        self.problem, self.M, self.first_step = problem, M, first_step
        self.red = Reducer()
        self.p = p0.detach().clone().reshape(-1)
        self.g = torch.empty_like(self.p)
        self.J = problem.gradient(self.p, self.g)
        self.S, self.Y = [], []
        self.k = 0
        self.n_evals = 1

    def iterate(self):
        red = self.red
        if self.S:
            d = two_loop(self.g, self.S, self.Y, red)
            _scale_into(-1.0, d, d)
            a1 = 1.0
        else:
            d = _scale_into(-1.0, self.g, torch.empty_like(self.g))
            a1 = self.first_step * float(self.p.abs().max().item()) / float(d.abs().max().item())
        d0 = float(red.dot(self.g, d).item())
        cache = {}

        def ev(a):
            if a not in cache:
                # a fresh tensor per trial point: the problem tracks its kept
                # forward run by tensor identity
                trial = _copy(self.p, torch.empty_like(self.p))
                axpy(a, d, trial)
                gt = torch.empty_like(self.p)
                Ja = self.problem.gradient(trial, gt)
                self.n_evals += 1
                cache[a] = (Ja, float(red.dot(gt, d).item()), trial, gt)
            return cache[a]

        a = strong_wolfe(lambda a: ev(a)[0], lambda a: ev(a)[1], self.J, d0, a1=a1)
        Jn, dn0, pn, gn = ev(a)
        # the accepted step: J and the directional derivative at both ends
        self.last_step = {"alpha": a, "J0": self.J, "d0": d0, "J": Jn, "slope": dn0, "c2": 0.9}
        s = torch.empty_like(self.p)
        blend(1.0, pn, pn, s)
        axpy(-1.0, self.p, s)
        y = torch.empty_like(self.p)
        blend(1.0, gn, gn, y)
        axpy(-1.0, self.g, y)
        ys = float(red.dot(y, s).item())
        if ys > 1e-10 * math.sqrt(float(red.dot(s, s).item()) * float(red.dot(y, y).item())):
            self.S.append(s)
            self.Y.append(y)
            if len(self.S) > self.M:
                self.S.pop(0)
                self.Y.pop(0)
        self.p, self.g, self.J = pn, gn, Jn
        self.k += 1
        return Jn


# ----------------------------------------------------------------------------
# nonlinear conjugate gradients
# ----------------------------------------------------------------------------

class NCG:
    """Polak-Ribiere+ nonlinear CG on a problem with ``gradient(p, g) -> J``.

    beta = max(0, g_{k+1}.(g_{k+1} - g_k) / g_k.g_k), d_{k+1} = -g_{k+1} + beta d_k,
    restarted with -g_{k+1} when not a descent direction; strong-Wolfe steps
    (c1 = 1e-4, c2 = 0.1) started at alpha_{k-1} g_{k-1}.d_{k-1} / g_k.d_k.
    The first step is scaled so that its largest entry is ``first_step``
    times the largest entry of p (the analogue of the fixed-step rule)."""

    def __init__(self, problem, p0, first_step=0.02, c2=0.1):
        self.problem, self.first_step, self.c2 = problem, first_step, c2
        self.red = Reducer()
        self.p = p0.detach().clone().reshape(-1)
        self.g = torch.empty_like(self.p)
        self.J = problem.gradient(self.p, self.g)
        self.d = _scale_into(-1.0, self.g, torch.empty_like(self.g))
        self.a_init = self.first_step * float(self.p.abs().max().item()) / float(self.d.abs().max().item())
        self.k = 0
        self.n_evals = 1

    def iterate(self):
        red, d = self.red, self.d
        d0 = float(red.dot(self.g, d).item())
        cache = {}

        def ev(a):
            if a not in cache:
                trial = _copy(self.p, torch.empty_like(self.p))
                axpy(a, d, trial)
                gt = torch.empty_like(self.p)
                Ja = self.problem.gradient(trial, gt)
                self.n_evals += 1
                cache[a] = (Ja, float(red.dot(gt, d).item()), trial, gt)
            return cache[a]

        a = strong_wolfe(lambda a: ev(a)[0], lambda a: ev(a)[1], self.J, d0, a1=self.a_init, c2=self.c2)
        Jn, dn0, pn, gn = ev(a)
        self.last_step = {"alpha": a, "J0": self.J, "d0": d0, "J": Jn, "slope": dn0, "c2": self.c2}
        gg = float(red.dot(self.g, self.g).item())
        beta = max(0.0, float(red.dot_diff(gn, gn, self.g).item()) / gg)
        dn = _scale_into(beta, d, torch.empty_like(d))
        axpy(-1.0, gn, dn)
        gd = float(red.dot(gn, dn).item())
        if gd >= 0.0:
            _scale_into(-1.0, gn, dn)
            gd = float(red.dot(gn, dn).item())
        self.a_init = a * d0 / gd
        self.p, self.g, self.d, self.J = pn, gn, dn, Jn
        self.k += 1
        return Jn
