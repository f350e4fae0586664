"""Algorithm 2 (l2-based Anderson acceleration for gradient descent) on the
HIP path, plus the problem wrappers it drives.

Every vector operation and every wave simulation runs in libaafwi.so; the
host only sequences the calls and reads the scalar misfits that the line
search compares (the one device-to-host synchronisation per trial).

Readings of the paper used here (Section "Method", Algorithm 2):
  * G(p) = p - eta dJ/dp with a fixed eta (eq. GD); f_k = -eta g_k.
  * p_1 = G(p_0); for k >= 1: pbar = G(p_k) (Step 1), gamma from the
    least-squares problem over the last M_k = min(M, k) differences (Step 2),
    ptilde from eq. AA2_update (Step 3), then the backtracking search over
    lambda in {1, 1/2, 1/4, 1/8} with the sufficient-decrease test
    J(p) <= J(p_k) + c1 <g_k, p - p_k> (Step 4), falling back to lambda = 0,
    and p_{k+1} = lambda ptilde + (1 - lambda) pbar (Step 5).
  * The accepted trial's forward run keeps its wavefield checkpoints, so the
    next gradient needs only the backward pass (no second forward).
  * Restart (the paper leaves the fallback's effect on the window open):
    when the search of iteration k fell back to lambda = 0 and that plain
    descent step decreased J (J(p_{k+1}) < J(p_k), known once the gradient
    at p_{k+1} is evaluated), the Anderson window is cleared before p_{k+1}
    enters it, so mixing restarts from the descent step; a descent step
    that did not decrease J keeps the window.
"""
from __future__ import annotations

import dataclasses
import json
import time

import torch

from ._lib import AA, Context, Reducer, axpy, blend, floor_, laplacian_filter, scale

LAMBDAS = (1.0, 0.5, 0.25, 0.125)
ARMIJO_C1 = 1e-4


class FWIProblem:
    """J(m) = 1/2 ||R F(m) - d_obs||^2 and its gradient on one Context."""

    def __init__(self, ctx: Context, d_obs: torch.Tensor):
        self.ctx = ctx
        self.d_obs = d_obs
        self.floor = ctx.floor  # the model's stable domain: m >= floor
        self.d = ctx._new(ctx.data_shape)
        self.r = ctx._new(ctx.data_shape)
        self.J = ctx._new((1,), torch.float64)
        self.kept = None  # the model whose forward run (and residual) is kept
        self.kept_gen = -1
        self.n_fwd = 0
        self.n_adj = 0

    def misfit_keep(self, m: torch.Tensor) -> float:
        """Forward with checkpoints kept (for the tensor object m); returns J
        (host sync)."""
        self.ctx.forward_model(m, self.d, keep_ckpt=True)
        self.ctx.residual_misfit(self.d, self.d_obs, self.r, self.J)
        self.kept, self.kept_gen = m, self.ctx.generation
        self.n_fwd += 1
        return float(self.J.item())

    def gradient(self, m: torch.Tensor, grad: torch.Tensor):
        """(J, grad) at m, reusing the kept forward run when it was at m (and
        no other run has replaced it on the Context since)."""
        if self.kept is not m or self.kept_gen != self.ctx.generation:
            self.misfit_keep(m)
        J = float(self.J.item())
        self.ctx.adjoint_from_residual(self.r, grad)
        self.n_adj += 1
        return J


class AutogradFWIProblem:
    """The same J(m) and gradient through the autograd form: f(m) is
    ``seismic_forward`` (a torch.autograd.Function over the HIP forward and
    adjoint) and J = ``misfit`` (a torch.autograd.Function over the library's
    residual kernel: r = f(m) - d_obs in FP32, J in FP64 in the same order as
    the C-ABI problem); ``J.backward()`` hands r to the adjoint.  The graph of
    the last misfit evaluation is kept, so the gradient at the accepted
    line-search trial reuses its forward run (its checkpoints)."""

    def __init__(self, ctx: Context, d_obs: torch.Tensor):
        self.ctx = ctx
        self.d_obs = d_obs
        self.floor = ctx.floor  # the model's stable domain: m >= floor
        self.kept = None
        self.kept_J = None
        self.kept_leaf = None
        self.n_fwd = 0
        self.n_adj = 0

    def misfit_keep(self, m: torch.Tensor) -> float:
        from .autograd import misfit, seismic_forward
        leaf = m.detach().view(self.ctx.nz, self.ctx.nx).requires_grad_(True)
        d = seismic_forward(leaf, self.ctx)
        J = misfit(d, self.d_obs, self.ctx)
        self.kept, self.kept_J, self.kept_leaf = m, J, leaf
        self.n_fwd += 1
        return float(J.item())

    def gradient(self, m: torch.Tensor, grad: torch.Tensor):
        if self.kept is not m:
            self.misfit_keep(m)
        J, leaf = self.kept_J, self.kept_leaf
        J.backward()
        grad.copy_(leaf.grad.reshape(grad.shape))
        self.kept, self.kept_J, self.kept_leaf = None, None, None
        self.n_adj += 1
        return float(J.item())


class LSRTMProblem:
    """J(x) = 1/2 ||L x - d_r||^2 at a fixed background m0 (eq. LSRTM)."""

    def __init__(self, ctx: Context, m0: torch.Tensor, d_r: torch.Tensor):
        self.ctx, self.m0, self.d_r = ctx, m0, d_r
        self.d = ctx._new(ctx.data_shape)
        self.r = ctx._new(ctx.data_shape)
        self.J = ctx._new((1,), torch.float64)
        self.kept = None
        self.n_fwd = 0
        self.n_adj = 0

    def misfit_keep(self, x: torch.Tensor) -> float:
        self.ctx.born(self.m0, x, self.d)
        self.ctx.residual_misfit(self.d, self.d_r, self.r, self.J)
        self.kept = x
        self.n_fwd += 1
        return float(self.J.item())

    def gradient(self, x: torch.Tensor, grad: torch.Tensor):
        if self.kept is not x:
            self.misfit_keep(x)
        J = float(self.J.item())
        self.ctx.born_adjoint(self.m0, self.r, grad)
        self.n_adj += 1
        return J

    def rtm_image(self):
        """m_RTM = L^T d_r (Section "FWI and LSRTM")."""
        img = self.ctx._new((self.ctx.nz, self.ctx.nx))
        self.ctx.born_adjoint(self.m0, self.d_r, img)
        self.kept = None
        self.n_fwd += 1
        self.n_adj += 1
        return img

    def filtered_rtm(self, h: float):
        """-Lap_h m_RTM, the Laplacian-filtered RTM image."""
        return laplacian_filter(self.rtm_image(), h)

    def scaled_start(self, h: float):
        """alpha f with f the filtered RTM image and alpha = <L f, d_r> / |L f|^2
        (the scale that minimises |alpha L f - d_r|); returns (x0, alpha)."""
        f = self.filtered_rtm(h)
        self.ctx.born(self.m0, f, self.d)
        self.kept = None  # self.d no longer holds the data of a kept iterate
        self.n_fwd += 1
        red = Reducer()
        num = float(red.dot(self.d, self.d_r).item())
        den = float(red.dot(self.d, self.d).item())
        alpha = num / den
        return scale(alpha, f), alpha

    def normal_op(self, x: torch.Tensor, out: torch.Tensor):
        """out = L^T L x (one Born and one Born adjoint)."""
        self.ctx.born(self.m0, x, self.d)
        self.ctx.born_adjoint(self.m0, self.d, out)
        self.n_fwd += 1
        self.n_adj += 1
        return out


@dataclasses.dataclass
class IterLog:
    k: int
    J: float
    lam: float
    mk: int
    n_grad: int
    n_fwd: int
    wall: float


class AADescent:
    """Algorithm 2 as a stepper: ``first()`` evaluates g_0 and sets p_1 = G(p_0);
    each ``iterate()`` performs one iteration k >= 1.

    M = 0 is steepest descent with the fixed step (the Picard iteration of G).
    aa_solver selects the least-squares solver ("gram" or "qr"), aa_beta the
    damping of the mixed step and aa_weights a weighted l2 norm for Step 2.
    floor: pbar and ptilde are kept at or above it (the model's stable
    domain); by default the problem's own floor (FWI), none for problems
    without one (LSRTM's reflectivity).
    The problem sees flat tensors; the accepted trial buffer becomes the new
    iterate itself, so the problem recognises (by object identity) that its
    kept forward run is at that iterate.
    """

    def __init__(self, problem, p0: torch.Tensor, eta: float | None, M: int, cond_max: float = 1e5,
                 lambdas=LAMBDAS, c1: float = ARMIJO_C1, linesearch: bool = True,
                 eta_frac: float = 0.02, aa_solver: str = "gram", aa_beta: float = 1.0, aa_weights=None,
                 restart: bool = True, floor="problem"):
        self.problem, self.M, self.eta = problem, M, eta
        self.floor = getattr(problem, "floor", None) if floor == "problem" else floor
        self.lambdas, self.c1, self.linesearch, self.eta_frac = lambdas, c1, linesearch, eta_frac
        self.restart = restart
        self.fell_back = False  # the last iteration's search took lambda = 0
        self.J_prev = None      # J(p_k) of the last iteration
        self.n_restart = 0
        self.shape = p0.shape
        self.aa = AA(p0.numel(), max(M, 1), cond_max, solver=aa_solver) if M > 0 else None
        if self.aa is not None:
            if aa_beta != 1.0:
                self.aa.set_damping(aa_beta)
            if aa_weights is not None:
                self.aa.set_weights(aa_weights.reshape(-1))
        self.red = Reducer()
        self.p = p0.detach().clone().reshape(-1)
        self.g = torch.empty_like(self.p)
        self.pbar = torch.empty_like(self.p)
        self.ptilde = torch.empty_like(self.p)
        self.trials = [torch.empty_like(self.p) for _ in range(2)]
        self.k = 0
        self.t0 = time.perf_counter()

    def _G(self):
        if self.aa is not None:
            self.aa.step(self.p, self.g, self.eta, self.pbar, self.ptilde)
        else:
            _gd_step(self.p, self.g, self.eta, self.pbar)
            self.ptilde.copy_(self.pbar)
        if self.floor is not None:
            floor_(self.pbar, self.floor)
            floor_(self.ptilde, self.floor)

    def first(self) -> IterLog:
        J = self.problem.gradient(self.p, self.g)
        self.J_prev = J
        if self.eta is None:
            self.eta = step_size(self.p, self.g, self.eta_frac)
        self._G()
        self.p = self.pbar.clone()
        return IterLog(0, J, 0.0, 0, self.problem.n_adj, self.problem.n_fwd, time.perf_counter() - self.t0)

    def iterate(self) -> IterLog:
        self.k += 1
        p, g = self.p, self.g
        J = self.problem.gradient(p, g)
        if self.restart and self.fell_back and self.aa is not None and J < self.J_prev:
            self.aa.reset()
            self.n_restart += 1
        self.J_prev = J
        self._G()
        lam_acc, p_next = 0.0, None
        if self.linesearch:
            for i, lam in enumerate(self.lambdas):
                trial = self.trials[i % 2]
                blend(lam, self.ptilde, self.pbar, trial)
                Jt = self.problem.misfit_keep(trial)
                slope = float(self.red.dot_diff(g, trial, p).item())
                if Jt <= J + self.c1 * slope:
                    lam_acc, p_next = lam, trial
                    self.trials[i % 2] = torch.empty_like(p)
                    break
        else:
            lam_acc, p_next = 1.0, self.ptilde
            self.ptilde = torch.empty_like(p)
        self.fell_back = self.linesearch and p_next is None
        if p_next is None:
            p_next = self.pbar
            self.pbar = torch.empty_like(p)
        self.p = p_next
        mk = int(self.aa.mk.item()) if self.aa is not None else 0
        return IterLog(self.k, J, lam_acc, mk, self.problem.n_adj, self.problem.n_fwd,
                       time.perf_counter() - self.t0)

    def close(self):
        if self.aa is not None:
            self.aa.close()
            self.aa = None


def aa_descent(problem, p0: torch.Tensor, eta: float | None, M: int, iters: int, cond_max: float = 1e5,
               lambdas=LAMBDAS, c1: float = ARMIJO_C1, linesearch: bool = True,
               keep_iterates: bool = True, log_path: str | None = None, callback=None, aa_solver: str = "gram",
               restart: bool = True):
    """Run Algorithm 2 for ``iters`` iterations after p_1 = G(p_0).
    Returns (iterates p_0..p_{iters+1}, history of IterLog, final p).
    aa_solver: "gram" (FP64 normal equations) or "qr" (rank-updated QR);
    restart: clear the window after a fallback step that decreased J."""
    run = AADescent(problem, p0, eta, M, cond_max, lambdas, c1, linesearch, aa_solver=aa_solver, restart=restart)
    iterates = [run.p.clone()] if keep_iterates else []
    hist = []
    out = open(log_path, "a") if log_path else None
    try:
        for i in range(iters + 1):
            rec = run.first() if i == 0 else run.iterate()
            if keep_iterates:
                iterates.append(run.p.clone())
            hist.append(rec)
            if out:
                out.write(json.dumps(dataclasses.asdict(rec)) + "\n")
            if callback:
                callback(rec)
    finally:
        if out:
            out.close()
        run.close()
    return iterates, hist, run.p.view(p0.shape)


def _gd_step(p, g, eta, out):
    """out = p - eta g (the map G of eq. GD)."""
    blend(1.0, p, p, out)
    axpy(-eta, g, out)


def step_size(m0: torch.Tensor, g0: torch.Tensor, frac: float = 0.02) -> float:
    """eta = frac * max(m0) / max|g0| (fixed for the whole run)."""
    return float(frac * m0.abs().max().item() / g0.abs().max().item())
