"""Algorithm 2 on many independent inversion instances at once.

Every instance runs its own Algorithm 2 (its own eta, Anderson window and
line search); all instances share each wave-equation launch through a Batch
(one launch per time step covers every instance's tiles; the launch
sequences are replayed as HIP graphs).  A line-search round runs a masked
batched forward for the instances still searching; an instance whose trial
is accepted keeps that forward run for its next gradient.

With the same inputs this produces, instance by instance, the same iterates
as ``inversion.AADescent`` on separate contexts (the kernels and their
arithmetic order are identical), restarts of the Anderson window after a
fallback step that decreased J included.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from ._lib import Batch, BatchAA, Reducer, axpy, blend, floor_
from .inversion import ARMIJO_C1, LAMBDAS


class BatchedAADescent:
    def __init__(self, batch: Batch, p0, M: int, etas=None, eta_frac: float = 0.02, cond_max: float = 1e5,
                 lambdas=LAMBDAS, c1: float = ARMIJO_C1, restart: bool = True, project: bool = True):
        self.b = batch
        # each instance's pbar and ptilde are kept at or above its floor (the
        # stable domain of its geometry), as in the single-instance driver
        self.floors = list(batch.floors) if project else None
        self.restart = restart
        self.N = batch.N
        self.M, self.lambdas, self.c1, self.eta_frac = M, lambdas, c1, eta_frac
        self.etas = None if etas is None else [float(e) for e in etas]
        s = batch.stream
        with torch.cuda.stream(s):
            self.p = [x.detach().reshape(-1).clone() for x in p0]
            self.pbar = [torch.empty_like(x) for x in self.p]
            self.ptilde = [torch.empty_like(x) for x in self.p]
            self.slope = torch.zeros(self.N, dtype=torch.float64, device=batch.device)
        # one Anderson state for all instances: every step is one launch
        # sequence over the whole batch
        self.aa = BatchAA([x.numel() for x in self.p], M, cond_max, stream=s) if M > 0 else None
        self.red = Reducer(stream=s)
        self.kept_ok = [False] * self.N
        self.fell_back = [False] * self.N
        self.J_prev = None
        self.k = 0
        self.n_forward_launches = 0
        self.n_backward_launches = 0
        self.t0 = time.perf_counter()

    # -- helpers ---------------------------------------------------------------
    def _m(self, i):
        return self.b.m[i].view(-1)

    def _g(self, i):
        return self.b.grad[i].view(-1)

    def _forward(self, mask):
        self.b.set_active(np.asarray(mask, np.uint8))
        self.b.forward(keep_ckpt=True)
        self.n_forward_launches += 1
        return self.b.misfits()

    def _gradients(self):
        """Gradients (and misfits) at the current iterates of all instances."""
        s = self.b.stream
        need = [not ok for ok in self.kept_ok]
        if any(need):
            for i in range(self.N):
                if need[i]:
                    blend(1.0, self.p[i], self.p[i], self._m(i), stream=s)
            self._forward(need)
        self.b.set_active(np.ones(self.N, np.uint8))
        self.b.backward()
        self.n_backward_launches += 1
        self.kept_ok = [True] * self.N
        return self.b.misfits()

    def _anderson(self):
        s = self.b.stream
        if self.aa is not None:
            self.aa.step(self.p, [self._g(i) for i in range(self.N)], self.etas, self.pbar, self.ptilde)
        else:
            for i in range(self.N):
                blend(1.0, self.p[i], self.p[i], self.pbar[i], stream=s)
                axpy(-self.etas[i], self._g(i), self.pbar[i], stream=s)
                blend(1.0, self.pbar[i], self.pbar[i], self.ptilde[i], stream=s)
        if self.floors is not None:
            for i in range(self.N):
                floor_(self.pbar[i], self.floors[i], stream=s)
                floor_(self.ptilde[i], self.floors[i], stream=s)

    # -- Algorithm 2 -------------------------------------------------------------
    def first(self):
        """g_0 at p_0 for every instance, then p_1 = G(p_0)."""
        J = self._gradients()
        self.J_prev = np.array(J, np.float64)
        if self.etas is None:
            self.etas = []
            with torch.cuda.stream(self.b.stream):
                for i in range(self.N):
                    self.etas.append(float(self.eta_frac * self.p[i].abs().max().item()
                                           / self._g(i).abs().max().item()))
        self._anderson()
        with torch.cuda.stream(self.b.stream):
            self.p = [x.clone() for x in self.pbar]
        self.kept_ok = [False] * self.N
        return J

    def iterate(self):
        """One iteration k >= 1 for every instance.

        Returns (J(p_k), lambdas, J(p_{k+1})), the last entry being the
        accepted trial's misfit, or NaN where the search fell back to pbar
        (whose misfit the next gradient evaluation computes)."""
        s = self.b.stream
        self.k += 1
        J = self._gradients()
        # restart after a fallback step that decreased J (as in AADescent)
        which = [self.restart and self.fell_back[i] and J[i] < self.J_prev[i] for i in range(self.N)]
        if self.aa is not None and any(which):
            self.aa.reset(which)
        self.J_prev = np.array(J, np.float64)
        self._anderson()
        pending = [True] * self.N
        lam = [0.0] * self.N
        new_p = [None] * self.N
        J_next = np.full(self.N, np.nan)
        for lv in self.lambdas:
            idx = [i for i in range(self.N) if pending[i]]
            if not idx:
                break
            for i in idx:
                blend(lv, self.ptilde[i], self.pbar[i], self._m(i), stream=s)
            Jt = self._forward(pending)
            for i in idx:
                self.red.dot_diff(self._g(i), self._m(i), self.p[i], out=self.slope[i:i + 1])
            with torch.cuda.stream(s):
                slope = self.slope.cpu().numpy()
            for i in idx:
                if Jt[i] <= J[i] + self.c1 * slope[i]:
                    with torch.cuda.stream(s):
                        new_p[i] = self._m(i).clone()
                    lam[i] = lv
                    J_next[i] = Jt[i]
                    pending[i] = False
        self.fell_back = list(pending)
        for i in range(self.N):
            if pending[i]:
                with torch.cuda.stream(s):
                    new_p[i] = self.pbar[i].clone()
                self.kept_ok[i] = False
        self.b.set_active(np.ones(self.N, np.uint8))
        self.p = new_p
        return J, lam, J_next

    def current_misfits(self):
        """J at the current iterates of all instances: a (masked) forward run
        for those whose last step was a fallback to pbar, whose misfit the
        line search did not compute; the others keep their accepted trial's."""
        s = self.b.stream
        need = [not ok for ok in self.kept_ok]
        if any(need):
            for i in range(self.N):
                if need[i]:
                    blend(1.0, self.p[i], self.p[i], self._m(i), stream=s)
            self._forward(need)
            self.kept_ok = [True] * self.N
        self.b.set_active(np.ones(self.N, np.uint8))
        return self.b.misfits()

    def close(self):
        if self.aa is not None:
            self.aa.close()
            self.aa = None
