"""The residual/misfit entry point that allocates nothing
(aafwi_residual_misfit_noalloc, static device scratch) against the context
entry point aafwi_residual_misfit on the same inputs: two calls in a row,
the second on a smaller data cube, both bitwise equal (same kernels, same
fixed summation order) in r and in J."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _cube(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape).astype(np.float32)


def test_noalloc_misfit_matches_context_entry_point_twice():
    import torch
    from paper_2008_11778_amd import Context
    from paper_2008_11778_amd._lib import residual_misfit_noalloc
    dev = torch.device("cuda", 0)
    big, _, _ = synth.config1()                     # 4 x 800 x 128 samples
    small, _ = synth.small_case(nshots=2, nt=150)   # 2 x 150 x 8 samples
    for i, g in enumerate((big, small)):
        shape = (g.nshots, g.nt, g.nrec)
        d = torch.from_numpy(_cube(shape, 100 + i)).to(dev)
        d_obs = torch.from_numpy(_cube(shape, 200 + i)).to(dev)
        with Context(g) as ctx:
            r_ref, J_ref = ctx.residual_misfit(d, d_obs)
            torch.cuda.synchronize()
            r = torch.full_like(d, float("nan"))
            J = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
            residual_misfit_noalloc(d, d_obs, r, J, stream=ctx.stream)
            torch.cuda.synchronize()
        J_np = float(J.item())
        # the residual is rounded to FP32 (it is an output), then squared and
        # summed in FP64
        r_host = (_cube(shape, 100 + i) - _cube(shape, 200 + i)).astype(np.float64)
        J_host = 0.5 * float(np.sum(r_host ** 2))
        print(f"call {i}: n = {d.numel()}, J = {J_np:.12e}, context entry point {float(J_ref.item()):.12e}, "
              f"FP64 host sum {J_host:.12e}")
        assert torch.equal(r, r_ref)
        assert J_np == float(J_ref.item())
        assert abs(J_np - J_host) <= 1e-12 * J_host


def test_noalloc_misfit_rejects_bad_sizes():
    import torch
    from paper_2008_11778_amd._lib import AafwiError, residual_misfit_noalloc
    x = torch.zeros(0, device="cuda")
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(AafwiError):
        residual_misfit_noalloc(x, x, x, J)
