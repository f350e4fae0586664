"""The FWI-gradient workload at full size (768 x 256 interior, 64 shots,
4000 steps, checkpoints every 50), in the launch shape the bench uses
(autotuned), checked where the oracle can reach:

* traces of two sampled shots over the first 600 steps against the oracle's
  run of those shots alone (samples before step 600 do not depend on later
  steps, and shots do not interact);
* the gradient against a central difference of J along a random smooth
  perturbation (a property of the exact adjoint at any size);
* the Born dot-product test <L x, y> = <x, L^T y>.
"""
import numpy as np
import pytest

import synth
from oracle import fd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    import torch
    from paper_2008_11778_amd import Context, autotune
    g, m_true, m0 = synth.config2()
    ctx = Context(g, ckpt_every=50)
    m0t = torch.from_numpy(m0).cuda()
    autotune.apply(ctx, autotune.tune(g, m0t))
    yield g, m_true, m0, ctx
    ctx.close()


def test_sampled_shot_traces_match_oracle(c2):
    import torch
    g, _, m0, ctx = c2
    d = ctx.forward_model(torch.from_numpy(m0).cuda()).cpu().numpy()
    nt_s = 600
    gs = synth.config2(nt=nt_s)[0]
    for s in (0, 37):
        ref = fd.forward_model(gs.subset_shots([s]), m0)[0]
        got = d[s, :nt_s]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"shot {s}: rel L2 {err:.2e}")
        assert err <= 1e-4, (s, err)


def test_gradient_directional_derivative(c2):
    import torch
    g, m_true, m0, ctx = c2
    d_obs = ctx.forward_model(torch.from_numpy(m_true).cuda()).clone()
    r = np.random.default_rng(17)
    dm = synth.smooth(r.standard_normal(m0.shape), 6.0)
    dm = (dm / np.abs(dm).max() * 0.002 * np.abs(m0).max()).astype(np.float32)
    m = torch.from_numpy(m0).cuda()
    grad, J = ctx.adjoint_gradient(m, d_obs)
    slope = float((grad.double() * torch.from_numpy(dm).cuda().double()).sum())
    Jp = ctx.adjoint_gradient(m + torch.from_numpy(dm).cuda(), d_obs)[1].item()
    Jm = ctx.adjoint_gradient(m - torch.from_numpy(dm).cuda(), d_obs)[1].item()
    fd_slope = (Jp - Jm) / 2.0
    print(f"J {J.item():.6e} slope {slope:.6e} central difference {fd_slope:.6e}")
    assert abs(fd_slope - slope) <= 1e-2 * abs(slope)


def test_born_dot_product(c2):
    import torch
    g, _, m0, ctx = c2
    r = np.random.default_rng(18)
    x = torch.from_numpy((synth.smooth(r.standard_normal(m0.shape), 2.0) * 1e-9).astype(np.float32)).cuda()
    y = torch.from_numpy(r.standard_normal((g.nshots, g.nt, g.nrec)).astype(np.float32)).cuda()
    m = torch.from_numpy(m0).cuda()
    lx = ctx.born(m, x)
    lty = ctx.born_adjoint(m, y)
    a = float((lx.double() * y.double()).sum())
    b = float((x.double() * lty.double()).sum())
    print(f"<Lx, y> {a:.9e} <x, L^T y> {b:.9e}")
    assert abs(a - b) <= 1e-4 * abs(a)


def test_large_grid_two_step_forward_sampled_shot():
    """The 1024 x 384, 96-shot forward step in its autotuned launch shape (two
    steps per launch on this grid), as the bench's large-grid measurement
    runs it: one sampled shot against the oracle over the 400 steps."""
    import torch
    from paper_2008_11778_amd import Context, autotune
    g, _, m0 = synth.config5(nt=400)
    with Context(g, ckpt_every=50) as ctx:
        m = torch.from_numpy(m0).cuda()
        autotune.apply(ctx, autotune.tune(g, m))
        print("launch modes (bit mask):", ctx.time_blocking())
        d = ctx.forward_model(m).cpu().numpy()
    s = 50
    ref = fd.forward_model(g.subset_shots([s]), m0)[0]
    err = float(np.linalg.norm(d[s] - ref) / np.linalg.norm(ref))
    print(f"shot {s}: rel L2 {err:.2e}")
    assert err <= 1e-4
