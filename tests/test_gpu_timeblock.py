"""Two time steps per launch against one step per launch: traces, misfits,
gradients and Born-adjoint images must be bitwise equal (the two-step
kernels evaluate every point with the one-step arithmetic in the same
order), over a ragged 64-column tiling, several strip heights (ragged
strips included), odd record lengths, odd and even checkpoint intervals, and
uneven batches."""
import numpy as np
import pytest

import synth
from oracle import fd

pytestmark = pytest.mark.gpu


def T(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def ragged_case(nshots=3, nt=301):
    """70 x 150 interior (90 x 170 padded: two full 64-column tiles and a
    42-column tail; strips of more than 64 rows apply to the two-step kernels
    only), sources in a corner, mid-grid and the far edge,
    receivers in two rows including the edge columns and a shared node."""
    g, m = synth.small_case(nz=70, nx=150, nb=10, nt=nt, nshots=nshots, nrec=12, f0=20.0, instance=3)
    rec_iz = np.tile(np.array([2] * 6 + [40] * 6, np.int32), (nshots, 1))
    rec_ix = np.tile(np.array([0, 31, 63, 64, 100, 149, 5, 5, 77, 120, 140, 149], np.int32), (nshots, 1))
    g = g.replace(rec_iz=rec_iz, rec_ix=rec_ix, src_iz=np.array([0, 35, 69][:nshots], np.int32),
                  src_ix=np.array([0, 75, 149][:nshots], np.int32))
    return g, m


def run(g, m, d_obs, k, rows, tb):
    from paper_2008_11778_amd import Context
    with Context(g, ckpt_every=k) as ctx:
        ctx.set_time_blocking(tb)
        assert ctx.time_blocking() == (7 if tb else 0)
        ctx.set_tile(rows)
        d = ctx.forward_model(T(m)).cpu().numpy()
        grad, J = ctx.adjoint_gradient(T(m), T(d_obs))
        img = ctx.born_adjoint(T(m), T(d_obs))
        return d, grad.cpu().numpy(), float(J.item()), img.cpu().numpy()


@pytest.mark.parametrize("k,rows", [(7, 0), (50, 13), (301, 37), (1, 64), (20, 4), (16, 120), (9, 77)])
def test_two_step_equals_one_step_bitwise(k, rows):
    g, m = ragged_case()
    r = np.random.default_rng(5)
    m_true = (m.astype(np.float64) * (1 + 0.02 * r.standard_normal(m.shape))).astype(np.float32)
    d_obs = fd.forward_model(g, m_true).astype(np.float32)
    one = run(g, m, d_obs, k, rows, False)
    two = run(g, m, d_obs, k, rows, True)
    assert np.array_equal(one[0], two[0])
    assert np.array_equal(one[1], two[1])
    assert one[2] == two[2]
    assert np.array_equal(one[3], two[3])


def test_two_step_gradient_matches_oracle():
    from paper_2008_11778_amd import Context
    g, m = ragged_case(nshots=2, nt=241)
    r = np.random.default_rng(6)
    m_true = (m.astype(np.float64) * (1 + 0.02 * r.standard_normal(m.shape))).astype(np.float32)
    d_obs = fd.forward_model(g, m_true).astype(np.float32)
    J_ref, g_ref = fd.adjoint_gradient(g, m, d_obs)
    d_ref = fd.forward_model(g, m)
    with Context(g, ckpt_every=25) as ctx:
        assert not ctx.time_blocking()  # small grids default to one step per launch
        ctx.set_time_blocking(True)
        d = ctx.forward_model(T(m)).cpu().numpy()
        grad, J = ctx.adjoint_gradient(T(m), T(d_obs))
    assert np.linalg.norm(d - d_ref) / np.linalg.norm(d_ref) <= 1e-4
    assert np.linalg.norm(grad.cpu().numpy() - g_ref) / np.linalg.norm(g_ref) <= 1e-3
    assert abs(float(J.item()) - J_ref) / J_ref <= 1e-3


def test_uneven_batch_two_step_equals_one_step():
    from paper_2008_11778_amd import Batch
    specs = [dict(nz=30, nx=70, nb=8, nt=130, nshots=2, nrec=9, h=10.0, dt=1e-3, f0=20.0, instance=11),
             dict(nz=44, nx=150, nb=12, nt=171, nshots=3, nrec=15, h=12.5, dt=1e-3, f0=15.0, instance=12),
             dict(nz=20, nx=40, nb=6, nt=95, nshots=1, nrec=7, h=8.0, dt=5e-4, f0=25.0, instance=13)]
    insts = []
    for sp in specs:
        g, m = synth.small_case(**sp)
        r = np.random.default_rng(sp["instance"])
        mt = (m.astype(np.float64) * (1 + 0.03 * r.standard_normal(m.shape))).astype(np.float32)
        insts.append((g, m, fd.forward_model(g, mt).astype(np.float32)))
    outs = []
    for tb in (False, True):
        with Batch([g for g, _, _ in insts], [d for _, _, d in insts], ckpt_every=15, use_graphs=True) as b:
            import torch
            b.set_time_blocking(tb)
            with torch.cuda.stream(b.stream):
                for i, (_, m, _) in enumerate(insts):
                    b.m[i].copy_(T(m))
            b.set_active(np.ones(b.N, np.uint8))
            b.forward(keep_ckpt=True)
            J = b.misfits()
            b.backward()
            b.stream.synchronize()
            outs.append([(b.grad[i].cpu().numpy(), float(J[i]), b.r[i].cpu().numpy()) for i in range(b.N)])
    for (ga, Ja, ra), (gb, Jb, rb) in zip(*outs):
        assert np.array_equal(ga, gb) and Ja == Jb and np.array_equal(ra, rb)


def test_tile_order_is_bitwise_neutral():
    """Tile orders: x-tiles of a strip adjacent, strips of a column
    adjacent, and shot groups of 2 (the last group ragged on 3 shots) and 4
    (larger than the shot count) innermost."""
    from paper_2008_11778_amd import Context
    g, m = ragged_case(nshots=3, nt=121)
    d_obs = np.zeros((g.nshots, g.nt, g.nrec), np.float32)
    outs = []
    for tb in (False, True):
        for order in (0, 1, 2, 4):
            with Context(g, ckpt_every=16) as ctx:
                ctx.set_time_blocking(tb)
                ctx.set_tile_order(order)
                ctx.set_tile(24)
                d = ctx.forward_model(T(m)).cpu().numpy()
                grad, _ = ctx.adjoint_gradient(T(m), T(d_obs + 1.0))
                outs.append((d, grad.cpu().numpy()))
    for d, gr in outs[1:]:
        assert np.array_equal(d, outs[0][0]) and np.array_equal(gr, outs[0][1])


def test_per_kernel_modes_are_bitwise_neutral():
    """Forward, recompute and adjoint choose one or two steps per launch
    independently; every combination gives the same traces and gradient."""
    from paper_2008_11778_amd import Context
    g, m = ragged_case(nshots=2, nt=97)
    d_obs = np.zeros((g.nshots, g.nt, g.nrec), np.float32) + 0.5
    outs = []
    for mask in range(8):
        with Context(g, ckpt_every=10) as ctx:
            for k in range(3):
                ctx.set_time_blocking(bool(mask >> k & 1), k)
            assert ctx.time_blocking() == mask
            d = ctx.forward_model(T(m)).cpu().numpy()
            grad, J = ctx.adjoint_gradient(T(m), T(d_obs))
            outs.append((d, grad.cpu().numpy(), float(J.item())))
    for d, gr, J in outs[1:]:
        assert np.array_equal(d, outs[0][0]) and np.array_equal(gr, outs[0][1]) and J == outs[0][2]
