"""Batched uneven instances (one launch per time step over all instances,
HIP-graph replays, masks) against single-instance contexts and the oracle."""
import numpy as np
import pytest

import synth
from oracle import fd

pytestmark = pytest.mark.gpu


def instances():
    """Three instances with different grids, spacings, time steps, record
    lengths (not multiples of the checkpoint interval), shots and receivers."""
    out = []
    specs = [dict(nz=30, nx=70, nb=8, nt=130, nshots=2, nrec=9, h=10.0, dt=1e-3, f0=20.0, instance=11),
             dict(nz=44, nx=150, nb=12, nt=171, nshots=3, nrec=15, h=12.5, dt=1e-3, f0=15.0, instance=12),
             dict(nz=20, nx=40, nb=6, nt=95, nshots=1, nrec=7, h=8.0, dt=5e-4, f0=25.0, instance=13)]
    for sp in specs:
        g, m = synth.small_case(**sp)
        r = np.random.default_rng(sp["instance"])
        mt = (m.astype(np.float64) * (1 + 0.03 * r.standard_normal(m.shape))).astype(np.float32)
        d_obs = fd.forward_model(g, mt).astype(np.float32)
        out.append((g, m, d_obs))
    return out


@pytest.fixture(scope="module")
def insts():
    return instances()


def single_results(insts, k):
    import torch
    from paper_2008_11778_amd import Context
    res = []
    for g, m, d_obs in insts:
        with Context(g, ckpt_every=k) as ctx:
            grad, J = ctx.adjoint_gradient(torch.from_numpy(m).cuda(), torch.from_numpy(d_obs).cuda())
            d = ctx.forward_model(torch.from_numpy(m).cuda())
            res.append((grad.cpu().numpy(), float(J.item()), (d.cpu().numpy() - d_obs)))
    return res


def run_batch(b, insts):
    import torch
    with torch.cuda.stream(b.stream):
        for i, (g, m, _) in enumerate(insts):
            b.m[i].copy_(torch.from_numpy(m).to(b.device))
    b.set_active(np.ones(b.N, np.uint8))
    b.forward(keep_ckpt=True)
    J = b.misfits()
    b.backward()
    b.stream.synchronize()
    return [(b.grad[i].cpu().numpy(), float(J[i]), b.r[i].cpu().numpy()) for i in range(b.N)]


def test_batch_equals_single_instances_bitwise(insts):
    from paper_2008_11778_amd import Batch
    k = 20
    ref = single_results(insts, k)
    with Batch([g for g, _, _ in insts], [d for _, _, d in insts], ckpt_every=k, use_graphs=False) as b:
        got = run_batch(b, insts)
    for (ga, Ja, ra), (gb, Jb, rb) in zip(got, ref):
        assert np.array_equal(ga, gb)
        assert Ja == Jb
        assert np.array_equal(ra, rb.astype(np.float32))


def test_batch_gradient_matches_oracle(insts):
    from paper_2008_11778_amd import Batch
    with Batch([g for g, _, _ in insts], [d for _, _, d in insts], ckpt_every=20, use_graphs=True) as b:
        got = run_batch(b, insts)
    for (g, m, d_obs), (grad, J, _) in zip(insts, got):
        J_ref, g_ref = fd.adjoint_gradient(g, m, d_obs)
        assert np.linalg.norm(grad - g_ref) / np.linalg.norm(g_ref) <= 1e-3
        assert abs(J - J_ref) / J_ref <= 1e-3


def test_graph_replays_equal_eager_and_masks(insts):
    import torch
    from paper_2008_11778_amd import Batch
    with Batch([g for g, _, _ in insts], [d for _, _, d in insts], ckpt_every=20, use_graphs=False) as b:
        eager = run_batch(b, insts)
    with Batch([g for g, _, _ in insts], [d for _, _, d in insts], ckpt_every=20, use_graphs=True) as b:
        for rep in range(3):
            got = run_batch(b, insts)
            torch.cuda.synchronize()
            for (ga, Ja, ra), (gb, Jb, rb) in zip(got, eager):
                assert np.array_equal(ga, gb) and Ja == Jb and np.array_equal(ra, rb), rep
        # a masked forward leaves the masked instance's residual and misfit alone
        r1 = b.r[1].cpu().numpy().copy()
        J1 = b.misfits()[1]
        with torch.cuda.stream(b.stream):
            b.m[0].mul_(1.01)
            b.m[1].mul_(1.01)
        b.set_active(np.array([1, 0, 1], np.uint8))
        b.forward(keep_ckpt=True)
        J = b.misfits()
        b.stream.synchronize()
        assert np.array_equal(b.r[1].cpu().numpy(), r1) and J[1] == J1
        assert J[0] != eager[0][1]


def test_batched_algorithm2_equals_per_instance_runs(insts):
    import torch
    from paper_2008_11778_amd import Batch, Context
    from paper_2008_11778_amd.batched import BatchedAADescent
    from paper_2008_11778_amd.inversion import AADescent, FWIProblem
    etas = []
    singles = []
    finals = []
    for g, m, d_obs in insts:
        with Context(g, ckpt_every=20) as ctx:
            prob = FWIProblem(ctx, torch.from_numpy(d_obs).cuda())
            run = AADescent(prob, torch.from_numpy(m).cuda(), None, M=3)
            run.first()
            etas.append(run.eta)
            its = [run.p.clone()]
            for _ in range(3):
                run.iterate()
                its.append(run.p.clone())
            finals.append(prob.misfit_keep(run.p))
            run.close()
            singles.append([x.cpu().numpy() for x in its])
    with Batch([g for g, _, _ in insts], [d for _, _, d in insts], ckpt_every=20, use_graphs=True) as b:
        br = BatchedAADescent(b, [torch.from_numpy(m).cuda() for _, m, _ in insts], M=3, etas=etas)
        br.first()
        bits = [[x.cpu().numpy() for x in br.p]]
        for _ in range(3):
            br.iterate()
            bits.append([x.cpu().numpy() for x in br.p])
        # misfits of the final iterates (a forward run where the last step fell back)
        J_end = list(br.current_misfits())
        br.close()
    for k in range(4):
        for i in range(len(insts)):
            assert np.array_equal(bits[k][i], singles[i][k]), (k, i)
    assert J_end == finals, (J_end, finals)


def _learned_singles(insts, w, scale=None, lambdas=None, iters=3):
    """LearnedAADescent on a separate context per instance (eta_theta times
    ``scale`` after the first step, if given): iterates, etas, eta_thetas,
    fallback counts and the final misfit."""
    import torch
    from paper_2008_11778_amd import CNN, Context
    from paper_2008_11778_amd.inversion import LAMBDAS, FWIProblem
    from paper_2008_11778_amd.learned import LearnedAADescent
    out = []
    for g, m, d_obs in insts:
        with Context(g, ckpt_every=20) as ctx, CNN(g.nz, g.nx, 1, w) as net:
            prob = FWIProblem(ctx, torch.from_numpy(d_obs).cuda())
            run = LearnedAADescent(prob, torch.from_numpy(m).cuda(), net, M=3,
                                   lambdas=LAMBDAS if lambdas is None else lambdas)
            run.first()
            if scale is not None:
                run.eta_theta *= scale
            its = [run.p.cpu().numpy()]
            for _ in range(iters):
                run.iterate()
                its.append(run.p.cpu().numpy())
            out.append(dict(its=its, eta=run.eta, eta_theta=run.eta_theta, fallbacks=run.n_fallback,
                            J_end=prob.misfit_keep(run.p)))
            run.close()
    return out


@pytest.mark.parametrize("scale,lambdas", [(None, None), (30.0, ()), (30.0, None)],
                         ids=["own-eta", "overshoot-no-trials", "overshoot"])
def test_batched_learned_equals_per_instance_runs(insts, scale, lambdas):
    """The batched learned form against LearnedAADescent per instance with
    the shipped network: at its own eta_theta, and with eta_theta 30 times
    larger from the second step on, which overshoots so that pbar_theta
    raises J and the iteration falls back to plain AA (with no line-search
    trials such an iteration takes the plain pbar; with the usual four, the
    searches run in whatever order the misfits dictate)."""
    import torch
    from paper_2008_11778_amd import Batch
    from paper_2008_11778_amd.inversion import LAMBDAS
    from paper_2008_11778_amd.learned import BatchedLearnedAADescent, shipped_weights
    w, _ = shipped_weights()
    ref = _learned_singles(insts, w, scale, lambdas)
    if lambdas == ():
        assert sum(r["fallbacks"] for r in ref) > 0, [r["fallbacks"] for r in ref]
    with Batch([g for g, _, _ in insts], [d for _, _, d in insts], ckpt_every=20, use_graphs=True) as b:
        br = BatchedLearnedAADescent(b, [torch.from_numpy(m).cuda() for _, m, _ in insts], w, M=3,
                                     lambdas=LAMBDAS if lambdas is None else lambdas)
        br.first()
        if scale is not None:
            br.eta_thetas = [e * scale for e in br.eta_thetas]
        bits = [[x.cpu().numpy() for x in br.p]]
        for _ in range(3):
            br.iterate()
            bits.append([x.cpu().numpy() for x in br.p])
        J_end = list(br.current_misfits())
        etas, eta_thetas, fallbacks = list(br.etas), list(br.eta_thetas), list(br.n_fallback)
        br.close()
    for i, r in enumerate(ref):
        assert etas[i] == r["eta"] and eta_thetas[i] == r["eta_theta"], i
        assert fallbacks[i] == r["fallbacks"], (i, fallbacks, [x["fallbacks"] for x in ref])
        for k in range(4):
            assert np.array_equal(bits[k][i], r["its"][k]), (k, i)
        assert J_end[i] == r["J_end"], (i, J_end[i], r["J_end"])
