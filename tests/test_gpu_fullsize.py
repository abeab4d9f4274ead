"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (every node of the slice in one batched call, the projector tiles the
autotuner picks for it): sampled nodes of the batched local update against the
oracle's Alg. 2, K-means consensus bit-exact on sampled segments, the plain
per-node loop against the replayed HIP graph bit for bit, and one node of the
2048^2, 64-node workload."""
import numpy as np
import pytest
import torch

import synthdata
from gpu_common import log, rel_l2, require_gpu, to_dev
from oracle import admm as oadmm
from oracle import joseph
from oracle.kmeans import kmeans_quantize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    require_gpu()
    from paper_2410_06106_amd import admm, tomoadmm
    return tomoadmm, admm


def _slice(T, A, ctx, w, seed=3):
    """A slice of the workload with random u, lambda and x (so every term of the
    update is exercised) and the workload's own data."""
    s = A.make_slice(ctx, w)
    rng = np.random.default_rng(seed)
    s.x.copy_(to_dev(rng.random((w.n, w.n)).astype(np.float32)))
    for u, lam in zip(s.u, s.lam):
        u.copy_(to_dev(rng.random((w.n, w.n)).astype(np.float32)))
        lam.copy_(to_dev((0.1 * rng.standard_normal((w.n, w.n))).astype(np.float32)))
    return s


@pytest.mark.parametrize("tiles", [(32, 32), (32, 16), (16, 64)])
def test_single_workload_local_update_sampled_nodes(mods, tiles):
    """512^2, 720 angles, 725 bins, 16 contiguous nodes: one batched E1 = 1 step,
    three sampled nodes against the oracle."""
    T, A = mods
    ctx = T.Context(0)
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_BAND, tiles[0])
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_JOB_WGS, tiles[1])
    w = synthdata.WORKLOADS["single"]
    s = _slice(T, A, ctx, w)
    s.eta1 = 2e-5
    before = [(u.cpu().numpy(), lam.cpu().numpy()) for u, lam in zip(s.u, s.lam)]
    x = s.x.cpu().numpy()
    run = A.DADMM(ctx, [s], rho=w.rho, e1=1)
    T.admm_local_update(ctx, run.nodes, 1)
    th = synthdata.angles(w.n_angles)
    parts = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)
    for m in (0, 7, 15):
        d = s.d[m].cpu().numpy()
        ref = oadmm.local_update(before[m][0], x, before[m][1], d, th[parts[m]], w.rho, s.eta1, 1)
        # compare the increments, so the gradient itself is checked to 1e-5
        err = rel_l2(s.u[m].cpu().numpy() - before[m][0], ref - before[m][0])
        log(f"  tiles {tiles} node {m}: rel-L2 of the step {err:.3g}")
        assert err <= 1e-5


def test_single_workload_kmeans_consensus_bit_exact(mods):
    """K-means with 8 levels on all 16 segments (16384 values each) in one call;
    E2 = 0 so each quantizer sees x itself, and sampled segments must match the
    oracle bit for bit (labels, centroids, the exchanged x)."""
    T, A = mods
    ctx = T.Context(0)
    w = synthdata.WORKLOADS["single"]
    s = _slice(T, A, ctx, w)
    x0 = s.x.cpu().numpy()
    labels = [torch.empty(r * w.n, dtype=torch.uint8, device="cuda") for _, r in s.segments]
    cents = [torch.empty(8, dtype=torch.float32, device="cuda") for _ in s.segments]
    msgs = T.make_msgs([dict(labels=l, centroids=c) for l, c in zip(labels, cents)])
    run = A.DADMM(ctx, [s], rho=w.rho, e2=0, quant=T.tomo_quant(T.TOMO_QUANT_KMEANS, 8, 30, 0), msgs=msgs)
    T.admm_consensus(ctx, run.nodes, T.TOMO_XUPDATE_SEGMENT, 0, run.quant, msgs)
    xq = s.x.cpu().numpy()
    for m in (0, 5, 15):
        r0, nr = s.segments[m]
        ref = kmeans_quantize(x0[r0:r0 + nr].reshape(-1), 8, 30)
        np.testing.assert_array_equal(labels[m].cpu().numpy(), ref.labels)
        np.testing.assert_array_equal(cents[m].cpu().numpy(), ref.centroids)
        np.testing.assert_array_equal(xq[r0:r0 + nr].reshape(-1), ref.a_hat)


def test_single_workload_graph_equals_plain_loop(mods):
    """Two full ADMM iterations (E1 = 5, SEG with E2 = 10, K-means 8): the per-node
    launch loop and the replayed one-iteration graph give the same x bit for bit."""
    T, A = mods
    ctx = T.Context(0)
    w = synthdata.WORKLOADS["single"]
    s = A.make_slice(ctx, w)
    s.eta1 = A.step_size(ctx, s, w.rho, 0.1)
    run = A.DADMM(ctx, [s], rho=w.rho, eta2=w.eta2, e1=w.inner_iters, e2=w.x_iters,
                  quant=T.tomo_quant(T.TOMO_QUANT_KMEANS, w.levels, 30, 0))
    for _ in range(2):
        run.step_plain()
    torch.cuda.synchronize()
    plain = s.x.clone()
    s.zero()
    run.step()                       # builds the batched plans outside capture
    s.zero()
    torch.cuda.synchronize()
    g = run.capture(1)
    s.zero()
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    assert torch.equal(plain, s.x)


def test_large_workload_local_update_sampled_node(mods):
    """2048^2, 1800 angles, 2897 bins, 64 nodes in one batched call: one node's
    E1 = 1 step against the oracle."""
    T, A = mods
    ctx = T.Context(0)
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_BAND, 16)
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_JOB_WGS, 32)
    w = synthdata.WORKLOADS["large"]
    rng = np.random.default_rng(4)
    th = synthdata.angles(w.n_angles)
    parts = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)
    n, nb = w.n, w.n_bins
    x = to_dev(rng.random((n, n)).astype(np.float32))
    m = 37
    ents, keep = [], None
    for i, p in enumerate(parts):
        u = to_dev(rng.random((n, n)).astype(np.float32)) if i == m else torch.zeros((n, n), device="cuda")
        lam = torch.zeros((n, n), device="cuda")
        d = to_dev(rng.standard_normal((len(p), nb)).astype(np.float32))
        if i == m:
            keep = (u.cpu().numpy(), d.cpu().numpy(), u)
        ents.append(dict(n=n, n_bins=nb, angles=to_dev(th[p], torch.float64), slice=0, d=d, u=u, lam=lam, x=x,
                         seg_row0=32 * i, seg_rows=32, rho=1.0, eta1=1e-6, eta2=0.2))
    T.admm_local_update(ctx, T.make_nodes(ents), 1)
    ref = oadmm.local_update(keep[0], x.cpu().numpy(), np.zeros((n, n)), keep[1], th[parts[m]], 1.0, 1e-6, 1)
    err = rel_l2(keep[2].cpu().numpy() - keep[0], ref - keep[0])
    log(f"  large node {m}: rel-L2 of the step {err:.3g}")
    assert err <= 1e-5


@pytest.mark.parametrize("tv_iters", [10, 11])
def test_single_workload_tv_block_z_update(mods, tv_iters):
    """The regularization block at bench.py --reg tv's settings on the 512^2,
    16-node slice (TV, mu = 0.02, 10 Chambolle iterations: two launches of 5
    iterations, the second also forming z and t_z; 11: launches of 6 and 5, the
    first using the whole halo of the tile): z, t_z and the field after two
    z-updates (the second warm-started from the first's field) against the
    oracle on the whole image."""
    from oracle import reg as oreg
    T, A = mods
    ctx = T.Context(0)
    w = synthdata.WORKLOADS["single"]
    s = _slice(T, A, ctx, w)
    run = A.DADMM(ctx, [s], reg=dict(kind=T.TOMO_REG_TV, mu=0.02, tv_iters=tv_iters))
    rng = np.random.default_rng(7)
    nu = (0.05 * rng.standard_normal((w.n, w.n))).astype(np.float32)
    s.reg["nu"].copy_(to_dev(nu))
    x = s.x.cpu().numpy().astype(np.float64)
    r = oreg.Reg(kind=oreg.TV, mu=0.02, rho=1.0, tv_iters=tv_iters)
    p = None
    for k in range(2):
        T.admm_reg_update(ctx, run.nodes, run.regs)
        torch.cuda.synchronize()
        z, p = oreg.z_update(r, x, nu.astype(np.float64), p)
        ez = rel_l2(s.reg["z"].cpu().numpy(), z)
        et = rel_l2(s.reg["tz"].cpu().numpy(), z + nu / 1.0)
        gp = s.reg["p"].cpu().numpy()
        ep = max(rel_l2(gp[0], p[0]), rel_l2(gp[1], p[1]))
        log(f"  z-update {k}: z rel {ez:.2e}, t_z rel {et:.2e}, field rel {ep:.2e}")
        assert ez <= 1e-5 and et <= 1e-5 and ep <= 1e-5


def test_single_workload_chord_local_update_sampled_nodes(mods):
    """bench.py --model chord's configuration: the 512^2, 16-node slice with the
    chord-length system matrix (band 32, 48 workgroups per node, the batched
    call with its dispatch table), one E1 = 1 step, two sampled nodes against
    the oracle's Alg. 2 with the chord projector."""
    from oracle import chord
    T, A = mods
    ctx = T.Context(0)
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_MODEL, 1)
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_BAND, 32)
    T.tomo_set_option(ctx, T.TOMO_OPT_PROJ_JOB_WGS, 48)
    w = synthdata.WORKLOADS["single"]
    s = _slice(T, A, ctx, w)
    s.eta1 = 2e-5
    before = [(u.cpu().numpy(), lam.cpu().numpy()) for u, lam in zip(s.u, s.lam)]
    x = s.x.cpu().numpy()
    run = A.DADMM(ctx, [s], rho=w.rho, e1=1)
    T.admm_local_update(ctx, run.nodes, 1)
    th = synthdata.angles(w.n_angles)
    parts = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)
    for m in (0, 9):
        d = s.d[m].cpu().numpy()
        ref = oadmm.local_update(before[m][0], x, before[m][1], d, th[parts[m]], w.rho, s.eta1, 1, proj=chord)
        err = rel_l2(s.u[m].cpu().numpy() - before[m][0], ref - before[m][0])
        log(f"  chord node {m}: rel-L2 of the step {err:.3g}")
        assert err <= 1e-5
