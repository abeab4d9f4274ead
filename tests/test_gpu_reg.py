"""GPU parity of the regularization block (admm_reg_update / admm_consensus_reg)
against the oracle (oracle/reg.py): the z-update (Tikhonov, TV with warm
start, even and odd iteration counts, several blocks of different sizes in one
call), the x-update with the block's term (SEG and AVG), the dual updates, the
K-means path, whole ADMM runs and a captured graph; argument errors."""
import numpy as np
import pytest
import torch

import synthdata
from gpu_common import log, rel_l2, require_gpu, to_dev
from oracle import admm as oadmm
from oracle import joseph, stepsize
from oracle import reg as oreg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    require_gpu()
    from paper_2410_06106_amd import admm, tomoadmm
    return tomoadmm, admm


@pytest.fixture(scope="module")
def ctx(mods):
    return mods[0].Context(0)


def _slice_nodes(T, n, n_nodes, x, us, lams, rho=1.0, eta2=0.2, slice_id=0):
    rows = n // n_nodes
    ents = []
    for m in range(n_nodes):
        r0 = m * rows
        nr = rows if m < n_nodes - 1 else n - r0
        ents.append(dict(n=n, n_bins=8, angles=torch.zeros(1, dtype=torch.float64, device="cuda"),
                         slice=slice_id, d=torch.zeros((1, 8), device="cuda"), u=us[m], lam=lams[m], x=x,
                         seg_row0=r0, seg_rows=nr, rho=rho, eta1=0.0, eta2=eta2))
    return ents


@pytest.mark.parametrize("iters", [0, 1, 7, 10, 11, 16, 17, 23])
def test_z_update_matches_oracle(mods, ctx, iters):
    """Two blocks in one call: TV on a 130 x 130 slice (several workgroups, a
    ragged tail) from a non-zero field, Tikhonov on a 37 x 37 slice.  11 and 23
    iterations make launches of 6 + 5 and 6 + 6 + 6 + 5: a launch of the full
    six iterations uses up the whole halo of the tile."""
    T, _ = mods
    rng = np.random.default_rng(10 + iters)
    blocks, ents = [], []
    for si, (n, kind) in enumerate(((130, T.TOMO_REG_TV), (37, T.TOMO_REG_TIKHONOV))):
        x = rng.standard_normal((n, n)).astype(np.float32)
        nu = (0.3 * rng.standard_normal((n, n))).astype(np.float32)
        p = (0.5 * rng.uniform(-1, 1, (2, n, n))).astype(np.float32)
        t = dict(x=to_dev(x), z=torch.zeros((n, n), device="cuda"), nu=to_dev(nu),
                 tz=torch.zeros((n, n), device="cuda"), p=to_dev(p))
        blocks.append((n, kind, x, nu, p, t))
        ents += _slice_nodes(T, n, 2, t["x"], [torch.zeros((n, n), device="cuda")] * 2,
                             [torch.zeros((n, n), device="cuda")] * 2, slice_id=si)
    nodes = T.make_nodes(ents)
    mu, rho, tau = 0.4, 1.3, 0.125
    regs = T.make_regs([dict(slice=si, kind=kind, mu=mu, rho=rho, tv_iters=iters, tau=tau, z=t["z"], nu=t["nu"],
                             tz=t["tz"], p=t["p"] if kind == T.TOMO_REG_TV else None)
                        for si, (n, kind, x, nu, p, t) in enumerate(blocks)])
    T.admm_reg_update(ctx, nodes, regs)
    torch.cuda.synchronize()
    for n, kind, x, nu, p, t in blocks:
        r = oreg.Reg(kind=oreg.TV if kind == T.TOMO_REG_TV else oreg.TIKHONOV, mu=mu, rho=rho, tv_iters=iters,
                     tau=tau)
        z, pz = oreg.z_update(r, x, nu, (p[0], p[1]) if kind == T.TOMO_REG_TV else None)
        ez = rel_l2(t["z"].cpu().numpy(), z)
        et = rel_l2(t["tz"].cpu().numpy(), z + nu / rho)
        log(f"  n={n} kind={kind} iters={iters}: z rel {ez:.2e}, t_z rel {et:.2e}")
        assert ez <= 1e-5 and et <= 1e-5
        if kind == T.TOMO_REG_TV:
            gp = t["p"].cpu().numpy()
            assert rel_l2(gp[0], pz[0]) <= 1e-5 and rel_l2(gp[1], pz[1]) <= 1e-5


@pytest.mark.parametrize("n", [1, 2, 9])
def test_z_update_tiny_images(mods, ctx, n):
    """TV z-updates on images smaller than one tile (1 x 1: no differences at
    all; 2 x 2; 9 x 9), 6 iterations from a non-zero field."""
    T, _ = mods
    rng = np.random.default_rng(30 + n)
    x = rng.standard_normal((n, n)).astype(np.float32)
    nu = (0.3 * rng.standard_normal((n, n))).astype(np.float32)
    p = (0.5 * rng.uniform(-1, 1, (2, n, n))).astype(np.float32)
    t = dict(x=to_dev(x), z=torch.zeros((n, n), device="cuda"), nu=to_dev(nu), tz=torch.zeros((n, n), device="cuda"),
             p=to_dev(p))
    nodes = T.make_nodes(_slice_nodes(T, n, 1, t["x"], [torch.zeros((n, n), device="cuda")],
                                      [torch.zeros((n, n), device="cuda")]))
    regs = T.make_regs([dict(slice=0, kind=T.TOMO_REG_TV, mu=0.3, rho=1.0, tv_iters=6, tau=0.125, z=t["z"],
                             nu=t["nu"], tz=t["tz"], p=t["p"])])
    T.admm_reg_update(ctx, nodes, regs)
    torch.cuda.synchronize()
    z, pz = oreg.z_update(oreg.Reg(kind=oreg.TV, mu=0.3, rho=1.0, tv_iters=6), x, nu, (p[0], p[1]))
    np.testing.assert_allclose(t["z"].cpu().numpy(), z, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(t["p"].cpu().numpy()[0], pz[0], rtol=1e-5, atol=1e-6)


def _consensus_case(T, rng, n, n_nodes):
    x = rng.standard_normal((n, n)).astype(np.float32)
    us = [rng.standard_normal((n, n)).astype(np.float32) for _ in range(n_nodes)]
    lams = [(0.2 * rng.standard_normal((n, n))).astype(np.float32) for _ in range(n_nodes)]
    z = rng.standard_normal((n, n)).astype(np.float32)
    nu = (0.2 * rng.standard_normal((n, n))).astype(np.float32)
    tz = (z + nu / 0.7).astype(np.float32)
    return x, us, lams, z, nu, tz


@pytest.mark.parametrize("mode", ["seg", "avg"])
def test_consensus_with_block_matches_oracle(mods, ctx, mode):
    T, _ = mods
    rng = np.random.default_rng(20)
    n, M, rho, rho_z, eta2, e2 = 67, 3, 1.0, 0.7, 0.2, 10
    x, us, lams, z, nu, tz = _consensus_case(T, rng, n, M)
    gx, gu, gl = to_dev(x), [to_dev(a) for a in us], [to_dev(a) for a in lams]
    gz, gnu, gtz = to_dev(z), to_dev(nu), to_dev(tz)
    nodes = T.make_nodes(_slice_nodes(T, n, M, gx, gu, gl, rho=rho, eta2=eta2))
    regs = T.make_regs([dict(slice=0, kind=T.TOMO_REG_TIKHONOV, mu=0.1, rho=rho_z, z=gz, nu=gnu, tz=gtz)])
    m = T.TOMO_XUPDATE_SEGMENT if mode == "seg" else T.TOMO_XUPDATE_AVERAGE
    T.admm_consensus_reg(ctx, nodes, m, e2, None, None, regs)
    torch.cuda.synchronize()
    f = lambda a: a.astype(np.float64)
    if mode == "seg":
        xo = f(x).copy()
        rows = n // M
        for k in range(M):
            sl = slice(k * rows, (k + 1) * rows if k < M - 1 else n)
            xo[sl] = oreg.x_update_segment(f(x)[sl], f(us[k])[sl], f(lams[k])[sl], rho, f(tz)[sl], rho_z, eta2, e2)
    else:
        xo = oreg.x_update_average([f(a) for a in us], [f(a) for a in lams], [rho] * M, f(tz), rho_z)
    ex = rel_l2(gx.cpu().numpy(), xo)
    enu = rel_l2(gnu.cpu().numpy(), oreg.dual_update(f(nu), f(z), xo, rho_z))
    el = max(rel_l2(gl[k].cpu().numpy(), oadmm.dual_update(f(lams[k]), f(us[k]), xo, rho)) for k in range(M))
    log(f"  {mode}: x rel {ex:.2e}, nu rel {enu:.2e}, lambda rel {el:.2e}")
    assert ex <= 1e-5 and enu <= 1e-5 and el <= 1e-5


@pytest.mark.parametrize("quant,n,M", [("kmeans", 64, 4), ("dct", 64, 4), ("kmeans", 256, 2)])
def test_quantized_consensus_with_block_equals_unquantized_then_quantizer(mods, ctx, quant, n, M):
    """The K-means kernel runs the x-update with the block's term on load, the
    DCT path before its transform: both equal the unquantized consensus followed
    by the standalone quantizer on each segment, bit for bit.  256 x 256 on two
    nodes gives segments of 32768 values, past the register-resident limit
    (the K-means variant with the global workspace)."""
    T, _ = mods
    rng = np.random.default_rng(21)
    x, us, lams, z, nu, tz = _consensus_case(T, rng, n, M)
    outs = []
    for q in (None, quant):
        gx, gu, gl = to_dev(x), [to_dev(a) for a in us], [to_dev(a) for a in lams]
        gz, gnu, gtz = to_dev(z), to_dev(nu), to_dev(tz)
        nodes = T.make_nodes(_slice_nodes(T, n, M, gx, gu, gl))
        regs = T.make_regs([dict(slice=0, kind=T.TOMO_REG_TV, mu=0.1, rho=0.7, tv_iters=3, z=gz, nu=gnu, tz=gtz,
                                 p=torch.zeros((2, n, n), device="cuda"))])
        tq = None
        if q == "kmeans":
            tq = T.tomo_quant(T.TOMO_QUANT_KMEANS, 8, 30, 50)
        elif q == "dct":
            tq = T.tomo_quant(T.TOMO_QUANT_DCT, 0, 0, 50)
        T.admm_consensus_reg(ctx, nodes, T.TOMO_XUPDATE_SEGMENT, 10, tq, None, regs)
        torch.cuda.synchronize()
        outs.append(gx)
    ref = outs[0].clone()
    rows = n // M
    for k in range(M):
        seg = ref[k * rows:(k + 1) * rows].contiguous()
        a_hat = torch.empty_like(seg)
        if quant == "kmeans":
            T.quantize_kmeans(ctx, seg, 8, 30, a_hat=a_hat.reshape(-1))
        else:
            T.quantize_dct(ctx, seg, 50, a_hat=a_hat)
        ref[k * rows:(k + 1) * rows] = a_hat
    assert torch.equal(outs[1], ref)


def _tiny(T, A, ctx):
    w = synthdata.WORKLOADS["tiny"]
    truth = synthdata.phantom(w, 0)
    th = synthdata.angles(w.n_angles)
    clean = joseph.project(truth, th, w.n_bins)
    d = synthdata.add_gaussian_noise(clean, w.noise_level, synthdata.sinogram_seed(w, 0))
    parts = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)
    v0 = np.random.default_rng(0).standard_normal((w.n, w.n))
    L = max(stepsize.normal_operator_norm(th[p], w.n, w.n_bins, v0) for p in parts)
    return w, truth, th, d, parts, L


@pytest.mark.parametrize("mode,kind", [("seg", "tv"), ("avg", "tv"), ("seg", "tikhonov")])
def test_admm_with_block_matches_oracle(mods, ctx, mode, kind):
    """The tiny workload, 30 iterations without a quantizer, with a TV or
    Tikhonov block: RMSE trajectory and final x against the oracle; then the
    same run replayed from a captured graph equals the eager run bit for bit."""
    T, A = mods
    w, truth, th, d, parts, L = _tiny(T, A, ctx)
    rho = 1.0
    c = 0.1 if mode == "seg" else 1.0
    eta1 = float(np.float32(c / (L + rho)))
    mu, iters = 0.02, 30
    prob = oadmm.Problem(w.n, w.n_bins, [th[p] for p in parts], [d[p].astype(np.float64) for p in parts],
                         synthdata.segment_rows(w.n, w.n_nodes), truth.astype(np.float64))
    r = oreg.Reg(kind=kind, mu=mu, rho=rho, tv_iters=8)
    x_o, _, _, tr = oadmm.run(prob, iters, rho, eta1, w.inner_iters, w.eta2, w.x_iters, mode=mode, cast32=True,
                              reg=r)
    s = A.make_slice(ctx, w, d_host=d, truth_host=truth)
    s.eta1 = eta1
    reg = dict(kind=T.TOMO_REG_TV if kind == "tv" else T.TOMO_REG_TIKHONOV, mu=mu, tv_iters=8)
    m = T.TOMO_XUPDATE_SEGMENT if mode == "seg" else T.TOMO_XUPDATE_AVERAGE
    run = A.DADMM(ctx, [s], rho=rho, eta2=w.eta2, e1=w.inner_iters, e2=w.x_iters, mode=m, reg=reg)
    rm, xs = [], []
    for _ in range(iters):
        run.step()
        rm.append(run.rmse())
        xs.append(s.x.clone())
    rm, rm_o = np.array(rm), np.array(tr.rmse)
    ex = rel_l2(s.x.cpu().numpy(), x_o)
    log(f"  {mode}/{kind}: rmse gpu {rm[-1]:.6g} oracle {rm_o[-1]:.6g}, x rel {ex:.2e}")
    assert np.all(np.abs(rm - rm_o) <= 1e-4 * rm_o)
    assert ex <= 1e-4
    # the plain per-node loop and a captured graph give the same iterates
    s.zero()
    for k in range(3):
        run.step_plain()
        assert torch.equal(s.x, xs[k]), f"plain loop iteration {k} differs"
    s.zero()
    torch.cuda.synchronize()
    g = run.capture(1)
    s.zero()
    torch.cuda.synchronize()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(8, device="cuda").sum().item()
        assert torch.equal(s.x, xs[k]), f"graph replay {k} differs"


def test_blocks_on_many_slices_batched_pipelined_and_plain_agree(mods, ctx):
    """Three slices of different sizes, each with a TV block (different
    iteration counts per z-update would not be expressible per slice here, so
    the blocks share them), K-means exchange: the plain per-slice loop, the
    batched step, the pipelined graph (z-update beside the local update, next
    projection beside the consensus) and the alternating two-iteration graph
    give the same iterates bit for bit."""
    T, A = mods
    slices = []
    for i, (n, k, b, m) in enumerate([(96, 90, 136, 3), (64, 70, 91, 2), (128, 120, 182, 4)]):
        w = synthdata.Workload(f"rs{i}", 9, n, k, b, m, "interleaved", 5, "gaussian", 0.02, 4)
        s = A.make_slice(ctx, w, slice_idx=i)
        s.eta1 = A.step_size(ctx, s, 1.0, 0.1)
        slices.append(s)
    run = A.DADMM(ctx, slices, quant=T.tomo_quant(T.TOMO_QUANT_KMEANS, 8, 30, 50),
                  reg=dict(kind=T.TOMO_REG_TV, mu=0.05, tv_iters=6))
    for _ in range(4):
        run.step_plain()
    plain = [t.cpu().clone() for s in slices for t in [s.x, s.reg["z"], s.reg["nu"]]]
    for s in slices:
        s.zero()
    for _ in range(4):
        run.step()
    got = [t.cpu() for s in slices for t in [s.x, s.reg["z"], s.reg["nu"]]]
    assert all(torch.equal(a, b) for a, b in zip(got, plain)), "batched step differs from the plain loop"
    g = run.capture(1, pipelined=True)
    for s in slices:
        s.zero()
    torch.cuda.synchronize()
    run.prime()
    for _ in range(4):
        g.replay()
    torch.cuda.synchronize()
    got = [t.cpu() for s in slices for t in [s.x, s.reg["z"], s.reg["nu"]]]
    assert all(torch.equal(a, b) for a, b in zip(got, plain)), "pipelined graph differs from the plain loop"
    g2 = run.capture(2, pipelined=True, alternate=True)
    for s in slices:
        s.zero()
    torch.cuda.synchronize()
    run.prime()
    for _ in range(2):
        g2.replay()
    torch.cuda.synchronize()
    got = [t.cpu() for s in slices for t in [s.x, s.reg["z"], s.reg["nu"]]]
    assert all(torch.equal(a, b) for a, b in zip(got, plain)), "alternating graph differs from the plain loop"


def test_block_lowers_error_on_noisy_data(mods, ctx):
    """A TV block on strongly noisy data of a piecewise-constant phantom ends
    with a lower RMSE than the plain method after the same iterations."""
    T, A = mods
    w = synthdata.Workload("noisy", 7, 64, 90, 91, 4, "interleaved", 5, "gaussian", 0.08, 4, gray_levels=3)
    out = []
    for reg in (None, dict(kind=T.TOMO_REG_TV, mu=0.5, tv_iters=10)):
        s = A.make_slice(ctx, w)
        s.eta1 = A.step_size(ctx, s, 1.0, 0.5)
        run = A.DADMM(ctx, [s], reg=reg)
        for _ in range(60):
            run.step()
        out.append(run.rmse())
    log(f"  rmse plain {out[0]:.5g}, with TV block {out[1]:.5g}")
    assert out[1] < out[0]


def test_reg_argument_errors(mods, ctx):
    T, _ = mods
    n = 16
    t = {k: torch.zeros((n, n), device="cuda") for k in ("x", "z", "nu", "tz")}
    p = torch.zeros((2, n, n), device="cuda")
    nodes = T.make_nodes(_slice_nodes(T, n, 2, t["x"], [torch.zeros((n, n), device="cuda")] * 2,
                                      [torch.zeros((n, n), device="cuda")] * 2))
    good = dict(slice=0, kind=T.TOMO_REG_TV, mu=0.1, rho=1.0, tv_iters=4, tau=0.125, z=t["z"], nu=t["nu"],
                tz=t["tz"], p=p)
    T.admm_reg_update(ctx, nodes, T.make_regs([good]))
    bad = [dict(good, kind=7), dict(good, rho=0.0), dict(good, mu=-1.0), dict(good, tau=0.3), dict(good, tau=0.0),
           dict(good, tv_iters=-1), dict(good, slice=5), dict(good, p=None), dict(good, tz=t["x"])]
    for b in bad:
        with pytest.raises(T.TomoError):
            T.admm_reg_update(ctx, nodes, T.make_regs([b]))
    with pytest.raises(T.TomoError):
        T.admm_reg_update(ctx, nodes, T.make_regs([good, good]))      # two blocks for one slice
    with pytest.raises(T.TomoError):
        T.admm_consensus_reg(ctx, nodes, T.TOMO_XUPDATE_SEGMENT, 2, None, None, T.make_regs([dict(good, rho=-1.0)]))
    torch.cuda.synchronize()
