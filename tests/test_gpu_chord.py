"""GPU parity of the chord-length model (TOMO_OPT_PROJ_MODEL = 1, the
intersection lengths of Eq. 2) against oracle/chord.py, through the C ABI:
projector and backprojector at ragged sizes and on the exact axis-aligned
angles where rays lie on pixel edges, the adjoint identity, every projector
launch option, the local update (Alg. 2) and the centralized baseline (Alg. 1).
Tolerance as for the Joseph model: rel-L2 <= 1e-5 (float32 values, float64
positions on the GPU, float64 oracle)."""
import numpy as np
import pytest
import torch

import synthdata
from gpu_common import log, rel_l2, require_gpu, to_dev
from oracle import admm as oadmm
from oracle import chord, joseph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    require_gpu()
    from paper_2410_06106_amd import tomoadmm
    return tomoadmm


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    T.tomo_set_option(c, T.TOMO_OPT_PROJ_MODEL, 1)
    return c


SPECIAL = np.array([0.0, np.pi / 4, np.pi / 2, 3 * np.pi / 4, np.pi - 1e-9, 1e-9, 1e-3, np.pi / 2 + 2e-3])


def _angles(kind, k, rng):
    if kind == "special":
        return SPECIAL
    if kind == "uniform":
        return synthdata.angles(k)          # includes 0 and pi/2 exactly
    return rng.uniform(0, np.pi, k)


CASES = [  # (n, n_bins, angle kind, n_angles); n and n_bins of different parity put rays on pixel edges
    (1, 1, "special", 0), (7, 11, "special", 0), (8, 9, "special", 0), (8, 8, "random", 9),
    (64, 91, "uniform", 90), (100, 143, "random", 13), (129, 150, "uniform", 30), (513, 727, "random", 6),
    (300, 200, "uniform", 8),    # detector narrower than the image
]


@pytest.mark.parametrize("n,nb,kind,k", CASES)
def test_chord_project_and_backproject_match_oracle(T, ctx, n, nb, kind, k):
    log(f"case chord n={n} nb={nb} kind={kind} k={k}")
    rng = np.random.default_rng(n * 5 + nb)
    th = _angles(kind, k, rng)
    img = rng.random((n, n)).astype(np.float32)
    sino = rng.standard_normal((th.size, nb)).astype(np.float32)
    ang = to_dev(th, torch.float64)
    got_p = T.tomo_project(ctx, ang, to_dev(img), nb).cpu().numpy()
    got_b = T.tomo_backproject(ctx, ang, to_dev(sino), n).cpu().numpy()
    ep, eb = rel_l2(got_p, chord.project(img, th, nb)), rel_l2(got_b, chord.backproject(sino, th, n))
    log(f"  rel-L2 project {ep:.3g} backproject {eb:.3g}")
    assert ep <= 1e-5 and eb <= 1e-5


def test_chord_axis_aligned_edges_exactly(T, ctx):
    """n = 4, 5 bins: at 0 and pi/2 every ray lies on a pixel edge; the half-open
    convention puts each in one pixel, so the sums are exact column/row sums."""
    img = (np.arange(16, dtype=np.float32).reshape(4, 4) + 1)
    got = T.tomo_project(ctx, to_dev(np.array([0.0, np.pi / 2]), torch.float64), to_dev(img), 5).cpu().numpy()
    np.testing.assert_array_equal(got[0], np.concatenate([img.sum(axis=0), [0.0]]))
    np.testing.assert_array_equal(got[1], np.concatenate([img.sum(axis=1), [0.0]]))


def test_chord_adjoint_identity(T, ctx):
    rng = np.random.default_rng(8)
    n, nb = 96, 137
    th = rng.uniform(0, np.pi, 17)
    th[:2] = (0.0, np.pi / 2)
    x = rng.standard_normal((n, n)).astype(np.float32)
    y = rng.standard_normal((th.size, nb)).astype(np.float32)
    ang = to_dev(th, torch.float64)
    px = T.tomo_project(ctx, ang, to_dev(x), nb).cpu().numpy().astype(np.float64)
    pty = T.tomo_backproject(ctx, ang, to_dev(y), n).cpu().numpy().astype(np.float64)
    lhs, rhs = float(np.sum(px * y)), float(np.sum(x * pty))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(px) * np.linalg.norm(y)


@pytest.mark.parametrize("band,job_wgs", [(16, 1), (16, 64), (32, 1), (32, 64), (32, 4096)])
def test_chord_launch_options_match_oracle(T, band, job_wgs):
    c = T.Context(0)
    T.tomo_set_option(c, T.TOMO_OPT_PROJ_MODEL, 1)
    T.tomo_set_option(c, T.TOMO_OPT_PROJ_BAND, band)
    T.tomo_set_option(c, T.TOMO_OPT_PROJ_JOB_WGS, job_wgs)
    rng = np.random.default_rng(band + job_wgs)
    n, nb = 300, 425
    th = synthdata.angles(24)
    img = rng.random((n, n)).astype(np.float32)
    got = T.tomo_project(c, to_dev(th, torch.float64), to_dev(img), nb).cpu().numpy()
    assert rel_l2(got, chord.project(img, th, nb)) <= 1e-5


def test_chord_ignores_the_region_resident_kernel(T, ctx):
    """The region-resident kernel is Joseph-only: with model 1 the band kernel runs."""
    c = T.Context(0)
    T.tomo_set_option(c, T.TOMO_OPT_PROJ_MODEL, 1)
    T.tomo_set_option(c, T.TOMO_OPT_PROJ_KERNEL, 1)
    rng = np.random.default_rng(3)
    th = to_dev(synthdata.angles(30), torch.float64)
    img = to_dev(rng.random((200, 200)).astype(np.float32))
    a = T.tomo_project(c, th, img, 283).cpu().numpy()
    b = T.tomo_project(ctx, th, img, 283).cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_chord_equals_joseph_at_45_degrees(T, ctx):
    j = T.Context(0)
    rng = np.random.default_rng(5)
    th = to_dev(np.array([np.pi / 4, 3 * np.pi / 4]), torch.float64)
    img = to_dev(rng.random((64, 64)).astype(np.float32))
    a = T.tomo_project(ctx, th, img, 91).cpu().numpy()
    b = T.tomo_project(j, th, img, 91).cpu().numpy()
    assert rel_l2(a, b) <= 1e-6


def test_chord_local_update_matches_oracle(T, ctx):
    n, nb, k, M = 64, 91, 90, 4
    rng = np.random.default_rng(21)
    th = synthdata.angles(k)
    parts = synthdata.partition_angles(k, M, "interleaved")
    truth = rng.random((n, n))
    d = [chord.project(truth, th[p], nb) for p in parts]
    x = rng.random((n, n)).astype(np.float32)
    us = [rng.random((n, n)).astype(np.float32) for _ in range(M)]
    lams = [(0.1 * rng.standard_normal((n, n))).astype(np.float32) for _ in range(M)]
    rho, eta1, e1 = 1.0, 1e-4, 5
    X = to_dev(x)
    U = [to_dev(u) for u in us]
    Lm = [to_dev(l) for l in lams]
    ents = [dict(n=n, n_bins=nb, angles=to_dev(th[p], torch.float64), slice=0, d=to_dev(d[m].astype(np.float32)),
                 u=U[m], lam=Lm[m], x=X, seg_row0=16 * m, seg_rows=16, rho=rho, eta1=eta1, eta2=0.2)
            for m, p in enumerate(parts)]
    T.admm_local_update(ctx, T.make_nodes(ents), e1)
    for m, p in enumerate(parts):
        ref = oadmm.local_update(us[m], x, lams[m], d[m].astype(np.float32), th[p], rho, eta1, e1, proj=chord)
        assert rel_l2(U[m].cpu().numpy(), ref) <= 1e-5


def test_chord_ctr_matches_oracle(T, ctx):
    n, k, nb, iters = 64, 90, 91, 6
    rng = np.random.default_rng(2)
    th = synthdata.angles(k)
    d = chord.project(rng.random((n, n)), th, nb).astype(np.float32)
    eta = 1e-4
    u = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    T.tomo_ctr_gd(ctx, to_dev(th, torch.float64), to_dev(d), u, eta, iters)
    ref = oadmm.ctr_gd(d.astype(np.float64), th, n, eta, iters, proj=chord)
    assert rel_l2(u.cpu().numpy(), ref) <= 1e-5
    # and it differs from the Joseph model (the option is in effect)
    assert rel_l2(u.cpu().numpy(), oadmm.ctr_gd(d.astype(np.float64), th, n, eta, iters, proj=joseph)) > 1e-4
