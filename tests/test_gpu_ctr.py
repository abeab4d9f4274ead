"""GPU parity of the centralized baseline (Alg. 1, tomo_ctr_gd) against the
oracle, and its argument checks."""
import numpy as np
import pytest
import torch

import synthdata
from gpu_common import log, rel_l2, require_gpu, to_dev
from oracle import admm as oadmm
from oracle import joseph, stepsize

pytestmark = pytest.mark.gpu

TOMO_OK, TOMO_EINVAL = 0, 1        # status codes of include/tomoadmm.h


@pytest.fixture(scope="module")
def T():
    require_gpu()
    from paper_2410_06106_amd import tomoadmm
    return tomoadmm


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


# (n, angles, bins): one region; regions split by the projector (129); a
# detector narrower than the image and a 2 x 2 region grid (300)
@pytest.mark.parametrize("n,n_ang,n_bins,iters", [(64, 90, 91, 12), (129, 60, 150, 8), (300, 40, 200, 5)])
def test_ctr_gradient_descent_matches_oracle(T, ctx, n, n_ang, n_bins, iters):
    log(f"case ctr n={n} angles={n_ang} bins={n_bins} iters={iters}")
    w = synthdata.Workload("ctr", 6, n, n_ang, n_bins, 1, "interleaved", 6, "gaussian", 0.01, iters)
    truth = synthdata.phantom(w).astype(np.float64)
    th = synthdata.angles(n_ang)
    d = synthdata.add_gaussian_noise(joseph.project(truth, th, n_bins), 0.01, synthdata.sinogram_seed(w))
    v0 = np.random.default_rng(1).standard_normal((n, n))
    eta = float(np.float32(1.0 / stepsize.normal_operator_norm(th, n, n_bins, v0)))
    u_o = oadmm.ctr_gd(d.astype(np.float64), th, n, eta, iters)
    u = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    T.tomo_ctr_gd(ctx, to_dev(th, torch.float64), to_dev(d), u, eta, iters)
    err = rel_l2(u.cpu().numpy(), u_o)
    log(f"  rel-L2 {err:.3g}")
    assert err <= 1e-5


def test_ctr_continues_from_the_given_image(T, ctx):
    """Two calls of k and m steps equal one call of k + m steps (u carries the state)."""
    n, n_ang, nb = 48, 30, 69
    th = to_dev(synthdata.angles(n_ang), torch.float64)
    d = torch.from_numpy(np.random.default_rng(2).standard_normal((n_ang, nb)).astype(np.float32)).cuda()
    a = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    T.tomo_ctr_gd(ctx, th, d, a, 1e-3, 5)
    T.tomo_ctr_gd(ctx, th, d, b, 1e-3, 2)
    T.tomo_ctr_gd(ctx, th, d, b, 1e-3, 3)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_ctr_argument_errors(T, ctx):
    n, n_ang, nb = 16, 8, 23
    th = to_dev(synthdata.angles(n_ang), torch.float64)
    d = torch.zeros((n_ang, nb), dtype=torch.float32, device="cuda")
    u = torch.ones((n, n), dtype=torch.float32, device="cuda")
    g = T.tomo_geom(n, nb)
    lib, P = T._lib, T._dev
    base = (ctx.handle, g, P(th, torch.float64, "a"), n_ang, P(d, torch.float32, "d"), P(u, torch.float32, "u"))
    assert lib.tomo_ctr_gd(*base, 0.1, -1, None) == TOMO_EINVAL
    assert lib.tomo_ctr_gd(*base, float("inf"), 1, None) == TOMO_EINVAL
    assert lib.tomo_ctr_gd(*base, float("nan"), 1, None) == TOMO_EINVAL
    assert lib.tomo_ctr_gd(ctx.handle, g, base[2], 0, base[4], base[5], 0.1, 1, None) == TOMO_EINVAL
    assert lib.tomo_ctr_gd(ctx.handle, g, base[2], n_ang, None, base[5], 0.1, 1, None) == TOMO_EINVAL
    # u overlapping d
    assert lib.tomo_ctr_gd(ctx.handle, g, base[2], n_ang, base[4], base[4], 0.1, 1, None) == TOMO_EINVAL
    # iters == 0 leaves u untouched
    assert lib.tomo_ctr_gd(*base, 0.1, 0, None) == TOMO_OK
    torch.cuda.synchronize()
    assert float(u.min()) == 1.0 and float(u.max()) == 1.0
