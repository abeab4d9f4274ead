"""Context workspace lifetime: a graph captured before the workspace grows
still replays correctly (the replaced allocation is kept), and tomo_release
frees cached plans after which calls rebuild them with identical results."""
import numpy as np
import pytest
import torch

import synthdata
from gpu_common import log, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    require_gpu()
    from paper_2410_06106_amd import tomoadmm
    return tomoadmm


def test_captured_projection_survives_workspace_growth(T):
    ctx = T.Context(0)
    rng = np.random.default_rng(0)
    n, nb = 300, 425
    ang = to_dev(synthdata.angles(24), torch.float64)
    img = to_dev(rng.random((n, n)).astype(np.float32))
    out = torch.empty((24, nb), dtype=torch.float32, device="cuda")
    T.tomo_project(ctx, ang, img, nb, out=out)          # allocates the split-region workspace
    torch.cuda.synchronize()
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            T.tomo_project(ctx, ang, img, nb, out=out)
    torch.cuda.current_stream().wait_stream(s)
    # a larger projection makes the context's workspace grow
    big = to_dev(rng.random((1024, 1024)).astype(np.float32))
    T.tomo_project(ctx, to_dev(synthdata.angles(64), torch.float64), big, 1449)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        log(f"  replay {rep}: max diff {float((out - ref).abs().max()):.3g}")
        assert torch.equal(out, ref)


def test_release_then_rebuild_gives_identical_results(T):
    ctx = T.Context(0)
    rng = np.random.default_rng(1)
    n, nb, k, M = 64, 91, 90, 4
    th = synthdata.angles(k)
    parts = synthdata.partition_angles(k, M, "interleaved")
    d = [to_dev(rng.standard_normal((len(p), nb)).astype(np.float32)) for p in parts]
    x = to_dev(rng.random((n, n)).astype(np.float32))
    u0 = [rng.random((n, n)).astype(np.float32) for _ in range(M)]
    lam = [torch.zeros((n, n), dtype=torch.float32, device="cuda") for _ in range(M)]

    def run():
        us = [to_dev(u) for u in u0]
        ents = [dict(n=n, n_bins=nb, angles=to_dev(th[p], torch.float64), slice=0, d=d[m], u=us[m], lam=lam[m],
                     x=x, seg_row0=16 * m, seg_rows=16, rho=1.0, eta1=1e-4, eta2=0.2) for m, p in enumerate(parts)]
        T.admm_local_update(ctx, T.make_nodes(ents), 3)
        torch.cuda.synchronize()
        return [u.cpu().numpy() for u in us]

    a = run()
    T.tomo_release(ctx)
    b = run()
    for ua, ub in zip(a, b):
        np.testing.assert_array_equal(ua, ub)
