"""quantize_dct_noalloc (the codec with its range partials in the library's
per-GPU scratch array, for callers that cannot allocate) against quantize_dct
through the C ABI: identical codes, range and decoded values, on two calls in a
row, the second with a smaller input (the scratch keeps the first call's
partials)."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_common import log, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _call(T, ctx, name, a, q):
    rows, cols = a.shape
    coeffs = torch.full((rows, cols), -7, dtype=torch.int16, device="cuda")
    lohi = torch.full((2,), -1.0, dtype=torch.float32, device="cuda")
    a_hat = torch.full_like(a, -3.0)
    P = ctypes.c_void_p
    rc = getattr(T._lib, name)(ctx.handle, P(a.data_ptr()), rows, cols, cols, q, P(coeffs.data_ptr()),
                               P(a_hat.data_ptr()), P(lohi.data_ptr()), P(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, T._lib.tomo_last_error(ctx.handle)
    torch.cuda.synchronize()
    return coeffs.cpu().numpy(), lohi.cpu().numpy(), a_hat.cpu().numpy()


def test_noalloc_dct_equals_allocating_entry_point():
    require_gpu()
    from paper_2410_06106_amd import tomoadmm as T
    ctx = T.Context(0)
    rng = np.random.default_rng(11)
    # first a 2048-wide segment with 64 row chunks' worth of partials, then a
    # smaller one whose partials cover only the start of the scratch array
    for rows, cols, q in ((512, 2048, 50), (16, 64, 90)):
        yy, xx = np.mgrid[0:rows, 0:cols]
        a = to_dev((np.sin(xx / 11.0) * np.cos(yy / 7.0) + 0.2 * rng.standard_normal((rows, cols)))
                   .astype(np.float32))
        log(f"case quantize_dct_noalloc rows={rows} cols={cols} q={q}")
        want = _call(T, ctx, "quantize_dct", a, q)
        got = _call(T, ctx, "quantize_dct_noalloc", a, q)
        np.testing.assert_array_equal(got[0], want[0])
        np.testing.assert_array_equal(got[1], want[1])
        np.testing.assert_array_equal(got[2], want[2])
        np.testing.assert_array_equal(got[1], [a.min().item(), a.max().item()])
    # argument errors are reported before anything is launched
    bad = to_dev(np.zeros((12, 16), np.float32))
    P = ctypes.c_void_p
    assert T._lib.quantize_dct_noalloc(ctx.handle, P(bad.data_ptr()), 12, 16, 16, 50, None, P(bad.data_ptr()),
                                       None, None) == 1
