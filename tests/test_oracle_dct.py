"""Pins of the oracle's JPEG-style segment quantizer.

The 8x8 transform is checked against scipy.fft.dctn (type II, orthonormal),
the quality scaling against the table at quality 50 and hand-worked steps, and
the whole codec against the error bound of rounding coefficients to integers.
"""
import numpy as np
import pytest
import scipy.fft

from oracle import dct


def test_dct_matrix_orthonormal():
    C = dct.dct_matrix()
    np.testing.assert_allclose(C @ C.T, np.eye(8), atol=1e-15)


def test_blockwise_transform_is_scipy_dct2():
    rng = np.random.default_rng(0)
    a = rng.uniform(-2, 3, (16, 24)).astype(np.float32)
    res = dct.dct_quantize(a, 50)
    lo, hi = float(a.min()), float(a.max())
    v = (a.astype(np.float64) - lo) * 255.0 / (hi - lo) - 128.0
    for br in range(2):
        for bc in range(3):
            blk = v[8 * br:8 * br + 8, 8 * bc:8 * bc + 8]
            ref = scipy.fft.dctn(blk, type=2, norm="ortho")
            np.testing.assert_allclose(res.F[8 * br:8 * br + 8, 8 * bc:8 * bc + 8], ref, atol=1e-11)


def test_constant_block_has_only_dc():
    a = np.zeros((8, 16), np.float32)
    a[:, 8:] = 1.0                      # lo = 0, hi = 1: left block v = -128, right v = 127
    res = dct.dct_quantize(a, 50)
    F = res.F
    assert abs(F[0, 0] - 8 * (-128.0)) < 1e-9 and abs(F[0, 8] - 8 * 127.0) < 1e-9
    F = F.copy()
    F[0, 0] = F[0, 8] = 0.0
    assert np.abs(F).max() < 1e-9
    # the DC codes are round(8 v / 16); half-way 1016 / 16 = 63.5 rounds to even
    assert res.coeffs[0, 0] == -64 and res.coeffs[0, 8] == 64
    assert np.count_nonzero(res.coeffs) == 2
    # with unit steps (quality 100) the DC codes are exact and so is the block
    np.testing.assert_allclose(dct.dct_quantize(a, 100).a_hat, a, atol=1e-5)


def test_quality_scaling():
    np.testing.assert_array_equal(dct.quant_steps(50), dct.LUMA_TABLE)
    np.testing.assert_array_equal(dct.quant_steps(25), 2 * dct.LUMA_TABLE)   # scale 200
    q90 = dct.quant_steps(90)                                                # scale 20
    assert q90[0, 0] == 3 and q90[0, 2] == 2 and q90[7, 7] == 20
    assert np.all(dct.quant_steps(100) == 1)
    assert np.all(dct.quant_steps(1) == 255)
    with pytest.raises(ValueError):
        dct.quant_steps(0)


def test_quality_100_error_bound():
    """With every step 1, each coefficient moves by at most 1/2, so each sample
    moves by at most 0.5 (sum_u |C[u][x]|)^2 <= 4 levels of (hi - lo)/255."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal((32, 64)).astype(np.float32)
    res = dct.dct_quantize(a, 100)
    scale = (res.hi - res.lo) / 255.0
    C = dct.dct_matrix()
    bound = 0.5 * np.abs(C).sum(axis=0).max() ** 2 * scale
    err = np.abs(res.a_hat.astype(np.float64) - a)
    assert err.max() <= bound + 1e-6
    assert np.sqrt(np.mean(err ** 2)) <= 0.5 * scale


def test_lower_quality_loses_more():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((64, 64)).astype(np.float32)
    errs = [np.sqrt(np.mean((dct.dct_quantize(a, q).a_hat - a) ** 2)) for q in (90, 50, 25)]
    assert errs[0] < errs[1] < errs[2]


def test_degenerate_inputs():
    a = np.full((8, 8), 3.0, np.float32)
    res = dct.dct_quantize(a, 50)
    np.testing.assert_array_equal(res.a_hat, a)
    assert np.all(res.coeffs == 0)
    with pytest.raises(ValueError):
        dct.dct_quantize(np.zeros((8, 12), np.float32), 50)
