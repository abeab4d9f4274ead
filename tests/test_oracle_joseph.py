"""Pins of the oracle's projector (Eq. 1-4) against things other than itself.

* the textbook Joseph algorithm (stepping along the driving axis with linear
  interpolation), written as plain loops on tiny grids;
* axis-aligned angles, where the projection reduces to column and row sums;
* analytic line integrals of a uniform disk and of ellipses (Kak and Slaney,
  Chapter 3, cited by the paper for the transform of Eq. 1), whose distance to
  the projection of the rasterised object must shrink like 1/N;
* the adjoint identity <P x, y> = <x, P^T y> and the dense transpose.
"""
import math

import numpy as np
import pytest

from oracle import joseph


def joseph_textbook(img, theta, n_bins):
    """Joseph's method: walk the ray one row (or column) at a time and
    interpolate linearly between the two nearest pixels of that row (column);
    scale by the path length per step."""
    n = img.shape[0]
    half = (n - 1) / 2.0
    c, s = math.cos(theta), math.sin(theta)
    out = np.zeros(n_bins)
    for b in range(n_bins):
        t = b - (n_bins - 1) / 2.0
        acc = 0.0
        if abs(c) >= abs(s):
            for r in range(n):
                y = r - half
                xi = (t - y * s) / c + half
                i0 = math.floor(xi)
                f = xi - i0
                v0 = img[r, i0] if 0 <= i0 < n else 0.0
                v1 = img[r, i0 + 1] if 0 <= i0 + 1 < n else 0.0
                acc += (1.0 - f) * v0 + f * v1
            out[b] = acc / abs(c)
        else:
            for col in range(n):
                x = col - half
                yi = (t - x * c) / s + half
                i0 = math.floor(yi)
                f = yi - i0
                v0 = img[i0, col] if 0 <= i0 < n else 0.0
                v1 = img[i0 + 1, col] if 0 <= i0 + 1 < n else 0.0
                acc += (1.0 - f) * v0 + f * v1
            out[b] = acc / abs(s)
    return out


@pytest.mark.parametrize("n,n_bins", [(6, 9), (7, 10), (8, 8), (5, 13)])
def test_matches_textbook_joseph(n, n_bins):
    rng = np.random.default_rng(n * 100 + n_bins)
    img = rng.standard_normal((n, n))
    thetas = np.concatenate([np.pi * np.arange(12) / 12, rng.uniform(0, np.pi, 5)])
    got = joseph.project(img, thetas, n_bins)
    for k, th in enumerate(thetas):
        ref = joseph_textbook(img, th, n_bins)
        np.testing.assert_allclose(got[k], ref, rtol=0, atol=1e-12)


def test_axis_angles_are_column_and_row_sums():
    rng = np.random.default_rng(3)
    n = 10
    img = rng.random((n, n))
    # same parity of N and B: bins sit on pixel centres
    p = joseph.project(img, [0.0, np.pi / 2], 12)
    np.testing.assert_allclose(p[0, 1:11], img.sum(axis=0), atol=1e-12)
    np.testing.assert_allclose(p[1, 1:11], img.sum(axis=1), atol=1e-12)
    assert p[0, 0] == 0 and p[0, 11] == 0
    # different parity: each bin sits between two pixel centres
    p = joseph.project(img, [0.0], 11)[0]
    cs = np.concatenate(([0.0], img.sum(axis=0), [0.0]))
    np.testing.assert_allclose(p, 0.5 * (cs[:-1] + cs[1:]), atol=1e-12)


def test_pixel_impulse_spreads_over_two_bins():
    n, n_bins = 9, 15
    img = np.zeros((n, n))
    img[2, 6] = 1.0
    thetas = np.random.default_rng(1).uniform(0, np.pi, 40)
    p = joseph.project(img, thetas, n_bins)
    for k, th in enumerate(thetas):
        assert np.count_nonzero(p[k] > 0) <= 2
        # the pixel's value is deposited as the area of a unit triangle (1/c * c)
        cth = max(abs(math.cos(th)), abs(math.sin(th)))
        assert 0.5 / cth - 1e-12 <= p[k].sum() <= 1.0 / cth + 1e-12


def _disk_error(n):
    R, x0, y0 = 0.3 * n, 0.1 * n, -0.05 * n
    half = (n - 1) / 2.0
    xs = np.arange(n) - half
    img = ((xs[None, :] - x0) ** 2 + (xs[:, None] - y0) ** 2 <= R * R).astype(float)
    n_bins = int(math.ceil(n * 1.5))
    thetas = np.pi * np.arange(12) / 12 + 0.05
    p = joseph.project(img, thetas, n_bins)
    tb = np.arange(n_bins) - (n_bins - 1) / 2.0
    ref = np.zeros_like(p)
    for k, th in enumerate(thetas):
        tau = tb - (x0 * math.cos(th) + y0 * math.sin(th))
        ref[k] = 2.0 * np.sqrt(np.maximum(R * R - tau ** 2, 0.0))
    return np.linalg.norm(p - ref) / np.linalg.norm(ref)


def _ellipse_error(n):
    a, b, phi, cx, cy = 0.35 * n, 0.18 * n, 0.6, 0.05 * n, 0.08 * n
    half = (n - 1) / 2.0
    xs = np.arange(n) - half
    X, Y = xs[None, :] - cx, xs[:, None] - cy
    P = X * math.cos(phi) + Y * math.sin(phi)
    Q = -X * math.sin(phi) + Y * math.cos(phi)
    img = ((P / a) ** 2 + (Q / b) ** 2 <= 1.0).astype(float)
    n_bins = int(math.ceil(n * 1.5))
    thetas = np.pi * np.arange(10) / 10 + 0.11
    p = joseph.project(img, thetas, n_bins)
    tb = np.arange(n_bins) - (n_bins - 1) / 2.0
    ref = np.zeros_like(p)
    for k, th in enumerate(thetas):
        a2 = a * a * math.cos(th - phi) ** 2 + b * b * math.sin(th - phi) ** 2
        tau = tb - (cx * math.cos(th) + cy * math.sin(th))
        ref[k] = 2.0 * a * b * np.sqrt(np.maximum(a2 - tau ** 2, 0.0)) / a2
    return np.linalg.norm(p - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("err_fn", [_disk_error, _ellipse_error])
def test_converges_to_analytic_line_integrals(err_fn):
    sizes = [32, 64, 128, 256]
    errs = [err_fn(n) for n in sizes]
    for n, e in zip(sizes, errs):
        assert e <= 3.0 / n, (n, e)
    for e1, e2 in zip(errs, errs[1:]):
        assert 1.4 <= e1 / e2 <= 2.8, errs


def test_adjoint_identity():
    rng = np.random.default_rng(7)
    n, n_bins = 33, 47
    thetas = rng.uniform(0, np.pi, 13)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((13, n_bins))
    Ax = joseph.project(x, thetas, n_bins)
    Aty = joseph.backproject(y, thetas, n)
    lhs, rhs = float(np.sum(Ax * y)), float(np.sum(x * Aty))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_dense_matrix_and_transpose():
    rng = np.random.default_rng(11)
    n, n_bins = 7, 12
    thetas = np.concatenate([[0.0, np.pi / 4, np.pi / 2], rng.uniform(0, np.pi, 4)])
    A = joseph.dense_matrix(n, n_bins, thetas)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((thetas.size, n_bins))
    np.testing.assert_allclose(A @ x.reshape(-1), joseph.project(x, thetas, n_bins).reshape(-1),
                               atol=1e-13)
    np.testing.assert_allclose(A.T @ y.reshape(-1), joseph.backproject(y, thetas, n).reshape(-1),
                               atol=1e-13)
    # the dense form agrees with the textbook loop as well
    for k, th in enumerate(thetas):
        np.testing.assert_allclose((A @ x.reshape(-1)).reshape(-1, n_bins)[k],
                                   joseph_textbook(x, th, n_bins), atol=1e-12)
