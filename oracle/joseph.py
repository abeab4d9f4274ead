"""Joseph parallel-beam projector and its exact transpose (float64).

Section 2.1 (Eq. 1) fixes the ray geometry: the ray at angle theta and signed
detector offset t is the line ``x cos(theta) + y sin(theta) = t``.  Eq. 2-4
discretise the transform into ``d = P u``.  The system matrix used here is the
Joseph one (linear interpolation along the driving axis), which in closed form is

    P[(theta, b), (r, c)] = max(0, 1 - |t_b - t_rc| / c_theta) / c_theta

with pixel centre ``x_c = c - (N-1)/2``, ``y_r = r - (N-1)/2`` (pixel units, y
grows with the row index), bin centre ``t_b = b - (B-1)/2``,
``t_rc = x_c cos(theta) + y_r sin(theta)`` and
``c_theta = max(|cos(theta)|, |sin(theta)|)``.  Every pixel touches at most two
bins per angle: with ``s = t_rc + (B-1)/2``, bins ``floor(s)`` and
``floor(s) + 1``.  Bins outside ``[0, B)`` are dropped (zero padding).
"""
from __future__ import annotations

import numpy as np


def _centres(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - (n - 1) / 2.0


def footprint(n: int, n_bins: int, theta: float):
    """Per-pixel (b0, w0, w1) for one angle: pixel weight w0 on bin b0, w1 on b0+1."""
    c, s = np.cos(theta), np.sin(theta)
    cth = max(abs(c), abs(s))
    t = _centres(n)[None, :] * c + _centres(n)[:, None] * s          # [r][c]
    pos = t + (n_bins - 1) / 2.0
    b0 = np.floor(pos)
    f = pos - b0
    w0 = np.maximum(0.0, 1.0 - f / cth) / cth
    w1 = np.maximum(0.0, 1.0 - (1.0 - f) / cth) / cth
    return b0.astype(np.int64), w0, w1


def project(image: np.ndarray, thetas, n_bins: int) -> np.ndarray:
    """sino[k][b] = sum_{r,c} P[(theta_k, b), (r, c)] image[r][c]  (Eq. 2)."""
    img = np.asarray(image, dtype=np.float64)
    n = img.shape[0]
    assert img.shape == (n, n)
    thetas = np.asarray(thetas, dtype=np.float64).reshape(-1)
    out = np.zeros((thetas.size, n_bins), dtype=np.float64)
    for k, th in enumerate(thetas):
        b0, w0, w1 = footprint(n, n_bins, th)
        for bb, ww in ((b0, w0), (b0 + 1, w1)):
            ok = (bb >= 0) & (bb < n_bins)
            out[k] += np.bincount(bb[ok], weights=(ww * img)[ok], minlength=n_bins)
    return out


def backproject(sino: np.ndarray, thetas, n: int) -> np.ndarray:
    """image[r][c] = sum_{k,b} P[(theta_k, b), (r, c)] sino[k][b]  (P transposed)."""
    sg = np.asarray(sino, dtype=np.float64)
    thetas = np.asarray(thetas, dtype=np.float64).reshape(-1)
    n_bins = sg.shape[1]
    assert sg.shape[0] == thetas.size
    out = np.zeros((n, n), dtype=np.float64)
    for k, th in enumerate(thetas):
        b0, w0, w1 = footprint(n, n_bins, th)
        row = np.concatenate(([0.0], sg[k], [0.0]))                  # index b+1, pads at -1 and B
        i0 = np.clip(b0, -1, n_bins) + 1
        i1 = np.clip(b0 + 1, -1, n_bins) + 1
        out += w0 * row[i0] + w1 * row[i1]
    return out


def dense_matrix(n: int, n_bins: int, thetas) -> np.ndarray:
    """The full [K*B][N*N] matrix from the closed form (tiny grids only)."""
    thetas = np.asarray(thetas, dtype=np.float64).reshape(-1)
    xc = _centres(n)
    tb = np.arange(n_bins, dtype=np.float64) - (n_bins - 1) / 2.0
    rows = []
    for th in thetas:
        c, s = np.cos(th), np.sin(th)
        cth = max(abs(c), abs(s))
        t = (xc[None, :] * c + xc[:, None] * s).reshape(-1)          # pixel order r*N + c
        rows.append(np.maximum(0.0, 1.0 - np.abs(tb[:, None] - t[None, :]) / cth) / cth)
    return np.concatenate(rows, axis=0)
