"""Intersection-length (chord) parallel-beam projector and its exact transpose
(float64): the discretisation Eq. 2 names, each measurement being the sum over
pixels of the pixel value times the length of the ray inside the pixel.

Geometry as in ``oracle.joseph``: pixel (r, c) is the unit square centred at
``x_c = c - (N-1)/2``, ``y_r = r - (N-1)/2``; the ray of bin b at angle theta is
the line ``x cos + y sin = t_b``, ``t_b = b - (B-1)/2``.

Length of a line inside one unit square.  With ``D = t_b - t_rc`` (signed
distance of the line from the pixel centre) it depends on D only, as a
trapezoid:

    L(D) = h * clamp((w2 - |D|) / (w2 - w1), 0, 1)
    h = 1 / max(|cos|, |sin|),  w1 = | |cos| - |sin| | / 2,  w2 = (|cos| + |sin|) / 2.

Support half-width w2 <= 1/sqrt(2), so a pixel meets at most the two bins
floor(s), floor(s) + 1 with s = t_rc + (B-1)/2, as in the Joseph model.

Conventions where the length is not determined by the formula:

* a cosine or sine within 1e-12 of zero is taken as exactly zero (the angle is
  axis-aligned; pi/2 in floating point has cos = 6e-17);
* for an axis-aligned line, pixels are half-open squares
  [x_c - 1/2, x_c + 1/2) x [y_r - 1/2, y_r + 1/2): a line on the edge between
  two pixels lies in the one on its +x (or +y) side and has length 1 there.
"""
from __future__ import annotations

import numpy as np

SNAP = 1e-12


def _centres(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - (n - 1) / 2.0


def trig(theta: float):
    """cos, sin with values within 1e-12 of zero set to zero (and the other to +-1)."""
    c, s = np.cos(theta), np.sin(theta)
    if abs(c) < SNAP:
        return 0.0, float(np.sign(s))
    if abs(s) < SNAP:
        return float(np.sign(c)), 0.0
    return float(c), float(s)


def footprint(n: int, n_bins: int, theta: float):
    """Per-pixel (b0, w0, w1) for one angle: length w0 on bin b0, w1 on b0 + 1."""
    c, s = trig(theta)
    t = _centres(n)[None, :] * c + _centres(n)[:, None] * s            # [r][c]
    pos = t + (n_bins - 1) / 2.0
    b0 = np.floor(pos)
    f = pos - b0                                                       # D = -f on b0, 1 - f on b0 + 1
    if c == 0.0 or s == 0.0:
        # axis-aligned: the line of bin b0 runs at coordinate (pixel centre - f)
        # along the axis its direction vector is normal to, oriented by the sign
        # of the nonzero component; inside the half-open pixel iff that offset is
        # in [-1/2, 1/2)
        sign = c if s == 0.0 else s
        on_b0 = (f <= 0.5) if sign > 0 else (f < 0.5)
        w0 = np.where(on_b0, 1.0, 0.0)
        return b0.astype(np.int64), w0, 1.0 - w0
    h = 1.0 / max(abs(c), abs(s))
    w1 = abs(abs(c) - abs(s)) / 2.0
    w2 = (abs(c) + abs(s)) / 2.0
    ramp = w2 - w1
    l0 = h * np.clip((w2 - f) / ramp, 0.0, 1.0)
    l1 = h * np.clip((w2 - (1.0 - f)) / ramp, 0.0, 1.0)
    return b0.astype(np.int64), l0, l1


def project(image: np.ndarray, thetas, n_bins: int) -> np.ndarray:
    """sino[k][b] = sum_{r,c} L_{k,b}(r, c) image[r][c]  (Eq. 2 with chord lengths)."""
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
    """The exact transpose of ``project``."""
    sg = np.asarray(sino, dtype=np.float64)
    thetas = np.asarray(thetas, dtype=np.float64).reshape(-1)
    n_bins = sg.shape[1]
    assert sg.shape[0] == thetas.size
    out = np.zeros((n, n), dtype=np.float64)
    for k, th in enumerate(thetas):
        b0, w0, w1 = footprint(n, n_bins, th)
        row = np.concatenate(([0.0], sg[k], [0.0]))
        i0 = np.clip(b0, -1, n_bins) + 1
        i1 = np.clip(b0 + 1, -1, n_bins) + 1
        out += w0 * row[i0] + w1 * row[i1]
    return out


def dense_matrix(n: int, n_bins: int, thetas) -> np.ndarray:
    """The full [K*B][N*N] matrix built from ``footprint`` (tiny grids only)."""
    thetas = np.asarray(thetas, dtype=np.float64).reshape(-1)
    A = np.zeros((thetas.size * n_bins, n * n))
    cols = np.arange(n * n)
    for k, th in enumerate(thetas):
        b0, w0, w1 = footprint(n, n_bins, th)
        for bb, ww in ((b0.reshape(-1), w0.reshape(-1)), (b0.reshape(-1) + 1, w1.reshape(-1))):
            ok = (bb >= 0) & (bb < n_bins)
            np.add.at(A, (k * n_bins + bb[ok], cols[ok]), ww[ok])
    return A
