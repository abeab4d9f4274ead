"""Pins of the chord-length oracle (oracle/chord.py) against routes it does not
take: exact clipping of each line against each pixel square, the chord of the
whole image square (lengths add up along a line), the half-open pixel
convention for lines on pixel edges, the Joseph model where the two coincide
(45 degrees), and the transpose."""
import math

import numpy as np
import pytest

from oracle import chord, joseph


def clip_length(t, theta, xc, yr):
    """Length of the line x cos + y sin = t inside the closed unit square centred at
    (xc, yr), by intersecting its parameter interval with the two slabs."""
    c, s = math.cos(theta), math.sin(theta)
    px, py = t * c, t * s                     # the point of the line closest to the origin
    dx, dy = -s, c                            # its direction
    lo, hi = -math.inf, math.inf
    for p, d, centre in ((px, dx, xc), (py, dy, yr)):
        a, b = centre - 0.5 - p, centre + 0.5 - p
        if abs(d) < 1e-15:
            if not (a <= 0.0 <= b):
                return 0.0
            continue
        l1, l2 = sorted((a / d, b / d))
        lo, hi = max(lo, l1), min(hi, l2)
    return max(0.0, hi - lo)


@pytest.mark.parametrize("theta", [0.3, 1.0, 2.0, 2.9, math.pi / 4 + 0.01, 1e-3, math.pi / 2 - 2e-3])
def test_matches_exact_clipping(theta):
    n, nb = 6, 9
    A = chord.dense_matrix(n, nb, [theta])
    xc = np.arange(n) - (n - 1) / 2.0
    tb = np.arange(nb) - (nb - 1) / 2.0
    for b in range(nb):
        for r in range(n):
            for c in range(n):
                assert A[b, r * n + c] == pytest.approx(clip_length(tb[b], theta, xc[c], xc[r]), abs=1e-12)


@pytest.mark.parametrize("theta", [0.2, 0.7, 1.3, 2.2, 3.0])
def test_constant_image_gives_the_chord_of_the_image_square(theta):
    n, nb = 24, 41
    sino = chord.project(np.ones((n, n)), [theta], nb)[0]
    c, s = abs(math.cos(theta)), abs(math.sin(theta))
    w1, w2, h = abs(c - s) / 2, (c + s) / 2, 1 / max(c, s)
    t = (np.arange(nb) - (nb - 1) / 2.0) / n                  # the square of side n scaled to side 1
    want = n * h * np.clip((w2 - np.abs(t)) / (w2 - w1), 0.0, 1.0)
    np.testing.assert_allclose(sino, want, atol=1e-11)


def test_axis_aligned_lines_on_pixel_edges_use_half_open_pixels():
    # n = 4 and 5 bins: at theta = 0 and pi/2 every ray lies on a pixel edge;
    # the ray at the image's -x (-y) edge is inside, the one at the +x (+y) edge is not
    img = np.arange(16, dtype=np.float64).reshape(4, 4) + 1
    s0 = chord.project(img, [0.0], 5)[0]
    np.testing.assert_array_equal(s0, np.concatenate([img.sum(axis=0), [0.0]]))
    s90 = chord.project(img, [np.pi / 2], 5)[0]               # cos(pi/2) = 6e-17 is snapped to 0
    np.testing.assert_array_equal(s90, np.concatenate([img.sum(axis=1), [0.0]]))
    # theta = pi: t = -x, the orientation flips and the other edge ray is inside
    s180 = chord.project(img, [np.pi], 5)[0]
    np.testing.assert_array_equal(s180, np.concatenate([[0.0], img.sum(axis=0)[::-1]]))
    # same parity: rays through pixel centres, every column once
    np.testing.assert_array_equal(chord.project(img, [0.0], 4)[0], img.sum(axis=0))


def test_equals_joseph_at_45_degrees():
    for theta in (math.pi / 4, 3 * math.pi / 4):
        np.testing.assert_allclose(chord.dense_matrix(7, 11, [theta]), joseph.dense_matrix(7, 11, [theta]),
                                   atol=1e-12)


def test_each_pixel_meets_at_most_two_bins_and_transpose_is_exact():
    rng = np.random.default_rng(4)
    n, nb = 9, 14
    th = np.sort(rng.uniform(0, np.pi, 11))
    th[0] = 0.0
    A = chord.dense_matrix(n, nb, th)
    assert (np.count_nonzero(A.reshape(len(th), nb, n * n), axis=1) <= 2).all()
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((len(th), nb))
    np.testing.assert_allclose(chord.project(x, th, nb).reshape(-1), A @ x.reshape(-1), atol=1e-12)
    np.testing.assert_allclose(chord.backproject(y, th, n).reshape(-1), A.T @ y.reshape(-1), atol=1e-12)
