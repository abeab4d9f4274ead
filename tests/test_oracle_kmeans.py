"""Pins of the oracle's scalar K-means quantizer (Alg. 5).

Checked against brute force (the optimal k-level scalar quantizer of a sorted
vector is a set of contiguous runs; enumerate every split on tiny inputs), the
Lloyd fixed-point conditions (each centre is its cluster's mean, each value sits
with a nearest centre), the paper's remark that an image with three grey levels
is represented exactly by K = 3, and degenerate cases.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle.kmeans import assign, initial_centres, kmeans_quantize


def _brute_force_distortion(a, k):
    s = np.sort(np.asarray(a, dtype=np.float64))
    n = s.size
    best = np.inf
    for cuts in itertools.combinations(range(1, n), k - 1):
        edges = (0,) + cuts + (n,)
        d = sum(((s[i:j] - s[i:j].mean()) ** 2).sum() for i, j in zip(edges, edges[1:]))
        best = min(best, d)
    return best


def _distortion(a, res):
    return float(((np.asarray(a, np.float64) - res.a_hat.astype(np.float64)) ** 2).sum())


@pytest.mark.parametrize("seed", range(12))
def test_never_beats_brute_force_and_matches_it_when_separated(seed):
    rng = np.random.default_rng(seed)
    n, k = int(rng.integers(5, 13)), int(rng.integers(1, 5))
    a = rng.standard_normal(n).astype(np.float32)
    res = kmeans_quantize(a, k)
    dstar = _brute_force_distortion(a, min(k, n))
    assert _distortion(a, res) >= dstar * (1 - 1e-6) - 1e-9
    # well separated clusters: Lloyd from spread-out initial centres finds the optimum
    centres = np.array([0.0, 10.0, 20.0, 30.0])[:k]
    b = (centres[rng.integers(0, k, n)] + 0.3 * rng.standard_normal(n)).astype(np.float32)
    b[:k] = centres                      # every cluster occupied
    res = kmeans_quantize(b, k)
    assert abs(_distortion(b, res) - _brute_force_distortion(b, k)) <= 1e-4 * max(1.0, _distortion(b, res))


@pytest.mark.parametrize("seed", range(5))
def test_lloyd_fixed_point_conditions(seed):
    rng = np.random.default_rng(100 + seed)
    a = np.concatenate([rng.normal(m, 0.05, 300) for m in (0.0, 0.4, 1.0, 1.7)]).astype(np.float32)
    res = kmeans_quantize(a, 6, max_iter=200)
    assert res.iters < 200
    a64, c64 = a.astype(np.float64), res.centroids.astype(np.float64)
    for j in range(6):
        sel = res.labels == j
        if sel.any():
            mean = a64[sel].mean()
            assert abs(c64[j] - mean) <= 2 * np.spacing(np.float32(abs(mean))) + 1e-12
    dist = np.abs(a64[:, None] - c64[None, :])
    own = dist[np.arange(a.size), res.labels]
    assert np.all(own <= dist.min(axis=1) + 2 * np.spacing(np.abs(a).max()))
    np.testing.assert_array_equal(res.a_hat, res.centroids[res.labels])


def test_three_grey_levels_are_exact_with_three_clusters():
    """Section 3.3: an image with three grey levels needs only K = 3."""
    rng = np.random.default_rng(9)
    levels = np.array([0.0, 0.35, 1.0], dtype=np.float32)
    a = levels[rng.integers(0, 3, 5000)]
    res = kmeans_quantize(a, 3)
    np.testing.assert_array_equal(res.a_hat, a)
    np.testing.assert_array_equal(np.sort(res.centroids), levels)


def test_single_cluster_is_the_mean():
    rng = np.random.default_rng(1)
    a = rng.uniform(-3, 5, 4097).astype(np.float32)
    res = kmeans_quantize(a, 1)
    mean = a.astype(np.float64).mean()
    assert abs(float(res.centroids[0]) - mean) <= np.spacing(np.float32(abs(mean)))
    assert np.all(res.labels == 0)


def test_labels_are_monotone_in_the_value():
    rng = np.random.default_rng(2)
    a = rng.standard_normal(3000).astype(np.float32)
    res = kmeans_quantize(a, 16)
    order = np.argsort(a, kind="stable")
    c = res.centroids
    assert np.all(np.diff(c) >= 0)
    assert np.all(np.diff(res.labels[order].astype(int)) >= 0)


def test_degenerate_inputs():
    a = np.full(17, 2.5, np.float32)
    res = kmeans_quantize(a, 4)
    assert res.iters == 0 and np.all(res.labels == 0) and np.all(res.centroids == 2.5)
    np.testing.assert_array_equal(res.a_hat, a)
    res = kmeans_quantize(np.zeros(0, np.float32), 4)
    assert res.labels.size == 0
    with pytest.raises(ValueError):
        kmeans_quantize(np.array([0.0, np.nan], np.float32), 2)
    with pytest.raises(ValueError):
        kmeans_quantize(np.array([0.0, 1.0], np.float32), 0)
    # more clusters than distinct values: the extra centres stay where they were put
    res = kmeans_quantize(np.array([0.0, 1.0, 1.0, 0.0], np.float32), 8)
    np.testing.assert_array_equal(res.a_hat, [0.0, 1.0, 1.0, 0.0])


@pytest.mark.parametrize("seed", range(6))
def test_assignment_is_the_exact_nearest_centre(seed):
    """The midpoint count equals the nearest centre found in exact rational
    arithmetic (distinct increasing centres), a value at a midpoint going to
    the lower centre."""
    rng = np.random.default_rng(50 + seed)
    k = int(rng.integers(2, 12))
    c = np.unique(rng.uniform(-2, 3, k).astype(np.float32))
    a = rng.uniform(-3, 4, 400).astype(np.float32)
    mids = ((c[:-1].astype(np.float64) + c[1:]) / 2).astype(np.float32)
    exact_mid = mids[mids.astype(np.float64) * 2 == c[:-1].astype(np.float64) + c[1:]]
    a = np.concatenate([a, exact_mid, c])
    got = assign(a, c)
    cf = [Fraction(float(x)) for x in c]
    for v, lab in zip(a, got):
        d = [abs(Fraction(float(v)) - x) for x in cf]
        assert lab == d.index(min(d)), (v, lab)


def test_initial_centres_are_the_cell_midpoints():
    """Alg. 5's initialisation (reading R14): the centres of k equal cells of
    [lo, hi].  Values chosen so that every centre is exact in float32."""
    np.testing.assert_array_equal(initial_centres(0.0, 1.0, 4), [0.125, 0.375, 0.625, 0.875])
    np.testing.assert_array_equal(initial_centres(-3.0, 1.0, 4), [-2.5, -1.5, -0.5, 0.5])
    np.testing.assert_array_equal(initial_centres(-8.0, -6.0, 2), [-7.5, -6.5])
    np.testing.assert_array_equal(initial_centres(2.0, 6.0, 1), [4.0])


@pytest.mark.parametrize("lo,hi,k", [(0.0, 1.0, 4), (-3.0, 1.0, 4), (-8.0, -6.0, 8), (-1.0, 3.0, 16)])
def test_zero_lloyd_iterations_is_the_uniform_quantizer(lo, hi, k):
    """With max_iter = 0 the output is the initial quantizer: the uniform
    k-cell quantizer of [lo, hi] (textbook midrise form), every value mapped to
    the midpoint of its cell, cell edges lo + (hi - lo) j / k.  Values sit away
    from the edges so the float32 rounding of a value cannot move it across."""
    rng = np.random.default_rng(k + int(hi - lo))
    w = (hi - lo) / k
    cell = rng.integers(0, k, 2000)
    frac = rng.uniform(0.01, 0.99, 2000)
    a = (lo + (cell + frac) * w).astype(np.float32)
    a[0], a[1] = lo, hi                   # the range is exactly [lo, hi]
    cell[0], cell[1] = 0, k - 1
    res = kmeans_quantize(a, k, max_iter=0)
    assert res.iters == 0
    np.testing.assert_array_equal(res.centroids, lo + (np.arange(k) + 0.5) * w)
    np.testing.assert_array_equal(res.labels, cell)
    np.testing.assert_array_equal(res.a_hat, (lo + (cell + 0.5) * w).astype(np.float32))
