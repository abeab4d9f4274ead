"""Checks of the synthetic input recipes that the oracle and the GPU path share
(no method arithmetic): the piecewise-constant phantom of the quality studies
and the node split of Section 3.2."""
import numpy as np
import pytest

import synthdata


@pytest.mark.parametrize("levels", [2, 3, 5])
def test_painted_phantom_has_exactly_the_requested_gray_levels(levels):
    rng = np.random.default_rng(7)
    img = synthdata.paint_levels(synthdata.ellipse_params(8, rng), 96, levels)
    vals = np.unique(img)
    np.testing.assert_allclose(vals, np.arange(levels) / (levels - 1), atol=0)
    assert img[0, 0] == 0.0 and img[48, 48] > 0.0          # background corner, body centre


def test_painted_phantom_rejects_a_single_level():
    with pytest.raises(ValueError):
        synthdata.paint_levels(synthdata.ellipse_params(2, np.random.default_rng(0)), 16, 1)


def test_quality_study_workload_matches_section_3():
    w = synthdata.WORKLOADS["elbow"]
    img = synthdata.phantom(w)
    assert img.shape == (512, 512) and img.dtype == np.float32
    assert sorted(np.unique(img).tolist()) == [0.0, 0.5, 1.0]
    parts = synthdata.partition_angles(w.n_angles, w.n_nodes, w.split)
    # two nodes: even- and odd-indexed angles, 402 each
    assert [len(p) for p in parts] == [402, 402]
    assert np.all(parts[0] % 2 == 0) and np.all(parts[1] % 2 == 1)
    # ten nodes: 4 x 81 + 6 x 80, node m holds m, m + 10, ...
    p10 = synthdata.partition_angles(w.n_angles, 10, w.split)
    assert [len(p) for p in p10] == [81] * 4 + [80] * 6
    assert p10[0][:3].tolist() == [0, 10, 20] and p10[1][-1] == 801
