"""Pins of the evaluation formulas (Eq. 19, 20, 25-27), the angle partition
of Section 3.2 and the compression arithmetic of Section 3.3, against the small
worked examples stored under tests/golden/."""
import math
import os

import numpy as np

import synthdata
from oracle import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def test_partition_matches_paper_example():
    g = {r[0]: r[1:] for r in _rows("partition_804x10.txt")}
    parts = synthdata.partition_angles(int(g["n_angles"][0]), int(g["n_nodes"][0]), "interleaved")
    assert [len(p) for p in parts] == [int(v) for v in g["counts"]]
    assert list(parts[0][:3]) == [int(v) for v in g["node0_first"]]
    assert parts[0][-1] == int(g["node0_last"][0])
    assert list(parts[1][:3]) == [int(v) for v in g["node1_first"]]
    assert parts[1][-1] == int(g["node1_last"][0])
    two = synthdata.partition_angles(804, 2, "interleaved")
    assert [len(p) for p in two] == [int(v) for v in g["two_node_counts"]]
    assert np.all(two[0] % 2 == 0) and np.all(two[1] % 2 == 1)
    # every angle is held exactly once, in either split
    for split in ("interleaved", "contiguous"):
        allidx = np.sort(np.concatenate(synthdata.partition_angles(804, 10, split)))
        np.testing.assert_array_equal(allidx, np.arange(804))


def test_memory_and_communication_models():
    X = 2048 * 2048 * 4 / 2 ** 20
    D = 2048 * 2048 * 4 / 2 ** 20
    for M, mem, comm in ((int(r[0]), float(r[1]), float(r[2])) for r in _rows("memory_comm_2048.txt")):
        assert metrics.memory_per_node(D, X, M) == mem
        assert metrics.comm_per_node(X, M) == comm
    assert abs(metrics.memory_per_node(D, X, 10 ** 9) - 3 * X) < 1e-6
    assert abs(metrics.comm_per_node(X, 10 ** 9) - 2 * X) < 1e-6


def test_compression_arithmetic():
    for K, bits, fold in ((int(r[0]), int(r[1]), float(r[2])) for r in _rows("compression.txt")):
        assert metrics.kmeans_bits(K) == bits
        assert 32 / bits == fold
        assert metrics.comm_per_node(32.0, 2, bits) == 32.0 / fold


def test_rmse_psnr_nsd():
    o = np.array([[0.0, 1.0], [2.0, 3.0]])
    x = o + np.array([[1.0, -1.0], [1.0, -1.0]])
    assert metrics.rmse(x, o) == 1.0
    assert abs(metrics.psnr(x, o) - 20 * math.log10(3.0)) < 1e-12
    assert abs(metrics.psnr(x, o, i_max=10.0) - 20.0) < 1e-12
    assert abs(metrics.nsd_percent(0.984, 410.0) - 0.24) < 1e-12


def test_segments_tile_the_image():
    for n, m in ((64, 4), (512, 16), (10, 3), (384, 16)):
        segs = synthdata.segment_rows(n, m)
        assert segs[0][0] == 0
        assert sum(r for _, r in segs) == n
        for (a, ra), (b, _) in zip(segs, segs[1:]):
            assert a + ra == b
