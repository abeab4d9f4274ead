"""Pins of the DCT entropy code (oracle/entropy.py): the zigzag scan order as
printed in ITU-T Rec. T.81 (Figure A.6), textbook Exp-Golomb codes, a block
encoded by hand, round trips across restart intervals, and the size of an
all-zero segment."""
import numpy as np
import pytest

from oracle import entropy


def test_zigzag_matches_the_jpeg_scan_order():
    # natural (row-major) index of the first 16 and last 4 positions of the scan
    nat = [8 * u + v for u, v in entropy.zigzag_order()]
    assert nat[:16] == [0, 1, 8, 16, 9, 2, 3, 10, 17, 24, 32, 25, 18, 11, 4, 5]
    assert nat[-6:] == [61, 54, 47, 55, 62, 63]
    assert sorted(nat) == list(range(64))


@pytest.mark.parametrize("x,code", [(0, "1"), (1, "010"), (2, "011"), (3, "00100"), (4, "00101"),
                                    (6, "00111"), (7, "0001000"), (14, "0001111")])
def test_exp_golomb_codes(x, code):
    assert entropy.eg_bits(x) == code


def test_block_encoded_by_hand():
    q = np.zeros((8, 8), np.int16)
    q[0, 0] = 5          # DC 5: d = 5 -> EG(10) = 0001011
    q[2, 0] = -2         # zigzag position 3, after two zeros: EG(3) = 00100, level EG(2*1 + 1) = 00100
    words, restart, total = entropy.encode(q)
    s = "0001011" + "00100" + "00100" + "1"
    assert total == len(s) == 18 and restart.tolist() == [0]
    assert words.tolist() == [int(s.ljust(32, "0"), 2)]


def test_round_trip_across_restart_intervals():
    rng = np.random.default_rng(9)
    rows, cols = 8 * 9, 8 * 17                      # 153 blocks: three intervals, the last partial
    q = np.where(rng.random((rows, cols)) < 0.15, rng.integers(-300, 300, (rows, cols)), 0).astype(np.int16)
    q[::8, ::8] = rng.integers(-2000, 2000, (9, 17))  # DCs
    words, restart, total = entropy.encode(q)
    assert len(restart) == 3 and restart[0] == 0
    np.testing.assert_array_equal(entropy.decode(words, restart, rows, cols), q)
    assert entropy.message_bytes(total, 153) == 4 * len(words) + 4 * 3 + 8


def test_all_zero_segment_costs_two_bits_per_block():
    words, restart, total = entropy.encode(np.zeros((16, 64), np.int16))
    # each block: DC difference EG(0) = "1", end of block EG(0) = "1"
    assert total == 2 * 16 and words.tolist() == [0xFFFFFFFF]
