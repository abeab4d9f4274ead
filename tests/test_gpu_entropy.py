"""GPU parity of the DCT entropy code (tomo_dct_encode / tomo_dct_decode)
against oracle/entropy.py: bit-exact words, restart table and total on sparse
and worst-case code arrays, round trips, a truncated stream reported as
malformed, and the codes of a real consensus message."""
import numpy as np
import pytest
import torch

from gpu_common import log, require_gpu, to_dev
from oracle import entropy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    require_gpu()
    from paper_2410_06106_amd import tomoadmm
    return tomoadmm


@pytest.fixture(scope="module")
def ctx(T):
    return T.Context(0)


def _codes(rows, cols, density, seed, amp=300):
    rng = np.random.default_rng(seed)
    q = np.where(rng.random((rows, cols)) < density, rng.integers(-amp, amp + 1, (rows, cols)), 0)
    q[::8, ::8] = rng.integers(-2000, 2001, (rows // 8, cols // 8))
    return q.astype(np.int16)


def _check(T, ctx, q):
    rows, cols = q.shape
    words, restart, total = T.tomo_dct_encode(ctx, to_dev(q, torch.int16))
    w_o, r_o, t_o = entropy.encode(q)
    tot = int(total.cpu().numpy().view(np.uint32)[0])
    assert tot == t_o
    got_w = words.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got_w[:len(w_o)], w_o)
    assert not got_w[len(w_o):].any()
    np.testing.assert_array_equal(restart.cpu().numpy().view(np.uint32)[:len(r_o)], r_o)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    back = T.tomo_dct_decode(ctx, words, restart, total, rows, cols, status=status)
    assert int(status.item()) == 0
    np.testing.assert_array_equal(back.cpu().numpy(), q)
    return tot


@pytest.mark.parametrize("rows,cols,density", [(8, 8, 0.3), (8, 136, 0.1), (72, 136, 0.15), (256, 512, 0.05),
                                               (64, 64, 0.0)])
def test_encode_matches_oracle_and_decodes(T, ctx, rows, cols, density):
    log(f"case entropy {rows}x{cols} density={density}")
    _check(T, ctx, _codes(rows, cols, density, rows + cols))


def test_worst_case_blocks(T, ctx):
    """Every code nonzero at the int16 extremes: the longest blocks the format has."""
    rng = np.random.default_rng(1)
    q = rng.choice(np.array([-32768, 32767, -1, 1], np.int16), size=(16, 24))
    tot = _check(T, ctx, q)
    assert tot <= 6 * 2302


def test_truncated_stream_is_reported(T, ctx):
    q = _codes(64, 64, 0.2, 5)
    words, restart, total = T.tomo_dct_encode(ctx, to_dev(q, torch.int16))
    short = torch.tensor([int(total.item()) // 2], dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    T.tomo_dct_decode(ctx, words, restart, short, 64, 64, status=status)
    assert int(status.item()) == 1


def test_consensus_dct_message_round_trip(T, ctx):
    """Codes admm_consensus emits for DCT-quantized segments encode to the
    oracle's stream and decode back; the message size follows oracle/entropy.py."""
    n, M = 64, 2
    rng = np.random.default_rng(6)
    X = to_dev(rng.random((n, n)).astype(np.float32))
    U = [to_dev(rng.random((n, n)).astype(np.float32)) for _ in range(M)]
    L = [torch.zeros((n, n), dtype=torch.float32, device="cuda") for _ in range(M)]
    dummy_d = to_dev(np.zeros((1, 8), np.float32))
    coeffs = [torch.empty((32, n), dtype=torch.int16, device="cuda") for _ in range(M)]
    lohi = [torch.empty(2, dtype=torch.float32, device="cuda") for _ in range(M)]
    ents = [dict(n=n, n_bins=8, angles=to_dev(np.zeros(1), torch.float64), slice=0, d=dummy_d, u=U[m],
                 lam=L[m], x=X, seg_row0=32 * m, seg_rows=32, rho=1.0, eta1=0.0, eta2=0.5) for m in range(M)]
    T.admm_consensus(ctx, T.make_nodes(ents), T.TOMO_XUPDATE_SEGMENT, 2, T.tomo_quant(T.TOMO_QUANT_DCT, 0, 0, 50),
                     T.make_msgs([dict(coeffs=coeffs[m], lohi=lohi[m]) for m in range(M)]))
    for m in range(M):
        q = coeffs[m].cpu().numpy()
        tot = _check(T, ctx, q)
        assert entropy.message_bytes(tot, 32) == 4 * ((tot + 31) // 32) + 4 + 8
