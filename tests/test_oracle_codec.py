"""Pins of the compressed interest-vector oracle (section "Private
Notifications": compressed Bloom-filter deltas; the stream format is this
build's reading, Golomb-Rice coded gaps)."""
import json
import os

import numpy as np
import pytest

import oracle


def _vec(m, positions):
    v = np.zeros((m + 7) // 8, dtype=np.uint8)
    for p in positions:
        v[p >> 3] |= np.uint8(1 << (p & 7))
    return v


def test_hand_worked_examples(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "interest_codec_examples.json")))
    for ex in g["examples"]:
        v = _vec(ex["m"], ex["positions"])
        assert oracle.iv_encode(v, ex["m"]).hex() == ex["stream"]
        m, back = oracle.iv_decode(bytes.fromhex(ex["stream"]))
        assert m == ex["m"] and np.array_equal(back, v)


def _expected_length(m, positions):
    """Stream length from the code's definition, in plain integer arithmetic."""
    c = len(positions)
    k = int(np.floor(np.log2(max(1, m // (c + 1)))))
    prev, bits = -1, 0
    for p in positions:
        g = p - prev - 1
        bits += (g >> k) + 1 + k
        prev = p
    return 24 + (bits + 7) // 8, k


@pytest.mark.parametrize("m,density,seed", [(1, 1.0, 1), (33, 0.5, 2), (1000, 0.01, 3), (4096, 0.3, 4),
                                            (1 << 17, 0.002, 5), (1 << 17, 0.9, 6), (100003, 0.05, 7)])
def test_round_trip_and_length(m, density, seed):
    rng = np.random.default_rng(seed)
    bits = rng.random(m) < density
    positions = np.flatnonzero(bits).tolist()
    v = np.packbits(bits, bitorder="little")
    s = oracle.iv_encode(v, m)
    want_len, k = _expected_length(m, positions)
    assert len(s) == want_len
    assert int.from_bytes(s[16:20], "little") == k
    assert int.from_bytes(s[8:16], "little") == len(positions)
    m2, back = oracle.iv_decode(s)
    assert m2 == m and np.array_equal(np.unpackbits(back, bitorder="little")[:m], bits.astype(np.uint8))


def test_sparse_deltas_compress():
    """A sparse delta (the case the paper's compressed filters target) costs far
    fewer bytes than the raw vector: about log2(mean gap) + 2 bits per bit set."""
    m = 1 << 17
    positions = np.sort(np.random.default_rng(8).choice(m, 600, replace=False))
    s = oracle.iv_encode(_vec(m, positions), m)
    assert len(s) < (m // 8) // 8
    assert len(s) <= 24 + 600 * (int(np.log2(m // 601)) + 3) // 8 + 1


def test_truncated_stream_rejected():
    s = oracle.iv_encode(_vec(1000, [5, 700]), 1000)
    with pytest.raises(ValueError):
        oracle.iv_decode(s[:-1])
