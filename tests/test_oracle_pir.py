"""Pins of the PIR oracle against what the paper and the mathematics fix.

None of these re-types the oracle's loop: each checks it against an
independent route (numpy's packbits bit order, numpy's XOR reduction, an
integer matrix product mod 2, the paper's 3-server reconstruction, linearity).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth


def _xor_reduce(D, mask):
    if not mask.any():
        return np.zeros(D.shape[1], dtype=np.uint8)
    return np.bitwise_xor.reduce(D[mask], axis=0)


def test_paper_three_server_example(golden_dir):
    """Section 'Background: PIR': l = 3 servers, n = 3 blocks, beta = 2."""
    g = json.load(open(os.path.join(golden_dir, "pir_three_server_example.json")))
    D = np.stack([np.frombuffer(bytes.fromhex(h), dtype=np.uint8) for h in g["blocks_hex"]])
    qs = [g["q1"], g["q2"], g["q3"]]
    # q3 = q' xor q1 xor q2 (client step 3)
    assert list(np.bitwise_xor.reduce(np.array([g["q_prime"], g["q1"], g["q2"]]), axis=0)) == g["q3"]
    R = [oracle.pir_read(D, synth.bits_to_rows(np.array([q])))[0] for q in qs]
    for r, h in zip(R, g["R_hex"]):
        assert r.tobytes().hex() == h
    rec = R[0] ^ R[1] ^ R[2]
    assert rec.tobytes().hex() == g["reconstructed_hex"]
    assert np.array_equal(rec, D[g["beta"] - 1])


@pytest.mark.parametrize("n", [1, 7, 8, 37, 64])
def test_zero_vector_gives_zero(n):
    D = synth.uniform_db(11, n, 24)
    req = np.zeros((3, synth.request_bytes(n)), dtype=np.uint8)
    assert not oracle.pir_read(D, req).any()


@pytest.mark.parametrize("n", [1, 9, 37, 64, 130])
def test_one_hot_returns_bucket(n):
    """e_i -> exactly bucket i, for every i; rows packed by numpy (LSB-first)."""
    D = synth.uniform_db(12, n, 40)
    bits = np.eye(n, dtype=bool)
    req = np.packbits(bits, axis=1, bitorder="little")
    resp = oracle.pir_read(D, req)
    assert np.array_equal(resp, D)


def test_all_ones_is_xor_of_every_bucket():
    n = 101
    D = synth.uniform_db(13, n, 64)
    req = synth.bits_to_rows(np.ones((1, n), dtype=bool))
    assert np.array_equal(oracle.pir_read(D, req)[0], np.bitwise_xor.reduce(D, axis=0))


def test_linearity():
    n = 200
    D = synth.uniform_db(14, n, 48)
    a = synth.bernoulli_requests(15, 6, n)
    b = synth.bernoulli_requests(16, 6, n)
    assert np.array_equal(oracle.pir_read(D, a ^ b), oracle.pir_read(D, a) ^ oracle.pir_read(D, b))


def test_three_share_reconstruction_random():
    """q3 = e_beta xor q1 xor q2 -> R1 xor R2 xor R3 = D[beta] (definition of correctness)."""
    n = 333
    D = synth.uniform_db(17, n, 32)
    for beta in [0, 1, 7, 8, 200, n - 1]:
        q1 = synth.bernoulli_requests(18 + beta, 1, n)
        q2 = synth.bernoulli_requests(1000 + beta, 1, n)
        e = synth.bits_to_rows(np.eye(n, dtype=bool)[[beta]])
        q3 = e ^ q1 ^ q2
        R = oracle.pir_read(D, np.concatenate([q1, q2, q3]))
        assert np.array_equal(R[0] ^ R[1] ^ R[2], D[beta])


def test_matches_numpy_xor_reduction():
    n = 257
    D = synth.uniform_db(19, n, 96)
    req = synth.bernoulli_requests(20, 9, n)
    bits = synth.rows_to_bits(req, n).astype(bool)
    resp = oracle.pir_read(D, req)
    for r in range(req.shape[0]):
        assert np.array_equal(resp[r], _xor_reduce(D, bits[r]))


@pytest.mark.parametrize("n", [1, 3, 8, 10])
def test_brute_force_gf2_matrix_product(n):
    """All 2^n request vectors; answer = (R_bits @ D_bits) mod 2, an integer product."""
    bucket = 3
    D = synth.uniform_db(21 + n, n, bucket)
    allv = ((np.arange(2 ** n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    req = synth.bits_to_rows(allv)
    Dbits = np.unpackbits(D, axis=1).astype(np.int64)          # [n, 8*bucket]
    expect = np.packbits((allv @ Dbits) % 2, axis=1).astype(np.uint8)
    assert np.array_equal(oracle.pir_read(D, req), expect)


def test_padding_bits_are_ignored():
    n = 37  # 5 bytes, 3 padding bits
    D = synth.uniform_db(22, n, 16)
    req = synth.bernoulli_requests(23, 4, n, p=0.3)
    noisy = req.copy()
    noisy[:, -1] |= 0xE0
    assert np.array_equal(oracle.pir_read(D, req), oracle.pir_read(D, noisy))


def test_row_stride_larger_than_needed():
    n = 50
    D = synth.uniform_db(24, n, 8)
    req = synth.bernoulli_requests(25, 3, n)
    padded = np.zeros((3, 16), dtype=np.uint8)
    padded[:, :req.shape[1]] = req
    assert np.array_equal(oracle.pir_read(D, req), oracle.pir_read(D, padded))


def test_threads_do_not_change_the_answer():
    n = 300
    D = synth.uniform_db(26, n, 128)
    req = synth.bernoulli_requests(27, 13, n)
    assert np.array_equal(oracle.pir_read(D, req, threads=1), oracle.pir_read(D, req, threads=4))


def test_empty_batch():
    D = synth.uniform_db(28, 10, 8)
    assert oracle.pir_read(D, np.zeros((0, 2), dtype=np.uint8)).shape == (0, 8)


def test_small_workload_end_to_end():
    """The 4 MiB / B = 8 workload in full, against the numpy reduction."""
    from synth.configs import C1
    D = synth.uniform_db(C1.db_seed, C1.n, C1.bucket_bytes)
    req = synth.bernoulli_requests(C1.req_seed, C1.B, C1.n)
    resp = oracle.pir_read(D, req, threads=4)
    bits = synth.rows_to_bits(req, C1.n).astype(bool)
    for r in range(C1.B):
        assert np.array_equal(resp[r], _xor_reduce(D, bits[r]))
