"""Pins of the serialized-PIR mask oracle (section "Serialized PIR").

The PRNG reading is ChaCha20 (RFC 8439 form); the oracle's keystream is pinned
to the RFC's published block-function example and, where the openssl tool is
installed, to an independent implementation (openssl's chacha20). The masked
answers are pinned by what the protocol requires: unmasking gives the plain
answer, and the leader's XOR of three servers' masked answers, unmasked with
the three masks, gives exactly the requested bucket.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth


def test_rfc8439_block_function_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "chacha20_rfc8439_block.json")))
    key = bytes.fromhex(g["key"])
    nonce = bytes.fromhex(g["nonce"])
    got = oracle.chacha20_stream(key, nonce, g["counter"], 64)
    assert got.tobytes().hex() == g["keystream"]


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl not installed")
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_keystream_matches_openssl(seed):
    rng = np.random.default_rng(seed)
    key = rng.integers(0, 256, 32, dtype=np.uint8).tobytes()
    nonce = rng.integers(0, 256, 12, dtype=np.uint8).tobytes()
    counter = int(rng.integers(0, 1 << 31))
    nbytes = int(rng.integers(1, 700))
    want = subprocess.run(
        ["openssl", "enc", "-chacha20", "-K", key.hex(),
         "-iv", counter.to_bytes(4, "little").hex() + nonce.hex()],
        input=bytes(nbytes), capture_output=True, check=True).stdout
    got = oracle.chacha20_stream(key, nonce, counter, nbytes)
    assert got.tobytes() == want


@pytest.mark.parametrize("row_bytes", [4096, 520, 24])
def test_mask_is_the_keystream_of_the_seed(row_bytes):
    """The mask of a seed is the first row_bytes of ChaCha20 keyed by the seed,
    all-zero nonce, block counter from 0: checked against the keystream
    function (pinned above to the RFC and openssl) and, where installed,
    against openssl directly."""
    seeds = synth.uniform_bytes(row_bytes, 3 * 32).reshape(3, 32)
    masks = oracle.apply_masks(np.zeros((3, row_bytes), dtype=np.uint8), seeds)
    for r in range(3):
        want = oracle.chacha20_stream(seeds[r].tobytes(), bytes(12), 0, row_bytes)
        assert np.array_equal(masks[r], want)
        if shutil.which("openssl"):
            ref = subprocess.run(["openssl", "enc", "-chacha20", "-K", seeds[r].tobytes().hex(), "-iv", "00" * 16],
                                 input=bytes(row_bytes), capture_output=True, check=True).stdout
            assert masks[r].tobytes() == ref


def test_masks_are_distinct_per_seed_and_position():
    seeds = synth.uniform_bytes(7, 2 * 32).reshape(2, 32)
    zero = np.zeros((2, 4096), dtype=np.uint8)
    masks = oracle.apply_masks(zero, seeds)
    assert not np.array_equal(masks[0], masks[1])
    blocks = masks[0].reshape(-1, 64)
    assert len({b.tobytes() for b in blocks}) == blocks.shape[0]   # counter advances per block


@pytest.mark.parametrize("n,bucket,B", [(64, 4096, 5), (100, 520, 3), (7, 24, 4)])
def test_unmasking_restores_the_plain_answer(n, bucket, B):
    D = synth.uniform_db(n + bucket, n, bucket)
    req = synth.bernoulli_requests(n, B, n)
    seeds = synth.uniform_bytes(B + 9, B * 32).reshape(B, 32)
    plain = oracle.pir_read(D, req)
    masked = oracle.pir_read_masked(D, req, seeds)
    assert not np.array_equal(masked, plain)
    assert np.array_equal(oracle.apply_masks(masked, seeds), plain)


def test_serialized_three_server_reconstruction():
    """Client: random q0, q1 and q2 = e_i ^ q0 ^ q1, seeds p0..p2; servers
    answer R_s ^ P_s; the leader XORs them; the client XORs the masks away and
    holds bucket i."""
    n, bucket = 300, 4096
    D = synth.uniform_db(31, n, bucket)
    rng = np.random.default_rng(32)
    for i in (0, 137, n - 1):
        q0 = synth.bernoulli_requests(int(rng.integers(1 << 30)), 1, n)
        q1 = synth.bernoulli_requests(int(rng.integers(1 << 30)), 1, n)
        q2 = q0 ^ q1 ^ synth.one_hot(n, i)
        seeds = [synth.uniform_bytes(int(rng.integers(1 << 30)), 32).reshape(1, 32) for _ in range(3)]
        answers = [oracle.pir_read_masked(D, q, p) for q, p in zip((q0, q1, q2), seeds)]
        combined = answers[0] ^ answers[1] ^ answers[2]
        for p in seeds:
            combined = oracle.apply_masks(combined, p)
        assert np.array_equal(combined[0], D[i])
