"""The bench's roofline accounting, checked on the CPU against brute force.

The plain XOR count of a batch is the number of set request bits below n
times the words per bucket; with Strassen leaves it is that of the 7^L leaf
products, whose request rows are XORs of request blocks (the A-combinations
of the leaf tables). Both are counted here bit by bit from unpacked bits,
and the LDS floor's byte counts are checked against a hand count of one
paired-table launch.
"""
import importlib.util
import os

import numpy as np
import pytest

import paper_2001_08250_amd as pir
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _bits(req, n):
    return np.unpackbits(req, axis=1, bitorder="little")[:, :n].astype(bool)


@pytest.mark.parametrize("n,B", [(1, 3), (13, 5), (1000, 97), (4096, 64)])
def test_popcount_rows_counts_bits_below_n(bench, n, B):
    req = synth.uniform_bytes(31 + n + B, B * ((n + 7) // 8)).reshape(B, -1)   # padding bits set too
    assert np.array_equal(bench.popcount_rows(req, n), _bits(req, n).sum(axis=1))


@pytest.mark.parametrize("n,B,levels", [(1000, 97, 1), (1000, 97, 2), (333, 5, 2), (4096, 64, 2), (4070, 600, 1)])
def test_leaf_request_bits_brute_force(bench, n, B, levels):
    req = synth.uniform_bytes(7 + n + B, B * ((n + 7) // 8)).reshape(B, -1)
    t = pir.preprocess_tables(levels)
    g = t["grid"]
    unit = 32 << levels
    nq = -(-n // unit) * unit >> levels
    bq = -(-B // g)
    bits = np.zeros((g * bq, g * nq), dtype=bool)
    bits[:B, :n] = _bits(req, n)
    total = 0
    for combo in t["a"]:
        acc = np.zeros((bq, nq), dtype=bool)
        for rb, cb in combo:
            acc ^= bits[rb * bq:(rb + 1) * bq, cb * nq:(cb + 1) * nq]
        total += int(acc.sum())
    assert bench.leaf_request_bits(pir, req, n, levels) == total


def test_leaf_bits_are_49_16ths_of_the_batch_on_average(bench):
    """At density 1/2 every leaf request bit is set with probability 1/2, so
    the 49 leaves of two levels hold 49 * (1/4 of the rows) * (1/4 of the
    bits) = 49/16 of the batch's set bits, up to sampling noise."""
    n, B = 1 << 14, 256
    req = synth.bernoulli_requests(5, B, n)
    ratio = bench.leaf_request_bits(pir, req, n, 2) / bench.popcount_rows(req, n).sum()
    assert abs(ratio - 49 / 16) < 0.02


class _Plan:
    def __init__(self, tile, unroll, flags):
        self.kind, self.tile, self.unroll, self.flags = 4, tile, unroll, flags


def test_lds_floor_hand_count(bench):
    """5-bucket pairs of 1 KiB entries, 256 requests a workgroup, and
    half-wave 6-bucket pairs of 512-byte entries, 512 a workgroup, over
    n = 2^20 rows of 1 KiB with 512 requests."""
    n, B, row = 1 << 20, 512, 1024
    p5 = _Plan(32, 8, pir.PLAN_PAIRS)
    steps = -(-n // 10)
    f = bench.lds_floor(p5, n, B, row)
    assert f["read_bytes"] == 1 * steps * B * 2 * 1024                # a slice, every request, two tables
    assert f["write_bytes"] == 1 * 2 * steps * 2 * 32 * 1024          # two request tiles build every table
    p6 = _Plan(64, 8, pir.PLAN_PAIRS | pir.PLAN_HALF_WAVES | pir.PLAN_PAIR_G6)
    steps = -(-n // 12)
    f = bench.lds_floor(p6, n, B, row)
    assert f["read_bytes"] == 2 * steps * B * 2 * 512                 # two 512-byte slices
    assert f["write_bytes"] == 2 * 1 * steps * 2 * 64 * 512           # one request tile per slice
