"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random bytes and shapes them; it holds none of the PIR
arithmetic, so both sides of every parity check consume the same bytes without
sharing any of the method's code.

A Talek server only ever sees ciphertext, which looks uniformly random, and
uniformly random request vectors (each server's share of an IT-PIR query is a
uniform bit vector; section "Background: PIR"). Uniform bytes for the database
and Bernoulli(1/2) request bits therefore reproduce exactly the distribution
the server path sees; the sizes follow the paper's workloads (1 KiB messages,
bucket depth 4; section "Evaluation").
"""
from __future__ import annotations

import hashlib
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK_BYTES = 1 << 26  # 64 MiB per independently seeded chunk


def _chunk_bytes(seed: int, chunk: int, nbytes: int) -> np.ndarray:
    bg = np.random.PCG64(np.random.SeedSequence([seed, chunk]))
    words = (nbytes + 7) // 8
    return bg.random_raw(words).view(np.uint8)[:nbytes]


def uniform_bytes(seed: int, nbytes: int, threads: int = 8, out: np.ndarray | None = None) -> np.ndarray:
    """nbytes uniform bytes; chunk c of 64 MiB comes from PCG64(SeedSequence([seed, c]))."""
    if out is None:
        out = np.empty(nbytes, dtype=np.uint8)
    flat = out.reshape(-1)
    assert flat.size == nbytes
    nchunks = (nbytes + CHUNK_BYTES - 1) // CHUNK_BYTES

    def fill(c):
        lo = c * CHUNK_BYTES
        hi = min(nbytes, lo + CHUNK_BYTES)
        flat[lo:hi] = _chunk_bytes(seed, c, hi - lo)

    if nchunks <= 1 or threads <= 1:
        for c in range(nchunks):
            fill(c)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(fill, range(nchunks)))
    return out


def uniform_db(seed: int, n: int, bucket_bytes: int, threads: int = 8) -> np.ndarray:
    """Database of n buckets of bucket_bytes uniform bytes: uint8 [n, bucket_bytes]."""
    return uniform_bytes(seed, n * bucket_bytes, threads).reshape(n, bucket_bytes)


def request_bytes(n: int) -> int:
    """Bytes of one request row: one bit per bucket, ceil(n / 8)."""
    return (n + 7) // 8


def bernoulli_requests(seed: int, B: int, n: int, p: float = 0.5) -> np.ndarray:
    """B request rows of n Bernoulli(p) bits, LSB-first in ceil(n/8) bytes.

    For p = 0.5 every byte is uniform, including the padding bits past n in the
    last byte (the server must ignore them). For other p the bits past n are 0.
    """
    rb = request_bytes(n)
    if p == 0.5:
        return uniform_bytes(seed, B * rb).reshape(B, rb)
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.random((B, n)) < p
    return np.packbits(bits, axis=1, bitorder="little")[:, :rb].copy()


def one_hot(n: int, idx) -> np.ndarray:
    """Rows e_i: exactly bit i set (LSB-first)."""
    idx = np.atleast_1d(np.asarray(idx, dtype=np.int64))
    rb = request_bytes(n)
    out = np.zeros((idx.size, rb), dtype=np.uint8)
    for r, i in enumerate(idx):
        out[r, i >> 3] |= np.uint8(1 << (int(i) & 7))
    return out


def bits_to_rows(bits: np.ndarray) -> np.ndarray:
    """Pack a bool/0-1 matrix [B, n] into request rows, LSB-first."""
    bits = np.asarray(bits).astype(bool)
    return np.packbits(bits, axis=1, bitorder="little")


def rows_to_bits(rows: np.ndarray, n: int) -> np.ndarray:
    """Unpack request rows into a 0/1 uint8 matrix [B, n]."""
    return np.unpackbits(np.asarray(rows, dtype=np.uint8), axis=1, bitorder="little")[:, :n]


def distinct_ids(seed: int, count: int) -> np.ndarray:
    """count distinct nonzero uint64 message ids (rejection of repeats)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ids = np.zeros(0, dtype=np.uint64)
    while ids.size < count:
        extra = rng.integers(1, np.iinfo(np.uint64).max, size=count - ids.size + 16, dtype=np.uint64,
                             endpoint=True)
        ids = np.concatenate([ids, extra])
        _, first = np.unique(ids, return_index=True)
        ids = ids[np.sort(first)]
    return ids[:count].copy()


def write_ops(seed: int, count: int, n: int, z: int, id_offset_seed: int | None = None):
    """Synthetic Write requests (beta1, beta2, data) for count messages.

    The candidate buckets are uniform in [0, n): they stand in for the client's
    PRF outputs (section "Writing into a Cuckoo Hash Table"). The z payload
    bytes stand in for the ciphertext; the first 8 bytes are the message id
    (little-endian) so a slot's content can be traced back to its message.
    Returns (ids uint64 [count], b1 uint64, b2 uint64, payload uint8 [count, z]).
    """
    ids = distinct_ids(seed if id_offset_seed is None else id_offset_seed, count)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
    b1 = rng.integers(0, n, size=count, dtype=np.uint64)
    b2 = rng.integers(0, n, size=count, dtype=np.uint64)
    payload = uniform_bytes(seed ^ 0x5A5A5A5A, count * z).reshape(count, z)
    if z >= 8:
        payload[:, :8] = ids.view(np.uint8).reshape(count, 8)
    return ids, b1, b2, payload


def uniform_indices(seed: int, count: int, n: int) -> np.ndarray:
    """count indices uniform in [0, n) (uint64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, n, size=count, dtype=np.uint64)


def batch_sizes(seed: int, count: int, lo: int = 1, hi: int = 1024) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=count).astype(np.uint32)


def poisson_arrivals(seed: int, rate: float, duration_s: float) -> np.ndarray:
    """Arrival times (seconds, increasing) of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    est = int(rate * duration_s * 1.2) + 64
    gaps = rng.exponential(1.0 / rate, size=est)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate, size=est)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]


def interest_positions(seed: int, writes: int, k: int, m_bits: int) -> np.ndarray:
    """k uniform bit positions in [0, m_bits) per write: uint32 [writes, k]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, m_bits, size=(writes, k), dtype=np.uint32)


def digest(a: np.ndarray) -> str:
    """Short content digest, recorded so both sides provably used the same bytes."""
    return hashlib.blake2b(np.ascontiguousarray(a).view(np.uint8).reshape(-1), digest_size=12).hexdigest()
