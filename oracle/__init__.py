"""CPU oracle for the Talek XOR-PIR server path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this package; the library under ``paper_2001_08250_amd``
never does, and this package never imports the library. It wraps the plain C
definitions in ``pir_oracle.c``, ``cuckoo_oracle.c`` and ``mask_oracle.c`` (built
with gcc by :func:`build`) through ctypes.

* :func:`pir_read` -- the server answer of IT-PIR (section "Background: PIR",
  server step; appendix "Security Proofs", answer functions): for each request
  row the XOR of every bucket whose request bit is set, bits LSB-first.
* :class:`Cuckoo` -- reference blocked cuckoo table with FIFO garbage
  collection (section "Writing into a Cuckoo Hash Table").
* :func:`interest_window` -- union of the interest-vector positions written
  in the last ``window`` epochs (section "Private Notifications").
* :func:`splitmix64` -- SplitMix64 stream (Steele, Lea, Flood 2014), the
  randomness the cuckoo walk draws from the shared seed.
* :func:`pir_read_masked`, :func:`apply_masks`, :func:`chacha20_stream` --
  serialized PIR (section "Serialized PIR"): each answer XORed with a one-time
  mask drawn from a per-request seed; the PRNG is read as ChaCha20 (RFC 8439
  form, seed as key, zero nonce, counter from 0).
* :func:`iv_encode`, :func:`iv_decode` -- the compressed interest-vector
  stream (Golomb-Rice coded gaps between set bits; section "Private
  Notifications": clients fetch compressed Bloom-filter deltas).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ["pir_oracle.c", "cuckoo_oracle.c", "mask_oracle.c", "codec_oracle.c"]
LIB_PATH = os.path.join(_HERE, "liboracle.so")
# A test may point the oracle at another build of these sources (the mutation
# check builds deliberately broken copies to show that the pins catch them).
LIB_PATH = os.environ.get("TALEK_ORACLE_LIB", LIB_PATH)
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra"]

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle C sources into ``liboracle.so`` (always rebuilds)."""
    cmd = ["gcc", *CFLAGS, "-o", LIB_PATH + ".tmp"] + [os.path.join(_HERE, s) for s in _SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_pir_read.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, u8p,
                                    ctypes.c_uint64, ctypes.c_uint32, u8p, ctypes.c_uint32]
    lib.oracle_pir_read.restype = ctypes.c_int
    lib.oracle_splitmix64_fill.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u64p]
    lib.oracle_splitmix64_fill.restype = None
    lib.oracle_cuckoo_new.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
    lib.oracle_cuckoo_new.restype = ctypes.c_void_p
    lib.oracle_cuckoo_free.argtypes = [ctypes.c_void_p]
    lib.oracle_cuckoo_free.restype = None
    lib.oracle_cuckoo_insert.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, u8p, u64p]
    lib.oracle_cuckoo_insert.restype = ctypes.c_int
    lib.oracle_cuckoo_insert_many.argtypes = [ctypes.c_void_p, ctypes.c_uint64, u64p, u64p, u64p,
                                              u8p, ctypes.POINTER(ctypes.c_int32), u64p]
    lib.oracle_cuckoo_insert_many.restype = ctypes.c_uint64
    lib.oracle_cuckoo_table.argtypes = [ctypes.c_void_p]
    lib.oracle_cuckoo_table.restype = ctypes.c_void_p
    lib.oracle_cuckoo_live.argtypes = [ctypes.c_void_p]
    lib.oracle_cuckoo_live.restype = ctypes.c_uint64
    lib.oracle_cuckoo_slots.argtypes = [ctypes.c_void_p, u64p, u8p]
    lib.oracle_cuckoo_slots.restype = None
    lib.oracle_cuckoo_slot_buckets.argtypes = [ctypes.c_void_p, u64p, u64p]
    lib.oracle_cuckoo_slot_buckets.restype = None
    lib.oracle_interest_window.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32), u64p,
                                           ctypes.c_uint32, ctypes.c_uint32, u8p]
    lib.oracle_interest_window.restype = ctypes.c_int
    lib.oracle_chacha20_stream.argtypes = [u8p, u8p, ctypes.c_uint32, u8p, ctypes.c_uint64]
    lib.oracle_chacha20_stream.restype = None
    lib.oracle_apply_masks.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32, u8p]
    lib.oracle_apply_masks.restype = None
    lib.oracle_iv_encode.argtypes = [u8p, ctypes.c_uint64, u8p, ctypes.c_uint64]
    lib.oracle_iv_encode.restype = ctypes.c_uint64
    lib.oracle_iv_decode.argtypes = [u8p, ctypes.c_uint64, u8p, ctypes.c_uint64]
    lib.oracle_iv_decode.restype = ctypes.c_uint64
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype=ctypes.c_uint8):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def pir_read(D: np.ndarray, req: np.ndarray, n: int | None = None, threads: int = 1) -> np.ndarray:
    """XOR-PIR answer for every request row.

    D   : uint8 [n, bucket_bytes] (or flat with n given).
    req : uint8 [B, stride] with stride >= ceil(n / 8); bits beyond n ignored.
    Returns uint8 [B, bucket_bytes].
    """
    lib = _load()
    D = np.ascontiguousarray(D, dtype=np.uint8)
    if n is None:
        n = D.shape[0]
    bucket_bytes = D.size // n if n else 0
    req = np.ascontiguousarray(req, dtype=np.uint8)
    if req.ndim == 1:
        req = req.reshape(1, -1)
    B = req.shape[0]
    resp = np.zeros((B, bucket_bytes), dtype=np.uint8)
    if B == 0:
        return resp
    rc = lib.oracle_pir_read(_ptr(D), n, bucket_bytes, _ptr(req), req.shape[1], B, _ptr(resp), threads)
    if rc != 0:
        raise ValueError("oracle_pir_read rejected its arguments")
    return resp


def splitmix64(seed: int, count: int) -> np.ndarray:
    lib = _load()
    out = np.zeros(count, dtype=np.uint64)
    lib.oracle_splitmix64_fill(seed, count, _ptr(out, ctypes.c_uint64))
    return out


class Cuckoo:
    """Reference blocked cuckoo table (n buckets x d slots x z bytes)."""

    OK, ERANGE, ENOMEM, EFULL = 0, -2, -3, -5

    def __init__(self, n: int, d: int, z: int, capacity: int = 0, seed: int = 0, max_kicks: int = 500):
        self._lib = _load()
        self.n, self.d, self.z = n, d, z
        self._h = self._lib.oracle_cuckoo_new(n, d, z, capacity, seed, max_kicks)
        if not self._h:
            raise MemoryError("oracle_cuckoo_new failed")

    def close(self):
        if self._h:
            self._lib.oracle_cuckoo_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def insert(self, id_: int, b1: int, b2: int, payload: np.ndarray):
        payload = np.ascontiguousarray(payload, dtype=np.uint8)
        assert payload.size == self.z
        dropped = ctypes.c_uint64(0)
        rc = self._lib.oracle_cuckoo_insert(self._h, id_, b1, b2, _ptr(payload), ctypes.byref(dropped))
        return rc, dropped.value

    def insert_many(self, ids, b1, b2, payloads):
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        b1 = np.ascontiguousarray(b1, dtype=np.uint64)
        b2 = np.ascontiguousarray(b2, dtype=np.uint64)
        payloads = np.ascontiguousarray(payloads, dtype=np.uint8)
        cnt = ids.size
        assert payloads.size == cnt * self.z
        status = np.zeros(cnt, dtype=np.int32)
        dropped = np.zeros(cnt, dtype=np.uint64)
        self._lib.oracle_cuckoo_insert_many(self._h, cnt, _ptr(ids, ctypes.c_uint64), _ptr(b1, ctypes.c_uint64),
                                            _ptr(b2, ctypes.c_uint64), _ptr(payloads),
                                            _ptr(status, ctypes.c_int32), _ptr(dropped, ctypes.c_uint64))
        return status, dropped

    def table(self) -> np.ndarray:
        """Copy of the table bytes as uint8 [n, d * z]."""
        p = self._lib.oracle_cuckoo_table(self._h)
        buf = (ctypes.c_uint8 * (self.n * self.d * self.z)).from_address(p)
        return np.frombuffer(buf, dtype=np.uint8).reshape(self.n, self.d * self.z).copy()

    def table_view(self) -> np.ndarray:
        """The table bytes as uint8 [n, d * z] without a copy: valid until the
        next insert or close (for reading large tables between inserts)."""
        p = self._lib.oracle_cuckoo_table(self._h)
        buf = (ctypes.c_uint8 * (self.n * self.d * self.z)).from_address(p)
        return np.frombuffer(buf, dtype=np.uint8).reshape(self.n, self.d * self.z)

    def live(self) -> int:
        return int(self._lib.oracle_cuckoo_live(self._h))

    def slots(self):
        """(ids uint64 [n, d], occupied bool [n, d])."""
        ids = np.zeros(self.n * self.d, dtype=np.uint64)
        occ = np.zeros(self.n * self.d, dtype=np.uint8)
        self._lib.oracle_cuckoo_slots(self._h, _ptr(ids, ctypes.c_uint64), _ptr(occ))
        return ids.reshape(self.n, self.d), occ.reshape(self.n, self.d).astype(bool)

    def slot_buckets(self):
        b1 = np.zeros(self.n * self.d, dtype=np.uint64)
        b2 = np.zeros(self.n * self.d, dtype=np.uint64)
        self._lib.oracle_cuckoo_slot_buckets(self._h, _ptr(b1, ctypes.c_uint64), _ptr(b2, ctypes.c_uint64))
        return b1.reshape(self.n, self.d), b2.reshape(self.n, self.d)


def interest_window(m_bits: int, epochs: list, last: int, window: int) -> np.ndarray:
    """OR of the positions of epochs max(0, last-window+1)..last.

    ``epochs`` is a list of uint32 position arrays, one per epoch.
    """
    lib = _load()
    pos = np.ascontiguousarray(np.concatenate([np.asarray(e, dtype=np.uint32) for e in epochs])
                               if epochs else np.zeros(0, np.uint32), dtype=np.uint32)
    starts = np.zeros(len(epochs) + 1, dtype=np.uint64)
    for i, e in enumerate(epochs):
        starts[i + 1] = starts[i] + len(e)
    out = np.zeros((m_bits + 7) // 8, dtype=np.uint8)
    if pos.size == 0:
        pos = np.zeros(1, dtype=np.uint32)
    rc = lib.oracle_interest_window(m_bits, _ptr(pos, ctypes.c_uint32), _ptr(starts, ctypes.c_uint64),
                                    last, window, _ptr(out))
    if rc != 0:
        raise ValueError("interest position out of range")
    return out


def chacha20_stream(key: bytes, nonce: bytes, counter: int, nbytes: int) -> np.ndarray:
    """nbytes of ChaCha20 keystream (32-byte key, 12-byte nonce, first block counter)."""
    k = np.frombuffer(bytes(key), dtype=np.uint8).copy()
    iv = np.frombuffer(bytes(nonce), dtype=np.uint8).copy()
    if k.size != 32 or iv.size != 12:
        raise ValueError("key must be 32 bytes and nonce 12 bytes")
    out = np.zeros(nbytes, dtype=np.uint8)
    _load().oracle_chacha20_stream(_ptr(k), _ptr(iv), counter, _ptr(out), nbytes)
    return out


def apply_masks(resp: np.ndarray, seeds: np.ndarray) -> np.ndarray:
    """resp[r] XOR P(seeds[r]) (section "Serialized PIR", steps 6-7 and 9): the
    mask is the first row-length bytes of the ChaCha20 keystream keyed by the
    32-byte seed, zero nonce, counter from 0. Returns a new array."""
    out = np.ascontiguousarray(resp, dtype=np.uint8).copy()
    seeds = np.ascontiguousarray(seeds, dtype=np.uint8).reshape(-1, 32)
    if out.ndim != 2 or seeds.shape[0] != out.shape[0]:
        raise ValueError("one 32-byte seed per response row")
    _load().oracle_apply_masks(_ptr(out), out.shape[1], out.shape[0], _ptr(seeds))
    return out


def pir_read_masked(D: np.ndarray, req: np.ndarray, seeds: np.ndarray, n: int | None = None,
                    threads: int = 1) -> np.ndarray:
    """A serialized-PIR server's answers: pir_read(D, req) XOR the one-time masks."""
    return apply_masks(pir_read(D, req, n=n, threads=threads), seeds)


def iv_encode(v: np.ndarray, m: int) -> bytes:
    """Compressed stream of an m-bit vector (uint8, ceil(m/8) bytes, LSB-first)."""
    v = np.ascontiguousarray(v, dtype=np.uint8).reshape(-1)
    if v.size < (m + 7) // 8:
        raise ValueError("vector shorter than m bits")
    lib = _load()
    size = lib.oracle_iv_encode(_ptr(v), m, None, 0)
    out = np.zeros(size, dtype=np.uint8)
    lib.oracle_iv_encode(_ptr(v), m, _ptr(out), size)
    return out.tobytes()


def iv_decode(stream: bytes) -> tuple[int, np.ndarray]:
    """(m, vector) from a compressed stream; ValueError if it is malformed."""
    s = np.frombuffer(bytes(stream), dtype=np.uint8).copy()
    if s.size < 24:
        raise ValueError("stream shorter than its header")
    m = int(s[:8].view(np.uint64)[0])
    v = np.zeros((m + 7) // 8, dtype=np.uint8)
    got = _load().oracle_iv_decode(_ptr(s), s.size, _ptr(v), v.size)
    if got != m:
        raise ValueError("malformed stream")
    return m, v
