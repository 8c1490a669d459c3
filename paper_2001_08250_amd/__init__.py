"""Talek XOR-PIR server engine for MI355X (gfx950): Python binding.

Argument marshalling only: every step of the read path runs in the HIP
library ``libtalek_pir.so`` (built in-tree by :func:`build`). The raw C entry
points are exposed under their C names (``pir_db_create``, ...); the classes
:class:`PirDB` and :class:`Cuckoo` wrap them for numpy arrays and torch
tensors. There is no CPU fallback: if the library is missing, importing the
binding's functions raises.

torch is only used for device memory and streams (``*_async`` calls take
device tensors and the current HIP stream) and is imported lazily.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtalek_pir.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "talek_pir.h")

PIR_OK, PIR_EINVAL, PIR_ERANGE, PIR_ENOMEM, PIR_EDEVICE, PIR_EFULL, PIR_EBUSY = 0, -1, -2, -3, -4, -5, -6
KERNEL_AUTO, KERNEL_MASK, KERNEL_SKIP, KERNEL_M4R = 0, 1, 2, 3


class PirError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class pir_plan(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tile", ctypes.c_uint32), ("splits", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32)]

    def __repr__(self):
        return f"pir_plan(kind={self.kind}, tile={self.tile}, splits={self.splits}, unroll={self.unroll})"


_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p
_u32, _u64, _i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32

# name -> (restype, argtypes); mirrors include/talek_pir.h
SIGNATURES = {
    "pir_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pir_version": (ctypes.c_char_p, []),
    "pir_db_create": (ctypes.c_int, [_u64, _u32, _u32, ctypes.POINTER(_vp)]),
    "pir_db_destroy": (None, [_vp]),
    "pir_db_shape": (ctypes.c_int, [_vp, _u64p, _u32p, _u32p, _u64p]),
    "pir_db_write_bucket": (ctypes.c_int, [_vp, _u64, _u8p]),
    "pir_db_write_range": (ctypes.c_int, [_vp, _u64, _u64, _u8p]),
    "pir_epoch_commit": (ctypes.c_int, [_vp, _u64p]),
    "pir_epoch": (_u64, [_vp]),
    "pir_read_batch": (ctypes.c_int, [_vp, _u8p, _u32, _u8p]),
    "pir_read_batch_async": (ctypes.c_int, [_vp, _vp, _u64, _u32, _vp, _u64, _vp]),
    "pir_read_stream_async": (ctypes.c_int, [_vp, _vp, _u64, _u32p, _u64p, _u32, _vp, _u64, _u64p, _vp]),
    "pir_set_plan": (ctypes.c_int, [_vp, ctypes.POINTER(pir_plan)]),
    "pir_get_plan": (ctypes.c_int, [_vp, _u32, ctypes.POINTER(pir_plan)]),
    "pir_tune": (ctypes.c_int, [_vp, _u32, _u32, ctypes.POINTER(pir_plan), ctypes.POINTER(ctypes.c_double)]),
    "pir_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "pir_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "pir_interest_config": (ctypes.c_int, [_vp, _u64, _u32]),
    "pir_interest_add": (ctypes.c_int, [_vp, _u32p, _u32]),
    "pir_interest_vector": (ctypes.c_int, [_vp, _u8p, _u64]),
    "pir_interest_vector_async": (ctypes.c_int, [_vp, _vp, _u64, _vp]),
    "pir_cuckoo_create": (ctypes.c_int, [_vp, _u64, _u64, _u32, ctypes.POINTER(_vp)]),
    "pir_cuckoo_create_detached": (ctypes.c_int, [_u64, _u32, _u32, _u64, _u64, _u32, ctypes.POINTER(_vp)]),
    "pir_cuckoo_destroy": (None, [_vp]),
    "pir_cuckoo_insert": (ctypes.c_int, [_vp, _u64, _u64, _u64, _u8p, _u64p]),
    "pir_cuckoo_insert_many": (ctypes.c_int, [_vp, _u64, _u64p, _u64p, _u64p, _u8p, _i32p, _u64p]),
    "pir_cuckoo_stage": (ctypes.c_int, [_vp, _u64p]),
    "pir_cuckoo_table": (ctypes.c_int, [_vp, _u8p, _u64]),
    "pir_cuckoo_slots": (ctypes.c_int, [_vp, _u64p, _u8p]),
    "pir_cuckoo_live": (_u64, [_vp]),
}

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the HIP library in-tree (hipcc, gfx950)."""
    from .buildlib import build as _build
    return _build(verbose=verbose)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2001_08250_amd.build() "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_symbols() -> list[str]:
    """Every function the public header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pir_[a-z0-9_]+)\s*\(", text)))


def strerror(code: int) -> str:
    return lib().pir_strerror(code).decode()


def version() -> str:
    return lib().pir_version().decode()


def _check(rc: int, what: str):
    if rc != PIR_OK:
        raise PirError(rc, what)


def _ptr(a: np.ndarray, ct=ctypes.c_uint8):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def __getattr__(name):  # raw C entry points under their own names
    if name in SIGNATURES:
        return getattr(lib(), name)
    raise AttributeError(name)


def _stream_handle(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class PirDB:
    """One server's PIR database (n buckets x d slots x msg_bytes)."""

    def __init__(self, n: int, d: int, msg_bytes: int):
        self._L = lib()
        h = _vp()
        _check(self._L.pir_db_create(n, d, msg_bytes, ctypes.byref(h)), "pir_db_create")
        self.h = h
        self.n, self.d, self.z = n, d, msg_bytes
        self.bucket_bytes = d * msg_bytes
        self.req_bytes = (n + 7) // 8

    def close(self):
        if getattr(self, "h", None):
            self._L.pir_db_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # writes ---------------------------------------------------------------
    def write_bucket(self, bucket: int, data: np.ndarray):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size != self.bucket_bytes:
            raise ValueError("bucket data has the wrong size")
        _check(self._L.pir_db_write_bucket(self.h, bucket, _ptr(data)), "pir_db_write_bucket")

    def write_range(self, first: int, data: np.ndarray):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if data.size % self.bucket_bytes:
            raise ValueError("range data is not a whole number of buckets")
        count = data.size // self.bucket_bytes
        _check(self._L.pir_db_write_range(self.h, first, count, _ptr(data)), "pir_db_write_range")

    def commit(self) -> int:
        e = ctypes.c_uint64(0)
        _check(self._L.pir_epoch_commit(self.h, ctypes.byref(e)), "pir_epoch_commit")
        return e.value

    def load(self, D: np.ndarray) -> int:
        """Write every bucket and publish them."""
        self.write_range(0, D)
        return self.commit()

    @property
    def epoch(self) -> int:
        return int(self._L.pir_epoch(self.h))

    # reads ----------------------------------------------------------------
    def read(self, req: np.ndarray) -> np.ndarray:
        req = np.ascontiguousarray(req, dtype=np.uint8)
        if req.ndim == 1:
            req = req.reshape(1, -1)
        if req.shape[1] != self.req_bytes:
            raise ValueError(f"request rows must be {self.req_bytes} bytes")
        B = req.shape[0]
        resp = np.empty((B, self.bucket_bytes), dtype=np.uint8)
        if B:
            _check(self._L.pir_read_batch(self.h, _ptr(req), B, _ptr(resp)), "pir_read_batch")
        return resp

    def read_async(self, req, resp, stream=None):
        """Device tensors: req uint8 [B, >= req_bytes], resp uint8 [B, >= bucket_bytes]."""
        B = req.shape[0]
        rp = req.stride(0) if B > 1 else req.shape[1]
        op = resp.stride(0) if B > 1 else resp.shape[1]
        _check(self._L.pir_read_batch_async(self.h, req.data_ptr(), rp, B, resp.data_ptr(), op,
                                            _stream_handle(stream)), "pir_read_batch_async")

    def read_stream_async(self, req, sizes, resp, req_first=None, resp_first=None, stream=None):
        sizes = np.ascontiguousarray(sizes, dtype=np.uint32)
        rf = None if req_first is None else np.ascontiguousarray(req_first, dtype=np.uint64)
        of = None if resp_first is None else np.ascontiguousarray(resp_first, dtype=np.uint64)
        _check(self._L.pir_read_stream_async(
            self.h, req.data_ptr(), req.stride(0), _ptr(sizes, ctypes.c_uint32),
            None if rf is None else _ptr(rf, ctypes.c_uint64), sizes.size, resp.data_ptr(), resp.stride(0),
            None if of is None else _ptr(of, ctypes.c_uint64), _stream_handle(stream)), "pir_read_stream_async")

    # schedule ---------------------------------------------------------------
    def set_plan(self, kind=KERNEL_AUTO, tile=0, splits=0, unroll=0):
        p = pir_plan(kind, tile, splits, unroll)
        _check(self._L.pir_set_plan(self.h, ctypes.byref(p)), "pir_set_plan")

    def get_plan(self, B: int) -> pir_plan:
        p = pir_plan()
        _check(self._L.pir_get_plan(self.h, B, ctypes.byref(p)), "pir_get_plan")
        return p

    def tune(self, B: int, iters: int = 5):
        p = pir_plan()
        us = ctypes.c_double(0)
        _check(self._L.pir_tune(self.h, B, iters, ctypes.byref(p), ctypes.byref(us)), "pir_tune")
        return p, us.value

    # interest vector --------------------------------------------------------
    def interest_config(self, m_bits: int = 1 << 20, window: int = 8):
        _check(self._L.pir_interest_config(self.h, m_bits, window), "pir_interest_config")
        self.m_bits = m_bits

    def interest_add(self, pos):
        pos = np.ascontiguousarray(pos, dtype=np.uint32).reshape(-1)
        _check(self._L.pir_interest_add(self.h, _ptr(pos, ctypes.c_uint32), pos.size), "pir_interest_add")

    def interest_vector(self) -> np.ndarray:
        m = getattr(self, "m_bits", 1 << 20)
        out = np.zeros((m + 7) // 8, dtype=np.uint8)
        _check(self._L.pir_interest_vector(self.h, _ptr(out), out.size), "pir_interest_vector")
        return out


class Cuckoo:
    """The server's blocked cuckoo working copy (bound to a PirDB, or detached)."""

    def __init__(self, db: PirDB | None = None, capacity: int = 0, seed: int = 0, max_kicks: int = 500,
                 shape: tuple | None = None):
        self._L = lib()
        h = _vp()
        if db is not None:
            _check(self._L.pir_cuckoo_create(db.h, capacity, seed, max_kicks, ctypes.byref(h)), "pir_cuckoo_create")
            self.n, self.d, self.z = db.n, db.d, db.z
        else:
            n, d, z = shape
            _check(self._L.pir_cuckoo_create_detached(n, d, z, capacity, seed, max_kicks, ctypes.byref(h)),
                   "pir_cuckoo_create_detached")
            self.n, self.d, self.z = n, d, z
        self.h = h
        self.db = db

    def close(self):
        if getattr(self, "h", None):
            self._L.pir_cuckoo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, id_: int, b1: int, b2: int, payload: np.ndarray):
        payload = np.ascontiguousarray(payload, dtype=np.uint8)
        dropped = ctypes.c_uint64(0)
        rc = self._L.pir_cuckoo_insert(self.h, id_, b1, b2, _ptr(payload), ctypes.byref(dropped))
        return rc, dropped.value

    def insert_many(self, ids, b1, b2, payloads):
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        b1 = np.ascontiguousarray(b1, dtype=np.uint64)
        b2 = np.ascontiguousarray(b2, dtype=np.uint64)
        payloads = np.ascontiguousarray(payloads, dtype=np.uint8)
        status = np.zeros(ids.size, dtype=np.int32)
        dropped = np.zeros(ids.size, dtype=np.uint64)
        _check(self._L.pir_cuckoo_insert_many(self.h, ids.size, _ptr(ids, ctypes.c_uint64), _ptr(b1, ctypes.c_uint64),
                                              _ptr(b2, ctypes.c_uint64), _ptr(payloads),
                                              _ptr(status, ctypes.c_int32), _ptr(dropped, ctypes.c_uint64)),
               "pir_cuckoo_insert_many")
        return status, dropped

    def stage(self) -> int:
        k = ctypes.c_uint64(0)
        _check(self._L.pir_cuckoo_stage(self.h, ctypes.byref(k)), "pir_cuckoo_stage")
        return k.value

    def table(self) -> np.ndarray:
        out = np.empty(self.n * self.d * self.z, dtype=np.uint8)
        _check(self._L.pir_cuckoo_table(self.h, _ptr(out), out.size), "pir_cuckoo_table")
        return out.reshape(self.n, self.d * self.z)

    def slots(self):
        ids = np.zeros(self.n * self.d, dtype=np.uint64)
        occ = np.zeros(self.n * self.d, dtype=np.uint8)
        _check(self._L.pir_cuckoo_slots(self.h, _ptr(ids, ctypes.c_uint64), _ptr(occ)), "pir_cuckoo_slots")
        return ids.reshape(self.n, self.d), occ.reshape(self.n, self.d).astype(bool)

    def live(self) -> int:
        return int(self._L.pir_cuckoo_live(self.h))
