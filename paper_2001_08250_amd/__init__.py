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
KERNEL_AUTO, KERNEL_MASK, KERNEL_SKIP, KERNEL_M4R, KERNEL_M4R_WIDE = 0, 1, 2, 3, 4
PLAN_SHARED_COLUMN = 1
PLAN_ROLLING = 1 << 12
PLAN_PAIRS = 1 << 13
PLAN_PAIR_G4 = 1 << 14     # with PLAN_PAIRS: 4-bucket tables
PLAN_PAIR_G3 = 2 << 14     # with PLAN_PAIRS: 3-bucket tables
PLAN_HALF_WAVES = 1 << 16  # with PLAN_PAIRS: 512-byte entries, a request per half wave
PLAN_PAIR_G6 = 1 << 17     # with PLAN_PAIRS | PLAN_HALF_WAVES: 6-bucket tables
PROFILE_MAX = 4096
IV_DEFAULT_BITS, IV_DEFAULT_WINDOW = 1 << 17, 100   # the library's interest-vector defaults


class PirError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class pir_plan(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tile", ctypes.c_uint32), ("splits", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32), ("flags", ctypes.c_uint32)]

    def __repr__(self):
        return (f"pir_plan(kind={self.kind}, tile={self.tile}, splits={self.splits}, unroll={self.unroll}, "
                f"flags={self.flags})")


_dp = ctypes.POINTER(ctypes.c_double)


class pir_serve_config(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("lanes", ctypes.c_uint32), ("mem_budget", ctypes.c_uint64),
                ("epoch_s", ctypes.c_double), ("interest_k", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class pir_serve_trace(ctypes.Structure):
    _fields_ = [("n_reads", ctypes.c_uint64), ("read_t", _dp), ("read_row", ctypes.POINTER(ctypes.c_uint32)),
                ("req_pool", ctypes.POINTER(ctypes.c_uint8)), ("pool_rows", ctypes.c_uint64),
                ("n_writes", ctypes.c_uint64), ("write_t", _dp), ("write_id", ctypes.POINTER(ctypes.c_uint64)),
                ("write_beta1", ctypes.POINTER(ctypes.c_uint64)), ("write_beta2", ctypes.POINTER(ctypes.c_uint64)),
                ("write_payload", ctypes.POINTER(ctypes.c_uint8)),
                ("write_interest", ctypes.POINTER(ctypes.c_uint32))]


class pir_serve_result(ctypes.Structure):
    _fields_ = [("latency_s", _dp), ("read_epoch", ctypes.POINTER(ctypes.c_uint64)), ("n_probe", ctypes.c_uint64),
                ("probe", ctypes.POINTER(ctypes.c_uint64)), ("probe_resp", ctypes.POINTER(ctypes.c_uint8)),
                ("probe_iv", ctypes.POINTER(ctypes.c_uint8)), ("write_epoch", ctypes.POINTER(ctypes.c_uint64)),
                ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("epochs", ctypes.c_uint64), ("writes_applied", ctypes.c_uint64),
                ("writes_failed", ctypes.c_uint64), ("max_queue", ctypes.c_uint64), ("wall_s", ctypes.c_double),
                ("reads_per_s", ctypes.c_double), ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("max_s", ctypes.c_double), ("mean_batch", ctypes.c_double)]


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
    "pir_db_write_bucket": (ctypes.c_int, [_vp, _u64, _vp]),
    "pir_db_write_range": (ctypes.c_int, [_vp, _u64, _u64, _u8p]),
    "pir_epoch_commit": (ctypes.c_int, [_vp, _u64p]),
    "pir_epoch": (_u64, [_vp]),
    "pir_read_batch": (ctypes.c_int, [_vp, _u8p, _u32, _u8p]),
    "pir_read_batch_async": (ctypes.c_int, [_vp, _vp, _u64, _u32, _vp, _u64, _vp]),
    "pir_read_batch_noalloc_async": (ctypes.c_int, [_vp, _vp, _u64, _u32, _vp, _u64, _vp]),
    "pir_read_stream_async": (ctypes.c_int, [_vp, _vp, _u64, _u32p, _u64p, _u32, _vp, _u64, _u64p, _vp]),
    "pir_read_batch_masked": (ctypes.c_int, [_vp, _u8p, _u32, _u8p, _u8p]),
    "pir_read_batch_masked_async": (ctypes.c_int, [_vp, _vp, _u64, _u32, _vp, _vp, _u64, _vp]),
    "pir_xor_combine_async": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(_vp), _u32, _u64, _u32, _u64, _vp]),
    "pir_set_plan": (ctypes.c_int, [_vp, ctypes.POINTER(pir_plan)]),
    "pir_get_plan": (ctypes.c_int, [_vp, _u32, ctypes.POINTER(pir_plan)]),
    "pir_tune": (ctypes.c_int, [_vp, _u32, _u32, ctypes.POINTER(pir_plan), ctypes.POINTER(ctypes.c_double)]),
    "pir_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "pir_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "pir_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "pir_profile_collect": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_uint32,
                                           ctypes.POINTER(ctypes.c_uint32)]),
    "pir_interest_config": (ctypes.c_int, [_vp, _u64, _u32]),
    "pir_interest_add": (ctypes.c_int, [_vp, _vp, _u32]),
    "pir_preprocess": (ctypes.c_int, [_vp, _u32, _u32]),
    "pir_preprocess_tables": (ctypes.c_int, [_u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pir_interest_vector": (ctypes.c_int, [_vp, _u8p, _u64]),
    "pir_interest_vector_async": (ctypes.c_int, [_vp, _vp, _u64, _vp]),
    "pir_interest_vector_encoded": (ctypes.c_int, [_vp, _u8p, _u64, _u64p]),
    "pir_interest_delta_encoded": (ctypes.c_int, [_vp, _u64, _u8p, _u64, _u64p]),
    "pir_cuckoo_create": (ctypes.c_int, [_vp, _u64, _u64, _u32, ctypes.POINTER(_vp)]),
    "pir_cuckoo_create_detached": (ctypes.c_int, [_u64, _u32, _u32, _u64, _u64, _u32, ctypes.POINTER(_vp)]),
    "pir_cuckoo_destroy": (None, [_vp]),
    "pir_cuckoo_insert": (ctypes.c_int, [_vp, _u64, _u64, _u64, _u8p, _u64p]),
    "pir_cuckoo_insert_many": (ctypes.c_int, [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pir_cuckoo_stage": (ctypes.c_int, [_vp, _u64p]),
    "pir_cuckoo_table": (ctypes.c_int, [_vp, _u8p, _u64]),
    "pir_cuckoo_slots": (ctypes.c_int, [_vp, _u64p, _u8p]),
    "pir_cuckoo_live": (_u64, [_vp]),
    "pir_serve_run": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(pir_serve_config), ctypes.POINTER(pir_serve_trace),
                                     ctypes.POINTER(pir_serve_result)]),
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


def _addr(a: np.ndarray) -> int:
    """Address of a contiguous array's data, for void-pointer arguments (a few
    times cheaper than building a typed ctypes pointer on every call)."""
    return a.__array_interface__["data"][0]


def __getattr__(name):  # raw C entry points under their own names
    if name in SIGNATURES:
        return getattr(lib(), name)
    raise AttributeError(name)


def xor_combine_async(out, ins, stream=None):
    """Leader combine: out[r] = XOR of ins[i][r] (device uint8 tensors [B, row_bytes])."""
    B, row = out.shape
    ptrs = (ctypes.c_void_p * len(ins))(*[t.data_ptr() for t in ins])
    op = out.stride(0) if B > 1 else row
    ip = ins[0].stride(0) if B > 1 else row
    if any(t.stride(0) != ins[0].stride(0) or tuple(t.shape) != (B, row) for t in ins):
        raise ValueError("inputs must share shape and row pitch")
    _check(lib().pir_xor_combine_async(out.data_ptr(), op, ptrs, len(ins), ip, B, row, _stream_handle(stream)),
           "pir_xor_combine_async")


def preprocess_tables(levels: int) -> dict:
    """The Strassen leaf tables of `levels` levels (see pir_preprocess_tables)."""
    leaves = np.zeros(1, dtype=np.uint32)
    a_cnt, d_cnt = np.zeros(49, np.uint8), np.zeros(49, np.uint8)
    a, d = np.zeros(196, np.uint8), np.zeros(196, np.uint8)
    o_cnt, o_leaf = np.zeros(16, np.uint8), np.zeros(256, np.uint8)
    _check(lib().pir_preprocess_tables(levels, _addr(leaves), _addr(a_cnt), _addr(a), _addr(d_cnt), _addr(d),
                                       _addr(o_cnt), _addr(o_leaf)), "pir_preprocess_tables")
    L = int(leaves[0])
    g = 1 << levels
    unpack = lambda v: (int(v) >> 4, int(v) & 15)
    return {"grid": g,
            "a": [[unpack(x) for x in a[4 * i:4 * i + int(a_cnt[i])]] for i in range(L)],
            "d": [[unpack(x) for x in d[4 * i:4 * i + int(d_cnt[i])]] for i in range(L)],
            "out": [[int(x) for x in o_leaf[16 * b:16 * b + int(o_cnt[b])]] for b in range(g * g)]}


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
        _check(self._L.pir_db_write_bucket(self.h, bucket, _addr(data)), "pir_db_write_bucket")

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

    def read_masked(self, req: np.ndarray, seeds: np.ndarray) -> np.ndarray:
        """Serialized-PIR answers: each row XOR the one-time mask of its 32-byte seed."""
        req = np.ascontiguousarray(req, dtype=np.uint8)
        if req.ndim == 1:
            req = req.reshape(1, -1)
        if req.shape[1] != self.req_bytes:
            raise ValueError(f"request rows must be {self.req_bytes} bytes")
        B = req.shape[0]
        seeds = np.ascontiguousarray(seeds, dtype=np.uint8).reshape(-1, 32)
        if seeds.shape[0] != B:
            raise ValueError("one 32-byte seed per request")
        resp = np.empty((B, self.bucket_bytes), dtype=np.uint8)
        if B:
            _check(self._L.pir_read_batch_masked(self.h, _ptr(req), B, _ptr(seeds), _ptr(resp)),
                   "pir_read_batch_masked")
        return resp

    def read_masked_async(self, req, seeds, resp, stream=None):
        """Device tensors: req [B, >= req_bytes], seeds uint8 [B, 32] (contiguous), resp [B, >= bucket_bytes]."""
        B = req.shape[0]
        rp = req.stride(0) if B > 1 else req.shape[1]
        op = resp.stride(0) if B > 1 else resp.shape[1]
        if tuple(seeds.shape) != (B, 32) or not seeds.is_contiguous():
            raise ValueError("seeds must be a contiguous [B, 32] uint8 tensor")
        _check(self._L.pir_read_batch_masked_async(self.h, req.data_ptr(), rp, B, seeds.data_ptr(),
                                                   resp.data_ptr(), op, _stream_handle(stream)),
               "pir_read_batch_masked_async")

    def read_stream_async(self, req, sizes, resp, req_first=None, resp_first=None, stream=None):
        sizes = np.ascontiguousarray(sizes, dtype=np.uint32)
        rf = None if req_first is None else np.ascontiguousarray(req_first, dtype=np.uint64)
        of = None if resp_first is None else np.ascontiguousarray(resp_first, dtype=np.uint64)
        _check(self._L.pir_read_stream_async(
            self.h, req.data_ptr(), req.stride(0), _ptr(sizes, ctypes.c_uint32),
            None if rf is None else _ptr(rf, ctypes.c_uint64), sizes.size, resp.data_ptr(), resp.stride(0),
            None if of is None else _ptr(of, ctypes.c_uint64), _stream_handle(stream)), "pir_read_stream_async")

    # schedule ---------------------------------------------------------------
    def set_plan(self, kind=KERNEL_AUTO, tile=0, splits=0, unroll=0, flags=0):
        p = pir_plan(kind, tile, splits, unroll, flags)
        _check(self._L.pir_set_plan(self.h, ctypes.byref(p)), "pir_set_plan")

    def get_plan(self, B: int) -> pir_plan:
        p = pir_plan()
        _check(self._L.pir_get_plan(self.h, B, ctypes.byref(p)), "pir_get_plan")
        return p

    def profile_enable(self, on: bool = True, every: int = 1):
        """Time the main read kernel of every `every`-th read from now on (False: stop)."""
        _check(self._L.pir_profile_enable(self.h, max(1, int(every)) if on else 0), "pir_profile_enable")

    def profile_collect(self) -> np.ndarray:
        """Main read kernel durations (ms) of the reads since profile_enable."""
        buf = np.zeros(PROFILE_MAX, dtype=np.float32)
        cnt = ctypes.c_uint32(0)
        _check(self._L.pir_profile_collect(self.h, _ptr(buf, ctypes.c_float), PROFILE_MAX, ctypes.byref(cnt)),
               "pir_profile_collect")
        return buf[:cnt.value].copy()

    def tune(self, B: int, iters: int = 5):
        p = pir_plan()
        us = ctypes.c_double(0)
        _check(self._L.pir_tune(self.h, B, iters, ctypes.byref(p), ctypes.byref(us)), "pir_tune")
        return p, us.value

    # interest vector --------------------------------------------------------
    def interest_config(self, m_bits: int = IV_DEFAULT_BITS, window: int = IV_DEFAULT_WINDOW):
        _check(self._L.pir_interest_config(self.h, m_bits, window), "pir_interest_config")
        self.m_bits = m_bits

    def preprocess(self, levels: int, min_batch: int = 0):
        """Strassen-preprocessed reads for batches of >= min_batch rows (0: 256 << levels);
        levels 0 turns them off."""
        _check(self._L.pir_preprocess(self.h, levels, min_batch), "pir_preprocess")

    def interest_add(self, pos):
        pos = np.ascontiguousarray(pos, dtype=np.uint32).reshape(-1)
        _check(self._L.pir_interest_add(self.h, _addr(pos), pos.size), "pir_interest_add")

    def interest_encoded(self, epoch: int | None = None) -> bytes:
        """Compressed stream of the global vector (epoch None) or of a published
        epoch's delta still in the window."""
        size = ctypes.c_uint64(0)
        if epoch is None:
            call = lambda buf, cap: self._L.pir_interest_vector_encoded(self.h, buf, cap, ctypes.byref(size))
        else:
            call = lambda buf, cap: self._L.pir_interest_delta_encoded(self.h, epoch, buf, cap, ctypes.byref(size))
        _check(call(None, 0), "interest_encoded (size)")
        out = np.zeros(size.value, dtype=np.uint8)
        _check(call(_ptr(out), out.size), "interest_encoded")
        return out.tobytes()

    def interest_vector(self) -> np.ndarray:
        m = getattr(self, "m_bits", IV_DEFAULT_BITS)
        out = np.zeros((m + 7) // 8, dtype=np.uint8)
        _check(self._L.pir_interest_vector(self.h, _ptr(out), out.size), "pir_interest_vector")
        return out


def serve(db: "PirDB", table: "Cuckoo | None", *, read_t, read_row, req_pool, write_t=None, writes=None,
          write_interest=None, max_batch=512, lanes=2, mem_budget=0, epoch_s=1.0, probe=None, with_iv=False):
    """Run the native serving loop (pir_serve_run) on a timed trace.

    writes = (ids, beta1, beta2, payload) arrays; write_interest uint32 [n_writes, k].
    Returns a dict with the summary, per-read latency/epoch and probe responses.
    """
    L = lib()
    read_t = np.ascontiguousarray(read_t, dtype=np.float64)
    read_row = np.ascontiguousarray(read_row, dtype=np.uint32)
    req_pool = np.ascontiguousarray(req_pool, dtype=np.uint8)
    tr = pir_serve_trace()
    tr.n_reads = read_t.size
    tr.read_t = read_t.ctypes.data_as(_dp)
    tr.read_row = _ptr(read_row, ctypes.c_uint32)
    tr.req_pool = _ptr(req_pool)
    tr.pool_rows = req_pool.shape[0]
    keep = [read_t, read_row, req_pool]
    k = 0
    if writes is not None and len(writes[0]):
        ids, b1, b2, pay = (np.ascontiguousarray(writes[0], dtype=np.uint64),
                            np.ascontiguousarray(writes[1], dtype=np.uint64),
                            np.ascontiguousarray(writes[2], dtype=np.uint64),
                            np.ascontiguousarray(writes[3], dtype=np.uint8))
        wt = np.ascontiguousarray(write_t, dtype=np.float64)
        tr.n_writes = ids.size
        tr.write_t = wt.ctypes.data_as(_dp)
        tr.write_id = _ptr(ids, ctypes.c_uint64)
        tr.write_beta1 = _ptr(b1, ctypes.c_uint64)
        tr.write_beta2 = _ptr(b2, ctypes.c_uint64)
        tr.write_payload = _ptr(pay)
        keep += [ids, b1, b2, pay, wt]
        if write_interest is not None:
            wi = np.ascontiguousarray(write_interest, dtype=np.uint32)
            k = wi.shape[1] if wi.ndim == 2 else 0
            tr.write_interest = _ptr(wi, ctypes.c_uint32)
            keep.append(wi)
    cfg = pir_serve_config(max_batch, lanes, mem_budget, epoch_s, k, 0)
    res = pir_serve_result()
    lat = np.zeros(read_t.size, dtype=np.float64)
    ep = np.zeros(read_t.size, dtype=np.uint64)
    res.latency_s = lat.ctypes.data_as(_dp)
    res.read_epoch = _ptr(ep, ctypes.c_uint64)
    probe = np.zeros(0, np.uint64) if probe is None else np.ascontiguousarray(np.sort(probe), dtype=np.uint64)
    presp = np.zeros((probe.size, db.bucket_bytes), dtype=np.uint8)
    piv = np.zeros((probe.size, (getattr(db, "m_bits", IV_DEFAULT_BITS) + 7) // 8), dtype=np.uint8) if with_iv else None
    res.n_probe = probe.size
    res.probe = _ptr(probe, ctypes.c_uint64)
    res.probe_resp = _ptr(presp)
    if piv is not None:
        res.probe_iv = _ptr(piv)
    wep = np.zeros(tr.n_writes, dtype=np.uint64)
    res.write_epoch = _ptr(wep, ctypes.c_uint64)
    _check(L.pir_serve_run(db.h, table.h if table is not None else None, ctypes.byref(cfg), ctypes.byref(tr),
                           ctypes.byref(res)), "pir_serve_run")
    out = {f: getattr(res, f) for f, _ in pir_serve_result._fields_
           if f not in ("latency_s", "read_epoch", "n_probe", "probe", "probe_resp", "probe_iv", "write_epoch")}
    out.update(latency_s=lat, read_epoch=ep, probe=probe, probe_resp=presp, probe_iv=piv, write_epoch=wep)
    del keep
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
        _check(self._L.pir_cuckoo_insert_many(self.h, ids.size, _addr(ids), _addr(b1), _addr(b2), _addr(payloads),
                                              _addr(status), _addr(dropped)), "pir_cuckoo_insert_many")
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
