"""The allocation-free read entry point (pir_read_batch_noalloc_async), called
through the C ABI: its answers equal pir_read_batch_async's (and the
oracle's) bit for bit, on two calls in a row, the second with a smaller
batch, including schedules whose splits must shrink to fit the static
scratch, the masked-kernel fallback and restaged (unaligned) rows."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2001_08250_amd as pir
import synth
from helpers import assert_rows_equal, gpu_available, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _noalloc(db, q, out, B, stream=0):
    L = pir.lib()
    rp = q.stride(0) if B > 1 else q.shape[1]
    op = out.stride(0) if B > 1 else out.shape[1]
    return L.pir_read_batch_noalloc_async(db.h, ctypes.c_void_p(q.data_ptr()), rp, B,
                                          ctypes.c_void_p(out.data_ptr()), op, ctypes.c_void_p(stream))


# (n, d, z, first B, second B): c2-shaped paired tables whose 64 splits of
# partials exceed the scratch; a batch whose Four-Russians offsets alone
# exceed it (masked kernel); ragged rows that are restaged both ways
CASES = [(65536, 4, 1024, 256, 40), (65536, 4, 1024, 2048, 300), (1000, 3, 100, 70, 9)]


@pytest.mark.parametrize("n,d,z,B1,B2", CASES)
def test_noalloc_equals_async(n, d, z, B1, B2):
    import torch
    dev = torch.device("cuda:0")
    D = synth.uniform_db(4401 + n, n, d * z)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        for k, B in enumerate((B1, B2)):
            req = synth.bernoulli_requests(4500 + 7 * k + B, B, n)
            q = torch.from_numpy(req).to(dev)
            if n % 32:
                # rows one byte off 4-byte alignment, answers at an odd pitch
                qbuf = torch.zeros((B, req.shape[1] + 3), dtype=torch.uint8, device=dev)
                qbuf[:, 1:1 + req.shape[1]] = q
                q = qbuf[:, 1:1 + req.shape[1]]
                out = torch.zeros((B, d * z + 5), dtype=torch.uint8, device=dev)[:, :d * z]
            else:
                out = torch.zeros((B, d * z), dtype=torch.uint8, device=dev)
            ref = torch.zeros((B, d * z), dtype=torch.uint8, device=dev)
            say(f"noalloc n={n} d={d} z={z} call {k + 1}: B={B}")
            assert _noalloc(db, q, out, B) == 0
            db.read_async(q, ref)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert_rows_equal(got, ref.cpu().numpy(), f"noalloc vs async, B={B}")
            rows = np.unique(np.linspace(0, B - 1, min(B, 12)).round().astype(np.int64))
            assert_rows_equal(got[rows], oracle.pir_read(D, req[rows], threads=8), f"noalloc vs oracle, B={B}")


def test_noalloc_allocates_nothing():
    """After one warm call, further calls (a smaller batch, then a larger one)
    leave the device's free memory unchanged."""
    import torch
    n, d, z = 4096, 4, 256
    D = synth.uniform_db(4601, n, d * z)
    dev = torch.device("cuda:0")
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        qs = [torch.from_numpy(synth.bernoulli_requests(4602 + B, B, n)).to(dev) for B in (200, 20, 130)]
        outs = [torch.zeros((q.shape[0], d * z), dtype=torch.uint8, device=dev) for q in qs]
        assert _noalloc(db, qs[0], outs[0], qs[0].shape[0]) == 0
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for q, out in zip(qs[1:], outs[1:]):
            assert _noalloc(db, q, out, q.shape[0]) == 0
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        for q, out in zip(qs, outs):
            want = oracle.pir_read(D, q.cpu().numpy(), threads=8)
            assert_rows_equal(out.cpu().numpy(), want, f"B={q.shape[0]}")


def test_noalloc_rejects_oversized_restaging():
    """Unaligned rows whose restaging alone would exceed the static scratch."""
    import torch
    n = (1 << 20) + 1          # ceil(n/8) = 131,073: rows are restaged
    B = 300                    # 300 x 131,088 bytes > 32 MiB
    with pir.PirDB(n, 1, 16) as db:
        q = torch.zeros((B, (n + 7) // 8), dtype=torch.uint8, device="cuda")
        out = torch.zeros((B, 16), dtype=torch.uint8, device="cuda")
        assert _noalloc(db, q, out, B) == pir.PIR_ERANGE
        assert _noalloc(db, q[:8], out[:8], 8) == 0
        torch.cuda.synchronize()
        assert not out.cpu().numpy().any()
