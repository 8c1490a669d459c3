"""Full-size parity: the paper-shaped workloads at their real sizes.

* n = 65,536 x 4 KiB, cuckoo-filled with 200,000 messages, B = 256: the
  library's cuckoo table must equal the oracle's byte for byte, and every one
  of the 256 answers must equal the oracle's.
* n = 2^20 x 4 KiB (4 GiB) uneven batch stream through the fused launch
  groups replayed from a HIP graph; n = 2^22 x 4 KiB (16 GiB) and n = 2^20 x 8 KiB (8 GiB) with
  B = 2048: seeded sampled rows against the oracle (each oracle row scans the
  whole database on the CPU).
Every kernel family is run at the full size too (sampled rows).
"""
import os

import numpy as np
import pytest

import oracle
import paper_2001_08250_amd as pir
import synth
from helpers import assert_rows_equal, gpu_available, say
from synth import configs

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def test_cuckoo_filled_65536_full_parity():
    w = configs.C2
    say("building the 200k-message cuckoo table (library and oracle)")
    ops = synth.write_ops(w.cuckoo_seed, w.cuckoo_items, w.n, w.z)
    ref = oracle.Cuckoo(w.n, w.d, w.z, capacity=w.cuckoo_items, seed=w.cuckoo_seed, max_kicks=500)
    st_ref, _ = ref.insert_many(*ops)
    D = ref.table()
    req = synth.bernoulli_requests(w.req_seed, w.B, w.n)
    with pir.PirDB(w.n, w.d, w.z) as db:
        ck = pir.Cuckoo(db, capacity=w.cuckoo_items, seed=w.cuckoo_seed, max_kicks=500)
        st, _ = ck.insert_many(*ops)
        assert np.array_equal(st, st_ref)
        assert np.array_equal(ck.table(), D), "library working copy differs from the oracle's table"
        ck.stage()
        db.commit()
        say("oracle: 256 rows over 256 MiB")
        want = oracle.pir_read(D, req, threads=THREADS)
        assert_rows_equal(db.read(req), want, "auto plan")
        R = pir.PLAN_ROLLING
        for kind, tile, unroll, fl in ((pir.KERNEL_MASK, 16, 8, 0), (pir.KERNEL_SKIP, 16, 4, 0),
                                       (pir.KERNEL_M4R, 16, 16, 0), (pir.KERNEL_M4R, 32, 8, 0),
                                       (pir.KERNEL_M4R_WIDE, 32, 8, 0), (pir.KERNEL_M4R_WIDE, 16, 16, 0),
                                       (pir.KERNEL_M4R_WIDE, 16, 16, R), (pir.KERNEL_M4R_WIDE, 32, 8, R),
                                       (pir.KERNEL_M4R_WIDE, 8, 4, R),
                                       (pir.KERNEL_M4R_WIDE, 32, 8, pir.PLAN_PAIRS),
                                       (pir.KERNEL_M4R_WIDE, 16, 8, pir.PLAN_PAIRS | pir.PLAN_PAIR_G4),
                                       (pir.KERNEL_M4R_WIDE, 8, 8, pir.PLAN_PAIRS | pir.PLAN_PAIR_G3)):
            db.set_plan(kind, tile, 0, unroll, fl)
            say(f"kind={kind} tile={tile} unroll={unroll} flags={fl:#x}")
            assert_rows_equal(db.read(req), want, f"kind={kind} tile={tile} unroll={unroll} flags={fl:#x}")


def _sampled(db, D, req, rows, what):
    got = db.read(req)
    want = oracle.pir_read(D, req[rows], threads=THREADS)
    assert_rows_equal(got[rows], want, what)
    return got


@pytest.mark.parametrize("key", ["c4b", "c4a"])
def test_large_batch_sampled_rows(key):
    w = configs.BY_KEY[key]
    say(f"generating {w.db_bytes >> 30} GiB database for {w.name}")
    D = synth.uniform_db(w.db_seed, w.n, w.bucket_bytes, threads=THREADS)
    req = synth.bernoulli_requests(w.req_seed, w.B, w.n)
    rows = np.sort(np.random.default_rng(w.req_seed).choice(w.B, size=16, replace=False))
    with pir.PirDB(w.n, w.d, w.z) as db:
        db.load(D)
        say(f"{w.name}: auto plan {db.get_plan(w.B)}")
        _sampled(db, D, req, rows, f"{w.name} auto")
        for kind, tile, unroll, fl in ((pir.KERNEL_MASK, 16, 8, 0), (pir.KERNEL_M4R, 32, 16, 0),
                                       (pir.KERNEL_M4R_WIDE, 32, 8, 0), (pir.KERNEL_M4R_WIDE, 16, 16, pir.PLAN_ROLLING),
                                       (pir.KERNEL_M4R_WIDE, 32, 8, pir.PLAN_PAIRS),
                                       (pir.KERNEL_M4R_WIDE, 16, 8, pir.PLAN_PAIRS | pir.PLAN_PAIR_G4)):
            db.set_plan(kind, tile, 0, unroll, fl)
            say(f"{w.name}: kind={kind} tile={tile}")
            _sampled(db, D, req, rows[:4], f"{w.name} kind={kind}")


def test_uneven_stream_1m_buckets_sampled():
    import torch
    w = configs.C3
    nb = 40
    sizes = synth.batch_sizes(w.batch_seed, nb)
    say(f"generating 4 GiB database; stream of {nb} batches, {int(sizes.sum())} reads")
    D = synth.uniform_db(w.db_seed, w.n, w.bucket_bytes, threads=THREADS)
    pool = synth.bernoulli_requests(w.req_seed, 1024, w.n)
    rng = np.random.default_rng(w.batch_seed)
    first = np.array([rng.integers(0, 1024 - s + 1) for s in sizes], dtype=np.uint64)
    total = int(sizes.sum())
    dev = torch.device("cuda:0")
    with pir.PirDB(w.n, w.d, w.z) as db:
        db.load(D)
        q = torch.from_numpy(pool).to(dev)
        out = torch.zeros((total, w.bucket_bytes), dtype=torch.uint8, device=dev)
        db.read_stream_async(q, sizes, out, req_first=first)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # two sampled rows from each of 8 sampled batches
        pick = np.sort(rng.choice(nb, size=8, replace=False))
        starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        rows, pool_rows = [], []
        for k in pick:
            for i in rng.choice(int(sizes[k]), size=min(2, int(sizes[k])), replace=False):
                rows.append(int(starts[k] + i))
                pool_rows.append(int(first[k] + i))
        say(f"oracle: {len(rows)} sampled rows over 4 GiB")
        want = oracle.pir_read(D, pool[pool_rows], threads=THREADS)
        assert_rows_equal(got[rows], want, "stream sampled rows")
