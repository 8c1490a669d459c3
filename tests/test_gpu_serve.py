"""Serving loop on the GPU: continuous batching with epoch writes.

Every probed read must equal the oracle's answer on the snapshot of the
epoch that served it (the oracle replays the same writes with its own cuckoo
table), and come back with that epoch's global interest vector; reads are
also re-asked alone (B = 1) and must give the same bytes (tolerance 0).
"""
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


N, DSLOT, Z = 4096, 4, 256
CAP = 12000
M_BITS, WINDOW, K = 1 << 16, 4, 6


def _trace(rate, duration, seed):
    read_t = synth.poisson_arrivals(seed, rate, duration)
    write_t = synth.poisson_arrivals(seed + 1, 0.1 * rate, duration)
    pool = synth.bernoulli_requests(seed + 2, 64, N)
    rows = np.random.default_rng(seed + 3).integers(0, 64, size=read_t.size).astype(np.uint32)
    return read_t, rows, pool, write_t


def _oracle_snapshots(pre, writes, write_epoch, first_epoch, last_epoch):
    """Oracle tables after each epoch first_epoch..last_epoch (writes in trace order)."""
    ref = oracle.Cuckoo(N, DSLOT, Z, capacity=CAP, seed=77, max_kicks=500)
    ref.insert_many(*pre)
    snaps = {first_epoch: ref.table()}
    ids, b1, b2, pay = writes
    for e in range(first_epoch + 1, last_epoch + 1):
        sel = np.nonzero(write_epoch == e)[0]
        if sel.size:
            ref.insert_many(ids[sel], b1[sel], b2[sel], pay[sel])
        snaps[e] = ref.table()
    return snaps


@pytest.mark.parametrize("max_batch,lanes,prep", [(64, 2, 0), (1, 3, 0), (256, 1, 0), (64, 2, 1)])
def test_serving_matches_oracle_per_epoch(max_batch, lanes, prep):
    """prep = 1: batches of 8 or more reads go through one-level Strassen
    leaves, rebuilt by every epoch commit while reads are in flight."""
    pre = synth.write_ops(501, 9000, N, Z)
    read_t, rows, pool, write_t = _trace(1500, 0.5, 600)
    writes = synth.write_ops(502, write_t.size, N, Z)
    interest = synth.interest_positions(503, write_t.size, K, M_BITS)
    with pir.PirDB(N, DSLOT, Z) as db:
        db.interest_config(M_BITS, WINDOW)
        table = pir.Cuckoo(db, capacity=CAP, seed=77)
        table.insert_many(*pre)
        table.stage()
        e0 = db.commit()
        if prep:
            db.preprocess(prep, min_batch=8)
        probe = np.arange(0, read_t.size, 3)
        say(f"serving {read_t.size} reads, {write_t.size} writes, batch<={max_batch}, lanes={lanes}")
        out = pir.serve(db, table, read_t=read_t, read_row=rows, req_pool=pool, write_t=write_t, writes=writes,
                        write_interest=interest, max_batch=max_batch, lanes=lanes, epoch_s=0.1, probe=probe,
                        with_iv=True)
        say({k: out[k] for k in ("completed", "batches", "epochs", "mean_batch", "p50_s", "p99_s")})
        assert out["completed"] == read_t.size
        assert (out["latency_s"] > 0).all()
        ep = out["read_epoch"]
        wep = out["write_epoch"]
        last = int(max(ep.max(), e0, db.epoch))
        snaps = _oracle_snapshots(pre, writes, wep, e0, last)
        # interest deltas per epoch (epoch e's delta holds the writes published by commit e)
        deltas = [np.zeros(0, np.uint32) for _ in range(last + 1)]
        for e in range(e0 + 1, last + 1):
            deltas[e] = interest[wep == e].reshape(-1)
        for k, rd in enumerate(out["probe"]):
            e = int(ep[rd])
            want = oracle.pir_read(snaps[e], pool[rows[rd]][None, :])
            assert_rows_equal(out["probe_resp"][k][None, :], want, f"read {rd} epoch {e}")
            iv = oracle.interest_window(M_BITS, deltas[1:e + 1], e - 1, WINDOW)
            assert np.array_equal(out["probe_iv"][k], iv), f"interest vector of read {rd} (epoch {e})"
        # alone (B = 1) on the published snapshot equals the oracle on it too,
        # and the probed reads that the mix answered from that snapshot give
        # the same bytes when asked again alone
        final = snaps[db.epoch]
        for r in range(0, 64, 9):
            assert_rows_equal(db.read(pool[r][None, :]), oracle.pir_read(final, pool[r][None, :]), "alone")
        again = [k for k, rd in enumerate(out["probe"]) if ep[rd] == db.epoch][:16]
        for k in again:
            rd = out["probe"][k]
            assert_rows_equal(db.read(pool[rows[rd]][None, :]), out["probe_resp"][k][None, :],
                              f"read {rd} alone vs in the mix")


def test_serving_rejects_bad_config():
    with pir.PirDB(64, 2, 16) as db:
        pool = synth.bernoulli_requests(1, 4, 64)
        with pytest.raises(pir.PirError):
            pir.serve(db, None, read_t=[0.0], read_row=[0], req_pool=pool, max_batch=0)
        with pytest.raises(pir.PirError) as e:
            pir.serve(db, None, read_t=[0.0], read_row=[9], req_pool=pool)
        assert e.value.code == pir.PIR_ERANGE


def test_serving_default_interest_vector_rows():
    """with_iv=True on a handle that kept the library's default interest
    configuration: every probed read returns the whole default-sized vector."""
    n = 256
    pre = synth.write_ops(711, 300, n, 64)
    read_t = synth.poisson_arrivals(712, 400, 0.2)
    write_t = synth.poisson_arrivals(714, 40, 0.2)
    pool = synth.bernoulli_requests(713, 8, n)
    rows = np.random.default_rng(715).integers(0, 8, size=read_t.size).astype(np.uint32)
    writes = synth.write_ops(716, write_t.size, n, 64)
    interest = synth.interest_positions(717, write_t.size, K, pir.IV_DEFAULT_BITS)
    with pir.PirDB(n, 2, 64) as db:
        table = pir.Cuckoo(db, capacity=600, seed=5)
        table.insert_many(*pre)
        table.stage()
        db.commit()
        probe = np.arange(read_t.size)
        out = pir.serve(db, table, read_t=read_t, read_row=rows, req_pool=pool, write_t=write_t, writes=writes,
                        write_interest=interest, max_batch=16, lanes=2, epoch_s=0.05, probe=probe, with_iv=True)
        assert out["probe_iv"].shape == (read_t.size, pir.IV_DEFAULT_BITS // 8)
        ep = out["read_epoch"]
        wep = out["write_epoch"]
        e_first = int(ep.min())
        deltas = [np.zeros(0, np.uint32) for _ in range(int(ep.max()) + 1)]
        for e in range(1, int(ep.max()) + 1):
            deltas[e] = interest[wep == e].reshape(-1)
        for k, rd in enumerate(probe):
            e = int(ep[rd])
            want = oracle.interest_window(pir.IV_DEFAULT_BITS, deltas[1:e + 1], e - 1, pir.IV_DEFAULT_WINDOW)
            assert np.array_equal(out["probe_iv"][k], want), f"read {rd} epoch {e} (first {e_first})"


def test_serving_budget_below_one_read_is_busy():
    """A memory budget that cannot hold one read (its request row and one
    response row) can never admit a read: PIR_EBUSY, nothing served."""
    n = 1024
    with pir.PirDB(n, 4, 256) as db:
        pool = synth.bernoulli_requests(3, 4, n)
        with pytest.raises(pir.PirError) as e:
            pir.serve(db, None, read_t=[0.0, 0.001], read_row=[0, 1], req_pool=pool, max_batch=4,
                      mem_budget=n // 8 + 4 * 256 - 1)
        assert e.value.code == pir.PIR_EBUSY
        out = pir.serve(db, None, read_t=[0.0, 0.001], read_row=[0, 1], req_pool=pool, max_batch=4,
                        mem_budget=n // 8 + 4 * 256)
        assert out["completed"] == 2
