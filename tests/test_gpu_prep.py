"""GPU parity of preprocessed (Strassen) reads against the CPU oracle.

The preprocessed path computes the same GF(2) product as the plain read by
another route (leaf databases formed at commit, 7^L leaf products, answers
XORed together); every answer must equal the plain definition bit for bit.
"""
import numpy as np
import pytest

import oracle
import paper_2001_08250_amd as pir
import synth
from helpers import assert_rows_equal, gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("n,d,z", [(2000, 2, 128), (4096, 4, 64), (333, 1, 64)])
def test_preprocessed_reads_match_oracle(levels, n, d, z):
    """Ragged n (block rows padded with zero buckets), B below, at and above
    multiples of 2^L (padded request rows), synchronous and async reads."""
    import torch
    D = synth.uniform_db(300 + n, n, d * z)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        db.preprocess(levels, min_batch=1)
        for B in (1, 3, 64, 301):
            req = synth.bernoulli_requests(400 + B, B, n)
            want = oracle.pir_read(D, req)
            assert_rows_equal(db.read(req), want, f"L={levels} B={B} sync")
            q = torch.from_numpy(req).cuda()
            out = torch.zeros((B, d * z), dtype=torch.uint8, device="cuda")
            db.read_async(q, out)
            torch.cuda.synchronize()
            assert_rows_equal(out.cpu().numpy(), want, f"L={levels} B={B} async")


_P = pir.PLAN_PAIRS
LEAF_PLANS = [(pir.KERNEL_M4R_WIDE, 32, 0, 8, _P), (pir.KERNEL_M4R_WIDE, 32, 3, 4, _P),
              (pir.KERNEL_M4R_WIDE, 16, 0, 8, _P | 4 << 8), (pir.KERNEL_M4R_WIDE, 8, 5, 8, _P | pir.PLAN_PAIR_G4),
              (pir.KERNEL_M4R_WIDE, 4, 0, 8, _P | pir.PLAN_PAIR_G3), (pir.KERNEL_M4R_WIDE, 8, 1, 8, _P | 4 << 8),
              (pir.KERNEL_M4R_WIDE, 64, 0, 8, _P | pir.PLAN_HALF_WAVES),
              (pir.KERNEL_M4R_WIDE, 32, 3, 8, _P | pir.PLAN_HALF_WAVES | pir.PLAN_PAIR_G6),
              (pir.KERNEL_M4R_WIDE, 16, 0, 8, pir.PLAN_ROLLING),
              (pir.KERNEL_MASK, 4, 0, 8, 0)]


@pytest.mark.parametrize("levels", [1, 2])
def test_leaf_reads_under_every_plan_family(levels):
    """Leaf reads under forced plans: the pair-table plans (offsets of every
    leaf staged in one launch from the request rows, every leaf answered by
    one launch) with 5-, 4- and 3-bucket tables, with and without splits and
    with ragged request tiles, and plans that read formed leaf request rows
    instead (rolling tables, masked XOR); ragged n and B, synchronous and
    async reads with unaligned request rows, all bit-exact against the
    oracle."""
    import torch
    n, d, z = 2000, 2, 512
    D = synth.uniform_db(960 + levels, n, d * z)
    reqs = {B: synth.bernoulli_requests(970 + B, B, n) for B in (5, 97, 600)}
    want = {B: oracle.pir_read(D, r, threads=8) for B, r in reqs.items()}
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        db.preprocess(levels, min_batch=1)
        for plan in LEAF_PLANS:
            db.set_plan(*plan)
            for B, req in reqs.items():
                assert_rows_equal(db.read(req), want[B], f"L={levels} plan={plan} B={B} sync")
            B = 97
            qb = reqs[B].shape[1]
            buf = torch.zeros((B, qb + 3), dtype=torch.uint8, device="cuda")
            buf[:, 1:1 + qb] = torch.from_numpy(reqs[B]).cuda()
            out = torch.zeros((B, d * z), dtype=torch.uint8, device="cuda")
            db.read_async(buf[:, 1:1 + qb], out)
            torch.cuda.synchronize()
            assert_rows_equal(out.cpu().numpy(), want[B], f"L={levels} plan={plan} B={B} async, unaligned rows")
        db.set_plan()


@pytest.mark.parametrize("levels", [1, 2])
def test_leaf_staging_16_byte_request_loads(levels):
    """Request rows of whole 16-byte units (n = 4070: 128 words, 6 bits of
    the last one used) and leaf blocks of whole 16-byte units: the staging
    loads 16 bytes at a time; host rows, device rows at a 16-byte pitch
    wider than the row, and rows at an odd pitch (restaged) all bit-exact."""
    import torch
    n, d, z = 4070, 2, 512
    D = synth.uniform_db(980 + levels, n, d * z)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        db.preprocess(levels, min_batch=1)
        for B in (97, 600):
            req = synth.bernoulli_requests(990 + B, B, n)
            want = oracle.pir_read(D, req, threads=8)
            assert_rows_equal(db.read(req), want, f"L={levels} B={B} host rows")
            qb = req.shape[1]
            for pitch, off in ((528, 0), (qb + 5, 1)):
                buf = torch.zeros((B, pitch + off), dtype=torch.uint8, device="cuda")
                buf[:, off:off + qb] = torch.from_numpy(req).cuda()
                out = torch.zeros((B, d * z), dtype=torch.uint8, device="cuda")
                db.read_async(buf[:, off:off + qb], out)
                torch.cuda.synchronize()
                assert_rows_equal(out.cpu().numpy(), want, f"L={levels} B={B} pitch {pitch} offset {off}")


@pytest.mark.parametrize("levels", [1, 2])
def test_preprocessed_reads_follow_epochs_and_masks(levels):
    """Commits that change the snapshot rebuild the leaves: reads after each
    commit see its data; masked reads give the masked answers; one-hot
    requests return single buckets; levels 0 returns to the plain path."""
    n, d, z, B = 1024, 2, 128, 96
    rng = np.random.default_rng(7 + levels)
    D = synth.uniform_db(500, n, d * z)
    req = synth.bernoulli_requests(501, B, n)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        db.preprocess(levels, min_batch=B)
        for e in range(3):
            published = D.copy()
            for b in rng.choice(n, size=17, replace=False):
                D[b] = rng.integers(0, 256, d * z, dtype=np.uint8)
                db.write_bucket(int(b), D[b])
            assert_rows_equal(db.read(req), oracle.pir_read(published, req), "staged, not yet published")
            db.commit()
            assert_rows_equal(db.read(req), oracle.pir_read(D, req), f"epoch {e}")
        seeds = synth.uniform_bytes(502, B * 32).reshape(B, 32)
        assert_rows_equal(db.read_masked(req, seeds), oracle.pir_read_masked(D, req, seeds), "masked")
        onehot = np.zeros((B, (n + 7) // 8), dtype=np.uint8)
        for r in range(B):
            j = (r * 37) % n
            onehot[r, j >> 3] = 1 << (j & 7)
        got = db.read(onehot)
        for r in range(B):
            assert np.array_equal(got[r], D[(r * 37) % n]), f"one-hot row {r}"
        db.preprocess(0)
        assert_rows_equal(db.read(req), oracle.pir_read(D, req), "plain path again")


def test_preprocess_rejects_bad_levels_and_shapes():
    """Blocks of buckets must be whole multiples of 16 bytes: 16 << levels
    must divide d * msg_bytes; at most two levels."""
    with pir.PirDB(64, 1, 24) as db:                # 24-byte buckets
        with pytest.raises(pir.PirError):
            db.preprocess(1)
    with pir.PirDB(64, 1, 32) as db:                # 32-byte buckets: one level only
        with pytest.raises(pir.PirError):
            db.preprocess(3)
        with pytest.raises(pir.PirError):
            db.preprocess(2)
        db.preprocess(1)
        db.preprocess(0)


def test_stream_and_commits_with_preprocessing_on():
    """With the leaves on, the uneven-batch stream (plain path) still answers
    every batch from the published snapshot, and commits between streams
    rebuild the leaves that a large read then uses."""
    import torch
    n, d, z = 2048, 2, 128
    rng = np.random.default_rng(91)
    D = synth.uniform_db(92, n, d * z)
    sizes = np.array([5, 70, 300, 1], dtype=np.uint64)
    pool = synth.bernoulli_requests(93, 400, n)
    first = np.array([0, 10, 50, 399], dtype=np.uint64)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        db.preprocess(1, min_batch=64)
        q = torch.from_numpy(pool).cuda()
        out = torch.zeros((int(sizes.sum()), d * z), dtype=torch.uint8, device="cuda")
        for rep in range(2):
            for b in rng.choice(n, size=9, replace=False):
                D[b] = rng.integers(0, 256, d * z, dtype=np.uint8)
                db.write_bucket(int(b), D[b])
            db.commit()
            out.zero_()
            db.read_stream_async(q, sizes, out, req_first=first)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            row = 0
            for k, s in enumerate(sizes):
                s = int(s)
                want = oracle.pir_read(D, pool[int(first[k]):int(first[k]) + s])
                assert_rows_equal(got[row:row + s], want, f"rep {rep} batch {k} (B={s})")
                row += s
            assert_rows_equal(db.read(pool[:300]), oracle.pir_read(D, pool[:300]), f"rep {rep} leaves")


@pytest.mark.parametrize("levels,n,d,z", [(1, 300, 1, 8192), (1, 300, 1, 16384), (2, 300, 1, 16384),
                                          (1, 301, 1, 96), (2, 77, 3, 64)])
def test_leaf_database_shapes(levels, n, d, z):
    """Leaf databases whose blocks are as wide as a workgroup of 16-byte
    columns or wider (one row per block, or several columns per thread), and
    blocks of a few columns that do not divide the workgroup: every answer
    bit-exact against the oracle."""
    D = synth.uniform_db(900 + n + z, n, d * z)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        db.preprocess(levels, min_batch=1)
        for B in (2, 33):
            req = synth.bernoulli_requests(950 + B + z, B, n)
            assert_rows_equal(db.read(req), oracle.pir_read(D, req), f"L={levels} n={n} bucket={d * z} B={B}")


@pytest.mark.parametrize("levels", [1, 2])
def test_commits_update_only_the_leaf_rows_they_feed(levels):
    """A commit of a few buckets recomputes only the leaf rows those buckets
    feed (buckets in different row blocks of one leaf row among them); a
    commit of many rebuilds every leaf; every read after every commit equals
    the oracle on the published snapshot."""
    n, d, z, B = 1000, 2, 64, 40
    nq = (-(-n // (1 << levels)) + 31) // 32 * 32   # bucket rows per block (the library pads to 32)
    rng = np.random.default_rng(70 + levels)
    D = synth.uniform_db(71, n, d * z)
    req = synth.bernoulli_requests(72, B, n)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        db.preprocess(levels, min_batch=1)
        plans = [[5, 5 + nq], [0, n - 1, nq - 1], list(rng.choice(n, size=3, replace=False)),
                 list(rng.choice(n, size=nq // 2, replace=False)), [7]]
        for e, rows in enumerate(plans):
            for b in rows:
                D[b] = rng.integers(0, 256, d * z, dtype=np.uint8)
                db.write_bucket(int(b), D[b])
            db.commit()
            assert_rows_equal(db.read(req), oracle.pir_read(D, req), f"L={levels} commit {e} ({len(rows)} buckets)")
