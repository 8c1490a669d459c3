"""GPU parity of the read path against the CPU oracle (bit-exact, tolerance 0).

Every read goes through the C ABI of libtalek_pir.so on the GPU; the expected
rows come from oracle/ on the same seeded inputs.
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


def _db(D, d, z):
    n = D.shape[0]
    db = pir.PirDB(n, d, z)
    db.load(D)
    return db


TILES = [1, 2, 4, 8, 16, 24, 32]


@pytest.mark.parametrize("kind", [pir.KERNEL_MASK, pir.KERNEL_SKIP])
def test_small_workload_every_tile_schedule(kind):
    """n = 1024, 4 KiB buckets, B = 8 (plus B = 37 for ragged tiles): all rows."""
    n, d, z = 1024, 4, 1024
    D = synth.uniform_db(1001, n, d * z)
    req8 = synth.bernoulli_requests(2001, 8, n)
    req37 = synth.bernoulli_requests(2101, 37, n)
    want8 = oracle.pir_read(D, req8, threads=8)
    want37 = oracle.pir_read(D, req37, threads=8)
    with _db(D, d, z) as db:
        for fl in (0, pir.PLAN_SHARED_COLUMN):
            for t in TILES:
                for u in (4, 8, 16):
                    if fl and (t < 4 or u == 16):
                        with pytest.raises(pir.PirError):
                            db.set_plan(kind, t, 0, u, fl)   # not compiled for this layout
                        continue
                    for s in (1, 0, 7):
                        say(f"kind={kind} tile={t} unroll={u} splits={s} flags={fl}")
                        db.set_plan(kind, t, s, u, fl)
                        assert_rows_equal(db.read(req8), want8, f"B=8 kind={kind} T={t} U={u} S={s} F={fl}")
                        assert_rows_equal(db.read(req37), want37, f"B=37 kind={kind} T={t} U={u} S={s} F={fl}")


M4R_SHAPES = [(4, 32), (4, 64), (8, 16), (8, 32), (8, 64), (16, 16), (16, 32)]
_R, _P = pir.PLAN_ROLLING, pir.PLAN_PAIRS
# (waves, requests per wave, flags = prefetch depth << 8 | lookup mode)
_G4 = pir.PLAN_PAIRS | pir.PLAN_PAIR_G4   # paired 4-bucket tables
_G3 = pir.PLAN_PAIRS | pir.PLAN_PAIR_G3   # paired 3-bucket tables
_HW = pir.PLAN_PAIRS | pir.PLAN_HALF_WAVES  # 512-byte entries, a request per half wave
_G6 = pir.PLAN_PAIR_G6                     # with _HW: paired 6-bucket tables
WIDE_SHAPES = [(4, 32, 2 << 8), (8, 16, 2 << 8), (8, 16, 4 << 8), (8, 32, 2 << 8), (8, 32, 3 << 8), (16, 16, 2 << 8),
               (4, 8, _R), (4, 16, _R), (8, 8, _R), (8, 16, _R), (8, 16, _R | 3 << 8), (8, 32, _R), (16, 16, _R),
               (4, 16, _P), (4, 32, _P), (8, 8, _P), (8, 16, _P), (8, 32, _P), (8, 32, _P | 3 << 8),
               (8, 4, _P | 4 << 8), (8, 8, _P | 4 << 8), (8, 16, _P | 4 << 8),
               (8, 4, _G4), (8, 4, _G4 | 4 << 8), (8, 8, _G4), (8, 8, _G4 | 4 << 8), (8, 16, _G4),
               (8, 4, _G3), (8, 4, _G3 | 4 << 8), (8, 8, _G3), (8, 8, _G3 | 4 << 8),
               (8, 64, _HW), (8, 64, _HW | 3 << 8), (8, 32, _HW), (4, 64, _HW), (8, 64, _HW | _G6), (8, 32, _HW | _G6)]
FOUR_RUSSIANS = ([(pir.KERNEL_M4R, (nw, tw, 0)) for nw, tw in M4R_SHAPES] +
                 [(pir.KERNEL_M4R_WIDE, s) for s in WIDE_SHAPES])


@pytest.mark.parametrize("kind", [pir.KERNEL_M4R, pir.KERNEL_M4R_WIDE])
def test_four_russians_every_shape(kind):
    """Four-Russians kernels: every (waves, requests/wave) shape, splits, ragged B."""
    n, d, z = 1024, 4, 1024
    D = synth.uniform_db(1001, n, d * z)
    reqs = {B: synth.bernoulli_requests(2200 + B, B, n) for B in (1, 37, 256, 300, 1100)}
    wants = {B: oracle.pir_read(D, r, threads=8) for B, r in reqs.items()}
    with _db(D, d, z) as db:
        for k, (nw, tw, fl) in FOUR_RUSSIANS:
            if k != kind:
                continue
            for sp in (1, 0, 7):
                db.set_plan(kind, tw, sp, nw, fl)
                for B, r in reqs.items():
                    say(f"kind={kind} nw={nw} tw={tw} flags={fl:#x} splits={sp} B={B}")
                    assert_rows_equal(db.read(r), wants[B], f"kind={kind} nw={nw} tw={tw} fl={fl:#x} S={sp} B={B}")


@pytest.mark.parametrize("n,d,z,B", [(37, 3, 20, 5), (1000, 1, 8, 70), (333, 2, 520, 17), (4097, 4, 1024, 133),
                                     (300, 2, 4096, 66), (2049, 8, 40, 2), (71, 1, 4, 9)])
def test_four_russians_ragged_shapes(n, d, z, B):
    D = synth.uniform_db(n * 11 + d, n, d * z)
    req = synth.bernoulli_requests(n + 3 * B, B, n)
    want = oracle.pir_read(D, req)
    with _db(D, d, z) as db:
        for nw, tw in ((4, 32), (8, 16), (16, 32)):
            db.set_plan(pir.KERNEL_M4R, tw, 0, nw)
            assert_rows_equal(db.read(req), want, f"m4r nw={nw} tw={tw}")
        for nw, tw, fl in WIDE_SHAPES:
            for sp in (0, 3):
                db.set_plan(pir.KERNEL_M4R_WIDE, tw, sp, nw, fl)
                assert_rows_equal(db.read(req), want, f"m4r-wide nw={nw} tw={tw} fl={fl:#x} S={sp}")


def test_four_russians_one_hot_and_densities():
    n, d, z = 1000, 2, 64
    D = synth.uniform_db(35, n, d * z)
    idx = [0, 1, 7, 8, 31, 32, 33, 63, 64, 255, 256, 511, 512, 991, 992, 998, 999]
    onehot = synth.bits_to_rows(np.eye(n, dtype=bool)[idx])
    with _db(D, d, z) as db:
        for kind, nw in ((pir.KERNEL_M4R, 8), (pir.KERNEL_M4R_WIDE, 8)):
            db.set_plan(kind, 16, 0, nw)
            assert_rows_equal(db.read(onehot), D[idx], f"kind={kind} one-hot")
            for p in (0.0, 0.01, 0.99, 1.0):
                req = synth.bernoulli_requests(36, 70, n, p=p)
                assert_rows_equal(db.read(req), oracle.pir_read(D, req), f"kind={kind} p={p}")


@pytest.mark.parametrize("p", [0.0, 0.01, 0.5, 0.99, 1.0])
def test_request_densities(p):
    n, d, z = 777, 4, 256
    D = synth.uniform_db(31, n, d * z)
    req = synth.bernoulli_requests(32, 19, n, p=p)
    want = oracle.pir_read(D, req)
    with _db(D, d, z) as db:
        for kind in (pir.KERNEL_MASK, pir.KERNEL_SKIP):
            db.set_plan(kind, 8, 0, 8)
            assert_rows_equal(db.read(req), want, f"p={p} kind={kind}")


def test_one_hot_rows_pin_bit_order_and_boundaries():
    n, d, z = 1000, 2, 64
    D = synth.uniform_db(33, n, d * z)
    idx = [0, 1, 7, 8, 31, 32, 33, 63, 64, 255, 256, 511, 512, 991, 992, 998, 999]
    req = synth.bits_to_rows(np.eye(n, dtype=bool)[idx])
    with _db(D, d, z) as db:
        for kind in (pir.KERNEL_MASK, pir.KERNEL_SKIP):
            for t in (1, 4, 16):
                db.set_plan(kind, t, 0, 8)
                assert_rows_equal(db.read(req), D[idx], f"one-hot kind={kind} T={t}")


@pytest.mark.parametrize("n,d,z,B", [(37, 3, 20, 5), (1, 1, 16, 3), (1000, 1, 8, 9), (333, 2, 520, 17),
                                     (4097, 4, 1024, 33), (300, 2, 4096, 6), (64, 5, 100, 64), (2049, 8, 40, 2)])
def test_ragged_shapes(n, d, z, B):
    D = synth.uniform_db(n * 7 + d, n, d * z)
    req = synth.bernoulli_requests(n + B, B, n)
    want = oracle.pir_read(D, req)
    with _db(D, d, z) as db:
        assert_rows_equal(db.read(req), want, "auto plan")
        for kind in (pir.KERNEL_MASK, pir.KERNEL_SKIP):
            for t in (1, 8, 32):
                db.set_plan(kind, t, 0, 8)
                assert_rows_equal(db.read(req), want, f"kind={kind} T={t}")
            db.set_plan(kind, 8, 0, 4, pir.PLAN_SHARED_COLUMN)
            assert_rows_equal(db.read(req), want, f"kind={kind} shared column")


@pytest.mark.parametrize("n,d,z", [(65533, 4, 1024), (8190, 1, 16), (4000, 3, 20)])
def test_split_reduction_small_answers_many_splits(n, d, z):
    """The split reduction spreads many splits of a small answer over the
    threads of a workgroup (LDS combine): every words-per-workgroup width it
    picks, odd split counts, plain and masked answers."""
    D = synth.uniform_db(n + 11, n, d * z)
    nwords = (n + 31) // 32
    with _db(D, d, z) as db:
        for B in (1, 3, 6):
            req = synth.bernoulli_requests(n + 17 * B, B, n)
            seeds = synth.uniform_bytes(n + 19 * B, B * 32).reshape(B, 32)
            want = oracle.pir_read(D, req, threads=8)
            want_m = oracle.pir_read_masked(D, req, seeds, threads=8)
            for s in sorted({nwords, nwords - 1, 513, 128, 127, 9, 2}):
                if s < 1 or s > nwords:
                    continue
                say(f"n={n} bucket={d * z} B={B} splits={s}")
                db.set_plan(pir.KERNEL_MASK, 1, s, 16)
                assert_rows_equal(db.read(req), want, f"B={B} splits={s}")
                assert_rows_equal(db.read_masked(req, seeds), want_m, f"masked B={B} splits={s}")
        db.set_plan()


def test_padding_bits_ignored_and_empty_batch():
    n, d, z = 37, 2, 32
    D = synth.uniform_db(41, n, d * z)
    req = synth.bernoulli_requests(42, 4, n, p=0.4)
    noisy = req.copy()
    noisy[:, -1] |= 0xE0
    with _db(D, d, z) as db:
        assert_rows_equal(db.read(noisy), oracle.pir_read(D, req), "padding bits")
        assert db.read(np.zeros((0, 5), np.uint8)).shape == (0, d * z)


def test_three_server_reconstruction_on_gpu():
    """l = 3 shares of e_beta answered by the GPU path reconstruct bucket beta."""
    n, d, z = 2048, 4, 256
    D = synth.uniform_db(43, n, d * z)
    with _db(D, d, z) as db:
        for beta in (0, 5, 1023, 2047):
            q1 = synth.bernoulli_requests(44 + beta, 1, n)
            q2 = synth.bernoulli_requests(99 + beta, 1, n)
            q3 = synth.bits_to_rows(np.eye(n, dtype=bool)[[beta]]) ^ q1 ^ q2
            R = db.read(np.concatenate([q1, q2, q3]))
            assert np.array_equal(R[0] ^ R[1] ^ R[2], D[beta])


def test_epoch_visibility_and_double_buffering():
    n, d, z = 256, 2, 64
    D0 = synth.uniform_db(51, n, d * z)
    req = synth.bernoulli_requests(52, 7, n)
    with pir.PirDB(n, d, z) as db:
        assert not db.read(req).any()                      # empty snapshot is zero
        db.write_range(0, D0)
        assert not db.read(req).any()                      # staged, not published
        db.commit()
        assert_rows_equal(db.read(req), oracle.pir_read(D0, req), "epoch 1")
        D1 = D0.copy()
        for b in (0, 17, 255):
            D1[b] = synth.uniform_db(60 + b, 1, d * z)[0]
            db.write_bucket(b, D1[b])
        D1[17] = synth.uniform_db(99, 1, d * z)[0]         # later write to the same bucket wins
        db.write_bucket(17, D1[17])
        assert_rows_equal(db.read(req), oracle.pir_read(D0, req), "still epoch 1")
        db.commit()
        assert_rows_equal(db.read(req), oracle.pir_read(D1, req), "epoch 2")
        D2 = D1.copy()
        D2[100] = 0
        db.write_bucket(100, D2[100])
        db.commit()                                         # back copy was mirrored
        assert_rows_equal(db.read(req), oracle.pir_read(D2, req), "epoch 3")
        db.commit()                                         # empty epoch keeps the data
        assert_rows_equal(db.read(req), oracle.pir_read(D2, req), "epoch 4")
        assert db.epoch == 4


@pytest.mark.parametrize("m_bits,window", [(1000, 1), (4096, 3), (1 << 17, 100)])
def test_interest_window_across_commits(m_bits, window):
    """Global interest vector after each commit = OR of the last `window`
    epochs' positions; epochs with no positions, with bucket writes (swap
    path) and without (vector-only path); the default configuration too."""
    n, d, z = 64, 2, 32
    rng = np.random.default_rng(m_bits + window)
    D = synth.uniform_db(93, n, d * z)
    with _db(D, d, z) as db:
        if (m_bits, window) != (pir.IV_DEFAULT_BITS, pir.IV_DEFAULT_WINDOW):
            db.interest_config(m_bits, window)
        epochs = [np.zeros(0, np.uint32)]          # commit 0 = the load
        for e in range(1, 12):
            k = 0 if e % 4 == 0 else int(rng.integers(1, 40))
            pos = rng.integers(0, m_bits, size=k, dtype=np.uint32)
            if k:
                db.interest_add(pos)
            if e % 3 == 1:
                db.write_bucket(int(rng.integers(0, n)), synth.uniform_bytes(e, d * z))
            db.commit()
            epochs.append(pos)
            want = oracle.interest_window(m_bits, epochs, len(epochs) - 1, window)
            assert np.array_equal(db.interest_vector(), want), f"epoch {e}"


@pytest.mark.parametrize("d,z", [(1, 512), (2, 520), (1, 496)])
def test_automatic_plan_around_the_half_wave_threshold(d, z):
    """The automatic schedule takes half-wave 6-bucket tables above 256
    requests over rows of 512 bytes or more (rows of 1040 bytes end in a
    ragged 16-byte column), 5-bucket pairs at 256 or over narrower rows;
    every answer bit-exact."""
    n = 2000
    D = synth.uniform_db(3100 + z, n, d * z)
    hw = pir.PLAN_PAIRS | pir.PLAN_HALF_WAVES | pir.PLAN_PAIR_G6
    with _db(D, d, z) as db:
        for B in (256, 257, 700):
            req = synth.bernoulli_requests(3200 + B + z, B, n)
            p = db.get_plan(B)
            want_hw = B > 256 and d * z >= 512
            assert (p.kind == pir.KERNEL_M4R_WIDE and p.flags == hw and p.tile == 64) == want_hw, (B, d * z, p)
            assert_rows_equal(db.read(req), oracle.pir_read(D, req, threads=8), f"auto B={B} row={d * z}")


def test_half_wave_plan_combinations_rejected():
    """Half waves take 5- or 6-bucket paired tables only, and 6-bucket
    tables only with half waves."""
    with pir.PirDB(64, 1, 1024) as db:
        for flags in (pir.PLAN_PAIR_G6 | pir.PLAN_PAIRS, pir.PLAN_HALF_WAVES | pir.PLAN_PAIRS | pir.PLAN_PAIR_G4,
                      pir.PLAN_HALF_WAVES):
            with pytest.raises(pir.PirError):
                db.set_plan(pir.KERNEL_M4R_WIDE, 64, 0, 8, flags)
        db.set_plan(pir.KERNEL_M4R_WIDE, 64, 0, 8, pir.PLAN_PAIRS | pir.PLAN_HALF_WAVES)
        db.set_plan()


def test_write_errors():
    with pir.PirDB(16, 2, 8) as db:
        with pytest.raises(pir.PirError) as e:
            db.write_bucket(16, np.zeros(16, np.uint8))
        assert e.value.code == pir.PIR_ERANGE
        with pytest.raises(pir.PirError):
            db.write_range(10, np.zeros((7, 16), np.uint8))


def test_async_device_api_pitches_and_alignment():
    import torch
    n, d, z = 1000, 4, 256          # ceil(n/8) = 125 bytes: not a multiple of 4 -> restaged
    D = synth.uniform_db(61, n, d * z)
    req = synth.bernoulli_requests(62, 12, n)
    want = oracle.pir_read(D, req)
    with _db(D, d, z) as db:
        dev = torch.device("cuda:0")
        q = torch.from_numpy(req).to(dev)
        out = torch.zeros((12, d * z), dtype=torch.uint8, device=dev)
        db.read_async(q, out)
        torch.cuda.synchronize()
        assert_rows_equal(out.cpu().numpy(), want, "contiguous")
        # padded request rows and padded, offset response rows
        qp = torch.zeros((12, 160), dtype=torch.uint8, device=dev)
        qp[:, :125] = q
        big = torch.zeros((12, d * z + 48), dtype=torch.uint8, device=dev)
        view = big[:, 16:16 + d * z]
        db.read_async(qp, view)
        torch.cuda.synchronize()
        assert_rows_equal(view.cpu().numpy(), want, "pitched")
        assert not big[:, :16].any() and not big[:, 16 + d * z:].any()


def test_stream_of_uneven_batches_matches_single_reads():
    import torch
    n, d, z = 4096, 4, 1024
    D = synth.uniform_db(71, n, d * z)
    sizes = synth.batch_sizes(72, 23, 1, 300)
    sizes[3] = 0
    total = int(sizes.sum())
    pool = synth.bernoulli_requests(73, 512, n)
    rng = np.random.default_rng(74)
    first = np.array([rng.integers(0, 512 - s + 1) for s in sizes], dtype=np.uint64)
    dev = torch.device("cuda:0")
    with _db(D, d, z) as db:
        q = torch.from_numpy(pool).to(dev)
        out = torch.zeros((total, d * z), dtype=torch.uint8, device=dev)
        for rep in range(3):                       # first call captures, then graph replays
            out.zero_()
            db.read_stream_async(q, sizes, out, req_first=first)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            row = 0
            for k, s in enumerate(sizes):
                s = int(s)
                want = oracle.pir_read(D, pool[int(first[k]):int(first[k]) + s], threads=8)
                assert_rows_equal(got[row:row + s], want, f"rep {rep} batch {k} (B={s})")
                row += s


def test_stream_fuses_batches_with_scattered_rows():
    """Batches fused into 1024-row launch groups (some batches split across
    two groups), request rows gathered from anywhere in the pool and responses
    scattered to permuted rows, replayed from the graph; then the same stream
    contiguous (no gather/scatter)."""
    import torch
    n, d, z = 2048, 4, 1024
    D = synth.uniform_db(75, n, d * z)
    sizes = synth.batch_sizes(76, 40, 1, 120)          # ~2400 rows: batches straddle 1024-row groups
    sizes[[0, 7, 39]] = 0
    total = int(sizes.sum())
    pool = synth.bernoulli_requests(77, 300, n)
    rng = np.random.default_rng(78)
    first = np.array([rng.integers(0, 300 - s + 1) for s in sizes], dtype=np.uint64)
    # response blocks in a permuted order with gaps between them
    order = rng.permutation(len(sizes))
    resp_first = np.zeros(len(sizes), dtype=np.uint64)
    row = 5
    for k in order:
        resp_first[k] = row
        row += int(sizes[k]) + 3
    dev = torch.device("cuda:0")
    want_rows = {}
    with _db(D, d, z) as db:
        q = torch.from_numpy(pool).to(dev)
        out = torch.zeros((row + 4, d * z), dtype=torch.uint8, device=dev)
        for rep in range(2):
            out.zero_()
            db.read_stream_async(q, sizes, out, req_first=first, resp_first=resp_first)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            touched = np.zeros(row + 4, dtype=bool)
            for k, s in enumerate(sizes):
                s = int(s)
                if s == 0:
                    continue
                if k not in want_rows:
                    want_rows[k] = oracle.pir_read(D, pool[int(first[k]):int(first[k]) + s], threads=8)
                r0 = int(resp_first[k])
                assert_rows_equal(got[r0:r0 + s], want_rows[k], f"rep {rep} batch {k} (B={s})")
                touched[r0:r0 + s] = True
            assert not got[~touched].any(), "rows outside the response blocks were written"
        # contiguous layout: no gather, no scatter
        out2 = torch.zeros((total, d * z), dtype=torch.uint8, device=dev)
        cat = np.concatenate([pool[int(first[k]):int(first[k]) + int(s)] for k, s in enumerate(sizes)])
        q2 = torch.from_numpy(cat).to(dev)
        db.read_stream_async(q2, sizes, out2)
        torch.cuda.synchronize()
        assert_rows_equal(out2.cpu().numpy(), oracle.pir_read(D, cat, threads=8), "contiguous stream")


def test_tuner_picks_a_correct_plan(tmp_path):
    n, d, z = 2048, 4, 1024
    D = synth.uniform_db(81, n, d * z)
    req = synth.bernoulli_requests(82, 40, n)
    want = oracle.pir_read(D, req)
    with _db(D, d, z) as db:
        plan, us = db.tune(40, iters=2)
        say(f"tuned {plan} {us:.1f} us")
        assert us > 0
        assert_rows_equal(db.read(req), want, "tuned plan")
        path = str(tmp_path / "tune.json")
        assert pir.lib().pir_tune_save(path.encode()) == 0
        assert pir.lib().pir_tune_load(path.encode()) == 0


def test_kernel_timing_records_each_read():
    import torch
    n, d, z = 4096, 4, 1024
    D = synth.uniform_db(91, n, d * z)
    req = synth.bernoulli_requests(92, 64, n)
    want = oracle.pir_read(D, req)
    with _db(D, d, z) as db:
        dev = torch.device("cuda:0")
        q = torch.from_numpy(req).to(dev)
        out = torch.zeros((64, d * z), dtype=torch.uint8, device=dev)
        db.read_async(q, out)                      # not recorded: timing is off
        db.profile_enable(True)
        for _ in range(3):
            db.read_async(q, out)
        assert_rows_equal(db.read(req), want, "sync read while timing")
        ms = db.profile_collect()
        assert ms.size == 4 and np.all(ms > 0) and np.all(ms < 1000)
        assert db.profile_collect().size == 0      # collect clears
        db.profile_enable(False)
        db.read_async(q, out)
        assert db.profile_collect().size == 0
        db.profile_enable(True, every=3)           # reads 0, 3 and 6 of seven
        for _ in range(7):
            db.read_async(q, out)
        ms = db.profile_collect()
        assert ms.size == 3 and np.all(ms > 0)
        db.profile_enable(False)
        torch.cuda.synchronize()
        assert_rows_equal(out.cpu().numpy(), want, "async read")


@pytest.mark.parametrize("forced", [None, (pir.KERNEL_M4R_WIDE, 8, 1, 8, pir.PLAN_PAIRS),
                                    (pir.KERNEL_SKIP, 16, 1, 4, 0)])
def test_async_reads_on_two_streams_see_their_epoch(forced):
    """Reads queued on two streams between commits, with no host wait, each
    answer from the snapshot published before they were issued: the commits'
    mirror copies wait for the reads still using the other copy (the read's
    last kernel marks its end), and the interest fetch beside each read gets
    the same epoch's vector. Automatic plan (split reduction last) and plans
    without splits (main kernel last)."""
    import torch
    n, d, z, B, m, window, epochs = 8192, 2, 1024, 64, 1 << 12, 3, 6
    rng = np.random.default_rng(95)
    D = synth.uniform_db(93, n, d * z)
    req = synth.bernoulli_requests(94, B, n)
    dev = torch.device("cuda:0")
    streams = [torch.cuda.current_stream(), torch.cuda.Stream(device=dev)]
    snaps, vecs = [], []
    with pir.PirDB(n, d, z) as db:
        db.interest_config(m, window)
        db.write_range(0, D)
        db.commit()
        if forced:
            db.set_plan(*forced)
        q = torch.from_numpy(req).to(dev)
        outs = [torch.zeros((B, d * z), dtype=torch.uint8, device=dev) for _ in range(epochs)]
        ivs = [torch.zeros((m // 8,), dtype=torch.uint8, device=dev) for _ in range(epochs)]
        pos_by_epoch = [np.zeros(0, np.uint32)]    # commit 0 = the load
        for e in range(epochs):
            for b in rng.choice(n, size=40, replace=False):
                D[b] = rng.integers(0, 256, d * z, dtype=np.uint8)
                db.write_bucket(int(b), D[b])
            pos = rng.integers(0, m, 30, dtype=np.uint32)
            db.interest_add(pos)
            db.commit()
            pos_by_epoch.append(pos)
            snaps.append(D.copy())
            vecs.append(oracle.interest_window(m, pos_by_epoch, len(pos_by_epoch) - 1, window))
            s = streams[e % 2]
            db.read_async(q, outs[e], stream=s)
            rc = pir.lib().pir_interest_vector_async(db.h, ivs[e].data_ptr(), ivs[e].numel(), int(s.cuda_stream))
            assert rc == 0
        torch.cuda.synchronize()
        for e in range(epochs):
            assert_rows_equal(outs[e].cpu().numpy(), oracle.pir_read(snaps[e], req), f"epoch {e + 1}")
            assert np.array_equal(ivs[e].cpu().numpy(), vecs[e]), f"interest vector of epoch {e + 1}"
