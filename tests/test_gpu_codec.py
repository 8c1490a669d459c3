"""Compressed interest vectors on the GPU: the device encoder's streams equal
the oracle's byte for byte (global vector and every delta in the window)."""
import numpy as np
import pytest

import oracle
import paper_2001_08250_amd as pir
import synth
from helpers import gpu_available, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _bits(m, positions):
    v = np.zeros((m + 7) // 8, dtype=np.uint8)
    for p in np.asarray(positions, dtype=np.int64):
        v[p >> 3] |= np.uint8(1 << (p & 7))
    return v


@pytest.mark.parametrize("m,window,per_epoch", [(1000, 3, 40), (4099, 5, 3), (1 << 17, 100, 600),
                                                (64, 2, 64), (1 << 20, 4, 20000)])
def test_encoded_vector_and_deltas(m, window, per_epoch):
    n, d, z = 64, 2, 32
    D = synth.uniform_db(7, n, d * z)
    rng = np.random.default_rng(m + window)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        db.interest_config(m, window)
        first = pir.lib().pir_epoch(db.h)
        epochs = {}
        for i in range(window + 3):
            k = 0 if i % 4 == 2 else int(rng.integers(1, per_epoch + 1))
            pos = rng.integers(0, m, size=k, dtype=np.uint32)
            if i == 1:
                pos = np.concatenate([pos, np.array([0, m - 1], dtype=np.uint32)])
            if k or i == 1:
                db.interest_add(pos)
            db.commit()
            e = pir.lib().pir_epoch(db.h)
            epochs[e] = pos
            g = db.interest_encoded()
            assert g == oracle.iv_encode(db.interest_vector(), m), f"global after epoch {e}"
            window_pos = [epochs[x] for x in sorted(epochs) if x > e - window]
            want_global = _bits(m, np.concatenate(window_pos) if window_pos else [])
            assert g == oracle.iv_encode(want_global, m)
        last = pir.lib().pir_epoch(db.h)
        for e in range(max(first + 1, last - window + 1), last + 1):
            say(f"m={m} delta of epoch {e}")
            assert db.interest_encoded(e) == oracle.iv_encode(_bits(m, epochs[e]), m), f"delta {e}"
        with pytest.raises(pir.PirError):
            db.interest_encoded(last - window)
        with pytest.raises(pir.PirError):
            db.interest_encoded(last + 1)


def test_dense_and_full_vectors():
    n, d, z = 16, 1, 16
    D = synth.uniform_db(9, n, d * z)
    with pir.PirDB(n, d, z) as db:
        db.load(D)
        for m in (33, 1000):
            db.interest_config(m, 1)
            db.interest_add(np.arange(m, dtype=np.uint32))
            db.commit()
            s = db.interest_encoded()
            assert s == oracle.iv_encode(np.full((m + 7) // 8, 0xFF, dtype=np.uint8), m)
            m2, v = oracle.iv_decode(s)
            assert m2 == m and np.unpackbits(v, bitorder="little")[:m].all()


@pytest.mark.parametrize("n_msg", [10_000, 100_000, 1_000_000])
def test_getupdates_payloads_at_the_papers_store_sizes(n_msg):
    """The paper's GetUpdates sizing (false-positive rate 0.02 over a TTL of
    100 write intervals, one position per message): after a full window of
    write intervals the device encodes the global vector and the last delta
    byte for byte as the oracle does."""
    from synth import configs
    sh = configs.getupdates_shape(n_msg)
    m, per, win = sh["m_bits"], sh["per_interval"], sh["window"]
    epochs = [synth.interest_positions(9000 + i, per, sh["k"], m).reshape(-1) for i in range(win)]
    with pir.PirDB(64, 2, 32) as db:
        db.interest_config(m, win)
        for pos in epochs:
            db.interest_add(pos)
            db.commit()
        last = pir.lib().pir_epoch(db.h)
        glob = oracle.interest_window(m, epochs, win - 1, win)
        want_g = oracle.iv_encode(glob, m)
        want_d = oracle.iv_encode(oracle.interest_window(m, epochs[-1:], 0, 1), m)
        got_g, got_d = db.interest_encoded(), db.interest_encoded(last)
        say(f"n={n_msg}: m={m} delta {len(got_d)} B, global {len(got_g)} B")
        assert got_g == want_g
        assert got_d == want_d
