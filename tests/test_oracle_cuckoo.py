"""Pins of the reference cuckoo table and interest-vector oracle."""
import json
import os

import numpy as np
import pytest

import oracle
import synth


def test_splitmix64_published_vector(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64_seed1234567.json")))
    out = oracle.splitmix64(g["seed"], len(g["outputs"]))
    assert [int(x) for x in out] == [int(x) for x in g["outputs"]]


def _payload(name, z):
    p = np.zeros(z, dtype=np.uint8)
    p[:len(name)] = np.frombuffer(name.encode(), dtype=np.uint8)
    p[-1] = 0xA5
    return p


@pytest.mark.parametrize("which", ["gc_fifo_d2", "eviction_cycle_d1", "beta2_then_random_victim_d2",
                                   "three_evictions_d4", "three_evictions_d3"])
def test_hand_worked_examples(golden_dir, which):
    g = json.load(open(os.path.join(golden_dir, "cuckoo_examples.json")))
    ex = next(e for e in g["examples"] if e["name"] == which)
    z = ex["z"]
    c = oracle.Cuckoo(ex["n"], ex["d"], z, capacity=ex["capacity"], seed=ex["seed"], max_kicks=ex["max_kicks"])
    names = {}
    status = []
    dropped = []
    for i, (name, b1, b2) in enumerate(ex["writes"]):
        names[i + 1] = name
        rc, drop = c.insert(i + 1, b1, b2, _payload(name, z))
        status.append(rc)
        if rc:
            dropped.append(names[drop])
    assert status == ex["status"]
    if "dropped" in ex:
        assert dropped == [ex["dropped"]]
    ids, occ = c.slots()
    table = c.table()
    for b in range(ex["n"]):
        for s in range(ex["d"]):
            want = ex["table"][b][s]
            row = table[b, s * z:(s + 1) * z]
            if want is None:
                assert not occ[b, s] and not row.any()
            else:
                assert occ[b, s] and names[int(ids[b, s])] == want
                assert np.array_equal(row, _payload(want, z))


def _fill(n, d, z, count, seed, capacity=0, max_kicks=500):
    ids, b1, b2, pay = synth.write_ops(seed, count, n, z)
    c = oracle.Cuckoo(n, d, z, capacity=capacity, seed=seed, max_kicks=max_kicks)
    status, dropped = c.insert_many(ids, b1, b2, pay)
    return c, (ids, b1, b2, pay), status, dropped


def test_invariants_after_random_fill():
    n, d, z = 512, 4, 16
    c, (ids, b1, b2, pay), status, dropped = _fill(n, d, z, int(0.9 * n * d), seed=7)
    sids, occ = c.slots()
    table = c.table().reshape(n, d, z)
    pos = {int(i): k for k, i in enumerate(ids)}
    live_ids = sids[occ]
    assert len(set(live_ids.tolist())) == live_ids.size          # no duplicates
    assert occ.sum() == c.live()
    lost = set(int(x) for x, s in zip(dropped, status) if s != 0)
    assert occ.sum() == len(ids) - len(lost)
    for b in range(n):
        for s in range(d):
            if not occ[b, s]:
                assert not table[b, s].any()
                continue
            k = pos[int(sids[b, s])]
            assert b in (int(b1[k]), int(b2[k]))                  # one of its two buckets
            assert np.array_equal(table[b, s], pay[k])            # payload moved intact


def test_d4_reaches_95_percent_load():
    """Section 'Evaluation': depth 4 supports a 95% load factor."""
    n, d, z = 4096, 4, 8
    ok = 0
    for seed in range(5):
        _, _, status, _ = _fill(n, d, z, int(0.95 * n * d), seed=100 + seed)
        ok += int((status == 0).all())
    assert ok >= 4


def test_overfull_table_reports_failure():
    n, d, z = 8, 2, 8
    _, _, status, dropped = _fill(n, d, z, n * d + 4, seed=3, max_kicks=50)
    assert (status == -5).sum() >= 4
    assert all(dropped[status == -5] != 0)


def test_fifo_garbage_collection_keeps_latest():
    n, d, z, cap = 256, 4, 8, 500
    c, (ids, *_), status, _ = _fill(n, d, z, 3 * cap, seed=9, capacity=cap)
    assert (status == 0).all()
    sids, occ = c.slots()
    assert set(sids[occ].tolist()) == set(int(x) for x in ids[-cap:])


def test_deterministic_under_seed():
    a, *_ = _fill(64, 4, 8, 240, seed=5)
    b, *_ = _fill(64, 4, 8, 240, seed=5)
    assert np.array_equal(a.table(), b.table())


def test_bucket_out_of_range():
    c = oracle.Cuckoo(4, 2, 8)
    rc, _ = c.insert(1, 4, 0, np.zeros(8, np.uint8))
    assert rc == -2


def test_interest_window_brute_force():
    m = 1000
    rng = np.random.default_rng(0)
    epochs = [rng.integers(0, m, size=rng.integers(0, 30)).astype(np.uint32) for _ in range(12)]
    for last in range(12):
        for window in (1, 3, 8, 20):
            got = oracle.interest_window(m, epochs, last, window)
            bits = set()
            for e in range(max(0, last - window + 1), last + 1):
                bits.update(int(p) for p in epochs[e])
            want = np.zeros(m, dtype=bool)
            want[list(bits)] = True
            assert np.array_equal(np.unpackbits(got, bitorder="little")[:m].astype(bool), want)


def test_interest_window_superset_and_idempotent():
    m = 256
    e = [np.array([1, 5, 200], np.uint32), np.array([5, 9], np.uint32)]
    one = oracle.interest_window(m, e[:1], 0, 4)
    two = oracle.interest_window(m, e, 1, 4)
    assert ((one & two) == one).all()                              # superset
    dup = oracle.interest_window(m, [np.concatenate([e[0], e[0]]), e[1]], 1, 4)
    assert np.array_equal(dup, two)                               # idempotent


def test_interest_rejects_out_of_range():
    with pytest.raises(ValueError):
        oracle.interest_window(64, [np.array([64], np.uint32)], 0, 1)
