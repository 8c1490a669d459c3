"""C-ABI library: loads, exports every declared symbol, host logic on the CPU.

No call here touches a GPU: the library's host-only cuckoo table (detached
from any database) is checked against the oracle's independent table.
"""
import numpy as np
import pytest

import oracle
import paper_2001_08250_amd as pir
import synth


def test_library_exports_every_header_symbol():
    L = pir.lib()
    declared = pir.header_symbols()
    assert len(declared) >= 25
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(pir.SIGNATURES) == declared


def test_strerror_and_version():
    assert pir.strerror(pir.PIR_EFULL).startswith("cuckoo insertion failed")
    assert pir.strerror(12345) == "unknown error"
    assert "gfx950" in pir.version()


def test_validation_without_device():
    import ctypes
    L = pir.lib()
    h = ctypes.c_void_p()
    assert L.pir_db_create(0, 4, 16, ctypes.byref(h)) == pir.PIR_EINVAL
    assert L.pir_db_create(16, 0, 16, ctypes.byref(h)) == pir.PIR_EINVAL
    assert L.pir_db_create(16, 4, 0, ctypes.byref(h)) == pir.PIR_EINVAL
    assert L.pir_db_create(16, 4, 16, None) == pir.PIR_EINVAL
    assert L.pir_read_batch(None, None, 0, None) == pir.PIR_EINVAL
    assert L.pir_epoch_commit(None, None) == pir.PIR_EINVAL
    assert L.pir_cuckoo_create(None, 0, 0, 500, ctypes.byref(h)) == pir.PIR_EINVAL
    assert L.pir_read_batch_masked(None, None, 0, None, None) == pir.PIR_EINVAL
    assert L.pir_read_batch_masked_async(None, None, 0, 0, None, None, 0, None) == pir.PIR_EINVAL
    two = (ctypes.c_void_p * 2)(16, 32)
    assert L.pir_xor_combine_async(None, 16, two, 2, 16, 0, 16, None) == pir.PIR_OK   # B = 0: no-op
    assert L.pir_xor_combine_async(None, 16, two, 2, 16, 1, 16, None) == pir.PIR_EINVAL
    assert L.pir_xor_combine_async(16, 16, two, 0, 16, 1, 16, None) == pir.PIR_EINVAL  # l = 0
    many = (ctypes.c_void_p * 17)(*([16] * 17))
    assert L.pir_xor_combine_async(16, 16, many, 17, 16, 1, 16, None) == pir.PIR_EINVAL  # l > 16
    assert L.pir_xor_combine_async(16, 16, two, 2, 16, 1, 24, None) == pir.PIR_EINVAL  # row % 16
    assert L.pir_xor_combine_async(16, 8, two, 2, 16, 1, 16, None) == pir.PIR_EINVAL   # pitch < row
    assert L.pir_profile_enable(None, 1) == pir.PIR_EINVAL
    assert L.pir_profile_collect(None, None, 0, None) == pir.PIR_EINVAL
    assert L.pir_preprocess(None, 1, 0) == pir.PIR_EINVAL
    buf = (ctypes.c_uint8 * 256)()
    leaves = ctypes.c_uint32(0)
    for bad in (0, 3):
        assert L.pir_preprocess_tables(bad, ctypes.byref(leaves), buf, buf, buf, buf, buf, buf) == pir.PIR_EINVAL
    assert L.pir_preprocess_tables(1, None, buf, buf, buf, buf, buf, buf) == pir.PIR_EINVAL
    L.pir_db_destroy(None)  # NULL-safe


def _lib_vs_oracle(n, d, z, count, seed, capacity=0, max_kicks=500):
    ids, b1, b2, pay = synth.write_ops(seed, count, n, z)
    ref = oracle.Cuckoo(n, d, z, capacity=capacity, seed=seed, max_kicks=max_kicks)
    st_ref, dr_ref = ref.insert_many(ids, b1, b2, pay)
    mine = pir.Cuckoo(None, capacity=capacity, seed=seed, max_kicks=max_kicks, shape=(n, d, z))
    st, dr = mine.insert_many(ids, b1, b2, pay)
    assert np.array_equal(st, st_ref)
    assert np.array_equal(dr, dr_ref)
    assert np.array_equal(mine.table(), ref.table())
    ids_m, occ_m = mine.slots()
    ids_r, occ_r = ref.slots()
    assert np.array_equal(occ_m, occ_r) and np.array_equal(ids_m, ids_r)
    assert mine.live() == ref.live()
    return st


@pytest.mark.parametrize("n,d,z,load,seed", [(512, 4, 16, 0.90, 1), (256, 2, 8, 0.80, 2), (97, 3, 12, 0.93, 3),
                                             (1024, 4, 32, 0.97, 4)])
def test_library_cuckoo_matches_oracle(n, d, z, load, seed):
    _lib_vs_oracle(n, d, z, int(load * n * d), seed)


def test_library_cuckoo_matches_oracle_with_gc_and_failures():
    st = _lib_vs_oracle(64, 2, 8, 400, seed=5, capacity=80)
    assert (st == 0).all()
    st = _lib_vs_oracle(16, 2, 8, 60, seed=6, max_kicks=20)
    assert (st == pir.PIR_EFULL).any()


def test_library_cuckoo_golden_examples(golden_dir):
    import json
    import os
    g = json.load(open(os.path.join(golden_dir, "cuckoo_examples.json")))
    for ex in g["examples"]:
        z = ex["z"]
        c = pir.Cuckoo(None, capacity=ex["capacity"], seed=ex["seed"], max_kicks=ex["max_kicks"],
                       shape=(ex["n"], ex["d"], z))
        names = {}
        status = []
        for i, (name, b1, b2) in enumerate(ex["writes"]):
            names[i + 1] = name
            p = np.zeros(z, np.uint8)
            p[:len(name)] = np.frombuffer(name.encode(), np.uint8)
            rc, _ = c.insert(i + 1, b1, b2, p)
            status.append(rc)
        assert status == ex["status"], ex["name"]
        ids, occ = c.slots()
        for b in range(ex["n"]):
            for s in range(ex["d"]):
                want = ex["table"][b][s]
                assert (names[int(ids[b, s])] if occ[b, s] else None) == want, ex["name"]


def test_detached_cuckoo_cannot_stage():
    c = pir.Cuckoo(None, shape=(8, 2, 8))
    with pytest.raises(pir.PirError):
        c.stage()


def test_cuckoo_rejects_out_of_range_bucket():
    c = pir.Cuckoo(None, shape=(8, 2, 8))
    rc, _ = c.insert(1, 8, 0, np.zeros(8, np.uint8))
    assert rc == pir.PIR_ERANGE
