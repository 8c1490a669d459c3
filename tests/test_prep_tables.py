"""CPU check of the library's Strassen leaf tables (no GPU).

Applied to random bit matrices A and byte matrices D, the leaf products that
the tables describe, XORed into the answer blocks they list, must give
exactly the GF(2) product A D computed directly (bucket rows XORed under the
request bits). This pins the block algebra of the preprocessed reads
independently of any kernel.
"""
import numpy as np
import pytest

import paper_2001_08250_amd as pir


def gf2_product(A: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Row r = XOR of the rows j of D with A[r, j] = 1."""
    out = np.zeros((A.shape[0], D.shape[1]), dtype=np.uint8)
    for r in range(A.shape[0]):
        sel = np.nonzero(A[r])[0]
        if sel.size:
            out[r] = np.bitwise_xor.reduce(D[sel], axis=0)
    return out


def block(M: np.ndarray, g: int, r: int, c: int) -> np.ndarray:
    h, w = M.shape[0] // g, M.shape[1] // g
    return M[r * h:(r + 1) * h, c * w:(c + 1) * w]


@pytest.mark.parametrize("levels", [1, 2])
def test_leaf_tables_reproduce_the_product(levels):
    t = pir.preprocess_tables(levels)
    g = t["grid"]
    assert g == 2 ** levels and len(t["a"]) == 7 ** levels == len(t["d"])
    assert all(len(x) <= 2 ** levels for x in t["a"] + t["d"])
    rng = np.random.default_rng(levels)
    for trial in range(3):
        A = rng.integers(0, 2, (6 * g, 10 * g), dtype=np.uint8)
        D = rng.integers(0, 256, (10 * g, 3 * g), dtype=np.uint8)
        want = gf2_product(A, D)
        got = np.zeros_like(want)
        prods = []
        for la, ld in zip(t["a"], t["d"]):
            Al = np.bitwise_xor.reduce([block(A, g, r, c) for r, c in la], axis=0)
            Dl = np.bitwise_xor.reduce([block(D, g, r, c) for r, c in ld], axis=0)
            prods.append(gf2_product(Al, Dl))
        h, w = want.shape[0] // g, want.shape[1] // g
        for b, leaves in enumerate(t["out"]):
            r, c = divmod(b, g)
            for l in leaves:
                got[r * h:(r + 1) * h, c * w:(c + 1) * w] ^= prods[l]
        assert np.array_equal(got, want), f"levels={levels} trial={trial}"


def test_leaf_tables_reject_other_levels():
    for levels in (0, 3):
        with pytest.raises(pir.PirError):
            pir.preprocess_tables(levels)
