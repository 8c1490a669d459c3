"""Shared helpers for the GPU tests (no PIR arithmetic here)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_rows_equal(got: np.ndarray, want: np.ndarray, what: str = ""):
    """Bit-exact comparison; on failure name the first differing row and byte."""
    assert got.shape == want.shape, f"{what}: shape {got.shape} != {want.shape}"
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, c = bad[0]
        raise AssertionError(f"{what}: {len(bad)} bytes differ; first at row {r} byte {c}: "
                             f"got {got[r, c]:#04x} want {want[r, c]:#04x}")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
