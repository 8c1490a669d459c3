"""GetUpdates payload sizes at the paper's store sizes (section "Evaluation",
cost of operations, GetUpdates row: 0.21 / 1.40 / 14.00 KB at 10K / 100K / 1M
messages, false-positive rate 0.02, TTL of 100 write intervals).

The global vector over the TTL window holds every stored message; a
GetUpdates sends one compressed delta (one write interval's messages). The
oracle encodes both; the checks are properties the sizing must have: the
window's false-positive rate is the paper's 0.02, the delta grows linearly
with the store, and it lands near the paper's row (the compressed format is
not the paper's, so not byte for byte)."""
import numpy as np
import pytest

import oracle
import synth
from synth import configs


def _payloads(n_msg: int, seed: int = 9000):
    sh = configs.getupdates_shape(n_msg)
    m, per, win = sh["m_bits"], sh["per_interval"], sh["window"]
    epochs = [synth.interest_positions(seed + i, per, sh["k"], m).reshape(-1) for i in range(win)]
    glob = oracle.interest_window(m, epochs, win - 1, win)
    delta = oracle.interest_window(m, epochs[-1:], 0, 1)
    return m, glob, oracle.iv_encode(glob, m), oracle.iv_encode(delta, m)


@pytest.mark.parametrize("n_msg", configs.GETUPDATES_MESSAGES)
def test_window_false_positive_rate(n_msg):
    m, glob, _, _ = _payloads(n_msg)
    fill = np.unpackbits(glob, bitorder="little")[:m].mean()   # one position per message
    assert abs(fill - configs.GETUPDATES_FP) < 0.002, fill


def test_delta_sizes_against_the_paper_row():
    sizes = {}
    for n_msg in configs.GETUPDATES_MESSAGES:
        m, _, g, d = _payloads(n_msg)
        sizes[n_msg] = len(d)
        paper = configs.GETUPDATES_PAPER_KB[n_msg] * 1000
        print(f"n={n_msg}: delta {len(d)} B (paper {paper:.0f} B), global {len(g)} B of {m // 8} raw")
        assert 0.75 * paper < len(d) < 1.5 * paper
    # linear in the store beyond the header: 10x the messages, about 10x the bytes
    assert 9.0 < sizes[1_000_000] / sizes[100_000] < 11.0
