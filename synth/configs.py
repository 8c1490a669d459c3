"""Workload shapes and seeds (synthetic stand-ins for the paper's workloads).

Sizes follow the paper's evaluation: 1 KiB messages and bucket depth d = 4
(section "Evaluation", cost of operations); n here counts buckets (the paper's
b). Each entry fixes its seeds so every run consumes the same bytes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

KiB = 1024
MiB = 1024 * KiB
GiB = 1024 * MiB


@dataclass(frozen=True)
class Workload:
    name: str
    n: int              # buckets
    d: int              # slots per bucket
    z: int              # bytes per slot (message size)
    B: int = 0          # request vectors per batch (fixed-batch workloads)
    db_seed: int = 0
    req_seed: int = 0
    fill: str = "uniform"   # "uniform" bytes or "cuckoo" fill with write_ops
    cuckoo_items: int = 0
    cuckoo_seed: int = 0    # seed of the write ops and of s_cuckoo
    batches: int = 0        # uneven-batch stream length
    batch_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def bucket_bytes(self) -> int:
        return self.d * self.z

    @property
    def db_bytes(self) -> int:
        return self.n * self.d * self.z


C1 = Workload("xorpir-n1024-d4-z1k-B8", n=1024, d=4, z=1 * KiB, B=8, db_seed=1001, req_seed=2001)
C2 = Workload("xorpir-n65536-d4-z1k-B256-cuckoo200k", n=65536, d=4, z=1 * KiB, B=256, req_seed=2002,
              fill="cuckoo", cuckoo_items=200_000, cuckoo_seed=3002)
C3 = Workload("xorpir-n1M-d4-z1k-uneven500", n=1 << 20, d=4, z=1 * KiB, db_seed=1003, req_seed=2003,
              batches=500, batch_seed=5003)
C3B64 = Workload("xorpir-n1M-d4-z1k-B64", n=1 << 20, d=4, z=1 * KiB, B=64, db_seed=1003, req_seed=2003)
C4A = Workload("xorpir-n4M-d4-z1k-B2048", n=1 << 22, d=4, z=1 * KiB, B=2048, db_seed=1004, req_seed=2004)
C4B = Workload("xorpir-n1M-d2-z4k-B2048", n=1 << 20, d=2, z=4 * KiB, B=2048, db_seed=1014, req_seed=2014)
C5 = Workload("serve-n1M-d4-z1k", n=1 << 20, d=4, z=1 * KiB, fill="cuckoo", cuckoo_items=3_145_728,
              cuckoo_seed=3005, req_seed=2005,
              extra={"arrival_seed": 4005, "rates": (5_000, 20_000, 50_000), "write_frac": 0.1,
                     "interest_bits": 1 << 20, "interest_k": 6, "window": 100, "epoch_s": 1.0})

ALL = {w.name: w for w in (C1, C2, C3, C3B64, C4A, C4B, C5)}
BY_KEY = {"c1": C1, "c2": C2, "c3": C3, "c4a": C4A, "c4b": C4B, "c5": C5}

# Blocked cuckoo parameters shared by every cuckoo-filled workload.
CUCKOO_MAX_KICKS = 500


# GetUpdates sizing (section "Evaluation", cost of operations: the interest
# vector grows linearly with the number n of stored messages so as to keep a
# false-positive rate of 0.02 over a TTL of 100 write intervals). Reading: a
# GetUpdates transfers one compressed delta, the messages of one write
# interval (n / TTL of them); each message sets one position (one hash, the
# compressed-Bloom-filter choice that minimises what is sent) in a vector of
# m = ceil(n / ln(1 / (1 - 0.02))) bits, so that the global vector over the
# TTL window of deltas (all n messages) has false-positive rate 0.02.
GETUPDATES_FP = 0.02
GETUPDATES_TTL = 100
GETUPDATES_MESSAGES = (10_000, 100_000, 1_000_000)
# the paper's GetUpdates row (KB) at those message counts
GETUPDATES_PAPER_KB = {10_000: 0.21, 100_000: 1.40, 1_000_000: 14.00}


def getupdates_shape(n_messages: int, fp: float = GETUPDATES_FP, ttl: int = GETUPDATES_TTL) -> dict:
    import math
    return {"m_bits": math.ceil(n_messages / -math.log1p(-fp)), "k": 1,
            "per_interval": n_messages // ttl, "window": ttl}
