"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle's C sources
(a dropped term, a wrong index, a wrong bit, a swapped operand), builds it
with gcc into a temporary directory and runs the oracle pin tests against
that build. Every case must make at least one pin fail: a mistake that no
pin catches would mean that part of the oracle is not pinned.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = ["tests/test_oracle_pir.py", "tests/test_oracle_cuckoo.py", "tests/test_oracle_mask.py",
        "tests/test_oracle_codec.py"]

# (name, source file, exact text, replacement)
MUTATIONS = [
    ("bit_order_msb_first", "pir_oracle.c", "(row[j >> 3] >> (j & 7)) & 1", "(row[j >> 3] >> (7 - (j & 7))) & 1"),
    ("last_bucket_dropped", "pir_oracle.c", "for (uint64_t j = 0; j < n; ++j) {",
     "for (uint64_t j = 0; j + 1 < n; ++j) {"),
    ("last_byte_skipped", "pir_oracle.c", "for (uint64_t k = 0; k < bucket_bytes; ++k)",
     "for (uint64_t k = 0; k + 1 < bucket_bytes; ++k)"),
    ("victim_high_word", "cuckoo_oracle.c", "uint64_t v = splitmix64_next(&c->rng) % c->d;",
     "uint64_t v = (splitmix64_next(&c->rng) >> 32) % c->d;"),
    ("victim_shifted", "cuckoo_oracle.c", "uint64_t v = splitmix64_next(&c->rng) % c->d;",
     "uint64_t v = (splitmix64_next(&c->rng) >> 1) % c->d;"),
    ("victim_masked", "cuckoo_oracle.c", "uint64_t v = splitmix64_next(&c->rng) % c->d;",
     "uint64_t v = splitmix64_next(&c->rng) & (c->d - 1);"),
    ("beta_e_inverted", "cuckoo_oracle.c", "(splitmix64_next(&c->rng) & 1) ? b2 : b1",
     "(splitmix64_next(&c->rng) & 1) ? b1 : b2"),
    ("beta2_probe_skipped", "cuckoo_oracle.c", "    s = free_slot(c, b2);\n    if (s >= 0) {",
     "    s = -1;\n    if (s >= 0) {"),
    ("gc_one_late", "cuckoo_oracle.c", "if (c->capacity && c->live >= c->capacity)",
     "if (c->capacity && c->live > c->capacity)"),
    ("alternate_bucket_wrong", "cuckoo_oracle.c",
     "be = (be == c->item_b1[victim]) ? c->item_b2[victim] : c->item_b1[victim];",
     "be = c->item_b2[victim];"),
    ("kick_bound_off_by_one", "cuckoo_oracle.c", "if (kicks == c->max_kicks) {", "if (kicks + 1 == c->max_kicks) {"),
    ("window_one_short", "cuckoo_oracle.c", "last + 1 >= window ? last + 1 - window : 0",
     "last >= window ? last - window + 2 : 0"),
    ("chacha_rotation", "mask_oracle.c", "x[b] = rotl(x[b], 7);", "x[b] = rotl(x[b], 8);"),
    ("chacha_no_feed_forward", "mask_oracle.c", "const uint32_t v = x[i] + s[i];", "const uint32_t v = x[i];"),
    ("chacha_counter_from_one", "mask_oracle.c", "        uint32_t counter = 0;", "        uint32_t counter = 1;"),
    ("rice_k_plus_one", "codec_oracle.c", "    while ((mean >> (k + 1)) != 0)\n        ++k;\n    return k;",
     "    while ((mean >> (k + 1)) != 0)\n        ++k;\n    return k + 1;"),
    ("gap_without_minus_one", "codec_oracle.c", "const uint64_t g = p - prev - 1;\n        for",
     "const uint64_t g = p - prev;\n        for"),
]


@pytest.mark.parametrize("name,src,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, name, src, old, new):
    for f in os.listdir(ORACLE):
        if f.endswith(".c"):
            shutil.copy(os.path.join(ORACLE, f), tmp_path / f)
    text = (tmp_path / src).read_text()
    assert text.count(old) >= 1, f"{name}: the text to mutate is no longer in {src}"
    (tmp_path / src).write_text(text.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    sources = sorted(str(tmp_path / f) for f in os.listdir(tmp_path) if f.endswith(".c"))
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", str(lib), *sources], check=True)
    env = dict(os.environ, TALEK_ORACLE_LIB=str(lib))
    run = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                          *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert run.returncode == 1, f"{name}: no pin failed\n{run.stdout[-2000:]}"
