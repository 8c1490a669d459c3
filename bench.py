"""Benchmark of the XOR-PIR server path on one MI355X.

Default workload: n = 2^22 buckets of 4 x 1 KiB (a 16 GiB database of uniform
bytes), answering batches of B = 2048 Bernoulli(1/2) request vectors through two
levels of Strassen leaves (formed once, then kept up to date by every commit for
the rows its buckets feed); then, as
a second case in the same line ("extra"), n = 65,536 buckets filled by
blocked-cuckoo insertion of 200,000 synthetic messages (256 MiB), B = 256.

One step = one served batch through the whole server path: ceil(B/10) new
Write requests (cuckoo insert with FIFO garbage collection, or whole-bucket
writes for the uniform database; 6 interest bits each) staged and published
as a new epoch, then the batch of B reads answered on that snapshot, then the
global interest vector fetched. Inputs are resident (requests and writes
prepared before the timed region). Prints ONE JSON line on stdout.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4a|c2|c1|c4b|c3b|c3|c5] [--step full|read]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from synth import configs  # noqa: E402

HBM_PEAK_GBS = 8000.0                      # MI355X HBM3E, published
# 32-bit VALU lane-operations per second: 256 CUs x 128 lanes per clock x 2.4 GHz
# = 78.6 T (the FP32 vector figure, 157.3 TFLOP/s, counts an FMA as two flops)
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# LDS rates measured by the roofline probe (bytes per clock and CU, 16-byte
# accesses, no bank conflicts), at 256 CUs and 2.4 GHz
LDS_READ_BPC, LDS_WRITE_BPC = 204.9, 75.4


def lds_floor(plan, n: int, B: int, bucket_bytes: int):
    """Algorithmic LDS traffic of a Four-Russians (wide) read launch and the
    time it takes at the measured LDS rates: every request looks up one table
    row slice per table (a 6-bucket table, or two G-bucket tables per step
    with paired tables: G = 5, 4 or 3, or 6 with half waves), and every
    workgroup writes its step's tables once. Slices are 1 KiB (64 lanes x 16
    bytes), or 512 bytes with half waves (a request per 32 lanes)."""
    if plan.kind != 4:
        return None
    pairs = bool(plan.flags & (1 << 13))
    half = pairs and bool(plan.flags & (1 << 16))
    if pairs:
        G = 6 if plan.flags & (1 << 17) else 5 - ((plan.flags >> 14) & 3)
        per_step, tables, entries = 2 * G, 2, 1 << G
    else:
        per_step, tables, entries = 6, 1, 64
    entry = 512 if half else 1024
    steps = -(-n // per_step)
    slices = -(-bucket_bytes // entry)
    R = plan.tile * plan.unroll
    tiles = -(-B // R)
    rows = -(-B // plan.tile) * plan.tile              # requests of the active waves
    rd = slices * steps * rows * tables * entry
    wr = slices * tiles * steps * tables * entries * entry
    clk = 256 * 2.4e9
    floor_s = rd / (LDS_READ_BPC * clk) + wr / (LDS_WRITE_BPC * clk)
    return {"read_bytes": rd, "write_bytes": wr, "floor_ms": round(1e3 * floor_s, 4)}
INTEREST_K = 6
IV_BITS = 1 << 17        # global interest vector: 16 KiB (the paper's ~14 KB at 1M messages)
IV_WINDOW = 100          # deltas kept: the paper's TTL of 100 write intervals
WRITE_FRAC = 0.1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {1: "xorpir_tile.hip", 2: "xorpir_tile.hip", 3: "xorpir_m4r.hip", 4: "xorpir_m4rw.hip"}


def kernel_source_digest(kind: int) -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_2001_08250_amd", "csrc", KERNEL_SOURCES.get(kind, ""))
    if not os.path.isfile(path):
        return ""
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def summary_key(workload: str, levels: int) -> str:
    """File-name key of a counter summary: the workload, and the Strassen levels
    when the read goes through preprocessed leaves."""
    return workload + (f"-strassen{levels}" if levels else "")


def _summary(kind: str, workload: str, plan):
    """The committed counter summary profiles/<kind>_<workload>.json, or None when
    none matches this workload and plan or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}.json")
    if not os.path.isfile(path):
        return None
    t = json.load(open(path))
    want = {"kind": plan.kind, "tile": plan.tile, "splits": plan.splits, "unroll": plan.unroll, "flags": plan.flags}
    if t.get("plan") != want or t.get("kernel_source_sha256_16") != kernel_source_digest(plan.kind):
        return None
    return t


def measured_valu(workload: str, plan) -> float | None:
    """VALU instructions (SQ_INSTS_VALU) of the main read kernel per read, from the
    committed counter summary (per launch times its launches per read)."""
    t = _summary("valu", workload, plan)
    return None if t is None else float(t["valu_insts_per_launch"]) * float(t.get("launches_per_read", 1))


def measured_traffic(workload: str, plan) -> float | None:
    """HBM bytes of the main read kernel per read, from the committed counter
    summary (per launch times its launches per read)."""
    t = _summary("traffic", workload, plan)
    return None if t is None else float(t["hbm_bytes_per_launch"]) * float(t.get("launches_per_read", 1))


KERNEL_NAMES = {1: "xorpir_tile_kernel", 2: "xorpir_tile_kernel", 3: "xorpir_m4r_kernel",
                4: "xorpir_m4rw_kernel"}
PLAN_PAIRS = 1 << 13
PLAN_HALF_WAVES = 1 << 16


def kernel_name(plan: dict) -> str:
    """Name of the main read kernel a plan launches."""
    if plan["kind"] == 4 and plan["flags"] & PLAN_PAIRS:
        return "xorpir_m4rh_kernel" if plan["flags"] & PLAN_HALF_WAVES else "xorpir_m4rp_kernel"
    return KERNEL_NAMES[plan["kind"]]


def _counter_rows(d: str, counter: str):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    if not rows:
        raise SystemExit(f"no {counter} rows under {d}")
    return rows


def _launches_per_read(rows, name: str, levels: int) -> float:
    """Main-kernel launches per read in a profiled run: 1 for a plain read; for
    a preprocessed one, its launches over the reads' final combining kernels."""
    if not levels:
        return 1.0
    main = {r["Dispatch_Id"] for r in rows if name in r["Kernel_Name"]}
    reads = {r["Dispatch_Id"] for r in rows if "prep_out_kernel" in r["Kernel_Name"]}
    if not reads:
        raise SystemExit("no prep_out_kernel dispatches in a preprocessed run")
    return len(main) / len(reads)


def _calibration_dispatch(rows):
    """The plain copy that --calib-copy-mib runs right after filling its source."""
    for a, b in zip(rows, rows[1:]):
        if "elementwise_kernel" in a["Kernel_Name"] and b["Kernel_Name"] == "__amd_rocclr_copyBuffer":
            return float(b["Counter_Value"])
    raise SystemExit("calibration copy not found (run the profiled bench with --calib-copy-mib)")


def traffic_summary(fetch_dir: str, write_dir: str, bench_json: str, calib_mib: int, command: str):
    """Write profiles/traffic_<workload>.json: HBM bytes per launch of the main read
    kernel from one FETCH_SIZE and one WRITE_SIZE rocprofv3 pass, each scaled by what
    the same counter reads for a plain device copy of calib_mib MiB in the same run."""
    line = json.loads([x for x in open(bench_json) if x.startswith("{")][-1])
    plan = line["config"]["plan"]
    name = kernel_name(plan)
    levels = line["config"].get("strassen_levels", 0)
    out = {"workload": summary_key(line["config"]["workload"], levels), "plan": plan,
           "kernel_source_sha256_16": kernel_source_digest(plan["kind"]), "kernel": name,
           "calibration_copy_kib": calib_mib * 1024, "command": command}
    total = 0.0
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, counter)
        copy_kib = _calibration_dispatch(rows)
        factor = calib_mib * 1024 / copy_kib
        vals = [float(r["Counter_Value"]) for r in rows if name in r["Kernel_Name"]]
        if not vals:
            raise SystemExit(f"no {name} dispatches in {d}")
        kib = float(np.mean(vals))
        out[counter.lower()] = {"copy_kib": copy_kib, "factor": round(factor, 4), "kernel_kib_mean": kib,
                                "dispatches": len(vals), "bytes": kib * factor * 1024}
        total += kib * factor * 1024
        out["launches_per_read"] = _launches_per_read(rows, name, levels)
    out["hbm_bytes_per_launch"] = round(total)
    path = os.path.join(ROOT, "profiles", f"traffic_{out['workload']}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def valu_summary(pmc_dir: str, bench_json: str, command: str):
    """Write profiles/valu_<workload>.json: VALU (and SALU, LDS) instructions per
    launch of the main read kernel from one rocprofv3 --pmc pass (SQ_INSTS_VALU,
    SQ_INSTS_SALU, SQ_INSTS_LDS, GRBM_GUI_ACTIVE) of the bench command."""
    line = json.loads([x for x in open(bench_json) if x.startswith("{")][-1])
    plan = line["config"]["plan"]
    name = kernel_name(plan)
    levels = line["config"].get("strassen_levels", 0)
    out = {"workload": summary_key(line["config"]["workload"], levels), "plan": plan,
           "kernel_source_sha256_16": kernel_source_digest(plan["kind"]), "kernel": name, "command": command}
    for counter, key in (("SQ_INSTS_VALU", "valu_insts_per_launch"), ("SQ_INSTS_SALU", "salu_insts_per_launch"),
                         ("SQ_INSTS_LDS", "lds_insts_per_launch"), ("GRBM_GUI_ACTIVE", "gui_active_per_launch")):
        rows = _counter_rows(pmc_dir, counter)
        vals = [float(r["Counter_Value"]) for r in rows if name in r["Kernel_Name"]]
        if not vals:
            raise SystemExit(f"no {name} dispatches with {counter} in {pmc_dir}")
        out[key] = float(np.mean(vals))
        out["dispatches"] = len(vals)
        out["launches_per_read"] = _launches_per_read(rows, name, levels)
    path = os.path.join(ROOT, "profiles", f"valu_{out['workload']}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def popcount_rows(req: np.ndarray, n: int) -> np.ndarray:
    """Set request bits < n per row."""
    r = np.ascontiguousarray(req[:, :(n + 7) // 8])
    if n % 8:
        r = r.copy()
        r[:, -1] &= np.uint8((1 << (n % 8)) - 1)
    return np.bitwise_count(r).sum(axis=1, dtype=np.int64)


def leaf_request_bits(pir, req: np.ndarray, n: int, levels: int) -> int:
    """Set bits of the request rows of all 7^L Strassen leaves of a read: leaf
    l's row r is the XOR of the request blocks its A-combination names (row
    block i: rows i * Bq + r; column block j: bits j * Nq .. + Nq), rows >= B
    and bits >= n zero; Nq and Bq as the library forms them."""
    t = pir.preprocess_tables(levels)
    g = t["grid"]
    unit = 32 << levels
    nq = -(-n // unit) * unit >> levels
    B = req.shape[0]
    bq = -(-B // g)
    nb = nq // 8
    R = np.zeros((g * bq, g * nb), dtype=np.uint8)
    R[:B, :(n + 7) // 8] = req[:, :(n + 7) // 8]
    if n % 8:
        R[:B, n // 8] &= np.uint8((1 << (n % 8)) - 1)
    total = 0
    for combo in t["a"]:
        acc = np.zeros((bq, nb), dtype=np.uint8)
        for rb, cb in combo:
            acc ^= R[rb * bq:(rb + 1) * bq, cb * nb:(cb + 1) * nb]
        total += int(np.bitwise_count(acc.view(np.uint32)).sum(dtype=np.int64))  # nb % 4 == 0
    return total


def serve_bench(args, pir, rates=None, duration=None, warmup_s=None, probes=None, baseline=True, emit=True):
    """Serving workload: open-loop Poisson reads with 10% writes published every
    epoch, each read returning its answer and the global interest vector.

    Per arrival rate: `warmup_s` + `duration` seconds of arrivals served by the
    continuous-batching loop (latency and throughput over the reads that arrive
    after the warm-up), then the one-launch-per-read baseline on the first
    `baseline_s` seconds of the same trace. Probed reads (64 per rate, spread
    over the run) are checked against the oracle's cuckoo replay on the
    snapshot of the epoch that answered them, and their interest vectors
    against the oracle's window over the published deltas."""
    import oracle
    w = configs.C5
    x = w.extra
    iv_bits = args.iv_bits or x["interest_bits"]
    dur = args.duration if duration is None else duration
    warm = args.warmup_s if warmup_s is None else warmup_s
    n_probes = args.probes if probes is None else probes
    t = time.perf_counter()
    db = pir.PirDB(w.n, w.d, w.z)
    db.interest_config(iv_bits, x["window"])
    pre = synth.write_ops(w.cuckoo_seed, w.cuckoo_items, w.n, w.z)
    ck = pir.Cuckoo(db, capacity=w.cuckoo_items, seed=w.cuckoo_seed, max_kicks=configs.CUCKOO_MAX_KICKS)
    ck.insert_many(*pre)
    ck.stage()
    e_pre = db.commit()
    ref = None
    if not args.no_parity:
        ref = oracle.Cuckoo(w.n, w.d, w.z, capacity=w.cuckoo_items, seed=w.cuckoo_seed,
                            max_kicks=configs.CUCKOO_MAX_KICKS)
        ref.insert_many(*pre)
    del pre
    log(f"[serve] {w.name}: database of {w.db_bytes >> 30} GiB ready in {time.perf_counter() - t:.1f}s")
    pool = synth.bernoulli_requests(w.req_seed, 1024, w.n)
    deltas = {}        # published epoch -> interest positions of the writes it published
    results = []
    parity_all = None if ref is None else True
    checked = 0

    def publish_rest(writes, wep, ipos):
        """Publish what the run left staged; feed the run's writes to the oracle in order."""
        e_end = db.commit()
        wep = wep.copy()
        wep[wep == np.iinfo(np.uint64).max] = e_end
        for e in np.unique(wep):
            deltas.setdefault(int(e), []).append(ipos[wep == e].reshape(-1))
        return wep

    for rate in rates or [r for r in x["rates"] if not args.rates or r in args.rates]:
        span = warm + dur
        read_t = synth.poisson_arrivals(x["arrival_seed"] + rate, rate, span)
        rows = synth.uniform_indices(x["arrival_seed"] + rate + 1, read_t.size, 1024).astype(np.uint32)
        write_t = synth.poisson_arrivals(x["arrival_seed"] + rate + 2, x["write_frac"] * rate, span)
        writes = synth.write_ops(w.cuckoo_seed + rate, write_t.size, w.n, w.z,
                                 id_offset_seed=w.cuckoo_seed + rate + 3)
        ipos = synth.interest_positions(x["arrival_seed"] + rate + 4, write_t.size, x["interest_k"], iv_bits)
        row = {"rate": rate, "reads": int(read_t.size), "writes": int(write_t.size)}
        for mode, mb, lanes in (("batched", args.max_batch, args.lanes), ("one_per_read", 1, 4)):
            if mode == "one_per_read" and (args.no_baseline or not baseline):
                continue
            # the one-launch-per-read baseline is given a shorter slice of the same trace
            n_r = read_t.size if mode == "batched" else int(np.searchsorted(read_t, min(span, args.baseline_s)))
            n_w = int(np.searchsorted(write_t, read_t[n_r - 1])) if n_r else 0
            post = np.nonzero(read_t[:n_r] >= (warm if mode == "batched" else 0.0))[0]
            probe = None
            if mode == "batched" and ref is not None and post.size:
                probe = post[np.unique(np.linspace(0, post.size - 1, n_probes).round().astype(np.int64))]
            log(f"[serve] rate {rate}/s {mode}: {n_r} reads, {n_w} writes")
            wsl = tuple(a[:n_w] for a in writes)
            out = pir.serve(db, ck, read_t=read_t[:n_r], read_row=rows[:n_r], req_pool=pool,
                            write_t=write_t[:n_w], writes=wsl, write_interest=ipos[:n_w], max_batch=mb,
                            lanes=lanes, epoch_s=x["epoch_s"], probe=probe, with_iv=probe is not None)
            lat = out["latency_s"][post]
            done_t = read_t[post] + lat
            t0 = warm if mode == "batched" else 0.0
            served = post.size / max(float(done_t.max()) - t0, 1e-9) if post.size else 0.0
            row[mode] = {"reads_per_s": round(served, 1), "p50_ms": round(1e3 * percentile(lat, 50), 3),
                         "p99_ms": round(1e3 * percentile(lat, 99), 3), "max_ms": round(1e3 * float(lat.max()), 3),
                         "measured_reads": int(post.size), "mean_batch": round(out["mean_batch"], 1),
                         "batches": int(out["batches"]), "epochs": int(out["epochs"]),
                         "wall_s": round(out["wall_s"], 3)}
            wep = publish_rest(wsl, out["write_epoch"], ipos[:n_w])
            if ref is not None:
                # the oracle replays the run's writes epoch by epoch and answers
                # each probed read on the snapshot of the epoch that served it
                ep = out["read_epoch"]
                need = {} if probe is None else {int(e): [] for e in ep[probe]}
                for k, rd in enumerate(probe if probe is not None else []):
                    need[int(ep[rd])].append(k)
                ok = True
                order = np.argsort(wep, kind="stable")
                pos = 0
                for e in sorted(set(int(v) for v in np.unique(wep)) | set(need)):
                    sel = []
                    while pos < order.size and int(wep[order[pos]]) <= e:
                        sel.append(order[pos])
                        pos += 1
                    if sel:
                        sel = np.sort(np.asarray(sel))
                        ref.insert_many(wsl[0][sel], wsl[1][sel], wsl[2][sel], wsl[3][sel])
                    if e in need:
                        ks = need[e]
                        rds = probe[ks]
                        want = oracle.pir_read(ref.table_view(), pool[rows[rds]], threads=16)
                        ok = ok and bool(np.array_equal(want, out["probe_resp"][ks]))
                        ev = [np.concatenate(deltas.get(i, [np.zeros(0, np.uint32)])) for i in range(1, e + 1)]
                        want_iv = oracle.interest_window(iv_bits, ev, e - 1, x["window"])
                        ok = ok and all(np.array_equal(want_iv, out["probe_iv"][k]) for k in ks)
                        checked += len(ks)
                if probe is not None:
                    row[mode]["parity"] = {"probed_reads": int(probe.size), "epochs": len(need), "bit_exact": ok}
                parity_all = parity_all and ok
            log(f"[serve]   {row[mode]}")
        results.append(row)
    db.close()
    best = max(results, key=lambda r: r["batched"]["reads_per_s"])
    line = {
        "metric": "PIR bucket-reads/sec at stated p99 (serving)",
        "value": best["batched"]["reads_per_s"],
        "unit": "reads/s",
        "n_gpus": 1,
        "steps": len(results),
        "warmup": 0,
        "ms_per_step": round(1e3 * dur, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_buckets": w.n, "d": w.d, "msg_bytes": w.z, "duration_s": dur,
                   "warmup_s": warm, "interest_bits": iv_bits, "interest_window": x["window"],
                   "max_batch": args.max_batch, "lanes": args.lanes, "parallelism": "single-gpu"},
        "p99_ms_at_best": best["batched"]["p99_ms"],
        "parity": parity_all,
        "parity_reads_checked": checked,
        "serving": results,
    }
    if emit:
        print(json.dumps(line), flush=True)
    return line


def stream_bench(args, pir, torch):
    """Uneven batches: n = 2^20 x 4 KiB, batch sizes uniform in [1, 1024].

    Four ways to answer the same stream, each timed over `steps` passes after
    one untimed pass: the fused launch groups of 1024 requests replayed from a
    HIP graph, and one launch sequence per batch, each first with the
    heuristic schedules and then with schedules that the tuner picked for
    every batch-size class the stream uses."""
    w = configs.C3
    nb = args.batches or w.batches
    sizes = synth.batch_sizes(w.batch_seed, nb)
    total = int(sizes.sum())
    t = time.perf_counter()
    D = synth.uniform_db(w.db_seed, w.n, w.bucket_bytes, threads=16)
    db = pir.PirDB(w.n, w.d, w.z)
    db.load(D)
    pool = synth.bernoulli_requests(w.req_seed, 1024, w.n)
    rng = np.random.default_rng(w.batch_seed)
    first = np.array([rng.integers(0, 1024 - s + 1) for s in sizes], dtype=np.uint64)
    log(f"[stream] {nb} batches, {total} reads; database ready in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    q = torch.from_numpy(pool).to(dev)
    out = torch.empty((total, w.bucket_bytes), dtype=torch.uint8, device=dev)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)

    def fused():
        db.read_stream_async(q, sizes, out, req_first=first)

    def per_batch():
        for k in range(nb):
            b = int(sizes[k])
            f = int(first[k])
            db.read_async(q[f:f + b], out[starts[k]:starts[k] + b])

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        return {"reads_per_s": round(total / dt, 1), "ms_per_stream": round(1e3 * dt, 2)}

    res = {}
    res["fused_graph_heuristic"] = timed(fused)
    res["per_batch_heuristic"] = timed(per_batch)
    if not args.no_tune:
        # every batch-size class (next power of two) that either form launches:
        # the fused groups (1024 requests, plus the last group's rest) and the
        # batches themselves
        rest = total % 1024
        classes = sorted({1 << int(np.ceil(np.log2(max(int(b), 1)))) for b in list(sizes) + [1024, rest or 1024]})
        t1 = time.perf_counter()
        tuned = {}
        for Bt in classes:
            p, us = db.tune(Bt, iters=2)
            tuned[Bt] = {"kind": p.kind, "tile": p.tile, "splits": p.splits, "unroll": p.unroll, "flags": p.flags,
                         "us": round(us, 1)}
            log(f"[stream] tuned B={Bt}: {p} {us:.0f} us")
        res["tuning_s"] = round(time.perf_counter() - t1, 1)
        res["tuned_plans"] = tuned
        res["fused_graph_tuned"] = timed(fused)
        res["per_batch_tuned"] = timed(per_batch)
    # sampled answers against the oracle (rows spread over the stream)
    import oracle
    rows = np.unique(np.linspace(0, total - 1, 16).round().astype(np.int64))
    k_of = np.searchsorted(starts, rows, side="right") - 1
    req_rows = pool[first[k_of].astype(np.int64) + (rows - starts[k_of])]
    want = oracle.pir_read(D, req_rows, threads=16)
    parity = bool(np.array_equal(want, out.cpu().numpy()[rows]))
    log(f"[stream] {res}; parity={parity}")
    rates = {k: v for k, v in res.items() if isinstance(v, dict) and "reads_per_s" in v}
    best = max(rates.values(), key=lambda r: r["reads_per_s"])
    line = {"metric": "PIR bucket-reads/sec (uneven batch stream)", "value": best["reads_per_s"], "unit": "reads/s",
            "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": best["ms_per_stream"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": w.name, "n_buckets": w.n, "d": w.d, "msg_bytes": w.z, "batches": nb,
                       "reads": total, "parallelism": "single-gpu"},
            "stream": res, "parity_sampled": parity}
    print(json.dumps(line), flush=True)
    db.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4a", choices=["c1", "c2", "c3", "c4a", "c4b", "c3b", "c5"])
    ap.add_argument("--duration", type=float, default=30.0, help="serving: measured seconds of arrivals per rate")
    ap.add_argument("--warmup-s", type=float, default=3.0, help="serving: seconds of arrivals before the measured ones")
    ap.add_argument("--iv-bits", type=int, default=0, help="serving: interest-vector bits (default 2^20)")
    ap.add_argument("--probes", type=int, default=64, help="serving: reads per rate checked against the oracle")
    ap.add_argument("--no-parity", action="store_true", help="serving: skip the oracle replay")
    ap.add_argument("--baseline-s", type=float, default=1.0, help="serving: seconds of the one-per-read baseline")
    ap.add_argument("--max-batch", type=int, default=256, help="serving: reads per launch (256: one request tile of the paired-table kernel)")
    ap.add_argument("--rates", type=int, nargs="*", default=[], help="serving: subset of the arrival rates")
    ap.add_argument("--lanes", type=int, default=2, help="serving: batches in flight")
    ap.add_argument("--no-baseline", action="store_true")
    ap.add_argument("--batches", type=int, default=0, help="uneven stream: number of batches (default 500)")
    ap.add_argument("--step", default="", choices=["", "full", "read"],
                    help="full = writes + commit + read + interest fetch (default for cuckoo workloads)")
    ap.add_argument("--B", type=int, default=0, help="override the batch size")
    ap.add_argument("--kind", type=int, default=0, help="force kernel family (1 mask, 2 skip, 3 four-russians)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--splits", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--flags", type=int, default=0, help="plan flags (1 = waves share a column chunk)")
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="uneven stream: skip the tuned schedules")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="oracle rows on all host cores (default: every row up to 1 GiB databases, else 48)")
    ap.add_argument("--cpu-rows-single", type=int, default=-1,
                    help="oracle rows on one core (default: 4 over databases above 1 GiB, else 16)")
    ap.add_argument("--latency-reads", type=int, default=20, help="batches issued alone for the latency figures")
    ap.add_argument("--no-extra", action="store_true", help="c4a: skip the 256 MiB second case")
    ap.add_argument("--read-streams", type=int, default=1,
                    help="read streams that consecutive batches take in turn (1 = every batch on one stream)")
    ap.add_argument("--prep", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="answer through L levels of Strassen leaves formed at commit and kept up to date row by "
                         "row (default: 2 for the 16 GiB workload, else 0)")
    ap.add_argument("--time-every", type=int, default=5,
                    help="time the main kernel of every k-th timed read with HIP events (1 = all)")
    ap.add_argument("--masked", action="store_true",
                    help="serialized PIR: every answer XORed with a ChaCha20 one-time mask from a per-request seed")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "BENCH_JSON"),
                    help="no GPU: turn two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) of a bench run "
                         "made with --calib-copy-mib into profiles/traffic_<workload>.json")
    ap.add_argument("--traffic-command", default="", help="the profiled command, recorded with the summary")
    ap.add_argument("--valu-summary", nargs=2, metavar=("PMC_DIR", "BENCH_JSON"),
                    help="no GPU: turn one rocprofv3 --pmc pass (SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_INSTS_LDS, "
                         "GRBM_GUI_ACTIVE) of a bench run into profiles/valu_<workload>.json")
    args = ap.parse_args()
    if args.traffic_summary:
        return traffic_summary(*args.traffic_summary, args.calib_copy_mib or 256, args.traffic_command)
    if args.valu_summary:
        return valu_summary(*args.valu_summary, args.traffic_command)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (one server's share runs on one "
              "MI355X); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2001_08250_amd as pir

    torch.cuda.set_device(0)
    if args.workload == "c5":
        return serve_bench(args, pir)
    if args.workload == "c3":
        return stream_bench(args, pir, torch)
    key = args.workload
    w = WORKLOADS[key]
    B = args.B or w.B or 1024
    if args.prep < 0:
        # Strassen leaves (maintained row by row at every commit) for the
        # 2048-request batches of the 16 GiB database, the plain read elsewhere
        args.prep = 2 if key == "c4a" and not (args.kind or args.masked or args.B) else 0
    big = w.db_bytes > (1 << 30)
    # oracle sample: about 10 s on all host cores and 8 s on one over the 16 GiB
    # database (5 and 0.5 reads/s)
    cpu_rows = args.cpu_rows or (48 if big else B)
    cpu_single = args.cpu_rows_single if args.cpu_rows_single >= 0 else (4 if big else 16)
    line = fixed_bench(args, pir, torch, w, B, args.steps, args.warmup, cpu_rows, cpu_single,
                       latency=args.latency_reads)
    if key == "c4a" and not args.no_extra and not (args.kind or args.masked or args.B):
        # the paper-scale 256 MiB database as a second, cache-sized case (plain
        # read: its 256-request batches are below the leaves' threshold)
        levels, args.prep = args.prep, 0
        keep = ("value", "ms_per_step", "config", "roofline", "cpu_baseline", "parity_sampled", "read_latency_ms")
        sub = fixed_bench(args, pir, torch, configs.C2, configs.C2.B, 50, 5, 16, 0, latency=50)
        line["extra"] = {"c2": {k: sub[k] for k in keep}}
        # a small batch over a database larger than the caches (4 GiB, B = 64):
        # the HBM-bound regime
        sub = fixed_bench(args, pir, torch, configs.C3B64, configs.C3B64.B, 20, 3, 4, 0, latency=20)
        line["extra"]["b64_4GiB"] = {k: sub[k] for k in keep}
        args.prep = levels
        # serving: 20k Poisson reads/s over 4 GiB for 5 s after 1 s, each with the
        # 128 KiB interest vector, 16 probed reads against the oracle's replay
        srv = serve_bench(args, pir, rates=[20_000], duration=5.0, warmup_s=1.0, probes=16, baseline=False,
                          emit=False)
        b = srv["serving"][0]["batched"]
        line["extra"]["serving"] = {"workload": srv["config"]["workload"], "offered_reads_per_s": 20_000,
                                    "served_reads_per_s": b["reads_per_s"], "p50_ms": b["p50_ms"],
                                    "p99_ms": b["p99_ms"], "max_ms": b["max_ms"], "duration_s": 5.0,
                                    "interest_bits": srv["config"]["interest_bits"], "parity": srv["parity"],
                                    "parity_reads_checked": srv["parity_reads_checked"]}
    print(json.dumps(line), flush=True)


WORKLOADS = {"c1": configs.C1, "c2": configs.C2, "c4a": configs.C4A, "c4b": configs.C4B, "c3b": configs.C3}


def host_info() -> dict:
    """Host cores the CPU baseline may use: count, affinity mask and model."""
    aff = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else list(range(os.cpu_count() or 1))
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    mask = 0
    for c in aff:
        mask |= 1 << c
    return {"nproc": os.cpu_count(), "affinity_cpus": len(aff), "affinity_mask": hex(mask), "cpu_model": model}


def percentile(x, q: float) -> float:
    """Nearest-rank percentile."""
    x = np.sort(np.asarray(x, dtype=np.float64))
    if x.size == 0:
        return float("nan")
    return float(x[min(x.size - 1, max(0, int(np.ceil(q / 100.0 * x.size)) - 1))])


def fixed_bench(args, pir, torch, w, B: int, K: int, W: int, cpu_rows: int, cpu_rows_single: int, latency: int):
    """One workload with a fixed batch size: K timed steps after W warm-up steps.

    A step is the whole server path for one batch: ceil(B/10) writes (cuckoo
    inserts with garbage collection for cuckoo-filled databases, whole-bucket
    writes otherwise) with 6 interest bits each, the epoch commit that publishes
    them, the read of the B request rows on the new snapshot, and the fetch of
    the global interest vector."""
    full = (args.step or "full") == "full"
    log(f"[bench] workload {w.name} n={w.n} d={w.d} z={w.z} B={B} step={'full' if full else 'read'}")

    # ---- database -------------------------------------------------------
    t = time.perf_counter()
    db = pir.PirDB(w.n, w.d, w.z)
    db.interest_config(IV_BITS, IV_WINDOW)
    ck = None
    pre = None
    if w.fill == "cuckoo":
        pre = synth.write_ops(w.cuckoo_seed, w.cuckoo_items, w.n, w.z)
        ck = pir.Cuckoo(db, capacity=w.cuckoo_items, seed=w.cuckoo_seed, max_kicks=configs.CUCKOO_MAX_KICKS)
        status, _ = ck.insert_many(*pre)
        ck.stage()
        D0 = None
    else:
        D0 = synth.uniform_db(w.db_seed, w.n, w.bucket_bytes, threads=16)
        db.write_range(0, D0)
    db.commit()
    log(f"[bench] database ready in {time.perf_counter() - t:.1f}s")

    # ---- per-step writes (prepared before timing) ---------------------------
    nw = max(1, -(-B // int(1 / WRITE_FRAC))) if full else 0
    total_w = nw * (W + K)
    if full:
        if ck is not None:
            wr = synth.write_ops(w.cuckoo_seed + 17, total_w, w.n, w.z, id_offset_seed=w.cuckoo_seed + 18)
        else:
            wr = (None, synth.uniform_indices(w.req_seed + 5, total_w, w.n), None,
                  synth.uniform_bytes(w.req_seed + 6, total_w * w.bucket_bytes).reshape(total_w, w.bucket_bytes))
        ipos = synth.interest_positions(w.req_seed + 7, total_w, INTEREST_K, IV_BITS)

    req = synth.bernoulli_requests(w.req_seed, B, w.n)
    if args.prep:
        t = time.perf_counter()
        db.preprocess(args.prep, 1)
        torch.cuda.synchronize()
        log(f"[bench] preprocessed ({args.prep} Strassen levels) in {time.perf_counter() - t:.2f}s")
    if args.kind:
        db.set_plan(args.kind, args.tile, args.splits, args.unroll, args.flags)
    if args.tune:
        p, us = db.tune(B, iters=3)
        log(f"[bench] tuned: {p} {us:.1f} us")
    plan = db.get_plan(B)
    log(f"[bench] plan {plan}")

    dev = torch.device("cuda:0")
    q = torch.from_numpy(req).to(dev)
    seeds = synth.uniform_bytes(w.req_seed + 99, B * 32).reshape(B, 32) if args.masked else None
    seeds_dev = torch.from_numpy(seeds).to(dev) if args.masked else None
    # Consecutive batches are independent; with R > 1 they go out on R read
    # streams in turn (default priority), so that one batch's split reduction
    # and the next batch's offset staging can overlap the neighbouring main
    # kernel. The main kernel's event-timed duration then includes its wait
    # for compute units, so the default is one stream.
    R = max(1, args.read_streams)
    read_streams = [torch.cuda.current_stream()] + [torch.cuda.Stream(device=dev) for _ in range(R - 1)]
    outs = [torch.empty((B, w.bucket_bytes), dtype=torch.uint8, device=dev) for _ in range(R)]
    iv = torch.empty((IV_BITS // 8,), dtype=torch.uint8, device=dev)
    # The interest-vector fetch depends only on the published epoch, not on
    # the read, so it goes out on a second stream (default priority) beside it.
    iv_stream = torch.cuda.Stream(device=dev)
    iv_sh = int(iv_stream.cuda_stream)
    L = pir.lib()

    # host seconds per part of the step, summed over the timed steps
    host_s = {"insert": 0.0, "stage": 0.0, "interest_add": 0.0, "commit": 0.0, "read_call": 0.0}

    def do_writes(k):
        sl = slice(k * nw, (k + 1) * nw)
        t0 = time.perf_counter()
        if ck is not None:
            ck.insert_many(wr[0][sl], wr[1][sl], wr[2][sl], wr[3][sl])
            t1 = time.perf_counter()
            ck.stage()
        else:
            for i in range(sl.start, sl.stop):
                db.write_bucket(int(wr[1][i]), wr[3][i])
            t1 = time.perf_counter()
        t2 = time.perf_counter()
        db.interest_add(ipos[sl])
        t3 = time.perf_counter()
        db.commit()
        t4 = time.perf_counter()
        for key, dt in (("insert", t1 - t0), ("stage", t2 - t1), ("interest_add", t3 - t2), ("commit", t4 - t3)):
            host_s[key] += dt

    def step(k):
        if full:
            do_writes(k)
        t = time.perf_counter()
        rs, out = read_streams[k % R], outs[k % R]
        if seeds_dev is not None:
            db.read_masked_async(q, seeds_dev, out, stream=rs)
        else:
            db.read_async(q, out, stream=rs)
        host_s["read_call"] += time.perf_counter() - t
        if full:
            rc = L.pir_interest_vector_async(db.h, iv.data_ptr(), iv.numel(), iv_sh)
            assert rc == 0, rc

    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                      # read and write calib_copy_mib MiB each
        torch.cuda.synchronize()
        del src, dst
    for k in range(W):
        step(k)
    torch.cuda.synchronize()
    # The main read kernel's dispatch records the start and end events of
    # every `time_every`-th read of the timed region on the read's stream
    # (a sample, so that the events' own cost stays out of the step time).
    db.profile_enable(True, args.time_every)
    for key in host_s:
        host_s[key] = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        step(W + k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = db.profile_collect()
    db.profile_enable(False)
    got = outs[(W + K - 1) % R].cpu().numpy()   # the last step's answers
    got_iv = iv.cpu().numpy()
    # Per-read latency: a read's answer is complete when its batch's is, so
    # each of `latency` batches is issued alone on the published snapshot
    # (requests already in device memory) and timed from the call to the
    # completion of its answers.
    lat = []
    rs0 = read_streams[0]
    for _ in range(latency):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        db.read_async(q, outs[0], stream=rs0)
        rs0.synchronize()
        lat.append(time.perf_counter() - t1)
    lat_ms = {"p50": round(1e3 * percentile(lat, 50), 4), "p99": round(1e3 * percentile(lat, 99), 4),
              "max": round(1e3 * max(lat), 4) if lat else None, "batches": len(lat), "reads_per_batch": B,
              "what": "call to completed answers of a batch issued alone (device-resident requests)"}
    # The synchronous call (host request rows in, host answers out, so the
    # PCIe copies included), after the timed region: never the headline value.
    n_sync = 10 if B <= 256 else 3
    db.read(req)
    t1 = time.perf_counter()
    for _ in range(n_sync):
        db.read(req)
    t_sync = (time.perf_counter() - t1) / n_sync
    pcie = {"call": "pir_read_batch (host buffers)", "ms_per_batch": round(1e3 * t_sync, 4),
            "reads_per_s": round(B / t_sync, 1)}
    codec = None
    if full:
        # GetUpdates payloads (not timed above): the published global vector and
        # the latest epoch's delta, raw and compressed, and the encode time
        t1 = time.perf_counter()
        g_bytes = len(db.interest_encoded())
        t_enc = time.perf_counter() - t1
        e_last = int(L.pir_epoch(db.h))
        codec = {"raw_bytes": IV_BITS // 8, "global_encoded_bytes": g_bytes,
                 "delta_encoded_bytes": len(db.interest_encoded(e_last)),
                 "global_encode_ms": round(1e3 * t_enc, 3)}
    assert kern.size == min(-(-K // args.time_every), pir.PROFILE_MAX)
    kern_ms = float(np.mean(kern))
    db.close()

    ms_per_step = 1000.0 * wall / K
    value = B * K / wall
    pops = popcount_rows(req, w.n)
    # plain dword-XOR count of the batch's product (one per selected bucket word)
    xor_ops = float(pops.sum()) * (w.bucket_bytes / 4)
    # ... and of the products the kernel computes: the 7^L leaf products (each
    # a plain GF(2) product of its own request rows with its leaf database,
    # Strassen's 7^L / 8^L of the batch's work) when the read uses the leaves
    xor_ops_alg = xor_ops
    if args.prep:
        xor_ops_alg = float(leaf_request_bits(pir, req, w.n, args.prep)) * ((w.bucket_bytes >> args.prep) / 4)
    alg_bytes = w.n * w.bucket_bytes + B * ((w.n + 7) // 8) + B * w.bucket_bytes
    t_kernel = kern_ms / 1000.0
    hbm_achieved = alg_bytes / t_kernel / 1e9
    alu_achieved = xor_ops_alg / t_kernel / 1e12
    answers_tops = xor_ops / t_kernel / 1e12
    t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
    t_alu = xor_ops_alg / (VALU_PEAK_TOPS * 1e12)
    if t_alu >= t_hbm:
        roof = {"bound": "alu", "achieved": round(alu_achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(alu_achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                "achieved_is": ("XORs of the plain method over the 7^L Strassen leaf products the kernel computes "
                                "(one 32-bit XOR per selected leaf-bucket word) per second of the main read kernel"
                                if args.prep else
                                "XORs of the plain method (one 32-bit XOR per selected bucket word) per second "
                                "of the main read kernel")}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "achieved_is": "algorithmic bytes (database once, requests, answers) per second of the main "
                               "read kernel"}
    # With Strassen leaves the main kernel answers 7^L leaves (products of
    # n/2^L buckets x d*z/2^L bytes x B/2^L requests), in one launch when their
    # offsets are staged together (else one launch per leaf); its figures are
    # summed over the read's leaves and kern_ms spans the first leaf's start to
    # the last one's end.
    leaves = 7 ** args.prep if args.prep else 1
    key = summary_key(w.name, args.prep)
    traffic = measured_traffic(key, plan)
    roof["traffic"] = traffic
    if args.prep:
        unit = 32 << args.prep
        nq, bq, cq = -(-w.n // unit) * unit >> args.prep, -(-B // (1 << args.prep)), w.bucket_bytes >> args.prep
        # the leaves take the automatic plan of their shape: the same family as
        # this batch's while both are above 256 requests
        one = lds_floor(plan, nq, bq, cq) if bq > 256 and B > 256 else None
        lds = None if one is None else {"read_bytes": one["read_bytes"] * leaves,
                                        "write_bytes": one["write_bytes"] * leaves,
                                        "floor_ms": round(one["floor_ms"] * leaves, 4), "leaves": leaves}
    else:
        lds = lds_floor(plan, w.n, B, w.bucket_bytes)
    if lds:
        lds["frac"] = round(lds["floor_ms"] / kern_ms, 4)   # of the LDS-bound floor
        roof["lds"] = lds
    # both plain-method fractions, whichever bound applies
    roof.update(kernel_ms=round(kern_ms, 4), hbm_gbs_alg=round(hbm_achieved, 1),
                hbm_frac=round(hbm_achieved / HBM_PEAK_GBS, 4), plain_xor_tops=round(alu_achieved, 3),
                valu_frac=round(alu_achieved / VALU_PEAK_TOPS, 4), alg_bytes=alg_bytes, plain_xor_ops=xor_ops_alg)
    if args.prep:
        # the whole batch's plain count per second: how fast answers come in
        # the plain method's units (not a utilisation: Strassen skips 1/8 of
        # the work per level, so it can pass the peak)
        roof.update(answers_plain_equiv_tops=round(answers_tops, 3),
                    answers_plain_equiv_frac=round(answers_tops / VALU_PEAK_TOPS, 4), answers_plain_xor_ops=xor_ops)
    inst = measured_valu(key, plan)
    if inst is not None:
        # VALU instructions the kernel really executes (counter summary), as lane-operations per second
        roof["valu_executed_frac"] = round(inst * 64 / t_kernel / (VALU_PEAK_TOPS * 1e12), 4)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        hi = host_info()
        threads = max(1, min(16, hi["affinity_cpus"]))
        # the oracle rebuilds the final snapshot from the same writes
        if ck is not None:
            ref = oracle.Cuckoo(w.n, w.d, w.z, capacity=w.cuckoo_items, seed=w.cuckoo_seed,
                                max_kicks=configs.CUCKOO_MAX_KICKS)
            ref.insert_many(*pre)
            if full:
                ref.insert_many(wr[0][:total_w], wr[1][:total_w], wr[2][:total_w], wr[3][:total_w])
            D = ref.table()
        else:
            D = D0                       # the device holds its own copy: apply the writes in place
            if full:
                for i in range(total_w):
                    D[int(wr[1][i])] = wr[3][i]
        # sampled rows spread over the batch (every block of a preprocessed read)
        rows = np.unique(np.linspace(0, B - 1, min(cpu_rows, B)).round().astype(np.int64))
        t1 = time.perf_counter()
        want = (oracle.pir_read_masked(D, req[rows], seeds[rows], threads=threads) if args.masked
                else oracle.pir_read(D, req[rows], threads=threads))
        dt = time.perf_counter() - t1
        parity = bool(np.array_equal(want, got[rows]))
        single = None
        if cpu_rows_single:
            r1 = rows[:cpu_rows_single]
            t1 = time.perf_counter()
            want1 = oracle.pir_read(D, req[r1], threads=1)
            dt1 = time.perf_counter() - t1
            parity = parity and bool(np.array_equal(want1, got[r1]))
            single = {"value": round(len(r1) / dt1, 3), "rows": int(len(r1)), "seconds": round(dt1, 3)}
        if full:
            last = W + K - 1
            epochs = [np.zeros(0, np.uint32)] + [ipos[k * nw:(k + 1) * nw].reshape(-1) for k in range(W + K)]
            want_iv = oracle.interest_window(IV_BITS, epochs, last + 1, IV_WINDOW)
            parity = parity and bool(np.array_equal(want_iv, got_iv))
        part = len(rows) < B
        cpu = {"value": round(len(rows) / dt, 3), "unit": "reads/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(rows)} of the {B} request rows of the last batch over the full "
                         f"{w.db_bytes >> 20} MiB snapshot, plain C byte loop (gcc -O2), {threads} threads, "
                         f"{dt:.2f} s" + ("; reads/s extrapolated from the sample" if part else ""),
               "extrapolated": part, "single_thread": single, **hi}
        log(f"[bench] oracle {cpu['value']} reads/s on {threads} threads"
            + (f", {single['value']} on one" if single else "") + f"; parity={parity}")
    del D0

    return {
        "metric": "PIR bucket-reads/sec",
        "value": round(value, 1),
        "unit": "reads/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_buckets": w.n, "d": w.d, "msg_bytes": w.z, "B": B,
                   "step": ("writes+commit+read+interest" if full else "read") + (" (masked)" if args.masked else ""),
                   "writes_per_step": nw, "read_streams": R, "strassen_levels": args.prep,
                   "plan": {"kind": plan.kind, "tile": plan.tile, "splits": plan.splits, "unroll": plan.unroll,
                            "flags": plan.flags},
                   "parallelism": "single-gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity_sampled": parity,
        "read_latency_ms": lat_ms,
        "host_ms_per_step": {key: round(1e3 * v / K, 4) for key, v in host_s.items()},
        "interest_codec": codec,
        "pcie_inclusive": pcie,
    }


if __name__ == "__main__":
    main()
