#!/usr/bin/env python3
"""Benchmark of the exact all-pairs Jaccard hot path on one MI355X.

One step = jas_encode (stage/validate, sort + dedup, compaction, batches, pack,
column sums) + jas_gram (packed-tile popcount Gram, row-list pairs, diagonal,
unions, J) over one synthetic collection that is already resident in HBM.
Prints one JSON line: the pair rate, the roofline of the dominant kernel, the
oracle's rate on a bounded sample, a serving run and per-kernel times.

  python bench.py [--steps K] [--warmup W] [--workload paperlike]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s
MFMA_I8_PEAK_TOPS = 5000.0     # dense int8 MFMA, TOP/s
MFMA_FP4_PEAK_TOPS = 10100.0   # dense fp4 MFMA, TFLOP/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash(kernel: str) -> str:
    src = {"radix_scatter": "radix.hip", "radix_onesweep": "radix.hip", "radix_hist": "radix.hip",
           "gram_popc": "gram.hip", "gram_mfma": "gram.hip", "gram_fp4": "gram.hip", "list_pairs": "gram.hip",
           "pair_count": "gram.hip", "cls_count": "encode.hip", "cls_write": "encode.hip",
           "local_cls": "encode.hip", "local_cls_wide": "encode.hip", "local_move": "encode.hip", "pair_emit": "encode.hip",
           "pair_sort": "radix.hip",
           "pack": "encode.hip", "build_keys": "encode.hip", "count_digits": "encode.hip"}.get(kernel)
    if src is None:
        return ""
    h = hashlib.sha256()
    for f in (src, "device_util.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1911_04200_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic(kernel: str, stats: dict, n: int, N: int, passes: int):
    """(bound, algorithmic amount per launch, unit, per-unit description) of a kernel."""
    if kernel in ("radix_scatter", "radix_onesweep"):
        return "hbm", 16.0 * N / 1e9, "GB/s", "16 B per key per pass (read 8 + write 8)"
    if kernel == "radix_hist":
        return "hbm", 8.0 * N / 1e9, "GB/s", "8 B per key per pass (read)"
    if kernel == "build_keys":
        return "hbm", 16.0 * N / 1e9, "GB/s", "16 B per entry (read ID 8 + write key 8)"
    if kernel == "count_digits":
        return "hbm", 8.0 * N / 1e9, "GB/s", "8 B per entry (read ID)"
    if kernel == "cls_count":
        return "hbm", 8.0 * N / 1e9, "GB/s", "8 B per sorted key (read)"
    if kernel == "cls_write":
        return ("hbm", (8.0 * N + 4.0 * stats["n_pairs"] + 16.0 * stats["n_shared_rows"]) / 1e9, "GB/s",
                "8 B per key read + 4 B per shared pair + 16 B per shared row written")
    if kernel in ("local_cls", "local_cls_wide"):
        shared = stats["n_pairs"] - (stats["n_rows"] - stats["n_shared_rows"])
        return ("hbm", (8.0 * N + 4.0 * shared + 16.0 * stats["n_shared_rows"]) / 1e9, "GB/s",
                "8 B per key read + 4 B per shared pair + 16 B per shared row written")
    if kernel == "local_move":
        return ("hbm", 44.0 * stats["n_shared_rows"] / 1e9, "GB/s",
                "per shared row: its ID, start and the next start read (24 B), its ID, start and degree written "
                "(20 B); the ranges' offsets are not counted")
    if kernel == "pair_sort":
        return "hbm", 8.0 * stats["list_pairs"] / 1e9, "GB/s", "8 B per 32-bit pair word per pass (read 4 + write 4)"
    if kernel == "pair_emit":
        return "hbm", 4.0 * stats["list_pairs"] / 1e9, "GB/s", "4 B per pair word written (+ the row lists read)"
    if kernel == "pair_count":
        return "hbm", 4.0 * stats["list_pairs"] / 1e9, "GB/s", "4 B per pair word read"
    if kernel == "pack":
        ldw = math.ceil(n / 128) * 128
        return "hbm", 8.0 * stats["n_word_rows"] * ldw / 1e9, "GB/s", "8 B per packed word written"
    if kernel == "list_pairs":
        lp, rows = stats["list_pairs"], stats["n_list_rows"]
        return ("hbm", (8.0 * lp + 4.0 * (2 * lp / max(rows, 1) + 1) * rows + 8.0 * rows) / 1e9, "GB/s",
                "8 B per pair increment (4-byte counter read + write) + 4 B per list entry + 8 B per row pointer")
    if kernel == "gram_mfma":
        nt = math.ceil(n / 128)
        macs = stats["n_word_rows"] * 64 * (nt * (nt + 1) // 2) * 128 * 128
        return "mfma", 2.0 * macs / 1e12, "TOP/s", "2 int8 ops per bit pair of every packed word pair (MACs x 2)"
    if kernel == "gram_fp4":
        nt = math.ceil(n / 128)
        macs = stats["n_word_rows"] * 64 * (nt * (nt + 1) // 2) * 128 * 128
        return ("mfma_fp4", 2.0 * macs / 1e12, "TFLOP/s",
                "2 fp4 flops per bit pair of every packed word pair (MACs x 2; each bit a 0/1 e2m1 value)")
    if kernel == "gram_popc":
        nt = math.ceil(n / 128)
        wp = stats["n_word_rows"] * (nt * (nt + 1) // 2) * 128 * 128
        return "alu", 4.0 * wp / 1e12, "TOP/s", "4 VALU lane-ops per 64-bit word pair (2 AND + 2 popcount-add)"
    return None


def kernel_label(name: str) -> str:
    """The timing label of a HIP kernel's name as rocprofv3 prints it
    (namespaces, template arguments and the parameter list around it)."""
    import re

    m = re.search(r"(?:^|::)(k_\w+)(?:<([^()]*)>)?(?:\(|$)", name)
    if m is None:
        return name.split("(")[0].split("::")[-1]
    base, tmpl = m.group(1)[2:], m.group(2) or ""
    if base == "radix_onesweep" and tmpl.startswith("unsigned int"):
        return "pair_sort"  # the same kernel on 32-bit pair words
    if base in ("gram_fp4_wide",):
        return "gram_fp4"
    if base in ("gram_mfma_wide",):
        return "gram_mfma"
    if base == "local_cls" and tmpl.startswith("unsigned long"):
        return "local_cls_wide"
    return base


def write_traffic(fetch_dir: str, write_dir: str, workload: str, copy_mib: int):
    """profiles/traffic.json entries of one workload from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, csv) of one bench step with no warm-up and the
    copy calibration: per kernel label, bytes per dispatch, each counter scaled
    by what it reads for the calibration copy of copy_mib MiB.  Prints a table."""
    import csv
    import glob

    def per_dispatch(d, counter):
        f = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
        out = {}
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            k = int(r["Dispatch_Id"])
            out.setdefault(k, [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
        return out

    fetch, write = per_dispatch(fetch_dir, "FETCH_SIZE"), per_dispatch(write_dir, "WRITE_SIZE")
    copy_bytes = copy_mib * 1024.0 * 1024.0
    cf = max(v for name, v in fetch.values() if "copyBuffer" in name) * 1024.0
    cw = max(v for name, v in write.values() if "copyBuffer" in name) * 1024.0
    ff, wf = copy_bytes / cf, copy_bytes / cw
    agg = {}
    for name, v in fetch.values():
        if "jas::" not in name:  # the calibration copy, torch's own kernels
            continue
        agg.setdefault(kernel_label(name), [0, 0.0, 0.0])
        a = agg[kernel_label(name)]
        a[0] += 1
        a[1] += v * 1024.0 * ff
    for name, v in write.values():
        if "jas::" not in name or kernel_label(name) not in agg:
            continue
        agg[kernel_label(name)][2] += v * 1024.0 * wf
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(tf)) if os.path.exists(tf) else {}
    rec = {k: v for k, v in rec.items() if not k.endswith(":" + workload)}
    print(f"| kernel | dispatches | read GB/dispatch | written GB/dispatch |  (fetch x {ff:.3f}, write x {wf:.3f})")
    print("|---|---|---|---|")
    for lab, (c, rd, wr) in sorted(agg.items(), key=lambda kv: -(kv[1][1] + kv[1][2]) / kv[1][0]):
        if (rd + wr) / c < 0.1e9:
            continue
        print(f"| {lab} | {c} | {rd / c / 1e9:.2f} | {wr / c / 1e9:.2f} |")
        rec[f"{lab}:{workload}"] = {"bytes_per_launch": round((rd + wr) / c / 1e9, 3), "unit": "GB",
                                    "read_GB": round(rd / c / 1e9, 3), "written_GB": round(wr / c / 1e9, 3),
                                    "source_hash": kernel_source_hash(lab), "fetch_factor": ff,
                                    "write_factor": wf}
    with open(tf, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


def cpu_baseline(spec, k: int, seed: int = 5):
    """The oracle timed on a bounded sample: k sets of the workload, all k(k+1)/2 pairs."""
    import numpy as np

    import oracle
    import synth
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(spec.n, size=min(k, spec.n), replace=False))
    ids, off = synth.generate_samples(spec, idx)
    t0 = time.perf_counter()
    s, so = oracle.normalize(ids, off)
    t1 = time.perf_counter()
    kk = idx.size
    iu, ju = np.triu_indices(kk)
    oracle.pairs_normalized(s, so, s, so, iu, ju)
    t2 = time.perf_counter()
    t_set = (t1 - t0) / kk
    t_pair = (t2 - t1) / iu.size
    n = spec.n
    full_pairs = n * (n + 1) // 2
    projected = full_pairs / (n * t_set + full_pairs * t_pair)
    return {"value": projected, "unit": "pairs/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": (f"{kk} of the {n} sets ({int(off[-1])} IDs), all {iu.size} pairs: set build "
                       f"{t1 - t0:.2f} s, pair merges {t2 - t1:.2f} s on {oracle.threads()} threads; value = "
                       f"n(n+1)/2 / (n * per-set + n(n+1)/2 * per-pair time) for the full n={n}")}


def run_serving(n_requests: int, n_saturation: int, n_warmup: int = 200, pool: int = 200, seed: int = 1):
    """Resident serving database (n=8192, U=36, 3.2e9 IDs); Poisson request stream at
    0.7 x the saturation rate measured by a closed pre-run; continuous batching over 4 slots
    within an 8 GiB HBM budget.  The requests cycle through `pool` seeded payloads (1-64
    query sets of 1e4-1e6 IDs each), so a long stream needs no more host memory than that."""
    import numpy as np
    import torch

    import synth
    from paper_1911_04200_amd import jas as cabi
    from paper_1911_04200_amd import serve

    spec = synth.workload("serving_db")
    off = synth.offsets(spec)
    N = int(off[-1])
    log(f"[serving] database n={spec.n} U={spec.universe_bits} N={N} ids")
    host = torch.empty(N, dtype=torch.int64, pin_memory=True)
    synth.generate(spec, out=host.numpy().view(np.uint64))
    ids_d = host.cuda()
    off_d = torch.from_numpy(off.view(np.int64)).cuda()
    del host
    torch.cuda.synchronize()
    opts = cabi.jas_encode_opts(spec.universe_bits, synth.BATCH_BITS["serving_db"], 0,
                                cabi.JAS_KEEP_IDS | cabi.JAS_QUERY_ONLY, 0)
    t = time.perf_counter()
    db, st = cabi.jas_encode(ids_d, off_d, spec.n, opts, None)
    enc_s = time.perf_counter() - t
    del ids_d
    torch.cuda.synchronize()
    log(f"[serving] encoded in {enc_s:.2f} s; generating requests")
    payload = serve.make_requests(spec, pool, seed=seed * 1000 + 3, first_id=300000, pinned=True)

    def stream_of(count, first):
        out = []
        for k in range(count):
            src = payload[(first + k) % pool]
            r = serve.Request(first + k, src.ids, src.offsets)
            r._payload = src
            out.append(r)
        return out

    warm = stream_of(n_warmup, 0)
    sat = stream_of(n_saturation, n_warmup)
    reqs = stream_of(n_requests, n_warmup + n_saturation)
    server = serve.Server(db, slots=4, budget_bytes=8 << 30, max_batch_sets=64, keep_results=False)
    arr_w = serve.poisson_arrivals(len(warm), 200.0, seed + 7)
    server.run(warm, arr_w)
    log(f"[serving] {len(warm)} warm-up requests done")
    t = time.perf_counter()
    server.run(sat)
    sat_rate = len(sat) / (time.perf_counter() - t)
    rate = 0.7 * sat_rate
    arrivals = serve.poisson_arrivals(len(reqs), rate, seed)
    log(f"[serving] saturation {sat_rate:.1f} req/s; Poisson stream at {rate:.1f} req/s")
    t = time.perf_counter()
    server.run(reqs, arrivals)
    wall = time.perf_counter() - t
    out = serve.summarize(reqs, spec.n, wall)
    out.update({"workload": f"serving_n{spec.n}_u{spec.universe_bits}", "db_ids": N,
                "db_encode_s": enc_s, "db_device_bytes": st["device_bytes"], "saturation_requests_per_s": sat_rate,
                "offered_requests_per_s": rate, "slots": 4, "hbm_budget_bytes": 8 << 30, "max_batch_sets": 64,
                "warmup_requests": len(warm), "saturation_requests": len(sat), "distinct_payloads": pool,
                "latency": "completion - Poisson arrival (host arrays in and out, queueing included)"})
    db.close()
    cabi.jas_trim()
    return out


def run_kmers(args):
    """The k-mer front end alone: 2-bit packed genomes resident in HBM -> the
    samples' canonical 31-mer IDs; prints one JSON line (bases per second)."""
    import numpy as np
    import torch

    import synth
    from paper_1911_04200_amd import jas as cabi

    n, length, k = 128, 1 << 22, 31
    samples = synth.random_genomes(n, length, n_refs=16, mutation=0.01, seqs_per_sample=4, seed=3)
    seqs = [s for smp in samples for s in smp]
    words, seq_off = synth.pack_2bit(seqs)
    smp_off = np.arange(0, 4 * n + 1, 4, dtype=np.uint64)
    ids_off = cabi.jas_kmer_offsets(seq_off, smp_off, k)
    torch.cuda.set_device(0)
    w = torch.from_numpy(words.view(np.int64)).cuda()
    ids = torch.empty(int(ids_off[-1]), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        cabi.jas_kmers(w, seq_off, k, cabi.JAS_CANONICAL, None, ids)
    cabi.jas_timing_enable(True)
    cabi.jas_timing_report()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cabi.jas_kmers(w, seq_off, k, cabi.JAS_CANONICAL, None, ids)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = cabi.jas_timing_report()
    cabi.jas_timing_enable(False)
    bases = int(seq_off[-1])
    sec = (t1 - t0) / args.steps
    c, ms = kt.get("kmers", (0, 0.0))
    launch_s = ms / max(c, 1) / 1e3
    traffic = bases / 4 + 8 * int(ids_off[-1])  # packed bases read once, IDs written
    print(json.dumps({"metric": "bases/s (canonical k-mer IDs, k = 31)", "value": bases / sec, "unit": "bases/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                      "data": "synthetic genomes (seeded, synth.random_genomes)",
                      "config": {"workload": f"kmers_n{n}_len{length}_k{k}", "bases": bases, "kmers": int(ids_off[-1])},
                      "roofline": {"kernel": "kmers", "bound": "hbm", "achieved": traffic / launch_s / 1e9,
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": traffic / launch_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
                                   "per_launch": "packed bases read (2 bits each) + 8 B per k-mer written",
                                   "avg_launch_ms": ms / max(c, 1)}}), flush=True)


def run_streamed(args):
    """The all-pairs step with the sets in host memory, streamed part by part
    (paper_1911_04200_amd.stream); prints one JSON line."""
    import numpy as np
    import torch

    import synth
    from paper_1911_04200_amd import jas as cabi
    from paper_1911_04200_amd import stream

    if args.workload not in synth.BERNOULLI:
        print(json.dumps({"error": "streaming needs ascending sets: use a bernoulli_p* workload"}))
        sys.exit(2)
    spec = synth.workload(args.workload)
    n, U, K = spec.n, spec.universe_bits, args.stream_part_bits
    t = time.perf_counter()
    ids, off = synth.generate(spec)
    bounds = stream.plan_parts(ids, off, U, K, check_sorted=False)
    log(f"[bench] {args.workload}: N={ids.size} ids in host memory, {1 << K} parts "
        f"({time.perf_counter() - t:.1f} s to generate and plan)")
    torch.cuda.set_device(0)

    def step():
        gf = cabi.JAS_GRAM_VARIANT(args.gram_variant) if args.gram_variant >= 0 else 0
        res = stream.all_pairs_streamed(ids, off, U, K, batch_bits=synth.BATCH_BITS[args.workload],
                                        dense_min_degree=args.dmin, upper=args.upper, bounds=bounds, gram_flags=gf)
        torch.cuda.synchronize()
        return res

    for w in range(args.warmup):
        step()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    cabi.jas_timing_enable(True)
    cabi.jas_timing_report()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    t1 = time.perf_counter()
    kt = cabi.jas_timing_report()
    cabi.jas_timing_enable(False)
    sec = (t1 - t0) / args.steps
    pairs = n * (n + 1) // 2
    kernels = {k: {"launches": c, "ms_per_step": ms / args.steps} for k, (c, ms) in kt.items()
               if not k.startswith("host:")}
    parts = res["parts"]
    out = {"metric": "sample-pair intersections/s (exact B, C, J of all pairs i <= j)", "value": pairs / sec,
           "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64 keys / i32 counts / f64 J", "data": "synthetic (seeded counter-based generator, synth/)",
           "config": {"workload": f"{args.workload}_n{n}_u{U}_streamed", "n": n, "universe_bits": U, "ids": int(ids.size),
                      "parts": 1 << K, "gram_variant": args.gram_variant,
                      "inputs": "host memory; gather into page-locked staging and host-to-device "
                      "copies inside the timed region", "layout": "upper" if args.upper else "full"},
           "roofline": None, "cpu_baseline": None,
           "detail": {"host_gather_s_per_step": res["host_gather_s"], "max_part_ids": res["max_part_ids"],
                      "max_part_encoding_bytes": max(p["device_bytes"] for p in parts),
                      "dense_min_degree": sorted(set(p["dense_min_degree"] for p in parts)),
                      "kernels": kernels}}
    print(json.dumps(out), flush=True)


def time_captured(args, ids_d, off_d, n, opts, flags, B, card, den, J, eager_ms):
    """The same step as one HIP graph: an encode plan made from these inputs,
    then plan encode + Gram + finalize captured once and replayed.  The
    replay's outputs are compared with the eager step's (left in B, den, J)."""
    import torch

    from paper_1911_04200_amd import jas as cabi

    torch.cuda.synchronize()
    ref = {"B": B.clone(), "den": den.clone(), "J": J.clone(), "card": card.clone()}
    t = time.perf_counter()
    plan = cabi.jas_plan_create(ids_d, off_d, n, opts, headroom=args.plan_headroom)
    create_s = time.perf_counter() - t
    db = plan.db
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # eager once on the plan's db: tunes the Gram tiles for its shape
        cabi.jas_plan_encode(plan, ids_d, off_d, s)
        cabi.jas_gram(db, flags | (cabi.JAS_TUNE if args.path == "auto" else 0), s, B, card, den, J)
    s.synchronize()
    cabi.jas_plan_check(plan, s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cabi.jas_plan_encode(plan, ids_d, off_d, s)
        cabi.jas_gram(db, flags, s, B, card, den, J)
    for w in range(args.warmup):
        g.replay()
        torch.cuda.synchronize()
    log("[bench] captured step: graph built and warmed up")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = cabi.jas_plan_check(plan, s)
    same = all(torch.equal(ref[k], v) for k, v in (("B", B), ("den", den), ("J", J), ("card", card)))
    log(f"[bench] {args.steps} captured steps done (outputs equal to the eager step's: {same})")
    del g
    plan.close()
    ms = (t1 - t0) / args.steps * 1e3
    pairs = n * (n + 1) // 2
    return {"ms_per_step": ms, "value": pairs / (ms / 1e3), "unit": "pairs/s", "eager_ms_per_step": eager_ms,
            "speedup_vs_eager": eager_ms / ms, "outputs_equal_eager": same, "plan_headroom": args.plan_headroom,
            "plan_create_s": create_s, "dense_min_degree": st["dense_min_degree"]}


def run_occupancy(workloads):
    """How much of the dense tile work a skip of empty blocks could save: the
    full-size encoding's words read back, per (K block of word rows x 128
    columns) whether any word is nonzero, and the executed word pairs of a Gram
    that skipped the empty blocks, over F; also with the word rows and the
    columns reordered by their nonzero counts, and with the columns grouped by
    the generator's cluster (known to the generator only).  One line per case."""
    import numpy as np
    import torch

    import synth
    from paper_1911_04200_amd import jas as cabi

    def skip_cost(nzm, n, nt, KB, T=128):
        nk = math.ceil(nzm.shape[0] / KB)
        m = torch.nn.functional.pad(nzm.to(torch.uint8), (0, nt * T - n, 0, nk * KB - nzm.shape[0]))
        occ = m.view(nk, KB, nt, T).amax(dim=(1, 3)).to(torch.float64)
        s = occ.sum(dim=1)
        both = (s * s + s) / 2  # tile pairs I <= J with both blocks occupied (o in {0, 1})
        return 1.0 - float(occ.mean()), float(both.sum()) * KB * T * T

    out = {}
    for name in workloads:
        spec = synth.workload(name)
        n = spec.n
        off = synth.offsets(spec)
        N = int(off[-1])
        host = torch.empty(N, dtype=torch.int64, pin_memory=True)
        synth.generate(spec, out=host.numpy().view(np.uint64))
        ids = host.cuda()
        offd = torch.from_numpy(off.view(np.int64)).cuda()
        del host
        db, st = cabi.jas_encode(ids, offd, n, cabi.jas_encode_opts(spec.universe_bits, synth.BATCH_BITS[name], 0, 0, 0),
                                 None)
        del ids
        H, stride = st["w_rows"], st["w_stride"]
        rec = {"n": n, "word_rows": H, "threshold": st["dense_min_degree"]}
        if H == 0:
            db.close()
            out[name] = rec
            continue
        W = torch.from_numpy(cabi.jas_db_read(db, cabi.JAS_DB_WORDS).view(np.int64)).cuda().view(H, stride)[:, :n]
        db.close()
        nz = W != 0
        del W
        z = nz.sum(dim=1, dtype=torch.int64)
        F = int((z * (z + 1) // 2).sum())
        nt = math.ceil(n / 128)
        dense = H * (nt * (nt + 1) // 2) * 128 * 128
        rec.update({"density": float(z.sum()) / (H * n), "F": F, "W_over_F": dense / F})
        colw = nz.sum(dim=0)
        cl = torch.tensor([synth.plan(spec, i)[3] for i in range(n)], device=nz.device)
        orders = {"stored": nz,
                  "rows and columns by nonzero count": nz[torch.argsort(z, descending=True)][:, torch.argsort(colw, descending=True)],
                  "columns by cluster, rows by count": nz[torch.argsort(z, descending=True)][:, torch.argsort(cl * (n + 1) + (n - colw.clamp(max=n)), stable=True)]}
        for oname, m in orders.items():
            for KB in (4, 16, 64):
                e, ws = skip_cost(m, n, nt, KB)
                rec[f"{oname}, {KB} rows"] = {"empty_blocks": e, "W_skip_over_F": ws / F}
        del nz, orders
        torch.cuda.empty_cache()
        cabi.jas_trim()
        out[name] = rec
        log(f"[occupancy] {name}: {json.dumps(rec)}")
    print(json.dumps({"occupancy": out}), flush=True)


def run_all_pairs(args, workload: str, upper: bool):
    """Time the all-pairs step (encode + Gram, inputs resident in HBM) on one
    full-size workload: (summary dict, encode stats, spec, N)."""
    import numpy as np
    import torch

    import synth
    from paper_1911_04200_amd import jas as cabi

    spec = synth.workload(workload)
    bb = synth.BATCH_BITS[workload]
    n = spec.n
    off = synth.offsets(spec)
    N = int(off[-1])
    log(f"[bench] workload {workload}: n={n} U={spec.universe_bits} N={N} ids, batch 2^{bb}")
    t = time.perf_counter()
    host = torch.empty(N, dtype=torch.int64, pin_memory=True)
    ids_np = host.numpy().view(np.uint64)
    synth.generate(spec, out=ids_np)
    log(f"[bench] generated in {time.perf_counter() - t:.1f} s")
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    ids_d = host.to(dev, non_blocking=False)
    off_d = torch.from_numpy(off.view(np.int64)).to(dev)
    del host, ids_np
    torch.cuda.synchronize()
    log("[bench] inputs resident in HBM")

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 17, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration} MiB done")
        del src, dst

    stream = torch.cuda.current_stream()
    length = n * (n + 1) // 2 if upper else n * n
    B = torch.empty(length, dtype=torch.int32, device=dev)
    card = torch.empty(n, dtype=torch.int64, device=dev)
    den = torch.empty(length, dtype=torch.int64, device=dev)
    J = torch.empty(length, dtype=torch.float64, device=dev)
    opts = cabi.jas_encode_opts(spec.universe_bits, bb, args.dmin, 0, 0)
    flags = cabi.JAS_UPPER if upper else 0
    flags |= {"auto": 0, "popcount": cabi.JAS_FORCE_POPCOUNT, "mfma": cabi.JAS_FORCE_MFMA}[args.path]

    def step(extra_flags=0):
        db, st = cabi.jas_encode(ids_d, off_d, n, opts, stream)
        cabi.jas_gram(db, flags | extra_flags, stream, B, card, den, J)
        db.close()
        return st

    # the Gram tile autotuner runs once, in the first warm-up step, timed apart
    tune_ms = None
    for w in range(args.warmup):
        if w == 0 and args.path == "auto":
            cabi.jas_timing_enable(True)
            cabi.jas_timing_report()
            st = step(cabi.JAS_TUNE)
            torch.cuda.synchronize()
            tune_ms = cabi.jas_timing_report().get("host:gram_tune", (0, None))[1]
            cabi.jas_timing_enable(False)
        else:
            st = step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    if args.timing:
        cabi.jas_timing_enable(True)
        cabi.jas_timing_report()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = cabi.jas_timing_report() if args.timing else {}
    cabi.jas_timing_enable(False)
    log(f"[bench] {args.steps} timed steps done")
    sec = (t1 - t0) / args.steps
    pairs = n * (n + 1) // 2
    value = pairs / sec

    # the dominant kernel and its roofline
    roof = None
    passes = math.ceil(spec.universe_bits / 8)
    kernels = {name: {"launches": c, "ms_per_step": ms / args.steps, "ms_per_launch": ms / max(c, 1)}
               for name, (c, ms) in kt.items() if not name.startswith("host:")}
    host_phases = {name[5:]: {"calls": c, "ms_per_step": ms / args.steps}
                   for name, (c, ms) in kt.items() if name.startswith("host:")}
    kt = {k: v for k, v in kt.items() if not k.startswith("host:")}
    if kt:
        dom = max(kt.items(), key=lambda kv: kv[1][1])[0]
        c, ms = kt[dom]
        alg = algorithmic(dom, st, n, N, passes)
        if alg:
            bound, amount, unit, desc = alg
            avg_s = ms / c / 1e3
            achieved = amount / avg_s
            peak = {"hbm": HBM_PEAK_GBS, "alu": VALU_PEAK_TOPS, "mfma": MFMA_I8_PEAK_TOPS,
                    "mfma_fp4": MFMA_FP4_PEAK_TOPS}[bound]
            if bound == "mfma_fp4":
                bound = "mfma"  # against the fp4 peak
            traffic = None
            tf = os.path.join(ROOT, "profiles", "traffic.json")
            if os.path.exists(tf):
                rec = json.load(open(tf)).get(f"{dom}:{workload}")
                if rec and rec.get("source_hash") == kernel_source_hash(dom):
                    traffic = rec.get("bytes_per_launch")
            roof = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                    "frac": achieved / peak, "traffic": traffic, "per_launch": desc,
                    "avg_launch_ms": ms / c}
    # word-pair rates of the popcount Gram
    gram_ms = (kt.get("gram_popc", (0, 0.0))[1] + kt.get("gram_mfma", (0, 0.0))[1] +
               kt.get("gram_fp4", (0, 0.0))[1]) / max(args.steps, 1)
    executed = st["word_pairs_W"]  # whole 128 x 128 tiles over every stored word row
    extra = {"gram_ms": gram_ms, "gram_autotune_ms": tune_ms,
             "word_pairs_W_over_F": (executed / st["word_pairs_F"]) if st["word_pairs_F"] else None,
             "G_bit_ANDs_per_s_executed": (64.0 * executed / (gram_ms / 1e3) / 1e9) if gram_ms else None,
             "G_bit_ANDs_per_s_algorithmic_F": (64.0 * st["word_pairs_F"] / (gram_ms / 1e3) / 1e9) if gram_ms
             else None,
             "encode_stats": st, "kernels": kernels, "host_phases": host_phases}

    captured = None
    if workload == "batching" and args.captured:
        try:
            captured = time_captured(args, ids_d, off_d, n, opts, flags, B, card, den, J, sec * 1e3)
        except Exception as e:  # reported, not fatal to the eager line
            captured = {"error": repr(e)}
    extra["captured"] = captured

    del ids_d, B, den, J
    cabi.jas_trim()
    summary = {"value": value, "unit": "pairs/s", "ms_per_step": sec * 1e3, "steps": args.steps,
               "config": {"workload": f"{workload}_n{n}_u{spec.universe_bits}", "n": n,
                          "universe_bits": spec.universe_bits, "batch_rows": f"2^{bb}", "ids": N,
                          "pairs_per_step": pairs, "layout": "upper" if upper else "full",
                          "dense_min_degree": args.dmin},
               "roofline": roof, "detail": extra}
    return summary, st, spec, N


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="paperlike",
                    choices=["tiny", "paperlike", "precision", "batching", "bernoulli_p1e-4", "bernoulli_p1e-3",
                             "bernoulli_p1e-2", "bernoulli_p1e-1", "graph_s13_ef64"],
                    help="bernoulli_p*: the paper's synthetic matrices (each entry 1 with probability p); "
                         "graph_*: neighbourhoods of an R-MAT graph (vertex similarity)")
    ap.add_argument("--dmin", type=int, default=0, help="dense_min_degree (0: library default)")
    ap.add_argument("--upper", action="store_true", help="packed upper-triangle outputs")
    ap.add_argument("--path", default="auto", choices=["auto", "popcount", "mfma"], help="Gram path for packed tiles")
    ap.add_argument("--cpu-sample", type=int, default=192, help="sets in the oracle's timed sample (0: skip)")
    ap.add_argument("--timing", type=int, default=1, help="per-kernel HIP-event timing in the timed region")
    ap.add_argument("--extra-configs", type=int, default=1,
                    help="with the paperlike workload: also time the precision and batching forms (0: skip)")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests in the timed Poisson serving run (0: no serving run)")
    ap.add_argument("--serving-saturation", type=int, default=200, help="requests in the closed saturation run")
    ap.add_argument("--stream-part-bits", type=int, default=0,
                    help="K > 0: keep the sets in host memory and stream them in 2^K ID-range parts "
                         "(Bernoulli workloads, whose sets are ascending); host-to-device copies are timed")
    ap.add_argument("--gram-variant", type=int, default=-1,
                    help="with --stream-part-bits: run MFMA tile variant V for every part (default: the library's)")
    ap.add_argument("--kmer-front-end", action="store_true",
                    help="time the GPU k-mer front end instead (128 genomes of 4 Mbases, k = 31, canonical): "
                         "bases/s, inputs resident in HBM")
    ap.add_argument("--occupancy", nargs="+", metavar="WORKLOAD",
                    help="report the packed words' block occupancy of these full-size workloads (no timing)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving stream (--serving-requests after the warm-up and saturation runs)")
    ap.add_argument("--captured", type=int, default=1,
                    help="batching form: also time the step as one replayed HIP graph through an encode plan")
    ap.add_argument("--plan-headroom", type=float, default=0.05, help="capacity headroom of that plan")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU: write profiles/traffic.json entries of --workload from two rocprofv3 --pmc csv "
                         "runs (FETCH_SIZE, WRITE_SIZE) of one step with --warmup 0 and --copy-calibration")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB copied device-to-device before the steps: a plain copy of known size that scales "
                         "the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.workload, args.copy_calibration or 4096)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1911_04200_amd import jas as cabi

    if args.occupancy:
        run_occupancy(args.occupancy)
        return
    if args.serving_only:
        out = run_serving(args.serving_requests, args.serving_saturation)
        print(json.dumps({"metric": "serving requests/s (resident db, Poisson arrivals)",
                          "value": out["requests_per_s"], "unit": "requests/s", "n_gpus": 1,
                          "higher_is_better": True, "data": "synthetic (seeded counter-based generator, synth/)",
                          "serving": out}), flush=True)
        return
    if args.stream_part_bits > 0:
        run_streamed(args)
        return
    if args.kmer_front_end:
        run_kmers(args)
        return
    upper = args.upper or args.workload == "batching"  # the batching form returns the upper triangle only
    main_res, st, spec, N = run_all_pairs(args, args.workload, upper)
    others = {}
    if args.workload == "paperlike" and args.extra_configs:
        # the precision and batching forms, timed the same way (their own dominant kernels)
        for name in ("precision", "batching"):
            try:
                r, _, _, _ = run_all_pairs(args, name, name == "batching")
                r["detail"] = {k: r["detail"][k] for k in ("gram_ms", "gram_autotune_ms", "encode_stats", "captured")} | {
                    "kernels": {k: v for k, v in r["detail"]["kernels"].items() if v["ms_per_step"] >= 0.5}}
                others[name] = r
            except Exception as e:  # reported, not fatal to the main line
                others[name] = {"error": repr(e)}
    serving = None
    if args.serving_requests > 0:
        try:
            serving = run_serving(args.serving_requests, args.serving_saturation)
        except Exception as e:  # reported, not fatal to the all-pairs line
            serving = {"error": repr(e)}

    cpu = None
    if args.cpu_sample > 0:
        log("[bench] timing the oracle on a sample")
        cpu = cpu_baseline(spec, args.cpu_sample)

    out = {"metric": "sample-pair intersections/s (exact B, C, J of all pairs i <= j)",
           "value": main_res["value"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": main_res["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": ("exact integers: u64 keys, i32 B, i64 C; packed Gram on fp4 (e2m1 0/1) MFMA operands with "
                     "f32 sums kept below 2^24 (exact); f64 J"),
           "data": "synthetic (seeded counter-based generator, synth/)",
           "config": main_res["config"], "roofline": main_res["roofline"], "cpu_baseline": cpu,
           "precision": others.get("precision"), "batching": others.get("batching"), "serving": serving,
           "detail": main_res["detail"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
