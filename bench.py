#!/usr/bin/env python
"""Throughput of the sparse polynomial product on one MI355X.

Workload (default): the large sparse 5-variable product
    f = (1+x+y+2z^2+3t^3+5u^5)^12,  g = (1+u+t+2z^2+3y^3+5x^5)^12
(6188 terms each, 38,291,344 term products -> 5,821,335 terms), exponents
packed 12 bits per variable, coefficients mod 2^61-1.  A step is one whole
pm_mul (validation, key compression, LDS tile combine, radix passes,
segmented reduction) with the operands resident in HBM, ending with the
result count read back.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sparse5_n12_modp_hbm_traffic.json")


KERNEL_SOURCES = ["pm_kernels.hip", "pm_bkt.hpp", "pm_ival.hpp", "pm_internal.hpp", "pm_plan.cpp", "pm_plan.hpp"]


def kernel_source_hash():
    """Hash of the sources that decide the product's kernels and launches."""
    import hashlib
    d = os.path.join(ROOT, "paper_1303_7425_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


def _traffic_profile():
    try:
        prof = json.load(open(TRAFFIC_PROFILE))
    except (OSError, ValueError):
        return None
    return prof if prof.get("kernel_source_sha256_16") == kernel_source_hash() else None


def measured_traffic(label):
    """Scaled rocprofv3 FETCH_SIZE + WRITE_SIZE bytes per launch of `label`,
    or None when the kernels changed since the counters were taken."""
    prof = _traffic_profile()
    e = None if prof is None else prof["per_launch"].get(label)
    return None if e is None else e["fetch_bytes"] + e["write_bytes"]


def measured_step_traffic():
    """Scaled counter bytes (read + write) of all the path's kernels per
    product, or None when the kernels changed since the counters were taken."""
    prof = _traffic_profile()
    if prof is None or not prof.get("steps"):
        return None
    return sum((e["fetch_bytes"] + e["write_bytes"]) * e["launches"] for e in prof["per_launch"].values()) / prof["steps"]


# rocprofv3 kernel names -> the labels used in the summaries
KERNEL_LABELS = [
    ("k_bk_count", "bk_count (fine-bin counts)"),
    ("k_bk_cut", "bk_cut (greedy cut into work items)"),
    ("k_bk_scan", "bk_scan"),
    ("k_bk_winfo", "bk_winfo"),
    ("k_bk_scatter", "bk_scatter (pair indices to work items)"),
    ("k_bk_reduce<", "bk_reduce (per-work-item LDS sum)"),
    ("k_bk_oscan", "bk_oscan"),
    ("k_bk_copy", "bk_copy (result placement)"),
    ("k_onesweep<unsigned int, unsigned int, 2, false, true>", "onesweep pass (pair indices)"),
    ("k_onesweep<unsigned int, unsigned int, 2, false, false>", "onesweep pass (pair indices, keys via cache)"),
    ("k_onesweep<unsigned int, unsigned int, 2, true, true>", "onesweep last pass (pair indices, writes keys)"),
    ("k_onesweep<unsigned int, unsigned int, 2, true, false>", "onesweep last pass (keys via cache)"),
    ("k_onesweep<unsigned int, unsigned int, 1, false, true>", "onesweep pass 0 (generates pair indices)"),
    ("k_onesweep<unsigned int, unsigned int, 1, true, true>", "onesweep single pass (generates, writes keys)"),
    ("k_onesweep<unsigned int, unsigned int, 1, true, false>", "onesweep pass 0 (generates, writes keys)"),
    ("k_onesweep<unsigned int, unsigned int, 0, true, false>", "onesweep pass (keys and pair indices)"),
    ("k_count<unsigned int, 2,", "count (pair indices)"),
    ("k_count<unsigned int, 1,", "count (generated pair indices)"),
    ("k_count<unsigned int, 0,", "count (staged keys)"),
    ("k_range_scan", "range_scan"),
    ("k_head_count<", "head_count"),
    ("k_head_scan", "head_scan"),
    ("k_reduce<", "reduce"),
    ("k_zero_compact<", "zero_compact"),
    ("k_seg_prepare", "seg_prepare"),
    ("k_stats", "stats"),
    ("k_compress<", "compress"),
    ("k_fill", "fill"),
]


def kernel_label(name):
    for key, label in KERNEL_LABELS:
        if key in name:
            return label
    return None


def traffic_summary(fetch_csv, write_csv, out_path=None, workload="sparse 5-var n=12 mod p", steps=None):
    """rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE counter CSVs of a
    `bench.py --copy-calibration` run -> per-launch HBM bytes, each counter
    scaled by what it reads for the 512 MiB calibration copies; writes the
    JSON that the roofline's `traffic` field is taken from and prints a table."""
    import csv
    import hashlib
    from collections import defaultdict

    def load(path, counter):
        per = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                per[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
        return per

    fe, wr = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    cal = float(1 << 29)
    fetch_scale = cal / max(v for k, vs in fe.items() if "copyBuffer" in k for v in vs)
    write_scale = cal / max(v for k, vs in wr.items() if "copyBuffer" in k for v in vs)
    per = {}
    for name, vs in fe.items():
        label = kernel_label(name)
        if label is None or name not in wr:
            continue
        per[label] = {"fetch_bytes": sum(vs) / len(vs) * fetch_scale,
                      "write_bytes": sum(wr[name]) / len(wr[name]) * write_scale, "launches": len(vs)}
    # products in the profiled run: launches of a kernel that runs once per
    # product (the statistics kernel also runs for the bound query)
    once = ("bk_reduce (per-work-item LDS sum)", "zero_compact", "compact")
    nsteps = steps or next((per[k]["launches"] for k in once if k in per), None)
    out = {"kernel_source_sha256_16": kernel_source_hash(),
           "workload": workload, "fetch_scale": fetch_scale, "write_scale": write_scale,
           "steps": nsteps, "per_launch": per}
    with open(out_path or TRAFFIC_PROFILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"fetch scale {fetch_scale:.4f}, write scale {write_scale:.4f}, kernel source {out['kernel_source_sha256_16']}, "
          f"{nsteps} products profiled")
    if nsteps:
        tot = sum((e["fetch_bytes"] + e["write_bytes"]) * e["launches"] for e in per.values()) / nsteps
        print(f"all kernels, per product: {tot / 1e6:.1f} MB read + written")
    print("| kernel | launches | read MB (scaled) | write MB (scaled) |")
    print("|---|---|---|---|")
    for label, e in sorted(per.items(), key=lambda kv: -(kv[1]["fetch_bytes"] + kv[1]["write_bytes"])):
        print(f"| {label} | {e['launches']} | {e['fetch_bytes'] / 1e6:.1f} | {e['write_bytes'] / 1e6:.1f} |")


def trace_summary(stats_csv):
    """rocprofv3 --kernel-trace --stats kernel_stats.csv -> markdown table."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print("| kernel | calls | average us | share of GPU time |")
    print("|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        print(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{100.0 * float(r['TotalDurationNs']) / tot:.1f}% |")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ring", default="modp", choices=["modp", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--workload", default="sparse", choices=["sparse", "batch", "serve", "drain", "dense"],
                    help="sparse: the large sparse product (default JSON line); batch: the 4096-product "
                         "batched workload, batched graph launches vs per-product calls; serve: Poisson "
                         "arrivals through the continuous-batching server; drain: batched products in "
                         "waves with results copied to host memory while the next wave runs; dense: the "
                         "degree-box products (dense n=10 int64, n=20 mod p, Example 1 n=40 mod p) against "
                         "the measured ceiling of their inner loop")
    ap.add_argument("--dense-cases", default="",
                    help="--workload dense: comma-separated case numbers to run (default: all; 5 and 6 are "
                         "the paper's Examples 3 and 2)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="tile shape of the LDS-combine and degree-box paths (-1 automatic, 0: 32x64, 1: 64x64, "
                         "2: 128x128)")
    ap.add_argument("--combine", type=int, default=-1,
                    help="sparse path mode for the sparse workload (-1 automatic, 0 pair-index radix sort, "
                         "1 LDS tile combine, 2 output-key intervals, 3 output-key work items)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy 512 MiB three times (counter scaling for HBM traffic)")
    ap.add_argument("--traffic-summary", nargs="+", metavar="CSV",
                    help="FETCH_CSV WRITE_CSV [OUT_JSON]: summarize rocprofv3 FETCH_SIZE / WRITE_SIZE counter CSVs "
                         "(no GPU needed); OUT_JSON defaults to the default workload's traffic profile")
    ap.add_argument("--trace-summary", metavar="KERNEL_STATS_CSV",
                    help="summarize a rocprofv3 --stats kernel_stats.csv (no GPU needed)")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--wave-gib", type=float, default=96.0, help="HBM per memory wave (outputs + workspace)")
    ap.add_argument("--batch-rings", default="both", choices=["both", "one"],
                    help="batch workload: mod p and FP64, or --ring only")
    ap.add_argument("--drain-products", type=int, default=512, help="first products of the batched workload")
    ap.add_argument("--drain-device-gib", type=float, default=64.0)
    ap.add_argument("--drain-host-gib", type=float, default=16.0)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.5, help="arrival rate as a fraction of saturation")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bench_batch(args):
    """Batched workload, like for like: every product of every memory wave is
    timed on its own (no extrapolation) in two pairings with the same
    validation policy on both sides:
      validated  one pm_mul_batch per wave        vs one pm_mul per product
      prepared   one HIP-graph replay per wave    vs one prepared single-product
                                                    graph replay per product
    The autotuner runs first on one product of each size class.  Mod p and
    FP64 (--batch-rings both)."""
    import math

    import numpy as np
    import torch

    from paper_1303_7425_amd import polymul as pm
    from paper_1303_7425_amd import workloads as W

    rings = ["modp", "f64"] if args.batch_rings == "both" else [args.ring]
    out = {}
    for ring in rings:
        sizes, rng = W.config4_sizes(count=args.batch_count)
        log(f"[batch] {ring}: generating {len(sizes)} pairs")
        fs, gs = [], []
        for na, nb in sizes.tolist():
            fs.append(pm.to_device(W.random_sparse(rng, int(na), 6, 10, 15, ring)))
            gs.append(pm.to_device(W.random_sparse(rng, int(nb), 6, 10, 15, ring)))
        lay = (6, 10, ring)
        total_pairs = int((sizes[:, 0] * sizes[:, 1]).sum())
        ws = pm.Workspace()
        # autotuner: the first product of each size class (floor(log2(pairs)))
        pm.autotune_reset()
        tuned = {}
        for q, (na, nb) in enumerate(sizes.tolist()):
            c = int(math.log2(na * nb))
            if c not in tuned:
                tuned[c] = pm.autotune(lay, fs[q], gs[q], ws)
        log(f"[batch] {ring}: autotuned {len(tuned)} size classes")
        # memory waves: bound-sized outputs (16 B/term) + workspace (about 24 B/pair)
        budget = args.wave_gib * (1 << 30)
        waves, cur, acc = [], [], 0.0
        for q, (na, nb) in enumerate(sizes.tolist()):
            need = na * nb * 40.0
            if cur and acc + need > budget:
                waves.append(cur)
                cur, acc = [], 0.0
            cur.append(q)
            acc += need
        if cur:
            waves.append(cur)
        t = {"batch_validated": 0.0, "single_validated": 0.0, "batch_graph": 0.0, "single_graph": 0.0}
        n_terms = 0

        def timed(fn):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        for w, idx in enumerate(waves):
            call = pm.BatchCall(lay, [fs[q] for q in idx], [gs[q] for q in idx], ws)
            call.run()
            t["batch_validated"] += timed(call.run)
            call.prepare_graph()
            call.launch_graph()
            t["batch_graph"] += timed(call.launch_graph)
            n_terms += int(call.out_n.sum().item())
            assert pm.last_call_status() == 0
            del call
            for q in idx:
                c = pm.MulCall(lay, fs[q], gs[q], ws)
                c.run()
                t["single_validated"] += timed(c.run)
                del c
                b = pm.BatchCall(lay, [fs[q]], [gs[q]], ws)
                b.prepare_graph()
                b.launch_graph()
                t["single_graph"] += timed(b.launch_graph)
                del b
            log(f"[batch] {ring} wave {w}: {len(idx)} products, {t}")
        out[ring] = {
            "term_products": total_pairs, "output_terms": n_terms, "waves": len(waves),
            "validated": {"batched_s": t["batch_validated"], "per_product_s": t["single_validated"],
                          "speedup": t["single_validated"] / t["batch_validated"]},
            "prepared": {"batched_graph_s": t["batch_graph"], "per_product_graph_s": t["single_graph"],
                         "speedup": t["single_graph"] / t["batch_graph"]},
            "autotuned_classes": {str(k): list(v) for k, v in sorted(tuned.items())},
        }
        del fs, gs, ws
        torch.cuda.empty_cache()
    main = out[rings[0]]
    return {
        "metric": "term-products/s (batched, prepared graph)", "value": main["term_products"] / main["prepared"]["batched_graph_s"],
        "unit": "term-products/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "u64" if rings[0] == "modp" else "f64", "data": "synthetic",
        "config": {"workload": f"{args.batch_count} random sparse 6-var products, 10 bits/var, exponents 0..15, "
                               "term counts log-uniform in [50, 20000], seed 4"},
        "rings": out,
    }


def bench_drain(args):
    """Batched products drained to pinned host memory wave by wave while the
    next wave runs (pm_mul_batch_drain), against the same waves computed with
    results left in HBM and against the D2H copy of the same bytes alone."""
    import numpy as np
    import torch

    from paper_1303_7425_amd import polymul as pm
    from paper_1303_7425_amd import workloads as W

    ring = args.ring
    sizes, rng = W.config4_sizes()
    sizes = sizes[:args.drain_products]
    log(f"[drain] generating {len(sizes)} pairs")
    fs, gs = [], []
    for na, nb in sizes.tolist():
        fs.append(pm.to_device(W.random_sparse(rng, int(na), 6, 10, 15, ring)))
        gs.append(pm.to_device(W.random_sparse(rng, int(nb), 6, 10, 15, ring)))
    pairs = int((sizes[:, 0] * sizes[:, 1]).sum())
    lay = (6, 10, ring)
    terms = [0]
    checksum = [0]

    def on_result(k, keys, coefs):
        terms[0] += keys.size
        if keys.size:
            checksum[0] ^= int(keys[-1])     # touch the drained data (last key of each result)

    dev_bytes = int(args.drain_device_gib * (1 << 30))
    host_bytes = int(args.drain_host_gib * (1 << 30))
    pm.mul_batch_drain(lay, fs[:8], gs[:8], on_result, dev_bytes, host_bytes)   # warm-up
    terms[0] = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    waves = pm.mul_batch_drain(lay, fs, gs, on_result, dev_bytes, host_bytes)
    t_drain = time.perf_counter() - t0
    drained_bytes = 16 * terms[0]
    log(f"[drain] {waves} waves, {terms[0]} terms, {t_drain:.3f} s")
    # the same products with results left in HBM (pm_mul_batch over chunks of
    # about 32 GiB of outputs and workspace)
    ws = pm.Workspace()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chunk, acc = [], 0.0
    for q, (na, nb) in enumerate(sizes.tolist() + [(0, 0)]):
        need = na * nb * 40.0
        if chunk and (q == len(sizes) or acc + need > 32.0 * (1 << 30)):
            call = pm.BatchCall(lay, [fs[i] for i in chunk], [gs[i] for i in chunk], ws)
            call.run()
            torch.cuda.synchronize()
            del call
            chunk, acc = [], 0.0
        if q < len(sizes):
            chunk.append(q)
            acc += need
    t_hbm = time.perf_counter() - t0
    del ws
    # the D2H copy of the same bytes alone, pinned, in 1 GiB pieces
    piece = 1 << 30
    src = torch.empty(piece, dtype=torch.uint8, device="cuda")
    dst = torch.empty(piece, dtype=torch.uint8, pin_memory=True)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    left = drained_bytes
    while left > 0:
        n = min(piece, left)
        dst[:n].copy_(src[:n], non_blocking=True)
        left -= n
    torch.cuda.synchronize()
    t_copy = time.perf_counter() - t0
    del src, dst
    return {
        "metric": "term-products/s (batched, results drained to host)", "value": pairs / t_drain,
        "unit": "term-products/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u64" if ring == "modp" else "f64",
        "data": "synthetic", "waves": waves, "drained_terms": terms[0], "drained_bytes": drained_bytes,
        "drain_s": t_drain, "results_in_hbm_s": t_hbm, "copy_alone_s": t_copy,
        "d2h_GBps_alone": drained_bytes / t_copy / 1e9,
        "overlap": (t_hbm + t_copy - t_drain) / min(t_hbm, t_copy),
        "config": {"workload": f"first {len(sizes)} products of the batched workload recipe (6 vars, 10 bits, "
                               "exponents 0..15, log-uniform term counts in [50, 20000], seed 4)",
                   "term_products": pairs, "device_buffer_GiB": args.drain_device_gib,
                   "host_buffer_GiB": args.drain_host_gib},
    }


def bench_dense(args):
    """Degree-box products: time per whole product (validation included, count
    read back) and term pairs/s against the measured ceiling of the dense
    tile's inner loop (mulmod or int64 product + LDS compare-and-swap + LDS
    atomic, no HBM traffic)."""
    import numpy as np
    import torch

    from paper_1303_7425_amd import polymul as pm
    from paper_1303_7425_amd import workloads as W

    def family(n, ring):
        f = W.dense_power(n, 4, 16, ring)
        return f, W.add_constant(f, 1), (4, 16, ring), None

    # (name, operands, timed steps); the output capacity of Examples 2 and 3
    # is their known term count rounded up (their bounds would be 118 GB and
    # more); Example 2's box takes 188 GB, so each case's memory is released
    # before the next
    cases = [("dense 4-var n=10, int64 (config 1)", lambda: family(10, "i64"), args.steps),
             ("dense 4-var n=20, mod 2^61-1 (config 2)", lambda: family(20, "modp"), args.steps),
             ("dense 4-var n=40, mod 2^61-1 (the paper's Example 1)", lambda: family(40, "modp"), 3),
             ("dense 4-var n=30, mod 2^61-1 (the serving mix's large request)", lambda: family(30, "modp"), args.steps),
             ("dense 5-var n=28, mod 2^61-1 (the paper's Example 3)",
              lambda: (*W.example3(28, 12, "modp"), (5, 12, "modp"), 150_000_000), 3),
             ("5-var n=25 through the degree box, mod 2^61-1 (the paper's Example 2)",
              lambda: (*W.config3("modp", n=25), (5, 12, "modp"), 320_000_000), 3)]
    if args.dense_cases:
        keep = {int(x) for x in args.dense_cases.split(",")}
        cases = [c for k, c in enumerate(cases, 1) if k in keep]
    ceil = {r: pm.dense_ceiling(r) for r in ("i64", "modp")}
    pm.set_tuning(args.tile, -1, True)
    rows = []
    for name, make, steps in cases:
        f, g, layout, capacity = make()
        ring = layout[2]
        call = pm.MulCall(layout, pm.to_device(f), pm.to_device(g), capacity=capacity)
        for _ in range(2):
            call.run()
            call.n()
        ts = []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            call.run()
            nout = call.n()
            ts.append(time.perf_counter() - t0)
        assert pm.last_call_status() == 0
        ms = 1e3 * float(np.median(ts))
        pairs = len(f) * len(g)
        rate = pairs / (ms * 1e-3)
        rows.append({"workload": name, "term_products": pairs, "output_terms": nout, "ms_per_product": ms,
                     "term_products_per_s": rate, "ceiling_per_s": ceil[ring], "frac_of_ceiling": rate / ceil[ring]})
        log(f"[dense] {name}: {ms:.3f} ms, {rate:.3e} pairs/s, {rate / ceil[ring]:.2f} of ceiling")
        del call
        torch.cuda.empty_cache()
    head = next((r for r in rows if "config 2" in r["workload"]), rows[0])
    return {"metric": "term-products/s (degree-box path) vs inner-loop ceiling", "value": head["term_products_per_s"],
            "unit": "term-products/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "roofline": {"bound": "alu", "kernel": "k_tile (dense)", "achieved": head["term_products_per_s"],
                         "peak": ceil["modp"], "unit": "term-products/s (measured inner-loop ceiling)",
                         "frac": head["frac_of_ceiling"]},
            "config": {"workload": "dense 4-var products f*(f+1), f = (1+x+y+z+t)^n, 16 bits/var; "
                                   "the paper's Examples 2 and 3 (5 vars, 12 bits/var)",
                       "tile": {-1: "automatic", 0: "32x64", 1: "64x64", 2: "128x128"}[args.tile]},
            "ceiling_per_s": ceil, "cases": rows}


def bench_serve(args):
    """Poisson arrivals through the server.  Latency runs from each request's
    scheduled arrival time to its completion (so a submit loop that falls
    behind is charged, not hidden), with the submit lateness recorded; result
    arrays come from pools per result-size class, so a busy slot of one class
    does not hold back another."""
    import numpy as np
    import torch

    from paper_1303_7425_amd import polymul as pm
    from paper_1303_7425_amd import workloads as W

    n_req = args.serve_requests
    reqs_all = W.config5_stream(n_req, rate_per_s=1.0, seed=5)   # arrival times rescaled below
    log(f"[serve] uploading {n_req} requests")
    dev = [(pm.to_device(r.f), pm.to_device(r.g)) for r in reqs_all]
    caps = [pm.bound((r.f.layout.nvars, r.f.layout.bits, "modp"), *d)[0] for r, d in zip(reqs_all, dev)]
    per_class = 16
    pools = {c: [pm.alloc_out(c, "modp") for _ in range(per_class)] for c in sorted(set(caps))}
    srv = pm.Server(64 << 30, nstreams=4)

    def run(rate):
        owner = {c: [None] * per_class for c in pools}
        nxt = {c: 0 for c in pools}
        tickets, t_sub = [], []
        arr = np.cumsum(np.random.Generator(np.random.PCG64(5)).exponential(1.0 / rate, size=n_req))
        t0 = time.perf_counter()
        for i, r in enumerate(reqs_all):
            c = caps[i]
            slot = nxt[c]
            nxt[c] = (slot + 1) % per_class
            if owner[c][slot] is not None:
                srv.wait(owner[c][slot])
            while time.perf_counter() - t0 < arr[i]:
                pass
            t_sub.append(time.perf_counter() - t0)
            owner[c][slot] = srv.submit((r.f.layout.nvars, r.f.layout.bits, "modp"), dev[i][0], dev[i][1],
                                        pools[c][slot])
            tickets.append(owner[c][slot])
        for t in tickets:
            assert srv.wait(t) == 0
        elapsed = time.perf_counter() - t0
        # latency from the scheduled arrival: submit lateness + server latency
        late = np.array(t_sub) - arr
        lat_ms = np.array([srv.latency_us(t) for t in tickets]) / 1e3 + late * 1e3
        return elapsed, tickets, lat_ms, late

    pairs = sum(len(r.f) * len(r.g) for r in reqs_all)
    t_sat, _, _, _ = run(1e12)   # saturation: all requests at once
    sat_rate = n_req / t_sat
    log(f"[serve] saturated: {sat_rate:.1f} req/s, {pairs / t_sat:.3e} pairs/s")
    rate = args.serve_load * sat_rate
    t_run, tickets, lat, late = run(rate)
    by_class = {}
    for kind in sorted({r.kind for r in reqs_all}):
        lk = np.array([x for x, r in zip(lat, reqs_all) if r.kind == kind])
        by_class[kind] = {"requests": int(lk.size), "p50_ms": float(np.percentile(lk, 50)),
                          "p99_ms": float(np.percentile(lk, 99))}
    srv.close()
    return {
        "metric": "serve latency p50/p99 (from scheduled arrival)", "value": float(np.percentile(lat, 50)),
        "unit": "ms (p50)", "p99_ms": float(np.percentile(lat, 99)), "n_gpus": 1, "higher_is_better": False,
        "dtype": "u64", "data": "synthetic", "arrival_rate_per_s": rate, "load_fraction_of_saturation": args.serve_load,
        "saturated_requests_per_s": sat_rate, "saturated_term_products_per_s": pairs / t_sat,
        "sustained_term_products_per_s": pairs / t_run, "requests": n_req, "latency_by_class": by_class,
        "submit_lateness_ms": {"p50": float(np.percentile(late, 50)) * 1e3, "p99": float(np.percentile(late, 99)) * 1e3,
                               "max": float(late.max()) * 1e3},
        "config": {"workload": "Poisson arrivals (seed 5): 98% sparse 5-var pairs at power U{6..12} with fresh "
                               "residues, 2% dense (1+x+y+z+t)^30 x (same+1), mod 2^61-1"},
    }


def host_cpu():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline(f, g, call):
    """The oracle's multiply on one host thread, timed around the C call alone
    (inputs converted and the output allocated beforehand), on whole products
    of the same workload until about 10 s of CPU work (at most 8)."""
    import ctypes

    import numpy as np

    import oracle
    log("[bench] oracle (CPU baseline)")
    lay = f.layout
    fk, fc = np.ascontiguousarray(f.keys, np.uint64), np.ascontiguousarray(f.coefs, oracle.COEF_DTYPE[lay.ring])
    gk, gc = np.ascontiguousarray(g.keys, np.uint64), np.ascontiguousarray(g.coefs, oracle.COEF_DTYPE[lay.ring])
    L = oracle.lib()
    b = ctypes.c_int64(0)
    assert L.oracle_bound(lay.nvars, lay.bits, fk.size, fk.ctypes.data, gk.size, gk.ctypes.data, ctypes.byref(b)) == 0
    cap = int(b.value)
    hk = np.zeros(cap, np.uint64)
    hc = np.zeros(cap, oracle.COEF_DTYPE[lay.ring])
    ha = np.zeros(cap, np.float64) if lay.ring == "f64" else None
    nh = ctypes.c_int64(0)
    reps, dt = 0, 0.0
    while reps < 8 and (reps == 0 or dt < 10.0):
        t = time.perf_counter()
        rc = L.oracle_mul(lay.nvars, lay.bits, oracle.RING_CODE[lay.ring], fk.size, fk.ctypes.data, fc.ctypes.data,
                          gk.size, gk.ctypes.data, gc.ctypes.data, cap, hk.ctypes.data, hc.ctypes.data,
                          ha.ctypes.data if ha is not None else None, ctypes.byref(nh))
        dt += time.perf_counter() - t
        assert rc == 0
        reps += 1
    n = int(nh.value)
    rk, rcf = call.result().numpy()
    same = bool(np.array_equal(rk, hk[:n]) and np.array_equal(rcf.view(np.uint64), hc[:n].view(np.uint64)))
    model, ncpu, naff = host_cpu()
    products = len(f) * len(g)
    return {"value": reps * products / dt, "unit": "term-products/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "nproc": naff, "cpu_count": ncpu,
            "sample": f"{reps} full products of the same workload, oracle_mul alone on one thread, {dt:.2f} s; "
                      f"GPU result {'identical' if same else 'DIFFERENT'}"}


def main():
    args = parse()
    if args.traffic_summary:
        if len(args.traffic_summary) not in (2, 3):
            sys.exit("--traffic-summary takes FETCH_CSV WRITE_CSV [OUT_JSON]")
        traffic_summary(*args.traffic_summary[:3])
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the product path is single-GPU in this "
              "build, see DESIGN.md for how it would shard", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1303_7425_amd import polymul as pm
    from paper_1303_7425_amd import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "drain":
        print(json.dumps(bench_drain(args)), flush=True)
        return
    if args.workload == "dense":
        print(json.dumps(bench_dense(args)), flush=True)
        return
    pm.set_tuning(-1, args.combine, True)
    f, g = W.config3(args.ring)
    layout = (5, 12, args.ring)
    fd, gd = pm.to_device(f), pm.to_device(g)
    call = pm.MulCall(layout, fd, gd)
    products = len(f) * len(g)
    stream = torch.cuda.current_stream()

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        call.run()
        n_out = call.n()
    assert pm.last_call_status() == 0, "device consistency check failed"

    # timed region: K whole products, count read back each step
    log(f"[bench] timed {args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        call.run()
        n_out = call.n()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps

    # same steps again with HIP events recorded around every kernel on the call's stream
    log("[bench] profiled")
    pm.profile_enable(True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        call.run()
        call.n()
    torch.cuda.synchronize()
    prof = pm.profile_read()
    pm.profile_enable(False)
    info = pm.last_call_info()
    staged, passes, kbytes, vbytes = info["staged"], info["passes"], info["key_bytes"], info["payload_bytes"]
    assert pm.last_call_status() == 0
    per_step = {k: round(v[0] / args.steps, 5) for k, v in prof.items()}
    # dominant kernel: the profiled scope with the most time per product
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    dom_ms, dom_n = prof[dom]
    dom_avg_ms = dom_ms / max(dom_n, 1)
    pair_item = 8  # staged (compressed key, pair index), two u32
    if dom == "bk_reduce":
        # reads every staged pair once, writes each result term's key (u32)
        # and coefficient (u64); operand coefficients come from cache
        dom_bytes = products * pair_item + n_out * 12 + (len(f) + len(g)) * 8
        dom_kernel, dom_label = "k_bk_reduce (per-work-item LDS sum)", "bk_reduce (per-work-item LDS sum)"
    elif dom == "bk_scatter":
        dom_bytes = products * pair_item
        dom_kernel, dom_label = "k_bk_scatter (pair indices to work items)", "bk_scatter (pair indices to work items)"
    else:
        # a radix pass that moves items only: pair-index sorts (4-byte payload)
        # read and write the index alone, combined sorts key + coefficient
        item_bytes = vbytes if vbytes == 4 else kbytes + vbytes
        dom_bytes = staged * item_bytes * 2
        dom_kernel, dom_label = f"{dom} (radix pass)", "onesweep pass (pair indices)"
    achieved = dom_bytes / (dom_avg_ms * 1e-3) / 1e9 if dom_avg_ms > 0 else 0.0
    # effective bandwidth: the product's algorithmic floor (22 B per term
    # product: inputs, output, one spill of combined tiles) over the whole step
    floor_bytes = 22.0 * products
    effective = floor_bytes / (ms_step * 1e-3) / 1e9

    if args.copy_calibration:
        src = torch.empty(1 << 29, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(f, g, call)

    out = {
        "metric": "term-products/s",
        "value": products / (ms_step * 1e-3),
        "unit": "term-products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64" if args.ring == "modp" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "sparse 5-var product (1+x+y+2z^2+3t^3+5u^5)^12 * (1+u+t+2z^2+3y^3+5x^5)^12, "
                        + ("coefficients mod 2^61-1" if args.ring == "modp" else "FP64 coefficients U[-1,1] seed 3"),
            "terms_f": len(f), "terms_g": len(g), "term_products": products, "output_terms": n_out,
            "bits_per_var": 12, "sparse_mode": {-1: "automatic", 0: "pair-index radix sort", 1: "LDS tile combine",
                                                2: "output-key intervals", 3: "output-key work items"}[args.combine],
        },
        "roofline": {"bound": "hbm", "kernel": dom_kernel, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom_label) if args.ring == "modp" else None,
                     "algorithmic_bytes_per_launch": dom_bytes, "avg_launch_ms": dom_avg_ms,
                     "effective": {"floor_bytes": floor_bytes, "achieved": effective,
                                   "frac": effective / HBM_PEAK_GBS},
                     "path_counter_bytes_per_product": measured_step_traffic() if args.ring == "modp" else None,
                     "sorted_items": staged, "passes": passes, "key_bytes": kbytes,
                     "payload_bytes": vbytes},
        "kernel_ms_per_step": per_step,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
