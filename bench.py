"""Benchmark of the exact pair-counting path on one MI355X.

One step = the whole hot path over one synthetic catalogue already resident
in HBM: validation and cell keys, radix sort, gather and cell offsets, work
list, ordering, the persistent counting kernel (FP32 distances, table
binning, FP64 edge recheck, LDS histograms) and the global merge.

Default workload (`--workload c2`): periodic cube L = 2000 Mpc/h, 1,000,000
clustered points (lognormal field on 256^3 cells, P(k) ~ k^-1.5, sigma_G = 1),
(s, mu) bins 40 x 100 over s in [0, 200), mu in [0, 1], line of sight z,
auto count, int64 counts plus FP64 weighted counts (weights U[0.5, 1.5)).

Prints one JSON line.  `value` is in-range pairs per second of the whole step.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
FLOP_PER_DISTANCE = 8      # 3 sub, 1 mul, 2 fma (counted as 2 flops each)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c5"])
    ap.add_argument("--unweighted", action="store_true", help="count without weights")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", default="", help="tuning overrides, e.g. cells_per_rmax=3,tile_points=128")
    return ap.parse_args()


def workload(name, weighted):
    from paper_2301_12557_amd import synth
    c = {"c1": 1, "c2": 2, "c5": 5}[name]
    w = synth.workload(c, weighted=weighted and c != 5)
    desc = {
        1: "C1 periodic L=1000, 20,000 uniform points, 40 linear s bins [0,200), auto",
        2: "C2 periodic L=2000, 1,000,000 lognormal points (256^3 field, P~k^-1.5, sigma_G=1), "
           "(s,mu) 40x100 bins s in [0,200) mu in [0,1], LOS z, auto",
        5: "C5 periodic L=3000, 10,000,000 lognormal points, 50 log s bins [0.1,50), auto",
    }[c]
    return w, desc


def measured_traffic(kernel_variant):
    """HBM bytes per launch of the counting kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (profiles/k_count_c2_traffic.json), if they were taken on the current
    kernel source and the same kernel variant; otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_count_c2_traffic.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2301_12557_amd", "csrc", "count.hip"), "rb").read()
        if rec.get("count_hip_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
            return None
        if rec.get("variant") != kernel_variant:
            return None
        return float(rec["hbm_bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(w, target_s):
    """The FP64 cell-list oracle, as it stands, on a sample: the cross count of a random subset of
    the catalogue against the whole catalogue (every pair of the subset with every point)."""
    import oracle
    x = w["x1"]
    kw = dict(kind=w["kind"], edges1=w["edges1"], edges2=w["edges2"], los=w["los"], box=w["box"])
    rng = np.random.default_rng(1)
    s0 = min(len(x), 1000)
    t = time.perf_counter()
    c, _ = oracle.count(x[rng.choice(len(x), s0, replace=False)], x, method="grid", **kw)
    dt0 = time.perf_counter() - t
    s = int(min(len(x), max(s0, s0 * target_s / max(dt0, 1e-3))))
    idx = rng.choice(len(x), s, replace=False)
    t = time.perf_counter()
    c, _ = oracle.count(x[idx], x, method="grid", **kw)
    dt = time.perf_counter() - t
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        pass
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = int(omp) if omp else cores
    return {"value": float(c.sum()) / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 cell-list oracle, cross count of {s} random points of the catalogue against all "
                      f"{len(x)} points: {int(c.sum())} in-range pairs in {dt:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import torch
    from paper_2301_12557_amd import fcfc

    weighted = not args.unweighted
    w, desc = workload(args.workload, weighted)
    weighted = weighted and w["w1"] is not None
    dev = torch.device("cuda:0")
    x = torch.from_numpy(w["x1"]).to(dev)
    wt = torch.from_numpy(w["w1"]).to(dev) if weighted else None
    tune = {}
    for kv in filter(None, args.tune.split(",")):
        k, v = kv.split("=")
        tune[k] = int(v)
    tune.setdefault("n_hint", len(w["x1"]))
    plan = fcfc.Plan(w["kind"], w["edges1"], w["edges2"], los=w["los"], box=w["box"], **tune)
    nb = plan.n1 * plan.n2
    out = torch.empty(nb, dtype=torch.int64, device=dev)
    wout = torch.empty(nb, dtype=torch.float64, device=dev) if weighted else None

    def step():
        cells = plan.build_cells(x, wt)
        plan.count(cells, weighted=weighted, out=out, wout=wout)
        st = plan.stats()
        cells.close()
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kms = []
    stats = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats = step()
        kms.append(stats["kernel_ms"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    pairs = int(stats["in_range"])
    cand = int(stats["candidates"])
    kernel_ms = float(np.mean(kms))
    achieved = FLOP_PER_DISTANCE * cand / (kernel_ms * 1e-3) / 1e12
    res = {
        "metric": "exact pairs/s (1 GPU, % FP32 roofline); mocks/s batched+learned vs plain",
        "value": pairs / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "points": len(w["x1"]), "bins": nb,
                   "weighted": bool(weighted), "tuning": tune},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(f"{args.workload}/{'weighted' if weighted else 'unweighted'}"),
                     "kernel": "k_count", "kernel_ms": kernel_ms,
                     "per_unit": f"{FLOP_PER_DISTANCE} flop per distance evaluation",
                     "units_per_launch": cand},
        "detail": {"in_range_pairs": pairs, "distance_evaluations": cand,
                   "candidates_per_pair": cand / max(pairs, 1),
                   "rechecks": int(stats["rechecks"]), "recheck_rate": stats["rechecks"] / max(cand, 1),
                   "kernel_pairs_per_s": pairs / (kernel_ms * 1e-3),
                   "kernel_distance_evals_per_s": cand / (kernel_ms * 1e-3),
                   "in_range_flop_frac": FLOP_PER_DISTANCE * pairs / (kernel_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                   "items": int(stats["items"]), "grid": stats["grid"], "cells_per_rmax": stats["cells_per_rmax"],
                   "wg_per_cu": stats["wg_per_cu"], "lut_entries": stats["lut_entries"],
                   "band_d2_rel": stats["band_d2_rel"], "device": torch.cuda.get_device_name(0)},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
