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
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--c3-rr", action="store_true", help="C3: also count RR (40M randoms, ~2e13 pairs)")
    ap.add_argument("--unweighted", action="store_true", help="count without weights")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", default="", help="tuning overrides, e.g. cells_per_rmax=3,tile_points=128")
    ap.add_argument("--no-c4", action="store_true", help="skip the batched-mocks comparison")
    ap.add_argument("--c4-mocks", type=int, default=200)
    ap.add_argument("--c4-repeats", type=int, default=12)
    ap.add_argument("--no-learned", action="store_true", help="skip training and the held-out C5 comparison")
    ap.add_argument("--no-peaks", action="store_true", help="skip the roofline microbenchmarks")
    ap.add_argument("--no-pairs", action="store_true", help="skip the multi-tracer pair-list comparison")
    ap.add_argument("--no-binning", action="store_true", help="skip the histogram-update microbenchmark")
    ap.add_argument("--binning-values", type=float, default=6.4e9, help="squared separations per binning call")
    ap.add_argument("--no-triplets", action="store_true", help="skip the triangle-count measurement")
    ap.add_argument("--no-c3", action="store_true", help="skip the full-size C3 survey counts (DD, DR, RR)")
    ap.add_argument("--no-fixed", action="store_true",
                    help="skip the roofline of C2 unweighted, C5 and C1 beside the headline")
    ap.add_argument("--shards", type=int, default=0,
                    help="also count each of G work-list shards (one GPU's share of a G-GPU run) and report "
                         "their kernel times")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (a plain copy of known size, to calibrate "
                         "HBM traffic counters against)")
    return ap.parse_args()


def workload(name, weighted):
    from paper_2301_12557_amd import synth
    c = {"c1": 1, "c2": 2, "c3": 3, "c5": 5}[name]
    w = synth.workload(c, weighted=weighted and c != 5)
    desc = {
        1: "C1 periodic L=1000, 20,000 uniform points, 40 linear s bins [0,200), auto",
        2: "C2 periodic L=2000, 1,000,000 lognormal points (256^3 field, P~k^-1.5, sigma_G=1), "
           "(s,mu) 40x100 bins s in [0,200) mu in [0,1], LOS z, auto",
        3: "C3 open survey shell r in [1000,2000], RA 60 deg x Dec 30 deg, data 2,000,000 + randoms 40,000,000, "
           "(s_perp,pi) 40x40 bins over [0,200), mid-point LOS, weights U[0.5,2); one step = bounds + both "
           "cell builds + DD + DR (+ RR with --c3-rr)",
        5: "C5 periodic L=3000, 10,000,000 lognormal points, 50 log s bins [0.1,50), auto",
    }[c]
    return w, desc


def measured_traffic(kernel_variant, sources=("count.hip",), key="count_hip_sha256_16"):
    """HBM bytes per launch of a kernel from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (profiles/*_traffic.md), if it was taken on the current
    kernel sources and the same kernel variant; else None."""
    import hashlib
    try:
        src = b"".join(open(os.path.join(ROOT, "paper_2301_12557_amd", "csrc", f), "rb").read() for f in sources)
        digest = hashlib.sha256(src).hexdigest()[:16]
        pdir = os.path.join(ROOT, "profiles")
        for fn in sorted(os.listdir(pdir)):
            if not fn.endswith("_traffic.md"):
                continue
            for line in open(os.path.join(pdir, fn)):
                if line.startswith("traffic-record:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("variant") == kernel_variant and rec.get(key) == digest:
                        return float(rec["hbm_bytes_per_launch"])
    except Exception:
        return None
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
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": float(c.sum()) / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "cpus_available": cores, "cpu_model": model,
            "sample": f"FP64 cell-list oracle, cross count of {s} random points of the catalogue against all "
                      f"{len(x)} points: {int(c.sum())} in-range pairs in {dt:.2f} s"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _sync_time(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, r


def record_timings(fcfc, x, kind, e1, e2, box, ks):
    """Per-item features and log2 times of counts of x at each cells-per-radius k."""
    import torch
    feats, ts = [], []
    for k in ks:
        plan = fcfc.Plan(kind, e1, e2, box=box, n_hint=len(x), cells_per_rmax=k, record_timing=1)
        c = plan.build_cells(x)
        plan.count(c)
        f, t = plan.timings()
        feats.append(f)
        ts.append(t)
        c.close()
        plan.close()
    return torch.cat(feats), torch.cat(ts)


def train_cost_model(fcfc, synth, x_c2, w_c2, mocks):
    """Train the cost model on item timings of the C2 catalogue (k = 2..4) and of
    four C4 mocks (smallest, largest, two others; k = 1..5)."""
    import torch
    feats, ts, src = [], [], []
    f, t = record_timings(fcfc, x_c2, "smu", w_c2["edges1"], w_c2["edges2"], w_c2["box"], [2, 3, 4])
    feats.append(f)
    ts.append(t)
    src.append(f"C2 k=2..4: {len(t)} items")
    sizes = [len(m) for m in mocks]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 0, 1})
    e1, e2 = synth.linear_edges(0, 200, 40), synth.mu_edges(100)
    for m in pick:
        f, t = record_timings(fcfc, mocks[m], "smu", e1, e2, 1000.0, [1, 2, 3, 4, 5])
        feats.append(f)
        ts.append(t)
        src.append(f"C4 mock {m} (N={sizes[m]}) k=1..5: {len(t)} items")
    F, T = torch.cat(feats), torch.cat(ts)
    md = fcfc.Model(seed=2301)
    ms, loss = _sync_time(lambda: md.train(F, T, epochs=6, batch=512, lr=2e-3, seed=7))
    return md, {"samples": int(len(T)), "epochs": 6, "batch": 512, "lr": 2e-3, "final_loss": loss,
                "train_s": ms / 1e3, "sources": src}


def make_mocks(synth, nmock):
    sizes = synth.mock_sizes(nmock)
    return [synth.lognormal_box_torch(int(n), 1000.0, synth.MOCK_SEED_BASE + m, device="cuda")
            for m, n in enumerate(sizes)]


def c4_section(fcfc, synth, mocks, model, repeats):
    """Catalogues/s of 200 C4 mocks: plain per-catalogue launches (P), the batched
    pipeline in a HIP graph (B), and the batched pipeline with the tuning that the
    autotuner picks with the learned model proposing (BL).  Every arm's histograms
    must equal P's."""
    import torch
    e1, e2 = synth.linear_edges(0, 200, 40), synth.mu_edges(100)
    nm = len(mocks)
    sizes = [len(m) for m in mocks]
    nhint = int(np.mean(sizes))
    nb = 40 * 100
    plan = fcfc.Plan("smu", e1, e2, box=1000.0, n_hint=nhint)
    outP = torch.empty(nm * nb, dtype=torch.int64, device="cuda")

    def run_plain():
        for i, x in enumerate(mocks):
            c = plan.build_cells(x)
            plan.count(c, out=outP[i * nb:(i + 1) * nb])
            c.close()

    run_plain()
    tP = [_sync_time(run_plain)[0] for _ in range(repeats)]
    st = plan.stats()

    def batch_arm(pl):
        out = torch.empty(nm * nb, dtype=torch.int64, device="cuda")
        create_ms, b = _sync_time(lambda: fcfc.Batch(pl, [(x, None) for x in mocks]))
        first_ms, _ = _sync_time(lambda: b.run(out, use_graph=True))
        b.check()
        ts = []
        for _ in range(repeats):
            ms, _ = _sync_time(lambda: b.run(out, use_graph=True))
            ts.append(ms)
        n_items, gpu_ms = b.check()
        equal = bool(torch.equal(out, outP))
        b.close()
        return ts, create_ms, first_ms, n_items, equal

    tB, cB, fB, iB, eqB = batch_arm(plan)
    med = int(np.argsort(sizes)[nm // 2])
    tune_ms, tuned = _sync_time(lambda: fcfc.autotune(mocks[med], model=model, kind="smu", edges1=e1, edges2=e2,
                                                      box=1000.0, n_hint=nhint))
    tk = {k: v for k, v in tuned[0].items() if k not in ("record_timing", "order")}

    # The proposal was measured on single counts of one mock; it is kept only if
    # it also beats the default on a batch of 20 mocks (best of 3 replays each).
    def sub_batch_ms(pl):
        sub = [(x, None) for x in mocks[:20]]
        out = torch.empty(len(sub) * nb, dtype=torch.int64, device="cuda")
        b = fcfc.Batch(pl, sub)
        b.run(out, use_graph=True)
        ms = min(_sync_time(lambda: b.run(out, use_graph=True))[0] for _ in range(3))
        b.close()
        return ms

    planT = fcfc.Plan("smu", e1, e2, box=1000.0, **tk)
    sub_tuned, sub_default = sub_batch_ms(planT), sub_batch_ms(plan)
    kept = sub_tuned < sub_default
    if not kept:
        tk = {"n_hint": nhint}
        planT.close()
        planT = plan
    tL, cL, fL, iL, eqL = batch_arm(planT)
    # the network's own gain on the work order: default tuning, items of each
    # mock ordered by the model's predicted time instead of the heuristic cost
    order_arm = None
    if model is not None:
        planO = fcfc.Plan("smu", e1, e2, box=1000.0, n_hint=nhint, order="learned")
        planO.set_model(model)
        tO, cO, fO, iO, eqO = batch_arm(planO)
        order_arm = (tO, cO, fO, iO, eqO)

    def arm(ts, extra=None):
        ts = np.asarray(ts)
        r = {"mocks_per_s": nm / (ts.mean() / 1e3), "mocks_per_s_sd": float(np.std(nm / (ts / 1e3))),
             "ms_mean": float(ts.mean()), "ms_sd": float(ts.std()), "runs": len(ts)}
        if extra:
            r.update(extra)
        return r

    return {
        "workload": f"C4: {nm} periodic L=1000 lognormal mocks, N uniform in [100k, 500k] "
                    f"(total {sum(sizes)} points), (s,mu) 40x100 bins s in [0,200), LOS z, auto, int64",
        "arms": {
            "P": arm(tP, {"what": "per-catalogue build + count launches on one stream, analytic tuning",
                          "cells_per_rmax": st["cells_per_rmax"]}),
            "B": arm(tB, {"what": "batched pipeline replayed from a HIP graph, analytic tuning",
                          "create_ms": cB, "first_run_ms": fB, "items": iB, "counts_equal_P": eqB}),
            "BL": arm(tL, {"what": "batched pipeline (HIP graph) with the autotuned tuning (cell sizes proposed by "
                                   "the learned model, tuned on the median-size mock), kept only if it also beats "
                                   "the default on a 20-mock sub-batch",
                           "tuning": tk, "autotune_ms": tune_ms, "autotune_trials": tuned[3],
                           "proposal": {k: v for k, v in tuned[0].items() if k not in ("record_timing", "order")},
                           "sub_batch_ms": {"proposal": sub_tuned, "default": sub_default}, "proposal_kept": kept,
                           "create_ms": cL, "first_run_ms": fL, "items": iL, "counts_equal_P": eqL}),
            **({"BO": arm(order_arm[0], {"what": "batched pipeline (HIP graph), default tuning, each mock's items in "
                                                "the order of the learned cost model's predicted time",
                                        "create_ms": order_arm[1], "first_run_ms": order_arm[2],
                                        "items": order_arm[3], "counts_equal_P": order_arm[4]})}
               if order_arm else {}),
        },
        **({"BO_over_B": float(np.mean(tB) / np.mean(order_arm[0]))} if order_arm else {}),
        "BL_over_P": float(np.mean(tP) / np.mean(tL)),
        "B_over_P": float(np.mean(tP) / np.mean(tB)),
        "BL_over_B": float(np.mean(tB) / np.mean(tL)),
    }


def c5_section(fcfc, synth, model):
    """Held-out C5 (not in the training set): the analytic cell size vs the model's
    choice vs the autotuned tuning, build + count time (best of 3) and kernel time."""
    e = synth.log_edges(0.1, 50.0, 50)
    x = synth.lognormal_box_torch(10_000_000, 3000.0, synth.config_seed(5), device="cuda")

    def measure(reps=3, mdl=None, **tune):
        tune.setdefault("n_hint", len(x))
        plan = fcfc.Plan("s", e, None, box=3000.0, **tune)
        if mdl is not None:
            plan.set_model(mdl)
        best, kern = np.inf, np.inf
        for _ in range(reps):
            def go():
                c = plan.build_cells(x)
                plan.count(c)
                return c
            ms, c = _sync_time(go)
            c.close()
            best = min(best, ms)
            kern = min(kern, plan.stats()["kernel_ms"])
        st = plan.stats()
        plan.close()
        return {"ms": best, "kernel_ms": kern, "cells_per_rmax": st["cells_per_rmax"], "order": st["order_used"]}

    kh, _ = fcfc.choose_cells(x, model=None, kind="s", edges1=e, box=3000.0)
    kl, pred = fcfc.choose_cells(x, model=model, kind="s", edges1=e, box=3000.0)
    tmsec, tuned = _sync_time(lambda: fcfc.autotune(x, model=model, kind="s", edges1=e, box=3000.0))
    tk = {k: v for k, v in tuned[0].items() if k != "record_timing"}
    res = {
        "workload": "C5: periodic L=3000, 10,000,000 lognormal points (GPU generator), 50 log s bins [0.1,50), auto",
        "analytic": measure(),
        "learned_k": dict(measure(cells_per_rmax=kl), predicted_ms_by_k=pred),
        "learned_order": measure(order="learned", mdl=model),
        "autotuned": dict(measure(mdl=model, **tk), tuning=tk, autotune_ms=tmsec, trials=tuned[3]),
    }
    res["learned_k_gain"] = res["analytic"]["ms"] / res["learned_k"]["ms"]
    res["autotuned_gain"] = res["analytic"]["ms"] / res["autotuned"]["ms"]
    return res


def fixed_axis_section(fcfc, synth, torch, x2):
    """The counting kernel's roofline on the other fixed-axis workloads: C2
    unweighted (the headline catalogue), C5 and C1.  Kernel time by HIP events,
    best of 3 launches on one cell set."""
    out = {}

    def run(name, desc, x, kind, e1, e2, box):
        plan = fcfc.Plan(kind, e1, e2, box=box, n_hint=len(x))
        cells = plan.build_cells(x)
        ks = []
        for _ in range(3):
            plan.count(cells)
            ks.append(plan.stats()["kernel_ms"])
        st = plan.stats()
        k = min(ks)
        achieved = FLOP_PER_DISTANCE * st["candidates"] / (k * 1e-3) / 1e12
        out[name] = {"workload": desc, "kernel_ms": k, "distance_evaluations": st["candidates"],
                     "in_range_pairs": st["in_range"], "kernel_pairs_per_s": st["in_range"] / (k * 1e-3),
                     "cells_per_rmax": st["cells_per_rmax"],
                     "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                  "frac": achieved / PEAK_FP32_TFLOPS}}
        cells.close()
        plan.close()

    w2 = synth.workload(2)
    run("c2_unweighted", "C2 catalogue, (s,mu) 40x100, LOS z, auto, unweighted", x2, "smu", w2["edges1"],
        w2["edges2"], 2000.0)
    x5 = synth.lognormal_box_torch(10_000_000, 3000.0, synth.config_seed(5), device="cuda")
    run("c5", "C5: periodic L=3000, 10,000,000 lognormal points (GPU generator), 50 log s bins [0.1,50), auto",
        x5, "s", synth.log_edges(0.1, 50.0, 50), None, 3000.0)
    del x5
    w1 = synth.workload(1)
    run("c1", "C1: periodic L=1000, 20,000 uniform points, 40 s bins [0,200), auto",
        torch.from_numpy(w1["x1"]).to("cuda"), "s", w1["edges1"], None, 1000.0)
    return out


def clustered_section(fcfc, synth, model):
    """Held-out catalogues far more clustered than the training boxes (Gaussian
    blobs): the analytic cell size vs the model's pure choice vs the measured
    search without and with the model proposing cell sizes; build + count time
    (best of 3) of each tuning, measured afresh after the search."""
    import torch
    L = 500.0
    e1 = synth.linear_edges(0, 40, 20)
    e2 = synth.mu_edges(10)
    out = {}
    for name, (nblob, rad, frac, seed) in (("blobs30", (30, 15.0, 0.8, 8)), ("blobs10", (10, 5.0, 0.9, 9))):
        x = torch.from_numpy(synth.blobs_box(300_000, L, nblob, rad, frac, seed)).to("cuda")

        def measure(mdl=None, **tune):
            tune.setdefault("n_hint", len(x))
            plan = fcfc.Plan("smu", e1, e2, box=L, **tune)
            if mdl is not None:
                plan.set_model(mdl)
            best = np.inf
            for _ in range(3):
                def go():
                    c = plan.build_cells(x)
                    plan.count(c)
                    return c
                ms, c = _sync_time(go)
                c.close()
                best = min(best, ms)
            k = plan.stats()["cells_per_rmax"]
            plan.close()
            return {"ms": best, "cells_per_rmax": k}

        kl, _ = fcfc.choose_cells(x, model=model, kind="smu", edges1=e1, edges2=e2, box=L)
        t0 = fcfc.autotune(x, kind="smu", edges1=e1, edges2=e2, box=L)
        t1 = fcfc.autotune(x, model=model, kind="smu", edges1=e1, edges2=e2, box=L)
        k0 = {k: v for k, v in t0[0].items() if k != "record_timing"}
        k1 = {k: v for k, v in t1[0].items() if k != "record_timing"}
        r = {"analytic": measure(), "learned_k": measure(cells_per_rmax=kl),
             "search_without_model": dict(measure(**k0), trials=t0[3]),
             "search_with_model": dict(measure(mdl=model, **k1), trials=t1[3])}
        a = r["analytic"]["ms"]
        r["gain_learned_k"] = a / r["learned_k"]["ms"]
        r["gain_search_without_model"] = a / r["search_without_model"]["ms"]
        r["gain_search_with_model"] = a / r["search_with_model"]["ms"]
        out[name] = r
        del x
    return {"workload": "300,000 points in [0,500)^3 periodic, 80 % in 30 Gaussian blobs of width 15 (blobs30) "
                        "or 90 % in 10 of width 5 (blobs10), rest uniform; (s,mu) 20x10 over [0,40)",
            **out}


# The multi-tracer pair list of the paper's quick guide (App. D): LRG data
# and randoms (L, R), ELG data and randoms (E, S).
TRACERS = (("L", 100_000), ("R", 500_000), ("E", 150_000), ("S", 750_000))
TRACER_PAIRS = ("LL", "LR", "RR", "EE", "ES", "SS", "LE", "LS", "RE", "RS")


def pairs_section(fcfc, synth, torch, repeats=3):
    """Multi-tracer counts (S) per pair, each a separate count over cell sets
    built once, against (M) one pair batch: one build, one work list, one
    counting launch, replayed from a HIP graph.  Survey patch as C3 (open box,
    mid-point line of sight, 40x40 (s_perp, pi) bins to 200), weights U[0.5, 2]."""
    lab = [t for t, _ in TRACERS]
    xs = [torch.from_numpy(synth.survey_shell(n, synth.config_seed(3) + 100 + i)).cuda()
          for i, (_, n) in enumerate(TRACERS)]
    ws = [torch.from_numpy(synth.uniform_weights(n, 0.5, 2.0, synth.config_seed(3) + 200 + i)).cuda()
          for i, (_, n) in enumerate(TRACERS)]
    pairs = [(lab.index(pq[0]), lab.index(pq[1])) for pq in TRACER_PAIRS]
    e = synth.linear_edges(0, 200, 40)
    plan = fcfc.Plan("spi", e, e, los="mid", box=0.0, n_hint=max(n for _, n in TRACERS))
    plan.fit_bounds([(x, None) for x in xs])
    nb = plan.n1 * plan.n2
    outS = torch.empty(len(pairs) * nb, dtype=torch.int64, device="cuda")
    woutS = torch.empty(len(pairs) * nb, dtype=torch.float64, device="cuda")

    def separate():
        cells = [plan.build_cells(x, w) for x, w in zip(xs, ws)]
        for q, (a, b) in enumerate(pairs):
            plan.count(cells[a], None if a == b else cells[b], weighted=True, out=outS[q * nb:(q + 1) * nb],
                       wout=woutS[q * nb:(q + 1) * nb])
        for c in cells:
            c.close()

    separate()
    tS = [_sync_time(separate)[0] for _ in range(repeats)]
    out = torch.empty_like(outS)
    wout = torch.empty_like(woutS)
    create_ms, b = _sync_time(lambda: fcfc.Batch(plan, list(zip(xs, ws)), pairs=pairs))
    first_ms, _ = _sync_time(lambda: b.run(out, wout, use_graph=True))
    tM = []
    for _ in range(repeats):
        ms, _ = _sync_time(lambda: b.run(out, wout, use_graph=True))
        tM.append(ms)
    n_items, gpu_ms = b.check()
    equal = bool(torch.equal(out, outS) and torch.equal(wout, woutS))
    b.close()
    plan.close()
    total = int(outS.sum().item())
    return {
        "workload": "multi-tracer survey patch (RA 60 deg, Dec +-15 deg, r 1000-2000, open box): "
                    + ", ".join(f"{t} {n}" for t, n in TRACERS) + "; pairs " + " ".join(TRACER_PAIRS)
                    + "; (s_perp, pi) 40x40 to 200, mid-point LOS, weights U[0.5, 2]",
        "in_range_pairs": total,
        "separate_ms": float(np.mean(tS)), "separate_ms_sd": float(np.std(tS)),
        "batch_ms": float(np.mean(tM)), "batch_ms_sd": float(np.std(tM)), "runs": repeats,
        "batch_create_ms": create_ms, "batch_first_run_ms": first_ms, "batch_items": n_items,
        "batch_over_separate": float(np.mean(tS) / np.mean(tM)),
        "in_range_pairs_per_s_batch": total / (np.mean(tM) * 1e-3),
        "counts_equal": equal,
    }


BIN_LAYOUTS = (("linear", 20), ("linear", 200), ("log", 20), ("log", 200))


def binning_section(fcfc, synth, torch, nvals, repeats=5, cpu_values=10_000_000, cpu=True):
    """The histogram update routine alone (App. C input: s^2 = x^(2/3) 200^2,
    nvals values resident in HBM; 20 and 200 bins, linear on [0, 200) and
    logarithmic on [0.1, 200)): kernel time over HIP events on the launch
    stream, against the HBM roofline of reading 8 B per value once; then the
    look-up table size scan on the 200 logarithmic bins; the oracle on a
    bounded sample for scale."""
    n = int(nvals)
    v = synth.s2_samples_torch(n, 200.0, synth.config_seed(6))
    torch.cuda.synchronize()
    rows = []
    for layout, nb in BIN_LAYOUTS:
        e = synth.linear_edges(0, 200, nb) if layout == "linear" else synth.log_edges(0.1, 200, nb)
        plan = fcfc.Plan("s", e, box=800.0)
        plan.bin_squared(v)
        ms = []
        for _ in range(repeats):
            plan.bin_squared(v)
            ms.append(plan.stats()["kernel_ms"])
        st = plan.stats()
        k = float(np.mean(ms))
        gbs = 8.0 * n / (k * 1e-3) / 1e9
        rows.append({"bins": nb, "layout": layout, "kernel_ms": k, "kernel_ms_sd": float(np.std(ms)),
                     "values_per_s": n / (k * 1e-3), "ps_per_value": k * 1e9 / n,
                     "hbm_gbps": gbs, "hbm_frac": gbs / 8000.0, "rechecks": int(st["rechecks"]),
                     "in_range": int(st["in_range"]), "lut_entries": int(st["lut_entries"])})
        plan.close()
    scan = []
    e = synth.log_edges(0.1, 200, 200)
    for lg in (8, 9, 10, 11, 12, 13, 14):
        plan = fcfc.Plan("s", e, box=800.0, lut_log2=lg)
        plan.bin_squared(v)
        ms = []
        for _ in range(3):
            plan.bin_squared(v)
            ms.append(plan.stats()["kernel_ms"])
        st = plan.stats()
        scan.append({"lut_log2": lg, "lut_entries": int(st["lut_entries"]), "kernel_ms": float(np.mean(ms)),
                     "recheck_rate": st["rechecks"] / n})
        plan.close()
    # CPU baseline: the oracle on a bounded sample of the same values
    sample = v[:cpu_values].cpu().numpy() if cpu else None
    del v
    torch.cuda.empty_cache()
    cpu_rows = []
    if cpu:
        from oracle import histogram as H
    for layout, nb in (BIN_LAYOUTS if cpu else ()):
        e = synth.linear_edges(0, 200, nb) if layout == "linear" else synth.log_edges(0.1, 200, nb)
        t0 = time.perf_counter()
        H.bin_squared(sample, e)
        cpu_rows.append({"bins": nb, "layout": layout, "values_per_s": len(sample) / (time.perf_counter() - t0)})
    return {
        "workload": f"{n} squared separations s^2 = x^(2/3) 200^2 (x uniform, App. C), FP64, resident in HBM",
        "kernel": "k_bin_squared",
        "roofline": {"bound": "hbm", "per_unit": "8 B per value (read once)", "peak": 8000.0, "unit": "GB/s",
                     "traffic": (measured_traffic("binning/6.4e9", ("binning.hip", "binlut.h"), "src_sha256_16")
                                 if n == 6_400_000_000 else None)},
        "layouts": rows,
        "lut_scan_log200": scan,
        "cpu_baseline": ({"kind": "oracle", "sample": f"first {cpu_values} values", "rows": cpu_rows,
                          "unit": "values/s", "cores": 1, "note": "numpy, one comparison pass per edge"}
                         if cpu else None),
        "paper_context": "about 2 ns per update on one Haswell core (scalar), not this machine",
    }


PEAK_FP64_TFLOPS = 78.6
FLOP_PER_SIDE = 8  # 3 sub, 3 mul, 2 add of one FP64 squared separation


def triplets_section(fcfc, synth, torch, n=2_000_000, L=1000.0, rmax=30.0, nbins=15, repeats=3, cpu=True):
    """Triangle counts (three-point extension): n uniform points in a periodic
    box, sides binned in nbins linear bins over [0, rmax).  Kernel time over
    HIP events on the launch stream; roofline of the FP64 side evaluations
    against the FP64 vector peak; the oracle (neighbour lists, all host cores)
    on a periodic sub-box of the same density for scale."""
    x = torch.from_numpy(synth.uniform_box(n, L, synth.config_seed(7))).cuda()
    e = synth.linear_edges(0, rmax, nbins)
    plan = fcfc.Plan("s", e, box=L, n_hint=n)
    cells = plan.build_cells(x)
    plan.count_triplets(cells)
    ms = []
    for _ in range(repeats):
        h, _ = plan.count_triplets(cells)
        ms.append(plan.stats()["kernel_ms"])
    st = plan.stats()
    tri = int(h.sum().item())
    k = float(np.mean(ms))
    sides = int(st["candidates"])
    achieved = FLOP_PER_SIDE * sides / (k * 1e-3) / 1e12
    cells.close()
    # weighted: weights U[0.5, 1.5]
    wt = torch.from_numpy(synth.uniform_weights(n, 0.5, 1.5, synth.config_seed(7) + 2)).cuda()
    cw = plan.build_cells(x, wt)
    plan.count_triplets(cw, weighted=True)
    msw = []
    for _ in range(repeats):
        hw, ww = plan.count_triplets(cw, weighted=True)
        msw.append(plan.stats()["kernel_ms"])
    same = bool(torch.equal(hw, h))
    cw.close()
    plan.close()
    # CPU baseline: the oracle on a periodic sub-box of the same density
    Ls = 200.0
    ns = int(round(n * (Ls / L) ** 3))
    base = None
    if cpu:
        import oracle
        xs = synth.uniform_box(ns, Ls, synth.config_seed(7) + 1)
        t0 = time.perf_counter()
        ref = oracle.triplets(xs, edges=e, box=Ls)
        cpu_s = time.perf_counter() - t0
        base = {"kind": "oracle", "sample": f"{ns} points in a periodic box {Ls:g} (same density)",
                "seconds": cpu_s, "triangles": int(ref.sum()), "value": int(ref.sum()) / cpu_s,
                "unit": "triangles/s", "cores": int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)}
    return {
        "workload": f"{n} uniform points, periodic box {L:g}, {nbins} linear side bins over [0, {rmax:g})",
        "kernel": "k_triplets", "kernel_ms": k, "kernel_ms_sd": float(np.std(ms)),
        "triangles": tri, "triangles_per_s": tri / (k * 1e-3),
        "side_evaluations": sides, "side_evaluations_per_s": sides / (k * 1e-3),
        "rechecks": int(st["rechecks"]),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "per_unit": f"{FLOP_PER_SIDE} FP64 flops per side evaluation"},
        "weighted": {"weights": "U[0.5, 1.5]", "kernel_ms": float(np.mean(msw)), "kernel_ms_sd": float(np.std(msw)),
                     "counts_equal_unweighted": same},
        "cpu_baseline": base,
    }


def c3_main(args, fcfc, torch):
    """C3 (open box, mid-point line of sight): DD and DR (and RR) per step."""
    weighted = not args.unweighted
    w, desc = workload("c3", weighted)
    dev = torch.device("cuda:0")
    d = torch.from_numpy(w["x1"]).to(dev)
    r = torch.from_numpy(w["x2"]).to(dev)
    wd = torch.from_numpy(w["w1"]).to(dev) if weighted else None
    wr = torch.from_numpy(w["w2"]).to(dev) if weighted else None
    tune = {}
    for kv in filter(None, args.tune.split(",")):
        k, v = kv.split("=")
        tune[k] = int(v)
    tune.setdefault("n_hint", len(w["x2"]))

    def step():
        plan = fcfc.Plan("spi", w["edges1"], w["edges2"], los="mid", box=0.0, **tune)
        plan.fit_bounds([(d, None), (r, None)])
        cd = plan.build_cells(d, wd)
        cr = plan.build_cells(r, wr)
        st = {}
        plan.count(cd, weighted=weighted)
        st["DD"] = plan.stats()
        plan.count(cd, cr, weighted=weighted)
        st["DR"] = plan.stats()
        if args.c3_rr:
            plan.count(cr, weighted=weighted)
            st["RR"] = plan.stats()
        cd.close()
        cr.close()
        plan.close()
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    pairs = sum(int(v["in_range"]) for v in st.values())
    dr = st["DR"]
    achieved = FLOP_PER_DISTANCE * dr["candidates"] / (dr["kernel_ms"] * 1e-3) / 1e12
    res = {
        "metric": "exact pairs/s (1 GPU, % FP32 roofline); mocks/s batched+learned vs plain",
        "value": pairs / (ms_step * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": desc, "data_points": len(w["x1"]), "random_points": len(w["x2"]),
                   "bins": 40 * 40, "weighted": bool(weighted), "tuning": tune},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None, "kernel": "k_count (DR)",
                     "kernel_ms": dr["kernel_ms"], "per_unit": f"{FLOP_PER_DISTANCE} flop per distance evaluation",
                     "units_per_launch": int(dr["candidates"])},
        "detail": {name: {"in_range_pairs": int(v["in_range"]), "distance_evaluations": int(v["candidates"]),
                          "kernel_ms": v["kernel_ms"], "kernel_pairs_per_s": v["in_range"] / (v["kernel_ms"] * 1e-3),
                          "candidates_per_pair": v["candidates"] / max(v["in_range"], 1),
                          "recheck_rate": v["rechecks"] / max(v["candidates"], 1), "grid": v["grid"],
                          "group_waves": v["group_waves"]} for name, v in st.items()},
    }
    print(json.dumps(res), flush=True)


def c3_section(fcfc, synth, torch, rr_shards=8):
    """C3 at full size in the default run: the survey shell's DD, DR and RR
    (2,000,000 data, 40,000,000 randoms, weighted (s_perp, pi) 40 x 40, mid-point
    line of sight, open box), each counted once after one DD warm-up.  RR is
    counted as rr_shards launches over disjoint shards of its work list (items
    i % G == g), whose histograms sum exactly to the whole count; a progress
    line follows each shard."""
    w = synth.workload(3, weighted=True)
    dev = torch.device("cuda:0")
    d = torch.from_numpy(w["x1"]).to(dev)
    r = torch.from_numpy(w["x2"]).to(dev)
    wd = torch.from_numpy(w["w1"]).to(dev)
    wr = torch.from_numpy(w["w2"]).to(dev)
    kw = dict(los="mid", box=0.0, n_hint=len(w["x2"]))
    plan = fcfc.Plan("spi", w["edges1"], w["edges2"], **kw)
    plan.fit_bounds([(d, None), (r, None)])
    builds = {}
    cells = {}
    for name, x, wt in (("data", d, wd), ("randoms", r, wr)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        cells[name] = plan.build_cells(x, wt)
        e1.record()
        torch.cuda.synchronize()
        builds[name] = e0.elapsed_time(e1)
    plan.count(cells["data"], weighted=True)  # warm-up
    out = {}

    def entry(st, kernel_ms, note=None):
        achieved = FLOP_PER_DISTANCE * st["candidates"] / (kernel_ms * 1e-3) / 1e12
        e = {"in_range_pairs": int(st["in_range"]), "distance_evaluations": int(st["candidates"]),
             "kernel_ms": kernel_ms, "kernel_pairs_per_s": st["in_range"] / (kernel_ms * 1e-3),
             "candidates_per_pair": st["candidates"] / max(st["in_range"], 1),
             "rechecks": int(st["rechecks"]), "recheck_rate": st["rechecks"] / max(st["candidates"], 1),
             "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                          "frac": achieved / PEAK_FP32_TFLOPS}}
        if note:
            e["note"] = note
        return e

    grid_hist = {}
    walls = {}
    walls["DD"], (c, wc) = _sync_time(lambda: plan.count(cells["data"], weighted=True))
    grid_hist["DD"] = (c.clone(), wc.clone())
    out["DD"] = entry(plan.stats(), plan.stats()["kernel_ms"])
    log(f"C3 DD: {out['DD']['kernel_ms']:.1f} ms")
    walls["DR"], (c, wc) = _sync_time(lambda: plan.count(cells["data"], cells["randoms"], weighted=True))
    grid_hist["DR"] = (c.clone(), wc.clone())
    st = plan.stats()
    out["DR"] = entry(st, st["kernel_ms"])
    log(f"C3 DR: {out['DR']['kernel_ms']:.0f} ms; RR in {rr_shards} shards next "
        f"(about {10 * out['DR']['kernel_ms'] / 1e3:.0f} s)")
    plan.close()
    for cl in cells.values():
        cl.close()
    # the same DD and DR through the k-d tree (leaves of 128 points)
    tree = {"leaf_points": 128}
    tplan = fcfc.Plan("spi", w["edges1"], w["edges2"], tree_leaf=128, **kw)
    tplan.fit_bounds([(d, None), (r, None)])
    tcells = {}
    tb = {}
    for name, x, wt in (("data", d, wd), ("randoms", r, wr)):
        tb[name], tcells[name] = _sync_time(lambda: tplan.build_cells(x, wt))
    tree["build_ms"] = tb
    tree["grid_build_ms"] = builds
    for name, args in (("DD", (tcells["data"],)), ("DR", (tcells["data"], tcells["randoms"]))):
        wall, (c, wc) = _sync_time(lambda: tplan.count(*args, weighted=True))
        st = tplan.stats()
        g_c, g_wc = grid_hist[name]
        tree[name] = dict(entry(st, st["kernel_ms"]), wall_ms=wall, items=int(st["items"]),
                          grid_wall_ms=walls[name], grid_kernel_ms=out[name]["kernel_ms"],
                          grid_distance_evaluations=out[name]["distance_evaluations"],
                          equal_to_grid=bool(torch.equal(c, g_c) and torch.equal(wc, g_wc)))
        log(f"C3 {name} tree: kernel {st['kernel_ms']:.1f} ms (grid {out[name]['kernel_ms']:.1f}), "
            f"wall {wall:.1f} ms (grid {walls[name]:.1f}), equal {tree[name]['equal_to_grid']}")
    for cl in tcells.values():
        cl.close()
    tplan.close()
    del grid_hist
    tot = {"in_range": 0, "candidates": 0, "rechecks": 0}
    kms = 0.0
    hist = None
    for g in range(rr_shards):
        ps = fcfc.Plan("spi", w["edges1"], w["edges2"], shard_count=rr_shards, shard_index=g, **kw)
        ps.fit_bounds([(d, None), (r, None)])
        cr = ps.build_cells(r, wr)
        c, wc = ps.count(cr, weighted=True)
        sg = ps.stats()
        hist = c.clone() if hist is None else hist + c
        for k in tot:
            tot[k] += int(sg[k])
        kms += sg["kernel_ms"]
        cr.close()
        ps.close()
        log(f"C3 RR shard {g + 1}/{rr_shards}: {sg['kernel_ms']:.0f} ms")
    tot["in_range"] = int(hist.sum())
    out["RR"] = entry(tot, kms, note=f"{rr_shards} launches over disjoint shards of the work list; "
                                     "kernel_ms is their sum, the histograms sum to the whole RR count")
    del d, r, wd, wr
    torch.cuda.empty_cache()
    return {"workload": "C3 open survey shell r in [1000,2000], RA 60 deg x Dec 30 deg, data 2,000,000 + "
                        "randoms 40,000,000, weighted (s_perp,pi) 40x40 over [0,200), mid-point LOS",
            "build_ms": builds, "counts": out, "tree": tree}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import torch
    from paper_2301_12557_amd import fcfc

    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "c3":
        c3_main(args, fcfc, torch)
        return
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
    log(f"{args.workload}: warmup done")
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
                   "wg_per_cu": stats["wg_per_cu"], "group_waves": stats["group_waves"],
                   "lut_entries": stats["lut_entries"],
                   "band_d2_rel": stats["band_d2_rel"], "device": torch.cuda.get_device_name(0)},
    }
    # the build (a1-a5) is HBM-bound: its algorithmic bytes are the inputs read
    # once and the sorted outputs written once, over HIP events on its stream
    # (which include the one synchronisation the build makes)
    bms = []
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        cb = plan.build_cells(x, wt)
        e1.record()
        torch.cuda.synchronize()
        bms.append(e0.elapsed_time(e1))
        cb.close()
    per_point = 24 + 16 + 24 + 4 + (16 if weighted else 0)
    build_bytes = per_point * len(x) + 4 * (int(np.prod(stats["grid"])) + 1)
    build_ms = float(min(bms))
    res["build_roofline"] = {"bound": "hbm", "achieved": build_bytes / (build_ms * 1e-3) / 1e9, "peak": 8000.0,
                             "unit": "GB/s", "frac": build_bytes / (build_ms * 1e-3) / 8e12, "ms": build_ms,
                             "algorithmic_bytes": build_bytes,
                             "per_unit": f"{per_point} B per point (positions{' and weights' if weighted else ''} "
                                         "read once; FP32 cell-local, FP64, key"
                                         f"{', weights' if weighted else ''} written once) + 4 B per cell"}
    log(f"build: {build_ms:.3f} ms, {res['build_roofline']['achieved']:.0f} GB/s")
    if args.shards > 1:
        G = args.shards
        cells = plan.build_cells(x, wt)
        sk, tot = [], None
        for g in range(G):
            ps = fcfc.Plan(w["kind"], w["edges1"], w["edges2"], los=w["los"], box=w["box"],
                           **dict(tune, shard_count=G, shard_index=g))
            cs = ps.build_cells(x, wt)
            best = np.inf
            for _ in range(3):
                c, _ = ps.count(cs, weighted=weighted)
                best = min(best, ps.stats()["kernel_ms"])
            tot = c.clone() if tot is None else tot + c
            sk.append(best)
            cs.close()
            ps.close()
        cells.close()
        res["shards"] = {"count": G, "kernel_ms": sk, "max_kernel_ms": max(sk),
                         "whole_kernel_ms": kernel_ms, "balance": float(np.mean(sk) / max(sk)),
                         "sum_equals_whole": bool(torch.equal(tot.reshape(-1), out.reshape(-1))),
                         "note": "each shard counted alone on this GPU, at its real shape; no multi-GPU time"}
        log(f"shards: max {max(sk):.3f} ms of whole {kernel_ms:.3f} ms")
    if not args.no_peaks:
        pk = fcfc.diag_peaks()
        kernel_s = kernel_ms * 1e-3
        atomic_time = pairs * (1.0 / pk["lds_u32_per_s"] + (2.0 / pk["lds_u64_per_s"] if weighted else 0.0))
        res["roofline"]["measured_peaks"] = {
            "fp32_fma_tflops_nonpacked": pk["fma_tflops"],
            "note": "one FMA per lane per instruction; the published 157.3 TFLOP/s counts packed FP32",
            "copy_gbps": pk["copy_gbps"], "lds_add_u32_per_s": pk["lds_u32_per_s"],
            "lds_add_u64_per_s": pk["lds_u64_per_s"]}
        res["lds_atomic_roofline"] = {
            "atomics_per_pair": "1 ds_add_u32" + (" + 2 ds_add_u64" if weighted else ""),
            "atomic_time_ms_at_peak": atomic_time * 1e3, "kernel_ms": kernel_ms,
            "frac": atomic_time / kernel_s}
        log(f"measured peaks: {pk}")
    if args.workload == "c2" and not args.no_fixed:
        from paper_2301_12557_amd import synth
        res["fixed_axis"] = fixed_axis_section(fcfc, synth, torch, x)
        log("fixed-axis workloads: " + " ".join(f"{k} {v['kernel_ms']:.2f} ms ({v['roofline']['frac']:.3f})"
                                                for k, v in res["fixed_axis"].items()))
    if not (args.no_c4 and args.no_learned):
        from paper_2301_12557_amd import synth
        mocks = make_mocks(synth, args.c4_mocks)
        log(f"generated {len(mocks)} C4 mocks")
        model, train = (None, None)
        if not args.no_learned:
            w2 = w if args.workload == "c2" else synth.workload(2)
            x2 = x if args.workload == "c2" else torch.from_numpy(w2["x1"]).to(dev)
            model, train = train_cost_model(fcfc, synth, x2, w2, mocks)
            res["learned"] = {"training": train}
            log(f"cost model trained on {train['samples']} items, loss {train['final_loss']:.3f}")
        if not args.no_c4:
            res["c4"] = c4_section(fcfc, synth, mocks, model, args.c4_repeats)
            log(f"C4 mocks/s: " + " ".join(f"{k} {v['mocks_per_s']:.1f}" for k, v in res['c4']['arms'].items()))
        del mocks
        torch.cuda.empty_cache()
        if not args.no_learned:
            res["learned"]["c5_heldout"] = c5_section(fcfc, synth, model)
            log("C5 held-out comparison done")
            res["learned"]["clustered_heldout"] = clustered_section(fcfc, synth, model)
            log("clustered held-out: " + " ".join(
                f"{k} analytic {v['analytic']['ms']:.2f} ms, search {v['search_without_model']['ms']:.2f}, "
                f"with model {v['search_with_model']['ms']:.2f}"
                for k, v in res["learned"]["clustered_heldout"].items() if k != "workload"))
    if not args.no_pairs:
        from paper_2301_12557_amd import synth
        res["pairs"] = pairs_section(fcfc, synth, torch)
        log(f"multi-tracer pairs: separate {res['pairs']['separate_ms']:.1f} ms, "
            f"one batch {res['pairs']['batch_ms']:.1f} ms, equal {res['pairs']['counts_equal']}")
    if not args.no_binning:
        from paper_2301_12557_amd import synth
        res["binning"] = binning_section(fcfc, synth, torch, args.binning_values, cpu=not args.no_cpu_baseline)
        log("binning: " + " ".join(f"{r['layout']}{r['bins']} {r['kernel_ms']:.2f} ms ({r['hbm_frac']:.2f})"
                                   for r in res["binning"]["layouts"]))
    if not args.no_triplets:
        from paper_2301_12557_amd import synth
        res["triplets"] = triplets_section(fcfc, synth, torch, cpu=not args.no_cpu_baseline)
        log(f"triplets: {res['triplets']['kernel_ms']:.2f} ms, {res['triplets']['triangles']} triangles, "
            f"{res['triplets']['roofline']['frac']:.3f} of FP64 peak")
    if not args.no_c3:
        from paper_2301_12557_amd import synth
        res["c3"] = c3_section(fcfc, synth, torch)
        log("C3: " + " ".join(f"{k} {v['kernel_ms']:.0f} ms ({v['roofline']['frac']:.3f})"
                              for k, v in res["c3"]["counts"].items()))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
