"""Benchmark of the exact coding-sequence design DP on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload batch256|plain300|plain925_1976|scale|served|motifs] [--no-cpu-baseline]

A step is one pass of the whole path over one batch of synthetic input.  Inputs are protein
strings handed to the C ABI; the library builds the automaton, uploads it, fills the DP on the
GPU, runs the canonical traceback on the GPU and returns the result strings.
  batch256 (default): 256 proteins, lengths log-uniform in [50, 1000] aa (seed 7), the first 128
                     at lambda = 0 and the rest at lambda = 4, in one persistent, graph-captured
                     launch per step.  The same 256 designs are also run once in plain mode (one
                     span-step launch per span length) and once through the continuous-batching
                     server at saturation, and reported beside the batched rate;
  plain300:          one 300-aa synthetic protein (Met + 298 uniform residues + stop, seed 1),
                     designed at lambda = 0 and lambda = 4 in plain mode;
  plain925_1976:     the 925-aa and 1,976-aa proteins (seed 1) at lambda = 0 and 4, plain mode;
  scale:             one 3,677-aa protein (seed 1) at lambda = 0 and 4, plain mode;
  served:            a Poisson request stream through the continuous-batching server, with the
                     learned candidate sizer against worst-case sizing (see served_workload);
  motifs:            one 105-aa protein avoiding 16 random 6-mers at lambda = 0 and 4 (the
                     generic-lattice path).

`value` is DP cells per second of fill time, summed over the step's designs (a cell is a state
pair (a, b) with rho(a) < rho(b)); fill time is the cost-only interval of the method: device
allocation, the O(N) input upload and the forward fill, without automaton build and traceback.
`complete_cells_per_s` and `designs_per_min` use complete time (input strings to result
strings).  One JSON line is printed.

Roofline of the dominant kernel (the persistent launch for batch256, the span step for the plain
workloads): algorithmic HBM bytes per launch = (72 B per cell for the V/B/S1/S2 writes + 20 B
per candidate visit + 12 B per appended candidate) / launches, divided by the kernel's average
duration measured with HIP events on the library's stream.  `traffic` comes from the committed
rocprofv3 counter summary if it was taken on the current kernel source, else null.
`cpu_baseline` times the CPU oracle (test infrastructure, dense O(N^3) reference) on a bounded
sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import random
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock
BYTES_PER_CELL = 72    # V (6 x int64) + B + S1 + S2 written once per cell
BYTES_PER_VISIT = 20   # candidate start state (4) + B(c,b) (8) + gathered S1(a,c) (8)
BYTES_PER_APPEND = 12  # appended (c, B) entry
# HIP events bracket every 16th span-step launch of the timed steps (spans 1, 17, 33, ...): an
# event between two launches adds a gap, so timing every launch would slow the fill being timed
KERNEL_TIMING_EVERY = 16
METRIC = "DP cells/s + designs/min at lambda in {0,4}, batched/served vs plain, oracle-exact"


def workload(name):
    import sdinputs as S
    if name == "plain300":
        p = S.protein(300, 1)
        return [(p, 0.0), (p, 4.0)], {"workload": "plain design, one 300-aa synthetic protein (seed 1), lambda 0 and 4",
                                      "aa": 300, "lambdas": [0, 4], "mode": "plain"}
    if name == "plain925_1976":
        items = [(S.protein(A, 1), lam) for A in (925, 1976) for lam in (0.0, 4.0)]
        return items, {"workload": "plain design, synthetic 925-aa and 1976-aa proteins (seed 1), lambda 0 and 4",
                       "aa": [925, 1976], "lambdas": [0, 4], "mode": "plain"}
    if name == "scale":
        p = S.protein(3677, 1)
        return [(p, 0.0), (p, 4.0)], {"workload": "plain design, one 3677-aa synthetic protein (seed 1; the length of the paper's largest design), lambda 0 and 4",
                                      "aa": 3677, "lambdas": [0, 4], "mode": "plain"}
    if name == "batch256":
        lens = S.batch_lengths(256, 50, 1000, seed=7)
        items = [(S.protein(A, 7000 + i), 0.0 if i < 128 else 4.0) for i, A in enumerate(lens)]
        return items, {"workload": "batched design, 256 synthetic proteins log-uniform in [50,1000] aa (seed 7), "
                                   "128 at lambda 0 and 128 at lambda 4, one persistent graph-captured launch per step; "
                                   "the same designs in plain mode and served, beside it",
                       "proteins": 256, "aa_range": [50, 1000], "lambdas": [0, 4], "mode": "batch"}
    if name == "motifs":
        p = S.protein(105, 1)
        return [(p, 0.0), (p, 4.0)], {"workload": "forbidden-motif design, one 105-aa synthetic protein (seed 1) avoiding 16 random 6-mers (seed 7), lambda 0 and 4",
                                      "aa": 105, "motifs": S.motifs(16, 7), "lambdas": [0, 4], "mode": "plain, generic lattice"}
    raise SystemExit(f"unknown workload {name}")


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("sd_kernels.hip", "sd_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2609_32308_amd", "csrc", f), "rb").read())
    return h.hexdigest()


COUNTER_FILES = {"plain300": "k_span_plain300_counters.json", "batch256": "k_persistent_waves_batch256_counters.json",
                 "motifs": "k_gen_closed_motifs_105aa_counters.json"}


def profile_record(name):
    """Counter summary committed under profiles/, if taken on the current kernel source."""
    if name not in COUNTER_FILES:
        return None
    path = os.path.join(ROOT, "profiles", COUNTER_FILES[name])
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256") != kernel_source_sha():
        return None  # counters were taken on an older kernel
    return d


def run_step(ctx, items, table, params, batch, motifs=None):
    if motifs:
        return [ctx.design_motifs(p, motifs, table, params, lam) for p, lam in items]
    if batch:
        return ctx.design_batch([p for p, _ in items], [l for _, l in items], table, params)
    return [ctx.design(p, table, params, lam) for p, lam in items]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(items, motifs=None):
    """The oracle, as it stands, on the host cores: every design of the sample on all cores,
    then the first one on a single thread (bounded to about 10-30 s of CPU work)."""
    import oracle as O
    import sdinputs as S
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    P = O.Params(S.default_params_path())
    w = S.codon_weights(2026)
    sample = [(p, lam) for p, lam in items if len(p) <= 400]
    note = "the workload's designs"
    if not sample:
        # proteins too long for the dense O(N^3) oracle: 300-residue prefixes stand in
        sample = [(p[:300], lam) for p, lam in items[:2]]
        note = "300-residue prefixes of the workload's first designs"
    sample = sample[:2]
    cells = 0
    t = time.time()
    def run(p, lam, nt):
        if motifs:
            return O.design_motifs(p, w, P, lam, motifs, nthreads=nt).n_cells
        return O.design(p, w, P, lam, nthreads=nt).n_cells
    for p, lam in sample:
        cells += run(p, lam, threads)
    dt = time.time() - t
    p1, lam1 = sample[0]
    if motifs:
        p1 = p1[:60]  # the single-thread leg on a 60-residue prefix keeps it to about 10 s
    t = time.time()
    c1 = run(p1, lam1, 1)
    dt1 = time.time() - t
    return {"value": cells / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"dense oracle{' (motif product lattice)' if motifs else ''} on {note}: {len(sample)} design(s) of {len(sample[0][0])} aa "
                      f"({cells} cells, {dt:.2f} s on {threads} threads); single thread {c1 / dt1:.4g} cells/s "
                      f"({dt1:.2f} s{', 60-residue prefix' if motifs else ''})",
            "single_thread_value": c1 / dt1, "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count()}


def per_design_stats(items, results):
    out = {}
    for (p, lam), r in list(zip(items, results))[:4]:
        n = 3 * len(p)
        out[f"{len(p)}aa_lambda{lam:g}"] = {
            "energy": r.energy, "objective_kcal": r.objective_kcal, "Z": r.n_candidates,
            "Z_over_n2": r.n_candidates / n ** 2, "Z_over_B_finite": r.n_candidates / max(r.n_feasible, 1),
            "visits": r.n_visits, "cells": r.n_cells, "t_fill_s": r.t_fill_s, "t_total_s": r.t_total_s}
    return out


def roofline_for(results_steps, counters, batch, kernel=None):
    alg_bytes = launches = timed = ktime = 0.0
    for step in results_steps:
        for r in step:
            alg_bytes += BYTES_PER_CELL * r.n_cells + BYTES_PER_VISIT * r.n_visits + BYTES_PER_APPEND * r.n_candidates
            launches += r.n_span_launches
            timed += r.n_timed_launches
            ktime += r.t_span_kernels_s
        if batch:
            launches += 1  # one persistent launch per batched call, timed whole
            timed += 1
    avg_launch_s = ktime / timed if timed else float("nan")
    per_launch = alg_bytes / launches if launches else 0.0
    achieved = per_launch / avg_launch_s / 1e9 if ktime > 0 else 0.0
    roof = {"bound": "hbm", "kernel": kernel or ("k_persistent" if batch else "k_span"), "achieved": achieved, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "traffic": counters.get("hbm_bytes_per_launch") if counters else None,
            "alg_bytes_per_launch": per_launch, "avg_launch_us": avg_launch_s * 1e6, "launches": int(launches),
            "timed_launches": int(timed)}
    if counters and counters.get("valu_insts_per_launch"):
        lane_ops = counters["valu_insts_per_launch"] * 64
        roof["valu_lane_ops_per_launch"] = lane_ops
        roof["valu_frac"] = lane_ops / avg_launch_s / PEAK_VALU_LANE_OPS
    return roof


def progress(msg):
    print(msg, file=sys.stderr, flush=True)


def side_legs(sd, items, table, params, batched_results, batched_elapsed_per_step):
    """The batch's own designs in plain mode (one pass) and through the server at saturation
    (one pass, worst-case candidate sizing, all requests submitted at once), each checked to give
    the batched designs, with their rates beside the batched ones."""
    cells = sum(r.n_cells for r in batched_results)
    key = lambda r: (r.energy, r.objective_fixed, r.mrna, r.structure)
    ctx = sd.Context(0)
    t0 = time.perf_counter()
    plain = []
    for i, (p, lam) in enumerate(items):
        plain.append(ctx.design(p, table, params, lam))
        if i % 64 == 63:
            progress(f"plain leg {i + 1}/{len(items)}")
    t_plain = time.perf_counter() - t0
    ctx.close()
    per_lam = {}
    for lam in sorted({l for _, l in items}):
        rs = [r for (p, l), r in zip(items, plain) if l == lam]
        per_lam[f"lambda{lam:g}"] = {"designs": len(rs), "fill_cells_per_s": sum(r.n_cells for r in rs) / sum(r.t_fill_s for r in rs),
                                     "complete_cells_per_s": sum(r.n_cells for r in rs) / sum(r.t_total_s for r in rs)}
    plain_fill = sum(r.t_fill_s for r in plain)
    out = {"plain": {"fill_cells_per_s": cells / plain_fill, "complete_cells_per_s": cells / t_plain,
                     "designs_per_min": len(items) / t_plain * 60.0, "fill_s": plain_fill, "complete_s": t_plain,
                     "per_lambda": per_lam,
                     "identical_to_batched": all(key(a) == key(b) for a, b in zip(plain, batched_results))}}
    progress("plain leg done")
    ctx = sd.Context(0)
    srv = sd.Server(ctx, table, params, pool_bytes=64 << 30, max_active=len(items), steps_per_round=64)
    t0 = time.perf_counter()
    tickets = [srv.submit(p, lam) for p, lam in items]
    served = [srv.wait(t) for t in tickets]
    t_srv = time.perf_counter() - t0
    st = srv.stats()
    srv.stop()
    ctx.close()
    lat = sorted(r.t_total_s for r in served)
    out["served_saturated"] = {
        "designs_per_min": len(items) / t_srv * 60.0, "complete_cells_per_s": cells / t_srv,
        "p50_s": lat[len(lat) // 2], "p99_s": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)],
        "rounds": st["rounds"], "peak_active": st["peak_active"], "fallbacks": st["fallbacks"],
        "pool_gib": 64, "identical_to_batched": all(key(a) == key(b) for a, b in zip(served, batched_results)),
        "all_persistent": all(r.path == sd.PATH_PERSISTENT for r in served)}
    progress("served leg done")
    out["batched_over_plain"] = {"fill": (cells / sum(r.t_fill_s for r in batched_results)) / (cells / plain_fill),
                                 "complete": t_plain / batched_elapsed_per_step}
    out["served_over_plain_complete"] = t_plain / t_srv
    return out


def served_workload(args, sd, S):
    """Continuous-batching server on a Poisson stream, learned sizer against worst-case sizing.

    Requests: lengths log-uniform in [50, 2000] aa, lambda uniform in {0, 4}, protein seeds
    200000 + i, arrival times from a seeded exponential.  The sizer is trained on the exact
    DP's own occupancy logs of synthetic proteins (seeds 100000 + i, same length law, both
    lambdas), 10 % held out.  The plain GPU DP on the same requests, one after another, gives
    the capacity that sets the offered load and the designs every served result must equal.

    A full run (2,000 requests, loads 0.5 / 0.8 / 0.95 and saturation, both policies) takes
    longer than one GPU call here, so it can be split: --save-sizer / --load-sizer keep the
    trained parameters between calls, --loads and --policies pick the runs, and --capacity
    reuses a measured plain capacity (the plain designs are then not recomputed, and served
    results are compared with a stored digest of them, --plain-digest).
    """
    import numpy as np
    params = sd.Params(S.default_params_path())
    table = sd.CodonTable(S.codon_weights(2026))
    ctx = sd.Context(0)
    nreq, ntrain, K = args.requests, args.train_proteins, 8
    sizer = sd.Sizer(ctx, 64, K, seed=11)
    sizer_info = {"train_proteins": ntrain, "train_aa_range": [50, 2000], "bins": K, "hidden": 64}
    if args.load_sizer:
        sizer.set_params(np.load(args.load_sizer))
        sizer_info["loaded_from"] = os.path.basename(args.load_sizer)
    else:
        # learned sizer: exact occupancy logs -> FP32 MLP trained on the GPU
        tl = S.batch_lengths(ntrain, 50, 2000, seed=100000)
        train = [S.protein(A, 100000 + i) for i, A in enumerate(tl)]
        tlam = [0.0 if i % 2 == 0 else 4.0 for i in range(ntrain)]
        t = time.time()
        Ys = []
        for i in range(0, ntrain, 100):  # chunks, so that a long log reports progress
            Ys.append(ctx.occupancy(train[i:i + 100], tlam[i:i + 100], table, params, K)[0])
            progress(f"occupancy log {min(ntrain, i + 100)}/{ntrain}")
        Y = np.concatenate(Ys)
        t_log = time.time() - t
        progress(f"occupancy log of {ntrain} proteins: {t_log:.1f} s")
        X = np.stack([sd.features(p, l) for p, l in zip(train, tlam)]).astype(np.float32)
        cut = int(0.9 * ntrain)
        t = time.time()
        sizer.train(X[:cut], Y[:cut], steps=2000, lr=3e-3)
        t_train = time.time() - t
        held = float(np.mean((sizer.predict(X[cut:]) - Y[cut:]) ** 2))
        progress(f"sizer trained in {t_train:.1f} s, held-out MSE {held:.3g}")
        sizer_info.update({"occupancy_log_s": t_log, "train_s": t_train, "heldout_mse": held})
        if args.save_sizer:
            np.save(args.save_sizer, sizer.get_params())
    # request stream
    rl = S.batch_lengths(nreq, 50, 2000, seed=11)
    rng = random.Random(11)
    reqs = [(S.protein(A, 200000 + i), rng.choice([0.0, 4.0])) for i, A in enumerate(rl)]
    key = lambda r: f"{r.energy}|{r.objective_fixed}|{r.mrna}|{r.structure}"
    if args.capacity > 0:
        capacity, t_plain, plain = args.capacity, None, None
        digest = args.plain_digest
        cells_total = None
    else:
        t = time.time()
        plain = []
        for i, (p, lam) in enumerate(reqs):
            plain.append(ctx.design(p, table, params, lam))
            if i % 20 == 19:
                progress(f"plain {i + 1}/{nreq}")
        t_plain = time.time() - t
        capacity = nreq / t_plain  # designs/s, plain, one after another
        digest = hashlib.sha256("\n".join(key(r) for r in plain).encode()).hexdigest()
    ctx.close()
    lat_plain = sorted(r.t_total_s for r in plain) if plain else None

    def serve(policy, rho):
        c = sd.Context(0)
        if policy == "mlp":
            c.set_sizer(sizer, margin=0.5, slack=8)
        srv = sd.Server(c, table, params, pool_bytes=args.pool_gib << 30, max_active=256, steps_per_round=64)
        arng = random.Random(12)
        t0 = time.perf_counter()
        tickets, t_sub = [], []
        next_t = 0.0
        for i, (p, lam) in enumerate(reqs):
            if rho > 0:
                next_t += arng.expovariate(rho * capacity)
                dt = t0 + next_t - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            t_sub.append(time.perf_counter() - t0)
            tickets.append(srv.submit(p, lam))
            if i % 50 == 49:  # paced arrivals take minutes at low load: report them as they go
                progress(f"submitted {policy} load {rho}: {i + 1}/{nreq}")
        res = []
        for i, tk in enumerate(tickets):
            res.append(srv.wait(tk))
            if i % 50 == 49:
                progress(f"served {policy} load {rho}: {i + 1}/{nreq}")
        st = srv.stats()
        srv.stop()
        c.close()
        lat = sorted(r.t_total_s for r in res)
        done = max(ts + r.t_total_s for ts, r in zip(t_sub, res))
        cells = sum(r.n_cells for r in res)
        same = hashlib.sha256("\n".join(key(r) for r in res).encode()).hexdigest() == digest
        return {"policy": policy, "offered_load": rho if rho > 0 else "saturated",
                "designs_per_min": nreq / done * 60.0, "cells_per_s": cells / done,
                "p50_s": lat[len(lat) // 2], "p99_s": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)],
                "peak_active": st["peak_active"], "fallbacks": st["fallbacks"], "rounds": st["rounds"],
                "reserved_bytes_per_request": st["reserved_bytes"] / nreq,
                "reserved_cand_bytes_per_request": st["reserved_cand_bytes"] / nreq,
                "pool_high_water": st["pool_high_water"], "gpu_busy_frac": st["gpu_seconds"] / done,
                "identical_to_plain": same,
                "all_persistent": all(r.path == sd.PATH_PERSISTENT for r in res)}

    runs = []
    for rho in args.loads:
        for policy in args.policies:
            runs.append(serve(policy, rho))
            progress(f"run {policy} {rho}: {runs[-1]['designs_per_min']:.1f} designs/min")
    head = runs[0]
    line = {
        "metric": METRIC, "value": head["cells_per_s"], "unit": "cells/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": nreq / head["designs_per_min"] * 60.0 * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"served: {nreq} requests, lengths log-uniform in [50,2000] aa, lambda in {{0,4}}, "
                               f"Poisson arrivals, pool {args.pool_gib} GiB", "requests": nreq,
                   "aa_range": [50, 2000], "mode": "served"},
        "plain_sequential": {"designs_per_min": capacity * 60.0, "capacity_designs_per_s": capacity,
                             "cells_per_s": (sum(r.n_cells for r in plain) / t_plain) if plain else None,
                             "p50_s": lat_plain[nreq // 2] if plain else None, "measured_in_this_run": plain is not None,
                             "results_digest": digest},
        "served_runs": runs,
        "sizer": sizer_info,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch256", choices=["batch256", "plain300", "plain925_1976", "scale", "served", "motifs"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side-legs", action="store_true",
                    help="batch256: skip the plain and served passes after the timed steps (profiling runs)")
    ap.add_argument("--retain-all", action="store_true",
                    help="plain workloads: also time the scalar-dense control (every finite direct "
                         "interval retained) and report its time and visit ratios to the sparse fill")
    ap.add_argument("--requests", type=int, default=100, help="served: number of requests")
    ap.add_argument("--train-proteins", type=int, default=120, help="served: proteins in the occupancy log")
    ap.add_argument("--pool-gib", type=int, default=8, help="served: device pool of the server")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.0, 0.8],
                    help="served: offered loads as fractions of the plain capacity (0: saturated)")
    ap.add_argument("--policies", nargs="+", default=["worst", "mlp"], choices=["worst", "mlp"],
                    help="served: candidate sizing policies to run at every load")
    ap.add_argument("--save-sizer", default="", help="served: write the trained sizer parameters (.npy)")
    ap.add_argument("--load-sizer", default="", help="served: use these sizer parameters instead of training")
    ap.add_argument("--capacity", type=float, default=0.0,
                    help="served: plain capacity in designs/s from an earlier run (skips the plain pass)")
    ap.add_argument("--plain-digest", default="", help="served: SHA-256 digest of the plain results of that run")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent designs would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib:
        import torch
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))
        return

    import paper_2609_32308_amd as sd
    import sdinputs as S

    if args.workload == "served":
        served_workload(args, sd, S)
        return
    items, config = workload(args.workload)
    batch = args.workload == "batch256"
    motifs = config.get("motifs")
    ctx = sd.Context(0, kernel_timing=KERNEL_TIMING_EVERY)
    params = sd.Params(S.default_params_path())
    table = sd.CodonTable(S.codon_weights(2026))
    last = None
    for i in range(args.warmup):
        last = run_step(ctx, items, table, params, batch, motifs)
        progress(f"warmup step {i + 1}/{args.warmup}")
    # the autotuners (batched schedule; plain span tiles per span band) explore one candidate per
    # call of a new size class: the timed steps start only once they have settled (untimed extra
    # calls if the warmup was shorter)
    extra = 0
    while (last is None or not all(r.sched_tuned for r in last)) and extra < 16:
        last = run_step(ctx, items, table, params, batch, motifs)
        extra += 1
        progress(f"untimed tuning step {extra}")
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(run_step(ctx, items, table, params, batch, motifs))
        if batch or i % 5 == 4:
            progress(f"timed step {i + 1}/{args.steps}")
    t1 = time.perf_counter()
    elapsed = t1 - t0
    step_cells = sum(r.n_cells for r in results[0])
    fill = sum(r.t_fill_s for s_ in results for r in s_)
    designs = len(items) * args.steps
    counters = profile_record(args.workload)
    kernel = "k_gen_closed+k_span_gen" if motifs else None
    if batch:
        # the persistent kernel the settled schedule ran; the committed counters count only if
        # they were taken on that kernel
        r0 = results[-1][0]
        kernel = "k_persistent_waves" if (r0.sched_item_waves == 1 and r0.sched_threads != 64) else "k_persistent"
        if counters and not counters.get("kernel", "").startswith(kernel + "<"):
            counters = None
    line = {
        "metric": METRIC,
        "value": step_cells * args.steps / fill,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": config,
        "complete_cells_per_s": step_cells * args.steps / elapsed,
        "designs_per_min": designs / elapsed * 60.0,
        "fill_ms_per_step": fill / args.steps * 1e3,
        "per_design": per_design_stats(items, results[-1]),
        "roofline": roofline_for(results, counters, batch, kernel),
        "params_sha256": params.sha256,
    }
    ctx.close()
    line["untimed_tuning_steps"] = extra
    if batch:
        line["batch"] = {"paths": sorted({r.path for r in results[-1]}),
                         "graph_captured": all(r.graph_captured == 1 for r in results[-1]),
                         "launch_s": sum(r.t_span_kernels_s for r in results[-1]),
                         "schedule": sorted({(r.sched_threads, r.sched_grid, r.sched_item_waves) for r in results[-1]}),
                         "schedule_settled": all(r.sched_tuned == 1 for s_ in results for r in s_)}
        if not args.no_side_legs:
            line.update(side_legs(sd, items, table, params, results[-1], elapsed / args.steps))
    if motifs:
        line["per_design"] = {k: dict(v, n_states=r.n_states) for (k, v), r in zip(line["per_design"].items(), results[-1])}
    if args.retain_all and not batch and not motifs:
        # scalar-dense control (Sec. 8.1 / Table 3): same designs, every finite B retained
        dctx = sd.Context(0, retain_all=True)
        run_step(dctx, items, table, params, False)
        dense = run_step(dctx, items, table, params, False)
        dctx.close()
        sparse = results[-1]
        fs, fd = sum(r.t_fill_s for r in sparse), sum(r.t_fill_s for r in dense)
        vs, vd = sum(r.n_visits for r in sparse), sum(r.n_visits for r in dense)
        assert all((a.mrna, a.structure, a.objective_fixed) == (b.mrna, b.structure, b.objective_fixed)
                   for a, b in zip(sparse, dense))
        line["scalar_dense_control"] = {"fill_s_sparse": fs, "fill_s_dense": fd, "time_ratio": fd / fs,
                                        "visits_sparse": vs, "visits_dense": vd, "visit_ratio": vd / max(vs, 1),
                                        "identical_designs": True}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(items, motifs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
