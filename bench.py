"""Benchmark of the exact coding-sequence design DP on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload config2|config3|batch]

A step is one pass of the whole path (input build, forward fill, canonical traceback, result
strings) over one batch of synthetic input:
  config2 (default): one 300-aa synthetic protein (Met + 298 uniform residues + stop, seed 1),
                     designed at lambda = 0 and lambda = 4 in plain mode (one span-step kernel
                     launch per span length);
  config3:           the 925-aa and 1,976-aa proteins at lambda = 0 and 4 (plain mode);
  batch:             256 proteins, lengths log-uniform in [50, 1000] aa, half at lambda = 0 and
                     half at lambda = 4, in one batched call.
`value` is DP cells per second over the timed steps (cells = state pairs (a, b) with
rho(a) < rho(b), summed over the step's designs).  One JSON line is printed.

Roofline of the dominant kernel (the span step): algorithmic HBM bytes per launch =
(72 B per cell for the V/B/S1/S2 writes + 20 B per candidate visit + 12 B per appended
candidate) / launches, divided by the kernel's average duration measured with HIP events on the
library's stream.  `traffic` comes from the committed rocprofv3 counter summary if it was taken
on the current kernel source, else null.  `cpu_baseline` times the CPU oracle (test
infrastructure, dense O(N^3) reference) on one design of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_CELL = 72    # V (6 x int64) + B + S1 + S2 written once per cell
BYTES_PER_VISIT = 20   # candidate start state (4) + B(c,b) (8) + gathered S1(a,c) (8)
BYTES_PER_APPEND = 12  # appended (c, B) entry
METRIC = "DP cells/s + designs/min at lambda in {0,4}, batched/served vs plain, oracle-exact"


def workload(name):
    import sdinputs as S
    if name == "config2":
        p = S.protein(300, 1)
        return [(p, 0.0), (p, 4.0)], {"workload": "plain design, one 300-aa synthetic protein (seed 1), lambda 0 and 4",
                                      "aa": 300, "lambdas": [0, 4], "mode": "plain"}
    if name == "config3":
        items = [(S.protein(A, 1), lam) for A in (925, 1976) for lam in (0.0, 4.0)]
        return items, {"workload": "plain design, synthetic 925-aa and 1976-aa proteins (seed 1), lambda 0 and 4",
                       "aa": [925, 1976], "lambdas": [0, 4], "mode": "plain"}
    if name == "batch":
        lens = S.batch_lengths(256, 50, 1000, seed=7)
        items = [(S.protein(A, 7000 + i), 0.0 if i < 128 else 4.0) for i, A in enumerate(lens)]
        return items, {"workload": "batched design, 256 synthetic proteins log-uniform in [50,1000] aa, half lambda 0 / half lambda 4",
                       "proteins": 256, "aa_range": [50, 1000], "mode": "batch"}
    raise SystemExit(f"unknown workload {name}")


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("sd_kernels.hip", "sd_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2609_32308_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_from_profiles(name):
    path = os.path.join(ROOT, "profiles", f"k_span_{name}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256") != kernel_source_sha():
        return None  # counters were taken on an older kernel
    return d.get("hbm_bytes_per_launch")


def run_step(ctx, items, table, params, batch):
    if batch:
        return ctx.design_batch([p for p, _ in items], [l for _, l in items], table, params)
    return [ctx.design(p, table, params, lam) for p, lam in items]


def cpu_baseline(items):
    import oracle as O
    import sdinputs as S
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    P = O.Params(S.default_params_path())
    w = S.codon_weights(2026)
    # bounded sample: the first design of the workload whose dense oracle finishes in ~30 s
    p, lam = min(items, key=lambda x: len(x[0]))
    if len(p) > 400:
        p = p[:300]  # a 300-residue prefix of the same protein keeps the sample bounded
    t = time.time()
    d = O.design(p, w, P, lam, nthreads=threads)
    dt = time.time() - t
    return {"value": d.n_cells / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"dense oracle, one design of {len(p)} aa at lambda={lam} ({d.n_cells} cells, {dt:.2f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config2", choices=["config2", "config3", "batch"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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

    items, config = workload(args.workload)
    batch = args.workload == "batch"
    ctx = sd.Context(0, kernel_timing=True)
    params = sd.Params(S.default_params_path())
    table = sd.CodonTable(S.codon_weights(2026))
    for _ in range(args.warmup):
        run_step(ctx, items, table, params, batch)
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(run_step(ctx, items, table, params, batch))
    t1 = time.perf_counter()
    elapsed = t1 - t0
    step_cells = sum(r.n_cells for r in results[0])
    designs = len(items) * args.steps
    value = step_cells * args.steps / elapsed
    # dominant kernel: the span step
    alg_bytes = launches = ktime = 0.0
    for step in results:
        for r in step:
            alg_bytes += BYTES_PER_CELL * r.n_cells + BYTES_PER_VISIT * r.n_visits + BYTES_PER_APPEND * r.n_candidates
            launches += r.n_span_launches
            ktime += r.t_span_kernels_s
    avg_launch_s = ktime / launches if launches else float("nan")
    per_launch = alg_bytes / launches if launches else 0.0
    achieved = per_launch / avg_launch_s / 1e9 if ktime > 0 else 0.0
    traffic = traffic_from_profiles(args.workload)
    line = {
        "metric": METRIC,
        "value": value,
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
        "designs_per_min": designs / elapsed * 60.0,
        "fill_cells_per_s": step_cells * args.steps / sum(r.t_fill_s for s_ in results for r in s_),
        "per_lambda": {str(lam): {"energy": r.energy, "objective_kcal": r.objective_kcal,
                                  "Z": r.n_candidates, "visits": r.n_visits, "t_fill_s": r.t_fill_s}
                       for (p, lam), r in list(zip(items, results[-1]))[:4]},
        "roofline": {"bound": "hbm", "kernel": "k_span", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": per_launch,
                     "avg_launch_us": avg_launch_s * 1e6, "launches": int(launches)},
    }
    ctx.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(items)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
