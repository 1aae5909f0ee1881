"""Write the oracle's designs for the larger seeded workloads to tests/golden/*.json.

Calls only oracle/ and sdinputs/ (the seeded generators); nothing here touches the GPU path.
The GPU parity tests compare against these files at sizes where running the dense oracle
inside a test would take minutes.

    python tests/golden/make_golden.py plain300 plain925_1976 [batch256] [stress] [motifs] [motifs_wide]

The stress families of Sec. 9.2 (poly-S and alternating YI, no Met and no stop) are keyed by
seed 0 (S) and seed -1 (YI).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import sdinputs as S  # noqa: E402

# the fixed-point range rule the stored designs were made under (the shift changes the stored
# objective_fixed, and designs made under another rule are not reused): per-pair energy bound
RULE = "pair-bound"

WORKLOADS = {
    "plain300": [(300, seed, lam) for seed in (1, 2, 3, 4) for lam in (0.0, 4.0)],
    "plain925_1976": [(925, 1, 0.0), (925, 1, 4.0), (1976, 1, 0.0), (1976, 1, 4.0)],
}


def batch_members():
    lens = S.batch_lengths(256, 50, 1000, seed=7)
    # member i: protein of length lens[i] from seed 7000 + i, lambda 0 for i < 128 else 4
    return [(A, 7000 + i, 0.0 if i < 128 else 4.0) for i, A in enumerate(lens)]


def stress_protein(A, seed):
    return "S" * A if seed == 0 else "YI" * (A // 2)


STRESS = [(256, fam, lam) for fam in (0, -1) for lam in (0.0, 4.0)]

# forbidden motifs: the 64- and 105-aa sizes of the finite-state constraint experiments, with an
# inventory of 16 random 6-mers (seed 7), and 300 aa as a larger case; "motifs_wide": 96 random
# 6- and 7-mers (seed 3) that widen a layer of the 60-aa automaton to 16 states, the kernel limit
MOTIF_SETS = {
    "motifs": (lambda: S.motifs(16, 7), [(A, 1, lam) for A in (64, 105, 300) for lam in (0.0, 4.0)]),
    "motifs_wide": (lambda: S.motifs(96, 3, 6, 7), [(60, 1, 0.0), (60, 1, 4.0)]),
}


def run(name, members, nthreads):
    params = S.default_params_path()
    P = O.Params(params)
    w = S.codon_weights(2026)
    path = os.path.join(HERE, f"{name}.json")
    out = {"params_sha256": S.sha256_file(params), "codon_seed": 2026, "fixed_point_rule": RULE,
           "designs": []}
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
        if old.get("params_sha256") == out["params_sha256"] and old.get("fixed_point_rule") == RULE:
            out = old
    done = {(d["A"], d["seed"], d["lambda"]) for d in out["designs"]}
    for (A, seed, lam) in members:
        if (A, seed, lam) in done:
            continue
        prot = stress_protein(A, seed) if name == "stress" else S.protein(A, seed)
        t = time.time()
        if name in MOTIF_SETS:
            out["motifs"] = MOTIF_SETS[name][0]()
            d = O.design_motifs(prot, w, P, lam, out["motifs"], nthreads=nthreads)
        else:
            d = O.design(prot, w, P, lam, nthreads=nthreads)
        dt = time.time() - t
        assert d.selfcheck_ok
        out["designs"].append({
            "A": A, "seed": seed, "lambda": lam, "protein": prot, "mrna": d.mrna,
            "structure": d.structure, "energy": d.energy, "objective_fixed": d.objective_fixed,
            "fixed_shift": d.fixed_shift, "codon_cost": d.codon_cost,
            "objective_kcal": d.objective_kcal, "n_states": d.n_states, "n_cells": d.n_cells,
            "n_feasible_direct": d.n_feasible_direct, "n_candidates": d.n_candidates,
            "visits_sparse": d.visits_sparse, "visits_dense": d.visits_dense,
            "oracle_seconds": round(dt, 3), "oracle_threads": nthreads,
        })
        with open(path + ".tmp", "w") as fh:
            json.dump(out, fh, indent=1)
        os.replace(path + ".tmp", path)
        print(name, A, seed, lam, round(dt, 1), flush=True)


if __name__ == "__main__":
    nthreads = int(os.environ.get("ORACLE_THREADS", "8"))
    for name in sys.argv[1:]:
        members = (batch_members() if name == "batch256" else STRESS if name == "stress"
                   else MOTIF_SETS[name][1] if name in MOTIF_SETS else WORKLOADS[name])
        run(name, members, nthreads)
