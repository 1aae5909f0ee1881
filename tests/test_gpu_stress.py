"""Stress and scale workloads (Sec. 9.2 families, a 3,677-aa synthetic design).

  * poly-S and alternating YI (no Met, no stop) at 32-128 aa against the dense oracle run here,
    and at 256 aa against stored oracle goldens (tests/golden/stress.json): these families keep
    far more candidates than random proteins, so the multiloop scan runs long lists;
  * a 3,677-aa synthetic protein (the length of the paper's largest design, Sec. 8.2), too large
    for the dense oracle: checked through properties that hold at any size -- the independent
    structure evaluator reproduces the reported energy, the fixed-point objective equals E * 2^s
    plus the codon costs recomputed from the emitted mRNA, the lambda exchange inequalities hold
    between lambda = 0 and 4, and the candidate count never exceeds the feasible direct cells.
"""
import json
import math
import os

import pytest

import oracle as O
import sdinputs as S

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def sd():
    import paper_2609_32308_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(sd):
    c = sd.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def gparams(sd, params_path):
    return sd.Params(params_path)


@pytest.fixture(scope="module")
def gtable(sd, weights):
    return sd.CodonTable(weights)


def family(name, A):
    return "S" * A if name == "S" else "YI" * (A // 2)


def same_as(r, d):
    assert r.energy == d["energy"] and r.objective_fixed == d["objective_fixed"]
    assert r.mrna == d["mrna"] and r.structure == d["structure"]
    assert r.n_candidates == d["n_candidates"]
    assert abs(r.objective_kcal - d["objective_kcal"]) <= 1e-9


@pytest.mark.parametrize("fam", ["S", "YI"])
@pytest.mark.parametrize("A", [32, 64, 128])
def test_stress_family_vs_oracle(fam, A, ctx, gtable, gparams, oparams, weights):
    p = family(fam, A)
    for lam in (0.0, 4.0):
        say("family", fam, A, lam)
        r = ctx.design(p, gtable, gparams, lam)
        d = O.design(p, weights, oparams, lam, nthreads=8)
        same_as(r, {"energy": d.energy, "objective_fixed": d.objective_fixed, "mrna": d.mrna,
                    "structure": d.structure, "n_candidates": d.n_candidates,
                    "objective_kcal": d.objective_kcal})
        assert r.n_visits == d.visits_sparse


def test_stress_family_256_goldens(ctx, gtable, gparams, params_path):
    path = os.path.join(HERE, "golden", "stress.json")
    gold = json.load(open(path))
    assert gold["params_sha256"] == S.sha256_file(params_path)
    assert len(gold["designs"]) == 4
    for d in gold["designs"]:
        say("family 256", d["seed"], d["lambda"])
        r = ctx.design(d["protein"], gtable, gparams, d["lambda"])
        same_as(r, d)
        assert r.n_visits == d["visits_sparse"]


def _round_half_away(x):
    r = math.floor(x)
    return r + 1 if x - r >= 0.5 else r


def test_scale_3677aa_properties(ctx, gtable, gparams, oparams, weights):
    p = S.protein(3677, 1)
    res = {}
    for lam in (0.0, 4.0):
        say("scale 3677", lam)
        r = ctx.design(p, gtable, gparams, lam)
        res[lam] = r
        assert len(r.mrna) == 3 * len(p) and len(r.structure) == len(r.mrna)
        # the emitted mRNA encodes the protein
        for k, aa in enumerate(p):
            assert r.mrna[3 * k:3 * k + 3] in S.GENETIC_CODE[aa]
        # independent loop-decomposition evaluator
        assert O.evaluate(r.mrna, r.structure, oparams) == r.energy
        # fixed-point objective = E * 2^s + sum of rounded codon costs, from the mRNA alone
        s = r.fixed_shift
        u = 0
        cost = 0.0
        for k in range(len(p)):
            q = -math.log(weights[S.codon_index(r.mrna[3 * k:3 * k + 3])])
            u += _round_half_away(math.ldexp(100.0 * lam * q, s))
            cost += q
        assert r.objective_fixed == r.energy * (1 << s) + u
        assert abs(r.codon_cost - cost) <= 1e-9 * max(1.0, cost)
        assert r.n_candidates <= r.n_feasible
    # lambda exchange: optimal codon cost does not grow, optimal energy does not fall
    assert res[4.0].codon_cost <= res[0.0].codon_cost + 1e-12
    assert res[4.0].energy >= res[0.0].energy
