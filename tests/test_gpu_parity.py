"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element.

Integer results (energy, fixed-point objective, candidate counts, every cell of the tables) must
be bit-exact; the emitted mRNA and structure must be identical under the canonical tie-break;
the FP64 objective is computed from the identical design and must agree within 1e-9.
"""
import json
import os

import numpy as np
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


def same(r, d):
    assert r.energy == d.energy
    assert r.objective_fixed == d.objective_fixed
    assert r.fixed_shift == d.fixed_shift
    assert r.mrna == d.mrna
    assert r.structure == d.structure
    assert abs(r.objective_kcal - d.objective_kcal) <= 1e-9
    assert r.codon_cost == d.codon_cost


@pytest.mark.parametrize("A,seed", [(A, s) for A in (6, 7, 8) for s in (1, 2, 3)])
@pytest.mark.parametrize("lam", [0.0, 4.0])
def test_bruteforce_sizes(A, seed, lam, ctx, gtable, gparams, oparams, weights):
    p = S.protein(A, seed)
    say("bruteforce-size", p, lam)
    r = ctx.design(p, gtable, gparams, lam)
    d = O.design(p, weights, oparams, lam)
    same(r, d)
    assert r.objective_fixed == O.bruteforce(p, weights, oparams, lam)["best_fixed"]


_ORACLE_TABLES = {}


def oracle_tables(p, lam, oparams, weights):
    k = (p, lam)
    if k not in _ORACLE_TABLES:
        _ORACLE_TABLES[k] = O.design(p, weights, oparams, lam, tables=True)
    return _ORACLE_TABLES[k]


@pytest.fixture(scope="module", params=[(0, 0), (64, 0), (256, 0), (512, 0), (1024, 0), (256, 1)],
                ids=["tuned", "64", "256", "512", "1024", "256waves"])
def span_ctx(request, sd):
    # (0, 0): the library's per-span-band choice (its tuner explores every candidate tile on the
    # first designs of a length class); the others force one span kernel for every span
    # (k_span<64>: one wave, three job parts; <256>: three parts; <512>: four parts, 80-VGPR cap;
    # <1024>: six parts; k_span_waves<256>: every wave on its own layer pair)
    threads, waves = request.param
    c = sd.Context(0, span_threads=threads, span_item_waves=waves)
    yield c
    c.close()


@pytest.mark.parametrize("A,seed", [(20, 1), (33, 2), (41, 3)])
@pytest.mark.parametrize("lam", [0.0, 4.0])
def test_cell_tables_equal_dense_oracle(A, seed, lam, span_ctx, gtable, gparams, oparams, weights):
    # every typed closed value, branch value and multiloop value equals the dense oracle's
    # (Theorem 1: sparse S1/S2 = dense D1/D2 at every interval, exactly in fixed point)
    p = S.protein(A, seed)
    say("tables", p, lam)
    r, T = span_ctx.design_tables(p, gtable, gparams, lam)
    d = oracle_tables(p, lam, oparams, weights)
    same(r, d)
    assert r.path == 0 and r.n_span_launches == 3 * A
    assert np.array_equal(T["V"], d.tables["V"])
    assert np.array_equal(T["B"], d.tables["B"])
    assert np.array_equal(T["S1"], d.tables["D1"])
    assert np.array_equal(T["S2"], d.tables["D2"])
    assert np.array_equal(T["X"], d.tables["X"])
    assert r.n_candidates == d.n_candidates
    assert r.n_visits == d.visits_sparse
    assert r.n_feasible == d.n_feasible_direct


@pytest.mark.parametrize("seed", range(1, 9))
@pytest.mark.parametrize("lam", [0.0, 4.0])
def test_plain50(seed, lam, ctx, gtable, gparams, oparams, weights):
    p = S.protein(50, seed)
    say("plain50", seed, lam)
    r = ctx.design(p, gtable, gparams, lam)
    d = O.design(p, weights, oparams, lam, nthreads=8)
    same(r, d)
    assert r.n_candidates == d.n_candidates and r.n_visits == d.visits_sparse


@pytest.mark.parametrize("p", ["M", "M*", "MW", "MKV", "MWMWMW", "YI" * 12, "W" * 9 + "*"])
def test_edge_cases(p, ctx, gtable, gparams, oparams, weights):
    say("edge", p)
    for lam in (0.0, 4.0):
        same(ctx.design(p, gtable, gparams, lam), O.design(p, weights, oparams, lam))


def test_retain_all_control_same_design(sd, gtable, gparams, oparams, weights):
    # scalar dense control: retains every finite direct interval; identical optimum and design
    c = sd.Context(0, retain_all=True)
    for seed in (1, 2):
        p = S.protein(50, seed)
        say("retain_all", seed)
        r = c.design(p, gtable, gparams, 0.0)
        d = O.design(p, weights, oparams, 0.0)
        same(r, d)
        assert r.n_candidates == d.n_candidates
        assert r.n_visits >= d.visits_sparse
    c.close()


def test_capacity_overflow_fallback(sd, gtable, gparams, oparams, weights):
    # a tiny per-endpoint capacity forces the overflow path; results are unchanged
    c = sd.Context(0, capacity_override=2)
    p = S.protein(50, 3)
    say("overflow")
    for lam in (0.0, 4.0):
        same(c.design(p, gtable, gparams, lam), O.design(p, weights, oparams, lam))
    c.close()


def test_invalid_inputs_on_device(sd, ctx, gtable, gparams):
    for p, code in [("", -2), ("MK*A", -2), ("MKZ", -2)]:
        with pytest.raises(sd.SDError) as e:
            ctx.design(p, gtable, gparams, 0.0)
        assert e.value.code == code
    for lam in (-1.0, float("nan"), float("inf")):
        with pytest.raises(sd.SDError) as e:
            ctx.design("MKV", gtable, gparams, lam)
        assert e.value.code == -5


def _golden(name, count):
    path = os.path.join(HERE, "golden", f"{name}.json")
    g = json.load(open(path))
    assert g["params_sha256"] == S.sha256_file(S.default_params_path())
    assert len(g["designs"]) == count
    return g["designs"]


def _check_golden(r, g):
    assert r.energy == g["energy"]
    assert r.objective_fixed == g["objective_fixed"]
    assert r.fixed_shift == g["fixed_shift"]
    assert r.mrna == g["mrna"]
    assert r.structure == g["structure"]
    assert abs(r.objective_kcal - g["objective_kcal"]) <= 1e-9
    assert r.n_candidates == g["n_candidates"]
    assert r.n_visits == g["visits_sparse"]
    assert r.n_cells == g["n_cells"]


@pytest.mark.parametrize("i", range(8))
def test_plain300_vs_golden(i, ctx, gtable, gparams):
    g = _golden("plain300", 8)[i]
    say("plain300", g["seed"], g["lambda"])
    _check_golden(ctx.design(g["protein"], gtable, gparams, g["lambda"]), g)


@pytest.mark.parametrize("i", range(4))
def test_plain925_1976_vs_golden(i, ctx, gtable, gparams):
    g = _golden("plain925_1976", 4)[i]
    say("plain925_1976", g["A"], g["lambda"])
    _check_golden(ctx.design(g["protein"], gtable, gparams, g["lambda"]), g)


def test_span_band_tuner_explores_then_settles(sd, gtable, gparams):
    # the first four designs of a length class each run one candidate tile for every span (every
    # launch timed); later designs of the class run each span band's fastest tile; the designs
    # are the same throughout
    c = sd.Context(0)
    p = S.protein(90, 5)
    flags, keys = [], {}
    for k in range(6):
        lam = 4.0 if k % 2 else 0.0
        say("span tuner design", k)
        r = c.design(p, gtable, gparams, lam)
        flags.append(r.sched_tuned)
        key = (r.mrna, r.structure, r.energy, r.objective_fixed, r.n_candidates, r.n_visits)
        assert keys.setdefault(lam, key) == key
    assert flags == [0, 0, 0, 0, 1, 1], flags
    fixed = sd.Context(0, span_threads=512)
    assert fixed.design(p, gtable, gparams, 0.0).sched_tuned == 1
    fixed.close()
    c.close()


@pytest.mark.parametrize("threads,waves", [(512, 1), (0, 1), (1024, 1), (256, 4)])
def test_invalid_span_item_waves_rejected(sd, threads, waves):
    with pytest.raises(sd.SDError) as e:
        sd.Context(0, span_threads=threads, span_item_waves=waves)
    assert e.value.code == -1  # SD_E_ARG
