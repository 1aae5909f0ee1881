"""Batched designs: one persistent launch (grid barrier per span, hipGraph-captured) must give
results identical to the plain per-design path and to the CPU oracle.  Every member must come
from the persistent launch itself (sd_result.path) replayed from a captured graph, so a silent
fallback to the plain path turns these tests red; under every persistent schedule the member
tables must equal the dense oracle's cell by cell."""
import functools
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
def gp(sd, params_path):
    return sd.Params(params_path)


@pytest.fixture(scope="module")
def gt(sd, weights):
    return sd.CodonTable(weights)


def key(r):
    return (r.energy, r.objective_fixed, r.mrna, r.structure, r.n_candidates, r.n_visits)


def persistent(sd, rs):
    # the result came from the persistent launch, replayed from a captured graph, with no
    # candidate overflow
    for r in rs:
        assert r.path == sd.PATH_PERSISTENT and r.graph_captured == 1 and r.cand_overflow == 0, \
            (r.path, r.graph_captured, r.cand_overflow)
        assert r.n_span_launches == 0
        assert (r.sched_threads, r.sched_item_waves) in ((64, 1), (256, 4), (256, 1), (512, 8)) and r.sched_grid > 0, \
            (r.sched_threads, r.sched_item_waves, r.sched_grid)


@functools.lru_cache(maxsize=None)
def oracle_tables(p, lam, params_path, wkey):
    return O.design(p, np.array(wkey), O.Params(params_path), lam, tables=True)


def test_small_mixed_batch_equals_plain_and_oracle(sd, ctx, gt, gp, oparams, weights):
    # 31-60 aa members exercise cross-span visibility through the grid barrier: a stale S1 of
    # the previous span inflates P_S and retains extra candidates (n_visits, n_candidates)
    lens = [6, 9, 15, 31, 40, 50, 12, 7, 44, 25, 60, 3]
    prots = [S.protein(A, 500 + i) for i, A in enumerate(lens)]
    lams = [0.0 if i % 2 == 0 else 4.0 for i in range(len(prots))]
    say("batch", len(prots))
    rb = ctx.design_batch(prots, lams, gt, gp)
    persistent(sd, rb)
    for p, lam, r in zip(prots, lams, rb):
        say("member", len(p), lam)
        rp = ctx.design(p, gt, gp, lam)
        assert key(r) == key(rp)
        d = O.design(p, weights, oparams, lam)
        assert (r.energy, r.objective_fixed, r.mrna, r.structure) == (d.energy, d.objective_fixed, d.mrna, d.structure)
        assert abs(r.objective_kcal - d.objective_kcal) <= 1e-9
        assert (r.n_candidates, r.n_visits, r.n_feasible) == (d.n_candidates, d.visits_sparse, d.n_feasible_direct)


def test_batch_with_duplicates_and_single(sd, ctx, gt, gp):
    p = S.protein(35, 9)
    rb = ctx.design_batch([p, p, p], [0.0, 4.0, 0.0], gt, gp)
    persistent(sd, rb)
    assert key(rb[0]) == key(rb[2])
    assert key(rb[1]) == key(ctx.design(p, gt, gp, 4.0))
    r1 = ctx.design_batch([p], [4.0], gt, gp)
    assert key(r1[0]) == key(rb[1])


def test_batch_rejects_bad_member(sd, ctx, gt, gp):
    with pytest.raises(sd.SDError) as e:
        ctx.design_batch(["MKV", "MKB"], [0.0, 0.0], gt, gp)
    assert e.value.code == -2  # SD_E_PROTEIN


def test_batch256_members_vs_golden(sd, ctx, gt, gp):
    path = os.path.join(HERE, "golden", "batch256.json")
    g = json.load(open(path))
    assert g["params_sha256"] == S.sha256_file(S.default_params_path())
    ds = g["designs"]
    assert len(ds) == 256
    say("batch256 golden members", len(ds))
    rb = ctx.design_batch([d["protein"] for d in ds], [d["lambda"] for d in ds], gt, gp)
    persistent(sd, rb)
    for r, d in zip(rb, ds):
        assert (r.energy, r.objective_fixed, r.mrna, r.structure) == (d["energy"], d["objective_fixed"], d["mrna"], d["structure"])
        assert r.n_candidates == d["n_candidates"] and r.n_visits == d["visits_sparse"]


@pytest.mark.parametrize("threads,per_cu,item_waves", [(64, 2, 0), (256, 1, 0), (512, 1, 0), (256, 3, 1), (256, 1, 1)])
def test_fixed_schedules_equal_plain(sd, gt, gp, threads, per_cu, item_waves):
    # every persistent schedule the caller can fix (workgroup size x workgroups per CU x waves per
    # work item) gives the plain results, whichever one the autotuner would have picked
    lens = [8, 33, 57, 21, 70]
    prots = [S.protein(A, 800 + i) for i, A in enumerate(lens)]
    lams = [0.0, 4.0, 0.0, 4.0, 2.0]
    c = sd.Context(0, batch_threads=threads, batch_per_cu=per_cu, batch_item_waves=item_waves)
    say("schedule", threads, per_cu, item_waves)
    rb = c.design_batch(prots, lams, gt, gp)
    persistent(sd, rb)
    for r in rb:  # the launch ran under the fixed schedule
        assert r.sched_threads == threads and r.sched_grid % per_cu == 0, (r.sched_threads, r.sched_grid)
        assert r.sched_item_waves == (item_waves or threads // 64)
    for p, lam, r in zip(prots, lams, rb):
        assert key(r) == key(c.design(p, gt, gp, lam))
    c.close()


@pytest.mark.parametrize("threads,per_cu,item_waves",
                         [(0, 0, 0), (64, 1, 0), (64, 2, 0), (256, 1, 0), (256, 2, 0), (512, 1, 0), (256, 1, 1),
                          (256, 3, 1)])
def test_member_tables_equal_dense_oracle(sd, gt, gp, params_path, weights, threads, per_cu, item_waves):
    # every typed value, branch value and multiloop value of each member, filled by the
    # persistent kernel under this schedule, equals the dense oracle's (Theorem 1); the members
    # span several layer-pair tiles and a ragged tail, both lambdas, in one launch
    prots = [S.protein(20, 1), S.protein(33, 2), S.protein(41, 3), S.protein(27, 4)]
    lams = [0.0, 4.0, 4.0, 0.0]
    c = sd.Context(0, batch_threads=threads, batch_per_cu=per_cu, batch_item_waves=item_waves)
    for m in range(len(prots)):
        say("batch tables", threads, per_cu, item_waves, "member", m)
        rb, T = c.design_batch_tables(prots, lams, gt, gp, m)
        persistent(sd, rb)
        d = oracle_tables(prots[m], lams[m], params_path, tuple(float(x) for x in weights))
        r = rb[m]
        assert (r.energy, r.objective_fixed, r.mrna, r.structure) == (d.energy, d.objective_fixed, d.mrna, d.structure)
        assert np.array_equal(T["V"], d.tables["V"])
        assert np.array_equal(T["B"], d.tables["B"])
        assert np.array_equal(T["S1"], d.tables["D1"])
        assert np.array_equal(T["S2"], d.tables["D2"])
        assert np.array_equal(T["X"], d.tables["X"])
        assert (r.n_candidates, r.n_visits, r.n_feasible) == (d.n_candidates, d.visits_sparse, d.n_feasible_direct)
    c.close()


def test_batch_tables_member_out_of_range(sd, ctx, gt, gp):
    with pytest.raises(sd.SDError) as e:
        ctx.design_batch_tables(["MKV"], [0.0], gt, gp, 1)
    assert e.value.code == -1


def test_invalid_options_rejected(sd):
    for kw in ({"span_threads": 100}, {"batch_threads": 128, "batch_per_cu": 1},
               {"batch_threads": 256}, {"batch_per_cu": 2}, {"batch_threads": 256, "batch_per_cu": 1000}):
        with pytest.raises(sd.SDError) as e:
            sd.Context(0, **kw)
        assert e.value.code == -1, kw


def test_envelope_invalid_ranges(ctx, sd, gt, gp):
    for lo, hi, code in ((-1.0, 4.0, -5), (2.0, 2.0, -5), (3.0, 1.0, -5), (0.0, float("inf"), -5)):
        with pytest.raises(sd.SDError) as e:
            ctx.lambda_envelope("MKV*", lo, hi, gt, gp)
        assert e.value.code == code
    with pytest.raises(sd.SDError) as e:
        ctx.lambda_envelope("MKV*", 0.0, 1.0, gt, gp, max_designs=1)
    assert e.value.code == -1


@pytest.mark.parametrize("threads,per_cu,item_waves", [(512, 1, 1), (0, 0, 1), (64, 1, 4), (256, 1, 2)])
def test_invalid_item_waves_rejected(sd, threads, per_cu, item_waves):
    with pytest.raises(sd.SDError) as e:
        sd.Context(0, batch_threads=threads, batch_per_cu=per_cu, batch_item_waves=item_waves)
    assert e.value.code == -1  # SD_E_ARG


def test_autotuner_explores_then_settles(sd, gt, gp):
    # a new size class runs one candidate schedule per call, then every later call runs the
    # fastest; the designs are the same under every schedule
    lens = [30 + 7 * i for i in range(16)]
    prots = [S.protein(A, 900 + i) for i, A in enumerate(lens)]
    lams = [0.0 if i % 2 == 0 else 4.0 for i in range(len(prots))]
    c = sd.Context(0)
    seen, ref = [], None
    for k in range(10):
        say("tuning call", k)
        rb = c.design_batch(prots, lams, gt, gp)
        persistent(sd, rb)
        keys = [key(r) for r in rb]
        ref = ref or keys
        assert keys == ref
        sched = {(r.sched_threads, r.sched_grid, r.sched_item_waves, r.sched_tuned) for r in rb}
        assert len(sched) == 1
        seen.append(sched.pop())
        if seen[-1][3] == 1:
            break
    explored = [x[:3] for x in seen if x[3] == 0]
    assert len(explored) >= 2 and len(set(explored)) == len(explored), seen
    assert seen[-1][3] == 1 and seen[-1][:3] in explored, seen
    rb = c.design_batch(prots, lams, gt, gp)
    assert {(r.sched_threads, r.sched_grid, r.sched_item_waves, r.sched_tuned) for r in rb} == {seen[-1]}
    c.close()


def test_batch_beyond_one_launch(sd, ctx, gt, gp):
    # more members than one persistent launch holds (1,024): the batch runs as consecutive
    # launches, and members on both sides of the split equal their plain designs
    n = 1030
    prots = [S.protein(4 + (i % 9), 3000 + i) for i in range(n)]
    lams = [0.0 if i % 3 else 4.0 for i in range(n)]
    say("batch of", n)
    rb = ctx.design_batch(prots, lams, gt, gp)
    assert len(rb) == n
    persistent(sd, rb)
    for i in (0, 1, 511, 1022, 1023, 1024, 1025, 1029):
        assert key(rb[i]) == key(ctx.design(prots[i], gt, gp, lams[i])), i
