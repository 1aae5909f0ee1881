"""Batched designs: one persistent launch (grid barrier per span, hipGraph-captured) must give
results identical to the plain per-design path and to the CPU oracle."""
import json
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
def gp(sd, params_path):
    return sd.Params(params_path)


@pytest.fixture(scope="module")
def gt(sd, weights):
    return sd.CodonTable(weights)


def key(r):
    return (r.energy, r.objective_fixed, r.mrna, r.structure, r.n_candidates, r.n_visits)


def test_small_mixed_batch_equals_plain_and_oracle(ctx, gt, gp, oparams, weights):
    lens = [6, 9, 15, 31, 40, 50, 12, 7, 44, 25, 60, 3]
    prots = [S.protein(A, 500 + i) for i, A in enumerate(lens)]
    lams = [0.0 if i % 2 == 0 else 4.0 for i in range(len(prots))]
    say("batch", len(prots))
    rb = ctx.design_batch(prots, lams, gt, gp)
    for p, lam, r in zip(prots, lams, rb):
        say("member", len(p), lam)
        rp = ctx.design(p, gt, gp, lam)
        assert key(r) == key(rp)
        d = O.design(p, weights, oparams, lam)
        assert (r.energy, r.objective_fixed, r.mrna, r.structure) == (d.energy, d.objective_fixed, d.mrna, d.structure)
        assert abs(r.objective_kcal - d.objective_kcal) <= 1e-9


def test_batch_with_duplicates_and_single(ctx, gt, gp):
    p = S.protein(35, 9)
    rb = ctx.design_batch([p, p, p], [0.0, 4.0, 0.0], gt, gp)
    assert key(rb[0]) == key(rb[2])
    assert key(rb[1]) == key(ctx.design(p, gt, gp, 4.0))
    r1 = ctx.design_batch([p], [4.0], gt, gp)
    assert key(r1[0]) == key(rb[1])


def test_batch_rejects_bad_member(sd, ctx, gt, gp):
    with pytest.raises(sd.SDError) as e:
        ctx.design_batch(["MKV", "MKB"], [0.0, 0.0], gt, gp)
    assert e.value.code == -2


def test_batch256_members_vs_golden(ctx, gt, gp):
    path = os.path.join(HERE, "golden", "batch256.json")
    if not os.path.exists(path):
        pytest.skip("batch256.json not generated")
    g = json.load(open(path))
    assert g["params_sha256"] == S.sha256_file(S.default_params_path())
    ds = g["designs"]
    if not ds:
        pytest.skip("no members generated yet")
    say("batch256 golden members", len(ds))
    rb = ctx.design_batch([d["protein"] for d in ds], [d["lambda"] for d in ds], gt, gp)
    for r, d in zip(rb, ds):
        assert (r.energy, r.objective_fixed, r.mrna, r.structure) == (d["energy"], d["objective_fixed"], d["mrna"], d["structure"])
        assert r.n_candidates == d["n_candidates"] and r.n_visits == d["visits_sparse"]


@pytest.mark.parametrize("threads,per_cu", [(64, 2), (256, 1), (512, 1)])
def test_fixed_schedules_equal_plain(sd, gt, gp, threads, per_cu):
    # every persistent schedule the caller can fix (workgroup size x workgroups per CU) gives the
    # plain results, whichever one the autotuner would have picked
    lens = [8, 33, 57, 21, 70]
    prots = [S.protein(A, 800 + i) for i, A in enumerate(lens)]
    lams = [0.0, 4.0, 0.0, 4.0, 2.0]
    c = sd.Context(0, batch_threads=threads, batch_per_cu=per_cu)
    say("schedule", threads, per_cu)
    rb = c.design_batch(prots, lams, gt, gp)
    for p, lam, r in zip(prots, lams, rb):
        assert key(r) == key(c.design(p, gt, gp, lam))
    c.close()


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
