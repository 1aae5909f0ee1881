"""Design server: continuous batching with memory-based admission.  Every served result must equal
the same design computed alone, requests arriving while others run must be admitted into the
running mix, and a small pool must make admission wait without changing results."""
import random
import threading
import time

import pytest

import sdinputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def sd():
    import paper_2609_32308_amd as m
    return m


@pytest.fixture(scope="module")
def env(sd, params_path, weights):
    return sd.Params(params_path), sd.CodonTable(weights)


def key(r):
    return (r.energy, r.objective_fixed, r.mrna, r.structure, r.n_candidates)


def _requests(n, seed, lo=20, hi=140):
    lens = S.batch_lengths(n, lo, hi, seed=seed)
    return [(S.protein(A, seed * 1000 + i), 0.0 if i % 2 == 0 else 4.0) for i, A in enumerate(lens)]


def _serve(sd, gp, gt, reqs, pool, max_active, steps, gaps):
    ctx = sd.Context(0)
    srv = sd.Server(ctx, gt, gp, pool_bytes=pool, max_active=max_active, steps_per_round=steps)
    tickets = []
    for (p, lam), gap in zip(reqs, gaps):
        tickets.append(srv.submit(p, lam))
        time.sleep(gap)
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.stop()
    ctx.close()
    return res, st


def test_served_equals_alone(sd, env):
    gp, gt = env
    reqs = _requests(24, 31)
    rng = random.Random(5)
    gaps = [rng.expovariate(200.0) for _ in reqs]  # Poisson arrivals, mean 5 ms apart
    say("serving", len(reqs))
    res, st = _serve(sd, gp, gt, reqs, pool=2 << 30, max_active=64, steps=16, gaps=gaps)
    say("stats", st)
    alone = sd.Context(0)
    for (p, lam), r in zip(reqs, res):
        a = alone.design(p, gt, gp, lam)
        assert key(r) == key(a)
    alone.close()
    assert st["admitted"] == len(reqs) and st["completed"] == len(reqs)
    assert st["peak_active"] > 1  # later arrivals joined a running mix
    assert st["rounds"] > 1


def test_small_pool_admission_waits(sd, env):
    gp, gt = env
    reqs = _requests(10, 32, 60, 120)
    say("small pool")
    res, st = _serve(sd, gp, gt, reqs, pool=40 << 20, max_active=64, steps=32, gaps=[0.0] * len(reqs))
    say("stats", st)
    assert st["pool_high_water"] <= 40 << 20
    assert st["peak_active"] < len(reqs)  # memory, not slots, limited the mix
    alone = sd.Context(0)
    for (p, lam), r in zip(reqs, res):
        assert key(r) == key(alone.design(p, gt, gp, lam))
    alone.close()


def test_invalid_request_and_stop_cancels(sd, env):
    gp, gt = env
    ctx = sd.Context(0)
    srv = sd.Server(ctx, gt, gp, pool_bytes=256 << 20, max_active=4, steps_per_round=8)
    bad = srv.submit("MKB", 0.0)
    with pytest.raises(sd.SDError) as e:
        srv.wait(bad)
    assert e.value.code == -2
    good = srv.submit(S.protein(30, 3), 0.0)
    assert srv.wait(good).mrna
    srv.stop()
    ctx.close()
