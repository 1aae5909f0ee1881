"""Design server: continuous batching with memory-based admission.  Every served result must equal
the oracle's design and the same design computed alone, must come from the persistent launch
(no plain fallback), requests arriving while others run must be admitted into the running mix,
and a small pool must make admission wait without changing results."""
import random
import threading
import time

import pytest

import oracle as O
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


def same_as_oracle(r, d):
    assert (r.energy, r.objective_fixed, r.fixed_shift, r.mrna, r.structure) == \
        (d.energy, d.objective_fixed, d.fixed_shift, d.mrna, d.structure)
    assert abs(r.objective_kcal - d.objective_kcal) <= 1e-9
    assert (r.n_candidates, r.n_visits, r.n_feasible) == (d.n_candidates, d.visits_sparse, d.n_feasible_direct)


def _requests(n, seed, lo=20, hi=140):
    lens = S.batch_lengths(n, lo, hi, seed=seed)
    return [(S.protein(A, seed * 1000 + i), 0.0 if i % 2 == 0 else 4.0) for i, A in enumerate(lens)]


def _serve(sd, gp, gt, reqs, pool, max_active, steps, gaps, **ctx_opts):
    ctx = sd.Context(0, **ctx_opts)
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


def test_served_equals_oracle_and_alone(sd, env, oparams, weights):
    gp, gt = env
    reqs = _requests(24, 31)
    rng = random.Random(5)
    gaps = [rng.expovariate(200.0) for _ in reqs]  # Poisson arrivals, mean 5 ms apart
    say("serving", len(reqs))
    res, st = _serve(sd, gp, gt, reqs, pool=2 << 30, max_active=64, steps=16, gaps=gaps)
    say("stats", st)
    assert st["fallbacks"] == 0
    alone = sd.Context(0)
    for (p, lam), r in zip(reqs, res):
        assert r.path == sd.PATH_PERSISTENT and r.cand_overflow == 0
        # the round that finished the request ran one of the two 256-thread schedules
        assert (r.sched_threads, r.sched_item_waves, r.sched_tuned) in ((256, 4, 1), (256, 1, 1)) and r.sched_grid > 0
        a = alone.design(p, gt, gp, lam)
        assert key(r) == key(a)
        say("oracle", len(p), lam)
        same_as_oracle(r, O.design(p, weights, oparams, lam, nthreads=8))
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
    assert st["fallbacks"] == 0
    alone = sd.Context(0)
    for (p, lam), r in zip(reqs, res):
        assert r.path == sd.PATH_PERSISTENT
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


def test_stop_with_requests_still_queued(sd, env):
    # a pool that holds one or two requests at a time keeps the rest queued while the server
    # thread admits; stopping then cancels the queued ones (the server thread takes a request
    # off the queue under the lock that reads it, so a request it is placing is never also
    # cancelled) and finishes the admitted ones; the context stays usable
    gp, gt = env
    reqs = _requests(16, 33, 80, 120)
    ctx = sd.Context(0)
    for delay in (0.0, 0.005, 0.05):
        srv = sd.Server(ctx, gt, gp, pool_bytes=48 << 20, max_active=8, steps_per_round=4)
        for p, lam in reqs:
            srv.submit(p, lam)
        time.sleep(delay)
        st = srv.stats()
        say("stop after", delay, st)
        srv.stop()
        with pytest.raises(sd.SDError):  # the handle is gone: null server
            srv.submit("MKV", 0.0)
    p, lam = reqs[0]
    assert key(ctx.design(p, gt, gp, lam)) == key(sd.Context(0).design(p, gt, gp, lam))
    ctx.close()


@pytest.mark.parametrize("item_waves", [1, 4])
def test_fixed_schedule_serving_equals_alone(sd, env, item_waves):
    # a schedule fixed in the context's options serves every round: independent waves and shared
    # items both give the designs of sd_design
    gp, gt = env
    reqs = _requests(12, 33)
    say("fixed schedule serving", item_waves)
    res, st = _serve(sd, gp, gt, reqs, pool=2 << 30, max_active=64, steps=16, gaps=[0.002] * len(reqs),
                     batch_threads=256, batch_per_cu=4, batch_item_waves=item_waves)
    assert st["fallbacks"] == 0 and st["completed"] == len(reqs)
    alone = sd.Context(0)
    for (p, lam), r in zip(reqs, res):
        assert r.path == sd.PATH_PERSISTENT
        assert (r.sched_threads, r.sched_item_waves, r.sched_tuned) == (256, item_waves, 1)
        assert key(r) == key(alone.design(p, gt, gp, lam))
    alone.close()
