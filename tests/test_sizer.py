"""Learned candidate-buffer sizing: the MLP's device gradients against a CPU FP64 reference, its
training, and the sizing policy's effect (less memory reserved, identical designs)."""
import numpy as np
import pytest

import oracle.mlp_ref as R
import sdinputs as S


def _rand_params(H, K, seed):
    rng = np.random.default_rng(seed)
    sizes = [H * 22, H, H * H, H, K * H, K]
    return np.concatenate([rng.normal(0, 0.3, n) for n in sizes]).astype(np.float32)


def test_reference_gradient_matches_finite_differences():
    # pins the FP64 reference itself (no GPU): central differences on random parameters
    H, K = 7, 3
    rng = np.random.default_rng(0)
    flat = _rand_params(H, K, 1).astype(np.float64)
    X = rng.random((11, 22))
    Y = rng.random((11, K))
    loss, g, _ = R.loss_and_grad(flat, X, Y, H, K)
    eps = 1e-6
    for i in rng.choice(flat.size, 40, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[i] += eps
        fm[i] -= eps
        num = (R.loss_and_grad(fp, X, Y, H, K)[0] - R.loss_and_grad(fm, X, Y, H, K)[0]) / (2 * eps)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num))


def test_reference_loss_is_mse_of_sigmoid_outputs():
    H, K = 4, 2
    flat = np.zeros(H * 22 + H + H * H + H + K * H + K)
    X = np.ones((3, 22))
    Y = np.full((3, K), 0.25)
    loss, g, yh = R.loss_and_grad(flat, X, Y, H, K)
    assert np.allclose(yh, 0.5) and abs(loss - 0.0625) < 1e-15


@pytest.fixture(scope="module")
def sd():
    import paper_2609_32308_amd as m
    return m


def _magnitudes(flat, X, Y, H, K):
    """Element-wise magnitude of each forward output and gradient entry: the same chain rule with
    every factor replaced by its absolute value.  An FP32 evaluation of a sum of such products
    is off by at most about (terms in the sum) * 2^-24 times this magnitude, so it scales the
    per-element tolerance (a wrong small entry, such as one bias gradient, still fails)."""
    W1, b1, W2, b2, W3, b3 = [np.abs(a) for a in R.unpack(flat, H, K)]
    Wr = R.unpack(flat, H, K)
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    z1 = X @ Wr[0].T + Wr[1]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ Wr[2].T + Wr[3]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ Wr[4].T + Wr[5]
    yh = 1.0 / (1.0 + np.exp(-z3))
    a1 = np.abs(X) @ W1.T + b1
    a2 = (a1 * (z1 > 0)) @ W2.T + b2
    a3 = (a2 * (z2 > 0)) @ W3.T + b3
    # |yh - Y| is computed from an FP32 yh: its error scales with yh, Y and the logit's magnitude
    d3 = 2.0 / (n * K) * (np.abs(yh - Y) + yh + np.abs(Y) + yh * (1 - yh) * a3) * yh * (1.0 - yh)
    gW3 = d3.T @ np.abs(h2)
    gb3 = d3.sum(0)
    d2 = (d3 @ W3) * (z2 > 0)
    gW2 = d2.T @ np.abs(h1)
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (z1 > 0)
    gW1 = d1.T @ np.abs(X)
    gb1 = d1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return g, yh * (1 - yh) * a3, min(np.abs(z1).min(), np.abs(z2).min())


def _inputs_clear_of_kinks(n, K, flat, H, seed):
    """Random inputs whose FP64 pre-activations all sit clear of the ReLU kink (a pre-activation
    within FP32 rounding of 0 could take the other branch on the device)."""
    for s in range(seed, seed + 50):
        rng = np.random.default_rng(s)
        X = rng.random((n, 22)).astype(np.float32)
        Y = rng.random((n, K)).astype(np.float32)
        if _magnitudes(flat, X, Y, H, K)[2] > 1e-4:
            return X, Y
    raise AssertionError("no input draw clear of the ReLU kinks")


@pytest.mark.gpu
def test_device_gradient_matches_cpu_fp64_elementwise(sd):
    ctx = sd.Context(0)
    H, K = 64, 8
    z = sd.Sizer(ctx, H, K, seed=3)
    flat = z.get_params()
    for n in (1, 37, 300):
        X, Y = _inputs_clear_of_kinks(n, K, flat, H, 5 + n)
        loss, g = z.gradient(X, Y)
        rl, rg, _ = R.loss_and_grad(flat, X, Y, H, K)
        mag, _, _ = _magnitudes(flat, X, Y, H, K)
        assert abs(loss - rl) <= 1e-5 * max(1e-3, abs(rl))
        terms = max(n, H, 22) + 4
        tol = 4 * terms * 2.0 ** -24 * mag + 1e-4 * np.abs(rg) + 1e-12
        bad = np.flatnonzero(np.abs(g - rg) > tol)
        print("n", n, "max |g - g_ref| / tol", float(np.max(np.abs(g - rg) / tol)), flush=True)
        assert bad.size == 0, (n, bad[:10], g[bad[:10]], rg[bad[:10]])
        # every block of the flat layout is exercised: no block is identically zero on both sides
        offs = np.cumsum([0, H * 22, H, H * H, H, K * H, K])
        for lo, hi in zip(offs[:-1], offs[1:]):
            assert np.any(rg[lo:hi] != 0.0)
    ctx.close()


@pytest.mark.gpu
def test_forward_device_and_host_match_cpu_fp64(sd):
    # the device forward pass (k_dense_fwd, used by training) and the host forward pass (used by
    # sizing and admission) against the FP64 reference, element by element, on the initial
    # parameters and after training
    ctx = sd.Context(0)
    H, K = 64, 8
    z = sd.Sizer(ctx, H, K, seed=11)
    rng = np.random.default_rng(12)
    Xt = rng.random((400, 22)).astype(np.float32)
    Yt = (0.1 + 0.5 * Xt[:, :8] * Xt[:, 8:16]).astype(np.float32)
    for stage in ("initial", "trained"):
        if stage == "trained":
            z.train(Xt, Yt, steps=300, lr=3e-3)
        flat = z.get_params()
        X, Y = _inputs_clear_of_kinks(64, K, flat, H, 40)
        _, _, yref = R.loss_and_grad(flat, X, Y, H, K)
        _, mag, _ = _magnitudes(flat, X, Y, H, K)
        tol = 4 * (H + 26) * 2.0 ** -24 * mag + 2e-7
        dev, host = z.predict(X), z.predict_host(X)
        print(stage, "device", float(np.max(np.abs(dev - yref) / tol)), "host",
              float(np.max(np.abs(host - yref) / tol)), flush=True)
        assert np.all(np.abs(dev - yref) <= tol)
        assert np.all(np.abs(host - yref) <= tol)
    ctx.close()


@pytest.mark.gpu
def test_device_training_reduces_loss(sd):
    ctx = sd.Context(0)
    z = sd.Sizer(ctx, 64, 8, seed=4)
    rng = np.random.default_rng(6)
    X = rng.random((500, 22)).astype(np.float32)
    Y = (0.1 + 0.5 * X[:, :8] * X[:, 8:16]).astype(np.float32)
    l0, _ = z.gradient(X, Y)
    l1 = z.train(X, Y, steps=1500, lr=3e-3)
    l2, _ = z.gradient(X, Y)
    assert l2 < 0.2 * l0 and l2 <= l1 * 1.01
    P = z.predict(X)
    assert np.mean((P - Y) ** 2) == pytest.approx(l2, rel=1e-3)
    ctx.close()


@pytest.mark.gpu
def test_features(sd):
    f = sd.features("MKKW*", 4.0)
    assert f[0] == pytest.approx(np.log(5) / np.log(2000), rel=1e-6)
    assert f[21] == 1.0 and f[1 + "ACDEFGHIKLMNPQRSTVWY".index("K")] == pytest.approx(0.4)


@pytest.mark.gpu
def test_sizing_policy_keeps_designs_and_saves_memory(sd, params_path, weights):
    ctx = sd.Context(0)
    gp, gt = sd.Params(params_path), sd.CodonTable(weights)
    K = 8
    train = [S.protein(A, 9000 + i) for i, A in enumerate(S.batch_lengths(160, 40, 160, seed=21))]
    lams = [0.0 if i % 2 == 0 else 4.0 for i in range(len(train))]
    Y, _ = ctx.occupancy(train, lams, gt, gp, K)
    assert np.all((Y >= 0) & (Y <= 1))
    X = np.stack([sd.features(p, l) for p, l in zip(train, lams)])
    z = sd.Sizer(ctx, 64, K, seed=7)
    z.train(X, Y, steps=2000, lr=3e-3)
    test = [S.protein(A, 9500 + i) for i, A in enumerate(S.batch_lengths(12, 60, 160, seed=22))]
    tl = [0.0 if i % 2 == 0 else 4.0 for i in range(len(test))]
    worst = ctx.design_batch(test, tl, gt, gp)
    ctx.set_sizer(z, margin=0.5, slack=8)
    sized = ctx.design_batch(test, tl, gt, gp)
    plain = [ctx.design(p, gt, gp, l) for p, l in zip(test, tl)]
    for a, b, c in zip(worst, sized, plain):
        assert (a.energy, a.objective_fixed, a.mrna, a.structure) == (b.energy, b.objective_fixed, b.mrna, b.structure)
        assert (b.mrna, b.structure) == (c.mrna, c.structure)
    # the host-side request estimate is exactly what the sized designs reserved
    for p, l, a, b, c in zip(test, tl, worst, sized, plain):
        est = z.request_bytes(p, l, margin=0.5, slack=8)
        assert est["cand_slots"] == b.cand_slots_first == c.cand_slots_first
        assert est["worst_slots"] == a.cand_slots_first and est["cand_bytes"] == 12 * est["cand_slots"]
    w = sum(r.cand_slots_first for r in worst)
    m = sum(r.cand_slots_first for r in sized)
    print("reserved slots worst", w, "mlp", m, "overflows", sum(r.cand_overflow for r in sized), flush=True)
    assert m < w
    # a sizer forced far too small overflows and falls back: results still identical
    ctx.set_sizer(z, margin=0.0, slack=0)
    zz = sd.Sizer(ctx, 64, K, seed=8)
    zz.set_params(np.full(zz.n_params, -0.5, np.float32))  # predicts tiny fractions
    ctx.set_sizer(zz, margin=0.0, slack=0)
    tiny = ctx.design_batch(test[:4], tl[:4], gt, gp)
    assert any(r.cand_overflow for r in tiny)
    for a, b in zip(tiny, worst[:4]):
        assert (a.energy, a.objective_fixed, a.mrna, a.structure) == (b.energy, b.objective_fixed, b.mrna, b.structure)
    ctx.set_sizer(None)
    ctx.close()


@pytest.mark.gpu
def test_learned_sizer_raises_admitted_concurrency(sd, params_path, weights, oparams):
    # What the trained network gains: under one fixed server pool, requests reserve less
    # candidate memory, so more of them run at once; every result stays the oracle's.
    import math
    import oracle as O
    ctx = sd.Context(0)
    gp, gt = sd.Params(params_path), sd.CodonTable(weights)
    K = 8
    train = [S.protein(A, 9100 + i) for i, A in enumerate(S.batch_lengths(120, 60, 260, seed=23))]
    lams = [0.0 if i % 2 == 0 else 4.0 for i in range(len(train))]
    Y, _ = ctx.occupancy(train, lams, gt, gp, K)
    X = np.stack([sd.features(p, l) for p, l in zip(train, lams)])
    z = sd.Sizer(ctx, 64, K, seed=7)
    z.train(X, Y, steps=2000, lr=3e-3)
    ctx.close()
    lam, margin = 4.0, 1.0

    def serve(p, sized, pool, copies, max_active):
        c = sd.Context(0)
        if sized:
            c.set_sizer(z, margin=margin, slack=8)
        srv = sd.Server(c, gt, gp, pool_bytes=pool, max_active=max_active, steps_per_round=64)
        tickets = [srv.submit(p, lam) for _ in range(copies)]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
        srv.stop()
        c.close()
        return res, st

    # reservation of one request under each policy, for a 200-aa request whose learned
    # reservation holds (an overflowing one is re-admitted with worst-case segments and then
    # reserves both)
    for seed in range(77, 87):
        p = S.protein(200, seed)
        _, st_s = serve(p, True, 1 << 30, 1, 4)
        if st_s["fallbacks"] == 0:
            break
    assert st_s["fallbacks"] == 0
    _, st_w = serve(p, False, 1 << 30, 1, 4)
    Ww, Ws = st_w["reserved_bytes"], st_s["reserved_bytes"]
    print("seed", seed, "reservation per request: worst-case", Ww, "learned", Ws, flush=True)
    assert Ws < Ww
    # a pool that holds k worst-case reservations but k + 1 learned ones
    d = Ww - Ws
    k = max(2, math.ceil(Ws / d))
    pool = k * Ww + d // 2
    assert (k + 1) * Ww > pool and (k + 1) * Ws <= pool
    res_w, st_w = serve(p, False, pool, k + 4, k + 8)
    res_s, st_s = serve(p, True, pool, k + 4, k + 8)
    print("pool", pool, "k", k, "peak worst", st_w["peak_active"], "peak learned", st_s["peak_active"],
          "overflows", st_s["fallbacks"], flush=True)
    assert st_w["peak_active"] == k
    assert st_s["peak_active"] >= k + 1
    d_or = O.design(p, weights, oparams, lam, nthreads=8)
    for r in res_w + res_s:
        assert (r.energy, r.objective_fixed, r.mrna, r.structure) == \
            (d_or.energy, d_or.objective_fixed, d_or.mrna, d_or.structure)
        assert r.path == sd.PATH_PERSISTENT
