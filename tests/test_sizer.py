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


@pytest.mark.gpu
def test_device_gradient_matches_cpu_fp64(sd):
    ctx = sd.Context(0)
    H, K = 64, 8
    z = sd.Sizer(ctx, H, K, seed=3)
    rng = np.random.default_rng(5)
    for n in (1, 37, 300):
        X = rng.random((n, 22)).astype(np.float32)
        Y = rng.random((n, K)).astype(np.float32)
        flat = z.get_params()
        loss, g = z.gradient(X, Y)
        rl, rg, _ = R.loss_and_grad(flat, X, Y, H, K)
        assert abs(loss - rl) <= 1e-5 * max(1e-3, abs(rl))
        err = np.linalg.norm(g - rg) / max(np.linalg.norm(rg), 1e-12)
        print("n", n, "relative gradient error", err, flush=True)
        assert err <= 1e-4
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
