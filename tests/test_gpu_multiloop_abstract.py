"""The exact-integer abstract multiloop test (Sec. 7.1) on the GPU code path: random layered
branching/merging DAGs with random integer direct costs B and unpaired-edge costs replace the
energy model, and the span step's own multiloop code (S2 over the committed candidate prefix,
P_S, S1, the online retention test B < P_S and the appends, eqs. 6-7) runs on them.  At every
forward interval S1 and S2 must equal the oracle's dense right-normal D1 and D2 (Theorem 1),
which tests/test_multiloop_abstract.py pins to brute-force path enumeration, and the retained
candidates must be exactly the dense retention set of eq. (6)."""
import numpy as np
import pytest

import oracle as O
from test_multiloop_abstract import SHAPES, random_dag

pytestmark = pytest.mark.gpu
INF = O.INF


@pytest.fixture(scope="module")
def ctx():
    import paper_2609_32308_amd as m
    c = m.Context(0)
    yield c
    c.close()


def check(ctx, layer, esrc, edst, eu, B):
    D1, D2, PD = O.multiloop_dense(layer, esrc, edst, eu, B)
    r = ctx.multiloop_abstract(layer, esrc, edst, eu, B)
    N = len(layer)
    fwd = layer[None, :] > layer[:, None]
    assert np.array_equal(r["S1"][fwd], D1[fwd])
    assert np.array_equal(r["S2"][fwd], D2[fwd])
    dense_set = fwd & (B < PD)
    assert np.array_equal(r["cand"].astype(bool), dense_set)
    assert r["Z"] == int(dense_set.sum())


# the shapes of the CPU test plus wider (up to the kernel's 4 states per layer) and longer DAGs
WIDE = [(12, 4), (20, 3), (30, 2)]
CASES = [(seed, *SHAPES[seed % len(SHAPES)]) for seed in range(300)] + \
        [(1000 + seed, *WIDE[seed % len(WIDE)]) for seed in range(60)]


@pytest.mark.parametrize("seed,L,w", CASES)
def test_gpu_multiloop_equals_dense(ctx, seed, L, w):
    rng = np.random.default_rng(seed)
    p_arc = 0.15 + 0.5 * rng.random()
    layer, esrc, edst, eu, B = random_dag(rng, L, w, p_edge=0.7, p_arc=p_arc)
    check(ctx, layer, esrc, edst, eu, B)


def test_gpu_ties_are_not_retained(ctx):
    layer = np.array([0, 1, 2])
    esrc, edst, eu = np.array([0, 1]), np.array([1, 2]), np.array([0, 0], dtype=np.int64)
    B = np.full((3, 3), INF, dtype=np.int64)
    B[0, 1], B[0, 2], B[1, 2] = 5, 5, 7  # (0,2) tied by arc (0,1) + edge (1,2): not a candidate
    check(ctx, layer, esrc, edst, eu, B)
    r = ctx.multiloop_abstract(layer, esrc, edst, eu, B)
    assert r["cand"][0, 2] == 0 and r["S1"][0, 2] == 5


def test_gpu_multiloop_rejects_malformed(ctx):
    import paper_2609_32308_amd as m
    B = np.full((3, 3), INF, dtype=np.int64)
    with pytest.raises(m.SDError) as e:  # an edge skipping a layer
        ctx.multiloop_abstract(np.array([0, 1, 2]), np.array([0]), np.array([2]), np.array([1]), B)
    assert e.value.code == -1
    with pytest.raises(m.SDError) as e:  # a layer of five states
        ctx.multiloop_abstract(np.array([0, 1, 1, 1, 1, 1, 2]), np.array([], np.int32), np.array([], np.int32),
                               np.array([], np.int64), np.full((7, 7), INF, dtype=np.int64))
    assert e.value.code == -1
