"""Exact-integer abstract multiloop test on random layered branching/merging DAGs.

Sec. 7.1 describes this check: random integer direct costs B and unpaired-edge costs u replace
the energy model, which isolates the multiloop recurrence logic.  The proof of Theorem 1 (Sec.
4.2) reads a multiloop fragment as a path of atomic branch arcs (finite B(a,b)) and unpaired
edges; D1 / D2 are the cheapest such paths with at least one / two arcs.  Here:
  * brute force enumerates every such path explicitly;
  * the oracle's dense right-normal recurrences (eqs. 3-5) must equal it at every interval;
  * the sparse recurrence (eq. 7 with the online test B < P_S, eq. 6) must equal dense at every
    interval (Theorem 1), and its candidates must be a subset of the finite direct intervals.
"""
import numpy as np
import pytest

import oracle as O

INF = O.INF


def random_dag(rng, L, wmax, p_edge, p_arc, arc_range=(-12, 12), u_range=(0, 6)):
    widths = [1] + [int(rng.integers(1, wmax + 1)) for _ in range(L - 1)] + [1]
    layer = []
    for l, w in enumerate(widths):
        layer += [l] * w
    N = len(layer)
    byl = {}
    for v, l in enumerate(layer):
        byl.setdefault(l, []).append(v)
    esrc, edst, eu = [], [], []
    for v in range(N):
        l = layer[v]
        if l + 1 in byl:
            for w in byl[l + 1]:
                if rng.random() < p_edge:
                    esrc.append(v); edst.append(w); eu.append(int(rng.integers(*u_range)))
    B = np.full((N, N), INF, dtype=np.int64)
    for a in range(N):
        for b in range(N):
            if layer[b] > layer[a] and rng.random() < p_arc:
                B[a, b] = int(rng.integers(*arc_range))
    return np.array(layer), np.array(esrc), np.array(edst), np.array(eu, dtype=np.int64), B


def brute(layer, esrc, edst, eu, B):
    """min cost over explicit item paths a -> b, split by arc count (1, >=2) and 'not sole arc'."""
    N = len(layer)
    out = {v: [] for v in range(N)}
    for s, d, u in zip(esrc, edst, eu):
        out[int(s)].append((int(d), int(u), 0))
    for a in range(N):
        for b in range(N):
            if B[a, b] < INF:
                out[a].append((b, int(B[a, b]), 1))
    D1 = np.full((N, N), INF, dtype=np.int64)
    D2 = np.full((N, N), INF, dtype=np.int64)
    PD = np.full((N, N), INF, dtype=np.int64)

    def dfs(a, v, cost, arcs, items):
        if arcs >= 1:
            if cost < D1[a, v]:
                D1[a, v] = cost
            if arcs >= 2 and cost < D2[a, v]:
                D2[a, v] = cost
            if not (items == 1 and arcs == 1) and cost < PD[a, v]:
                PD[a, v] = cost
        for (w, c, isarc) in out[v]:
            dfs(a, w, cost + c, min(arcs + isarc, 2), items + 1)

    for a in range(N):
        dfs(a, a, 0, 0, 0)
    return D1, D2, PD


def sparse(layer, esrc, edst, eu, B):
    """eq. (7): S2 scans only candidates c in C_b with rho(c) > rho(a); online retention B < P_S."""
    N = len(layer)
    ins = {v: [] for v in range(N)}
    outs = {v: [] for v in range(N)}
    for s, d, u in zip(esrc, edst, eu):
        ins[int(d)].append((int(s), int(u)))
        outs[int(s)].append((int(d), int(u)))
    S1 = np.full((N, N), INF, dtype=np.int64)
    S2 = np.full((N, N), INF, dtype=np.int64)
    cands = {b: [] for b in range(N)}  # (c, B(c,b))
    add = lambda x, y: INF if (x >= INF or y >= INF) else x + y
    maxl = int(max(layer))
    for g in range(1, maxl + 1):
        new = []
        for a in range(N):
            for b in range(N):
                if layer[b] - layer[a] != g:
                    continue
                s2 = INF
                for (bp, u) in ins[b]:
                    if layer[bp] > layer[a]:
                        s2 = min(s2, add(S2[a, bp], u))
                for (c, bc) in cands[b]:
                    assert layer[c] > layer[a]  # the guard holds for every committed entry
                    s2 = min(s2, add(S1[a, c], bc))
                ps = s2
                for (ap, u) in outs[a]:
                    if layer[ap] < layer[b]:
                        ps = min(ps, add(u, S1[ap, b]))
                for (bp, u) in ins[b]:
                    if layer[bp] > layer[a]:
                        ps = min(ps, add(S1[a, bp], u))
                S2[a, b] = s2
                S1[a, b] = min(int(B[a, b]), ps)
                if B[a, b] < ps:
                    new.append((b, a, int(B[a, b])))
        for (b, a, bv) in new:  # appended after the span, so never consumed at the same span
            cands[b].append((a, bv))
    Z = sum(len(v) for v in cands.values())
    return S1, S2, cands, Z


SHAPES = [(5, 2), (6, 2), (7, 2), (6, 3), (8, 2)]
CASES = [(seed, *SHAPES[seed % len(SHAPES)]) for seed in range(500)]


@pytest.mark.parametrize("seed,L,w", CASES)
def test_dense_equals_brute_force_and_sparse(seed, L, w):
    rng = np.random.default_rng(seed)
    p_arc = 0.15 + 0.5 * rng.random()
    layer, esrc, edst, eu, B = random_dag(rng, L, w, p_edge=0.7, p_arc=p_arc)
    D1, D2, PD = O.multiloop_dense(layer, esrc, edst, eu, B)
    bD1, bD2, bPD = brute(layer, esrc, edst, eu, B)
    N = len(layer)
    fwd = np.array([[layer[b] > layer[a] for b in range(N)] for a in range(N)])
    assert np.array_equal(D1[fwd], bD1[fwd])
    assert np.array_equal(D2[fwd], bD2[fwd])
    assert np.array_equal(PD[fwd], bPD[fwd])
    # zero-span and reverse intervals are infeasible
    assert (D1[~fwd] == INF).all() and (D2[~fwd] == INF).all()
    S1, S2, cands, Z = sparse(layer, esrc, edst, eu, B)
    assert np.array_equal(S1[fwd], D1[fwd])
    assert np.array_equal(S2[fwd], D2[fwd])
    # candidates: exactly the dense retention set of eq. (6), a subset of finite direct arcs
    dense_set = {(int(c), int(b)) for c in range(N) for b in range(N) if fwd[c, b] and B[c, b] < PD[c, b]}
    sparse_set = {(c, b) for b in cands for (c, _) in cands[b]}
    assert sparse_set == dense_set
    assert all(B[c, b] < INF for (c, b) in sparse_set)


def test_ties_are_not_retained():
    # a direct arc that is only tied by a partitionable alternative is not a candidate
    layer = np.array([0, 1, 2])
    esrc, edst, eu = np.array([0, 1]), np.array([1, 2]), np.array([0, 0], dtype=np.int64)
    B = np.full((3, 3), INF, dtype=np.int64)
    B[0, 1] = 5
    B[0, 2] = 5   # tied by arc (0,1) + edge (1,2)
    B[1, 2] = 7
    D1, D2, PD = O.multiloop_dense(layer, esrc, edst, eu, B)
    assert PD[0, 2] == 5 and not (B[0, 2] < PD[0, 2])
    S1, S2, cands, Z = sparse(layer, esrc, edst, eu, B)
    assert (0, 5) not in cands[2] and S1[0, 2] == 5
