"""CPU pins of the oracle against facts fixed by the paper and by mathematics.

Every check here runs without a GPU.  The oracle (oracle/) is the plain dense lattice DP; these
tests tie it to things other than itself:
  * an exact count printed in the paper (Sec. 9.2: alternating YI, 256 aa, no stop, has 186,565
    feasible direct intervals) -- energy-independent, pins the codon DFA, the pair set, the
    minimum hairpin and "no implicit stop";
  * lattice sizes of the seeded workloads (cells and feasible intervals per configuration);
  * brute-force enumeration of every synonymous mRNA with an independent fixed-sequence Zuker
    MFE (Sec. 7.1 runs the same kind of check);
  * special cases that reduce to a textbook routine (Met/Trp-only proteins have one synonymous
    sequence, so the design optimum is that sequence's Zuker MFE);
  * refolding and independent evaluation of every emitted design;
  * the lambda exchange argument (optimal C is non-increasing, optimal E non-decreasing, F*
    concave and non-decreasing in lambda);
  * hand-worked loop energies from explicit table entries, one per loop class.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import sdinputs as S

# ---------------------------------------------------------------------------------------------
# Exact lattice counts
# ---------------------------------------------------------------------------------------------


def test_p1_yi_feasible_direct_intervals():
    # Sec. 9.2: alternating YI at 256 aa and lambda = 0 retains 146,306 of 186,565 feasible
    # direct intervals; the denominator depends only on the automaton and the pairing rules.
    st = O.stats("YI" * 128)
    assert st["n_feasible_direct"] == 186565


@pytest.mark.parametrize("aa,expect", [(32, 2717), (64, 11317), (128, 46181)])
def test_yi_feasible_counts_smaller(aa, expect):
    # brute-force count over the width-1 YI lattice: pairable (i,j) with j - i >= 4
    seq_states = "YI" * (aa // 2)
    assert O.stats(seq_states)["n_feasible_direct"] == expect


def _brute_feasible_pairs_width1(rna_sets):
    """Count (i,j), j-i>=4, where some choice of bases at i and j pairs (position-only lattice
    when every layer has one state)."""
    pairs = {("A", "U"), ("C", "G"), ("G", "C"), ("G", "U"), ("U", "A"), ("U", "G")}
    n = len(rna_sets)
    cnt = 0
    for i in range(n):
        for j in range(i + 4, n):
            if any((x, y) in pairs for x in rna_sets[i] for y in rna_sets[j]):
                cnt += 1
    return cnt


def test_yi_count_matches_position_brute_force():
    # Y = UA{C,U}, I = AU{A,C,U}: every layer of the trie has width 1 for this protein
    sets = []
    for aa in "YI" * 16:
        cods = S.GENETIC_CODE[aa]
        for pos in range(3):
            sets.append({c[pos] for c in cods})
    assert O.stats("YI" * 16)["n_feasible_direct"] == _brute_feasible_pairs_width1(sets)


@pytest.mark.parametrize("A,seed,N,E,cells,feas", [
    (50, 1, 170, 278, 14346, 8163),
    (300, 1, 1012, 1679, 511455, 302134),
])
def test_workload_lattice_sizes(A, seed, N, E, cells, feas):
    st = O.stats(S.protein(A, seed))
    assert (st["n_states"], st["n_edges"], st["n_cells"], st["n_feasible_direct"]) == (N, E, cells, feas)


def test_trie_state_count_formula():
    # one state per codon boundary plus one per distinct first base and per distinct 2-prefix
    p = S.protein(80, 3)
    n_states = len(p) + 1
    for aa in p:
        cods = S.GENETIC_CODE[aa]
        n_states += len({c[0] for c in cods}) + len({c[:2] for c in cods})
    assert O.stats(p)["n_states"] == n_states


# ---------------------------------------------------------------------------------------------
# Brute force over all synonymous sequences (independent Zuker per sequence)
# ---------------------------------------------------------------------------------------------

BRUTE = [(A, seed) for A in (6, 7, 8) for seed in range(1, 13)]


@pytest.mark.parametrize("A,seed", BRUTE)
@pytest.mark.parametrize("lam", [0.0, 0.5, 4.0])
def test_bruteforce_objective(A, seed, lam, oparams, weights):
    p = S.protein(A, seed)
    d = O.design(p, weights, oparams, lam)
    bf = O.bruteforce(p, weights, oparams, lam)
    assert d.selfcheck_ok
    assert d.fixed_shift == bf["shift"]
    # same fixed point: exactly equal
    assert d.objective_fixed == bf["best_fixed"]
    # FP64 objective of eq. (1) within 1e-9 of the brute-force optimum
    assert abs(d.objective_kcal - bf["best_kcal"]) <= 1e-9
    # the emitted design is a synonymous sequence whose refold equals the claimed energy
    assert translate(d.mrna) == p
    assert O.zuker(d.mrna, oparams)[0] == d.energy
    assert O.evaluate(d.mrna, d.structure, oparams) == d.energy


def translate(mrna):
    inv = {c: aa for aa, cods in S.GENETIC_CODE.items() for c in cods}
    return "".join(inv[mrna[i:i + 3]] for i in range(0, len(mrna), 3))


@pytest.mark.parametrize("seed", range(1, 9))
def test_bruteforce_other_parameter_sets(seed, weights, tmp_path):
    # a different synthetic table set (and ML_base = 0) exercises other optima and ties
    path = str(tmp_path / f"p{seed}.par")
    S.write_params(path, S.synthetic_params(seed=100 + seed, ml_base=0 if seed % 2 else None))
    P = O.Params(path)
    p = S.protein(7, 40 + seed)
    for lam in (0.0, 2.0):
        d = O.design(p, weights, P, lam)
        bf = O.bruteforce(p, weights, P, lam)
        assert d.objective_fixed == bf["best_fixed"] and d.selfcheck_ok


# ---------------------------------------------------------------------------------------------
# Special cases and invariants
# ---------------------------------------------------------------------------------------------


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_met_trp_reduces_to_fixed_sequence_zuker(seed, oparams, weights):
    # one codon per residue: Syn(p) has a single sequence, so F* is its Zuker MFE (any length)
    rng = np.random.default_rng(seed)
    p = "".join(rng.choice(["M", "W"], 60))
    seq = "".join({"M": "AUG", "W": "UGG"}[a] for a in p)
    for lam in (0.0, 4.0):
        d = O.design(p, weights, oparams, lam)
        z, zs = O.zuker(seq, oparams)
        assert d.mrna == seq
        assert d.energy == z
        assert d.objective_fixed == z * (1 << d.fixed_shift)
        assert O.evaluate(seq, d.structure, oparams) == z
        assert O.evaluate(seq, zs, oparams) == z


@pytest.mark.parametrize("p", ["M", "M*", "K"])
def test_too_short_for_any_pair(p, oparams, weights):
    # fewer than five nucleotides: no pair fits, E = 0, and max w = 1 per family gives C = 0
    d = O.design(p, weights, oparams, 4.0)
    assert d.energy == 0 and d.objective_fixed == 0 and d.codon_cost == 0.0
    assert set(d.structure) == {"."}


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_lambda_exchange_invariants(seed, oparams, weights):
    p = S.protein(40, seed)
    lams = [0.0, 0.25, 1.0, 2.0, 4.0, 8.0]
    ds = [O.design(p, weights, oparams, lam) for lam in lams]
    F = [d.objective_kcal for d in ds]
    for (l1, d1), (l2, d2) in zip(zip(lams, ds), zip(lams[1:], ds[1:])):
        assert d2.codon_cost <= d1.codon_cost + 1e-12
        assert d2.energy >= d1.energy
        # each optimum is no worse than the other design re-priced at its own lambda
        assert d1.objective_kcal <= d2.energy / 100 + l1 * d2.codon_cost + 1e-9
        assert d2.objective_kcal <= d1.energy / 100 + l2 * d1.codon_cost + 1e-9
    assert all(b >= a - 1e-9 for a, b in zip(F, F[1:]))
    for i in range(1, len(lams) - 1):  # concavity on the grid
        t = (lams[i] - lams[i - 1]) / (lams[i + 1] - lams[i - 1])
        assert F[i] >= (1 - t) * F[i - 1] + t * F[i + 1] - 1e-9


@pytest.mark.parametrize("seed", range(1, 9))
@pytest.mark.parametrize("lam", [0.0, 4.0])
def test_plain50_refold_and_evaluate(seed, lam, oparams, weights):
    p = S.protein(50, seed)
    d = O.design(p, weights, oparams, lam, nthreads=4)
    assert d.selfcheck_ok
    assert translate(d.mrna) == p
    assert O.evaluate(d.mrna, d.structure, oparams) == d.energy
    assert O.zuker(d.mrna, oparams)[0] == d.energy
    # candidates are a subset of the finite direct intervals (Sec. 7.1) and visits shrink
    assert 0 < d.n_candidates <= d.n_feasible_direct
    assert d.visits_sparse <= d.visits_dense
    # C(r) recomputed in FP64 from the emitted codons, codon order
    C = sum(-math.log(weights[S.codon_index(d.mrna[i:i + 3])]) for i in range(0, len(d.mrna), 3))
    assert d.codon_cost == C


def test_invalid_inputs(oparams, weights):
    assert O.design_status("", weights, oparams, 0.0) == -2
    assert O.design_status("MK*A", weights, oparams, 0.0) == -2
    assert O.design_status("MKB", weights, oparams, 0.0) == -2
    assert O.design_status("MK", weights, oparams, -1.0) == -5
    assert O.design_status("MK", weights, oparams, float("nan")) == -5
    w = weights.copy()
    w[S.codon_index("AAA")] = 0.0
    assert O.design_status("MK", w, oparams, 0.0) == -3
    w = weights.copy()
    w[S.codon_index("AAA")] = w[S.codon_index("AAG")] = 0.5
    assert O.design_status("MK", w, oparams, 0.0) == -3


# ---------------------------------------------------------------------------------------------
# Hand-worked loop energies (one structure per loop class, expected value from explicit entries)
# ---------------------------------------------------------------------------------------------

AU, CG, GC, GU, UA, UG = range(6)
A_, C_, G_, U_ = range(4)


def _tabs():
    p = S.synthetic_params(2004)
    a = p.arrays
    return p, a, p.scalars


def _special_set(p):
    return {s for k in p.specials for s, _ in p.specials[k]}


def test_hand_hairpin_stack(oparams):
    p, a, sc = _tabs()
    # GGGAAACCC, (((...))): two GC/CG stacks and a 3-loop closed by G-C
    seq, st = "GGGAAACCC", "(((...)))"
    assert "GAAAC" not in _special_set(p)
    expect = 2 * a["stack"][GC][CG] + a["hairpin"][3]
    assert O.evaluate(seq, st, oparams) == expect


def test_hand_hairpin_terminal_and_mismatch(oparams):
    p, a, sc = _tabs()
    seq, st = "AAAAAU", "(....)"  # 4-loop closed by A-U: mismatch uses x_{i+1}=A, x_{j-1}=A
    assert seq not in _special_set(p)
    assert O.evaluate(seq, st, oparams) == a["hairpin"][4] + a["mismatch_hairpin"][AU][A_][A_] + sc["TerminalAU"]
    seq, st = "UCCCA", "(...)"  # triloop closed by U-A: terminal penalty instead of a mismatch
    assert seq not in _special_set(p)
    assert O.evaluate(seq, st, oparams) == a["hairpin"][3] + sc["TerminalAU"] + sc["TerminalAU"]


def test_hand_special_tetraloop(oparams):
    p, a, sc = _tabs()
    s, e = p.specials["tetraloop"][0]
    tau = ["AU", "CG", "GC", "GU", "UA", "UG"].index(s[0] + s[-1])
    au = sc["TerminalAU"] if tau in (AU, GU, UA, UG) else 0
    assert O.evaluate(s, "(....)", oparams) == e + au  # listed total + exterior terminal term


def test_hand_bulges(oparams):
    p, a, sc = _tabs()
    # G(GAAAC)C with a 1-bulge: G C  G AAA C A C ... build explicitly
    seq = "GA" + "GAAAC" + "C"   # pairs (0,7) G-C, (2,6) G-C, bulge of 1 (A at 1)
    st = "(.(...))"
    hp = a["hairpin"][3]
    assert O.evaluate(seq, st, oparams) == a["bulge"][1] + a["stack"][GC][CG] + hp
    seq = "GAAA" + "GAAAC" + "C"  # bulge of 3
    st = "(...(...))"
    assert O.evaluate(seq, st, oparams) == a["bulge"][3] + 0 + 0 + hp


def test_hand_interior_tables(oparams):
    p, a, sc = _tabs()
    hp = a["hairpin"][3]
    # 1x1: G A [G AAA C] C C  -> x_{i+1}=A, x_{j-1}=C
    seq, st = "GAGAAACCC", "(.(...).)"
    assert O.evaluate(seq, st, oparams) == a["int11"][GC][CG][A_][C_] + hp
    # 1x2: G A [G AAA C] U C C -> x_{i+1}=A, x_{l+1}=U, x_{j-1}=C
    seq, st = "GAGAAACUCC", "(.(...)..)"
    assert O.evaluate(seq, st, oparams) == a["int21"][GC][CG][A_][U_][C_] + hp
    # 2x1: G A U [G AAA C] C C -> rotated table: [inner][outer][x_{l+1}][x_{i+1}][x_{k-1}]
    seq, st = "GAUGAAACCC", "(..(...).)"
    assert O.evaluate(seq, st, oparams) == a["int21"][CG][GC][C_][A_][U_] + hp
    # 2x2: G A U [G AAA C] G C C
    seq, st = "GAUGAAACGCC", "(..(...)..)"
    assert O.evaluate(seq, st, oparams) == a["int22"][GC][CG][A_][U_][G_][C_] + hp


def test_hand_generic_interior(oparams):
    p, a, sc = _tabs()
    hp = a["hairpin"][3]
    nin = lambda d: min(sc["NinioMax"], sc["Ninio"] * d)
    # 1x3 (mismatch_interior_1n): G A [G AAA C] U U G C  -> x_{i+1}=A x_{k-1}=A x_{l+1}=U x_{j-1}=G
    seq, st = "GAGAAACUUGC", "(.(...)...)"
    expect = a["interior"][4] + nin(2) + a["mismatch_interior_1n"][GC][A_][G_] + a["mismatch_interior_1n"][CG][U_][A_] + hp
    assert O.evaluate(seq, st, oparams) == expect
    # 2x3 (mismatch_interior_23)
    seq, st = "GACGAAACUUGC", "(..(...)...)"
    expect = a["interior"][5] + nin(1) + a["mismatch_interior_23"][GC][A_][G_] + a["mismatch_interior_23"][CG][U_][C_] + hp
    assert O.evaluate(seq, st, oparams) == expect
    # 3x4 generic (mismatch_interior)
    seq, st = "GACUGAAACAAAGC", "(...(...)....)"
    expect = a["interior"][7] + nin(1) + a["mismatch_interior"][GC][A_][G_] + a["mismatch_interior"][CG][A_][U_] + hp
    assert O.evaluate(seq, st, oparams) == expect


def test_hand_multiloop_and_exterior(oparams):
    p, a, sc = _tabs()
    hp = a["hairpin"][3]
    # A (GAAAC) A (UAAAA) A U : multiloop closed by A-U with two branches and 2 unpaired
    seq = "A" + "A" + "GAAAC" + "A" + "UCCCA" + "U"
    st = "(." + "(...)" + "." + "(...)" + ")"
    assert "UCCCA" not in _special_set(p)
    ml = sc["ML_closing"] + sc["ML_intern"] + sc["TerminalAU"]  # closing pair A-U
    ml += (sc["ML_intern"] + 0) + (sc["ML_intern"] + sc["TerminalAU"])  # branches G-C, U-A
    ml += 2 * sc["ML_base"]
    hps = hp + (hp + sc["TerminalAU"])
    ext = sc["TerminalAU"]
    assert O.evaluate(seq, st, oparams) == ml + hps + ext
    # exterior loop with two helices: terminal penalties only
    seq, st = "GAAACAUCCCA", "(...).(...)"
    assert O.evaluate(seq, st, oparams) == hp + (hp + sc["TerminalAU"]) + sc["TerminalAU"]


def test_evaluator_scores_beyond_the_cap(oparams):
    # the 30-unpaired cap restricts the optimisation domain only (Sec. 3); the evaluator scores
    # a 31-unpaired bulge with the lxc extrapolation
    p, a, sc = _tabs()
    seq = "G" + "A" * 31 + "GAAAC" + "C"
    st = "(" + "." * 31 + "(...))"
    ext = a["bulge"][30] + round_half_away(sc["lxc"] * math.log(31 / 30))
    assert O.evaluate(seq, st, oparams) == ext + a["hairpin"][3]


def round_half_away(x):
    return int(math.floor(abs(x) + 0.5)) * (1 if x >= 0 else -1)


# ---------------------------------------------------------------------------------------------
# Zuker vs evaluator on random sequences (two independent codes)
# ---------------------------------------------------------------------------------------------


@pytest.mark.parametrize("seed", range(12))
def test_zuker_structure_evaluates_to_its_energy(seed, oparams):
    rng = np.random.default_rng(seed)
    seq = "".join(rng.choice(list("ACGU"), 30 + 7 * seed))
    e, st = O.zuker(seq, oparams)
    assert O.evaluate(seq, st, oparams) == e


@pytest.mark.parametrize("seed", range(6))
def test_zuker_is_minimal_over_enumerated_structures(seed, oparams):
    # tiny sequences: enumerate every structure in S_{3,30} and compare with Zuker
    rng = np.random.default_rng(100 + seed)
    seq = "".join(rng.choice(list("ACGU"), 13))
    best = min(O.evaluate(seq, s, oparams) for s in _all_structures(seq))
    assert O.zuker(seq, oparams)[0] == best


def _all_structures(seq):
    pairs = {"AU", "CG", "GC", "GU", "UA", "UG"}
    n = len(seq)
    memo = {}

    def rec(i, j):  # structures of seq[i..j]
        if i > j:
            return [""]
        if (i, j) in memo:
            return memo[(i, j)]
        out = ["." + s for s in rec(i + 1, j)]
        for k in range(i + 4, j + 1):
            if seq[i] + seq[k] in pairs:
                for inner in rec(i + 1, k - 1):
                    for rest in rec(k + 1, j):
                        out.append("(" + inner + ")" + rest)
        memo[(i, j)] = out
        return out

    return rec(0, n - 1)
