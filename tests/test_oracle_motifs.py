"""CPU pins of the oracle's forbidden-motif design (Sec. 3: the codon DFA intersected with a
deterministic motif matcher; Sec. 9 reports designs that avoid a whole inventory).

The product automaton and the constrained DP are tied to things other than themselves:
  * the language of the product equals the set of synonymous mRNAs with no motif as a substring,
    counted by brute-force enumeration with plain substring search;
  * the constrained optimum equals the brute-force minimum over those mRNAs, each folded by the
    independent fixed-sequence Zuker recursion;
  * hand-worked small automata (sizes, the single surviving sequence, infeasible languages);
  * invariants: the design avoids every motif, constraints never lower the objective, a motif
    longer than the mRNA changes nothing, and more motifs never lower it either.
"""
import itertools

import pytest

import oracle as O
import sdinputs as S


def translate(mrna):
    inv = {c: aa for aa, cods in S.GENETIC_CODE.items() for c in cods}
    return "".join(inv[mrna[i:i + 3]] for i in range(0, len(mrna), 3))


def n_synonymous(p):
    n = 1
    for aa in p:
        n *= len(S.GENETIC_CODE[aa])
    return n


def motif_free(p, motifs):
    """All synonymous mRNAs of p that contain no motif (plain enumeration)."""
    out = []
    for cods in itertools.product(*[S.GENETIC_CODE[aa] for aa in p]):
        r = "".join(cods)
        if not any(m in r for m in motifs):
            out.append(r)
    return out


CASES = [(A, seed) for A in (4, 5, 6, 7) for seed in range(1, 7)]


@pytest.mark.parametrize("A,seed", CASES)
def test_product_language_is_the_motif_free_set(A, seed):
    p = S.protein(A, seed)
    motifs = S.motifs_in(p, 1 + seed % 3, seed)
    allowed = motif_free(p, motifs)
    if not allowed:
        with pytest.raises(O.OracleError) as e:
            O.motif_lattice(p, motifs)
        assert e.value.code == O.INFEASIBLE
        return
    st = O.motif_lattice(p, motifs)
    # a deterministic automaton accepts each string along exactly one path
    assert st["n_paths"] == len(allowed)
    assert st["n_paths"] < n_synonymous(p)
    bf = O.bruteforce_motifs(p, S.codon_weights(2026), O.Params(S.default_params_path()), 0.0, motifs)
    assert bf["n_seqs"] == len(allowed)


@pytest.mark.parametrize("A,seed", [(A, s) for A in (5, 6, 7) for s in range(1, 9)])
@pytest.mark.parametrize("lam", [0.0, 0.5, 4.0])
def test_constrained_design_equals_bruteforce(A, seed, lam, oparams, weights):
    p = S.protein(A, seed)
    motifs = S.motifs_in(p, 1 + seed % 3, 100 + seed)
    bf = O.bruteforce_motifs(p, weights, oparams, lam, motifs)
    if bf["n_seqs"] == 0:
        with pytest.raises(O.OracleError) as e:
            O.design_motifs(p, weights, oparams, lam, motifs)
        assert e.value.code == O.INFEASIBLE
        return
    d = O.design_motifs(p, weights, oparams, lam, motifs)
    assert d.selfcheck_ok
    assert d.fixed_shift == bf["shift"]
    assert d.objective_fixed == bf["best_fixed"]
    assert abs(d.objective_kcal - bf["best_kcal"]) <= 1e-9
    assert translate(d.mrna) == p
    assert not any(m in d.mrna for m in motifs)
    assert O.zuker(d.mrna, oparams)[0] == d.energy
    assert O.evaluate(d.mrna, d.structure, oparams) == d.energy


def test_hand_worked_automata(oparams, weights):
    # K = AA{A,G}, M = AUG.  "GA" occurs in AAGAUG only, so AAAAUG is the one coding sequence
    # left: the trie's 7 states survive (the state after AAG with matcher state "G" has no
    # allowed continuation and is removed), 6 edges, one path.
    st = O.motif_lattice("KM", ["GA"])
    assert (st["n_states"], st["n_edges"], st["width"], st["n_paths"]) == (7, 6, 1, 1)
    d = O.design_motifs("KM", weights, oparams, 0.0, ["GA"])
    assert d.mrna == "AAAAUG" and d.structure == "......"
    # "AAAA" removes AAAAUG instead
    d = O.design_motifs("KM", weights, oparams, 0.0, ["AAAA"])
    assert d.mrna == "AAGAUG"
    # both motifs: nothing is left
    for call in (lambda: O.motif_lattice("KM", ["GA", "AAAA"]),
                 lambda: O.design_motifs("KM", weights, oparams, 0.0, ["GA", "AAAA"])):
        with pytest.raises(O.OracleError) as e:
            call()
        assert e.value.code == O.INFEASIBLE
    # a single base forbids every sequence containing it
    with pytest.raises(O.OracleError) as e:
        O.design_motifs("M*", weights, oparams, 0.0, ["G"])
    assert e.value.code == O.INFEASIBLE
    # a motif longer than the mRNA: the matcher splits states but the language is unchanged
    st = O.motif_lattice("KM", ["A" * 7])
    assert st["n_paths"] == 2 and st["n_states"] > 7


def test_bad_motifs_rejected(oparams, weights):
    for bad in ([""], ["ACGT"], ["A" * 33], ["acg"]):
        with pytest.raises(O.OracleError) as e:
            O.design_motifs("MK*", weights, oparams, 0.0, bad)
        assert e.value.code == -1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_constraint_invariants(seed, oparams, weights):
    p = S.protein(40, seed)
    inv = S.motifs(8, seed, 4, 5)
    free = O.design(p, weights, oparams, 4.0, nthreads=8)
    prev = free.objective_fixed
    for k in (2, 4, 8):
        try:
            d = O.design_motifs(p, weights, oparams, 4.0, inv[:k], nthreads=8)
        except O.OracleError as e:
            assert e.code == O.INFEASIBLE
            break
        assert d.selfcheck_ok and translate(d.mrna) == p
        assert not any(m in d.mrna for m in inv[:k])
        # constraining the language can only raise the minimum
        assert d.objective_fixed >= prev
        prev = d.objective_fixed
        assert O.evaluate(d.mrna, d.structure, oparams) == d.energy
    # motifs that cannot occur leave the optimum unchanged
    long = O.design_motifs(p, weights, oparams, 4.0, ["A" * 32, "C" * 32], nthreads=8)
    assert long.objective_fixed == free.objective_fixed and long.energy == free.energy


def test_paper_scale_state_growth():
    # 16 six-base motifs widen the automata of 64- and 105-aa proteins by about 2.7x, to width
    # 10 (the paper's 217 -> 598 and 362 -> 966 nodes, width 2 -> 8 and 10, are of the same order)
    for A, lo, hi in ((64, 2.2, 3.2), (105, 2.2, 3.2)):
        p = S.protein(A, 1)
        base = O.stats(p)["n_states"]
        st = O.motif_lattice(p, S.motifs(16, 7))
        assert lo * base <= st["n_states"] <= hi * base
        assert 8 <= st["width"] <= 12
