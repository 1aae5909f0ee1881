"""Pins of the fixed-point reading (CPU only).

The paper states the objective E + lambda * C(r) over reals (Sec. 3, eq. 1) and computes it in
doubles.  Here both the oracle and the library run an int64 fixed point: energies times 2^s plus
codon costs rounded to multiples of 2^-s.  The shift s comes from a range rule: every finite
DP value is the value of a partial design, bounded by the largest rounded codon costs plus a
bound on the energy of any partial structure, and that total must stay below 2^60.

What is pinned here, each against something other than the two implementations:
  * the rule itself, recomputed from its statement with this file's own parser of the
    parameter file, at the configured lengths (50, 300, 925, 1,976, 3,677 aa) and lambda 0 / 4,
    against the oracle and the library (host entry point sd_fixed_shift);
  * the range error: a lambda so large that no s >= 16 qualifies gives the range status on
    both sides;
  * soundness of the energy bound: every finite entry of the oracle's dense tables lies inside
    the interval the rule assumes, for the default parameters and for parameter sets drawn to
    make loops strongly negative or strongly positive;
  * the rounding claim: a design's fixed-point objective divided by 2^s is within
    A * 2^-(s+1) internal units of its FP64 objective E + 100 * lambda * C(r).
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_2609_32308_amd as sd
import sdinputs as S

LENGTHS = (50, 300, 925, 1976, 3677)


def parse_params(path):
    """Independent reader of the project's parameter text format."""
    arrays, scalars, specials = {}, {}, {}
    sec, want, buf = None, 0, []
    for raw in open(path):
        line = raw.split("#", 1)[0].strip()
        if not line or line.startswith("SPARSEDESIGN-PARAMS"):
            continue
        if line.startswith("["):
            name = line[1:line.index("]")]
            rest = line[line.index("]") + 1:].strip()
            sec = name
            if name in ("name", "scalars", "end"):
                continue
            want, buf = int(rest), []
            if name in ("triloop", "tetraloop", "hexaloop"):
                specials[name] = []
            continue
        if sec == "scalars":
            k, v = line.split()
            scalars[k] = float(v) if k == "lxc" else int(v)
        elif sec in ("triloop", "tetraloop", "hexaloop"):
            seq, e = line.split()
            specials[sec].append(int(e))
        else:
            buf.extend(line.split())
            if len(buf) == want:
                arrays[sec] = [None if t == "INF" else int(t) for t in buf]
    return arrays, scalars, specials


def loop_init(tab, lxc, m):
    if m <= 30:
        return tab[m]
    x = lxc * math.log(m / 30.0)
    return tab[30] + int(math.floor(abs(x) + 0.5)) * (1 if x >= 0 else -1)


def energy_bound(params, n):
    """max(|lower|, upper) bound on the energy of a partial structure on n nucleotides."""
    A, sc, sp = params
    tau = sc["TerminalAU"]
    au = (min(0, tau), max(0, tau))
    lows, highs = [], []
    mh = A["mismatch_hairpin"]
    inits = [loop_init(A["hairpin"], sc["lxc"], m) for m in range(3, max(n, 3) + 1)]
    lows.append(min(inits) + min(au[0], min(mh), 0))
    highs.append(max(inits) + max(au[1], max(mh), 0))
    for es in sp.values():
        lows += es
        highs += es
    st = A["stack"]
    lows += [min(st), A["bulge"][1] + min(st)]
    highs += [max(st), A["bulge"][1] + max(st)]
    for l in range(2, 31):
        lows.append(A["bulge"][l] + 2 * au[0])
        highs.append(A["bulge"][l] + 2 * au[1])
    for k in ("int11", "int21", "int22"):
        lows.append(min(A[k]))
        highs.append(max(A[k]))
    mm = A["mismatch_interior"] + A["mismatch_interior_1n"] + A["mismatch_interior_23"]
    asym = (min(0, sc["NinioMax"], 28 * sc["Ninio"]), max(0, sc["NinioMax"]))
    for l in range(2, 31):
        lows.append(A["interior"][l] + asym[0] + 2 * min(0, min(mm)))
        highs.append(A["interior"][l] + asym[1] + 2 * max(0, max(mm)))
    mlc = sc["ML_closing"] + sc["ML_intern"]
    lows.append(mlc + au[0])
    highs.append(mlc + au[1])
    br = (min(0, sc["ML_intern"] + au[0], au[0]), max(0, sc["ML_intern"] + au[1], au[1]))
    pairs = n // 2
    e_lo = pairs * (min(0, min(lows)) + br[0]) + n * min(0, sc["ML_base"])
    e_hi = pairs * (max(0, max(highs)) + br[1]) + n * max(0, sc["ML_base"])
    return e_lo, e_hi


def rounded(x):
    """llround of a non-negative double that is exactly representable after scaling."""
    f = math.floor(x)
    return int(f) + (1 if x - f >= 0.5 else 0)


def max_codon_costs(protein, w, lam, s):
    out = []
    for aa in protein:
        out.append(max(rounded(math.ldexp(100.0 * lam * -math.log(w[S.codon_index(c)]), s))
                       for c in S.GENETIC_CODE[aa]))
    return out


def shift_rule(protein, w, params, lam):
    e_lo, e_hi = energy_bound(params, 3 * len(protein))
    eb = max(-e_lo, e_hi)
    for s in range(40, 15, -1):
        if sum(max_codon_costs(protein, w, lam, s)) + eb * (1 << s) < (1 << 60):
            return s
    return None


@pytest.fixture(scope="module")
def parsed(params_path):
    return parse_params(params_path)


@pytest.fixture(scope="module")
def lib_inputs(params_path, weights):
    return sd.Params(params_path), sd.CodonTable(weights)


@pytest.mark.parametrize("A", LENGTHS)
@pytest.mark.parametrize("lam", [0.0, 4.0])
def test_shift_rule_recomputed(A, lam, parsed, oparams, weights, lib_inputs):
    p = S.protein(A, 1)
    s = shift_rule(p, weights, parsed, lam)
    assert s is not None
    assert O.fixed_shift(p, weights, oparams, lam) == s
    gp, gt = lib_inputs
    assert sd.fixed_shift(p, gt, gp, lam) == s


def test_shift_values_at_the_configured_lengths(parsed, weights):
    # the values stated with their rounding bounds in the design notes
    got = {(A, lam): shift_rule(S.protein(A, 1), weights, parsed, lam)
           for A in LENGTHS for lam in (0.0, 4.0)}
    assert got == {(50, 0.0): 40, (50, 4.0): 40, (300, 0.0): 40, (300, 4.0): 40,
                   (925, 0.0): 39, (925, 4.0): 38, (1976, 0.0): 37, (1976, 4.0): 37,
                   (3677, 0.0): 37, (3677, 4.0): 36}


def test_shift_monotone(parsed, weights):
    p = S.protein(400, 3)
    shifts = [shift_rule(p, weights, parsed, lam) for lam in (0.0, 1.0, 4.0, 16.0, 64.0)]
    assert shifts == sorted(shifts, reverse=True)
    lens = [shift_rule(S.protein(A, 3), weights, parsed, 4.0) for A in (20, 200, 2000, 6000)]
    assert lens == sorted(lens, reverse=True)


@pytest.mark.parametrize("lam", [1e12, 1e15])
def test_range_error_on_both_sides(lam, parsed, oparams, weights, lib_inputs):
    p = S.protein(40, 2)
    assert shift_rule(p, weights, parsed, lam) is None
    assert O.fixed_shift(p, weights, oparams, lam) == -6
    assert O.design_status(p, weights, oparams, lam) == -6
    gp, gt = lib_inputs
    with pytest.raises(sd.SDError) as e:
        sd.fixed_shift(p, gt, gp, lam)
    assert e.value.code == -6


def _extreme_params(seed, sign):
    """A synthetic set pushed so that loops are strongly negative (sign < 0) or positive."""
    ps = S.synthetic_params(seed=seed)
    a = {k: np.array(v, dtype=np.int64) for k, v in ps.arrays.items()}
    if sign < 0:
        a["stack"] = a["stack"] * 3
        a["mismatch_hairpin"] = a["mismatch_hairpin"] * 2
        ps.scalars["ML_intern"] = -150
        ps.scalars["ML_base"] = -5
        ps.scalars["ML_closing"] = 50
    else:
        a["stack"] = np.abs(a["stack"])
        for k in ("hairpin", "bulge", "interior"):
            a[k] = np.where(a[k] < 0, a[k], a[k] * 2)
        ps.scalars["ML_base"] = 20
        ps.scalars["ML_intern"] = 60
    ps.arrays.update(a)
    return ps


@pytest.mark.parametrize("which", ["default", "negative", "positive"])
@pytest.mark.parametrize("lam", [0.0, 4.0])
def test_tables_inside_the_bound(which, lam, params_path, weights, tmp_path):
    path = params_path
    if which != "default":
        path = str(tmp_path / f"{which}.par")
        S.write_params(path, _extreme_params(77, -1 if which == "negative" else 1))
    P = O.Params(path)
    parsed_p = parse_params(path)
    for A, seed in ((24, 3), (36, 5)):
        p = S.protein(A, seed)
        d = O.design(p, weights, P, lam, tables=True)
        s = d.fixed_shift
        assert s == shift_rule(p, weights, parsed_p, lam)
        e_lo, e_hi = energy_bound(parsed_p, 3 * A)
        lo = e_lo * (1 << s)
        hi = sum(max_codon_costs(p, weights, lam, s)) + e_hi * (1 << s)
        for k in ("V", "B", "D1", "D2", "X"):
            t = d.tables[k]
            fin = t[t < (1 << 61)]
            assert fin.size > 0
            assert int(fin.min()) >= lo, (k, int(fin.min()), lo)
            assert int(fin.max()) <= hi, (k, int(fin.max()), hi)


@pytest.mark.parametrize("A,seed", [(30, 1), (60, 2), (120, 3), (300, 1)])
def test_rounding_bound(A, seed, oparams, weights):
    p = S.protein(A, seed)
    d = O.design(p, weights, oparams, 4.0)
    s = d.fixed_shift
    exact = d.energy + 100.0 * 4.0 * d.codon_cost  # internal units, FP64
    err = abs(d.objective_fixed / 2.0 ** s - exact)
    # A codons each rounded by at most 2^-(s+1), plus the FP64 error of the comparison itself
    assert err <= A * 2.0 ** -(s + 1) + 1e-12 * max(1.0, abs(exact))


GOLDENS = {"plain300": 8, "plain925_1976": 4, "batch256": 256, "stress": 4, "motifs": 6, "motifs_wide": 2}


@pytest.mark.parametrize("name", sorted(GOLDENS))
def test_goldens_complete_under_this_rule(name, params_path, oparams, weights):
    # every stored oracle design was made under the current range rule: its shift is the one the
    # rule gives for its protein (the motif designs use the unconstrained design's shift)
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}.json")
    g = json.load(open(path))
    assert g["params_sha256"] == S.sha256_file(params_path)
    assert g["fixed_point_rule"] == "pair-bound"
    assert len(g["designs"]) == GOLDENS[name]
    for d in g["designs"]:
        assert O.fixed_shift(d["protein"], weights, oparams, d["lambda"]) == d["fixed_shift"]
