"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the design method: it only draws proteins, codon-usage
weights and a nearest-neighbour parameter file from seeded generators, and writes them in the
formats the two independent implementations parse.

* Proteins follow the workload recipe: Met, then residues drawn i.i.d. uniformly from the 20
  amino acids, then an explicit stop; the stop occupies one codon position and no stop is
  added implicitly (Section 3, problem definition).
* Codon weights are relative adaptiveness values w(c) = f(c) / max over synonymous f, so every
  family has maximum exactly 1 (Section 3).
* Forbidden motifs: uniform random 6-mers (16 of them widen the 64- and 105-aa automata by about
  2.7x, to width 10, as the paper's motif inventories do), or substrings of random coding
  sequences of a protein for small cases where the constraint must bind.
* Energy parameters: the genuine Turner-2004 tables are not available, so ``synthetic_params``
  draws a table set with the same array shapes and plausible signs and magnitudes. It is a
  stand-in, never the real model.
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field

import numpy as np

NUC = "ACGU"
AMINO = "ACDEFGHIKLMNPQRSTVWY"

# The standard genetic code; '*' is the stop family.
GENETIC_CODE = {
    "A": ["GCA", "GCC", "GCG", "GCU"],
    "C": ["UGC", "UGU"],
    "D": ["GAC", "GAU"],
    "E": ["GAA", "GAG"],
    "F": ["UUC", "UUU"],
    "G": ["GGA", "GGC", "GGG", "GGU"],
    "H": ["CAC", "CAU"],
    "I": ["AUA", "AUC", "AUU"],
    "K": ["AAA", "AAG"],
    "L": ["CUA", "CUC", "CUG", "CUU", "UUA", "UUG"],
    "M": ["AUG"],
    "N": ["AAC", "AAU"],
    "P": ["CCA", "CCC", "CCG", "CCU"],
    "Q": ["CAA", "CAG"],
    "R": ["AGA", "AGG", "CGA", "CGC", "CGG", "CGU"],
    "S": ["AGC", "AGU", "UCA", "UCC", "UCG", "UCU"],
    "T": ["ACA", "ACC", "ACG", "ACU"],
    "V": ["GUA", "GUC", "GUG", "GUU"],
    "W": ["UGG"],
    "Y": ["UAC", "UAU"],
    "*": ["UAA", "UAG", "UGA"],
}


def codon_index(codon: str) -> int:
    """Index 16*b1 + 4*b2 + b3 with A<C<G<U."""
    return 16 * NUC.index(codon[0]) + 4 * NUC.index(codon[1]) + NUC.index(codon[2])


def protein(A: int, seed: int) -> str:
    """Synthetic protein with A codon positions: 'M' + (A-2) uniform residues + '*'."""
    if A < 2:
        raise ValueError("A must count at least Met and the stop")
    rng = np.random.default_rng(seed)
    mid = rng.choice(list(AMINO), A - 2)
    return "M" + "".join(mid) + "*"


def codon_freqs(seed: int = 2026, floor: float = 0.05) -> np.ndarray:
    """Per-codon usage frequencies f ~ U(floor, 1], indexed by codon_index; unused codons 0."""
    rng = np.random.default_rng(seed)
    f = np.zeros(64)
    for aa in sorted(GENETIC_CODE):
        for c in GENETIC_CODE[aa]:
            f[codon_index(c)] = floor + (1.0 - floor) * (1.0 - rng.random())
    return f


def codon_weights(seed: int = 2026, floor: float = 0.05) -> np.ndarray:
    """Relative adaptiveness w = f / max over the synonymous family (max exactly 1)."""
    f = codon_freqs(seed, floor)
    w = np.zeros(64)
    for aa, cods in GENETIC_CODE.items():
        idx = [codon_index(c) for c in cods]
        mx = max(f[i] for i in idx)
        for i in idx:
            w[i] = f[i] / mx
    return w


def motifs(count: int, seed: int, lo: int = 6, hi: int = 6) -> list[str]:
    """Forbidden-motif inventory: `count` distinct uniform random strings over ACGU with lengths
    uniform in [lo, hi] (a stand-in for restriction sites and similar short sequence signals)."""
    rng = np.random.default_rng(seed)
    out: list[str] = []
    while len(out) < count:
        L = int(rng.integers(lo, hi + 1))
        m = "".join(NUC[i] for i in rng.integers(0, 4, L))
        if m not in out:
            out.append(m)
    return out


def motifs_in(protein_: str, count: int, seed: int, lo: int = 3, hi: int = 4) -> list[str]:
    """Motifs cut from random synonymous mRNAs of the protein (so that they do occur): each is a
    substring of length uniform in [lo, hi] at a uniform position of a fresh random coding
    sequence."""
    rng = np.random.default_rng(seed)
    out: list[str] = []
    tries = 0
    while len(out) < count and tries < 1000:
        tries += 1
        rna = "".join(GENETIC_CODE[aa][int(rng.integers(0, len(GENETIC_CODE[aa])))] for aa in protein_)
        L = int(rng.integers(lo, hi + 1))
        if L > len(rna):
            continue
        i = int(rng.integers(0, len(rna) - L + 1))
        m = rna[i:i + L]
        if m not in out:
            out.append(m)
    return out


def batch_lengths(count: int, lo: int, hi: int, seed: int) -> list[int]:
    """Lengths A = round(exp(U(ln lo, ln hi))) (log-uniform)."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(count)]


# ----------------------------------------------------------------------------------------------
# Synthetic nearest-neighbour parameter set (same shapes as a Turner-2004 d0 table set).
# ----------------------------------------------------------------------------------------------
PAIRS = ["AU", "CG", "GC", "GU", "UA", "UG"]
_STRENGTH = {"AU": 2, "CG": 3, "GC": 3, "GU": 1, "UA": 2, "UG": 1}


@dataclass
class ParamSet:
    name: str
    scalars: dict
    arrays: dict = field(default_factory=dict)  # name -> np.ndarray (int), INF as None-masked
    specials: dict = field(default_factory=dict)  # 'triloop'/'tetraloop'/'hexaloop' -> [(seq, e)]


def _pairable(x: str, y: str) -> bool:
    return (x + y) in PAIRS


def synthetic_params(seed: int = 2004, ml_base: int | None = None) -> ParamSet:
    """Draw a seeded parameter set with Turner-2004 d0 array shapes (values are synthetic)."""
    rng = np.random.default_rng(seed)
    r = lambda lo, hi, size=None: rng.integers(lo, hi + 1, size=size)

    stack = np.zeros((6, 6), dtype=np.int64)
    for i in range(6):
        for j in range(i, 6):
            s = _STRENGTH[PAIRS[i]] + _STRENGTH[PAIRS[j]]
            v = -(45 * s) + int(r(-40, 60))
            stack[i, j] = stack[j, i] = v

    def loop_init(base, slope, lo_m):
        arr = np.full(31, -1, dtype=np.int64)  # -1 marks INF (unused sizes)
        for m in range(lo_m, 31):
            arr[m] = int(round(base + slope * math.log(m / lo_m))) + int(r(-25, 25))
        return arr

    hairpin = loop_init(int(r(480, 580)), float(rng.uniform(80, 120)), 3)
    bulge = loop_init(int(r(300, 420)), float(rng.uniform(80, 120)), 1)
    interior = loop_init(int(r(80, 140)), float(rng.uniform(90, 130)), 2)

    mmH = r(-180, -20, (6, 4, 4)).astype(np.int64)
    mmI = r(-110, 10, (6, 4, 4)).astype(np.int64)
    mm1n = r(-60, 40, (6, 4, 4)).astype(np.int64)
    mm23 = r(-120, 20, (6, 4, 4)).astype(np.int64)
    int11 = r(-60, 200, (6, 6, 4, 4)).astype(np.int64)
    int21 = r(60, 380, (6, 6, 4, 4, 4)).astype(np.int64)
    int22 = r(-160, 320, (6, 6, 4, 4, 4, 4)).astype(np.int64)

    scalars = {
        "ML_closing": int(r(180, 420)),
        "ML_intern": int(r(-110, 40)),
        "ML_base": int(r(0, 15)) if ml_base is None else int(ml_base),
        "TerminalAU": int(r(25, 65)),
        "Ninio": int(r(40, 70)),
        "NinioMax": int(r(250, 330)),
        "lxc": round(float(rng.uniform(95.0, 120.0)), 4),
    }

    def special(m, count, lo, hi):
        out, seen = [], set()
        while len(out) < count:
            s = "".join(rng.choice(list(NUC), m + 2))
            if not _pairable(s[0], s[-1]) or s in seen:
                continue
            seen.add(s)
            out.append((s, int(r(lo, hi))))
        return sorted(out)

    specials = {
        "triloop": special(3, 4, 200, 650),
        "tetraloop": special(4, 40, 100, 500),
        "hexaloop": special(6, 8, 100, 450),
    }
    arrays = {
        "stack": stack, "mismatch_hairpin": mmH, "mismatch_interior": mmI,
        "mismatch_interior_1n": mm1n, "mismatch_interior_23": mm23,
        "int11": int11, "int21": int21, "int22": int22,
        "hairpin": hairpin, "bulge": bulge, "interior": interior,
    }
    return ParamSet(name=f"T04-shaped-synthetic-seed{seed}", scalars=scalars, arrays=arrays,
                    specials=specials)


ARRAY_ORDER = ["stack", "mismatch_hairpin", "mismatch_interior", "mismatch_interior_1n",
               "mismatch_interior_23", "int11", "int21", "int22", "hairpin", "bulge", "interior"]
SCALAR_ORDER = ["ML_closing", "ML_intern", "ML_base", "TerminalAU", "Ninio", "NinioMax", "lxc"]


def params_text(p: ParamSet) -> str:
    """Serialise a ParamSet in the project's plain-text parameter format (version 1)."""
    lines = ["SPARSEDESIGN-PARAMS 1", f"# {p.name}", f"[name] {p.name}", "[scalars]"]
    for k in SCALAR_ORDER:
        lines.append(f"{k} {p.scalars[k]}")
    for k in ARRAY_ORDER:
        a = np.asarray(p.arrays[k]).reshape(-1)
        lines.append(f"[{k}] {a.size}")
        toks = ["INF" if (k in ("hairpin", "bulge", "interior") and v < 0) else str(int(v))
                for v in a]
        for i in range(0, len(toks), 16):
            lines.append(" ".join(toks[i:i + 16]))
    for k in ("triloop", "tetraloop", "hexaloop"):
        lines.append(f"[{k}] {len(p.specials[k])}")
        for s, e in p.specials[k]:
            lines.append(f"{s} {e}")
    lines.append("[end]")
    return "\n".join(lines) + "\n"


def write_params(path: str, p: ParamSet | None = None) -> str:
    """Write a parameter file and return its SHA-256 hex digest."""
    p = p or synthetic_params()
    txt = params_text(p)
    with open(path, "w") as fh:
        fh.write(txt)
    return hashlib.sha256(txt.encode()).hexdigest()


HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "t04_synthetic_seed2004.par")


def default_params_path() -> str:
    """Path of the committed default synthetic parameter file (seed 2004)."""
    return DEFAULT_PARAMS


def sha256_file(path: str) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


if __name__ == "__main__":  # regenerate the committed default parameter file
    print(write_params(DEFAULT_PARAMS))
