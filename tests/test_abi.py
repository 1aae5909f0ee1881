"""Host-only checks of the C ABI library (no GPU needed).

The library must load, export every function declared in include/sparsedesign.h, parse the
parameter file with the same SHA-256 as hashlib, size lattices like the oracle, and reject bad
inputs before touching a device.
"""
import hashlib
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2609_32308_amd as sd
import sdinputs as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sparsedesign.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sd_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(sd.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = sd.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_params_sha256_matches_hashlib(params_path):
    P = sd.Params(params_path)
    assert P.sha256 == hashlib.sha256(open(params_path, "rb").read()).hexdigest()
    P2 = sd.Params(params_path, expect_sha256=P.sha256)
    assert P2.sha256 == P.sha256
    with pytest.raises(sd.SDError) as e:
        sd.Params(params_path, expect_sha256="0" * 64)
    assert e.value.code == -4


def test_params_rejects_malformed(tmp_path, params_path):
    txt = open(params_path).read()
    bad = tmp_path / "bad.par"
    bad.write_text(txt.replace("[int22] 9216", "[int22] 9215"))
    with pytest.raises(sd.SDError) as e:
        sd.Params(str(bad))
    assert e.value.code == -4
    with pytest.raises(sd.SDError):
        sd.Params(str(tmp_path / "missing.par"))


@pytest.mark.parametrize("p", ["M", "MK*", "YI" * 20, "MLRSTWY*", S.protein(300, 2)])
def test_lattice_size_matches_oracle(p):
    N, cells = sd.lattice_size(p)
    st = O.stats(p)
    assert (N, cells) == (st["n_states"], st["n_cells"])


@pytest.mark.parametrize("p", ["", "MK*A", "MKB", "mk", "M**"])
def test_lattice_size_rejects_bad_proteins(p):
    with pytest.raises(sd.SDError) as e:
        sd.lattice_size(p)
    assert e.value.code == -2


def test_codon_table_validation(weights):
    sd.CodonTable(weights)
    w = weights.copy()
    w[3] = 0.0
    with pytest.raises(sd.SDError) as e:
        sd.CodonTable(w)
    assert e.value.code == -3
    w[3] = 1.5
    with pytest.raises(sd.SDError):
        sd.CodonTable(w)
    f = S.codon_freqs(2026)
    sd.CodonTable(freqs=f)


def test_status_strings():
    L = sd.lib()
    for code in sd.STATUS:
        assert L.sd_status_str(code)


@pytest.mark.parametrize("A,seed,k", [(20, 1, 4), (64, 1, 16), (105, 1, 16), (60, 1, 96)])
def test_motif_lattice_size_matches_oracle(A, seed, k):
    # the library's product automaton (host only) has the oracle's state count; its cell count is
    # the row layout's (every state pair with rho(a) < rho(b))
    import oracle as O
    p = S.protein(A, seed)
    motifs = S.motifs(k, 7) if k != 96 else S.motifs(96, 3, 6, 7)
    N, cells = sd.motif_lattice_size(p, motifs)
    st = O.motif_lattice(p, motifs)
    assert N == st["n_states"]
    assert N * (N - 1) // 2 >= cells > 0


def test_motif_lattice_size_errors():
    with pytest.raises(sd.SDError) as e:
        sd.motif_lattice_size("KM", ["GA", "AAAA"])
    assert e.value.code == -12
    for bad in ([], [""], ["ACGT"], ["A" * 33]):
        with pytest.raises(sd.SDError) as e:
            sd.motif_lattice_size("MK*", bad)
        assert e.value.code == -1
    with pytest.raises(sd.SDError) as e:
        sd.motif_lattice_size(S.protein(30, 1), S.motifs(200, 3, 6, 7))
    assert e.value.code == -6
    with pytest.raises(sd.SDError) as e:
        sd.motif_lattice_size("MZ", ["GA"])
    assert e.value.code == -2


def _c_layout(tmp_path, structs):
    """sizeof and every field's offset of the header's structs, from a C program built with gcc"""
    import subprocess
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "sparsedesign.h"', "int main(void) {"]
    for cname, fields in structs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines))
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


def test_binding_structs_match_the_header_layout(tmp_path):
    # the ctypes mirrors of the header's structs have the same size and field offsets
    import ctypes
    pairs = [("sd_options", sd.Options), ("sd_result", sd._Result), ("sd_server_cfg", sd.ServerCfg),
             ("sd_server_stats", sd.ServerStats)]
    c = _c_layout(tmp_path, [(cn, [f for f, _ in py._fields_]) for cn, py in pairs])
    for cn, py in pairs:
        assert c[(cn, "size")] == ctypes.sizeof(py), cn
        for f, _ in py._fields_:
            assert c[(cn, f)] == getattr(py, f).offset, (cn, f)
