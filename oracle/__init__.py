"""ctypes binding of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this package.
The product path (the GPU library and its Python binding) never imports, links or runs it.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
INF = 1 << 62

_lib = None


class _Res(C.Structure):
    _fields_ = [
        ("energy", C.c_int32), ("objective_fixed", C.c_int64), ("path_u", C.c_int64),
        ("fixed_shift", C.c_int32), ("codon_cost", C.c_double), ("objective_kcal", C.c_double),
        ("n_states", C.c_int64), ("n_edges", C.c_int64), ("n_cells", C.c_int64),
        ("n_feasible_direct", C.c_int64), ("n_candidates", C.c_int64),
        ("visits_dense", C.c_int64), ("visits_sparse", C.c_int64), ("selfcheck_ok", C.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P64 = C.POINTER(C.c_int64)
        L.or_params_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
        L.or_params_free.argtypes = [C.c_void_p]
        L.or_design.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.c_void_p, C.c_double, C.c_int,
                                C.c_char_p, C.c_char_p, C.POINTER(_Res), P64, P64, P64, P64, P64]
        L.or_lattice_stats.argtypes = [C.c_char_p, P64, P64, P64, P64]
        L.or_fixed_shift.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.c_void_p, C.c_double]
        L.or_zuker.argtypes = [C.c_char_p, C.c_void_p, C.POINTER(C.c_int32), C.c_char_p]
        L.or_eval.argtypes = [C.c_char_p, C.c_char_p, C.c_void_p, C.POINTER(C.c_int32)]
        L.or_bruteforce.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.c_void_p, C.c_double,
                                    P64, C.POINTER(C.c_double), P64, C.POINTER(C.c_int32)]
        PC = C.POINTER(C.c_char_p)
        L.or_design_motifs.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.c_void_p, C.c_double, PC,
                                       C.c_int, C.c_int, C.c_char_p, C.c_char_p, C.POINTER(_Res)]
        L.or_design_motifs_tables.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.c_void_p, C.c_double, PC,
                                              C.c_int, C.c_int, C.c_char_p, C.c_char_p, C.POINTER(_Res),
                                              P64, P64, P64, P64, P64]
        L.or_motif_lattice.argtypes = [C.c_char_p, PC, C.c_int, P64, P64, P64, P64]
        L.or_bruteforce_motifs.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.c_void_p, C.c_double,
                                           PC, C.c_int, P64, C.POINTER(C.c_double), P64,
                                           C.POINTER(C.c_int32)]
        L.or_multiloop_dense.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int),
                                         C.POINTER(C.c_int), P64, P64, P64, P64, P64]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


class Params:
    def __init__(self, path: str):
        h = C.c_void_p()
        rc = lib().or_params_load(path.encode(), C.byref(h))
        if rc:
            raise OracleError(rc, "or_params_load")
        self.h = h
        self.path = path

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_params_free(self.h)
            self.h = None


def _w(w):
    a = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    assert a.shape == (64,)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Design:
    mrna: str
    structure: str
    energy: int
    objective_fixed: int
    path_u: int
    fixed_shift: int
    codon_cost: float
    objective_kcal: float
    n_states: int
    n_edges: int
    n_cells: int
    n_feasible_direct: int
    n_candidates: int
    visits_dense: int
    visits_sparse: int
    selfcheck_ok: bool
    tables: dict | None = None


def design(protein: str, w, params: Params, lam: float, nthreads: int = 0, tables: bool = False) -> Design:
    """Dense oracle design; tables=True also returns V (6,N,N), B, D1, D2 (N,N), X (N)."""
    n = 3 * len(protein)
    mr = C.create_string_buffer(n + 1)
    st = C.create_string_buffer(n + 1)
    res = _Res()
    wa, wp = _w(w)
    ptrs = [None] * 5
    arrs = None
    if tables:
        N = stats(protein)["n_states"]
        arrs = {"V": np.empty((6, N, N), np.int64), "B": np.empty((N, N), np.int64),
                "D1": np.empty((N, N), np.int64), "D2": np.empty((N, N), np.int64),
                "X": np.empty(N, np.int64)}
        ptrs = [arrs[k].ctypes.data_as(C.POINTER(C.c_int64)) for k in ("V", "B", "D1", "D2", "X")]
    rc = lib().or_design(protein.encode(), wp, params.h, lam, nthreads, mr, st, C.byref(res), *ptrs)
    if rc:
        raise OracleError(rc, "or_design")
    return Design(mr.value.decode(), st.value.decode(), res.energy, res.objective_fixed, res.path_u,
                  res.fixed_shift, res.codon_cost, res.objective_kcal, res.n_states, res.n_edges,
                  res.n_cells, res.n_feasible_direct, res.n_candidates, res.visits_dense,
                  res.visits_sparse, bool(res.selfcheck_ok), arrs)


def _motif_array(motifs):
    arr = (C.c_char_p * max(len(motifs), 1))(*[m.encode() for m in motifs])
    return arr, len(motifs)


INFEASIBLE = -12


def design_motifs(protein: str, w, params: Params, lam: float, motifs, nthreads: int = 0,
                  tables: bool = False) -> Design:
    """Dense oracle design over the product with the forbidden-motif matcher; tables=True also
    returns V (6,N,N), B, D1, D2 (N,N), X (N) over the product's states."""
    n = 3 * len(protein)
    mr = C.create_string_buffer(n + 1)
    st = C.create_string_buffer(n + 1)
    res = _Res()
    wa, wp = _w(w)
    arr, nm = _motif_array(motifs)
    arrs = None
    if tables:
        N = motif_lattice(protein, motifs)["n_states"]
        arrs = {"V": np.empty((6, N, N), np.int64), "B": np.empty((N, N), np.int64),
                "D1": np.empty((N, N), np.int64), "D2": np.empty((N, N), np.int64),
                "X": np.empty(N, np.int64)}
        ptrs = [arrs[k].ctypes.data_as(C.POINTER(C.c_int64)) for k in ("V", "B", "D1", "D2", "X")]
        rc = lib().or_design_motifs_tables(protein.encode(), wp, params.h, lam, arr, nm, nthreads, mr, st,
                                           C.byref(res), *ptrs)
    else:
        rc = lib().or_design_motifs(protein.encode(), wp, params.h, lam, arr, nm, nthreads, mr, st,
                                    C.byref(res))
    if rc:
        raise OracleError(rc, "or_design_motifs")
    return Design(mr.value.decode(), st.value.decode(), res.energy, res.objective_fixed, res.path_u,
                  res.fixed_shift, res.codon_cost, res.objective_kcal, res.n_states, res.n_edges,
                  res.n_cells, res.n_feasible_direct, res.n_candidates, res.visits_dense,
                  res.visits_sparse, bool(res.selfcheck_ok), arrs)


def motif_lattice(protein: str, motifs) -> dict:
    v = [C.c_int64() for _ in range(4)]
    arr, nm = _motif_array(motifs)
    rc = lib().or_motif_lattice(protein.encode(), arr, nm, *[C.byref(x) for x in v])
    if rc:
        raise OracleError(rc, "or_motif_lattice")
    return dict(zip(["n_states", "n_edges", "width", "n_paths"], [x.value for x in v]))


def design_status(protein: str, w, params: Params, lam: float) -> int:
    n = 3 * max(len(protein), 1)
    mr = C.create_string_buffer(n + 1)
    st = C.create_string_buffer(n + 1)
    res = _Res()
    wa, wp = _w(w)
    return lib().or_design(protein.encode(), wp, params.h, lam, 1, mr, st, C.byref(res),
                           None, None, None, None, None)


def stats(protein: str) -> dict:
    v = [C.c_int64() for _ in range(4)]
    rc = lib().or_lattice_stats(protein.encode(), *[C.byref(x) for x in v])
    if rc:
        raise OracleError(rc, "or_lattice_stats")
    return dict(zip(["n_states", "n_edges", "n_cells", "n_feasible_direct"], [x.value for x in v]))


def fixed_shift(protein: str, w, params: Params, lam: float) -> int:
    wa, wp = _w(w)
    return lib().or_fixed_shift(protein.encode(), wp, params.h, lam)


def zuker(seq: str, params: Params):
    e = C.c_int32()
    st = C.create_string_buffer(len(seq) + 1)
    rc = lib().or_zuker(seq.encode(), params.h, C.byref(e), st)
    if rc:
        raise OracleError(rc, "or_zuker")
    return e.value, st.value.decode()


def evaluate(seq: str, structure: str, params: Params) -> int:
    e = C.c_int32()
    rc = lib().or_eval(seq.encode(), structure.encode(), params.h, C.byref(e))
    if rc:
        raise OracleError(rc, "or_eval")
    return e.value


def bruteforce(protein: str, w, params: Params, lam: float):
    bf, bk, ns, sh = C.c_int64(), C.c_double(), C.c_int64(), C.c_int32()
    wa, wp = _w(w)
    rc = lib().or_bruteforce(protein.encode(), wp, params.h, lam, C.byref(bf), C.byref(bk),
                             C.byref(ns), C.byref(sh))
    if rc:
        raise OracleError(rc, "or_bruteforce")
    return {"best_fixed": bf.value, "best_kcal": bk.value, "n_seqs": ns.value, "shift": sh.value}


def bruteforce_motifs(protein: str, w, params: Params, lam: float, motifs):
    bf, bk, ns, sh = C.c_int64(), C.c_double(), C.c_int64(), C.c_int32()
    wa, wp = _w(w)
    arr, nm = _motif_array(motifs)
    rc = lib().or_bruteforce_motifs(protein.encode(), wp, params.h, lam, arr, nm, C.byref(bf),
                                    C.byref(bk), C.byref(ns), C.byref(sh))
    if rc:
        raise OracleError(rc, "or_bruteforce_motifs")
    return {"best_fixed": bf.value, "best_kcal": bk.value, "n_seqs": ns.value, "shift": sh.value}


def multiloop_dense(layer, esrc, edst, eu, B):
    """Abstract dense multiloop recurrences on a layered DAG (eqs. 3-5)."""
    layer = np.ascontiguousarray(layer, dtype=np.int32)
    esrc = np.ascontiguousarray(esrc, dtype=np.int32)
    edst = np.ascontiguousarray(edst, dtype=np.int32)
    eu = np.ascontiguousarray(eu, dtype=np.int64)
    B = np.ascontiguousarray(B, dtype=np.int64)
    N = len(layer)
    D1, D2, PD = (np.empty((N, N), np.int64) for _ in range(3))
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
    lp = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
    rc = lib().or_multiloop_dense(N, ip(layer), len(esrc), ip(esrc), ip(edst), lp(eu), lp(B),
                                  lp(D1), lp(D2), lp(PD))
    if rc:
        raise OracleError(rc, "or_multiloop_dense")
    return D1, D2, PD
