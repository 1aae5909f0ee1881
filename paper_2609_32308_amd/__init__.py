"""Python binding of libsparsedesign.so (argument marshalling only).

Every step of the design DP runs in the library's gfx950 kernels; this module only converts
arguments and results.  There is no fallback: if the shared library is missing the import of
`lib()` raises, and without a gfx950 device `Context()` raises SDError(SD_E_DEVICE).

Sharing a process with PyTorch (e.g. `Context.external` on a torch stream and tensor): import
torch first.  Torch ships its own HIP runtime under the same soname as the system one the
library links; a process loads only the first, and torch cannot initialise the GPU on a runtime
the library loaded before it, while the library runs on torch's.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsparsedesign.so")
INF = 1 << 62
# sd_result.path
PATH_PLAIN, PATH_PERSISTENT, PATH_PLAIN_AFTER_BARRIER, PATH_PLAIN_AFTER_OVERFLOW = 0, 1, 2, 3

STATUS = {0: "SD_OK", -1: "SD_E_ARG", -2: "SD_E_PROTEIN", -3: "SD_E_CODON_TABLE",
          -4: "SD_E_PARAMS", -5: "SD_E_LAMBDA", -6: "SD_E_RANGE", -7: "SD_E_NOMEM",
          -8: "SD_E_DEVICE", -9: "SD_E_BUSY", -10: "SD_E_CANCELLED", -11: "SD_E_INTERNAL",
          -12: "SD_E_INFEASIBLE"}

# every function declared in include/sparsedesign.h
EXPORTS = [
    "sd_params_load", "sd_params_sha256", "sd_params_free", "sd_codon_table_from_weights",
    "sd_codon_table_from_freqs", "sd_codon_table_free", "sd_context_create", "sd_context_destroy",
    "sd_design", "sd_design_batch", "sd_design_tables", "sd_lattice_size", "sd_result_free",
    "sd_status_str", "sd_last_error", "sd_sizer_create", "sd_sizer_free", "sd_sizer_num_params",
    "sd_sizer_get_params", "sd_sizer_set_params", "sd_sizer_gradient", "sd_sizer_train",
    "sd_sizer_predict", "sd_sizer_features", "sd_context_set_sizer", "sd_occupancy",
    "sd_server_start", "sd_server_submit", "sd_server_poll", "sd_server_wait", "sd_server_get_stats",
    "sd_server_stop", "sd_lambda_envelope", "sd_design_motifs", "sd_inverse_lambda",
    "sd_design_motifs_tables", "sd_motif_lattice_size", "sd_context_create_external",
    "sd_sizer_request_bytes", "sd_fixed_shift", "sd_design_batch_tables",
    "sd_sizer_predict_host", "sd_design_noalloc", "sd_multiloop_abstract",
    "sd_tuning_save", "sd_tuning_load",
]


class SDError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        super().__init__(f"{where}: {STATUS.get(code, code)} {detail}".strip())
        self.code = code


class Options(C.Structure):
    _fields_ = [("retain_all", C.c_int), ("capacity_override", C.c_int), ("kernel_timing", C.c_int),
                ("span_threads", C.c_int), ("span_item_waves", C.c_int), ("batch_threads", C.c_int),
                ("batch_per_cu", C.c_int),
                ("batch_item_waves", C.c_int), ("span_check", C.c_int)]


class ServerCfg(C.Structure):
    _fields_ = [("pool_bytes", C.c_size_t), ("max_active", C.c_int), ("steps_per_round", C.c_int),
                ("reserved", C.c_int * 6)]


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "admitted", "completed", "fallbacks", "rounds",
                                          "peak_active", "active", "queued", "pool_in_use",
                                          "pool_high_water", "reserved_bytes", "reserved_cand_bytes")] + \
               [("gpu_seconds", C.c_double)]


class _Result(C.Structure):
    _fields_ = [
        ("mrna", C.c_void_p), ("structure", C.c_void_p), ("energy_centi", C.c_int32),
        ("codon_cost", C.c_double), ("objective_kcal", C.c_double), ("objective_fixed", C.c_int64),
        ("fixed_shift", C.c_int32), ("cai", C.c_double), ("n_states", C.c_int64),
        ("n_cells", C.c_int64), ("n_candidates", C.c_int64), ("n_visits", C.c_int64),
        ("n_feasible", C.c_int64), ("t_fill_s", C.c_double), ("t_total_s", C.c_double),
        ("t_span_kernels_s", C.c_double), ("n_span_launches", C.c_int64),
        ("cand_slots", C.c_int64), ("cand_slots_first", C.c_int64), ("cand_overflow", C.c_int32),
        ("n_timed_launches", C.c_int64), ("path", C.c_int32), ("graph_captured", C.c_int32),
        ("sched_threads", C.c_int32), ("sched_grid", C.c_int32), ("sched_item_waves", C.c_int32),
        ("sched_tuned", C.c_int32),
    ]


_lib = None


def lib():
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2609_32308_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, P64 = C.c_void_p, C.POINTER(C.c_int64)
        L.sd_params_load.argtypes = [C.c_char_p, C.c_char_p, C.POINTER(vp)]
        L.sd_params_sha256.argtypes = [vp, C.c_char_p]
        L.sd_params_free.argtypes = [vp]
        L.sd_codon_table_from_weights.argtypes = [C.POINTER(C.c_double), C.POINTER(vp)]
        L.sd_codon_table_from_freqs.argtypes = [C.POINTER(C.c_double), C.POINTER(vp)]
        L.sd_codon_table_free.argtypes = [vp]
        L.sd_context_create.argtypes = [C.c_int, C.POINTER(Options), C.POINTER(vp)]
        L.sd_context_destroy.argtypes = [vp]
        L.sd_tuning_save.argtypes = [vp, C.c_char_p]
        L.sd_tuning_load.argtypes = [vp, C.c_char_p]
        L.sd_design.argtypes = [vp, C.c_char_p, vp, vp, C.c_double, C.POINTER(_Result)]
        L.sd_design_noalloc.argtypes = [vp, C.c_char_p, vp, vp, C.c_double, C.POINTER(_Result)]
        L.sd_design_motifs.argtypes = [vp, C.c_char_p, C.POINTER(C.c_char_p), C.c_int, vp, vp, C.c_double,
                                       C.POINTER(_Result)]
        L.sd_inverse_lambda.argtypes = [vp, C.c_char_p, C.c_double, C.c_double, C.c_int, vp, vp,
                                        C.POINTER(_Result), C.POINTER(C.c_double)]
        L.sd_design_motifs_tables.argtypes = [vp, C.c_char_p, C.POINTER(C.c_char_p), C.c_int, vp, vp,
                                              C.c_double, C.POINTER(_Result), P64, P64, P64, P64, P64]
        L.sd_motif_lattice_size.argtypes = [C.c_char_p, C.POINTER(C.c_char_p), C.c_int, P64, P64]
        L.sd_context_create_external.argtypes = [vp, vp, C.c_size_t, C.POINTER(Options), C.POINTER(vp)]
        L.sd_sizer_request_bytes.argtypes = [vp, C.c_char_p, C.c_double, C.c_float, C.c_int, P64, P64, P64]
        L.sd_design_batch.argtypes = [vp, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                                      vp, vp, C.POINTER(_Result)]
        L.sd_design_tables.argtypes = [vp, C.c_char_p, vp, vp, C.c_double, C.POINTER(_Result),
                                       P64, P64, P64, P64, P64]
        L.sd_design_batch_tables.argtypes = [vp, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                                             vp, vp, C.POINTER(_Result), C.c_int, P64, P64, P64, P64, P64]
        L.sd_lattice_size.argtypes = [C.c_char_p, P64, P64]
        P32 = C.POINTER(C.c_int32)
        L.sd_multiloop_abstract.argtypes = [vp, C.c_int, P32, C.c_int, P32, P32, P64, P64, P64, P64,
                                            C.POINTER(C.c_int8), P64]
        L.sd_fixed_shift.argtypes = [C.c_char_p, vp, vp, C.c_double, C.POINTER(C.c_int32)]
        L.sd_result_free.argtypes = [C.POINTER(_Result)]
        L.sd_status_str.argtypes = [C.c_int]
        L.sd_status_str.restype = C.c_char_p
        L.sd_last_error.argtypes = []
        L.sd_last_error.restype = C.c_char_p
        PF = C.POINTER(C.c_float)
        L.sd_sizer_create.argtypes = [vp, C.c_int, C.c_int, C.c_uint64, C.POINTER(vp)]
        L.sd_sizer_free.argtypes = [vp]
        L.sd_sizer_num_params.argtypes = [vp]
        L.sd_sizer_num_params.restype = C.c_int64
        L.sd_sizer_get_params.argtypes = [vp, PF]
        L.sd_sizer_set_params.argtypes = [vp, PF]
        L.sd_sizer_gradient.argtypes = [vp, C.c_int, PF, PF, PF, PF]
        L.sd_sizer_train.argtypes = [vp, C.c_int, PF, PF, C.c_int, C.c_float, PF]
        L.sd_sizer_predict.argtypes = [vp, C.c_int, PF, PF]
        L.sd_sizer_predict_host.argtypes = [vp, C.c_int, PF, PF]
        L.sd_sizer_features.argtypes = [C.c_char_p, C.c_double, PF]
        L.sd_context_set_sizer.argtypes = [vp, vp, C.c_float, C.c_int]
        L.sd_lambda_envelope.argtypes = [vp, C.c_char_p, C.c_double, C.c_double, C.c_int, vp, vp,
                                         C.POINTER(_Result), C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.sd_occupancy.argtypes = [vp, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_double), vp, vp,
                                   C.c_int, PF, C.POINTER(_Result)]
        L.sd_server_start.argtypes = [vp, vp, vp, C.POINTER(ServerCfg), C.POINTER(vp)]
        L.sd_server_submit.argtypes = [vp, C.c_char_p, C.c_double, C.POINTER(C.c_uint64)]
        L.sd_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(_Result)]
        L.sd_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(_Result)]
        L.sd_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.sd_server_stop.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != 0:
        raise SDError(rc, where, lib().sd_last_error().decode(errors="replace"))


class Params:
    def __init__(self, path: str, expect_sha256: str | None = None):
        h = C.c_void_p()
        _check(lib().sd_params_load(path.encode(), expect_sha256.encode() if expect_sha256 else None,
                                    C.byref(h)), "sd_params_load")
        self.h = h

    @property
    def sha256(self) -> str:
        buf = C.create_string_buffer(65)
        _check(lib().sd_params_sha256(self.h, buf), "sd_params_sha256")
        return buf.value.decode()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sd_params_free(self.h)
            self.h = None


class CodonTable:
    def __init__(self, weights=None, freqs=None):
        h = C.c_void_p()
        if weights is not None:
            a = np.ascontiguousarray(weights, dtype=np.float64)
            _check(lib().sd_codon_table_from_weights(a.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)),
                   "sd_codon_table_from_weights")
        else:
            a = np.ascontiguousarray(freqs, dtype=np.float64)
            _check(lib().sd_codon_table_from_freqs(a.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)),
                   "sd_codon_table_from_freqs")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sd_codon_table_free(self.h)
            self.h = None


@dataclass
class Result:
    mrna: str
    structure: str
    energy: int
    codon_cost: float
    objective_kcal: float
    objective_fixed: int
    fixed_shift: int
    cai: float
    n_states: int
    n_cells: int
    n_candidates: int
    n_visits: int
    n_feasible: int
    t_fill_s: float
    t_total_s: float
    t_span_kernels_s: float
    n_span_launches: int
    cand_slots: int
    cand_slots_first: int
    cand_overflow: int
    n_timed_launches: int
    path: int
    graph_captured: int
    sched_threads: int
    sched_grid: int
    sched_item_waves: int
    sched_tuned: int


def _convert(r: _Result) -> Result:
    out = Result(C.string_at(r.mrna).decode(), C.string_at(r.structure).decode(), r.energy_centi,
                 r.codon_cost, r.objective_kcal, r.objective_fixed, r.fixed_shift, r.cai, r.n_states,
                 r.n_cells, r.n_candidates, r.n_visits, r.n_feasible, r.t_fill_s, r.t_total_s,
                 r.t_span_kernels_s, r.n_span_launches, r.cand_slots, r.cand_slots_first,
                 r.cand_overflow, r.n_timed_launches, r.path, r.graph_captured, r.sched_threads,
                 r.sched_grid, r.sched_item_waves, r.sched_tuned)
    lib().sd_result_free(C.byref(r))
    return out


class Context:
    def __init__(self, device: int = 0, retain_all: bool = False, capacity_override: int = 0,
                 kernel_timing: int = 0, span_threads: int = 0, batch_threads: int = 0,
                 batch_per_cu: int = 0, span_check: int = 0, batch_item_waves: int = 0,
                 span_item_waves: int = 0):
        opt = Options(int(retain_all), int(capacity_override), int(kernel_timing), int(span_threads),
                      int(span_item_waves), int(batch_threads), int(batch_per_cu), int(batch_item_waves),
                      int(span_check))
        h = C.c_void_p()
        _check(lib().sd_context_create(device, C.byref(opt), C.byref(h)), "sd_context_create")
        self.h = h

    @classmethod
    def external(cls, stream: int, pool_ptr: int, pool_bytes: int, retain_all: bool = False,
                 capacity_override: int = 0, kernel_timing: int = 0):
        """Context on a caller-owned HIP stream handle and device pool (raw addresses; the caller
        keeps both alive, e.g. torch.cuda.Stream().cuda_stream and a uint8 CUDA tensor)."""
        self = cls.__new__(cls)
        opt = Options(int(retain_all), int(capacity_override), int(kernel_timing), 0, 0, 0)
        h = C.c_void_p()
        _check(lib().sd_context_create_external(C.c_void_p(stream), C.c_void_p(pool_ptr), pool_bytes,
                                                C.byref(opt), C.byref(h)), "sd_context_create_external")
        self.h = h
        return self

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sd_context_destroy(self.h)
            self.h = None

    __del__ = close

    def tuning_save(self, path: str) -> None:
        """Writes the context's settled schedule choices to a text file (sd_tuning_save)."""
        _check(lib().sd_tuning_save(self.h, str(path).encode()), "sd_tuning_save")

    def tuning_load(self, path: str) -> None:
        """Installs a tuning file's choices as settled (sd_tuning_load; all or nothing)."""
        _check(lib().sd_tuning_load(self.h, str(path).encode()), "sd_tuning_load")

    def design(self, protein: str, table: CodonTable, params: Params, lam: float) -> Result:
        r = _Result()
        _check(lib().sd_design(self.h, protein.encode(), table.h, params.h, float(lam), C.byref(r)), "sd_design")
        return _convert(r)

    def design_noalloc(self, protein: str, table: CodonTable, params: Params, lam: float) -> Result:
        """sd_design with the device state in the library's static scratch array (no allocation)."""
        r = _Result()
        _check(lib().sd_design_noalloc(self.h, protein.encode(), table.h, params.h, float(lam), C.byref(r)),
               "sd_design_noalloc")
        return _convert(r)

    def design_motifs(self, protein: str, motifs, table: CodonTable, params: Params, lam: float) -> Result:
        """Design whose mRNA contains none of the motifs (strings over ACGU)."""
        m = list(motifs)
        arr = (C.c_char_p * max(len(m), 1))(*[x.encode() for x in m])
        r = _Result()
        _check(lib().sd_design_motifs(self.h, protein.encode(), arr, len(m), table.h, params.h, float(lam),
                                      C.byref(r)), "sd_design_motifs")
        return _convert(r)

    def inverse_lambda(self, protein: str, target_cai: float, lambda_hi: float, table: CodonTable,
                       params: Params, max_designs: int = 64):
        """(lambda, design): the smallest lambda <= lambda_hi whose supported design has CAI >= target."""
        r = _Result()
        lam = C.c_double()
        _check(lib().sd_inverse_lambda(self.h, protein.encode(), float(target_cai), float(lambda_hi),
                                       max_designs, table.h, params.h, C.byref(r), C.byref(lam)),
               "sd_inverse_lambda")
        return lam.value, _convert(r)

    def design_batch(self, proteins, lambdas, table: CodonTable, params: Params):
        n = len(proteins)
        arr = (C.c_char_p * n)(*[p.encode() for p in proteins])
        lam = (C.c_double * n)(*[float(x) for x in lambdas])
        res = (_Result * n)()
        _check(lib().sd_design_batch(self.h, n, arr, lam, table.h, params.h, res), "sd_design_batch")
        return [_convert(res[i]) for i in range(n)]

    def lambda_envelope(self, protein: str, lo: float, hi: float, table: CodonTable, params: Params,
                        max_designs: int = 64):
        """Supported designs on [lo, hi] in increasing lambda and their breakpoints."""
        res = (_Result * max_designs)()
        br = (C.c_double * (max_designs + 1))()
        n = C.c_int()
        _check(lib().sd_lambda_envelope(self.h, protein.encode(), float(lo), float(hi), int(max_designs),
                                        table.h, params.h, res, br, C.byref(n)), "sd_lambda_envelope")
        return [_convert(res[i]) for i in range(n.value)], [br[i] for i in range(n.value + 1)]

    def set_sizer(self, sizer, margin: float = 0.5, slack: int = 8):
        _check(lib().sd_context_set_sizer(self.h, sizer.h if sizer else None, float(margin), int(slack)),
               "sd_context_set_sizer")
        self._sizer = sizer  # keep alive

    def occupancy(self, proteins, lambdas, table: CodonTable, params: Params, K: int):
        """Exact per-bin candidate occupancy fractions (n, K) plus the designs."""
        n = len(proteins)
        arr = (C.c_char_p * n)(*[p.encode() for p in proteins])
        lam = (C.c_double * n)(*[float(x) for x in lambdas])
        Y = np.zeros((n, K), np.float32)
        res = (_Result * n)()
        _check(lib().sd_occupancy(self.h, n, arr, lam, table.h, params.h, K,
                                  Y.ctypes.data_as(C.POINTER(C.c_float)), res), "sd_occupancy")
        return Y, [_convert(res[i]) for i in range(n)]

    def design_tables(self, protein: str, table: CodonTable, params: Params, lam: float):
        N, _ = lattice_size(protein)
        V = np.empty((6, N, N), np.int64)
        B, S1, S2 = (np.empty((N, N), np.int64) for _ in range(3))
        X = np.empty(N, np.int64)
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
        r = _Result()
        _check(lib().sd_design_tables(self.h, protein.encode(), table.h, params.h, float(lam), C.byref(r),
                                      p(V), p(B), p(S1), p(S2), p(X)), "sd_design_tables")
        return _convert(r), {"V": V, "B": B, "S1": S1, "S2": S2, "X": X}

    def design_batch_tables(self, proteins, lambdas, table: CodonTable, params: Params, member: int):
        """design_batch plus the dense tables of one member."""
        n = len(proteins)
        N = lattice_size(proteins[member])[0] if 0 <= member < n else 1  # the library rejects the index
        arr = (C.c_char_p * n)(*[p.encode() for p in proteins])
        lam = (C.c_double * n)(*[float(x) for x in lambdas])
        res = (_Result * n)()
        V = np.empty((6, N, N), np.int64)
        B, S1, S2 = (np.empty((N, N), np.int64) for _ in range(3))
        X = np.empty(N, np.int64)
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
        _check(lib().sd_design_batch_tables(self.h, n, arr, lam, table.h, params.h, res, int(member),
                                            p(V), p(B), p(S1), p(S2), p(X)), "sd_design_batch_tables")
        return [_convert(res[i]) for i in range(n)], {"V": V, "B": B, "S1": S1, "S2": S2, "X": X}

    def multiloop_abstract(self, layer, esrc, edst, eu, B):
        """The multiloop recurrences on an abstract layered DAG: dict of dense S1, S2, cand, Z."""
        layer = np.ascontiguousarray(layer, np.int32)
        N = len(layer)
        es = np.ascontiguousarray(esrc, np.int32)
        ed = np.ascontiguousarray(edst, np.int32)
        u = np.ascontiguousarray(eu, np.int64)
        Bm = np.ascontiguousarray(B, np.int64)
        S1 = np.empty((N, N), np.int64)
        S2 = np.empty((N, N), np.int64)
        cand = np.zeros((N, N), np.int8)
        z = C.c_int64()
        p32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        p64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
        _check(lib().sd_multiloop_abstract(self.h, N, p32(layer), len(es), p32(es), p32(ed), p64(u), p64(Bm),
                                           p64(S1), p64(S2), cand.ctypes.data_as(C.POINTER(C.c_int8)),
                                           C.byref(z)), "sd_multiloop_abstract")
        return {"S1": S1, "S2": S2, "cand": cand, "Z": z.value}

    def design_motifs_tables(self, protein: str, motifs, table: CodonTable, params: Params, lam: float):
        m = list(motifs)
        N, _ = motif_lattice_size(protein, m)
        arr = (C.c_char_p * max(len(m), 1))(*[x.encode() for x in m])
        V = np.empty((6, N, N), np.int64)
        B, S1, S2 = (np.empty((N, N), np.int64) for _ in range(3))
        X = np.empty(N, np.int64)
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
        r = _Result()
        _check(lib().sd_design_motifs_tables(self.h, protein.encode(), arr, len(m), table.h, params.h,
                                             float(lam), C.byref(r), p(V), p(B), p(S1), p(S2), p(X)),
               "sd_design_motifs_tables")
        return _convert(r), {"V": V, "B": B, "S1": S1, "S2": S2, "X": X}


def motif_lattice_size(protein: str, motifs):
    m = list(motifs)
    arr = (C.c_char_p * max(len(m), 1))(*[x.encode() for x in m])
    n, c = C.c_int64(), C.c_int64()
    _check(lib().sd_motif_lattice_size(protein.encode(), arr, len(m), C.byref(n), C.byref(c)),
           "sd_motif_lattice_size")
    return n.value, c.value


def fixed_shift(protein: str, table: CodonTable, params: Params, lam: float) -> int:
    """The fixed-point shift s a design of these inputs uses (host only)."""
    s = C.c_int32()
    _check(lib().sd_fixed_shift(protein.encode(), table.h, params.h, float(lam), C.byref(s)), "sd_fixed_shift")
    return s.value


def lattice_size(protein: str):
    n, c = C.c_int64(), C.c_int64()
    _check(lib().sd_lattice_size(protein.encode(), C.byref(n), C.byref(c)), "sd_lattice_size")
    return n.value, c.value


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def features(protein: str, lam: float) -> np.ndarray:
    out = np.zeros(22, np.float32)
    _check(lib().sd_sizer_features(protein.encode(), float(lam), _fp(out)), "sd_sizer_features")
    return out


class Sizer:
    """FP32 MLP 22 -> hidden -> hidden -> K trained on the device (learned candidate sizing)."""

    def __init__(self, ctx: Context, hidden: int = 64, n_out: int = 8, seed: int = 1):
        h = C.c_void_p()
        _check(lib().sd_sizer_create(ctx.h, hidden, n_out, seed, C.byref(h)), "sd_sizer_create")
        self.h, self.hidden, self.K, self.ctx = h, hidden, n_out, ctx

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sd_sizer_free(self.h)
            self.h = None

    def request_bytes(self, protein: str, lam: float, margin: float = 0.5, slack: int = 8) -> dict:
        """Candidate slots / bytes this sizer reserves for one request, beside the worst case."""
        v = [C.c_int64() for _ in range(3)]
        _check(lib().sd_sizer_request_bytes(self.h, protein.encode(), float(lam), float(margin), int(slack),
                                            *[C.byref(x) for x in v]), "sd_sizer_request_bytes")
        return dict(zip(["cand_slots", "cand_bytes", "worst_slots"], [x.value for x in v]))

    @property
    def n_params(self) -> int:
        return lib().sd_sizer_num_params(self.h)

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        _check(lib().sd_sizer_get_params(self.h, _fp(out)), "sd_sizer_get_params")
        return out

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().sd_sizer_set_params(self.h, _fp(a)), "sd_sizer_set_params")

    def gradient(self, X, Y):
        X = np.ascontiguousarray(X, np.float32)
        Y = np.ascontiguousarray(Y, np.float32)
        loss = np.zeros(1, np.float32)
        g = np.zeros(self.n_params, np.float32)
        _check(lib().sd_sizer_gradient(self.h, len(X), _fp(X), _fp(Y), _fp(loss), _fp(g)), "sd_sizer_gradient")
        return float(loss[0]), g

    def train(self, X, Y, steps: int = 2000, lr: float = 3e-3) -> float:
        X = np.ascontiguousarray(X, np.float32)
        Y = np.ascontiguousarray(Y, np.float32)
        loss = np.zeros(1, np.float32)
        _check(lib().sd_sizer_train(self.h, len(X), _fp(X), _fp(Y), steps, lr, _fp(loss)), "sd_sizer_train")
        return float(loss[0])

    def predict(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, np.float32)
        Y = np.zeros((len(X), self.K), np.float32)
        _check(lib().sd_sizer_predict(self.h, len(X), _fp(X), _fp(Y)), "sd_sizer_predict")
        return Y

    def predict_host(self, X) -> np.ndarray:
        """The host forward pass that sizing and admission use."""
        X = np.ascontiguousarray(X, np.float32)
        Y = np.zeros((len(X), self.K), np.float32)
        _check(lib().sd_sizer_predict_host(self.h, len(X), _fp(X), _fp(Y)), "sd_sizer_predict_host")
        return Y


class Server:
    """Continuous-batching design server on one context (the context is reserved while it runs)."""

    def __init__(self, ctx: Context, table: CodonTable, params: Params, pool_bytes: int = 8 << 30,
                 max_active: int = 256, steps_per_round: int = 64):
        cfg = ServerCfg(int(pool_bytes), int(max_active), int(steps_per_round))
        h = C.c_void_p()
        _check(lib().sd_server_start(ctx.h, table.h, params.h, C.byref(cfg), C.byref(h)), "sd_server_start")
        self.h, self._keep = h, (ctx, table, params)

    def submit(self, protein: str, lam: float) -> int:
        t = C.c_uint64()
        _check(lib().sd_server_submit(self.h, protein.encode(), float(lam), C.byref(t)), "sd_server_submit")
        return t.value

    def poll(self, ticket: int):
        r = _Result()
        rc = lib().sd_server_poll(self.h, ticket, C.byref(r))
        if rc == -9:
            return None
        _check(rc, "sd_server_poll")
        return _convert(r)

    def wait(self, ticket: int) -> Result:
        r = _Result()
        _check(lib().sd_server_wait(self.h, ticket, C.byref(r)), "sd_server_wait")
        return _convert(r)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().sd_server_get_stats(self.h, C.byref(st)), "sd_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def stop(self):
        if getattr(self, "h", None):
            _check(lib().sd_server_stop(self.h), "sd_server_stop")
            self.h = None

    __del__ = stop
