// Host-side helpers shared by the plain/batched driver and the design server.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/sparsedesign.h"
#include "sd_device.h"
#include "sd_lattice.h"
#include "sd_traceback.h"

struct sd_params {
    sd::Params p;
    uint64_t uid;
};
struct sd_codon_table {
    sd::CodonTable t;
};

namespace sd {
sd_status fail(sd_status s, const std::string& msg);
sd_status hip_fail(hipError_t e, const char* where);
double now_s();
sd_status ensure_params(sd_context* c, const sd_params* p);
// into: caller memory of table_bytes(L) (pinned for full-speed copies); else the context's
// pinned buffer, or host memory owned by T with own_storage
size_t table_bytes(const Lattice& L);
sd_status fetch_tables(sd_context* c, const Lattice& L, const Inst& I, TraceTables& T, bool own_storage = false,
                       char* into = nullptr);
sd_status fill_result(const Lattice& L, const TraceResult& R, int64_t xs, int64_t Z, int64_t visits,
                      int64_t feasible, sd_result* out);
// Copies the device traceback's O(n + N) outputs of an instance whose k_trace has run on the
// context's stream (synchronises it); counts are the strict candidates per right endpoint.
sd_status fetch_trace(sd_context* c, const Lattice& L, const Inst& I, TraceOut& T);
// Runs the traceback of one placed, filled instance and completes its result on the host.
sd_status trace_and_finish(sd_context* c, const Lattice& L, const Inst& I, int64_t visits, int64_t feasible,
                           TraceOut& T, sd_result* out);
sd_status trace_and_finish_on(sd_context* c, const Lattice& L, const Inst& I, const EnergyTables* Et,
                              const int32_t* spec, int64_t visits, int64_t feasible, TraceOut& T, sd_result* out);
// Plain-mode fill of a placed instance (one span-step launch per span) with explicit energy
// tables; kernel_timing as in sd_options (0: no events).  *overflow_span: 0 or the first span
// whose candidate appends overflowed.
sd_status run_plain_on(sd_context* c, const Lattice& L, Inst& I, const EnergyTables* Et, const int32_t* spec,
                       int kernel_timing, int64_t* overflow_span);
// Device address of this device's static scratch array (sd_noalloc.cpp), set when a context is
// created on it; null if that set-up failed.
char* scratch_base(int device);
sd_status scratch_setup(int device);
// Largest retained fraction of the worst-case slots per position bin (occupancy logging).
void occupancy_bins(const Lattice& L, const std::vector<int32_t>& counts, int K, float* y);
sd_status design_plain(sd_context* c, const char* protein, const sd_codon_table* table,
                       const sd_params* params, double lambda, sd_result* out, TraceTables* keep,
                       Lattice* keepL, const std::vector<std::string>* motifs = nullptr,
                       TraceOut* keep_trace = nullptr);
CapPolicy policy_for(const sd_context* c, const char* protein, double lambda, std::vector<float>& frac);
// destinations of the dense test layout (any may be null)
struct DenseOut {
    int64_t *V = nullptr, *B = nullptr, *S1 = nullptr, *S2 = nullptr, *X = nullptr;
};
void dense_tables(const Lattice& L, const TraceTables& T, const DenseOut& D);
}  // namespace sd
