// Context object and kernel launch entry points (library-internal).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/sparsedesign.h"
#include "sd_internal.h"

struct sd_context {
    int device = 0;
    int num_cu = 0;
    sd_options opt{};
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    void* E_dev = nullptr;     // EnergyTables
    void* spec_dev = nullptr;  // special hairpin table
    uint64_t params_uid = 0;
    int64_t last_visits = 0, last_appends = 0, last_feasible = 0, last_overflow_span = 0;
    double last_kernel_ms = 0.0;
    int64_t last_launches = 0;
    std::vector<hipEvent_t> tev;  // kernel_timing: event pairs around span launches
};

namespace sd {
hipError_t upload_pair_order();
hipError_t launch_init(const Inst& I, hipStream_t st);
hipError_t launch_span(const Inst& I, const EnergyTables* E, const int32_t* spec, int g,
                       int ext_layer, hipStream_t st);
hipError_t launch_ext(const Inst& I, const EnergyTables* E, int L, hipStream_t st);
}  // namespace sd

sd_status design_batch_impl(sd_context* ctx, int n, const char* const* proteins,
                            const double* lambdas, const sd_codon_table* table,
                            const sd_params* params, sd_result* outs);
