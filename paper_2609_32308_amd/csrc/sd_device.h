// Context object and kernel launch entry points (library-internal).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <map>
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
    bool external = false;  // arena and stream belong to the caller (sd_context_create_external)
    void* staging = nullptr;  // pinned host image of the input region
    size_t staging_bytes = 0;
    struct Sched {
        int grid = 0, threads = 256, item_waves = 4;
    };
    // Tuner state per (length, member-count) class: the candidate schedules, run one per batched
    // call until each has been measured, then the fastest for every later call of the class.
    struct Tune {
        std::vector<Sched> cands;
        std::vector<double> score;  // launch seconds per DP cell (infinite: the barrier gave up)
        int next = 0;
        bool settled = false;
        Sched best;
    };
    std::map<int, Tune> tune;
    char* tbuf = nullptr;  // pinned download buffer of the dense-table test hooks
    size_t tbuf_bytes = 0;
    bool last_graph = false;  // last batch ran as a captured graph
    double last_batch_kernel_s = 0.0, last_batch_fill_s = 0.0;
    int64_t last_batch_fallbacks = 0;
    // learned sizing policy (sd_context_set_sizer) and exact occupancy capture (sd_occupancy)
    const sd_sizer* sizer = nullptr;
    float sz_margin = 0.f;
    int sz_slack = 0;
    int force_worst = 0;
    int occ_K = 0;
    std::vector<float> occ;
    void* E_dev = nullptr;     // EnergyTables
    void* spec_dev = nullptr;  // special hairpin table
    uint64_t params_uid = 0;
    int64_t last_visits = 0, last_appends = 0, last_feasible = 0, last_overflow_span = 0;
    double last_kernel_ms = 0.0;
    int64_t last_launches = 0;
    int64_t last_timed = 0;
    std::vector<hipEvent_t> tev;  // kernel_timing / span tuning: event pairs around span launches
    // Per-span-band tile of the plain span step (layer pairs of the span -> band floor log2),
    // tuned per length class (floor log2 of the layer count): the first designs of a class run
    // one candidate tile each for every span, timed per band between events at the band
    // boundaries (spans run in order of decreasing pairs, so a band is a run of back-to-back
    // launches); then each band keeps the default tile unless another was faster by a margin.
    struct SpanTile {
        int threads = 256, item_waves = 4;
    };
    static constexpr int kSpanBands = 16, kSpanCands = 4;
    struct SpanTune {
        int next = 0;
        bool settled = false;
        double us[kSpanCands][kSpanBands] = {};
        int cnt[kSpanCands][kSpanBands] = {};
        SpanTile best[kSpanBands];
        bool tuned[kSpanBands] = {};
    };
    std::map<int, SpanTune> span_tune;
    std::vector<hipEvent_t> bev;  // span tuning: events at band boundaries
    bool last_span_settled = true;  // the last plain design's tiles were settled or fixed
    // span_check debug mode: snapshots of the committed counts and counters, digests
    char* dbg = nullptr;
    size_t dbg_bytes = 0;
};

namespace sd {
struct InstLayout {
    size_t a_bytes, b_bytes;
};
struct Lattice;
struct Params;
InstLayout layout_instance(const Lattice& L, char* A, char* B, Inst& I);
hipError_t read_stats(const Inst& I, hipStream_t st, unsigned long long out[4]);
void stage_inputs(const Lattice& L, const Inst& I, const char* devA, char* image);
hipError_t upload_pair_order();
hipError_t launch_init(const Inst& I, hipStream_t st);
// one span step: threads per workgroup with item_waves = threads / 64 (the waves share each layer
// pair), or 256 threads with item_waves = 1 (every wave on its own pair)
hipError_t launch_span(const Inst& I, const EnergyTables* E, const int32_t* spec, int g,
                       int ext_layer, int threads, int item_waves, hipStream_t st);
hipError_t launch_ext(const Inst& I, const EnergyTables* E, int L, hipStream_t st);
// canonical traceback of one design (one workgroup of eight wavefronts) / of every design of a
// device Inst array (one such workgroup each)
hipError_t launch_trace(const Inst& I, const EnergyTables* E, const int32_t* spec, hipStream_t st);
hipError_t launch_trace_many(const Inst* insts_dev, int n, const EnergyTables* E, const int32_t* spec,
                             hipStream_t st);
// multiloop recurrences of span g on an abstract DAG whose direct costs sit in the V array
hipError_t launch_ml_abstract(const Inst& I, int g, hipStream_t st);
// digest of what span step g wrote (g = 0: of every cell of a finished design) into *out
hipError_t launch_checksum(const Inst& I, int g, unsigned long long* out, hipStream_t st);
// strict candidates per right endpoint into cstrict (retain-all control)
hipError_t launch_strict_count(const Inst& I, hipStream_t st);
hipError_t launch_span_gen(const Inst& I, const EnergyTables* E, const int32_t* spec, int g,
                           int ext_layer, int num_cu, hipStream_t st);
hipError_t launch_batch_init(const Inst* insts_dev, int ninst, BatchCtl* ctl, hipStream_t st);
// persistent schedules: (64, 1), (256, 4), (256, 1), (512, 8) as (threads, waves per work item)
bool persistent_schedule_valid(int threads, int item_waves);
hipError_t persistent_occupancy(int threads, int item_waves, int* blocks_per_cu);
hipError_t launch_persistent(const Inst* insts_dev, int ninst, int nsteps, const EnergyTables* E,
                             const int32_t* spec, BatchCtl* ctl, int grid, int threads, int item_waves,
                             unsigned spin_cap, hipStream_t st);
}  // namespace sd


