// sd_design_noalloc: the plain design of sd_design with every device byte it needs (energy
// tables, the instance's input region and its DP tables, rings and candidate segments) placed in
// one file-scope static device array instead of library or caller allocations.  For callers that
// cannot allocate device memory.
//
// Layout of the array: [energy tables | special hairpin table | instance region A | region B],
// each start 256-byte aligned.  The array lives on every device the library runs on until the
// process ends.  Host code never uses its name as an address: at set-up (context creation on a
// device, with that device current) hipGetSymbolAddress gives this device's copy, which is kept
// per device and passed to the kernels like any other pointer.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "sd_host.h"

using namespace sd;

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // 256 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_ptr[kMaxDevices];         // this device's address of `scratch` (null until set up)
uint64_t g_params_uid[kMaxDevices];  // parameter set whose tables the array holds (0: none)

constexpr size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kEOff = 0;
constexpr size_t kSpecOff = al256(sizeof(EnergyTables));
constexpr size_t kInstOff = al256(kSpecOff + sizeof(int32_t) * kSpecSize);

}  // namespace

namespace sd {

sd_status scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(SD_E_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return SD_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the caller made `device` current
    if (e != hipSuccess || !p) {
        hipGetLastError();
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch symbol address");
    }
    g_ptr[device] = (char*)p;
    return SD_OK;
}

char* scratch_base(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace sd

extern "C" sd_status sd_design_noalloc(sd_context* c, const char* protein, const sd_codon_table* table,
                                       const sd_params* params, double lambda_kcal, sd_result* out) {
    try {
        const double t0 = now_s();
        if (!c || !table || !params || !out) return fail(SD_E_ARG, "null argument");
        hipError_t e = hipSetDevice(c->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        char* base = scratch_base(c->device);
        if (!base) return fail(SD_E_DEVICE, "the static scratch array has no address on this device");
        Lattice L;
        std::string err;
        std::vector<float> frac;
        int rc = build_lattice(protein, table->t, params->p, lambda_kcal, policy_for(c, protein, lambda_kcal, frac), L,
                               err);
        if (rc) return fail((sd_status)rc, err);
        const int64_t slots_first = L.cand_slots;
        // energy tables: uploaded when the array holds another parameter set
        const EnergyTables* Et = (const EnergyTables*)(base + kEOff);
        const int32_t* spec = (const int32_t*)(base + kSpecOff);
        {
            std::lock_guard<std::mutex> lk(g_mu);
            if (g_params_uid[c->device] != params->uid) {
                e = hipMemcpyAsync(base + kEOff, &params->p.E, sizeof(EnergyTables), hipMemcpyHostToDevice, c->stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(base + kSpecOff, params->p.spec_table.data(), sizeof(int32_t) * kSpecSize,
                                       hipMemcpyHostToDevice, c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
                if (e != hipSuccess) {
                    g_params_uid[c->device] = 0;
                    return hip_fail(e, "scratch parameter upload");
                }
                g_params_uid[c->device] = params->uid;
            }
        }
        const double tf0 = now_s();
        int overflowed = 0;
        Inst I;
        for (int attempt = 0; attempt < 2; attempt++) {
            memset(&I, 0, sizeof(I));
            InstLayout sz = layout_instance(L, nullptr, nullptr, I);
            if (!sz.a_bytes) return fail(SD_E_INTERNAL, "instance layout does not hold its arrays");
            const size_t need = kInstOff + sz.a_bytes + sz.b_bytes;
            if (need > kScratchBytes)
                return fail(SD_E_NOMEM, "the design needs " + std::to_string(need) + " bytes of device memory; the static "
                                        "scratch array of sd_design_noalloc holds " + std::to_string(kScratchBytes) +
                                        " (use sd_design)");
            char* A = base + kInstOff;
            layout_instance(L, A, A + sz.a_bytes, I);
            I.retain_all = c->opt.retain_all;
            std::vector<char> image(sz.a_bytes, 0);  // pageable host image of region A
            stage_inputs(L, I, A, image.data());
            e = hipMemcpyAsync(A, image.data(), sz.a_bytes, hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return hip_fail(e, "scratch input upload");
            int64_t ovf = 0;
            sd_status s = run_plain_on(c, L, I, Et, spec, 0, &ovf);
            if (s) return s;
            if (!ovf) break;
            if (attempt == 1) return fail(SD_E_INTERNAL, "candidate overflow with worst-case capacity");
            overflowed = 1;  // a learned reservation overflowed: exact worst-case segments
            rc = build_lattice(protein, table->t, params->p, lambda_kcal, CapPolicy(), L, err);
            if (rc) return fail((sd_status)rc, err);
        }
        const double tf1 = now_s();
        TraceOut T;
        sd_status s = trace_and_finish_on(c, L, I, Et, spec, c->last_visits, c->last_feasible, T, out);
        if (s) return s;
        out->t_fill_s = tf1 - tf0;
        out->t_total_s = now_s() - t0;
        out->n_span_launches = c->last_launches;
        out->cand_slots = L.cand_slots;
        out->cand_slots_first = slots_first;
        out->cand_overflow = overflowed;
        out->path = SD_PATH_PLAIN;
        out->sched_tuned = c->last_span_settled ? 1 : 0;
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}
