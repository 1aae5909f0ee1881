// C ABI of the library: handles, validation, device memory and the plain span-step driver.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <algorithm>
#include <thread>
#include <vector>

#include "../../include/sparsedesign.h"
#include "sd_device.h"
#include "sd_lattice.h"
#include "sd_traceback.h"
#include "sd_host.h"

using namespace sd;


namespace {
thread_local std::string g_err;
uint64_t g_uid = 1;
std::mutex g_uid_mu;
const char kCode64[65] = "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";
}  // namespace

namespace sd {
sd_status fail(sd_status s, const std::string& msg) {
    g_err = msg;
    return s;
}
sd_status hip_fail(hipError_t e, const char* where) {
    return fail(SD_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}
double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace sd

// ------------------------------------------------------------------------------------------------
extern "C" const char* sd_status_str(sd_status s) {
    switch (s) {
        case SD_OK: return "ok";
        case SD_E_ARG: return "invalid argument";
        case SD_E_PROTEIN: return "invalid protein";
        case SD_E_CODON_TABLE: return "invalid codon table";
        case SD_E_PARAMS: return "invalid parameter file";
        case SD_E_LAMBDA: return "invalid lambda";
        case SD_E_RANGE: return "fixed-point range exceeded";
        case SD_E_NOMEM: return "out of memory";
        case SD_E_DEVICE: return "device error";
        case SD_E_BUSY: return "busy";
        case SD_E_CANCELLED: return "cancelled";
        case SD_E_INTERNAL: return "internal error";
        case SD_E_INFEASIBLE: return "no coding sequence meets the constraints";
    }
    return "unknown status";
}

extern "C" const char* sd_last_error(void) { return g_err.c_str(); }

extern "C" sd_status sd_params_load(const char* path, const char* expect_sha256, sd_params** out) {
    if (!path || !out) return fail(SD_E_ARG, "null argument");
    *out = nullptr;
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(SD_E_PARAMS, std::string("cannot open ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    std::string text = ss.str();
    sd_params* p = new (std::nothrow) sd_params();
    if (!p) return fail(SD_E_NOMEM, "host allocation");
    std::string err;
    int rc = parse_params(text, p->p, err);
    if (rc) {
        delete p;
        return fail((sd_status)rc, err);
    }
    p->p.sha256 = sha256_hex(text);
    if (expect_sha256 && p->p.sha256 != expect_sha256) {
        delete p;
        return fail(SD_E_PARAMS, "parameter file SHA-256 mismatch");
    }
    {
        std::lock_guard<std::mutex> lk(g_uid_mu);
        p->uid = g_uid++;
    }
    *out = p;
    return SD_OK;
}

extern "C" sd_status sd_params_sha256(const sd_params* p, char out[65]) {
    if (!p || !out) return fail(SD_E_ARG, "null argument");
    memcpy(out, p->p.sha256.c_str(), 65);
    return SD_OK;
}

extern "C" void sd_params_free(sd_params* p) { delete p; }

extern "C" sd_status sd_codon_table_from_weights(const double w[64], sd_codon_table** out) {
    if (!w || !out) return fail(SD_E_ARG, "null argument");
    for (int i = 0; i < 64; i++)
        if (!(w[i] > 0.0 && w[i] <= 1.0)) return fail(SD_E_CODON_TABLE, "weights must lie in (0,1]");
    sd_codon_table* t = new (std::nothrow) sd_codon_table();
    if (!t) return fail(SD_E_NOMEM, "host allocation");
    memcpy(t->t.w, w, sizeof(double) * 64);
    *out = t;
    return SD_OK;
}

extern "C" sd_status sd_codon_table_from_freqs(const double f[64], sd_codon_table** out) {
    if (!f || !out) return fail(SD_E_ARG, "null argument");
    double w[64];
    for (int i = 0; i < 64; i++) {
        if (!(f[i] > 0.0) || !std::isfinite(f[i])) return fail(SD_E_CODON_TABLE, "frequencies must be positive");
        double mx = 0.0;
        for (int j = 0; j < 64; j++)
            if (kCode64[j] == kCode64[i]) mx = std::max(mx, f[j]);
        w[i] = f[i] / mx;
    }
    return sd_codon_table_from_weights(w, out);
}

extern "C" void sd_codon_table_free(sd_codon_table* t) { delete t; }

// ------------------------------------------------------------------------------------------------
namespace {
// Context on `device`; with ext_pool the caller's stream and device pool replace the library's own.
sd_status context_create(int device, const sd_options* opt, bool ext, void* ext_stream, void* ext_pool,
                         size_t ext_bytes, sd_context** out) {
    if (!out) return fail(SD_E_ARG, "null argument");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(SD_E_DEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(SD_E_ARG, "device index out of range");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SD_E_DEVICE, std::string("kernels are built for gfx950, device is ") + prop.gcnArchName);
    sd_context* c = new (std::nothrow) sd_context();
    if (!c) return fail(SD_E_NOMEM, "host allocation");
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    if (opt) c->opt = *opt;
    if (c->opt.span_threads != 0 && c->opt.span_threads != 64 && c->opt.span_threads != 256 &&
        c->opt.span_threads != 512 && c->opt.span_threads != 1024) {
        delete c;
        return fail(SD_E_ARG, "span_threads must be 0, 64, 256, 512 or 1024");
    }
    if (c->opt.span_item_waves != 0 && !(c->opt.span_item_waves == 1 && c->opt.span_threads == 256)) {
        delete c;
        return fail(SD_E_ARG, "span_item_waves must be 0, or 1 with span_threads 256");
    }
    if (c->opt.kernel_timing < 0) {
        delete c;
        return fail(SD_E_ARG, "kernel_timing must be >= 0");
    }
    if (c->opt.span_check < 0 || c->opt.span_check > 2) {
        delete c;
        return fail(SD_E_ARG, "span_check must be 0, 1 or 2");
    }
    if ((c->opt.batch_threads != 0 && c->opt.batch_threads != 64 && c->opt.batch_threads != 256 &&
         c->opt.batch_threads != 512) ||
        (c->opt.batch_threads != 0) != (c->opt.batch_per_cu > 0) || c->opt.batch_per_cu < 0) {
        delete c;
        return fail(SD_E_ARG, "batch_threads must be 0, 64, 256 or 512, with batch_per_cu > 0 exactly when it is set");
    }
    if (c->opt.batch_item_waves != 0 &&
        (c->opt.batch_threads == 0 || !persistent_schedule_valid(c->opt.batch_threads, c->opt.batch_item_waves))) {
        delete c;
        return fail(SD_E_ARG, "batch_item_waves must be 0 or one of (batch_threads, batch_item_waves) = "
                              "(64, 1), (256, 4), (256, 1), (512, 8)");
    }
    e = hipSetDevice(device);
    if (e == hipSuccess && c->opt.batch_threads) {
        int per_cu = 0;
        const int iw = c->opt.batch_item_waves ? c->opt.batch_item_waves : c->opt.batch_threads / 64;
        if (persistent_occupancy(c->opt.batch_threads, iw, &per_cu) != hipSuccess || c->opt.batch_per_cu > per_cu) {
            delete c;
            return fail(SD_E_ARG, "batch_per_cu exceeds the co-resident workgroups per CU");
        }
    }
    if (ext) {
        c->external = true;
        c->stream = (hipStream_t)ext_stream;
        c->arena = ext_pool;
        c->arena_bytes = ext_bytes;
    } else if (e == hipSuccess) {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    }
    if (e == hipSuccess) e = upload_pair_order();
    // this device's address of the static scratch array of sd_design_noalloc (its own error
    // is reported by that entry point; the other entry points do not use the array)
    if (e == hipSuccess && scratch_setup(device) != SD_OK) g_err.clear();
    if (e == hipSuccess) e = hipEventCreate(&c->ev0);
    if (e == hipSuccess) e = hipEventCreate(&c->ev1);
    if (e != hipSuccess) {
        if (c->ev0) hipEventDestroy(c->ev0);
        if (!c->external && c->stream) hipStreamDestroy(c->stream);
        delete c;
        return hip_fail(e, "context setup");
    }
    *out = c;
    return SD_OK;
}
}  // namespace

extern "C" sd_status sd_context_create(int device, const sd_options* opt, sd_context** out) {
    return context_create(device, opt, false, nullptr, nullptr, 0, out);
}

extern "C" sd_status sd_context_create_external(void* hip_stream, void* dev_pool, size_t pool_bytes,
                                                const sd_options* opt, sd_context** out) {
    if (!out) return fail(SD_E_ARG, "null argument");
    *out = nullptr;
    if (!dev_pool || pool_bytes < 4096 || ((uintptr_t)dev_pool & 255))
        return fail(SD_E_ARG, "the device pool must be a 256-byte aligned device allocation of at least 4 KiB");
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, dev_pool);
    if (e != hipSuccess || at.type != hipMemoryTypeDevice) {
        hipGetLastError();
        return fail(SD_E_ARG, "the pool is not device memory");
    }
    return context_create(at.device, opt, true, hip_stream, dev_pool, pool_bytes, out);
}

extern "C" void sd_context_destroy(sd_context* c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    if (c->arena && !c->external) hipFree(c->arena);
    if (c->staging) hipHostFree(c->staging);
    if (c->tbuf) hipHostFree(c->tbuf);
    if (c->E_dev) hipFree(c->E_dev);
    if (c->spec_dev) hipFree(c->spec_dev);
    if (c->ev0) hipEventDestroy(c->ev0);
    if (c->ev1) hipEventDestroy(c->ev1);
    for (hipEvent_t ev : c->tev) hipEventDestroy(ev);
    for (hipEvent_t ev : c->bev) hipEventDestroy(ev);
    if (c->dbg) hipFree(c->dbg);
    if (c->stream && !c->external) hipStreamDestroy(c->stream);
    delete c;
}

namespace sd {

sd_status ensure_params(sd_context* c, const sd_params* p) {
    if (c->params_uid == p->uid) return SD_OK;
    hipError_t e = hipSuccess;
    if (!c->E_dev) e = hipMalloc(&c->E_dev, sizeof(EnergyTables));
    if (e == hipSuccess && !c->spec_dev) e = hipMalloc(&c->spec_dev, sizeof(int32_t) * kSpecSize);
    if (e == hipSuccess) e = hipMemcpy(c->E_dev, &p->p.E, sizeof(EnergyTables), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->spec_dev, p->p.spec_table.data(), sizeof(int32_t) * kSpecSize, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "parameter upload");
    c->params_uid = p->uid;
    return SD_OK;
}

sd_status ensure_arena(sd_context* c, size_t bytes) {
    if (bytes <= c->arena_bytes) return SD_OK;
    if (c->external)
        return fail(SD_E_NOMEM, "the caller's device pool of " + std::to_string(c->arena_bytes) + " bytes cannot hold " +
                                    std::to_string(bytes) + " bytes");
    if (c->arena) {
        hipStreamSynchronize(c->stream);
        hipFree(c->arena);
        c->arena = nullptr;
        c->arena_bytes = 0;
    }
    size_t want = bytes + bytes / 8;
    hipError_t e = hipMalloc(&c->arena, want);
    if (e != hipSuccess) {
        hipGetLastError();
        return fail(SD_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    c->arena_bytes = want;
    return SD_OK;
}

// Device layout of one instance (see the Inst declaration): region A holds the read-only inputs
// and the small mutable arrays (uploaded from one staged host image), region B the O(N^2)
// tables and the rings.  With null bases only the sizes are computed.  Every array's extent is
// checked against its slot on the host, so a kernel indexing within an array's documented
// size stays inside the instance's regions.
InstLayout layout_instance(const Lattice& L, char* A, char* B, Inst& I) {
    const int64_t N = L.N, n = L.n;
    int64_t m = std::max<int64_t>(N + 2, std::max<int64_t>(n + 2, (int64_t)L.A + 1));
    I.U = (8 * m + 255) & ~(int64_t)255;
    I.ra = A;
    I.rb = B;
    I.nE = (int64_t)L.in_src.size();
    I.nF = (int64_t)L.fwd_meta.size();
    I.nB = (int64_t)L.bwd_meta.size();
    I.cells = L.cells;
    I.slots = L.cand_slots;
    I.n = L.n;
    I.N = L.N;
    I.A = L.A;
    I.shift = L.shift;
    I.mlbase_fx = L.mlbase_fx;
    I.retain_all = 0;
    I.g0 = 1;
    I.gwin = L.generic ? L.gwin : 0;
    I.wmax = L.wmax;
    I.njobs = L.generic ? (int64_t)L.gjobs.size() / 2 : 0;
    // extents against slots (units of U in region A, of R in region B)
    struct Ext { const void* p; int64_t bytes; int64_t slot; };
    const int64_t U = I.U, R = I.R();
    const Ext ea[] = {
        {I.layer(), 4 * N, U}, {I.off(), 4 * (n + 2), U}, {I.in_start(), 4 * (N + 1), U},
        {I.tail(), 8 * N, U}, {I.pfx(), 4 * N, U}, {I.P(), 8 * ((int64_t)L.A + 1), U},
        {I.hp_init(), 4 * (n + 1), U}, {I.rowoff(), 8 * N, U}, {I.coff(), 8 * N, U},
        {I.ccap(), 4 * N, U}, {I.ccnt(), 4 * N, U}, {I.X(), 8 * N, U},
        {I.out_dst(), 16 * N, 2 * U}, {I.out_U(), 32 * N, 4 * U}, {I.alphaU(), 32 * N, 4 * U},
        {I.betaU(), 32 * N, 4 * U}, {I.fwd_off(), 4 * (int64_t)L.fwd_off.size(), 3 * U},
        {I.bwd_off(), 4 * (int64_t)L.bwd_off.size(), 3 * U}, {I.hpB(), 8 * (int64_t)L.hpB.size(), 16 * U},
        {I.OB(), 8 * (int64_t)L.OB.size(), 72 * U}, {I.OA(), 8 * (int64_t)L.OA.size(), 72 * U},
        {I.stats(), 96, U}, {I.visits(), 8 * (n + 1), U}, {I.feasible(), 8 * (n + 1), U},
        {I.inmask(), 4 * N, U}, {I.tr_seq(), 4 * n, U}, {I.tr_pair(), 4 * n, U},
        {I.tr_stack(), 16 * (n + 2), 2 * U}, {I.cstrict(), 4 * N, U},
        {I.LM(), 8 * (int64_t)kLMRing * (n + 1) * 2, 2 * R}, {I.IDL(), 8 * (int64_t)kLMRing * N * 12, 12 * R},
        {I.JDL(), 8 * (int64_t)kLMRing * N * 12, 12 * R}, {I.BI(), 8 * (int64_t)kLMRing * N, R},
        {I.BJ(), 8 * (int64_t)kLMRing * N, R}, {I.RS(), 8 * (int64_t)kLMRing * N * 16, 16 * R},
        {I.LS(), 8 * (int64_t)kLMRing * N * 16, 16 * R}, {I.MINI(), 8 * (int64_t)kLMRing * (n + 1) * 2, 2 * R}};
    bool ok = L.fwd_crow.size() == L.fwd_meta.size() && (int64_t)L.inmask.size() == N && (int64_t)L.fwd_off.size() == 4 * N + 1 && (int64_t)L.bwd_off.size() == 4 * N + 1 &&
              (int64_t)L.hpB.size() == 16 * N && (int64_t)L.OB.size() == 72 * N && (int64_t)L.OA.size() == 72 * N;
    for (const Ext& e : ea) ok = ok && e.bytes <= e.slot;
    // the span kernels locate the cells of edge neighbours from the layering: every edge must
    // join consecutive layers (the in-edges are the out-edges reversed)
    for (int64_t e = 0; ok && e < 4 * N && e < (int64_t)L.out_dst.size(); e++) {
        const int d = L.out_dst[e];
        ok = d < 0 || (d < N && L.layer[d] == L.layer[e / 4] + 1);
    }
    if (!ok) {
        // a layout that does not hold its arrays, or an automaton whose edges skip layers, is a
        // library bug: refuse to place the instance
        InstLayout bad;
        bad.a_bytes = bad.b_bytes = 0;
        return bad;
    }
    InstLayout r;
    r.a_bytes = (I.a_bytes() + 255) & ~(int64_t)255;
    r.b_bytes = (I.b_bytes() + 255) & ~(int64_t)255;
    return r;
}

// Copy the inputs of one instance into the host image of region A (image base = device A base).
void stage_inputs(const Lattice& L, const Inst& I, const char* devA, char* image) {
    auto put = [&](const void* dptr, const void* h, size_t bytes) {
        if (bytes) memcpy(image + ((const char*)dptr - devA), h, bytes);
    };
    put(I.layer(), L.layer.data(), L.layer.size() * 4);
    put(I.off(), L.off.data(), L.off.size() * 4);
    put(I.out_dst(), L.out_dst.data(), L.out_dst.size() * 4);
    put(I.out_U(), L.out_U.data(), L.out_U.size() * 8);
    put(I.in_start(), L.in_start.data(), L.in_start.size() * 4);
    put(I.in_src(), L.in_src.data(), L.in_src.size() * 4);
    put(I.in_lab(), L.in_lab.data(), L.in_lab.size() * 4);
    put(I.in_U(), L.in_U.data(), L.in_U.size() * 8);
    put(I.tail(), L.tail.data(), L.tail.size() * 8);
    put(I.inmask(), L.inmask.data(), L.inmask.size() * 4);
    put(I.pfx(), L.pfx.data(), L.pfx.size() * 4);
    put(I.P(), L.P.data(), L.P.size() * 8);
    put(I.hp_init(), L.hp_init.data(), L.hp_init.size() * 4);
    put(I.rowoff(), L.rowoff.data(), L.rowoff.size() * 8);
    put(I.coff(), L.coff.data(), L.coff.size() * 8);
    put(I.ccap(), L.ccap.data(), L.ccap.size() * 4);
    put(I.alphaU(), L.alphaU.data(), L.alphaU.size() * 8);
    put(I.betaU(), L.betaU.data(), L.betaU.size() * 8);
    put(I.fwd_off(), L.fwd_off.data(), L.fwd_off.size() * 4);
    put(I.fwd_meta(), L.fwd_meta.data(), L.fwd_meta.size() * 4);
    put(I.fwd_cost(), L.fwd_cost.data(), L.fwd_cost.size() * 8);
    put(I.fwd_crow(), L.fwd_crow.data(), L.fwd_crow.size() * 8);
    put(I.bwd_off(), L.bwd_off.data(), L.bwd_off.size() * 4);
    put(I.bwd_meta(), L.bwd_meta.data(), L.bwd_meta.size() * 4);
    put(I.bwd_cost(), L.bwd_cost.data(), L.bwd_cost.size() * 8);
    put(I.hpB(), L.hpB.data(), L.hpB.size() * 8);
    put(I.OB(), L.OB.data(), L.OB.size() * 8);
    put(I.OA(), L.OA.data(), L.OA.size() * 8);
    if (L.generic) {
        put(I.gjob_off(), L.gjob_off.data(), L.gjob_off.size() * 8);
        put(I.gjobs(), L.gjobs.data(), L.gjobs.size() * 4);
    }
}

sd_status ensure_staging(sd_context* c, size_t bytes) {
    if (bytes <= c->staging_bytes) return SD_OK;
    if (c->staging) hipHostFree(c->staging);
    c->staging = nullptr;
    c->staging_bytes = 0;
    size_t want = bytes + bytes / 4;
    hipError_t e = hipHostMalloc(&c->staging, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        hipGetLastError();
        return fail(SD_E_NOMEM, "pinned host allocation failed");
    }
    c->staging_bytes = want;
    return SD_OK;
}

// Place one instance at the start of the arena and upload its inputs with one copy.
sd_status place_and_upload(sd_context* c, const Lattice& L, Inst& I) {
    InstLayout sz = layout_instance(L, nullptr, nullptr, I);
    if (!sz.a_bytes) return fail(SD_E_INTERNAL, "instance layout does not hold its arrays");
    sd_status s = ensure_arena(c, sz.a_bytes + sz.b_bytes);
    if (s) return s;
    s = ensure_staging(c, sz.a_bytes);
    if (s) return s;
    char* A = (char*)c->arena;
    layout_instance(L, A, A + sz.a_bytes, I);
    hipError_t e = hipStreamSynchronize(c->stream);  // staging buffer may still feed a copy
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    stage_inputs(L, I, A, (char*)c->staging);
    e = hipMemcpyAsync(A, c->staging, sz.a_bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "input upload");
    return SD_OK;
}

// Counters of a finished instance: out[0] candidate visits, out[2] earliest overflow span (all
// ones if none), out[3] cells with finite B; out[1] is unused.  Synchronises the stream.
hipError_t read_stats(const Inst& I, hipStream_t st, unsigned long long out[4]) {
    std::vector<unsigned long long> v(I.n + 1), f(I.n + 1);
    hipError_t e = hipMemcpyAsync(out, I.stats(), 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(v.data(), I.visits(), v.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(f.data(), I.feasible(), f.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    out[0] = out[1] = out[3] = 0;
    for (size_t i = 0; i < v.size(); i++) {
        out[0] += v[i];
        out[3] += f[i];
    }
    return hipSuccess;
}

// Tile of the span step for a span with `pairs` layer pairs when no tuning data decide it.  Eight
// or sixteen waves per pair shorten each pair's critical path (more of its typed-value job parts
// run at once) but leave fewer workgroups resident per CU (three of eight waves, against four of
// four), so eight pay only up to about SPAN_WIDE_PER_CU pairs per CU (of 2, 3, 4, 6, 12 and 64,
// 12 was fastest on a 1,976-aa design and 4 to 64 tied on a 300-aa one), and sixteen while there
// is at most one pair per CU.
#ifndef SPAN_WIDE_PER_CU
#define SPAN_WIDE_PER_CU 12
#endif
#ifndef SPAN_XWIDE_PER_CU
#define SPAN_XWIDE_PER_CU 1
#endif
sd_status run_plain_on(sd_context* c, const Lattice& L, Inst& I, const EnergyTables* Et, const int32_t* spec,
                       int kernel_timing, int64_t* overflow_span);

namespace {
using SpanTile = sd_context::SpanTile;
// candidate tiles of the span-band tuner, in the order the exploring designs run them
constexpr int kSpanCandThreads[sd_context::kSpanCands] = {1024, 512, 256, 256};
constexpr int kSpanCandWaves[sd_context::kSpanCands] = {16, 8, 4, 1};

SpanTile span_tile_default(const sd_context* c, int pairs) {
    SpanTile t;
    t.threads = pairs <= SPAN_XWIDE_PER_CU * c->num_cu ? 1024 : pairs <= SPAN_WIDE_PER_CU * c->num_cu ? 512 : 256;
    t.item_waves = t.threads / 64;
    return t;
}
int span_band(int pairs) {
    int b = 0;
    while ((2 << b) <= pairs && b + 1 < sd_context::kSpanBands) b++;
    return b;  // floor log2(pairs), capped
}
int span_class(const Lattice& L) { return (int)std::floor(std::log2(std::max(1, L.n))); }
}  // namespace

// Plain mode: one span-step launch per span length.  Returns the overflow span (0 if none).
sd_status run_plain(sd_context* c, const Lattice& L, Inst& I, int64_t* overflow_span) {
    return run_plain_on(c, L, I, (const EnergyTables*)c->E_dev, (const int32_t*)c->spec_dev, c->opt.kernel_timing,
                        overflow_span);
}

// The same with explicit energy tables and kernel timing (0: none).
sd_status run_plain_on(sd_context* c, const Lattice& L, Inst& I, const EnergyTables* Et, const int32_t* spec,
                       int kernel_timing, int64_t* overflow_span) {
    hipStream_t st = c->stream;
    hipError_t e = launch_init(I, st);
    // the span tiles: fixed by the caller, else the tuner's per-band choice for this length class;
    // while the class explores, this design runs the next candidate tile for every span, with
    // every launch timed
    const bool fixed = c->opt.span_threads != 0 || L.generic || c->opt.span_check != 0;
    sd_context::SpanTune* tune = fixed ? nullptr : &c->span_tune[span_class(L)];
    const bool explore = tune && !tune->settled;
    const int cand = explore ? tune->next : -1;
    c->last_span_settled = !explore;
    auto tile_for = [&](int pairs) {
        SpanTile t;
        if (c->opt.span_threads) {
            t.threads = c->opt.span_threads;
            t.item_waves = c->opt.span_item_waves ? c->opt.span_item_waves : c->opt.span_threads / 64;
        } else if (explore) {
            t.threads = kSpanCandThreads[cand];
            t.item_waves = kSpanCandWaves[cand];
        } else if (tune && tune->tuned[span_band(pairs)]) {
            t = tune->best[span_band(pairs)];
        } else {
            t = span_tile_default(c, pairs);
        }
        return t;
    };
    const bool timing = kernel_timing != 0;
    while (explore && (int)c->bev.size() < sd_context::kSpanBands + 1 && e == hipSuccess) {
        hipEvent_t ev;
        e = hipEventCreate(&ev);
        if (e == hipSuccess) c->bev.push_back(ev);
    }
    int band_now = -1, nbev = 0;
    int bev_band[sd_context::kSpanBands + 1], bev_spans[sd_context::kSpanBands + 1];
    if (timing && (int)c->tev.size() < 2 * L.n) {
        while ((int)c->tev.size() < 2 * L.n && e == hipSuccess) {
            hipEvent_t ev;
            e = hipEventCreate(&ev);
            if (e == hipSuccess) c->tev.push_back(ev);
        }
    }
    const int every = kernel_timing > 0 ? kernel_timing : 1;
    // span_check debug mode (codon trie only): snapshot of the committed candidate counts and the
    // per-layer counters, restored before every second run of a step
    const bool check = c->opt.span_check != 0 && !L.generic;
    unsigned long long* dsum = nullptr;
    char *snap_cnt = nullptr, *snap_vis = nullptr, *snap_fea = nullptr;
    const size_t cnt_b = 4 * (size_t)L.N, ctr_b = 8 * ((size_t)L.n + 1);
    if (check && e == hipSuccess) {
        const size_t need = 256 + ((cnt_b + 255) & ~(size_t)255) + 2 * ((ctr_b + 255) & ~(size_t)255);
        if (need > c->dbg_bytes) {
            if (c->dbg) hipFree(c->dbg);
            c->dbg = nullptr;
            c->dbg_bytes = 0;
            e = hipMalloc((void**)&c->dbg, need);
            if (e == hipSuccess) c->dbg_bytes = need;
        }
        dsum = (unsigned long long*)c->dbg;
        snap_cnt = c->dbg + 256;
        snap_vis = snap_cnt + ((cnt_b + 255) & ~(size_t)255);
        snap_fea = snap_vis + ((ctr_b + 255) & ~(size_t)255);
    }
    for (int g = 1; g <= L.n && e == hipSuccess; g++) {
        const bool timed = timing && (g - 1) % every == 0;
        if (explore && e == hipSuccess) {
            const int b = span_band(L.n - g + 1);  // non-increasing in g
            if (b != band_now && nbev < sd_context::kSpanBands) {
                e = hipEventRecord(c->bev[nbev], st);
                bev_band[nbev] = b;
                bev_spans[nbev] = 0;
                nbev++;
                band_now = b;
            }
            bev_spans[nbev - 1]++;
        }
        const int ext = g >= 2 ? L.n - g + 1 : -1;
        if (check) {
            e = hipMemcpyAsync(snap_cnt, I.ccnt(), cnt_b, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(snap_vis, I.visits(), ctr_b, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(snap_fea, I.feasible(), ctr_b, hipMemcpyDeviceToDevice, st);
        }
        if (timed && e == hipSuccess) e = hipEventRecord(c->tev[2 * (g - 1)], st);
        const SpanTile tile = tile_for(L.n - g + 1);
        if (e == hipSuccess && L.generic)
            e = launch_span_gen(I, Et, spec, g, ext, c->num_cu, st);
        else if (e == hipSuccess)
            e = launch_span(I, Et, spec, g, ext, tile.threads, tile.item_waves, st);
        if (timed && e == hipSuccess) e = hipEventRecord(c->tev[2 * (g - 1) + 1], st);
        if (check && e == hipSuccess) {
            // the same step again with another workgroup size from the same inputs
            e = launch_checksum(I, g, dsum, st);
            if (e == hipSuccess) e = hipMemcpyAsync(I.ccnt(), snap_cnt, cnt_b, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess && c->opt.span_check != 2)
                e = hipMemcpyAsync(I.visits(), snap_vis, ctr_b, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(I.feasible(), snap_fea, ctr_b, hipMemcpyDeviceToDevice, st);
            // another tile: sixteen shared waves, or independent waves after sixteen
            SpanTile other;
            other.threads = tile.threads == 1024 ? 256 : 1024;
            other.item_waves = tile.threads == 1024 ? 1 : 16;
            if (e == hipSuccess) e = launch_span(I, Et, spec, g, ext, other.threads, other.item_waves, st);
            if (e == hipSuccess) e = launch_checksum(I, g, dsum + 1, st);
            unsigned long long h[2] = {0, 0};
            if (e == hipSuccess) e = hipMemcpyAsync(h, dsum, sizeof(h), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e == hipSuccess && h[0] != h[1])
                return fail(SD_E_INTERNAL, "span check: span " + std::to_string(g) + " wrote different values when run "
                                           "again with " + std::to_string(other.threads) + " threads and " +
                                           std::to_string(other.item_waves) + " waves per pair instead of " +
                                           std::to_string(tile.threads) + " and " + std::to_string(tile.item_waves));
        }
    }
    if (explore && nbev > 0 && e == hipSuccess) e = hipEventRecord(c->bev[nbev], st);
    if (e == hipSuccess) e = launch_ext(I, Et, 0, st);
    unsigned long long stats[4];
    if (e == hipSuccess) e = read_stats(I, st, stats);
    if (e != hipSuccess) return hip_fail(e, "span wavefront");
    *overflow_span = stats[2] == ~0ull ? 0 : (int64_t)stats[2];
    c->last_kernel_ms = 0.0;
    c->last_launches = L.n;
    c->last_timed = 0;
    if (kernel_timing)
        for (int g = 1; g <= L.n; g += every) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, c->tev[2 * (g - 1)], c->tev[2 * (g - 1) + 1]);
            if (e != hipSuccess) return hip_fail(e, "kernel timing");
            c->last_kernel_ms += ms;
            c->last_timed++;
        }
    if (explore) {
        // time per span of each band under this candidate; after the last candidate, each band
        // keeps its default tile unless another candidate was faster by more than 3 % over at
        // least 16 spans (the smallest bands hold a few spans each, too few to rank tiles)
        for (int i = 0; i < nbev; i++) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, c->bev[i], c->bev[i + 1]);
            if (e != hipSuccess) return hip_fail(e, "span tuning timing");
            tune->us[cand][bev_band[i]] += 1e3 * ms;
            tune->cnt[cand][bev_band[i]] += bev_spans[i];
        }
        if (++tune->next == sd_context::kSpanCands) {
            for (int b = 0; b < sd_context::kSpanBands; b++) {
                const SpanTile d = span_tile_default(c, (1 << b) + (1 << b) / 2);  // the band's middle
                int dk = -1, best = -1;
                double best_us = 0;
                for (int k = 0; k < sd_context::kSpanCands; k++) {
                    if (kSpanCandThreads[k] == d.threads && kSpanCandWaves[k] == d.item_waves) dk = k;
                    if (!tune->cnt[k][b]) continue;
                    const double m = tune->us[k][b] / tune->cnt[k][b];
                    if (best < 0 || m < best_us) {
                        best = k;
                        best_us = m;
                    }
                }
                if (best < 0) continue;
                if (dk >= 0 && tune->cnt[dk][b] && best != dk &&
                    (tune->cnt[best][b] < 16 || best_us > 0.97 * (tune->us[dk][b] / tune->cnt[dk][b])))
                    best = dk;
                tune->best[b].threads = kSpanCandThreads[best];
                tune->best[b].item_waves = kSpanCandWaves[best];
                tune->tuned[b] = true;
            }
            tune->settled = true;
        }
    }
    c->last_visits = (int64_t)stats[0];
    c->last_feasible = (int64_t)stats[3];
    return SD_OK;
}

// Download a design's tables (dense test hooks).  By default into the context's pinned buffer (grown
// on demand, no host zeroing, DMA at full link speed; valid until the next download on this
// context); with own_storage into host memory owned by T (for results traced back later).
size_t table_bytes(const Lattice& L) {
    const size_t cells = (size_t)L.cells, N = (size_t)L.N, slots = (size_t)L.cand_slots;
    return cells * 72 + N * 8 + ((N * 4 + 7) & ~(size_t)7) + ((slots * 4 + 7) & ~(size_t)7) +
           (L.generic ? cells * 8 : 0);
}

sd_status fetch_tables(sd_context* c, const Lattice& L, const Inst& I, TraceTables& T, bool own_storage,
                       char* into) {
    hipStream_t st = c->stream;
    const size_t cells = (size_t)L.cells, N = (size_t)L.N, slots = (size_t)L.cand_slots;
    const size_t bytes = table_bytes(L);
    char* base;
    if (into) {
        base = into;
        T.own.reset();
    } else if (own_storage) {
        T.own.reset(new (std::nothrow) char[bytes]);
        if (!T.own) return fail(SD_E_NOMEM, "host table buffer");
        base = T.own.get();
    } else {
        if (bytes > c->tbuf_bytes) {
            hipError_t e = hipStreamSynchronize(st);
            if (e == hipSuccess && c->tbuf) e = hipHostFree(c->tbuf);
            c->tbuf = nullptr;
            c->tbuf_bytes = 0;
            const size_t want = bytes + bytes / 4;
            if (e == hipSuccess) e = hipHostMalloc((void**)&c->tbuf, want, hipHostMallocDefault);
            if (e != hipSuccess) {
                c->tbuf = nullptr;
                return hip_fail(e, "pinned table buffer");
            }
            c->tbuf_bytes = want;
        }
        base = c->tbuf;
        T.own.reset();
    }
    int64_t* V = (int64_t*)base;
    int64_t* B = V + cells * 6;
    int64_t* S1 = B + cells;
    int64_t* S2 = S1 + cells;
    int64_t* X = S2 + cells;
    int* ccnt = (int*)(X + N);
    int* cc = (int*)((char*)ccnt + ((N * 4 + 7) & ~(size_t)7));
    int64_t* G = L.generic ? (int64_t*)((char*)cc + ((slots * 4 + 7) & ~(size_t)7)) : nullptr;
    hipError_t e = hipMemcpyAsync(V, I.V(), cells * 48, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(B, I.Bt(), cells * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(S1, I.S1(), cells * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(S2, I.S2(), cells * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(X, I.X(), N * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ccnt, I.ccnt(), N * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && slots) e = hipMemcpyAsync(cc, I.cc(), slots * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && G) e = hipMemcpyAsync(G, I.Gt(), cells * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "table download");
    T.V = V;
    T.B = B;
    T.S1 = S1;
    T.S2 = S2;
    T.X = X;
    T.ccnt = ccnt;
    T.cc = cc;
    T.G = G;
    return SD_OK;
}

char* dup_str(const std::string& s) {
    char* p = (char*)malloc(s.size() + 1);
    if (p) memcpy(p, s.c_str(), s.size() + 1);
    return p;
}

sd_status fill_result(const Lattice& L, const TraceResult& R, int64_t xs, int64_t Z, int64_t visits,
                      int64_t feasible, sd_result* out) {
    sd_result r;
    memset(&r, 0, sizeof(r));
    r.mrna = dup_str(R.mrna);
    r.structure = dup_str(R.structure);
    if (!r.mrna || !r.structure) {
        free(r.mrna);
        free(r.structure);
        return fail(SD_E_NOMEM, "host allocation");
    }
    r.energy_centi = R.energy;
    r.codon_cost = R.codon_cost;
    r.objective_kcal = (double)R.energy / 100.0 + L.lambda * R.codon_cost;
    r.objective_fixed = xs;
    r.fixed_shift = L.shift;
    r.cai = exp(-R.codon_cost / (double)L.A);
    r.n_states = L.N;
    r.n_cells = L.cells;
    r.n_candidates = Z;
    r.n_visits = visits;
    r.n_feasible = feasible;
    *out = r;
    return SD_OK;
}

void sizer_predict_host(const sd_sizer* z, const float* x, float* y);
int sizer_bins(const sd_sizer* z);

// Candidate capacity policy of a context for one request (frac must outlive the policy).
CapPolicy policy_for(const sd_context* c, const char* protein, double lambda, std::vector<float>& frac) {
    CapPolicy cp;
    if (c->force_worst) return cp;
    if (c->opt.capacity_override > 0) {
        cp.override_slots = c->opt.capacity_override;
        return cp;
    }
    if (c->sizer) {
        float x[22];
        if (sd_sizer_features(protein, lambda, x) == SD_OK) {
            frac.assign(sizer_bins(c->sizer), 0.f);
            sizer_predict_host(c->sizer, x, frac.data());
            cp.frac = frac.data();
            cp.K = (int)frac.size();
            cp.margin = c->sz_margin;
            cp.slack = c->sz_slack;
        }
    }
    return cp;
}

}  // namespace sd

// Candidate reservation of one request under a sizer (what a sized context or a server reserves
// for it before any overflow), beside the worst case; 12 bytes per slot (start state + B).
extern "C" sd_status sd_sizer_request_bytes(const sd_sizer* z, const char* protein, double lambda_kcal,
                                            float margin, int slack, int64_t* cand_slots,
                                            int64_t* cand_bytes, int64_t* worst_slots) {
    using namespace sd;
    try {
        if (!z || !protein || !cand_slots || !cand_bytes || !worst_slots || !(margin >= 0.f) || slack < 0)
            return fail(SD_E_ARG, "null argument, negative margin or negative slack");
        float x[22];
        sd_status s = sd_sizer_features(protein, lambda_kcal, x);
        if (s) return s;
        std::vector<float> frac(sizer_bins(z));
        sizer_predict_host(z, x, frac.data());
        CodonTable T;
        for (int i = 0; i < 64; i++) T.w[i] = 1.0;
        Params P;
        memset(&P.E, 0, sizeof(P.E));
        CapPolicy cp;
        cp.frac = frac.data();
        cp.K = (int)frac.size();
        cp.margin = margin;
        cp.slack = slack;
        Lattice L;
        std::string err;
        int rc = build_lattice(protein, T, P, 0.0, cp, L, err);
        if (rc) return fail((sd_status)rc, err);
        *cand_slots = L.cand_slots;
        *cand_bytes = 12 * L.cand_slots;
        rc = build_lattice(protein, T, P, 0.0, CapPolicy(), L, err);
        if (rc) return fail((sd_status)rc, err);
        *worst_slots = L.cand_slots;
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    }
}

namespace sd {

// Exact occupancy of one finished design: per position bin, the largest fraction of its
// worst-case slots that any right endpoint of the bin filled with retained strict candidates
// (endpoints with fewer than 64 worst-case slots are left to the sizing slack).  A reservation
// of this fraction covers every endpoint of the bin, which is what an overflow-free size needs.
void occupancy_bins(const Lattice& L, const std::vector<int32_t>& counts, int K, float* y) {
    std::vector<double> mx(K, 0.0);
    for (int b = 0; b < L.N; b++) {
        const int lb = L.layer[b], k = position_bin(lb, L.n, K);
        const int worst = lb >= 5 ? L.off[lb - 4] : 0;
        if (worst < 64) continue;
        mx[k] = std::max(mx[k], (double)counts[b] / worst);
    }
    for (int k = 0; k < K; k++) y[k] = (float)mx[k];
}

sd_status fetch_trace(sd_context* c, const Lattice& L, const Inst& I, TraceOut& T) {
    hipStream_t st = c->stream;
    T.seq.resize(L.n);
    T.pair.resize(L.n);
    T.counts.resize(L.N);
    long long res[4];
    hipError_t e = hipSuccess;
    if (L.n > 0) e = hipMemcpyAsync(T.seq.data(), I.tr_seq(), 4 * (size_t)L.n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && L.n > 0)
        e = hipMemcpyAsync(T.pair.data(), I.tr_pair(), 4 * (size_t)L.n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(res, I.tr_res(), sizeof(res), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(T.counts.data(), I.retain_all ? I.cstrict() : I.ccnt(), 4 * (size_t)L.N,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "traceback download");
    T.energy = res[0];
    T.path_u = res[1];
    T.status = res[2];
    T.xs = res[3];
    return SD_OK;
}

sd_status trace_and_finish(sd_context* c, const Lattice& L, const Inst& I, int64_t visits, int64_t feasible,
                           TraceOut& T, sd_result* out) {
    return trace_and_finish_on(c, L, I, (const EnergyTables*)c->E_dev, (const int32_t*)c->spec_dev, visits,
                               feasible, T, out);
}

sd_status trace_and_finish_on(sd_context* c, const Lattice& L, const Inst& I, const EnergyTables* Et,
                              const int32_t* spec, int64_t visits, int64_t feasible, TraceOut& T, sd_result* out) {
    hipError_t e = launch_trace(I, Et, spec, c->stream);
    if (e == hipSuccess && I.retain_all) e = launch_strict_count(I, c->stream);
    if (e != hipSuccess) return hip_fail(e, "traceback launch");
    sd_status s = fetch_trace(c, L, I, T);
    if (s) return s;
    TraceResult R;
    std::string why;
    if (finish_trace(L, T, R, &why)) return fail(SD_E_INTERNAL, "traceback self-check failed: " + why);
    int64_t Z = 0;
    for (int v = 0; v < L.N; v++) Z += T.counts[v];
    return fill_result(L, R, T.xs, Z, visits, feasible, out);
}

// One plain design; optionally keeps its tables (dense test hooks: downloaded), its lattice and
// the traceback outputs.
sd_status design_plain(sd_context* c, const char* protein, const sd_codon_table* table,
                       const sd_params* params, double lambda, sd_result* out, TraceTables* keep,
                       Lattice* keepL, const std::vector<std::string>* motifs, TraceOut* keep_trace) {
    const double t0 = now_s();
    if (!c || !table || !params || !out) return fail(SD_E_ARG, "null argument");
    hipError_t he = hipSetDevice(c->device);
    if (he != hipSuccess) return hip_fail(he, "hipSetDevice");
    Lattice L;
    std::string err;
    std::vector<float> frac;
    CapPolicy cp0;
    if (!motifs) {
        cp0 = policy_for(c, protein, lambda, frac);
    } else if (c->opt.capacity_override > 0 && !c->force_worst) {
        cp0.override_slots = c->opt.capacity_override;  // the sizer knows unconstrained lattices only
    }
    auto build = [&](const CapPolicy& cp) {
        return motifs ? build_motif_lattice(protein, table->t, params->p, lambda, cp, *motifs, L, err)
                      : build_lattice(protein, table->t, params->p, lambda, cp, L, err);
    };
    int rc = build(cp0);
    if (rc) return fail((sd_status)rc, err);
    sd_status s = ensure_params(c, params);
    if (s) return s;
    const double tf0 = now_s();
    const int64_t slots_first = L.cand_slots;
    int overflowed = 0;
    Inst I;
    memset(&I, 0, sizeof(I));
    for (int attempt = 0; attempt < 2; attempt++) {
        s = place_and_upload(c, L, I);
        if (s) return s;
        I.retain_all = c->opt.retain_all;
        int64_t ovf = 0;
        s = run_plain(c, L, I, &ovf);
        if (s) return s;
        if (!ovf) break;
        // overflow of a predicted / overridden capacity: fall back to exact worst-case segments
        if (attempt == 1) return fail(SD_E_INTERNAL, "candidate overflow with worst-case capacity");
        c->last_overflow_span = ovf;
        overflowed = 1;
        rc = build(CapPolicy());
        if (rc) return fail((sd_status)rc, err);
    }
    const double tf1 = now_s();
    TraceOut T;
    s = trace_and_finish(c, L, I, c->last_visits, c->last_feasible, T, out);
    if (s) return s;
    out->t_fill_s = tf1 - tf0;
    out->t_total_s = now_s() - t0;
    out->t_span_kernels_s = c->last_kernel_ms * 1e-3;
    out->n_span_launches = c->last_launches;
    out->n_timed_launches = c->last_timed;
    out->sched_tuned = c->last_span_settled ? 1 : 0;
    out->cand_slots = L.cand_slots;
    out->cand_slots_first = slots_first;
    out->cand_overflow = overflowed;
    if (keep) {
        s = fetch_tables(c, L, I, *keep, true);
        if (s) {
            sd_result_free(out);
            return s;
        }
    }
    if (keep_trace) *keep_trace = std::move(T);
    if (keepL) *keepL = std::move(L);
    return SD_OK;
}

}  // namespace sd

extern "C" sd_status sd_design(sd_context* ctx, const char* protein, const sd_codon_table* table,
                               const sd_params* params, double lambda_kcal, sd_result* out) {
    try {
        return design_plain(ctx, protein, table, params, lambda_kcal, out, nullptr, nullptr, nullptr);
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}

extern "C" sd_status sd_design_motifs(sd_context* ctx, const char* protein, const char* const* motifs,
                                      int n_motifs, const sd_codon_table* table, const sd_params* params,
                                      double lambda_kcal, sd_result* out) {
    try {
        if (!motifs || n_motifs < 1 || n_motifs > kMaxMotifs) return fail(SD_E_ARG, "need 1 to 256 motifs");
        std::vector<std::string> ms;
        for (int i = 0; i < n_motifs; i++) {
            if (!motifs[i]) return fail(SD_E_ARG, "null motif");
            ms.push_back(motifs[i]);
        }
        return design_plain(ctx, protein, table, params, lambda_kcal, out, nullptr, nullptr, &ms);
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}

extern "C" sd_status sd_lattice_size(const char* protein, int64_t* n_states, int64_t* n_cells) {
    if (!n_states || !n_cells) return fail(SD_E_ARG, "null argument");
    int rc = check_protein(protein);
    if (rc) return fail((sd_status)rc, "invalid protein");
    CodonTable T;
    for (int i = 0; i < 64; i++) T.w[i] = 1.0;
    Params P;
    memset(&P.E, 0, sizeof(P.E));
    Lattice L;
    std::string err;
    rc = build_lattice(protein, T, P, 0.0, CapPolicy(), L, err);
    if (rc) return fail((sd_status)rc, err);
    *n_states = L.N;
    *n_cells = L.cells;
    return SD_OK;
}

extern "C" sd_status sd_fixed_shift(const char* protein, const sd_codon_table* table, const sd_params* params,
                                   double lambda_kcal, int32_t* shift) {
    try {
        if (!table || !params || !shift) return fail(SD_E_ARG, "null argument");
        Lattice L;
        std::string err;
        int rc = build_lattice(protein, table->t, params->p, lambda_kcal, CapPolicy(), L, err);
        if (rc) return fail((sd_status)rc, err);
        *shift = L.shift;
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    }
}

namespace sd {
// Copies downloaded tables into the dense test layout [a * N + b] (V: [tau][a][b]); entries with
// rho(a) >= rho(b) are INF.  Null destinations are skipped.
void dense_tables(const Lattice& L, const TraceTables& T, const DenseOut& D) {
    const size_t N = L.N;
    auto dense = [&](int64_t* dst, const int64_t* src, int stride, int t) {
        if (!dst) return;
        for (size_t a = 0; a < N; a++)
            for (size_t b = 0; b < N; b++) {
                int64_t v = kINF;
                if (L.layer[a] < L.layer[b]) v = src[(L.rowoff[a] + (b - L.off[L.layer[a] + 1])) * stride + t];
                dst[a * N + b] = v;
            }
    };
    for (int t = 0; t < 6 && D.V; t++) dense(D.V + (size_t)t * N * N, T.V, 6, t);
    dense(D.B, T.B, 1, 0);
    dense(D.S1, T.S1, 1, 0);
    dense(D.S2, T.S2, 1, 0);
    if (D.X) memcpy(D.X, T.X, N * 8);
}
}  // namespace sd

namespace {
sd_status design_tables_impl(sd_context* ctx, const char* protein, const std::vector<std::string>* motifs,
                             const sd_codon_table* table, const sd_params* params, double lambda_kcal,
                             sd_result* out, int64_t* V, int64_t* B, int64_t* S1, int64_t* S2, int64_t* X) {
    try {
        TraceTables T;
        Lattice L;
        sd_status s = design_plain(ctx, protein, table, params, lambda_kcal, out, &T, &L, motifs);
        if (s) return s;
        dense_tables(L, T, DenseOut{V, B, S1, S2, X});
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}
}  // namespace

extern "C" sd_status sd_motif_lattice_size(const char* protein, const char* const* motifs, int n_motifs,
                                           int64_t* n_states, int64_t* n_cells) {
    try {
        if (!n_states || !n_cells || !motifs || n_motifs < 1 || n_motifs > kMaxMotifs)
            return fail(SD_E_ARG, "null argument or motif count outside 1..256");
        std::vector<std::string> ms;
        for (int i = 0; i < n_motifs; i++) {
            if (!motifs[i]) return fail(SD_E_ARG, "null motif");
            ms.push_back(motifs[i]);
        }
        CodonTable T;
        for (int i = 0; i < 64; i++) T.w[i] = 1.0;
        Params P;
        memset(&P.E, 0, sizeof(P.E));
        Lattice L;
        std::string err;
        int rc = build_motif_lattice(protein, T, P, 0.0, CapPolicy(), ms, L, err);
        if (rc) return fail((sd_status)rc, err);
        *n_states = L.N;
        *n_cells = L.cells;
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    }
}

extern "C" sd_status sd_multiloop_abstract(sd_context* c, int N, const int32_t* layer, int n_edges,
                                          const int32_t* esrc, const int32_t* edst, const int64_t* eu,
                                          const int64_t* B, int64_t* S1, int64_t* S2, int8_t* cand, int64_t* Z) {
    try {
        if (!c || N < 1 || !layer || n_edges < 0 || (n_edges > 0 && (!esrc || !edst || !eu)) || !B || !S1 || !S2 ||
            !cand || !Z)
            return fail(SD_E_ARG, "null argument or bad size");
        hipError_t e = hipSetDevice(c->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        // layered DAG: layers 0.. in state order, each non-empty and at most kMaxWidth wide,
        // edges from a layer to the next, at most four out of a state
        if (layer[0] != 0) return fail(SD_E_ARG, "the first state must be in layer 0");
        for (int v = 1; v < N; v++)
            if (layer[v] != layer[v - 1] && layer[v] != layer[v - 1] + 1)
                return fail(SD_E_ARG, "layers must be consecutive and in state order");
        Lattice L;
        L.N = N;
        L.n = layer[N - 1];
        L.A = 1;
        L.layer.assign(layer, layer + N);
        L.off.assign(L.n + 2, 0);
        for (int v = N - 1; v >= 0; v--) L.off[layer[v]] = v;
        L.off[L.n + 1] = N;
        for (int l = 0; l <= L.n; l++) {
            L.wmax = std::max(L.wmax, L.off[l + 1] - L.off[l]);
            if (L.off[l + 1] - L.off[l] > kMaxWidth) return fail(SD_E_ARG, "a layer is wider than 4 states");
        }
        L.out_dst.assign(4 * (size_t)N, -1);
        L.out_cod.assign(4 * (size_t)N, -1);
        L.out_q.assign(4 * (size_t)N, 0.0);
        L.out_U.assign(4 * (size_t)N, 0);
        std::vector<int> outdeg(N, 0);
        struct InE { int src, lab, dst; int64_t u; };
        std::vector<InE> ins;
        for (int k = 0; k < n_edges; k++) {
            const int a = esrc[k], b = edst[k];
            if (a < 0 || a >= N || b < 0 || b >= N || layer[b] != layer[a] + 1)
                return fail(SD_E_ARG, "an edge must join consecutive layers");
            if (outdeg[a] == 4) return fail(SD_E_ARG, "more than four edges leave a state");
            if (eu[k] < -((int64_t)1 << 40) || eu[k] > ((int64_t)1 << 40)) return fail(SD_E_RANGE, "edge cost out of range");
            const int lab = outdeg[a]++;
            L.out_dst[4 * (size_t)a + lab] = b;
            L.out_U[4 * (size_t)a + lab] = eu[k];
            ins.push_back({a, lab, b, eu[k]});
        }
        std::stable_sort(ins.begin(), ins.end(), [](const InE& x, const InE& y) {
            return x.dst != y.dst ? x.dst < y.dst : (x.src != y.src ? x.src < y.src : x.lab < y.lab);
        });
        L.in_start.assign(N + 1, 0);
        L.inmask.assign(N, 0);
        for (const InE& x : ins) {
            L.in_start[x.dst + 1]++;
            L.in_src.push_back(x.src);
            L.in_lab.push_back(x.lab);
            L.in_U.push_back(x.u);
            L.in_cod.push_back(-1);
            L.inmask[x.dst] |= 1 << x.lab;
        }
        for (int v = 0; v < N; v++) L.in_start[v + 1] += L.in_start[v];
        L.tail.assign(N, 0);
        L.pfx.assign(N, 0);
        L.P.assign(2, 0);
        L.hp_init.assign(L.n + 1, 0);
        L.alphaU.assign(4 * (size_t)N, kINF);
        L.betaU.assign(4 * (size_t)N, kINF);
        L.fwd_off.assign(4 * (size_t)N + 1, 0);
        L.bwd_off.assign(4 * (size_t)N + 1, 0);
        L.hpB.assign(16 * (size_t)N, kINF);
        L.OB.assign(72 * (size_t)N, kINF);
        L.OA.assign(72 * (size_t)N, kINF);
        // cells in row layout; worst-case candidate segments (a direct arc may have any span)
        L.rowoff.assign(N, 0);
        L.coff.assign(N, 0);
        L.ccap.assign(N, 0);
        int64_t cells = 0, slots = 0;
        for (int a = 0; a < N; a++) {
            L.rowoff[a] = cells;
            cells += N - L.off[layer[a] + 1];
            L.coff[a] = slots;
            L.ccap[a] = L.off[layer[a]];
            slots += L.ccap[a];
        }
        L.cells = cells;
        L.cand_slots = slots;
        std::vector<int64_t> Bc(std::max<int64_t>(cells, 1), kINF);
        for (int a = 0; a < N; a++)
            for (int b = L.off[layer[a] + 1]; b < N; b++) {
                const int64_t v = B[(size_t)a * N + b];
                if (v < kHalfINF && (v < -((int64_t)1 << 40) || v > ((int64_t)1 << 40)))
                    return fail(SD_E_RANGE, "direct cost out of range");
                Bc[L.rowoff[a] + (b - L.off[layer[a] + 1])] = v >= kHalfINF ? kINF : v;
            }
        Inst I;
        memset(&I, 0, sizeof(I));
        sd_status st = place_and_upload(c, L, I);
        if (st) return st;
        I.retain_all = 0;
        e = hipMemcpyAsync(I.V(), Bc.data(), 8 * (size_t)cells, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = launch_init(I, c->stream);
        for (int g = 1; g <= L.n && e == hipSuccess; g++) e = launch_ml_abstract(I, g, c->stream);
        std::vector<int64_t> s1(std::max<int64_t>(cells, 1)), s2(std::max<int64_t>(cells, 1));
        std::vector<int> cnt(N), cc(std::max<int64_t>(slots, 1));
        if (e == hipSuccess && cells) e = hipMemcpyAsync(s1.data(), I.S1(), 8 * (size_t)cells, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && cells) e = hipMemcpyAsync(s2.data(), I.S2(), 8 * (size_t)cells, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(cnt.data(), I.ccnt(), 4 * (size_t)N, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && slots) e = hipMemcpyAsync(cc.data(), I.cc(), 4 * (size_t)slots, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "abstract multiloop run");
        int64_t z = 0;
        memset(cand, 0, (size_t)N * N);
        for (int a = 0; a < N; a++)
            for (int b = 0; b < N; b++) {
                const bool f = layer[a] < layer[b];
                const int64_t k = f ? L.rowoff[a] + (b - L.off[layer[a] + 1]) : 0;
                S1[(size_t)a * N + b] = f ? s1[k] : kINF;
                S2[(size_t)a * N + b] = f ? s2[k] : kINF;
            }
        for (int b = 0; b < N; b++)
            for (int k = 0; k < cnt[b]; k++) {
                const int raw = cc[L.coff[b] + k];
                if (raw >= 0) cand[(size_t)raw * N + b] = 1;
                z++;
            }
        *Z = z;
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    }
}

extern "C" sd_status sd_design_tables(sd_context* ctx, const char* protein, const sd_codon_table* table,
                                      const sd_params* params, double lambda_kcal, sd_result* out,
                                      int64_t* V, int64_t* B, int64_t* S1, int64_t* S2, int64_t* X) {
    return design_tables_impl(ctx, protein, nullptr, table, params, lambda_kcal, out, V, B, S1, S2, X);
}

extern "C" sd_status sd_design_motifs_tables(sd_context* ctx, const char* protein, const char* const* motifs,
                                             int n_motifs, const sd_codon_table* table, const sd_params* params,
                                             double lambda_kcal, sd_result* out, int64_t* V, int64_t* B,
                                             int64_t* S1, int64_t* S2, int64_t* X) {
    try {
        if (!motifs || n_motifs < 1 || n_motifs > kMaxMotifs) return fail(SD_E_ARG, "need 1 to 256 motifs");
        std::vector<std::string> ms;
        for (int i = 0; i < n_motifs; i++) {
            if (!motifs[i]) return fail(SD_E_ARG, "null motif");
            ms.push_back(motifs[i]);
        }
        return design_tables_impl(ctx, protein, &ms, table, params, lambda_kcal, out, V, B, S1, S2, X);
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    }
}

extern "C" void sd_result_free(sd_result* r) {
    if (!r) return;
    free(r->mrna);
    free(r->structure);
    r->mrna = nullptr;
    r->structure = nullptr;
}

namespace sd {

// Runs the batched persistent launch for lattices Ls (already validated) and returns the device
// instance descriptors (in the arena) through Is.  *barrier_ok is false when the grid barrier
// reported a wait beyond its spin limit (the caller then recomputes in plain mode).
sd_status run_batch(sd_context* c, std::vector<Lattice>& Ls, std::vector<Inst>& Is, const sd_context::Sched& sc,
                    bool* barrier_ok, double* kernel_s, Inst** insts_out) {
    const int n = (int)Ls.size();
    Is.assign(n, Inst{});
    std::vector<InstLayout> lay(n);
    size_t totA = 0, totB = 0;
    for (int i = 0; i < n; i++) {
        lay[i] = layout_instance(Ls[i], nullptr, nullptr, Is[i]);
        if (!lay[i].a_bytes) return fail(SD_E_INTERNAL, "instance layout does not hold its arrays");
        totA += lay[i].a_bytes;
        totB += lay[i].b_bytes;
    }
    const size_t inst_bytes = ((sizeof(Inst) * n + 255) / 256) * 256;
    sd_status s = ensure_arena(c, totA + totB + inst_bytes + sizeof(BatchCtl) + 256);
    if (s) return s;
    s = ensure_staging(c, totA);
    if (s) return s;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    char* A = (char*)c->arena;
    char* B = A + totA;
    Inst* insts_dev = (Inst*)(B + totB);
    BatchCtl* ctl = (BatchCtl*)((char*)insts_dev + inst_bytes);
    size_t oa = 0, ob = 0;
    for (int i = 0; i < n; i++) {
        layout_instance(Ls[i], A + oa, B + ob, Is[i]);
        Is[i].retain_all = c->opt.retain_all;
        Is[i].g0 = 1;
        stage_inputs(Ls[i], Is[i], A, (char*)c->staging);
        oa += lay[i].a_bytes;
        ob += lay[i].b_bytes;
    }
    e = hipMemcpyAsync(A, c->staging, totA, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(insts_dev, Is.data(), sizeof(Inst) * n, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
    int maxn = 0;
    for (auto& L : Ls) maxn = std::max(maxn, L.n);
    const unsigned spin_cap = 1u << 22;  // a few seconds of polling before the barrier gives up
    // one captured graph: per-instance initialisation, then the persistent span wavefront
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool captured = false;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        hipError_t e1 = launch_batch_init(insts_dev, n, ctl, c->stream);
        hipError_t e2 = e1 == hipSuccess ? launch_persistent(insts_dev, n, maxn + 1, (const EnergyTables*)c->E_dev,
                                                             (const int32_t*)c->spec_dev, ctl, sc.grid, sc.threads, sc.item_waves,
                                                             spin_cap, c->stream)
                                         : e1;
        hipError_t e3 = hipStreamEndCapture(c->stream, &graph);
        if (e2 == hipSuccess && e3 == hipSuccess && graph &&
            hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess)
            captured = true;
    }
    hipGetLastError();
    e = hipEventRecord(c->ev0, c->stream);
    if (captured) {
        if (e == hipSuccess) e = hipGraphLaunch(exec, c->stream);
    } else {
        if (e == hipSuccess) e = launch_batch_init(insts_dev, n, ctl, c->stream);
        if (e == hipSuccess)
            e = launch_persistent(insts_dev, n, maxn + 1, (const EnergyTables*)c->E_dev, (const int32_t*)c->spec_dev,
                                  ctl, sc.grid, sc.threads, sc.item_waves, spin_cap, c->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(c->ev1, c->stream);
    BatchCtl hctl;
    if (e == hipSuccess) e = hipMemcpyAsync(&hctl, ctl, sizeof(hctl), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev0, c->ev1);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "batched wavefront");
    c->last_graph = captured;
    *kernel_s = ms * 1e-3;
    *barrier_ok = hctl.err.v == 0 && hctl.steps_done.v == (unsigned)(maxn + 1);  // nsteps = maxn + 1
    if (insts_out) *insts_out = insts_dev;
    return SD_OK;
}

// Autotuned schedule of the persistent launch: threads per workgroup, resident workgroups per CU,
// and waves per work item (one layer pair): the four waves of a workgroup share each item, or
// every wave works on its own items.  Every schedule gives bit-identical results, so the tuner
// explores on the caller's own batches: the first calls of a size class run one candidate each,
// scored by launch time per DP cell, and later calls of the class run the fastest.  A size class
// is (floor log2 of the mean length, floor log2 of the member count, capped at 16 members).  A
// probe on a sample of the batch would misjudge the waves dimension: a dozen members leave the
// launch latency-bound, where shared items win, while hundreds keep it throughput-bound, where
// independent waves win.
namespace {
int size_class(const std::vector<Lattice>& batch) {
    double mean_n = 0;
    for (const Lattice& L : batch) mean_n += L.n;
    mean_n /= std::max<size_t>(1, batch.size());
    const int cls_n = (int)std::floor(std::log2(std::max(1.0, mean_n)));
    const int cls_m = std::min(4, (int)std::floor(std::log2((double)std::max<size_t>(1, batch.size()))));
    return cls_n * 8 + cls_m;
}
}  // namespace

// The schedule of the next batched call; *settled is false while the class is still exploring.
sd_status tuned_schedule(sd_context* c, const std::vector<Lattice>& batch, sd_context::Sched* out, int* cls_out,
                         bool* settled) {
    *cls_out = -1;
    if (c->opt.batch_threads > 0) {  // fixed by the caller
        out->threads = c->opt.batch_threads;
        out->grid = c->opt.batch_per_cu * c->num_cu;
        out->item_waves = c->opt.batch_item_waves ? c->opt.batch_item_waves : c->opt.batch_threads / 64;
        *settled = true;
        return SD_OK;
    }
    const int cls = size_class(batch);
    *cls_out = cls;
    sd_context::Tune& T = c->tune[cls];
    if (T.cands.empty()) {
        // candidates in the order they are tried: independent waves first (the best schedule
        // for large batches); one workgroup per CU and 64-thread workgroups only for batches of
        // fewer than 12 members, where the grid barrier's participants weigh more than residency
        int pc_w = 0, pc_s = 0, pc_64 = 0;
        hipError_t e = persistent_occupancy(256, 1, &pc_w);
        if (e == hipSuccess) e = persistent_occupancy(256, 4, &pc_s);
        if (e == hipSuccess) e = persistent_occupancy(64, 1, &pc_64);
        if (e != hipSuccess || pc_w <= 0 || pc_s <= 0 || pc_64 <= 0) {
            c->tune.erase(cls);
            return hip_fail(e, "occupancy query");
        }
        auto add = [&](int threads, int iw, int per_cu) {
            sd_context::Sched sc;
            sc.threads = threads;
            sc.item_waves = iw;
            sc.grid = per_cu * c->num_cu;
            for (const auto& x : T.cands)
                if (x.threads == sc.threads && x.item_waves == sc.item_waves && x.grid == sc.grid) return;
            T.cands.push_back(sc);
        };
        add(256, 1, pc_w);
        add(256, 4, pc_s);
        add(256, 1, std::max(1, pc_w / 2));
        add(256, 4, std::max(1, pc_s / 2));
        if (batch.size() < 12) {
            add(256, 4, 1);
            add(64, 1, pc_64);
        }
        T.score.assign(T.cands.size(), 0.0);
    }
    *settled = T.settled;
    *out = T.settled ? T.best : T.cands[T.next];
    return SD_OK;
}

// Records the measured launch of an exploring call (ok: the grid barrier completed).
void tune_record(sd_context* c, int cls, const std::vector<Lattice>& batch, bool ok, double kernel_s) {
    auto it = c->tune.find(cls);
    if (it == c->tune.end() || it->second.settled) return;
    sd_context::Tune& T = it->second;
    double cells = 0;
    for (const Lattice& L : batch) cells += (double)L.cells;
    T.score[T.next] = ok ? kernel_s / std::max(1.0, cells) : HUGE_VAL;
    if (++T.next < (int)T.cands.size()) return;
    int b = 0;
    for (int k = 1; k < (int)T.cands.size(); k++)
        if (T.score[k] < T.score[b]) b = k;
    T.best = T.cands[b];
    T.settled = true;
}

}  // namespace sd

namespace {
// Digests of every member's tables after the launch just run; then the same batch under another
// persistent schedule; the digests must agree member by member.
sd_status check_batch_rerun(sd_context* ctx, std::vector<Lattice>& Ls, std::vector<Inst>& Is,
                            const sd_context::Sched& sc, Inst** insts_dev) {
    const int m = (int)Ls.size();
    const size_t need = 256 + 16 * (size_t)m;
    hipError_t e = hipSuccess;
    if (need > ctx->dbg_bytes) {
        if (ctx->dbg) hipFree(ctx->dbg);
        ctx->dbg = nullptr;
        ctx->dbg_bytes = 0;
        e = hipMalloc((void**)&ctx->dbg, need);
        if (e != hipSuccess) return hip_fail(e, "span check buffer");
        ctx->dbg_bytes = need;
    }
    unsigned long long* d = (unsigned long long*)ctx->dbg;
    for (int i = 0; i < m && e == hipSuccess; i++) e = launch_checksum(Is[i], 0, d + i, ctx->stream);
    std::vector<unsigned long long> h1(m), h2(m);
    if (e == hipSuccess) e = hipMemcpyAsync(h1.data(), d, 8 * (size_t)m, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "span check digests");
    // another schedule: shared items <-> one wave per item
    sd_context::Sched s2;
    s2.threads = sc.threads == 256 && sc.item_waves == 4 ? 64 : 256;
    s2.item_waves = s2.threads == 64 ? 1 : 4;
    int per_cu = 0;
    e = persistent_occupancy(s2.threads, s2.item_waves, &per_cu);
    if (e != hipSuccess || per_cu <= 0) return hip_fail(e, "occupancy query");
    s2.grid = std::min(per_cu, 2) * ctx->num_cu;
    bool ok2 = false;
    double ks2 = 0;
    std::vector<Inst> Is2;
    sd_status s = run_batch(ctx, Ls, Is2, s2, &ok2, &ks2, insts_dev);
    if (s) return s;
    if (!ok2) return fail(SD_E_INTERNAL, "span check: the re-run's grid barrier gave up");
    for (int i = 0; i < m && e == hipSuccess; i++) e = launch_checksum(Is2[i], 0, d + i, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h2.data(), d, 8 * (size_t)m, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "span check digests");
    for (int i = 0; i < m; i++)
        if (h1[i] != h2[i])
            return fail(SD_E_INTERNAL, "span check: batch member " + std::to_string(i) + " filled different tables "
                                       "under the schedules " + std::to_string(sc.threads) + "/" +
                                       std::to_string(sc.item_waves) + " and " + std::to_string(s2.threads) + "/" +
                                       std::to_string(s2.item_waves) + " (threads per workgroup / waves per item)");
    Is = std::move(Is2);
    return SD_OK;
}

// sd_design_batch; with dump_member in [0, n) that member's tables also go to D (dense layout)
sd_status design_batch_impl(sd_context* ctx, int n, const char* const* proteins, const double* lambdas,
                            const sd_codon_table* table, const sd_params* params, sd_result* outs,
                            int dump_member, const DenseOut& D) {
    try {
        if (!ctx || !table || !params || n < 0 || (n > 0 && (!proteins || !lambdas || !outs)))
            return fail(SD_E_ARG, "null argument");
        // every entry starts empty, so that freeing the outputs on an error path only ever
        // frees strings this call allocated, whatever the caller's array held
        memset(outs, 0, sizeof(sd_result) * (size_t)n);
        hipError_t he = hipSetDevice(ctx->device);
        if (he != hipSuccess) return hip_fail(he, "hipSetDevice");
        int done = 0;
        while (done < n) {
            const int m = std::min(n - done, kMaxBatch);
            const double t0 = now_s();
            // the members' automata and layouts, built on up to 16 host threads (each build reads
            // only its protein, the shared read-only tables and the sizer); the first failing
            // member in order is reported
            std::vector<Lattice> Ls(m);
            std::vector<int> rcs(m, 0);
            std::vector<std::string> errs(m);
            {
                const int nt = std::max(1, std::min({m, 16, (int)std::thread::hardware_concurrency()}));
                auto work = [&](int t) {
                    for (int i = t; i < m; i += nt) {
                        try {
                            std::vector<float> frac;
                            rcs[i] = build_lattice(proteins[done + i], table->t, params->p, lambdas[done + i],
                                                   policy_for(ctx, proteins[done + i], lambdas[done + i], frac), Ls[i],
                                                   errs[i]);
                        } catch (const std::bad_alloc&) {
                            rcs[i] = SD_E_NOMEM;
                            errs[i] = "host allocation";
                        }
                    }
                };
                std::vector<std::thread> pool;
                for (int t = 1; t < nt; t++) pool.emplace_back(work, t);
                work(0);
                for (auto& th : pool) th.join();
            }
            for (int i = 0; i < m; i++)
                if (rcs[i]) {
                    for (int j = 0; j < done; j++) sd_result_free(&outs[j]);
                    return fail((sd_status)rcs[i], "batch member " + std::to_string(done + i) + ": " + errs[i]);
                }
            sd_status s = ensure_params(ctx, params);
            sd_context::Sched sc;
            int cls = -1;
            bool settled = true;
            if (!s) s = tuned_schedule(ctx, Ls, &sc, &cls, &settled);
            const double tf0 = now_s();
            std::vector<Inst> Is;
            bool ok = false;
            double ks = 0;
            Inst* insts_dev = nullptr;
            if (!s) s = run_batch(ctx, Ls, Is, sc, &ok, &ks, &insts_dev);
            const double tf1 = now_s();
            if (!s && !settled) tune_record(ctx, cls, Ls, ok, ks);
            // span_check debug mode: the whole launch again under another schedule, then a digest
            // of every member's tables from each run must agree
            if (!s && ok && ctx->opt.span_check) s = check_batch_rerun(ctx, Ls, Is, sc, &insts_dev);
            // the canonical traceback of every member in one launch (eight wavefronts each)
            if (!s && ok) {
                hipError_t e = launch_trace_many(insts_dev, m, (const EnergyTables*)ctx->E_dev,
                                                 (const int32_t*)ctx->spec_dev, ctx->stream);
                for (int i = 0; i < m && e == hipSuccess; i++)
                    if (Is[i].retain_all) e = launch_strict_count(Is[i], ctx->stream);
                if (e != hipSuccess) s = hip_fail(e, "batched traceback launch");
            }
            if (s) {
                for (int j = 0; j < done; j++) sd_result_free(&outs[j]);
                return s;
            }
            ctx->last_batch_kernel_s = ks;
            ctx->last_batch_fill_s = tf1 - tf0;
            for (int i = 0; i < m && s == SD_OK; i++) {
                const int gi = done + i;
                unsigned long long st[4];
                hipError_t e = read_stats(Is[i], ctx->stream, st);
                if (e != hipSuccess) {
                    s = hip_fail(e, "batch stats");
                    break;
                }
                if (!ok || st[2] != ~0ull) {
                    // barrier failure or candidate overflow: exact recomputation in plain mode
                    // with worst-case segments
                    TraceTables T2;
                    Lattice L2;
                    TraceOut O2;
                    const int fw = ctx->force_worst;
                    ctx->force_worst = 1;
                    s = design_plain(ctx, proteins[gi], table, params, lambdas[gi], &outs[gi],
                                     gi == dump_member ? &T2 : nullptr, &L2, nullptr, &O2);
                    ctx->force_worst = fw;
                    ctx->last_batch_fallbacks++;
                    if (!s && gi == dump_member) dense_tables(L2, T2, D);
                    if (!s) {
                        outs[gi].cand_slots_first = Ls[i].cand_slots;
                        outs[gi].cand_overflow = st[2] != ~0ull;
                        outs[gi].path = ok ? SD_PATH_PLAIN_AFTER_OVERFLOW : SD_PATH_PLAIN_AFTER_BARRIER;
                        if (ctx->occ_K > 0) occupancy_bins(L2, O2.counts, ctx->occ_K, &ctx->occ[(size_t)gi * ctx->occ_K]);
                    }
                    continue;
                }
                TraceOut T;
                s = fetch_trace(ctx, Ls[i], Is[i], T);
                if (s) break;
                if (gi == dump_member) {
                    TraceTables TT;
                    s = fetch_tables(ctx, Ls[i], Is[i], TT, true);
                    if (s) break;
                    dense_tables(Ls[i], TT, D);
                }
                TraceResult R;
                std::string why;
                if (finish_trace(Ls[i], T, R, &why)) {
                    s = fail(SD_E_INTERNAL, "traceback self-check failed for batch member " + std::to_string(gi) +
                                                " (" + std::to_string(Ls[i].n) + " layers): " + why);
                    break;
                }
                int64_t Z = 0;
                for (int v = 0; v < Ls[i].N; v++) Z += T.counts[v];
                s = fill_result(Ls[i], R, T.xs, Z, (int64_t)st[0], (int64_t)st[3], &outs[gi]);
                if (s) break;
                outs[gi].t_fill_s = (tf1 - tf0) / m;
                outs[gi].t_total_s = now_s() - t0;
                outs[gi].t_span_kernels_s = ks / m;
                outs[gi].n_span_launches = 0;
                outs[gi].cand_slots = Ls[i].cand_slots;
                outs[gi].cand_slots_first = Ls[i].cand_slots;
                outs[gi].cand_overflow = 0;
                outs[gi].path = SD_PATH_PERSISTENT;
                outs[gi].graph_captured = ctx->last_graph ? 1 : 0;
                outs[gi].sched_threads = sc.threads;
                outs[gi].sched_grid = sc.grid;
                outs[gi].sched_item_waves = sc.item_waves;
                outs[gi].sched_tuned = settled ? 1 : 0;
                if (ctx->occ_K > 0) occupancy_bins(Ls[i], T.counts, ctx->occ_K, &ctx->occ[(size_t)gi * ctx->occ_K]);
            }
            if (s) {
                for (int j = 0; j < done + m; j++) sd_result_free(&outs[j]);
                return s;
            }
            done += m;
        }
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}

}  // namespace

extern "C" sd_status sd_design_batch(sd_context* ctx, int n, const char* const* proteins,
                                     const double* lambdas, const sd_codon_table* table,
                                     const sd_params* params, sd_result* outs) {
    return design_batch_impl(ctx, n, proteins, lambdas, table, params, outs, -1, DenseOut{});
}

extern "C" sd_status sd_design_batch_tables(sd_context* ctx, int n, const char* const* proteins,
                                            const double* lambdas, const sd_codon_table* table,
                                            const sd_params* params, sd_result* outs, int member,
                                            int64_t* V, int64_t* B, int64_t* S1, int64_t* S2, int64_t* X) {
    if (member < 0 || member >= n) return fail(SD_E_ARG, "member index outside the batch");
    return design_batch_impl(ctx, n, proteins, lambdas, table, params, outs, member, DenseOut{V, B, S1, S2, X});
}

extern "C" sd_status sd_context_set_sizer(sd_context* ctx, const sd_sizer* z, float margin, int slack) {
    if (!ctx || margin < 0.f || slack < 0) return fail(SD_E_ARG, "bad sizing policy");
    ctx->sizer = z;
    ctx->sz_margin = margin;
    ctx->sz_slack = slack;
    return SD_OK;
}

extern "C" sd_status sd_occupancy(sd_context* ctx, int n, const char* const* proteins, const double* lambdas,
                                  const sd_codon_table* table, const sd_params* params, int K, float* Y,
                                  sd_result* outs) {
    if (!ctx || !Y || K <= 0 || K > 64 || n < 0) return fail(SD_E_ARG, "bad occupancy arguments");
    std::vector<sd_result> tmp;
    sd_result* res = outs;
    if (!res) {
        tmp.resize(n);
        res = tmp.data();
    }
    ctx->occ.assign((size_t)n * K, 0.f);
    ctx->occ_K = K;
    const int fw = ctx->force_worst;
    ctx->force_worst = 1;
    sd_status s = sd_design_batch(ctx, n, proteins, lambdas, table, params, res);
    ctx->force_worst = fw;
    ctx->occ_K = 0;
    if (s) return s;
    memcpy(Y, ctx->occ.data(), sizeof(float) * (size_t)n * K);
    if (!outs)
        for (auto& r : tmp) sd_result_free(&r);
    return SD_OK;
}

// Tuning file (text): a header line, the device line (architecture, CU count), then one line per
// settled persistent schedule ("batch class grid threads item_waves") and per tuned span band
// ("span class band threads item_waves").
extern "C" sd_status sd_tuning_save(const sd_context* c, const char* path) {
    using namespace sd;
    if (!c || !path) return fail(SD_E_ARG, "null argument");
    try {
        std::ostringstream os;
        os << "sparsedesign-tuning 1\n" << "device gfx950 " << c->num_cu << "\n";
        for (const auto& kv : c->tune)
            if (kv.second.settled)
                os << "batch " << kv.first << " " << kv.second.best.grid << " " << kv.second.best.threads << " "
                   << kv.second.best.item_waves << "\n";
        for (const auto& kv : c->span_tune)
            if (kv.second.settled)
                for (int b = 0; b < sd_context::kSpanBands; b++)
                    if (kv.second.tuned[b])
                        os << "span " << kv.first << " " << b << " " << kv.second.best[b].threads << " "
                           << kv.second.best[b].item_waves << "\n";
        std::ofstream f(path, std::ios::trunc);
        f << os.str();
        f.close();
        if (!f) return fail(SD_E_ARG, std::string("cannot write ") + path);
        return SD_OK;
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}

extern "C" sd_status sd_tuning_load(sd_context* c, const char* path) {
    using namespace sd;
    if (!c || !path) return fail(SD_E_ARG, "null argument");
    try {
        hipError_t e = hipSetDevice(c->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        std::ifstream f(path);
        if (!f) return fail(SD_E_ARG, std::string("cannot read ") + path);
        std::string line;
        if (!std::getline(f, line) || line != "sparsedesign-tuning 1") return fail(SD_E_ARG, "not a tuning file");
        std::string w1, arch;
        int cus = 0;
        if (!std::getline(f, line)) return fail(SD_E_ARG, "tuning file without a device line");
        {
            std::istringstream is(line);
            if (!(is >> w1 >> arch >> cus) || w1 != "device") return fail(SD_E_ARG, "malformed device line");
            if (arch != "gfx950" || cus != c->num_cu)
                return fail(SD_E_ARG, "tuning file written for " + arch + " with " + std::to_string(cus) +
                                          " CUs; this device is gfx950 with " + std::to_string(c->num_cu));
        }
        // parse and validate everything before installing anything
        std::map<int, sd_context::Sched> batch;
        std::map<int, std::map<int, sd_context::SpanTile>> span;
        for (int ln = 3; std::getline(f, line); ln++) {
            if (line.empty()) continue;
            std::istringstream is(line);
            std::string kind;
            int cls = 0, x = 0, threads = 0, iw = 0;
            const std::string where = " at line " + std::to_string(ln);
            if (!(is >> kind >> cls >> x >> threads >> iw)) return fail(SD_E_ARG, "malformed tuning line" + where);
            if (kind == "batch") {
                int per_cu = 0;
                if (!persistent_schedule_valid(threads, iw) || persistent_occupancy(threads, iw, &per_cu) != hipSuccess ||
                    x <= 0 || x % c->num_cu != 0 || x / c->num_cu > per_cu)
                    return fail(SD_E_ARG, "persistent schedule this device cannot run" + where);
                sd_context::Sched sc;
                sc.grid = x;
                sc.threads = threads;
                sc.item_waves = iw;
                batch[cls] = sc;
            } else if (kind == "span") {
                bool ok = false;
                for (int k = 0; k < sd_context::kSpanCands; k++)
                    ok |= kSpanCandThreads[k] == threads && kSpanCandWaves[k] == iw;
                ok &= x >= 0 && x < sd_context::kSpanBands;
                if (!ok) return fail(SD_E_ARG, "span tile this library does not have" + where);
                sd_context::SpanTile t;
                t.threads = threads;
                t.item_waves = iw;
                span[cls][x] = t;
            } else {
                return fail(SD_E_ARG, "unknown tuning entry" + where);
            }
        }
        for (const auto& kv : batch) {
            sd_context::Tune& T = c->tune[kv.first];
            T = sd_context::Tune();
            T.settled = true;
            T.best = kv.second;
        }
        for (const auto& kv : span) {
            sd_context::SpanTune& T = c->span_tune[kv.first];
            T = sd_context::SpanTune();
            T.settled = true;
            for (const auto& bt : kv.second) {
                T.tuned[bt.first] = true;
                T.best[bt.first] = bt.second;
            }
        }
        return SD_OK;
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}
