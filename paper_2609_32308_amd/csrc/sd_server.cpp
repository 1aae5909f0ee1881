// Design server: continuous batching of design requests at span-step boundaries.
//
// A server thread repeats rounds.  Each round it
//   1. admits queued requests (FIFO) while a slot is free and the request's device state fits
//      the remaining pool: the O(N^2) tables are known exactly from the automaton, the candidate
//      segments come from the context's sizing policy (learned sizer or worst case);
//   2. runs one persistent launch of `steps_per_round` span steps over every active instance,
//      each at its own span (new instances start at span 1 and are initialised by the launch);
//   3. retires instances that passed their last span: the canonical traceback of all of them
//      runs on the device in one launch (one workgroup of eight wavefronts each), only its O(n)
//      outputs are copied back, and their pool memory is released at once.
// An instance whose candidate reservation overflowed is recomputed exactly in plain mode with
// worst-case segments, so every result equals the standalone design.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include <atomic>

#include "sd_host.h"

using namespace sd;

namespace {

// auxiliary device buffer: the round's instance descriptors, the barrier state, then the
// descriptors of the instances retiring in the round (traceback launch)
constexpr size_t kAuxTrace = ((sizeof(Inst) * kMaxBatch + sizeof(BatchCtl) + 255) / 256) * 256;

// first-fit allocator over one device buffer (offsets, 256-byte granularity)
struct Pool {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    size_t used = 0, high = 0;
    void init(size_t n) {
        size = n;
        free_.clear();
        free_[0] = n;
        used = high = 0;
    }
    bool alloc(size_t n, size_t* off) {
        n = (n + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used += n;
                high = std::max(high, used);
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) & ~(size_t)255;
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    uint64_t ticket;
    std::string protein;
    double lambda;
    double t_submit, t_admit = 0;
    bool worst = false;  // re-admitted after a candidate overflow: worst-case segments
    int64_t first_slots = 0;
};

struct Active {
    Request rq;
    Lattice L;
    Inst I;
    size_t off = 0, bytes = 0;
    int g = 1;  // next span to process
};

struct Done {
    sd_status status;
    sd_result res;
};

}  // namespace

struct sd_server {
    sd_context* ctx;
    const sd_codon_table* table;
    const sd_params* params;
    sd_server_cfg cfg;
    Pool pool;
    char* pool_dev = nullptr;
    char* aux_dev = nullptr;  // instance descriptors + barrier state
    void* staging = nullptr;
    size_t staging_bytes = 0;
    int grid = 0, threads = 256, item_waves = 4;  // the schedule of the current round
    bool fixed = false;                           // fixed by the caller's options
    int grid_shared = 0, grid_waves = 0;          // full-residency grids of the two schedules

    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Request> queue;
    std::map<uint64_t, Done> done;
    std::vector<Active> active;
    uint64_t next_ticket = 1;
    std::atomic<bool> stop{false};
    std::thread loop;
    sd_server_stats st{};
};

namespace {

// Answer a request; `completed` counts it as a finished design (a cancellation is not one).
void finish(sd_server* S, uint64_t ticket, sd_status status, const sd_result& r, bool completed = true) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->done[ticket] = Done{status, r};
    if (completed) S->st.completed++;
    S->cv_done.notify_all();
}

sd_status ensure_srv_staging(sd_server* S, size_t bytes) {
    if (bytes <= S->staging_bytes) return SD_OK;
    if (S->staging) hipHostFree(S->staging);
    S->staging = nullptr;
    S->staging_bytes = 0;
    if (hipHostMalloc(&S->staging, bytes * 2, hipHostMallocDefault) != hipSuccess) return SD_E_NOMEM;
    S->staging_bytes = bytes * 2;
    return SD_OK;
}

// Admit queued requests that fit; returns after uploading their inputs.  A request is taken off
// the queue under the lock that reads it, so sd_server_stop (which answers every queued request
// SD_E_CANCELLED and clears the queue from the caller's thread) never sees a request that this
// thread is placing.  A request that has to wait for pool memory goes back to the head of the
// queue, or is answered SD_E_CANCELLED if the server was stopped meanwhile.
sd_status admit(sd_server* S) {
    for (;;) {
        Request rq;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->queue.empty() || (int)S->active.size() >= S->cfg.max_active) return SD_OK;
            rq = S->queue.front();
            S->queue.pop_front();
        }
        Active a;
        a.rq = rq;
        std::string err;
        std::vector<float> frac;
        int rc = build_lattice(rq.protein.c_str(), S->table->t, S->params->p, rq.lambda,
                               rq.worst ? CapPolicy() : policy_for(S->ctx, rq.protein.c_str(), rq.lambda, frac),
                               a.L, err);
        if (rc) {  // invalid request: answer it right away
            sd_result r;
            memset(&r, 0, sizeof(r));
            finish(S, rq.ticket, (sd_status)rc, r);
            continue;
        }
        memset(&a.I, 0, sizeof(a.I));
        InstLayout lay = layout_instance(a.L, nullptr, nullptr, a.I);
        a.bytes = lay.a_bytes + lay.b_bytes;
        if (!lay.a_bytes) {
            sd_result r;
            memset(&r, 0, sizeof(r));
            finish(S, rq.ticket, SD_E_INTERNAL, r);
            continue;
        }
        if (a.bytes > S->pool.size) {  // can never fit: recompute in plain mode outside the pool
            sd_result r;
            memset(&r, 0, sizeof(r));
            sd_status s = design_plain(S->ctx, rq.protein.c_str(), S->table, S->params, rq.lambda, &r, nullptr, nullptr);
            if (!s) r.t_total_s = now_s() - rq.t_submit;
            finish(S, rq.ticket, s, r);
            continue;
        }
        size_t off;
        if (!S->pool.alloc(a.bytes, &off)) {  // wait for memory to free up
            bool cancelled = false;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (S->stop) cancelled = true;
                else S->queue.push_front(rq);
            }
            if (cancelled) {
                sd_result r;
                memset(&r, 0, sizeof(r));
                finish(S, rq.ticket, SD_E_CANCELLED, r, false);
            }
            return SD_OK;
        }
        a.off = off;
        char* A = S->pool_dev + off;
        layout_instance(a.L, A, A + lay.a_bytes, a.I);
        a.I.retain_all = S->ctx->opt.retain_all;
        a.I.g0 = 1;
        sd_status s = ensure_srv_staging(S, lay.a_bytes);
        if (s) {
            S->pool.release(off, a.bytes);
            std::lock_guard<std::mutex> lk(S->mu);
            S->queue.push_front(rq);  // failed with the device failure handling of the caller
            return s;
        }
        hipError_t e = hipStreamSynchronize(S->ctx->stream);
        if (e == hipSuccess) {
            stage_inputs(a.L, a.I, A, (char*)S->staging);
            e = hipMemcpyAsync(A, S->staging, lay.a_bytes, hipMemcpyHostToDevice, S->ctx->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(S->ctx->stream);
        if (e != hipSuccess) {
            S->pool.release(off, a.bytes);
            std::lock_guard<std::mutex> lk(S->mu);
            S->queue.push_front(rq);
            return hip_fail(e, "server upload");
        }
        a.rq.t_admit = now_s();
        S->st.admitted++;
        S->st.reserved_bytes += a.bytes;
        S->st.reserved_cand_bytes += a.L.cand_slots * 12;
        S->active.push_back(std::move(a));
        S->st.peak_active = std::max<int64_t>(S->st.peak_active, (int64_t)S->active.size());
        S->st.pool_high_water = std::max<int64_t>(S->st.pool_high_water, (int64_t)S->pool.high);
    }
}

sd_status round_once(sd_server* S) {
    const int n = (int)S->active.size();
    std::vector<Inst> Is(n);
    for (int i = 0; i < n; i++) {
        Is[i] = S->active[i].I;
        Is[i].g0 = S->active[i].g;
    }
    Inst* insts = (Inst*)S->aux_dev;
    BatchCtl* ctl = (BatchCtl*)(S->aux_dev + sizeof(Inst) * kMaxBatch);
    hipStream_t st = S->ctx->stream;
    const double t0 = now_s();
    if (!S->fixed) {
        // Every wave on its own items when the round starts with at least 12 layer pairs per
        // resident wave; else four waves share each item.  A mix of about 30 requests (an 8 GiB
        // pool) holds too few pairs per step for independent waves (715 against 687 designs/min);
        // 256 requests (a 64 GiB pool) hold enough (1.24x).
        int64_t items = 0;
        for (int i = 0; i < n; i++) items += std::max(0, S->active[i].L.n - S->active[i].g + 1);
        const bool waves = items >= 12 * (int64_t)S->grid_waves * 4;
        S->threads = 256;
        S->item_waves = waves ? 1 : 4;
        S->grid = waves ? S->grid_waves : S->grid_shared;
    }
    hipError_t e = hipMemcpyAsync(insts, Is.data(), sizeof(Inst) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_batch_init(insts, n, ctl, st);
    if (e == hipSuccess)
        e = launch_persistent(insts, n, S->cfg.steps_per_round, (const EnergyTables*)S->ctx->E_dev,
                              (const int32_t*)S->ctx->spec_dev, ctl, S->grid, S->threads, S->item_waves, 1u << 22,
                              st);
    BatchCtl h;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "server round");
    const double dt = now_s() - t0;
    S->st.rounds++;
    S->st.gpu_seconds += dt;
    const bool ok = h.err.v == 0 && h.steps_done.v == (unsigned)S->cfg.steps_per_round;
    // advance and retire
    std::vector<Active> keep;
    std::vector<int> retiring;
    std::vector<int64_t> visits, feasible;
    for (int i = 0; i < n; i++) {
        Active& a = S->active[i];
        a.g += S->cfg.steps_per_round;
        if (ok && a.g <= a.L.n + 1) {
            keep.push_back(std::move(a));
            continue;
        }
        unsigned long long stats[4];
        e = read_stats(a.I, st, stats);
        if (e != hipSuccess) return hip_fail(e, "server stats");
        if (ok && stats[2] != ~0ull) {
            // candidate overflow of a predicted reservation: the request goes back to the head
            // of the queue and is redone with worst-case segments (exact; the mix keeps running)
            S->pool.release(a.off, a.bytes);
            Request rq = a.rq;
            rq.worst = true;
            rq.first_slots = a.L.cand_slots;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->queue.push_front(rq);
            }
            S->st.fallbacks++;
            continue;
        }
        if (!ok) {
            // barrier failure: exact recomputation in plain mode
            S->pool.release(a.off, a.bytes);
            sd_result r;
            const int fw = S->ctx->force_worst;
            S->ctx->force_worst = 1;
            sd_status s = design_plain(S->ctx, a.rq.protein.c_str(), S->table, S->params, a.rq.lambda, &r, nullptr, nullptr);
            S->ctx->force_worst = fw;
            if (!s) {
                r.t_total_s = now_s() - a.rq.t_submit;
                r.cand_overflow = stats[2] != ~0ull;
                r.cand_slots_first = a.L.cand_slots;
                r.path = SD_PATH_PLAIN_AFTER_BARRIER;
            }
            S->st.fallbacks++;
            finish(S, a.rq.ticket, s, r);
            continue;
        }
        retiring.push_back(i);
        visits.push_back((int64_t)stats[0]);
        feasible.push_back((int64_t)stats[3]);
    }
    // canonical traceback of every retiring instance on the device, then O(n) results per request
    if (!retiring.empty()) {
        const int nt = (int)retiring.size();
        std::vector<Inst> Ts(nt);
        for (int k = 0; k < nt; k++) Ts[k] = S->active[retiring[k]].I;
        Inst* tdev = (Inst*)(S->aux_dev + kAuxTrace);
        e = hipMemcpyAsync(tdev, Ts.data(), sizeof(Inst) * nt, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = launch_trace_many(tdev, nt, (const EnergyTables*)S->ctx->E_dev, (const int32_t*)S->ctx->spec_dev, st);
        for (int k = 0; k < nt && e == hipSuccess; k++)
            if (Ts[k].retain_all) e = launch_strict_count(Ts[k], st);
        if (e != hipSuccess) return hip_fail(e, "server traceback");
        for (int k = 0; k < nt; k++) {
            Active& a = S->active[retiring[k]];
            TraceOut T;
            sd_status s = fetch_trace(S->ctx, a.L, a.I, T);
            S->pool.release(a.off, a.bytes);
            if (s) return s;
            sd_result r;
            memset(&r, 0, sizeof(r));
            TraceResult R;
            std::string why;
            s = finish_trace(a.L, T, R, &why) ? fail(SD_E_INTERNAL, "traceback self-check failed: " + why) : SD_OK;
            if (!s) {
                int64_t Z = 0;
                for (int v = 0; v < a.L.N; v++) Z += T.counts[v];
                s = fill_result(a.L, R, T.xs, Z, visits[k], feasible[k], &r);
            }
            if (!s) {
                r.path = SD_PATH_PERSISTENT;
                r.graph_captured = 0;
                r.sched_threads = S->threads;
                r.sched_grid = S->grid;
                r.sched_item_waves = S->item_waves;
                r.sched_tuned = 1;
                r.t_fill_s = a.rq.t_admit > 0 ? now_s() - a.rq.t_admit : 0.0;
                r.t_total_s = now_s() - a.rq.t_submit;
                r.cand_slots = a.L.cand_slots;
                r.cand_slots_first = a.rq.worst ? a.rq.first_slots : a.L.cand_slots;
                r.cand_overflow = a.rq.worst ? 1 : 0;
            }
            finish(S, a.rq.ticket, s, r);
        }
    }
    S->active = std::move(keep);
    return SD_OK;
}

void server_main(sd_server* S) {
    hipSetDevice(S->ctx->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait_for(lk, std::chrono::milliseconds(5),
                           [&] { return S->stop || !S->queue.empty() || !S->active.empty(); });
            if (S->stop && S->active.empty()) break;
        }
        sd_status s = admit(S);
        if (!s && !S->active.empty()) s = round_once(S);
        if (s) {  // device failure: fail everything that is in flight or queued
            std::lock_guard<std::mutex> lk(S->mu);
            for (auto& a : S->active) S->done[a.rq.ticket] = Done{s, sd_result{}};
            for (auto& q : S->queue) S->done[q.ticket] = Done{s, sd_result{}};
            S->active.clear();
            S->queue.clear();
            S->cv_done.notify_all();
        }
    }
}

}  // namespace

extern "C" sd_status sd_server_start(sd_context* ctx, const sd_codon_table* table, const sd_params* params,
                                     const sd_server_cfg* cfg, sd_server** out) {
    if (!ctx || !table || !params || !cfg || !out) return fail(SD_E_ARG, "null argument");
    if (cfg->pool_bytes < (1u << 20) || cfg->max_active <= 0 || cfg->max_active > kMaxBatch ||
        cfg->steps_per_round <= 0)
        return fail(SD_E_ARG, "bad server configuration");
    *out = nullptr;
    sd_status s = ensure_params(ctx, params);
    if (s) return s;
    sd_server* S = new (std::nothrow) sd_server();
    if (!S) return fail(SD_E_NOMEM, "host allocation");
    S->ctx = ctx;
    S->table = table;
    S->params = params;
    S->cfg = *cfg;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMalloc((void**)&S->pool_dev, cfg->pool_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&S->aux_dev, kAuxTrace + sizeof(Inst) * kMaxBatch);
    if (e != hipSuccess) {
        if (S->pool_dev) hipFree(S->pool_dev);
        delete S;
        hipGetLastError();
        return fail(SD_E_NOMEM, "server pool allocation");
    }
    S->pool.init(cfg->pool_bytes);
    // the schedule: fixed by the caller (validated at context creation), else chosen per round
    // from the mix (round_once) between the full-residency grids of the two 256-thread schedules
    if (ctx->opt.batch_threads > 0) {
        S->fixed = true;
        S->threads = ctx->opt.batch_threads;
        S->grid = ctx->opt.batch_per_cu * ctx->num_cu;
        S->item_waves = ctx->opt.batch_item_waves ? ctx->opt.batch_item_waves : ctx->opt.batch_threads / 64;
    } else {
        int pc_s = 0, pc_w = 0;
        e = persistent_occupancy(256, 4, &pc_s);
        if (e == hipSuccess) e = persistent_occupancy(256, 1, &pc_w);
        if (e != hipSuccess || pc_s <= 0 || pc_w <= 0) {
            hipFree(S->pool_dev);
            hipFree(S->aux_dev);
            delete S;
            return hip_fail(e, "occupancy query");
        }
        S->grid_shared = pc_s * ctx->num_cu;
        S->grid_waves = pc_w * ctx->num_cu;
        S->grid = S->grid_shared;
    }
    S->loop = std::thread(server_main, S);
    *out = S;
    return SD_OK;
}

extern "C" sd_status sd_server_submit(sd_server* S, const char* protein, double lambda, uint64_t* ticket) {
    if (!S || !protein || !ticket) return fail(SD_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(SD_E_CANCELLED, "server stopped");
    Request r{S->next_ticket++, protein, lambda, now_s()};
    S->queue.push_back(r);
    S->st.submitted++;
    *ticket = r.ticket;
    S->cv.notify_one();
    return SD_OK;
}

extern "C" sd_status sd_server_poll(sd_server* S, uint64_t ticket, sd_result* out) {
    if (!S || !out) return fail(SD_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) return SD_E_BUSY;
    sd_status s = it->second.status;
    *out = it->second.res;
    S->done.erase(it);
    return s;
}

extern "C" sd_status sd_server_wait(sd_server* S, uint64_t ticket, sd_result* out) {
    if (!S || !out) return fail(SD_E_ARG, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->done.count(ticket) > 0; });
    auto it = S->done.find(ticket);
    sd_status s = it->second.status;
    *out = it->second.res;
    S->done.erase(it);
    return s;
}

extern "C" sd_status sd_server_get_stats(sd_server* S, sd_server_stats* out) {
    if (!S || !out) return fail(SD_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->pool_in_use = (int64_t)S->pool.used;
    out->active = (int64_t)S->active.size();
    out->queued = (int64_t)S->queue.size();
    return SD_OK;
}

extern "C" sd_status sd_server_stop(sd_server* S) {
    if (!S) return fail(SD_E_ARG, "null argument");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (auto& q : S->queue) S->done[q.ticket] = Done{SD_E_CANCELLED, sd_result{}};
        S->queue.clear();
        S->cv.notify_all();
        S->cv_done.notify_all();
    }
    if (S->loop.joinable()) S->loop.join();
    for (auto& kv : S->done) sd_result_free(&kv.second.res);
    hipFree(S->pool_dev);
    hipFree(S->aux_dev);
    if (S->staging) hipHostFree(S->staging);
    delete S;
    return SD_OK;
}
