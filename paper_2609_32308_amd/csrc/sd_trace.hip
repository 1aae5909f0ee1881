// Canonical first-match traceback on the device (Sec. 5: the traceback is deferred until the
// fill is complete and reconstructs every decision from the stored costs; Sec. 7: optima are
// often tied, so one fixed order of alternatives makes the emitted design reproducible).
//
// A workgroup of eight wavefronts per design replays the decisions from X(s).  A decision either
// continues in the same wave or also defers an independent sub-interval (the rest of the external
// loop beside a closed pair, the left part of a multiloop split), which a free wave takes from a
// shared stack.  At each decision the alternatives are enumerated in a fixed order and the first
// whose value equals the stored value exactly is taken, so the design does not depend on which
// wave replays which interval:
//   X(a):   unpaired out-edges by label; then branches (b by state index, pair type in the order
//           AU, CG, GC, GU, UA, UG)
//   V_t:    hairpin (sizes 3, 4, 6: paths in lexicographic base order; other sizes: x_{i+1} by
//           base, the closing in-edge of b, the in-edge of b1), then two-loops (l1 ascending,
//           l2 ascending, closing in-edge of b, inner c by index, d by index, inner type, left
//           segment, right segment), then the multiloop (closing in-edge of b)
//   S1:     direct branch, S2, left unpaired edge (by label), right unpaired edge (in-edge order)
//   S2:     right unpaired edge (in-edge order), then candidates c of C_b by state index (eq. 7)
//   branch: pair type order
//   gaps:   the minimum-cost path that takes the smallest base staying on a minimum path
// The lanes of a wave evaluate alternatives side by side and the first match is the lowest set
// lane of a ballot (or the wave minimum of the matching indices), which is what a sequential
// replay in this order picks.  Two-loop alternatives are grouped by (l1, l2, closing edge, c, d); a group
// is enumerated only if an exact lower bound (segment costs at their minima, the gap costs;
// the loop energy at the minimum of its table over boundary bases and inner types) does not
// already exceed the stored value.  The decisions only read the completed tables, so the design
// does not depend on how the fill was scheduled.
//
// Only O(n) results leave the device: the base at every position, the partner of every paired
// position, the energy, the path cost, a status and X(s).
#include <hip/hip_runtime.h>

#include <limits.h>

#include "sd_devutil.h"
#include "sd_internal.h"
#include "sd_trace_status.h"

namespace sd {
namespace {

enum : int { kFX = 0, kFV = 1, kFS1 = 2, kFS2 = 3, kFBR = 4 };

__device__ __forceinline__ int64_t sadd(int64_t a, int64_t b) { return (a >= kINF || b >= kINF) ? kINF : a + b; }
__device__ __forceinline__ int first_lane(unsigned long long m) { return __ffsll((unsigned long long)m) - 1; }
__device__ __forceinline__ int bcast(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int wmin_int(int v) { return (int)wave_min((int64_t)v); }

// minimum path cost u -> v (INF if unreachable): the trie's closed form, or the device gap table
// of a generic lattice
__device__ __forceinline__ int64_t tgap(const Inst& I, int u, int v) {
    const int lu = I.layer()[u], lv = I.layer()[v];
    if (lu == lv) return u == v ? 0 : kINF;
    if (lu > lv) return kINF;
    if (I.gwin) return I.Gt()[I.rowoff()[u] + (v - I.off()[lu + 1])];
    const int ku = lu / 3, kv = lv / 3;
    if (ku == kv) {
        if (lu % 3 == 0) return 0;
        return (I.pfx()[v] >> 2) == I.pfx()[u] ? 0 : kINF;
    }
    return I.tail()[u] + I.P()[kv] - I.P()[ku + 1];
}
__device__ __forceinline__ int64_t tcell(const Inst& I, int a, int b) {
    return I.rowoff()[a] + (b - I.off()[I.layer()[a] + 1]);
}
__device__ __forceinline__ bool fwd(const Inst& I, int a, int b) { return I.layer()[a] < I.layer()[b]; }
__device__ __forceinline__ int64_t tV(const Inst& I, int t, int a, int b) { return fwd(I, a, b) ? I.V()[tcell(I, a, b) * 6 + t] : kINF; }
__device__ __forceinline__ int64_t tB(const Inst& I, int a, int b) { return fwd(I, a, b) ? I.Bt()[tcell(I, a, b)] : kINF; }
__device__ __forceinline__ int64_t tS1(const Inst& I, int a, int b) { return fwd(I, a, b) ? I.S1()[tcell(I, a, b)] : kINF; }
__device__ __forceinline__ int64_t tS2(const Inst& I, int a, int b) { return fwd(I, a, b) ? I.S2()[tcell(I, a, b)] : kINF; }

// loop energy of a two-loop (stack, bulge, interior) closed by t around the reversed inner type tr
__device__ __forceinline__ int32_t two_loop_e(const SmallE& S, int t, int tr, int l1, int l2, int xi, int xk, int xl,
                                              int xj) {
    if (l1 == 0 && l2 == 0) return S.stack[t][tr];
    if (l1 == 0 || l2 == 0) return bulge_e(S, t, tr, l1 + l2);
    return interior_e(S, nullptr, t, tr, l1, l2, xi, xk, xl, xj);
}

// lower bounds of two-loop energies per closing type over boundary bases and inner types
struct LoopMin {
    int32_t stack[6], int11[6], int12[6], int21[6], int22[6];
    int32_t mm_out[3][6];  // min over (x_{i+1}, x_{j-1}) of mm_X[t]
    int32_t mm_in[3];      // min over inner types and boundary bases of mm_X
    int32_t au_min;
};

__device__ void loop_minima(const SmallE& S, LoopMin& M, int lane) {
    for (int t = 0; t < 6; t++) {
        int64_t st = lane < 6 ? S.stack[t][lane] : kINF, i11 = kINF, i12 = kINF, i21 = kINF, i22 = kINF;
        for (int k = lane; k < 96; k += 64) i11 = mn(i11, (&S.int11[t][0][0][0])[k]);
        for (int k = lane; k < 384; k += 64) {
            i12 = mn(i12, (&S.int21[t][0][0][0][0])[k]);
            i21 = mn(i21, (&S.int21[k >> 6][t][0][0][0])[k & 63]);
        }
        for (int k = lane; k < 1536; k += 64) i22 = mn(i22, (&S.int22[t][0][0][0][0][0])[k]);
        st = wave_min(st);
        i11 = wave_min(i11);
        i12 = wave_min(i12);
        i21 = wave_min(i21);
        i22 = wave_min(i22);
        int64_t mo[3];
        for (int X = 0; X < 3; X++) mo[X] = wave_min(lane < 16 ? (int64_t)mmx(S, X, t, lane >> 2, lane & 3) : kINF);
        if (lane == 0) {
            M.stack[t] = (int32_t)st;
            M.int11[t] = (int32_t)i11;
            M.int12[t] = (int32_t)i12;
            M.int21[t] = (int32_t)i21;
            M.int22[t] = (int32_t)i22;
            for (int X = 0; X < 3; X++) M.mm_out[X][t] = (int32_t)mo[X];
        }
    }
    for (int X = 0; X < 3; X++) {
        int64_t v = kINF;
        for (int k = lane; k < 96; k += 64) v = mn(v, mmx(S, X, k >> 4, (k >> 2) & 3, k & 3));
        v = wave_min(v);
        if (lane == 0) M.mm_in[X] = (int32_t)v;
    }
    if (lane == 0) M.au_min = S.terminal_au < 0 ? S.terminal_au : 0;
}

// lower bound of two_loop_e(t, *, l1, l2, *) over inner types and boundary bases
__device__ __forceinline__ int32_t two_loop_lb(const SmallE& S, const LoopMin& M, int t, int l1, int l2) {
    if (l1 == 0 && l2 == 0) return M.stack[t];
    if (l1 == 0 || l2 == 0) {
        const int l = l1 + l2;
        return l == 1 ? S.bulge[1] + M.stack[t] : S.bulge[l] + au_pen(S, t) + M.au_min;
    }
    if (l1 == 1 && l2 == 1) return M.int11[t];
    if (l1 == 1 && l2 == 2) return M.int12[t];
    if (l1 == 2 && l2 == 1) return M.int21[t];
    if (l1 == 2 && l2 == 2) return M.int22[t];
    const int X = mm_class(l1, l2);
    return interior_base(S, l1, l2) + M.mm_out[X][t] + M.mm_in[X];
}

struct Seg {
    int e1, e2, gfrom, gto, xa, xb;  // out-edge id of the first base, in-edge index of the last
    int64_t cost;
};

// The idx-th segment of l bases from u to v in canonical order (first base, then the in-edge of
// v in CSR order); false if there are fewer.  With idx < 0 the count is returned in *count.
__device__ bool seg_at(const Inst& I, int u, int v, int l, int idx, Seg& s, int* count = nullptr) {
    int k = 0;
    if (l == 0) {
        if (u == v) {
            if (k == idx) {
                s = Seg{-1, -1, -1, -1, 0, 0, 0};
                return true;
            }
            k++;
        }
    } else if (l == 1) {
        for (int x = 0; x < 4; x++) {
            const int e = u * 4 + x;
            if (I.out_dst()[e] != v) continue;
            if (k == idx) {
                s = Seg{e, -1, -1, -1, x, x, I.out_U()[e]};
                return true;
            }
            k++;
        }
    } else {
        const int j0 = I.in_start()[v], j1 = I.in_start()[v + 1];
        for (int x = 0; x < 4; x++) {
            const int e = u * 4 + x, u2 = I.out_dst()[e];
            if (u2 < 0) continue;
            for (int j = j0; j < j1; j++) {
                const int64_t gg = tgap(I, u2, I.in_src()[j]);
                if (gg >= kINF) continue;
                if (k == idx) {
                    s = Seg{e, j, u2, I.in_src()[j], x, I.in_lab()[j], I.out_U()[e] + gg + I.in_U()[j]};
                    return true;
                }
                k++;
            }
        }
    }
    if (count) *count = k;
    return false;
}

// The segments of l bases from u to v, one at a time, in seg_at's order.
struct SegIter {
    int u, v, l, x, j, j0, j1;
    bool done;
    __device__ SegIter(const Inst& I, int u_, int v_, int l_) : u(u_), v(v_), l(l_), x(0), done(false) {
        j0 = l >= 2 ? I.in_start()[v] : 0;
        j1 = l >= 2 ? I.in_start()[v + 1] : 0;
        j = j0;
    }
    __device__ bool next(const Inst& I, Seg& s) {
        if (l == 0) {
            if (done || u != v) return false;
            done = true;
            s = Seg{-1, -1, -1, -1, 0, 0, 0};
            return true;
        }
        if (l == 1) {
            while (x < 4) {
                const int e = u * 4 + x++;
                if (I.out_dst()[e] == v) {
                    s = Seg{e, -1, -1, -1, e & 3, e & 3, I.out_U()[e]};
                    return true;
                }
            }
            return false;
        }
        while (x < 4) {
            const int e = u * 4 + x, u2 = I.out_dst()[e];
            if (u2 >= 0)
                while (j < j1) {
                    const int jj = j++;
                    const int64_t gg = tgap(I, u2, I.in_src()[jj]);
                    if (gg < kINF) {
                        s = Seg{e, jj, u2, I.in_src()[jj], x, I.in_lab()[jj], I.out_U()[e] + gg + I.in_U()[jj]};
                        return true;
                    }
                }
            x++;
            j = j0;
        }
        return false;
    }
};

// Waves per design: deferred decisions of independent sub-intervals (the rest of the external
// loop beside a closed pair; the left part of a multiloop split beside its last branch) are taken
// by whichever wave is free.
constexpr int kTraceWaves = 8;
constexpr unsigned kTraceSpinCap = 1u << 24;  // polls before a wait is declared failed

// one wave's scratch for the decision it is working on
struct TraceScratch {
    int pre[kNumPairs + 1];  // tuples of the two-loop pairs before pair k
    int jl[64];              // in-edges of b labelled y (closing edge of a pair)
    int hpre[65];            // generic hairpins: prefix of in-degrees of the b1 of jl
};

struct TraceLds {
    SmallE S;
    LoopMin M;
    unsigned char pl1[kNumPairs], pl2[kNumPairs];
    TraceScratch w[kTraceWaves];
    // the shared stack of deferred frames (frames in region A, its top here), guarded by `lock`
    int lock, sp, busy, failed, dup;
    unsigned long long E, U;  // sums over the waves (two's complement)
};

// A wavefront's replay state; every lane holds the same values.
struct Tracer {
    const Inst& I;
    TraceLds& L;
    TraceScratch& W;
    const int32_t* spec;
    int lane;
    int64_t E = 0, U = 0;
    bool fail = false;
    bool dup = false;  // a position emitted twice (lane 0's view, broadcast at the end)
    TFrame next;
    bool have_next = false;

    __device__ Tracer(const Inst& I_, TraceLds& L_, TraceScratch& W_, const int32_t* sp_, int ln)
        : I(I_), L(L_), W(W_), spec(sp_), lane(ln) {}

    __device__ int64_t fxe(int64_t e) const { return e * ((int64_t)1 << I.shift); }

    // the stack's lock: lane 0 spins, the whole wave then orders its accesses after it
    __device__ bool lock() {
        int ok = 1;
        if (lane == 0) {
            unsigned spins = 0;
            while (atomicCAS(&L.lock, 0, 1) != 0) {
                if (++spins > kTraceSpinCap) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        ok = bcast(ok);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (!ok) fail_all(kTrWait);
        return ok;
    }
    // A workgroup-scope release waits only for LDS operations, so the frame a push stored, or the
    // frame a take is still loading from a slot a later push may reuse, is waited for explicitly
    // (vmcnt 0) before the lock is given up.  All waves of the design share this CU's L2.
    __device__ void unlock() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt untouched
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) atomicExch(&L.lock, 0);
    }
    // ends every wave's replay; the first reason recorded is the one reported
    __device__ void fail_all(int reason) {
        fail = true;
        if (lane == 0) atomicCAS(&L.failed, 0, reason);
    }
    // Frames move between waves through region A.  Stack slots are reused, so they are written
    // and read with agent-scope atomic accesses (to L2, past this CU's L1 copy of the slot); the
    // lock's release and acquire order them.
    __device__ static void store_frame(TFrame* p, const TFrame& f) {
        __hip_atomic_store(&p->kind, f.kind, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&p->a, f.a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&p->b, f.b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&p->t, f.t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static TFrame load_frame(TFrame* p) {
        return TFrame{__hip_atomic_load(&p->kind, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(&p->a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(&p->b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(&p->t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
    }
    // defers a decision to the shared stack (at most n + 2 frames: each covers a disjoint interval)
    __device__ void push(int kind, int a, int b, int t) {
        if (!lock()) return;
        int over = 0;
        if (lane == 0) {
            const int slot = L.sp;
            if (slot >= I.n + 2) {
                over = 1;
            } else {
                store_frame(I.tr_stack() + slot, TFrame{kind, a, b, t});
                L.sp = slot + 1;
            }
        }
        unlock();
        if (bcast(over)) fail_all(kTrStack);
    }
    // The next deferred frame once this wave's chain has ended (a wave counted busy stops being
    // busy first): true with a frame (the wave is busy again), false when no wave is busy and the
    // stack is empty, or on failure.  Waiting waves poll the stack's state with plain loads and
    // take the lock only to pop a frame or to confirm the end, so that they do not keep the lock
    // from the busy waves' pushes.
    __device__ bool take(TFrame& f, bool was_busy) {
        if (was_busy) {
            if (!lock()) return false;
            if (lane == 0) L.busy--;
            unlock();
        }
        for (unsigned spins = 0;; spins++) {
            int look = 0;  // 1: a frame to pop or a possible end, 2: failed
            if (lane == 0) {
                const int fl = __hip_atomic_load(&L.failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const int sp = __hip_atomic_load(&L.sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const int bz = __hip_atomic_load(&L.busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                look = fl ? 2 : (sp > 0 || bz == 0) ? 1 : 0;
            }
            look = bcast(look);
            if (look == 2) return false;
            if (look == 1) {
                if (!lock()) return false;
                int st = 0;  // 0: wait, 1: frame, 2: done
                TFrame h{0, 0, 0, 0};
                if (lane == 0) {
                    if (L.failed) {
                        st = 2;
                    } else if (L.sp > 0) {
                        h = load_frame(I.tr_stack() + --L.sp);
                        L.busy++;
                        st = 1;
                    } else if (L.busy == 0) {
                        st = 2;
                    }
                }
                unlock();
                st = bcast(st);
                if (st == 1) {
                    f = TFrame{bcast(h.kind), bcast(h.a), bcast(h.b), bcast(h.t)};
                    // a frame names states of this design (a corrupted one would index out of range)
                    if (f.kind < kFX || f.kind > kFBR || f.a < 0 || f.a >= I.N || f.b < -1 || f.b >= I.N ||
                        f.t < -1 || f.t >= 6) {
                        fail_all(kTrFrame);
                        return false;
                    }
                    return true;
                }
                if (st == 2) return false;
            }
            if (spins > kTraceSpinCap) {
                fail_all(kTrWait);
                return false;
            }
            __builtin_amdgcn_s_sleep(4);
        }
    }
    __device__ void go(int kind, int a, int b, int t) {
        next = TFrame{kind, a, b, t};
        have_next = true;
    }
    __device__ void emit_at(int pos, int lab, int64_t cost) {
        if (lane == 0) {
            if (I.tr_seq()[pos] >= 0) dup = true;
            I.tr_seq()[pos] = lab;
        }
        U += cost;
    }
    __device__ void emit_out(int e) { emit_at(I.layer()[e >> 2], e & 3, I.out_U()[e]); }
    __device__ void emit_in(int j) { emit_at(I.layer()[I.in_src()[j]], I.in_lab()[j], I.in_U()[j]); }
    // the minimum-cost path u -> v, smallest base first at every step (lanes 0..3 try the bases)
    __device__ void emit_gap(int u, int v) {
        while (u != v && !fail) {
            const int64_t g = tgap(I, u, v);
            bool ok = false;
            int d = -1;
            if (lane < 4) {
                const int e = u * 4 + lane;
                d = I.out_dst()[e];
                ok = d >= 0 && sadd(I.out_U()[e], tgap(I, d, v)) == g;
            }
            const unsigned long long m = __ballot(ok);
            if (!m) {
                fail = true;
                return;
            }
            const int x = first_lane(m);
            emit_out(u * 4 + x);
            u = I.out_dst()[u * 4 + x];
        }
    }
    __device__ void emit_seg(const Seg& s) {
        if (s.e1 >= 0) emit_out(s.e1);
        if (s.e2 >= 0) {
            emit_gap(s.gfrom, s.gto);
            emit_in(s.e2);
        }
    }

    __device__ void ext(int a);
    __device__ void closed(int a, int b, int t);
    __device__ bool hairpin(int a, int b, int t, int64_t v, int ea, int a1);
    __device__ bool twoloop(int a, int b, int t, int64_t v, int ea, int a1);
    __device__ void s1(int a, int b);
    __device__ void s2(int a, int b);
    __device__ void branch(int a, int b);
};

__device__ void Tracer::ext(int a) {
    if (I.layer()[a] == I.n) return;
    const int64_t x = I.X()[a];
    bool ok = false;
    if (lane < 4) {
        const int d = I.out_dst()[a * 4 + lane];
        ok = d >= 0 && sadd(I.out_U()[a * 4 + lane], I.X()[d]) == x;
    }
    unsigned long long m = __ballot(ok);
    if (m) {
        const int y = first_lane(m), e = a * 4 + y;
        emit_out(e);
        go(kFX, I.out_dst()[e], -1, -1);
        return;
    }
    // branches b (state order), pair types in order; one state per lane
    const int la = I.layer()[a];
    const int b0 = la + 5 <= I.n ? I.off()[la + 5] : I.N;
    for (int base = b0; base < I.N; base += 64) {
        const int bb = base + lane;
        int hit = INT_MAX;
        if (bb < I.N) {
            const int64_t* vr = I.V() + tcell(I, a, bb) * 6;
            const int64_t xb = I.X()[bb];
            for (int t = 0; t < 6; t++)
                if (sadd(sadd(vr[t], fxe(au_pen(L.S, t))), xb) == x) {
                    hit = bb * 8 + t;
                    break;
                }
        }
        hit = wmin_int(hit);
        if (hit != INT_MAX) {
            const int b = hit >> 3, t = hit & 7;
            E += au_pen(L.S, t);
            push(kFX, b, -1, -1);
            go(kFV, a, b, t);
            return;
        }
    }
    fail = true;
}

__device__ bool Tracer::hairpin(int a, int b, int t, int64_t v, int ea, int a1) {
    const int g = I.layer()[b] - I.layer()[a], m = g - 2;
    if (m < 3) return false;
    if (m == 3 || m == 4 || m == 6) {
        // every label path of g edges from a whose first base is x and last base y, in
        // lexicographic order: the middle g - 2 bases are the digits of the lane's combination
        const int mid = g - 2, combos = 1 << (2 * mid);
        const int off = m == 3 ? kSpecOff5 : m == 4 ? kSpecOff6 : kSpecOff8;
        for (int base = 0; base < combos; base += 64) {
            const int cmb = base + lane;
            bool ok = false;
            int32_t en = 0;
            if (cmb < combos) {
                int st = a, key = 0, l1 = 0, lm = 0;
                int64_t cost = 0;
                ok = true;
                for (int i = 0; i < g && ok; i++) {
                    const int lab = i == 0 ? kTX[t] : i == g - 1 ? kTY[t] : (cmb >> (2 * (mid - i))) & 3;
                    if (i == 1) l1 = lab;
                    if (i == g - 2) lm = lab;
                    const int e = st * 4 + lab, d = I.out_dst()[e];
                    if (d < 0) ok = false;
                    else {
                        cost += I.out_U()[e];
                        key = key * 4 + lab;
                        st = d;
                    }
                }
                if (ok && st == b) {
                    en = spec[off + key];
                    if (en == kNoSpecial) en = I.hp_init()[m] + (m == 3 ? au_pen(L.S, t) : L.S.mmH[t][l1][lm]);
                    ok = cost + fxe(en) == v;
                } else {
                    ok = false;
                }
            }
            const unsigned long long msk = __ballot(ok);
            if (msk) {
                const int win = base + first_lane(msk);
                int st = a, key = 0, l1 = 0, lm = 0;
                for (int i = 0; i < g; i++) {
                    const int lab = i == 0 ? kTX[t] : i == g - 1 ? kTY[t] : (win >> (2 * (mid - i))) & 3;
                    if (i == 1) l1 = lab;
                    if (i == g - 2) lm = lab;
                    emit_out(st * 4 + lab);
                    key = key * 4 + lab;
                    st = I.out_dst()[st * 4 + lab];
                }
                int32_t e2 = spec[off + key];
                if (e2 == kNoSpecial) e2 = I.hp_init()[m] + (m == 3 ? au_pen(L.S, t) : L.S.mmH[t][l1][lm]);
                E += e2;
                return true;
            }
        }
        return false;
    }
    // generic size: a -x-> a1 -x2-> a2 ~~> b2 -z-> b1 -y-> b, alternatives (x2, closing in-edge of
    // b, in-edge of b1) in order, flattened over the lanes with the prefix of the b1 in-degrees
    const int y = kTY[t];
    const int ib0 = I.in_start()[b], ib1 = I.in_start()[b + 1];
    int nj = 0;
    for (int j0 = ib0; j0 < ib1; j0 += 64) {
        const int j = j0 + lane;
        const bool lab = j < ib1 && I.in_lab()[j] == y;
        const unsigned long long msk = __ballot(lab);
        const int at = nj + __popcll(msk & ((1ull << lane) - 1));
        if (lab && at < 64) W.jl[at] = j;
        nj += __popcll(msk);
    }
    if (nj > 64) nj = 64;  // a state has at most 64 in-edges (4 labels x 16 sources)
    __builtin_amdgcn_wave_barrier();
    int deg = 0;
    if (lane < nj) {
        const int b1 = I.in_src()[W.jl[lane]];
        deg = I.in_start()[b1 + 1] - I.in_start()[b1];
    }
    int incl = deg;
    for (int o = 1; o < 64; o <<= 1) {
        const int w = __shfl_up(incl, o, 64);
        if (lane >= o) incl += w;
    }
    if (lane < nj) W.hpre[lane + 1] = incl;
    if (lane == 0) W.hpre[0] = 0;
    __builtin_amdgcn_wave_barrier();
    const int per = bcast(__shfl(incl, 63, 64));
    const int total = 4 * per;
    const int64_t Ua = I.out_U()[ea];
    for (int base = 0; base < total; base += 64) {
        const int idx = base + lane;
        bool ok = false;
        if (idx < total) {
            const int x2 = idx / per, r = idx - x2 * per;
            int jj = 0;
            while (jj + 1 < nj && W.hpre[jj + 1] <= r) jj++;
            const int j = W.jl[jj], b1 = I.in_src()[j];
            const int j2 = I.in_start()[b1] + (r - W.hpre[jj]);
            const int e1 = a1 * 4 + x2, a2 = I.out_dst()[e1];
            if (a2 >= 0) {
                const int64_t gg = tgap(I, a2, I.in_src()[j2]);
                if (gg < kINF) {
                    const int32_t en = I.hp_init()[m] + L.S.mmH[t][x2][I.in_lab()[j2]];
                    ok = Ua + I.out_U()[e1] + gg + I.in_U()[j2] + I.in_U()[j] + fxe(en) == v;
                }
            }
        }
        const unsigned long long msk = __ballot(ok);
        if (msk) {
            const int win = base + first_lane(msk);
            const int x2 = win / per, r = win - x2 * per;
            int jj = 0;
            while (jj + 1 < nj && W.hpre[jj + 1] <= r) jj++;
            const int j = W.jl[jj], b1 = I.in_src()[j];
            const int j2 = I.in_start()[b1] + (r - W.hpre[jj]);
            const int e1 = a1 * 4 + x2;
            emit_out(ea);
            emit_out(e1);
            emit_gap(I.out_dst()[e1], I.in_src()[j2]);
            emit_in(j2);
            emit_in(j);
            E += I.hp_init()[m] + L.S.mmH[t][x2][I.in_lab()[j2]];
            return true;
        }
    }
    return false;
}

__device__ bool Tracer::twoloop(int a, int b, int t, int64_t v, int ea, int a1) {
    const int la = I.layer()[a], lb = I.layer()[b], g = lb - la;
    if (g < 7) return false;
    const int y = kTY[t];
    // closing in-edges of b labelled y, in CSR order
    const int ib0 = I.in_start()[b], ib1 = I.in_start()[b + 1];
    int nj = 0;
    for (int j0 = ib0; j0 < ib1; j0 += 64) {
        const int j = j0 + lane;
        const bool lab = j < ib1 && I.in_lab()[j] == y;
        const unsigned long long msk = __ballot(lab);
        const int at = nj + __popcll(msk & ((1ull << lane) - 1));
        if (lab && at < 64) W.jl[at] = j;
        nj += __popcll(msk);
    }
    if (nj > 64) nj = 64;
    if (nj == 0) return false;
    // tuples (pair k, closing edge, c, d) per pair: nj * width(cl) * width(dl) when the pair fits
    // (l1 + l2 <= g - 7); prefix over the pairs in canonical order, eight pairs per lane
    {
        int cnt[8], sum = 0;
        for (int i = 0; i < 8; i++) {
            const int k = lane * 8 + i;
            int c = 0;
            if (k < kNumPairs) {
                const int l1 = L.pl1[k], l2 = L.pl2[k];
                if (l1 + l2 <= g - 7) {
                    const int cl = la + 1 + l1, dl = lb - 1 - l2;
                    c = nj * (I.off()[cl + 1] - I.off()[cl]) * (I.off()[dl + 1] - I.off()[dl]);
                }
            }
            cnt[i] = c;
            sum += c;
        }
        int incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const int w = __shfl_up(incl, o, 64);
            if (lane >= o) incl += w;
        }
        int acc = incl - sum;
        for (int i = 0; i < 8; i++) {
            const int k = lane * 8 + i;
            if (k <= kNumPairs) W.pre[k] = acc;
            acc += cnt[i];
        }
        __builtin_amdgcn_wave_barrier();
    }
    const int total = W.pre[kNumPairs];
    const int64_t Ua = I.out_U()[ea];
    // four groups per lane and round (group T = base + lane + 64 k): their independent loads are
    // issued together, then each group's lower bound is tested and, rarely, its alternatives
    // enumerated; the lane's first match is its smallest matching group
    constexpr int kPer = 4;
    for (int base = 0; base < total; base += 64 * kPer) {
        int code = INT_MAX;  // the lane's first matching group and its (tp, p, q)
        int wtp = 0, wp = 0, wq = 0;
        int tl1[kPer], tl2[kPer], tc[kPer], td[kPer], tj[kPer], tb1[kPer];
        int64_t tU[kPer], tgl[kPer], tgr[kPer];
        const int64_t* tvr[kPer];
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const int T = base + lane + 64 * k;
            tl1[k] = -1;
            if (T >= total) continue;
            int lo = 0, hi = kNumPairs - 1;  // last pair whose prefix <= T
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (W.pre[mid] <= T) lo = mid;
                else hi = mid - 1;
            }
            const int l1 = L.pl1[lo], l2 = L.pl2[lo];
            const int cl = la + 1 + l1, dl = lb - 1 - l2;
            const int c0 = I.off()[cl], d0 = I.off()[dl];
            const int wc = I.off()[cl + 1] - c0, wd = I.off()[dl + 1] - d0;
            const int r = T - W.pre[lo], jj = r / (wc * wd), ci = (r / wd) % wc, di = r % wd;
            tl1[k] = l1;
            tl2[k] = l2;
            tc[k] = c0 + ci;
            td[k] = d0 + di;
            tj[k] = W.jl[jj];
        }
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            if (tl1[k] < 0) continue;
            tb1[k] = I.in_src()[tj[k]];
            tU[k] = I.in_U()[tj[k]];
            tvr[k] = I.V() + tcell(I, tc[k], td[k]) * 6;
        }
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            if (tl1[k] < 0) continue;
            tgl[k] = tl1[k] == 0 ? (a1 == tc[k] ? 0 : kINF) : tgap(I, a1, tc[k]);
            tgr[k] = tl2[k] == 0 ? (td[k] == tb1[k] ? 0 : kINF) : tgap(I, td[k], tb1[k]);
        }
        for (int k = 0; k < kPer && code == INT_MAX; k++) {
            if (tl1[k] < 0 || tgl[k] >= kINF || tgr[k] >= kINF) continue;
            const int l1 = tl1[k], l2 = tl2[k], c = tc[k], d = td[k], b1 = tb1[k];
            const int64_t* vr = tvr[k];
            int64_t vmin = kINF;
            for (int tp = 0; tp < 6; tp++) vmin = mn(vmin, vr[tp]);
            // exact lower bound of every alternative of the group
            const int64_t lb0 = Ua + tgl[k] + tgr[k] + tU[k] + fxe(two_loop_lb(L.S, L.M, t, l1, l2));
            if (vmin >= kINF || lb0 + vmin > v) continue;
            // enumerate (inner type, left segment, right segment) in order
            for (int tp = 0; tp < 6 && code == INT_MAX; tp++) {
                const int64_t vin = vr[tp];
                if (vin >= kINF || lb0 + vin > v) continue;
                const int tr = kRev[tp];
                Seg sl, sr;
                SegIter li(I, a1, c, l1);
                for (int p = 0; code == INT_MAX && li.next(I, sl); p++) {
                    SegIter ri(I, d, b1, l2);
                    for (int q = 0; code == INT_MAX && ri.next(I, sr); q++) {
                        const int32_t e2 = two_loop_e(L.S, t, tr, l1, l2, sl.xa, sl.xb, sr.xa, sr.xb);
                        if (Ua + sl.cost + vin + sr.cost + tU[k] + fxe(e2) == v) {
                            code = base + lane + 64 * k;
                            wtp = tp;
                            wp = p;
                            wq = q;
                        }
                    }
                }
            }
        }
        const int best = wmin_int(code);
        if (best == INT_MAX) continue;
        const int wl = first_lane(__ballot(code == best));
        const int tp = __shfl(wtp, wl, 64), p = __shfl(wp, wl, 64), q = __shfl(wq, wl, 64);
        // decode the winning tuple (uniform)
        int lo = 0, hi = kNumPairs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (W.pre[mid] <= best) lo = mid;
            else hi = mid - 1;
        }
        const int k = lo, l1 = L.pl1[k], l2 = L.pl2[k];
        const int cl = la + 1 + l1, dl = lb - 1 - l2;
        const int wc = I.off()[cl + 1] - I.off()[cl], wd = I.off()[dl + 1] - I.off()[dl];
        const int r = best - W.pre[k], jj = r / (wc * wd), ci = (r / wd) % wc, di = r % wd;
        const int j = W.jl[jj], b1 = I.in_src()[j], c = I.off()[cl] + ci, d = I.off()[dl] + di;
        Seg sl, sr;
        seg_at(I, a1, c, l1, p, sl);
        seg_at(I, d, b1, l2, q, sr);
        const int32_t e2 = two_loop_e(L.S, t, kRev[tp], l1, l2, sl.xa, sl.xb, sr.xa, sr.xb);
        emit_out(ea);
        emit_seg(sl);
        emit_seg(sr);
        emit_in(j);
        E += e2;
        go(kFV, c, d, tp);
        return true;
    }
    return false;
}

__device__ void Tracer::closed(int a, int b, int t) {
    const int64_t v = tV(I, t, a, b);
    const int i = I.layer()[a], j = I.layer()[b] - 1;
    if (lane == 0) {
        I.tr_pair()[i] = j;
        I.tr_pair()[j] = i;
    }
    const int ea = a * 4 + kTX[t], a1 = I.out_dst()[ea];
    if (a1 < 0 || v >= kINF) {
        fail = true;
        return;
    }
    if (hairpin(a, b, t, v, ea, a1)) return;
    if (twoloop(a, b, t, v, ea, a1)) return;
    // multiloop: closing in-edge of b labelled y, in CSR order
    if (I.layer()[b] - I.layer()[a] >= 12) {
        const int y = kTY[t];
        const int32_t mlc = L.S.ml_closing + L.S.ml_intern + au_pen(L.S, t);
        const int64_t Ua = I.out_U()[ea];
        const int ib0 = I.in_start()[b], ib1 = I.in_start()[b + 1];
        for (int j0 = ib0; j0 < ib1; j0 += 64) {
            const int jj = j0 + lane;
            bool ok = false;
            if (jj < ib1 && I.in_lab()[jj] == y) {
                const int b1 = I.in_src()[jj];
                ok = I.layer()[b1] - I.layer()[a1] >= 10 && sadd(Ua + I.in_U()[jj] + fxe(mlc), tS2(I, a1, b1)) == v;
            }
            const unsigned long long msk = __ballot(ok);
            if (msk) {
                const int jw = j0 + first_lane(msk);
                emit_out(ea);
                emit_in(jw);
                E += mlc;
                go(kFS2, a1, I.in_src()[jw], -1);
                return;
            }
        }
    }
    fail = true;
}

__device__ void Tracer::branch(int a, int b) {
    const int64_t v = tB(I, a, b);
    bool ok = false;
    if (lane < 6) ok = sadd(tV(I, lane, a, b), fxe(L.S.ml_intern + au_pen(L.S, lane))) == v;
    const unsigned long long m = __ballot(ok);
    if (!m) {
        fail = true;
        return;
    }
    const int t = first_lane(m);
    E += L.S.ml_intern + au_pen(L.S, t);
    go(kFV, a, b, t);
}

__device__ void Tracer::s1(int a, int b) {
    const int64_t v = tS1(I, a, b);
    // items: 0 direct branch, 1 S2, 2..5 left unpaired edge by label, 6.. right unpaired in-edge
    const int ib0 = I.in_start()[b], ib1 = I.in_start()[b + 1], total = 6 + (ib1 - ib0);
    const int la = I.layer()[a], lb = I.layer()[b];
    for (int base = 0; base < total; base += 64) {
        const int it = base + lane;
        bool ok = false;
        if (it == 0) ok = tB(I, a, b) == v;
        else if (it == 1) ok = tS2(I, a, b) == v;
        else if (it < 6) {
            const int e = a * 4 + it - 2, ap = I.out_dst()[e];
            ok = ap >= 0 && I.layer()[ap] < lb && sadd(I.out_U()[e] + I.mlbase_fx, tS1(I, ap, b)) == v;
        } else if (it < total) {
            const int j = ib0 + it - 6, bp = I.in_src()[j];
            ok = I.layer()[bp] > la && sadd(tS1(I, a, bp), I.in_U()[j] + I.mlbase_fx) == v;
        }
        const unsigned long long m = __ballot(ok);
        if (!m) continue;
        const int w = base + first_lane(m);
        if (w == 0) go(kFBR, a, b, -1);
        else if (w == 1) go(kFS2, a, b, -1);
        else if (w < 6) {
            const int e = a * 4 + w - 2;
            emit_out(e);
            E += L.S.ml_base;
            go(kFS1, I.out_dst()[e], b, -1);
        } else {
            const int j = ib0 + w - 6;
            emit_in(j);
            E += L.S.ml_base;
            go(kFS1, a, I.in_src()[j], -1);
        }
        return;
    }
    fail = true;
}

__device__ void Tracer::s2(int a, int b) {
    const int64_t v = tS2(I, a, b);
    const int ib0 = I.in_start()[b], ib1 = I.in_start()[b + 1];
    const int la = I.layer()[a];
    for (int j0 = ib0; j0 < ib1; j0 += 64) {
        const int j = j0 + lane;
        bool ok = false;
        if (j < ib1) {
            const int bp = I.in_src()[j];
            ok = I.layer()[bp] > la && sadd(tS2(I, a, bp), I.in_U()[j] + I.mlbase_fx) == v;
        }
        const unsigned long long m = __ballot(ok);
        if (m) {
            const int jw = j0 + first_lane(m);
            emit_in(jw);
            E += L.S.ml_base;
            go(kFS2, a, I.in_src()[jw], -1);
            return;
        }
    }
    // strict candidates c of C_b with layer(c) > layer(a): the smallest matching state index
    const int64_t cbase = I.coff()[b];
    const int cnt = I.ccnt()[b];
    int best = INT_MAX;
    for (int k = lane; k < cnt; k += 64) {
        const int raw = I.cc()[cbase + k];
        if (raw < 0 || raw >= best || I.layer()[raw] <= la) continue;  // non-strict entries have bit 31 set
        if (sadd(tS1(I, a, raw), tB(I, raw, b)) == v) best = raw;
    }
    best = wmin_int(best);
    if (best == INT_MAX) {
        fail = true;
        return;
    }
    push(kFS1, a, best, -1);
    go(kFBR, best, b, -1);
}

__device__ void trace_instance(const Inst& I, const EnergyTables* __restrict__ E, const int32_t* __restrict__ spec,
                               TraceLds& L) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    stage_tables(L.S, E);
    for (int k = tid; k < kNumPairs; k += blockDim.x) {  // (l1, l2) in canonical order
        int l1 = 0, r = k;
        while (r >= 31 - l1) {
            r -= 31 - l1;
            l1++;
        }
        L.pl1[k] = (unsigned char)l1;
        L.pl2[k] = (unsigned char)r;
    }
    for (int p = tid; p < I.n; p += blockDim.x) {
        I.tr_seq()[p] = -1;
        I.tr_pair()[p] = -1;
    }
    if (tid == 0) {
        L.lock = 0;
        L.sp = 0;
        L.busy = 1;  // wave 0 starts busy with X(s)
        L.failed = 0;
        L.dup = 0;
        L.E = 0;
        L.U = 0;
    }
    __syncthreads();  // every wave's share of the energy tables is staged
    if (wave == 0) loop_minima(L.S, L.M, lane);
    // A position is initialised by one wave and later written by whichever wave emits it: every
    // wave waits for its initialising stores before the barrier (which by itself waits only for
    // LDS operations), so that no -1 can land after an emitted value.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    Tracer tr(I, L, L.w[wave], spec, lane);
    const int64_t xs = I.X()[0];
    if (wave == 0) {
        if (xs >= kINF) tr.fail_all(kTrUnreachable);
        tr.go(kFX, 0, -1, -1);
    }
    bool busy = wave == 0;
    for (;;) {
        if (tr.fail) {
            tr.fail_all(kTrNoMatch);  // a no-match decision (other reasons were recorded already)
            break;
        }
        TFrame f;
        if (tr.have_next) {
            f = tr.next;
            tr.have_next = false;
        } else {
            // this wave's chain has ended (or it never had one): a deferred frame, or the end
            const bool got = tr.take(f, busy);
            busy = got;
            if (!got) break;
        }
        switch (f.kind) {
            case kFX: tr.ext(f.a); break;
            case kFV: tr.closed(f.a, f.b, f.t); break;
            case kFS1: tr.s1(f.a, f.b); break;
            case kFS2: tr.s2(f.a, f.b); break;
            default: tr.branch(f.a, f.b); break;
        }
    }
    const int dup = bcast(tr.dup ? 1 : 0);
    if (lane == 0) {
        atomicAdd(&L.E, (unsigned long long)tr.E);
        atomicAdd(&L.U, (unsigned long long)tr.U);
        if (dup) atomicOr(&L.dup, 1);
    }
    __syncthreads();
    if (tid == 0) {
        I.tr_res()[0] = (long long)L.E;
        I.tr_res()[1] = (long long)L.U;
        I.tr_res()[2] = L.failed ? L.failed : L.dup ? kTrDup : kTrOk;
        I.tr_res()[3] = xs;
    }
}

__global__ __launch_bounds__(64 * kTraceWaves) void k_trace(Inst I, const EnergyTables* __restrict__ E,
                                                            const int32_t* __restrict__ spec) {
    __shared__ TraceLds L;
    trace_instance(I, E, spec, L);
}

__global__ __launch_bounds__(64 * kTraceWaves) void k_trace_many(const Inst* __restrict__ insts,
                                                                 const EnergyTables* __restrict__ E,
                                                                 const int32_t* __restrict__ spec) {
    __shared__ TraceLds L;
    const Inst I = insts[blockIdx.x];
    trace_instance(I, E, spec, L);
}

// strict candidates per right endpoint (retain-all control: non-strict entries carry bit 31)
__global__ void k_strict_count(Inst I) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= I.N) return;
    const int64_t base = I.coff()[b];
    int c = 0;
    for (int k = 0; k < I.ccnt()[b]; k++) c += I.cc()[base + k] >= 0;
    I.cstrict()[b] = c;
}

}  // namespace

hipError_t launch_trace(const Inst& I, const EnergyTables* E, const int32_t* spec, hipStream_t st) {
    hipLaunchKernelGGL(k_trace, dim3(1), dim3(64 * kTraceWaves), 0, st, I, E, spec);
    return hipGetLastError();
}

hipError_t launch_trace_many(const Inst* insts_dev, int n, const EnergyTables* E, const int32_t* spec,
                             hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trace_many, dim3(n), dim3(64 * kTraceWaves), 0, st, insts_dev, E, spec);
    return hipGetLastError();
}

hipError_t launch_strict_count(const Inst& I, hipStream_t st) {
    hipLaunchKernelGGL(k_strict_count, dim3((I.N + 255) / 256), dim3(256), 0, st, I);
    return hipGetLastError();
}

}  // namespace sd
