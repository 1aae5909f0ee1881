// gfx950 kernels of the span wavefront (Sec. 5, Algorithm 1, re-designed for the GPU).
//
// One launch per span length g.  A wavefront (64 lanes) owns one layer pair (p, q = p + g) and
// therefore every cell (a, b) with a in layer p and b in layer q; it is the only writer of the
// candidate segments C_b of its right endpoints in this step (the endpoint-ownership rule of
// Sec. 5), so appends need no atomics and land in start-state order.  Inside a cell the lanes
// split the closed-value enumeration (hairpin paths / two-loop (l1,l2) pairs / multiloop
// in-edges) and the candidate-prefix scan of eq. (7), then reduce with wavefront min shuffles.
// An extra workgroup per launch fills the external column one layer behind the wavefront.
#include <hip/hip_runtime.h>

#include "sd_internal.h"

namespace sd {

__constant__ int kTX[6] = {0, 1, 2, 2, 3, 3};  // 5' base of AU CG GC GU UA UG
__constant__ int kTY[6] = {3, 2, 1, 3, 0, 2};  // 3' base
__constant__ int kPairType[16] = {-1, -1, -1, 0, -1, -1, 1, -1, -1, 2, -1, 3, 4, -1, 5, -1};
// (l1, l2) pairs in canonical order: l1 ascending, then l2 ascending, l1 + l2 <= 30
__constant__ unsigned char kL1[kNumPairs];
__constant__ unsigned char kL2[kNumPairs];

__device__ __forceinline__ int ptype(int x, int y) { return kPairType[x * 4 + y]; }
__device__ __forceinline__ int32_t au_pen(const EnergyTables* E, int t) {
    return (t == 1 || t == 2) ? 0 : E->terminal_au;
}
__device__ __forceinline__ int64_t mn(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t fx(int32_t e, int s) { return (int64_t)e * ((int64_t)1 << s); }
__device__ __forceinline__ int64_t norm_inf(int64_t v) { return v >= kHalfINF ? kINF : v; }

__device__ __forceinline__ int64_t shfl_xor64(int64_t v, int m) {
    int lo = __shfl_xor((int)(uint32_t)(uint64_t)v, m, 64);
    int hi = __shfl_xor((int)(uint32_t)((uint64_t)v >> 32), m, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
__device__ __forceinline__ int64_t wave_min(int64_t v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = mn(v, shfl_xor64(v, m));
    return v;
}

__device__ __forceinline__ int64_t cell_of(const Inst& I, int a, int b) {
    return I.rowoff[a] + (b - I.off[I.layer[a] + 1]);
}

// Minimum path cost between states of the codon trie (closed form; INF if unreachable).
__device__ __forceinline__ int64_t gap(const Inst& I, int a, int b) {
    int la = I.layer[a], lb = I.layer[b];
    if (la == lb) return a == b ? 0 : kINF;
    int ka = la / 3, kb = lb / 3;
    if (ka == kb) {
        if (la % 3 == 0) return 0;
        return (I.pfx[b] >> 2) == I.pfx[a] ? 0 : kINF;
    }
    return I.tail[a] + I.P[kb] - I.P[ka + 1];
}

__device__ int32_t two_loop_e(const EnergyTables* __restrict__ E, int t, int tr, int l1, int l2,
                              int xi1, int xk1, int xl1, int xj1) {
    if (l1 == 0 && l2 == 0) return E->stack[t][tr];
    if (l1 == 0 || l2 == 0) {
        int l = l1 + l2;
        if (l == 1) return E->bulge[1] + E->stack[t][tr];
        return E->bulge[l] + au_pen(E, t) + au_pen(E, tr);
    }
    if (l1 == 1 && l2 == 1) return E->int11[t][tr][xi1][xj1];
    if (l1 == 1 && l2 == 2) return E->int21[t][tr][xi1][xl1][xj1];
    if (l1 == 2 && l2 == 1) return E->int21[tr][t][xl1][xi1][xk1];
    if (l1 == 2 && l2 == 2) return E->int22[t][tr][xi1][xk1][xl1][xj1];
    int d = l1 > l2 ? l1 - l2 : l2 - l1;
    int32_t asym = E->ninio * d;
    asym = asym < E->ninio_max ? asym : E->ninio_max;
    int32_t e = E->interior[l1 + l2] + asym;
    if (l1 == 1 || l2 == 1) return e + E->mm1n[t][xi1][xj1] + E->mm1n[tr][xl1][xk1];
    if (l1 + l2 == 5 && (l1 == 2 || l1 == 3)) return e + E->mm23[t][xi1][xj1] + E->mm23[tr][xl1][xk1];
    return e + E->mmI[t][xi1][xj1] + E->mmI[tr][xl1][xk1];
}

// ---- hairpin closure ------------------------------------------------------------------------
// Sizes 3, 4, 6 may match a listed special loop, so each lane walks the paths whose bases at
// positions 1..3 equal its lane id in base 4; other sizes decompose into the two outer edges on
// each side plus a minimum-cost unpaired interior.
__device__ int64_t hairpin_lane(const Inst& I, const EnergyTables* __restrict__ E,
                                const int32_t* __restrict__ spec, int a, int b, int t, int a1,
                                int64_t Ua, int lane) {
    const int la = I.layer[a], g = I.layer[b] - la, m = g - 2, s = I.shift;
    const int x = kTX[t], y = kTY[t];
    int64_t best = kINF;
    if (m == 3 || m == 4 || m == 6) {
        int l1 = (lane >> 4) & 3, l2 = (lane >> 2) & 3, l3 = lane & 3;
        int st = a1;
        int64_t cost = Ua;
        int key = x;
        int labs[3] = {l1, l2, l3};
        for (int i = 0; i < 3; i++) {
            int e = st * 4 + labs[i];
            int d = I.out_dst[e];
            if (d < 0) return kINF;
            cost += I.out_U[e];
            key = key * 4 + labs[i];
            st = d;
        }
        // remaining free positions: g - 5 (0, 1 or 3), then the last base y into b
        const int nfree = g - 5;
        const int combos = 1 << (2 * nfree);
        for (int k = 0; k < combos; k++) {
            int st2 = st, key2 = key, ok = 1, lastfree = l3;
            int64_t c2 = cost;
            for (int i = nfree - 1; i >= 0; i--) {
                int lab = (k >> (2 * i)) & 3;
                int e = st2 * 4 + lab;
                int d = I.out_dst[e];
                if (d < 0) { ok = 0; break; }
                c2 += I.out_U[e];
                key2 = key2 * 4 + lab;
                st2 = d;
                lastfree = lab;
            }
            if (!ok) {
                // skip the whole subtree below the failing position would be faster; sizes are tiny
                continue;
            }
            int e = st2 * 4 + y;
            if (I.out_dst[e] != b) continue;
            c2 += I.out_U[e];
            key2 = key2 * 4 + y;
            int off = m == 3 ? kSpecOff5 : m == 4 ? kSpecOff6 : kSpecOff8;
            int32_t en = spec[off + key2];
            if (en == kNoSpecial) {
                en = I.hp_init[m] + (m == 3 ? au_pen(E, t) : E->mmH[t][l1][lastfree]);
            }
            best = mn(best, c2 + fx(en, s));
        }
        return best;
    }
    // generic: a -x-> a1 -x2-> a2 ~~> b2 -z-> b1 -y-> b
    const int ib0 = I.in_start[b], ib1 = I.in_start[b + 1];
    const int nb = ib1 - ib0;
    for (int k = lane; k < 4 * 8 * 8; k += 64) {
        int x2 = k & 3, i1 = (k >> 2) & 7, i2 = k >> 5;
        if (i1 >= nb) continue;
        int eb = ib0 + i1;
        if (I.in_lab[eb] != y) continue;
        int b1 = I.in_src[eb];
        int j0 = I.in_start[b1];
        if (i2 >= I.in_start[b1 + 1] - j0) continue;
        int eb2 = j0 + i2;
        int e1 = a1 * 4 + x2;
        int a2 = I.out_dst[e1];
        if (a2 < 0) continue;
        int b2 = I.in_src[eb2];
        int64_t gg = gap(I, a2, b2);
        if (gg >= kINF) continue;
        int32_t en = I.hp_init[m] + E->mmH[t][x2][I.in_lab[eb2]];
        best = mn(best, Ua + I.out_U[e1] + gg + I.in_U[eb2] + I.in_U[eb] + fx(en, s));
    }
    return best;
}

// ---- two-loop closure: stack, bulge, interior with l1 + l2 <= 30 -------------------------------
struct Seg {
    int xa, xb;
    int64_t cost;
};
constexpr int kMaxSegs = 24;  // 4 first bases x at most 6 in-edges (codon family size)

// unpaired segment u ~> v with l bases (l >= 1); boundary labels (first, last)
__device__ __forceinline__ int segs(const Inst& I, int u, int v, int l, Seg* out) {
    int k = 0;
    if (l == 1) {
        for (int x = 0; x < 4; x++) {
            int e = u * 4 + x;
            if (I.out_dst[e] == v && k < kMaxSegs) out[k++] = Seg{x, x, I.out_U[e]};
        }
        return k;
    }
    const int j0 = I.in_start[v], j1 = I.in_start[v + 1];
    for (int x = 0; x < 4; x++) {
        int e = u * 4 + x;
        int u2 = I.out_dst[e];
        if (u2 < 0) continue;
        for (int j = j0; j < j1; j++) {
            int64_t gg = gap(I, u2, I.in_src[j]);
            if (gg >= kINF || k >= kMaxSegs) continue;
            out[k++] = Seg{x, I.in_lab[j], I.out_U[e] + gg + I.in_U[j]};
        }
    }
    return k;
}

__device__ int64_t twoloop_lane(const Inst& I, const EnergyTables* __restrict__ E, int a, int b,
                                int t, int a1, int64_t Ua, int lane) {
    const int la = I.layer[a], lb = I.layer[b], s = I.shift, y = kTY[t];
    const int ib0 = I.in_start[b], ib1 = I.in_start[b + 1];
    int64_t best = kINF;
    Seg L[kMaxSegs], R[kMaxSegs];
    for (int pi = lane; pi < kNumPairs; pi += 64) {
        const int l1 = kL1[pi], l2 = kL2[pi];
        const int cl = la + 1 + l1, dl = lb - 1 - l2;
        if (dl - cl < 5) continue;
        for (int eb = ib0; eb < ib1; eb++) {
            if (I.in_lab[eb] != y) continue;
            const int b1 = I.in_src[eb];
            const int64_t Uab = Ua + I.in_U[eb];
            for (int c = I.off[cl]; c < I.off[cl + 1]; c++) {
                int nl;
                if (l1 == 0) {
                    if (c != a1) continue;
                    nl = 1;
                    L[0] = Seg{0, 0, 0};
                } else {
                    nl = segs(I, a1, c, l1, L);
                    if (!nl) continue;
                }
                const int64_t crow = I.rowoff[c] - I.off[cl + 1];
                for (int d = I.off[dl]; d < I.off[dl + 1]; d++) {
                    const int64_t* vcd = I.V + (crow + d) * 6;
                    int nr = -1;
                    for (int tp = 0; tp < 6; tp++) {
                        const int64_t vin = vcd[tp];
                        if (vin >= kINF) continue;
                        if (nr < 0) {
                            if (l2 == 0) {
                                nr = d == b1 ? 1 : 0;
                                R[0] = Seg{0, 0, 0};
                            } else {
                                nr = segs(I, d, b1, l2, R);
                            }
                        }
                        if (!nr) break;
                        const int tr = ptype(kTY[tp], kTX[tp]);
                        for (int i = 0; i < nl; i++)
                            for (int j = 0; j < nr; j++) {
                                int32_t e2 = two_loop_e(E, t, tr, l1, l2, L[i].xa, L[i].xb, R[j].xa, R[j].xb);
                                best = mn(best, Uab + L[i].cost + vin + R[j].cost + fx(e2, s));
                            }
                    }
                }
            }
        }
    }
    return best;
}

// ---- multiloop closure ------------------------------------------------------------------------
__device__ int64_t multiloop_lane(const Inst& I, const EnergyTables* __restrict__ E, int a, int b,
                                  int t, int a1, int64_t Ua, int lane) {
    const int y = kTY[t];
    const int ib0 = I.in_start[b], ib1 = I.in_start[b + 1];
    const int32_t mlc = E->ml_closing + E->ml_intern + au_pen(E, t);
    int64_t best = kINF;
    for (int eb = ib0 + lane; eb < ib1; eb += 64) {
        if (I.in_lab[eb] != y) continue;
        int b1 = I.in_src[eb];
        if (I.layer[b1] - I.layer[a1] < 10) continue;
        int64_t s2 = I.S2[cell_of(I, a1, b1)];
        best = mn(best, s2 + Ua + I.in_U[eb] + fx(mlc, I.shift));  // s2 may be INF: normalised later
    }
    return best;
}

// ---- external column: X(a) for every a of layer L (one workgroup) ------------------------------
__device__ void ext_column(const Inst& I, const EnergyTables* __restrict__ E, int L) {
    __shared__ int64_t red[256];
    const int tid = threadIdx.x;
    for (int a = I.off[L]; a < I.off[L + 1]; a++) {
        int64_t v = kINF;
        if (tid < 4) {
            int d = I.out_dst[a * 4 + tid];
            if (d >= 0) v = I.out_U[a * 4 + tid] + I.X[d];
        }
        if (L + 5 <= I.n) {
            const int bstart = I.off[L + 5];
            const int64_t base = I.rowoff[a] - I.off[L + 1];
            for (int bb = bstart + tid; bb < I.N; bb += blockDim.x) {
                const int64_t* vr = I.V + (base + bb) * 6;
                const int64_t xb = I.X[bb];
#pragma unroll
                for (int t = 0; t < 6; t++) {
                    int64_t vt = vr[t];
                    if (vt < kINF) v = mn(v, vt + fx(au_pen(E, t), I.shift) + xb);
                }
            }
        }
        red[tid] = v;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] = mn(red[tid], red[tid + w]);
            __syncthreads();
        }
        if (tid == 0) I.X[a] = norm_inf(red[0]);
        __syncthreads();
    }
}

// ---- the span step ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_span(Inst I, const EnergyTables* __restrict__ E,
                                              const int32_t* __restrict__ spec, int g,
                                              int ext_layer, int nblk_cells) {
    if ((int)blockIdx.x >= nblk_cells) {
        if (ext_layer >= 0) ext_column(I, E, ext_layer);
        return;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + wave, q = p + g;
    if (q > I.n) return;
    const int s = I.shift;
    const int a_lo = I.off[p], a_hi = I.off[p + 1], b_lo = I.off[q], b_hi = I.off[q + 1];
    unsigned long long visits = 0, appends = 0, feasible = 0;
    for (int b = b_lo; b < b_hi; b++) {
        const int committed = I.ccnt[b];  // entries of spans < g only (this wave owns C_b now)
        const int64_t cbase = I.coff[b];
        int added = 0;
        for (int a = a_lo; a < a_hi; a++) {
            const int64_t cell = I.rowoff[a] + (b - I.off[p + 1]);
            // phase 1: typed closed values and the scalar branch (eq. 2)
            int64_t Bv = kINF;
            for (int t = 0; t < 6; t++) {
                int64_t v = kINF;
                if (g >= 5) {
                    const int ea = a * 4 + kTX[t];
                    const int a1 = I.out_dst[ea];
                    if (a1 >= 0) {
                        const int64_t Ua = I.out_U[ea];
                        v = hairpin_lane(I, E, spec, a, b, t, a1, Ua, lane);
                        v = mn(v, twoloop_lane(I, E, a, b, t, a1, Ua, lane));
                        if (g >= 12) v = mn(v, multiloop_lane(I, E, a, b, t, a1, Ua, lane));
                        v = norm_inf(wave_min(v));
                    }
                }
                if (lane == 0) I.V[cell * 6 + t] = v;
                if (v < kINF) Bv = mn(Bv, v + fx(E->ml_intern + au_pen(E, t), s));
            }
            // phase 2: S2 (eq. 7), P_S, S1 and the strict retention test (eq. 6)
            int64_t s2 = kINF;
            const int ib0 = I.in_start[b], ib1 = I.in_start[b + 1];
            for (int eb = ib0 + lane; eb < ib1; eb += 64) {
                int bp = I.in_src[eb];
                if (I.layer[bp] > p) s2 = mn(s2, I.S2[cell_of(I, a, bp)] + I.in_U[eb] + I.mlbase_fx);
            }
            const int64_t arow = I.rowoff[a] - I.off[p + 1];
            for (int k = lane; k < committed; k += 64) {
                const int c = I.cc[cbase + k] & 0x7fffffff;
                s2 = mn(s2, I.S1[arow + c] + I.cB[cbase + k]);
            }
            s2 = norm_inf(wave_min(s2));
            int64_t ps = s2;
            if (lane < 4) {
                int ap = I.out_dst[a * 4 + lane];
                if (ap >= 0 && I.layer[ap] < q) ps = mn(ps, I.S1[cell_of(I, ap, b)] + I.out_U[a * 4 + lane] + I.mlbase_fx);
            }
            for (int eb = ib0 + lane; eb < ib1; eb += 64) {
                int bp = I.in_src[eb];
                if (I.layer[bp] > p) ps = mn(ps, I.S1[cell_of(I, a, bp)] + I.in_U[eb] + I.mlbase_fx);
            }
            ps = norm_inf(wave_min(ps));
            visits += (unsigned long long)committed;
            if (lane == 0) {
                I.Bt[cell] = Bv;
                I.S2[cell] = s2;
                I.S1[cell] = mn(Bv, ps);
            }
            const bool strict = Bv < ps;
            const bool keep = I.retain_all ? (Bv < kINF) : strict;
            feasible += Bv < kINF;
            if (keep) {
                const int slot = committed + added;
                if (slot < I.ccap[b]) {
                    if (lane == 0) {
                        I.cc[cbase + slot] = a | (strict ? 0 : (int)0x80000000);
                        I.cB[cbase + slot] = Bv;
                    }
                } else if (lane == 0) {
                    atomicMin((unsigned long long*)&I.stats[2], (unsigned long long)g);
                }
                added++;
                appends++;
            }
        }
        if (lane == 0 && added) I.ccnt[b] = min(committed + added, I.ccap[b]);
    }
    if (lane == 0) {
        if (visits) atomicAdd(&I.stats[0], visits);
        if (appends) {
            atomicAdd(&I.stats[1], appends);
            if (I.span_appends) atomicAdd(&I.span_appends[g], appends);
        }
        if (feasible) atomicAdd(&I.stats[3], feasible);
    }
}

__global__ void k_ext(Inst I, const EnergyTables* __restrict__ E, int L) { ext_column(I, E, L); }

__global__ void k_init(Inst I) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = tid; i < I.N; i += gridDim.x * blockDim.x) {
        I.ccnt[i] = 0;
        I.X[i] = (i == I.N - 1) ? 0 : kINF;
    }
    if (tid < 4) I.stats[tid] = tid == 2 ? ~0ull : 0ull;
    if (I.span_appends)
        for (int i = tid; i <= I.n; i += gridDim.x * blockDim.x) I.span_appends[i] = 0;
}

}  // namespace sd

// ---- host launch wrappers (C++ linkage, used by the library host code) --------------------------
namespace sd {

hipError_t upload_pair_order() {
    unsigned char l1[kNumPairs], l2[kNumPairs];
    int k = 0;
    for (int a = 0; a <= kMaxLoop; a++)
        for (int b = 0; a + b <= kMaxLoop; b++) {
            l1[k] = (unsigned char)a;
            l2[k] = (unsigned char)b;
            k++;
        }
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(kL1), l1, sizeof(l1));
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(kL2), l2, sizeof(l2));
}

hipError_t launch_init(const Inst& I, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3(64), dim3(256), 0, st, I);
    return hipGetLastError();
}

// one span step: cells of span g plus the external column of layer ext_layer (or -1)
hipError_t launch_span(const Inst& I, const EnergyTables* E, const int32_t* spec, int g,
                       int ext_layer, hipStream_t st) {
    const int layers = I.n - g + 1;
    const int nblk = layers > 0 ? (layers + 3) / 4 : 0;
    const int total = nblk + (ext_layer >= 0 ? 1 : 0);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_span, dim3(total), dim3(256), 0, st, I, E, spec, g, ext_layer, nblk);
    return hipGetLastError();
}

hipError_t launch_ext(const Inst& I, const EnergyTables* E, int L, hipStream_t st) {
    hipLaunchKernelGGL(k_ext, dim3(1), dim3(256), 0, st, I, E, L);
    return hipGetLastError();
}

}  // namespace sd
