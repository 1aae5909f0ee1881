// Device helpers shared by the span-step kernels and the traceback kernel: pair types, the loop
// tables staged in LDS, fixed-point and INF arithmetic, wavefront reductions over DPP moves, cell
// addressing and the codon trie's closed-form gap (Sec. 4.3), and the loop energies of the
// nearest-neighbour model (Sec. 3).
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include "sd_internal.h"

namespace sd {

static __constant__ int kTX[6] = {0, 1, 2, 2, 3, 3};  // 5' base of AU CG GC GU UA UG
static __constant__ int kTY[6] = {3, 2, 1, 3, 0, 2};  // 3' base
static __constant__ int kRev[6] = {4, 2, 1, 5, 0, 3}; // type of the reversed pair
static __constant__ int kPairType[16] = {-1, -1, -1, 0, -1, -1, 1, -1, -1, 2, -1, 3, 4, -1, 5, -1};

// Loop tables staged in LDS per workgroup (~27 KB; the 1x2 and 2x2 full-loop tables as 16-bit
// copies).
struct SmallE {
    alignas(16) int16_t int21[6][6][4][4][4];    // 1x2 loops (staged from the 16-bit copies)
    alignas(16) int16_t int22[6][6][4][4][4][4]; // 2x2 loops
    int32_t stack[6][6];
    int32_t mmH[6][4][4], mmI[6][4][4], mm1n[6][4][4], mm23[6][4][4];
    int32_t int11[6][6][4][4];
    int32_t hairpin[31], bulge[31], interior[31];
    int32_t ml_closing, ml_intern, ml_base, terminal_au, ninio, ninio_max;
};

__device__ inline void stage_tables(SmallE& S, const EnergyTables* __restrict__ E) {
    const int t = threadIdx.x, nt = blockDim.x;
    {
        static_assert(sizeof(S.int21) + sizeof(S.int22) == 23040, "int21 + int22 copies");
        static_assert(offsetof(EnergyTables, int22h) == offsetof(EnergyTables, int21h) + sizeof(S.int21),
                      "adjacent 16-bit tables");
        const uint4* src = reinterpret_cast<const uint4*>(&E->int21h[0][0][0][0][0]);
        uint4* dst = reinterpret_cast<uint4*>(&S.int21[0][0][0][0][0]);
        for (int i = t; i < 23040 / 16; i += nt) dst[i] = src[i];
    }
    for (int i = t; i < 36; i += nt) (&S.stack[0][0])[i] = (&E->stack[0][0])[i];
    for (int i = t; i < 96; i += nt) {
        (&S.mmH[0][0][0])[i] = (&E->mmH[0][0][0])[i];
        (&S.mmI[0][0][0])[i] = (&E->mmI[0][0][0])[i];
        (&S.mm1n[0][0][0])[i] = (&E->mm1n[0][0][0])[i];
        (&S.mm23[0][0][0])[i] = (&E->mm23[0][0][0])[i];
    }
    for (int i = t; i < 576; i += nt) (&S.int11[0][0][0][0])[i] = (&E->int11[0][0][0][0])[i];
    for (int i = t; i < 31; i += nt) {
        S.hairpin[i] = E->hairpin[i];
        S.bulge[i] = E->bulge[i];
        S.interior[i] = E->interior[i];
    }
    if (t == 0) {
        S.ml_closing = E->ml_closing;
        S.ml_intern = E->ml_intern;
        S.ml_base = E->ml_base;
        S.terminal_au = E->terminal_au;
        S.ninio = E->ninio;
        S.ninio_max = E->ninio_max;
    }
}

__device__ __forceinline__ int ptype(int x, int y) { return kPairType[x * 4 + y]; }
__device__ __forceinline__ int32_t au_pen(const SmallE& S, int t) {
    return (t == 1 || t == 2) ? 0 : S.terminal_au;
}
__device__ __forceinline__ int64_t mn(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t fx(int32_t e, int s) { return (int64_t)e * ((int64_t)1 << s); }
__device__ __forceinline__ int64_t norm_inf(int64_t v) { return v >= kHalfINF ? kINF : v; }

__device__ __forceinline__ int64_t shfl_xor64(int64_t v, int m) {
    int lo = __shfl_xor((int)(uint32_t)(uint64_t)v, m, 64);
    int hi = __shfl_xor((int)(uint32_t)((uint64_t)v >> 32), m, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
// DPP moves of a 64-bit value within rows of 16 lanes (no LDS traffic).  Callers run with every
// lane of the wave active.
template <int CTRL>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
    const int lo = (int)(uint32_t)(uint64_t)v, hi = (int)(uint32_t)((uint64_t)v >> 32);
    const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    return (int64_t)(((uint64_t)(uint32_t)h2 << 32) | (uint64_t)(uint32_t)l2);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E;               // quad_perm [1,0,3,2], [2,3,0,1]
constexpr int kDppHalfMirror = 0x141, kDppMirror = 0x140;     // lane i <-> 7-i, 15-i of its row
constexpr int kDppRor4 = 0x124, kDppRor8 = 0x128;             // rotate the row by 4, 8 lanes
__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
// minimum over the whole wave (every lane active): DPP within each row of 16 lanes, then the
// four row minima on the scalar unit
__device__ __forceinline__ int64_t wave_min(int64_t v) {
    v = mn(v, dpp64<kDppXor1>(v));
    v = mn(v, dpp64<kDppXor2>(v));
    v = mn(v, dpp64<kDppHalfMirror>(v));
    v = mn(v, dpp64<kDppMirror>(v));
    return mn(mn(readlane64(v, 0), readlane64(v, 16)), mn(readlane64(v, 32), readlane64(v, 48)));
}

template <class IT>
__device__ __forceinline__ int64_t cell_of(const IT& I, int a, int b) {
    return I.rowoff()[a] + (b - I.off()[I.layer()[a] + 1]);
}

// Minimum path cost between states of the codon trie (closed form; INF if unreachable).
template <class IT>
__device__ __forceinline__ int64_t gap(const IT& I, int a, int b) {
    int la = I.layer()[a], lb = I.layer()[b];
    if (la == lb) return a == b ? 0 : kINF;
    int ka = la / 3, kb = lb / 3;
    if (ka == kb) {
        if (la % 3 == 0) return 0;
        return (I.pfx()[b] >> 2) == I.pfx()[a] ? 0 : kINF;
    }
    return I.tail()[a] + I.P()[kb] - I.P()[ka + 1];
}

__device__ __forceinline__ int32_t bulge_e(const SmallE& S, int t, int tr, int l) {
    return l == 1 ? S.bulge[1] + S.stack[t][tr] : S.bulge[l] + au_pen(S, t) + au_pen(S, tr);
}

__device__ __forceinline__ int32_t interior_base(const SmallE& S, int l1, int l2) {
    int d = l1 > l2 ? l1 - l2 : l2 - l1;
    int32_t asym = S.ninio * d;
    return S.interior[l1 + l2] + (asym < S.ninio_max ? asym : S.ninio_max);
}

// interior loop with l1, l2 >= 1
__device__ inline int32_t interior_e(const SmallE& S, const EnergyTables* __restrict__ E, int t, int tr,
                              int l1, int l2, int xi1, int xk1, int xl1, int xj1) {
    if (l1 == 1 && l2 == 1) return S.int11[t][tr][xi1][xj1];
    if (l1 == 1 && l2 == 2) return S.int21[t][tr][xi1][xl1][xj1];
    if (l1 == 2 && l2 == 1) return S.int21[tr][t][xl1][xi1][xk1];
    if (l1 == 2 && l2 == 2) return S.int22[t][tr][xi1][xk1][xl1][xj1];
    int32_t e = interior_base(S, l1, l2);
    if (l1 == 1 || l2 == 1) return e + S.mm1n[t][xi1][xj1] + S.mm1n[tr][xl1][xk1];
    if (l1 + l2 == 5 && (l1 == 2 || l1 == 3)) return e + S.mm23[t][xi1][xj1] + S.mm23[tr][xl1][xk1];
    return e + S.mmI[t][xi1][xj1] + S.mmI[tr][xl1][xk1];
}

__device__ __forceinline__ int pair_class(int l1, int l2) {  // 1: 2x3 mismatch table, 0: generic
    return (l1 + l2 == 5 && (l1 == 2 || l1 == 3)) ? 1 : 0;
}
// mismatch class of an interior loop: 0 generic, 1 2x3, 2 1xn
__device__ __forceinline__ int mm_class(int l1, int l2) {
    return (l1 == 1 || l2 == 1) ? 2 : pair_class(l1, l2);
}
__device__ __forceinline__ int32_t mmx(const SmallE& S, int X, int t, int i, int j) {
    return X == 0 ? S.mmI[t][i][j] : X == 1 ? S.mm23[t][i][j] : S.mm1n[t][i][j];
}

}  // namespace sd
