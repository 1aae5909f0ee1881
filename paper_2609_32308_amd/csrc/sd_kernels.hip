// gfx950 kernels of the span wavefront (Sec. 5, Algorithm 1, re-designed for the GPU).
//
// One step per span length g.  A team owns one layer pair (p, q = p + g) and therefore every
// cell (a, b) with a in layer p and b in layer q: a workgroup of 4, 8 or 16 wavefronts, or one
// wavefront of a workgroup whose waves work on pairs of their own.  It is the only writer of the
// candidate segments C_b of its right endpoints in this step (the endpoint-ownership rule of
// Sec. 5), so appends need no atomics and land in start-state order.  Its waves split the
// (cell, type) jobs of the closed values into parts, and inside a part or a cell the lanes split
// the enumeration and the candidate-prefix scan of eq. (7), then reduce with wavefront min
// shuffles.  One extra team fills the external column one layer behind.
// Generic lattices (a forbidden-motif matcher intersected with the codon automaton) have their
// own span kernels in a section of their own below.
//
// Two-loop closure (stack / bulge / interior, l1 + l2 <= 30).  For a generic interior loop the
// energy is init(l1+l2) + asymmetry + mm[t][x_{i+1}][x_{j-1}] + mm[t'][x_{l+1}][x_{k-1}]: the
// outer mismatch couples only the two bases next to the closing pair and the inner mismatch only
// the two bases next to the inner pair.  When each unpaired segment crosses a codon boundary the
// trie's minimum segment cost splits the same way (first edge + rest of its codon, whole codons,
// last edge), so the whole term separates into
//     OUT(a1, b1, t)  [closing-pair side]  +  IN(c, d)  [inner-pair side]  +  layer constants.
// IN depends on the inner cell only, so its minimum over the states of a layer pair, LM, is
// stored once per layer pair (ring over the last 64 spans) when that pair is finished; a later
// cell then needs one lookup per (l1, l2) instead of an enumeration.  Every other (l1, l2)
// (bulges, 1xn, 1x1/1x2/2x2 tables, segments inside one codon) is enumerated explicitly.
#include <hip/hip_runtime.h>

#include <stddef.h>
#include <string.h>

#include <type_traits>

#include "sd_devutil.h"
#include "sd_internal.h"

namespace sd {

// (l1, l2) pairs in canonical order: l1 ascending, then l2 ascending, l1 + l2 <= 30
__constant__ unsigned char kL1[kNumPairs];
__constant__ unsigned char kL2[kNumPairs];
// Two-loop (l1, l2) pairs by category for each phase (p mod 3, q mod 3), each list sorted by
// l1 + l2 so that the pairs allowed at span g (l1 + l2 <= g - 7) form a prefix.  Entries:
// l1 | l2 << 5 | side << 10 (side 1: left side separable).  Counts: kCnt[list][phase][cap].
enum { kListBulge = 0, kListOne = 1, kListLab = 2, kListFast = 3, kListBulgeSep = 4 };
__constant__ unsigned short kPairList[5][9][kNumPairs];
__constant__ unsigned short kPairCnt[5][9][31];

// (l1, l2) handled by the separable layer-pair tables: both segments of length >= 2 crossing a
// codon boundary, generic or 2x3 interior class.
__device__ __forceinline__ bool fast_pair(int p, int q, int l1, int l2) {
    if (l1 < 2 || l2 < 2 || (l1 == 2 && l2 == 2)) return false;
    if ((q - 1 - l2) - (p + 1 + l1) < 5) return false;
    return (p + 2) / 3 != (p + l1) / 3 && (q - l2) / 3 != (q - 2) / 3;
}

// ---- hairpin closure ------------------------------------------------------------------------
template <class IT>
__device__ int64_t hairpin_lane(const IT& I, const SmallE& S, const int32_t* __restrict__ spec,
                                int a, int b, int t, int a1, int64_t Ua, int la, int g, int lane) {
    const int m = g - 2, s = I.shift;
    const int x = kTX[t], y = kTY[t];
    int64_t best = kINF;
    if (m == 3 || m == 4 || m == 6) {
        // each lane walks the paths whose bases at positions 1..3 spell its lane id in base 4
        const int l1 = (lane >> 4) & 3, l2 = (lane >> 2) & 3, l3 = lane & 3;
        int st = a1, key = x;
        int64_t cost = Ua;
        const int labs[3] = {l1, l2, l3};
        for (int i = 0; i < 3; i++) {
            const int e = st * 4 + labs[i], d = I.out_dst()[e];
            if (d < 0) return kINF;
            cost += I.out_U()[e];
            key = key * 4 + labs[i];
            st = d;
        }
        const int nfree = g - 5;  // 0, 1 or 3 free positions before the final base y
        const int combos = 1 << (2 * nfree);
        for (int k = 0; k < combos; k++) {
            int st2 = st, key2 = key, ok = 1, last = l3;
            int64_t c2 = cost;
            for (int i = nfree - 1; i >= 0; i--) {
                const int lab = (k >> (2 * i)) & 3, e = st2 * 4 + lab, d = I.out_dst()[e];
                if (d < 0) { ok = 0; break; }
                c2 += I.out_U()[e];
                key2 = key2 * 4 + lab;
                st2 = d;
                last = lab;
            }
            if (!ok) continue;
            const int e = st2 * 4 + y;
            if (I.out_dst()[e] != b) continue;
            c2 += I.out_U()[e];
            key2 = key2 * 4 + y;
            const int off = m == 3 ? kSpecOff5 : m == 4 ? kSpecOff6 : kSpecOff8;
            int32_t en = spec[off + key2];
            if (en == kNoSpecial) en = I.hp_init()[m] + (m == 3 ? au_pen(S, t) : S.mmH[t][l1][last]);
            best = mn(best, c2 + fx(en, s));
        }
        return best;
    }
    // generic size m >= 5: a -x-> a1 -x2-> a2 ~~> b2 -z-> b1 -y-> b.  a2 and b2 are >= 3 layers
    // apart, so the gap is tail(a2) + whole codons and the minimum separates into
    // alpha(a1, x2) + mmH[t][x2][z] + HB(b, y, z) plus layer constants.
    if (lane < 16) {
        const int x2 = lane >> 2, z = lane & 3;
        const int64_t al = I.alphaU()[a1 * 4 + x2], hb = I.hpB()[b * 16 + y * 4 + z];
        if (al < kINF && hb < kINF)
            best = Ua + al + hb + I.P()[(la + g - 2) / 3] - I.P()[(la + 2) / 3 + 1] +
                   fx(I.hp_init()[m] + S.mmH[t][x2][z], s);
    }
    return best;
}

// ---- two-loop closure: bulges and stacks ----------------------------------------------------------
// No boundary bases enter a bulge or stack energy, so each unpaired side costs its minimum
// (the gap).  The explicit pairs (stack, bulges of 1 and 2) are flattened over the lanes as
// (pair, inner left state, inner right state), counting only the states the inner layers hold;
// each lane evaluates the six inner types.
template <class IT>
__device__ __forceinline__ int64_t gap_l(const IT& I, int a, int la, int b, int lb) {  // gap() with known layers
    if (la == lb) return a == b ? 0 : kINF;
    const int ka = la / 3, kb = lb / 3;
    if (ka == kb) {
        if (la % 3 == 0) return 0;
        return (I.pfx()[b] >> 2) == I.pfx()[a] ? 0 : kINF;
    }
    return I.tail()[a] + I.P()[kb] - I.P()[ka + 1];
}

template <class IT>
__device__ int64_t bulge_lanes(const IT& I, const SmallE& S, int t, int a1, int b1, int64_t Uab, int p,
                               int q, int cap, int lane) {
    const int s = I.shift;
    // The explicit pairs (l1, l2) are (0,0), (0,1), (1,0), (0,2), (2,0), those with l1 + l2 <= cap.
    // One side of a bulge is empty, so after the stack each pair's items are the states of its one
    // inner layer: q-2, p+2, q-3, p+3.
    const int r1 = cap >= 1 ? I.off()[q - 2] : 0, nr1 = cap >= 1 ? I.off()[q - 1] - r1 : 0;
    const int l1s = cap >= 1 ? I.off()[p + 2] : 0, nl1 = cap >= 1 ? I.off()[p + 3] - l1s : 0;
    const int r2 = cap >= 2 ? I.off()[q - 3] : 0, nr2 = cap >= 2 ? r1 - r2 : 0;
    const int l2s = cap >= 2 ? I.off()[p + 3] : 0, nl2 = cap >= 2 ? I.off()[p + 4] - l2s : 0;
    const int tot = 1 + nr1 + nl1 + nr2 + nl2;
    int64_t best = kINF;
    for (int idx = lane; idx < tot; idx += 64) {
        int l1 = 0, l2 = 0, c = a1, d = b1, r = idx - 1;
        if (idx == 0) {
        } else if (r < nr1) {
            l2 = 1;
            d = r1 + r;
        } else if ((r -= nr1) < nl1) {
            l1 = 1;
            c = l1s + r;
        } else if ((r -= nl1) < nr2) {
            l2 = 2;
            d = r2 + r;
        } else {
            r -= nr2;
            l1 = 2;
            c = l2s + r;
        }
        const int cl = p + 1 + l1, dl = q - 1 - l2;
        const int64_t gl = l1 == 0 ? 0 : gap_l(I, a1, p + 1, c, cl);
        const int64_t gr = l2 == 0 ? 0 : gap_l(I, d, dl, b1, q - 1);
        if (gl >= kINF || gr >= kINF) continue;
        const int64_t* v = I.V() + (I.rowoff()[c] - I.off()[cl + 1] + d) * 6;
        const int l = l1 + l2;
#pragma unroll
        for (int tp = 0; tp < 6; tp++) {
            const int64_t vin = v[tp];
            const int32_t e2 = l == 0 ? S.stack[t][kRev[tp]] : bulge_e(S, t, kRev[tp], l);
            if (vin < kINF) best = mn(best, Uab + gl + vin + gr + fx(e2, s));
        }
    }
    return best;
}

// ---- two-loop closure: both segments explicit (each has 1..4 bases inside one codon) -------------
// Left segments are the label paths of l1 edges out of a1, right segments the paths of l2 edges
// into b1.  The (pair, left path, right path) combinations of all such pairs are flattened over
// the lanes: lane k < #pairs publishes its pair's combination count, a wave prefix sum gives
// the offsets, and every lane decodes its own combinations.  When nh waves share the list, the
// wave with index h takes the blocks of 64 combinations h, h + nh, ...
struct LabPair {
    int f0, nl, r0, nr, l1, l2, start;
};

template <class IT>
__device__ int64_t labelled_pairs(const IT& I, const SmallE& S, const EnergyTables* __restrict__ E,
                                  int t, int a1, int b1, int64_t Uab, int ph, int cap, int lane,
                                  LabPair* lp, int h, int nh) {
    const int s = I.shift;
    const int npairs = kPairCnt[kListLab][ph][cap];  // <= 16
    int cnt = 0;
    if (lane < npairs) {
        const int code = kPairList[kListLab][ph][lane], l1 = code & 31, l2 = (code >> 5) & 31;
        LabPair x;
        x.f0 = I.fwd_off()[a1 * 4 + l1 - 1];
        x.nl = I.fwd_off()[a1 * 4 + l1] - x.f0;
        x.r0 = I.bwd_off()[b1 * 4 + l2 - 1];
        x.nr = I.bwd_off()[b1 * 4 + l2] - x.r0;
        x.l1 = l1;
        x.l2 = l2;
        cnt = x.nl * x.nr;
        lp[lane] = x;
    }
    // inclusive prefix over lanes 0..15 (the first row) by DPP row shifts; a shifted-in lane
    // from outside the row reads 0
    int incl = cnt;
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xF, 0xF, false);  // row_shr:1
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xF, 0xF, false);  // row_shr:2
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xF, 0xF, false);  // row_shr:4
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xF, 0xF, false);  // row_shr:8
    if (lane < npairs) lp[lane].start = incl - cnt;
    const int total = __builtin_amdgcn_readlane(incl, 15);
    // pair starts on the scalar unit (a lane at or past npairs starts at total)
    int pst[16];
#pragma unroll
    for (int j = 1; j < 16; j++) pst[j] = __builtin_amdgcn_readlane(incl - cnt, j);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    int64_t best = kINF;
    for (int idx = lane + 64 * h; idx < total; idx += 64 * nh) {
        int k = 0;  // the last pair whose start is <= idx
#pragma unroll
        for (int j = 1; j < 16; j++) k += pst[j] <= idx;
        const LabPair x = lp[k];
        const int r = idx - x.start, i = r / x.nr, j = r - i * x.nr;
        const int fm = I.fwd_meta()[x.f0 + i], bm = I.bwd_meta()[x.r0 + j];
        const int c = fm >> 4, xi = (fm >> 2) & 3, xk = fm & 3;
        const int d = bm >> 4, xl = (bm >> 2) & 3, xj = bm & 3;
        const int64_t base = Uab + I.fwd_cost()[x.f0 + i] + I.bwd_cost()[x.r0 + j];
        const int64_t* v = I.V() + (I.fwd_crow()[x.f0 + i] + d) * 6;
        for (int tp = 0; tp < 6; tp++) {
            const int64_t vin = v[tp];
            if (vin >= kINF) continue;
            const int32_t e2 = interior_e(S, E, t, kRev[tp], x.l1, x.l2, xi, xk, xl, xj);
            best = mn(best, base + vin + fx(e2, s));
        }
    }
    __builtin_amdgcn_wave_barrier();
    return best;
}

// ---- one-sided separable two-loops --------------------------------------------------------------
// A side is separable when its segment has >= 2 bases and its two end edges lie in different
// codons (then its minimum cost is first-edge part + last-edge part + whole codons).  With the
// right side separable and the left side explicit (one edge, or both ends inside one codon):
//   value = U_ab + base + PR + left cost + OB_X(b1, t, x_{i+1}) + IDL_X(c, span, x_{k-1})
// and symmetrically with the left side separable:
//   value = U_ab + base + PL + right cost + OA_X(a1, t, x_{j-1}) + JDL_X(d, span, x_{l+1}).
__device__ __forceinline__ bool sep_left(int p, int l1) { return l1 >= 2 && (p + 2) / 3 != (p + l1) / 3; }
__device__ __forceinline__ bool sep_right(int q, int l2) { return l2 >= 2 && (q - l2) / 3 != (q - 2) / 3; }
// per-state rings [state][class][label][span mod 64]: a consumer walks consecutive spans
__device__ __forceinline__ int64_t ring_idx(int state, int span, int X, int lab) {
    return (((int64_t)state * 3 + X) * 4 + lab) * kLMRing + (span & (kLMRing - 1));
}
// per-layer-pair ring [left layer][class][span mod 64]
__device__ __forceinline__ int64_t lm_idx(int layer, int span, int X) {
    return ((int64_t)layer * 2 + X) * kLMRing + (span & (kLMRing - 1));
}
// ring of prepared both-separable minima [layer p][span mod 64][class]
__device__ __forceinline__ int64_t mini_idx(int p, int span, int X) {
    return ((int64_t)p * kLMRing + (span & (kLMRing - 1))) * 2 + X;
}
template <class IT>
__device__ __forceinline__ int64_t PLt(const IT& I, int p, int l1) { return I.P()[(p + l1) / 3] - I.P()[(p + 2) / 3 + 1]; }
template <class IT>
__device__ __forceinline__ int64_t PRt(const IT& I, int q, int l2) { return I.P()[(q - 2) / 3] - I.P()[(q - l2) / 3 + 1]; }

// Outer minima of one-sided loops come from per-state tables built with the automaton:
//   OB(b1, t)[X][x_{i+1}] = min_{x_{j-1}} beta(b1, x_{j-1}) + mm_X[t][x_{i+1}][x_{j-1}]
//   OA(a1, t)[X][x_{j-1}] = min_{x_{i+1}} alpha(a1, x_{i+1}) + mm_X[t][x_{i+1}][x_{j-1}]

// left segment explicit (paths of l1 edges out of a1), right segment separable
template <class IT>
__device__ int64_t rsep_pair(const IT& I, const SmallE& S, int a1, int64_t Uab, int l1, int l2,
                             int cl, int dl, int q, const int64_t* __restrict__ ob, int first, int step) {
    const int X = mm_class(l1, l2), g2 = dl - cl;
    const int64_t base = Uab + fx(interior_base(S, l1, l2), I.shift) + PRt(I, q, l2);
    const int f0 = I.fwd_off()[a1 * 4 + l1 - 1], f1 = I.fwd_off()[a1 * 4 + l1];
    int64_t best = kINF;
    for (int i = f0 + first; i < f1; i += step) {
        const int fm = I.fwd_meta()[i], c = fm >> 4, xi = (fm >> 2) & 3, xk = fm & 3;
        const int64_t o = ob[X * 4 + xi], idl = I.IDL()[ring_idx(c, g2, X, xk)];
        if (o < kINF && idl < kINF) best = mn(best, base + I.fwd_cost()[i] + o + idl);
    }
    return best;
}

// left segment separable, right segment explicit (paths of l2 edges into b1)
template <class IT>
__device__ int64_t lsep_pair(const IT& I, const SmallE& S, int b1, int64_t Uab, int l1, int l2,
                             int cl, int dl, int p, const int64_t* __restrict__ oa, int first, int step) {
    const int X = mm_class(l1, l2), g2 = dl - cl;
    const int64_t base = Uab + fx(interior_base(S, l1, l2), I.shift) + PLt(I, p, l1);
    const int r0 = I.bwd_off()[b1 * 4 + l2 - 1], r1 = I.bwd_off()[b1 * 4 + l2];
    int64_t best = kINF;
    for (int j = r0 + first; j < r1; j += step) {
        const int bm = I.bwd_meta()[j], d = bm >> 4, xl = (bm >> 2) & 3, xj = bm & 3;
        const int64_t o = oa[X * 4 + xj], jdl = I.JDL()[ring_idx(d, g2, X, xl)];
        if (o < kINF && jdl < kINF) best = mn(best, base + I.bwd_cost()[j] + o + jdl);
    }
    return best;
}

// ---- one-sided pairs through the per-state tables RS / LS ---------------------------------------
// The explicit side's short label paths are enumerated once; the separable side's length was
// minimised by the producer.  The 2x3 and 3x2 pairs (whose mismatch class differs from the rest
// of their row) are evaluated per pair.
__device__ __forceinline__ int64_t rs_idx(int state, int span, int l, int lab) {
    return ((int64_t)state * kLMRing + (span & (kLMRing - 1))) * 16 + (l - 1) * 4 + lab;
}

template <bool kSpread, class IT>
__device__ int64_t one_sided(const IT& I, const SmallE& S, int a1, int b1, int64_t Uab, int p, int q,
                             int cap, int lane, const int64_t* __restrict__ ob,
                             const int64_t* __restrict__ oa) {
    const int g = q - p;
    int start[9];
    int tot = 0;
    for (int l = 1; l <= 4; l++) {  // left explicit (right separable) path lists
        start[l - 1] = tot;
        const bool ok = !sep_left(p, l) && g - 2 - l >= 8;
        tot += ok ? I.fwd_off()[a1 * 4 + l] - I.fwd_off()[a1 * 4 + l - 1] : 0;
    }
    for (int l = 1; l <= 4; l++) {  // right explicit (left separable) path lists
        start[3 + l] = tot;
        const bool ok = !sep_right(q, l) && g - 2 - l >= 8;
        tot += ok ? I.bwd_off()[b1 * 4 + l] - I.bwd_off()[b1 * 4 + l - 1] : 0;
    }
    start[8] = tot;
    int64_t best = kINF;
    for (int idx = lane; idx < tot; idx += 64) {
        int k = 0;
        while (k < 7 && start[k + 1] <= idx) k++;
        const int i = idx - start[k];
        if (k < 4) {
            const int l1 = k + 1, X = l1 == 1 ? 2 : 0, e = I.fwd_off()[a1 * 4 + l1 - 1] + i;
            const int fm = I.fwd_meta()[e], c = fm >> 4, xi = (fm >> 2) & 3, xk = fm & 3;
            const int64_t rs = I.RS()[rs_idx(c, g - 2 - l1, l1, xk)], o = ob[X * 4 + xi];
            if (rs < kINF && o < kINF) best = mn(best, Uab + I.fwd_cost()[e] + o + rs);
        } else {
            const int l2 = k - 3, X = l2 == 1 ? 2 : 0, e = I.bwd_off()[b1 * 4 + l2 - 1] + i;
            const int bm = I.bwd_meta()[e], d = bm >> 4, xl = (bm >> 2) & 3, xj = bm & 3;
            const int64_t ls = I.LS()[rs_idx(d, g - 2 - l2, l2, xl)], o = oa[X * 4 + xj];
            if (ls < kINF && o < kINF) best = mn(best, Uab + I.bwd_cost()[e] + o + ls);
        }
    }
    // 2x3 with the left side explicit, 3x2 with the right side explicit: with kSpread one label
    // path of the explicit side per lane, else lane 0 (2x3) and lane 1 (3x2) walk them all (the
    // spread costs the 8- and 16-wave span kernels registers they do not have under their caps)
    if (kSpread) {
        if (cap >= 5 && !sep_left(p, 2) && sep_right(q, 3))
            best = mn(best, rsep_pair(I, S, a1, Uab, 2, 3, p + 3, q - 4, q, ob, lane, 64));
        if (cap >= 5 && sep_left(p, 3) && !sep_right(q, 2))
            best = mn(best, lsep_pair(I, S, b1, Uab, 3, 2, p + 4, q - 3, p, oa, lane, 64));
    } else {
        if (lane == 0 && cap >= 5 && !sep_left(p, 2) && sep_right(q, 3))
            best = mn(best, rsep_pair(I, S, a1, Uab, 2, 3, p + 3, q - 4, q, ob, 0, 1));
        if (lane == 1 && cap >= 5 && sep_left(p, 3) && !sep_right(q, 2))
            best = mn(best, lsep_pair(I, S, b1, Uab, 3, 2, p + 4, q - 3, p, oa, 0, 1));
    }
    return best;
}

// ---- the work of one layer pair (p, q) in span step g: one workgroup of several waves ----------
struct GroupCounters {
    unsigned long long visits, feasible;
};


// The threads that work on one layer pair: the whole workgroup (ordered by workgroup barriers),
// or a single wavefront of a workgroup whose waves each work on their own pair (ordered within the
// wave; a workgroup barrier there would pair up unrelated points of different waves).
struct BlockTeam {
    __device__ int tid() const { return threadIdx.x; }
    __device__ int lane() const { return threadIdx.x & 63; }
    __device__ int size() const { return blockDim.x; }
    __device__ void sync() const { __syncthreads(); }
};
struct WaveTeam {
    __device__ int tid() const { return threadIdx.x & 63; }
    // The lane index produced per call: a one-wave team runs inside the persistent loop, and lane
    // predicates derived from threadIdx would be hoisted to the kernel entry and held for the
    // whole launch, where they crowd the scalar registers and are spilled to vector lanes.
    __device__ int lane() const {
        int l;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
        return l;
    }
    __device__ int size() const { return 64; }
    __device__ void sync() const {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// A value every lane of the wave holds (read from one LDS address), moved to a scalar register so
// that the addresses and loop bounds derived from it stay scalar.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
    const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32)), lo = __builtin_amdgcn_readfirstlane((int)x);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int NW>  // waves per workgroup
struct GroupShared {
    int64_t vbuf[kMaxWidth * kMaxWidth][6];  // typed closed values of this layer pair's cells
    int64_t cellB[kMaxWidth * kMaxWidth];
    int keep[kMaxWidth * kMaxWidth];          // 0 none, 1 strict, 2 retained non-strict
    uint8_t combo[kMaxWidth * kMaxWidth * 6]; // (cell, type) jobs with an out-edge of label x
    int ncombo;
    int64_t red[NW][2];
    int64_t red2[NW][2];
    LabPair lab[NW][16];
    // the pair's automaton and segment metadata, read once per pair
    int adst[kMaxWidth][4];      // out-edge targets of the left states by label (-1 none)
    int64_t aU[kMaxWidth][4];    //   and their costs
    int bin[kMaxWidth + 1];      // in-edge range starts of the right states (and the end)
    int bcnt[kMaxWidth], bcap[kMaxWidth];
    int64_t boff[kMaxWidth];     // committed count, capacity and offset of each C_b
};

// Bulges of >= 3 bases through the in-edge b1 -> b: the unpaired side costs its gap (tail +
// whole codons), read from the BI / BJ rings.
template <class IT>
__device__ int64_t long_bulges(const IT& I, const SmallE& S, int t, int a1, int b1, int64_t Uab, int p,
                               int q, int cap, int lane) {
    const int s = I.shift;
    int64_t v = kINF;
    for (int k = lane; k < kPairCnt[kListBulgeSep][0][cap]; k += 64) {
        const int code = kPairList[kListBulgeSep][0][k], l1 = code & 31, l2 = (code >> 5) & 31;
        const int l = l1 + l2, cl = p + 1 + l1, dl = q - 1 - l2;
        int64_t w;
        if (l1 == 0) {
            const int64_t bi = I.BI()[(int64_t)a1 * kLMRing + ((dl - cl) & (kLMRing - 1))];
            w = bi >= kINF ? kINF : Uab + bi + I.P()[(q - 1) / 3] - I.P()[dl / 3 + 1];
        } else {
            const int64_t bj = I.BJ()[(int64_t)b1 * kLMRing + ((dl - cl) & (kLMRing - 1))];
            w = bj >= kINF ? kINF : Uab + bj + I.tail()[a1] + I.P()[cl / 3] - I.P()[(p + 1) / 3 + 1];
        }
        if (w < kINF) v = mn(v, w + fx(S.bulge[l] + au_pen(S, t), s));
    }
    return v;
}

// One part of the typed closed value V_t(a, b), with the lanes of one wave:
//   part 0: hairpin, stacks and bulges of 1-2 bases;
//   part 1: interior loops with a separable side (one-sided, both separable);
//   parts 2 .. nparts-1: interior loops with both sides explicit (labelled short paths), whose
//   flattened items are dealt to these parts in blocks of 64;
//   bulges of >= 3 bases and the multiloop closure: the last part when nparts >= 4, else part 0.
// Returns this lane's minimum.  The parts of one (cell, type) run on different waves and meet in
// an LDS minimum, or, in a one-wave group, run one after another into one wave reduction.
template <bool kSpread, class IT>
__device__ __forceinline__ int64_t closed_lanes(const IT& I, const SmallE& S, const EnergyTables* __restrict__ E,
                               const int32_t* __restrict__ spec, int a, int b, int t, int p, int q,
                               int part, int nparts, int64_t mini0, int64_t mini1, int lane, LabPair* lab,
                               int a1, int64_t Ua, int ib0, int ib1) {
    // a1 / Ua: the out-edge of a labelled x (type t's first base) and its cost; ib0 / ib1: b's
    // in-edge range
    const int g = q - p, s = I.shift;
    const int y = kTY[t];
    const int ph = (p % 3) * 3 + (q % 3), cap = min(g - 7, kMaxLoop);
    int64_t v = kINF;
    // bulges of >= 3 bases and the multiloop closure go with the last labelled part when the
    // labelled list is split, else with part 0
    const bool long_here = part == (nparts >= 4 ? nparts - 1 : 0);
    // multiloop closure (ML_closing + ML_intern + AU + S2 of the interior (a1, b1)) over the same
    // in-edges: b1 lies in layer q - 1 and a1 in layer p + 1, at least 10 layers apart from
    // g = 12 on; its S2 value is read before the in-edge's other loops so that it overlaps them
    const bool ml_here = long_here && g >= 12;
    const int64_t a1row = ml_here ? I.rowoff()[a1] - I.off()[p + 2] : 0;
    const int64_t mlc = fx(S.ml_closing + S.ml_intern + au_pen(S, t), s);
    if (part == 0) {
        v = hairpin_lane(I, S, spec, a, b, t, a1, Ua, p, g, lane);
        if (g >= 7) {
            for (int eb = ib0; eb < ib1; eb++) {
                if (I.in_lab()[eb] != y) continue;
                const int b1 = I.in_src()[eb];
                const int64_t Uab = Ua + I.in_U()[eb];
                const int64_t s2 = ml_here ? I.S2()[a1row + b1] : kINF;
                v = mn(v, bulge_lanes(I, S, t, a1, b1, Uab, p, q, cap, lane));
                if (long_here) v = mn(v, long_bulges(I, S, t, a1, b1, Uab, p, q, cap, lane));
                if (s2 < kINF) v = mn(v, s2 + Uab + mlc);
            }
        }
    } else if (part >= 2) {
        if (g >= 7) {
            for (int eb = ib0; eb < ib1; eb++) {
                if (I.in_lab()[eb] != y) continue;
                const int b1 = I.in_src()[eb];
                const int64_t Uab = Ua + I.in_U()[eb];
                const int64_t s2 = ml_here ? I.S2()[a1row + b1] : kINF;
                v = mn(v, labelled_pairs(I, S, E, t, a1, b1, Uab, ph, cap, lane, lab, part - 2, nparts - 2));
                if (long_here) v = mn(v, long_bulges(I, S, t, a1, b1, Uab, p, q, cap, lane));
                if (s2 < kINF) v = mn(v, s2 + Uab + mlc);
            }
        }
    } else {
        if (g >= 7) {
            const int64_t* oa = I.OA() + (int64_t)(a1 * 6 + t) * 12;
            for (int eb = ib0; eb < ib1; eb++) {
                if (I.in_lab()[eb] != y) continue;
                const int b1 = I.in_src()[eb];
                const int64_t Uab = Ua + I.in_U()[eb];
                v = mn(v, one_sided<kSpread>(I, S, a1, b1, Uab, p, q, cap, lane, I.OB() + (int64_t)(b1 * 6 + t) * 12, oa));
            }
        }
        if (g >= 12) {
            // both segments separable: OUT(a1, b1, t) + layer-pair minimum
            const int nbx = (ib1 - ib0) * 32;
            for (int k = lane; k < nbx; k += 64) {
                const int eb = ib0 + (k >> 5), X = (k >> 4) & 1, xi = (k >> 2) & 3, xj = k & 3;
                if (I.in_lab()[eb] != y) continue;
                const int64_t mini = X ? mini1 : mini0;
                const int64_t al = I.alphaU()[a1 * 4 + xi], be = I.betaU()[I.in_src()[eb] * 4 + xj];
                if (mini >= kINF || al >= kINF || be >= kINF) continue;
                v = mn(v, Ua + I.in_U()[eb] + al + be + fx(mmx(S, X, t, xi, xj), s) + mini);
            }
        }
    }
    return v;  // this lane's minimum
}

template <bool kSpread, class IT>
__device__ int64_t closed_part(const IT& I, const SmallE& S, const EnergyTables* __restrict__ E,
                               const int32_t* __restrict__ spec, int a, int b, int t, int p, int q,
                               int part, int nparts, int64_t mini0, int64_t mini1, int lane, LabPair* lab,
                               int a1, int64_t Ua, int ib0, int ib1) {
    return norm_inf(wave_min(closed_lanes<kSpread>(I, S, E, spec, a, b, t, p, q, part, nparts, mini0, mini1, lane,
                                                   lab, a1, Ua, ib0, ib1)));
}

// Per-state tables of span g for later two-loops, one state per wave (lanes as noted):
//   left state c (layer p):  RS(c, g), IDL(c, g), BI(c, g) and its LM contribution;
//   right state d (layer q): LS(d, g), JDL(d, g), BJ(d, g).
// RS / LS read IDL / JDL of spans <= g - 3 only; the rest reads this group's typed values.
template <int NW, class IT>
__device__ void produce_state(const IT& I, const SmallE& S, const GroupShared<NW>& G, int p, int g,
                              int k, int a_lo, int b_lo, int wa, int wb, int lane,
                              int64_t& lm0, int64_t& lm1) {
    const int s = I.shift;
    const bool left = k < wa;
    const int i = left ? k : k - wa, st = left ? a_lo + i : b_lo + i;
    // one-sided tables: lane = 4 * grp + lab covers separable lengths 3 + grp and 19 + grp;
    // outputs per explicit length 1..4, minimised over the 16 lane groups
    {
        const int lab = lane & 3, grp = lane >> 2;
        const int qc = p + g + 1, pc = p - 1;  // consumer closing layers (left / right state)
        int64_t o[4] = {kINF, kINF, kINF, kINF};
        // one separable length at a time in workgroup teams: unrolling keeps both lengths' ring
        // values and tails live at once, which made the 80-VGPR instantiation spill here; a
        // one-wave team (128 VGPRs) issues both lengths' loads together
#pragma unroll (NW == 1 ? 2 : 1)
        for (int h = 0; h < 2; h++) {
            const int ls = 3 + grp + 16 * h, g2 = g - ls;
            if (ls > 29 || g2 < 5) continue;
            if (left ? !sep_right(qc, ls) : (pc < 0 || !sep_left(pc, ls))) continue;
            const int64_t ptail = left ? PRt(I, qc, ls) : PLt(I, pc, ls);
            const int64_t in0 = left ? I.IDL()[ring_idx(st, g2, 0, lab)] : I.JDL()[ring_idx(st, g2, 0, lab)];
            const int64_t in2 = left ? I.IDL()[ring_idx(st, g2, 2, lab)] : I.JDL()[ring_idx(st, g2, 2, lab)];
#pragma unroll
            for (int le = 1; le <= 4; le++) {
                if (le + ls > kMaxLoop || (le == 2 && ls == 3)) continue;
                const int64_t in = le == 1 ? in2 : in0;
                if (in >= kINF) continue;
                const int32_t eb = left ? interior_base(S, le, ls) : interior_base(S, ls, le);
                o[le - 1] = mn(o[le - 1], in + fx(eb, s) + ptail);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            // over the lanes that share lane & 3: rotations by 4 and 8 within each row, then rows
            o[j] = mn(o[j], dpp64<kDppRor4>(o[j]));
            o[j] = mn(o[j], dpp64<kDppRor8>(o[j]));
            o[j] = mn(o[j], shfl_xor64(o[j], 16));
            o[j] = mn(o[j], shfl_xor64(o[j], 32));
        }
        if (grp == 0) {
            int64_t* T = left ? I.RS() : I.LS();
#pragma unroll
            for (int j = 0; j < 4; j++) T[rs_idx(st, g, j + 1, lab)] = norm_inf(o[j]);
        }
    }
    // inner minima: lane = 16 * X + 4 * xx + z (48 lanes), minimised over z
    {
        const int X = lane >> 4, xx = (lane >> 2) & 3, z = lane & 3;
        int64_t acc = kINF;
        if (X < 3) {
            const int nother = left ? wb : wa;
            for (int o = 0; o < nother; o++) {
                const int ci = left ? i * wb + o : o * wb + i;
                // left: vary x_{l+1} = z with alpha(d); right: vary x_{k-1} = z with beta(c)
                const int64_t w = left ? I.alphaU()[(b_lo + o) * 4 + z] : I.betaU()[(a_lo + o) * 4 + z];
                if (w >= kINF) continue;
                for (int tp = 0; tp < 6; tp++) {
                    const int64_t vin = G.vbuf[ci][tp];
                    if (vin < kINF)
                        acc = mn(acc, vin + w + fx(left ? mmx(S, X, kRev[tp], z, xx) : mmx(S, X, kRev[tp], xx, z), s));
                }
            }
        }
        acc = mn(acc, dpp64<kDppXor1>(acc));
        acc = mn(acc, dpp64<kDppXor2>(acc));
        acc = norm_inf(acc);
        if (X < 3 && z == 0) {
            if (left) {
                I.IDL()[ring_idx(st, g, X, xx)] = acc;
                const int64_t be = I.betaU()[st * 4 + xx];
                if (acc < kINF && be < kINF) {
                    if (X == 0) lm0 = mn(lm0, acc + be);
                    if (X == 1) lm1 = mn(lm1, acc + be);
                }
            } else {
                I.JDL()[ring_idx(st, g, X, xx)] = acc;
            }
        }
    }
    // bulge rings: lane = 6 * other + type (24 lanes)
    {
        const int o = lane / 6, tp = lane - 6 * o;
        int64_t acc = kINF;
        if (lane < 24 && o < (left ? wb : wa)) {
            const int64_t vin = G.vbuf[left ? i * wb + o : o * wb + i][tp];
            if (vin < kINF) acc = vin + (left ? I.tail()[b_lo + o] : 0) + fx(au_pen(S, tp), s);
        }
        acc = norm_inf(wave_min(acc));
        if (lane == 0) {
            if (left) I.BI()[(int64_t)st * kLMRing + (g & (kLMRing - 1))] = acc;
            else I.BJ()[(int64_t)st * kLMRing + (g & (kLMRing - 1))] = acc;
        }
    }
}

// The multiloop part of one cell (a, b) of layer pair (p, q) given its direct branch cost Bv
// (eq. 2), by one wave: S2 (eq. 7: in-edge extensions, then the committed prefix of C_b with
// the gathered S1(a, c)), P_S, S1 = min(B, P_S) and the retention test B < P_S (eq. 6).  Every
// scan reads only entries committed by earlier spans (their start states lie in layers after
// p, so the guard of eq. 7 holds for each).  Lane 0 writes B, S2 and S1 and returns the keep
// flag: 0 none, 1 strict, 2 retained non-strict (retain-all control).
template <class IT>
__device__ int multiloop_cell(const IT& I, int a, int b, int p, int q, int64_t cell, int64_t Bv, int lane,
                              GroupCounters& ctr, int committed, int64_t cbase, int ib0, int ib1,
                              const int* adst, const int64_t* aU) {
    // Every edge joins consecutive layers, so the in-edge sources of b lie in layer q - 1 and the
    // out-edge targets of a in layer p + 1: both are inner states of the pair exactly when g >= 2,
    // and their cells are found without reading their layers.  committed / cbase: C_b's count and
    // offset; ib0 / ib1: b's in-edge range; adst / aU: a's out-edge targets by label (-1 none)
    // and their costs.
    const int g = q - p;
    const int64_t arow = cell - b;  // cell(a, c) = arow + c for every c
    const int64_t* __restrict__ S1r = I.S1() + arow;
    const int64_t* __restrict__ S2r = I.S2() + arow;
    int64_t s2 = kINF;
    if (g >= 2)
        for (int eb = ib0 + lane; eb < ib1; eb += 64) s2 = mn(s2, S2r[I.in_src()[eb]] + I.in_U()[eb] + I.mlbase_fx);
    const int* __restrict__ cc = I.cc() + cbase;
    const int64_t* __restrict__ cB = I.cB() + cbase;
    // four entries per lane and round, their loads issued together: the gathers of S1(a, c)
    // depend on the start states, so one entry at a time would serialise two load latencies
    // per 64 entries
    int k = lane;
    for (; k + 192 < committed; k += 256) {
        const int c0 = cc[k] & 0x7fffffff, c1 = cc[k + 64] & 0x7fffffff;
        const int c2 = cc[k + 128] & 0x7fffffff, c3 = cc[k + 192] & 0x7fffffff;
        const int64_t b0 = cB[k], b1 = cB[k + 64], b2 = cB[k + 128], b3 = cB[k + 192];
        const int64_t s0 = S1r[c0], s1v = S1r[c1], s2v = S1r[c2], s3 = S1r[c3];
        s2 = mn(s2, mn(mn(s0 + b0, s1v + b1), mn(s2v + b2, s3 + b3)));
    }
    for (; k < committed; k += 64) s2 = mn(s2, S1r[cc[k] & 0x7fffffff] + cB[k]);
    s2 = norm_inf(wave_min(s2));
    int64_t ps = s2;
    if (g >= 2) {
        if (lane < 4) {
            const int ap = adst[lane];
            if (ap >= 0) ps = mn(ps, I.S1()[I.rowoff()[ap] + (b - I.off()[p + 2])] + aU[lane] + I.mlbase_fx);
        }
        for (int eb = ib0 + lane; eb < ib1; eb += 64) ps = mn(ps, S1r[I.in_src()[eb]] + I.in_U()[eb] + I.mlbase_fx);
    }
    ps = norm_inf(wave_min(ps));
    int keep = 0;
    if (lane == 0) {
        I.Bt()[cell] = Bv;
        I.S2()[cell] = s2;
        I.S1()[cell] = mn(Bv, ps);
        const bool strict = Bv < ps;
        keep = I.retain_all ? (Bv < kINF ? (strict ? 1 : 2) : 0) : (strict ? 1 : 0);
    }
    ctr.visits += (unsigned long long)committed;
    ctr.feasible += Bv < kINF;
    return keep;
}

// The same with the per-pair metadata read from the instance.
template <class IT>
__device__ int multiloop_cell(const IT& I, int a, int b, int p, int q, int64_t cell, int64_t Bv, int lane,
                              GroupCounters& ctr) {
    return multiloop_cell(I, a, b, p, q, cell, Bv, lane, ctr, I.ccnt()[b], I.coff()[b], I.in_start()[b],
                          I.in_start()[b + 1], I.out_dst() + a * 4, I.out_U() + a * 4);
}

// Appends the retained entries (a, B(a, b)) of layer pair (p, q) to the segments C_b in
// start-state order, one lane per right endpoint: the caller's workgroup owns these segments in
// step g (endpoint ownership), so no atomics are needed and the layout is deterministic.  An
// append beyond a segment's capacity records the earliest overflowing span instead.
template <class IT>
__device__ void append_candidates(const IT& I, int a_lo, int wa, int b_lo, int wb, const int* keep,
                                  const int64_t* cellB, int g, int lane, int committed, int cap,
                                  int64_t base) {
    // committed / cap / base: lane < wb's segment C_(b_lo + lane), count, capacity and offset
    int added = 0;
    if (lane < wb) {
        for (int ia = 0; ia < wa; ia++) {
            const int ci = ia * wb + lane;
            if (!keep[ci]) continue;
            const int slot = committed + added;
            if (slot < cap) {
                I.cc()[base + slot] = (a_lo + ia) | (keep[ci] == 1 ? 0 : (int)0x80000000);
                I.cB()[base + slot] = cellB[ci];
            } else {
                atomicMin(&I.stats()[2], (unsigned long long)g);
            }
            added++;
        }
        if (added) I.ccnt()[b_lo + lane] = min(committed + added, cap);
    }
}

// The same with the segments' counts, capacities and offsets read from the instance.
template <class IT>
__device__ void append_candidates(const IT& I, int a_lo, int wa, int b_lo, int wb, const int* keep,
                                  const int64_t* cellB, int g, int lane) {
    const bool mine = lane < wb;
    append_candidates(I, a_lo, wa, b_lo, wb, keep, cellB, g, lane, mine ? I.ccnt()[b_lo + lane] : 0,
                      mine ? I.ccap()[b_lo + lane] : 0, mine ? I.coff()[b_lo + lane] : 0);
}

template <int NW, class IT, class Team = BlockTeam>
__device__ GroupCounters span_group(const IT& I, const SmallE& S, const EnergyTables* __restrict__ E,
                                    const int32_t* __restrict__ spec, int p, int q, GroupShared<NW>& G,
                                    Team T = Team()) {
    const int g = q - p, s = I.shift;
    const int tid = T.tid(), wave = tid >> 6, lane = T.lane(), nw = T.size() >> 6;
    GroupCounters ctr{0, 0};
    const int a_lo = I.off()[p], a_hi = I.off()[p + 1], b_lo = I.off()[q], b_hi = I.off()[q + 1];
    const int wa = a_hi - a_lo, wb = b_hi - b_lo, ncell = wa * wb;
    // both-separable interior minima of this layer pair, per class (prepared one step ahead)
    int64_t mini0 = kINF, mini1 = kINF;
    if (g >= 12) {
        mini0 = I.MINI()[mini_idx(p, g, 0)];
        mini1 = I.MINI()[mini_idx(p, g, 1)];
    }
    // (cell, type) jobs: the type's first label leaves a and its last label enters b (any other
    // type is infeasible for the cell); typed values cleared.  Alongside, the pair's metadata is
    // read once: lanes 0-15 the out-edges of the left states, 16-20 the in-edge range starts of
    // the right states (and the end of the last), 32-35 their candidate segments.
    if (wave == 0) {
        if (lane < 4 * wa) {
            const int e = a_lo * 4 + lane;
            G.adst[lane >> 2][lane & 3] = I.out_dst()[e];
            G.aU[lane >> 2][lane & 3] = I.out_U()[e];
        } else if (lane >= 16 && lane <= 16 + wb) {
            G.bin[lane - 16] = I.in_start()[b_lo + lane - 16];
        } else if (lane >= 32 && lane < 32 + wb) {
            const int b = b_lo + lane - 32;
            G.bcnt[lane - 32] = I.ccnt()[b];
            G.bcap[lane - 32] = I.ccap()[b];
            G.boff[lane - 32] = I.coff()[b];
        }
        int base = 0;
        for (int k0 = 0; k0 < ncell * 6; k0 += 64) {
            const int k = k0 + lane;
            bool job = false;
            if (k < ncell * 6) {
                const int ci = k / 6, t = k - 6 * ci;
                G.vbuf[ci][t] = kINF;
                job = g >= 5 && I.out_dst()[(a_lo + ci / wb) * 4 + kTX[t]] >= 0 &&
                      ((I.inmask()[b_lo + ci % wb] >> kTY[t]) & 1);
            }
            const unsigned long long m = __ballot(job);
            if (job) G.combo[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint8_t)k;
            base += __popcll(m);
        }
        if (lane == 0) G.ncombo = base;
    }
    T.sync();
    // phase 1: typed closed values; the parts of every (cell, type) job on separate waves
    // labelled pairs over 1, 2 or 4 waves: wide workgroups run spans with few layer pairs
    constexpr int nparts = NW >= 16 ? 6 : NW >= 8 ? 4 : 3;
    if constexpr (NW == 1) {
        // one wave runs every part of a job: one reduction per job, and the value is stored
        // directly (each (cell, type) is one job)
        for (int j = 0; j < G.ncombo; j++) {
            const int cmb = G.combo[j], ci = cmb / 6, t = cmb - 6 * ci;
            const int ia = ci / wb, ib = ci - wb * ia, a = a_lo + ia, b = b_lo + ib;
            const int a1 = uni(G.adst[ia][kTX[t]]), i0 = uni(G.bin[ib]), i1 = uni(G.bin[ib + 1]);
            const int64_t Ua = uni(G.aU[ia][kTX[t]]);
            int64_t v = kINF;
#pragma unroll
            for (int part = 0; part < nparts; part++)
                v = mn(v, closed_lanes<true>(I, S, E, spec, a, b, t, p, q, part, nparts, mini0, mini1, lane,
                                             G.lab[wave], a1, Ua, i0, i1));
            v = norm_inf(wave_min(v));
            if (lane == 0) G.vbuf[ci][t] = v;
        }
    }
    const int njobs = NW == 1 ? 0 : nparts * G.ncombo;
    for (int k = wave; k < njobs; k += nw) {
        const int cmb = G.combo[k / nparts], ci = cmb / 6, t = cmb - 6 * ci;
        const int ia = ci / wb, ib = ci - wb * ia, a = a_lo + ia, b = b_lo + ib;
        const int64_t v = closed_part<(NW <= 4)>(I, S, E, spec, a, b, t, p, q, k % nparts, nparts, mini0, mini1, lane,
                                                  G.lab[wave], uni(G.adst[ia][kTX[t]]), uni(G.aU[ia][kTX[t]]),
                                                  uni(G.bin[ib]), uni(G.bin[ib + 1]));
        if (lane == 0 && v < kINF)
            __hip_atomic_fetch_min(&G.vbuf[ci][t], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    T.sync();
    // phase 2: branch value (eq. 2), S2 (eq. 7), P_S, S1 and the retention test (eq. 6); one
    // cell per wave from the first wave on.  Every scan reads only entries committed by earlier
    // spans.
    for (int ci = wave; ci < ncell; ci += nw) {
        const int ia = ci / wb, ib = ci - wb * ia, a = a_lo + ia, b = b_lo + ib;
        const int64_t cell = I.rowoff()[a] + (b - I.off()[p + 1]);
        int64_t Bv = kINF;
        for (int t = 0; t < 6; t++) {
            const int64_t v = G.vbuf[ci][t];
            if (lane == t) I.V()[cell * 6 + t] = v;
            if (v < kINF) Bv = mn(Bv, v + fx(S.ml_intern + au_pen(S, t), s));
        }
        const int keep = multiloop_cell(I, a, b, p, q, cell, Bv, lane, ctr, uni(G.bcnt[ib]), uni(G.boff[ib]),
                                        uni(G.bin[ib]), uni(G.bin[ib + 1]), G.adst[ia], G.aU[ia]);
        if (lane == 0) {
            G.keep[ci] = keep;
            G.cellB[ci] = Bv;
        }
    }
    // producers for later two-loops, one state per wave from the last wave down, so that they
    // overlap phase 2 (they read typed values and earlier spans only)
    int64_t lm0 = kINF, lm1 = kINF;
    if (g >= 5)
        for (int k = nw - 1 - wave; k < wa + wb; k += nw)
            produce_state(I, S, G, p, g, k, a_lo, b_lo, wa, wb, lane, lm0, lm1);
    lm0 = wave_min(lm0);
    lm1 = wave_min(lm1);
    if (lane == 0) {
        G.red[wave][0] = lm0;
        G.red[wave][1] = lm1;
    }
    T.sync();
    if (wave == 0) {
        // LM: layer-pair minimum of the both-separable form
        if (lane == 0 && g >= 5) {
            int64_t r0 = kINF, r1 = kINF;
            for (int w = 0; w < nw; w++) {
                r0 = mn(r0, G.red[w][0]);
                r1 = mn(r1, G.red[w][1]);
            }
            I.LM()[lm_idx(p, g, 0)] = norm_inf(r0);
            I.LM()[lm_idx(p, g, 1)] = norm_inf(r1);
        }
        // appends in start-state order, one lane per right endpoint (this group owns C_b in
        // this step)
        const bool mine = lane < wb;
        append_candidates(I, a_lo, wa, b_lo, wb, G.keep, G.cellB, g, lane, mine ? G.bcnt[lane] : 0,
                          mine ? G.bcap[lane] : 0, mine ? G.boff[lane] : (int64_t)0);
    }
    // both-separable minima of the next span's pair (p, q + 1), by the waves other than wave 0
    // (busy with the appends): they read LM of spans <= g - 7, complete before this step
    if (g + 1 >= 12 && q + 1 <= I.n) {
        const int w0 = nw > 1 ? 1 : 0;
        if (wave >= w0) {
            int64_t m0 = kINF, m1 = kINF;
            const int qn = q + 1, ph = (p % 3) * 3 + (qn % 3), cap = min(g + 1 - 7, kMaxLoop);
            for (int k = tid - 64 * w0; k < kPairCnt[kListFast][ph][cap]; k += T.size() - 64 * w0) {
                const int code = kPairList[kListFast][ph][k], l1 = code & 31, l2 = (code >> 5) & 31;
                const int cl = p + 1 + l1, dl = qn - 1 - l2, X = pair_class(l1, l2);
                const int64_t lm = I.LM()[lm_idx(cl, dl - cl, X)];
                if (lm >= kINF) continue;
                const int64_t v = lm + fx(interior_base(S, l1, l2), s) + PLt(I, p, l1) + PRt(I, qn, l2);
                if (X) m1 = mn(m1, v);
                else m0 = mn(m0, v);
            }
            m0 = wave_min(m0);
            m1 = wave_min(m1);
            if (lane == 0) {
                G.red2[wave][0] = m0;
                G.red2[wave][1] = m1;
            }
        }
        T.sync();
        if (tid == 64 * w0) {
            int64_t r0 = kINF, r1 = kINF;
            for (int w = w0; w < nw; w++) {
                r0 = mn(r0, G.red2[w][0]);
                r1 = mn(r1, G.red2[w][1]);
            }
            I.MINI()[mini_idx(p, g + 1, 0)] = norm_inf(r0);
            I.MINI()[mini_idx(p, g + 1, 1)] = norm_inf(r1);
        }
    }
    return ctr;
}

// ---- external column: X(a) for every a of layer L (one workgroup) ------------------------------
template <class IT, class Team = BlockTeam>
__device__ void ext_column(const IT& I, const SmallE& S, int L, int64_t* red, Team T = Team()) {
    const int tid = T.tid(), nt = T.size();
    for (int a = I.off()[L]; a < I.off()[L + 1]; a++) {
        int64_t v = kINF;
        if (tid < 4) {
            const int d = I.out_dst()[a * 4 + tid];
            if (d >= 0) v = I.out_U()[a * 4 + tid] + I.X()[d];
        }
        if (L + 5 <= I.n) {
            const int bstart = I.off()[L + 5];
            const int64_t base = I.rowoff()[a] - I.off()[L + 1];
            for (int bb = bstart + tid; bb < I.N; bb += nt) {
                const int64_t* vr = I.V() + (base + bb) * 6;
                const int64_t xb = I.X()[bb];
#pragma unroll
                for (int t = 0; t < 6; t++) {
                    const int64_t vt = vr[t];
                    if (vt < kINF) v = mn(v, vt + fx(au_pen(S, t), I.shift) + xb);
                }
            }
        }
        if constexpr (std::is_same<Team, WaveTeam>::value) {
            v = wave_min(v);
        } else {  // tree over the workgroup (the wave reduction costs the 512-thread span kernel a spill)
            red[tid] = v;
            T.sync();
            for (int w = nt / 2; w > 0; w >>= 1) {
                if (tid < w) red[tid] = mn(red[tid], red[tid + w]);
                T.sync();
            }
            v = red[0];
        }
        if (tid == 0) I.X()[a] = norm_inf(v);
        T.sync();
    }
}

template <class IT>
__device__ __forceinline__ void flush_counters(const IT& I, const GroupCounters& c, int p, int lane) {
    if (lane != 0) return;
    if (c.visits) atomicAdd(&I.visits()[p], c.visits);
    if (c.feasible) atomicAdd(&I.feasible()[p], c.feasible);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i on XCD i mod 8), each with
// its own L2.  Neighbouring layer pairs read each other's rows and rings, so every XCD gets one
// contiguous band of layer pairs: a bijection of [0, nb) that sends the workgroups of residue x
// to the x-th band.
__device__ __forceinline__ int xcd_band(int i, int nb) {
    const int x = i & 7, k = i >> 3;
    int base = 0;
    for (int r = 0; r < x; r++) base += (nb - r + 7) >> 3;
    return base + k;
}

// ---- the span step (plain mode): layer pair xcd_band(x) for block x < layer pairs ---------------
// The 512-thread instantiation is held to 80 VGPRs so that three of its workgroups fit a CU.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 512 ? 6 : 1)))
void k_span(Inst I, const EnergyTables* __restrict__ E, const int32_t* __restrict__ spec, int g,
            int ext_layer, int nblk_cells) {
    __shared__ SmallE S;
    __shared__ int64_t red[NT];
    __shared__ GroupShared<NT / 64> G;
    stage_tables(S, E);
    __syncthreads();
    if ((int)blockIdx.x >= nblk_cells) {
        if (ext_layer >= 0) ext_column(I, S, ext_layer, red);
        return;
    }
    const int p = xcd_band(blockIdx.x, nblk_cells), q = p + g;
    GroupCounters c = span_group(I, S, E, spec, p, q, G);
    // each wave counted its own cells
    const int lane = threadIdx.x & 63;
    flush_counters(I, c, p, lane);
}

// The span step with every wave on its own layer pair: four pairs per workgroup and one staging of
// the energy tables, for spans with many more layer pairs than the chip holds workgroups.  Items
// are the span's layer pairs, then the external column; workgroup x takes the four consecutive
// items of band xcd_band(x).  No workgroup barrier follows the staging: the waves' items are
// independent and some waves have none.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_span_waves(
    Inst I, const EnergyTables* __restrict__ E, const int32_t* __restrict__ spec, int g, int ext_layer, int npairs) {
    constexpr int NWV = NT / 64;
    __shared__ SmallE S;
    __shared__ GroupShared<1> G[NWV];
    stage_tables(S, E);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int items = npairs + (ext_layer >= 0 ? 1 : 0);
    const int nblk = (items + NWV - 1) / NWV;
    const int item = xcd_band(blockIdx.x, nblk) * NWV + wave;
    const WaveTeam T;
    if (item < npairs) {
        GroupCounters c = span_group(I, S, E, spec, item, item + g, G[wave], T);
        flush_counters(I, c, item, lane);
    } else if (item == npairs && ext_layer >= 0) {
        ext_column(I, S, ext_layer, nullptr, T);
    }
}

__global__ __launch_bounds__(256) void k_ext(Inst I, const EnergyTables* __restrict__ E, int L) {
    __shared__ SmallE S;
    __shared__ int64_t red[256];
    stage_tables(S, E);
    __syncthreads();
    ext_column(I, S, L, red);
}

__global__ void k_init(Inst I) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
    for (int i = tid; i < I.N; i += nt) {
        I.ccnt()[i] = 0;
        I.X()[i] = I.layer()[i] == I.n ? 0 : kINF;  // every state of the last layer is a sink
    }
    for (size_t i = tid; i < (size_t)(I.n + 1) * 2 * kLMRing; i += nt) I.LM()[i] = kINF;
    for (size_t i = tid; i < (size_t)I.N * kLMRing * 12; i += nt) {
        I.IDL()[i] = kINF;
        I.JDL()[i] = kINF;
    }
    for (size_t i = tid; i < (size_t)I.N * kLMRing; i += nt) {
        I.BI()[i] = kINF;
        I.BJ()[i] = kINF;
    }
    for (size_t i = tid; i < (size_t)I.N * kLMRing * 16; i += nt) {
        I.RS()[i] = kINF;
        I.LS()[i] = kINF;
    }
    if (tid < 4) I.stats()[tid] = tid == 2 ? ~0ull : 0ull;
    for (int i = tid; i <= I.n; i += nt) {
        I.visits()[i] = 0;
        I.feasible()[i] = 0;
    }
    if (I.gwin) {  // generic lattices: typed values are folded in with atomic minima
        for (int64_t i = tid; i < I.cells * 6; i += nt) I.V()[i] = kINF;
        for (int i = tid; i <= I.n; i += nt) I.gtickets()[i] = 0;
    }
}

// ---- the multiloop recurrences alone on an abstract layered DAG (test hook) -----------------------
// Direct branch costs B are given per cell (row layout, in the V array of the instance) instead of
// coming from loop energies; the unpaired-edge costs are the automaton's edge costs (ML_base 0).
// One wave per layer pair of span g runs the span step's own multiloop_cell and
// append_candidates: the exact-integer abstract test of Sec. 7.1 on the GPU code path.
__global__ __launch_bounds__(64) void k_ml_abstract(Inst I, int g) {
    __shared__ int keep[kMaxWidth * kMaxWidth];
    __shared__ int64_t cellB[kMaxWidth * kMaxWidth];
    const int p = blockIdx.x, q = p + g, lane = threadIdx.x;
    const int a_lo = I.off()[p], wa = I.off()[p + 1] - a_lo, b_lo = I.off()[q], wb = I.off()[q + 1] - b_lo;
    GroupCounters ctr{0, 0};
    for (int ci = 0; ci < wa * wb; ci++) {
        const int a = a_lo + ci / wb, b = b_lo + ci % wb;
        const int64_t cell = I.rowoff()[a] + (b - I.off()[p + 1]);
        const int64_t Bv = I.V()[cell];
        const int k = multiloop_cell(I, a, b, p, q, cell, Bv, lane, ctr);
        if (lane == 0) {
            keep[ci] = k;
            cellB[ci] = Bv;
        }
    }
    __syncthreads();
    append_candidates(I, a_lo, wa, b_lo, wb, keep, cellB, g, lane);
    flush_counters(I, ctr, p, lane);
}

// ---- span checksums (debug mode) -----------------------------------------------------------------
// An order-independent digest (wrapping sum of mixed (tag, index, value) words) of what a span
// step writes: the cells of span g (V, B, S1, S2), the committed candidate counts and entries,
// the visit and feasibility counters, the external column and the ring slots of span g.  With
// g = 0 it covers every cell and no ring slot (the whole tables of a finished design).  Two runs
// of a step that read the same inputs must give the same digest whatever their schedule.
__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ unsigned long long dword(int tag, int64_t idx, int64_t v) {
    return mix64((unsigned long long)v ^ mix64(((unsigned long long)idx << 4) | (unsigned)tag));
}

__global__ void k_checksum(Inst I, int g, unsigned long long* out) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (int64_t)gridDim.x * blockDim.x;
    unsigned long long h = 0;
    // cells: of span g (p = 0 .. n - g), or every cell
    const int plo = 0, phi = g > 0 ? I.n - g : I.n;
    for (int p = plo; p <= phi; p++) {
        const int q0 = g > 0 ? p + g : p + 1, q1 = g > 0 ? p + g : I.n;
        if (q0 > I.n) break;
        const int a0 = I.off()[p], a1 = I.off()[p + 1], b0 = I.off()[q0], b1 = I.off()[q1 + 1];
        const int64_t wb = b1 - b0, tot = (int64_t)(a1 - a0) * wb;
        for (int64_t k = tid; k < tot; k += nt) {
            const int a = a0 + (int)(k / wb), b = b0 + (int)(k % wb);
            const int64_t c = I.rowoff()[a] + (b - I.off()[p + 1]);
            for (int t = 0; t < 6; t++) h += dword(1 + t, c, I.V()[c * 6 + t]);
            h += dword(7, c, I.Bt()[c]) + dword(8, c, I.S1()[c]) + dword(9, c, I.S2()[c]);
        }
    }
    for (int64_t b = tid; b < I.N; b += nt) {
        const int cnt = I.ccnt()[b];
        h += dword(10, b, cnt) + dword(11, b, I.X()[b]);
        const int64_t base = I.coff()[b];
        for (int k = 0; k < cnt; k++) h += dword(12, base + k, I.cc()[base + k]) + dword(13, base + k, I.cB()[base + k]);
    }
    for (int64_t l = tid; l <= I.n; l += nt) h += dword(14, l, (int64_t)I.visits()[l]) + dword(15, l, (int64_t)I.feasible()[l]);
    if (g > 0) {
        const int r = g & (kLMRing - 1), r1 = (g + 1) & (kLMRing - 1);
        for (int64_t st = tid; st < I.N; st += nt) {
            for (int k = 0; k < 12; k++) {
                h += dword(16, st * 12 + k, I.IDL()[(st * 12 + k) * kLMRing + r]);
                h += dword(17, st * 12 + k, I.JDL()[(st * 12 + k) * kLMRing + r]);
            }
            for (int k = 0; k < 16; k++) {
                h += dword(18, st * 16 + k, I.RS()[(st * kLMRing + r) * 16 + k]);
                h += dword(19, st * 16 + k, I.LS()[(st * kLMRing + r) * 16 + k]);
            }
            h += dword(20, st, I.BI()[st * kLMRing + r]) + dword(21, st, I.BJ()[st * kLMRing + r]);
        }
        for (int64_t l = tid; l <= I.n; l += nt)
            for (int X = 0; X < 2; X++) {
                h += dword(22, l * 2 + X, I.LM()[(l * 2 + X) * kLMRing + r]);
                h += dword(23, l * 2 + X, I.MINI()[(l * kLMRing + r1) * 2 + X]);
            }
    }
    // wave sum, then one atomic per wave (wrapping, so the total is order independent)
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, h);
}

// ---- generic lattice: the codon automaton intersected with a forbidden-motif matcher --------------
// Nothing below relies on the codon trie.  Minimum path costs come from two tables that the span
// step fills for its own cells and that later spans read:
//   G(a, b)        minimum path cost a -> b (cell layout);
//   LG(u, v, x, y) minimum cost of a path u -> v whose first edge is labelled x and last edge y,
//                  for layer distances 1..30 (the unpaired segments of a two-loop).
// A generic interior loop couples its segments only through the four bases next to the two
// pairs (outer mismatch: x_{i+1}, x_{j-1}; inner mismatch: x_{l+1}, x_{k-1}), so for an inner
// cell (c, d) the minimum over those bases is a min-plus product over a 4-cycle: eliminate x_{j-1}
// with the right segment and the outer mismatch, x_{k-1} with the left segment and the inner
// mismatch, then take the minimum over (x_{i+1}, x_{l+1}).  Loops with both sides of <= 2 bases
// (the 1x1, 1x2, 2x2 tables) enumerate all boundary bases.
// per (cell, type): part 0 hairpin, stack, bulges, multiloop; part l1 = 1..29 the interior loops
// whose left segment has l1 bases (one ticket each, so that a span's work balances finely)
constexpr int kGenParts = 30;

template <class IT>
__device__ __forceinline__ int64_t gen_gap(const IT& I, int a, int la, int b, int lb) {
    if (la == lb) return a == b ? 0 : kINF;
    return I.Gt()[I.rowoff()[a] + (b - I.off()[la + 1])];
}
template <class IT>
__device__ __forceinline__ const int64_t* gen_lg(const IT& I, int u, int lu, int v) {
    return I.LG() + ((int64_t)u * I.gwin + (v - I.off()[lu + 1])) * 16;
}

struct GenShared {
    int64_t cellB[kGenMaxWidth * kGenMaxWidth];
    int keep[kGenMaxWidth * kGenMaxWidth];
};

// interior loop (l1, l2 >= 1) closed by type t around inner cell values vin[6], with the left
// and right segment tables L = LG(a1, c), R = LG(d, b1)
__device__ int64_t gen_interior(const SmallE& S, const EnergyTables* __restrict__ E, int t, int l1, int l2,
                                const int64_t* __restrict__ Lp, const int64_t* __restrict__ Rp,
                                const int64_t vin[6], int s) {
    int64_t best = kINF;
    if (l1 <= 2 && l2 <= 2) {
        for (int i = 0; i < 16; i++) {
            const int64_t li = Lp[i];
            if (li >= kINF) continue;
            for (int j = 0; j < 16; j++) {
                const int64_t rj = Rp[j];
                if (rj >= kINF) continue;
#pragma unroll
                for (int tp = 0; tp < 6; tp++) {
                    if (vin[tp] >= kINF) continue;
                    const int32_t e2 = interior_e(S, E, t, kRev[tp], l1, l2, i >> 2, i & 3, j >> 2, j & 3);
                    best = mn(best, li + rj + vin[tp] + fx(e2, s));
                }
            }
        }
        return best;
    }
    const int X = mm_class(l1, l2);
    // T2[xl][xi] = min over xj of R[xl][xj] + mm_X[t][xi][xj]
    int64_t T2[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int xl = k >> 2, xi = k & 3;
        int64_t acc = kINF;
#pragma unroll
        for (int xj = 0; xj < 4; xj++) {
            const int64_t r = Rp[xl * 4 + xj];
            if (r < kINF) acc = mn(acc, r + fx(mmx(S, X, t, xi, xj), s));
        }
        T2[k] = acc;
    }
    for (int tp = 0; tp < 6; tp++) {
        if (vin[tp] >= kINF) continue;
        const int tr = kRev[tp];
        for (int xi = 0; xi < 4; xi++)
            for (int xl = 0; xl < 4; xl++) {
                const int64_t t2 = T2[xl * 4 + xi];
                if (t2 >= kINF) continue;
                int64_t t1 = kINF;  // min over xk of L[xi][xk] + mm_X[tr][xl][xk]
#pragma unroll
                for (int xk = 0; xk < 4; xk++) {
                    const int64_t l = Lp[xi * 4 + xk];
                    if (l < kINF) t1 = mn(t1, l + fx(mmx(S, X, tr, xl, xk), s));
                }
                if (t1 < kINF) best = mn(best, t1 + t2 + vin[tp]);
            }
    }
    return best >= kINF ? kINF : best + fx(interior_base(S, l1, l2), s);
}

// Interior loop of mismatch class X with both segment tables known, when the left segment's
// part is pre-reduced: A[xk][xj] = min over xi of L[xi][xk] + mm_X[t][xi][xj] (per inner left
// state c).  Then min over (xk, xl) of [min over xj of A[xk][xj] + R[xl][xj]] + IN(xk, xl), with
// IN(xk, xl) = min over inner types of V + mm_X[reversed type][xl][xk].
__device__ __forceinline__ int64_t gen_interior_fast(const SmallE& S, int X, const int64_t A[16],
                                                     const int64_t* __restrict__ Rp, const int64_t vin[6],
                                                     int l1, int l2, int s) {
    int64_t R[16];
#pragma unroll
    for (int k = 0; k < 16; k++) R[k] = Rp[k];
    int64_t best = kINF;
#pragma unroll
    for (int xk = 0; xk < 4; xk++)
#pragma unroll
        for (int xl = 0; xl < 4; xl++) {
            int64_t out = kINF;
#pragma unroll
            for (int xj = 0; xj < 4; xj++) {
                const int64_t a = A[xk * 4 + xj], r = R[xl * 4 + xj];
                if (a < kINF && r < kINF) out = mn(out, a + r);
            }
            if (out >= kINF) continue;
            int64_t in = kINF;
#pragma unroll
            for (int tp = 0; tp < 6; tp++)
                if (vin[tp] < kINF) in = mn(in, vin[tp] + fx(mmx(S, X, kRev[tp], xl, xk), s));
            if (in < kINF) best = mn(best, out + in);
        }
    return best >= kINF ? kINF : best + fx(interior_base(S, l1, l2), s);
}

// One part of V_t(a, b) on a generic lattice, with the lanes of one wave (min over lanes).
template <class IT>
__device__ int64_t gen_closed_part(const IT& I, const SmallE& S, const EnergyTables* __restrict__ E,
                                   const int32_t* __restrict__ spec, int a, int b, int t, int p, int q,
                                   int part, int lane) {
    const int g = q - p, s = I.shift;
    const int a1 = I.out_dst()[a * 4 + kTX[t]];
    const int64_t Ua = I.out_U()[a * 4 + kTX[t]];
    const int y = kTY[t];
    const int ib0 = I.in_start()[b], ib1 = I.in_start()[b + 1];
    int64_t v = kINF;
    if (part == 0) {
        const int m = g - 2;
        if (m == 3 || m == 4 || m == 6) {
            v = hairpin_lane(I, S, spec, a, b, t, a1, Ua, p, g, lane);  // path enumeration only
        } else if (m >= 5) {
            // a -x-> a1 -x2-> a2 ~~> b2 -z-> b1 -y-> b: lanes over (x2, in-edge of b1)
            for (int eb = ib0; eb < ib1; eb++) {
                if (I.in_lab()[eb] != y) continue;
                const int b1 = I.in_src()[eb];
                const int j0 = I.in_start()[b1], nj = I.in_start()[b1 + 1] - j0;
                for (int k = lane; k < 4 * nj; k += 64) {
                    const int x2 = k & 3, j = j0 + (k >> 2);
                    const int a2 = I.out_dst()[a1 * 4 + x2];
                    if (a2 < 0) continue;
                    const int64_t gg = gen_gap(I, a2, p + 2, I.in_src()[j], q - 2);
                    if (gg >= kINF) continue;
                    v = mn(v, Ua + I.out_U()[a1 * 4 + x2] + gg + I.in_U()[j] + I.in_U()[eb] +
                                  fx(I.hp_init()[m] + S.mmH[t][x2][I.in_lab()[j]], s));
                }
            }
        }
        if (g >= 7) {
            // stack (item 0), left bulges (inner c of layer p+1+l, d = b1), right bulges (c = a1,
            // inner d of layer q-1-l); inner span >= 5 and l <= 30
            const int cl_hi = min(p + 31, q - 6), dl_lo = max(q - 31, p + 6);
            const int c0 = I.off()[p + 2], c1 = cl_hi >= p + 2 ? I.off()[cl_hi + 1] : c0;
            const int d1 = I.off()[q - 1], d0 = dl_lo <= q - 2 ? I.off()[dl_lo] : d1;
            const int nc = c1 - c0, nd = d1 - d0;
            for (int eb = ib0; eb < ib1; eb++) {
                if (I.in_lab()[eb] != y) continue;
                const int b1 = I.in_src()[eb];
                const int64_t Uab = Ua + I.in_U()[eb];
                for (int k = lane; k < 1 + nc + nd; k += 64) {
                    int c = a1, d = b1, lc = p + 1, l = 0;
                    int64_t gl = 0;
                    if (k >= 1 && k <= nc) {
                        c = c0 + k - 1;
                        lc = I.layer()[c];
                        l = lc - (p + 1);
                        gl = gen_gap(I, a1, p + 1, c, lc);
                    } else if (k > nc) {
                        d = d0 + k - 1 - nc;
                        const int ld = I.layer()[d];
                        l = (q - 1) - ld;
                        gl = gen_gap(I, d, ld, b1, q - 1);
                    }
                    if (gl >= kINF) continue;
                    const int64_t* vv = I.V() + (I.rowoff()[c] - I.off()[lc + 1] + d) * 6;
#pragma unroll
                    for (int tp = 0; tp < 6; tp++) {
                        const int64_t vin = vv[tp];
                        if (vin >= kINF) continue;
                        const int32_t e2 = l == 0 ? S.stack[t][kRev[tp]] : bulge_e(S, t, kRev[tp], l);
                        v = mn(v, Uab + gl + vin + fx(e2, s));
                    }
                }
            }
        }
        if (g >= 12) {
            // multiloop closure (ML_closing + ML_intern + AU) + S2 of the interior
            const int32_t mlc = S.ml_closing + S.ml_intern + au_pen(S, t);
            for (int eb = ib0 + lane; eb < ib1; eb += 64) {
                if (I.in_lab()[eb] != y) continue;
                const int b1 = I.in_src()[eb];
                if (I.layer()[b1] - (p + 1) < 10) continue;
                v = mn(v, I.S2()[cell_of(I, a1, b1)] + Ua + I.in_U()[eb] + fx(mlc, s));
            }
        }
    } else if (g >= 9) {
        // interior loops with l1 = part (29 parts cover every l1): the inner left state c runs
        // over the layer of l1, the lanes over every inner right state d with 1 <= l2 <= 30 - l1
        // and inner span >= 5 (one contiguous state range).  Pairs of the class that dominates
        // the row (1xn for l1 = 1, generic otherwise) take the pre-reduced form; 1x1/1x2/2x2,
        // 2x3 and 1xn with l1 > 1 the full one.
        for (int eb = ib0; eb < ib1; eb++) {
            if (I.in_lab()[eb] != y) continue;
            const int b1 = I.in_src()[eb];
            const int64_t Uab = Ua + I.in_U()[eb];
            for (int l1 = part; l1 <= kGenLoopWin - 1; l1 += kGenParts - 1) {
                const int lc = p + 1 + l1;
                const int dl_lo = max(q - 1 - (kGenLoopWin - l1), lc + 5), dl_hi = q - 2;
                if (dl_lo > dl_hi) break;
                const int d0 = I.off()[dl_lo], d1 = I.off()[dl_hi + 1];
                const int Xc = l1 == 1 ? 2 : 0;
                for (int c = I.off()[lc]; c < I.off()[lc + 1]; c++) {
                    const int64_t* lgl = gen_lg(I, a1, p + 1, c);
                    const int64_t crow = I.rowoff()[c] - I.off()[lc + 1];
                    int64_t A[16];
                    bool anyA = false;
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        const int xk = k >> 2, xj = k & 3;
                        int64_t acc = kINF;
#pragma unroll
                        for (int xi = 0; xi < 4; xi++) {
                            const int64_t l = lgl[xi * 4 + xk];
                            if (l < kINF) acc = mn(acc, l + fx(mmx(S, Xc, t, xi, xj), s));
                        }
                        A[k] = acc;
                        anyA = anyA || acc < kINF;
                    }
                    if (!anyA) continue;  // no path a1 -> c of l1 edges
                    for (int d = d0 + lane; d < d1; d += 64) {
                        const int64_t* vv = I.V() + (crow + d) * 6;
                        int64_t vin[6];
                        bool any = false;
#pragma unroll
                        for (int tp = 0; tp < 6; tp++) {
                            vin[tp] = vv[tp];
                            any = any || vin[tp] < kINF;
                        }
                        if (!any) continue;
                        const int ld = I.layer()[d], l2 = q - 1 - ld;
                        const int64_t* lgr = gen_lg(I, d, ld, b1);
                        const bool fast = !(l1 <= 2 && l2 <= 2) && mm_class(l1, l2) == Xc;
                        const int64_t w = fast ? gen_interior_fast(S, Xc, A, lgr, vin, l1, l2, s)
                                               : gen_interior(S, E, t, l1, l2, lgl, lgr, vin, s);
                        if (w < kINF) v = mn(v, Uab + w);
                    }
                }
            }
        }
    }
    return norm_inf(wave_min(v));
}

template <int NW, class IT>
__device__ GroupCounters gen_span_group(const IT& I, const SmallE& S, const EnergyTables* __restrict__ E,
                                        const int32_t* __restrict__ spec, int p, int q, GenShared& G) {
    const int g = q - p, s = I.shift;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, nw = blockDim.x >> 6;
    GroupCounters ctr{0, 0};
    const int a_lo = I.off()[p], a_hi = I.off()[p + 1], b_lo = I.off()[q], b_hi = I.off()[q + 1];
    const int wa = a_hi - a_lo, wb = b_hi - b_lo, ncell = wa * wb;
    // gap tables of this span's cells (only later spans read them)
    for (int ci = tid; ci < ncell; ci += blockDim.x) {
        const int a = a_lo + ci / wb, b = b_lo + ci % wb;
        int64_t gv = kINF;
        for (int eb = I.in_start()[b]; eb < I.in_start()[b + 1]; eb++) {
            const int bp = I.in_src()[eb];
            const int64_t gp = g == 1 ? (bp == a ? 0 : kINF) : I.Gt()[cell_of(I, a, bp)];
            if (gp < kINF) gv = mn(gv, gp + I.in_U()[eb]);
        }
        I.Gt()[cell_of(I, a, b)] = gv;
    }
    if (g <= kGenLoopWin) {
        for (int k = tid; k < ncell * 16; k += blockDim.x) {
            const int ci = k >> 4, x = (k >> 2) & 3, yy = k & 3;
            const int a = a_lo + ci / wb, b = b_lo + ci % wb;
            const int u1 = I.out_dst()[a * 4 + x];
            int64_t lv = kINF;
            if (u1 >= 0) {
                if (g == 1) {
                    if (u1 == b && x == yy) lv = I.out_U()[a * 4 + x];
                } else {
                    for (int eb = I.in_start()[b]; eb < I.in_start()[b + 1]; eb++) {
                        if (I.in_lab()[eb] != yy) continue;
                        const int v1 = I.in_src()[eb];
                        const int64_t gg = g == 2 ? (u1 == v1 ? 0 : kINF) : I.Gt()[cell_of(I, u1, v1)];
                        if (gg < kINF) lv = mn(lv, I.out_U()[a * 4 + x] + gg + I.in_U()[eb]);
                    }
                }
            }
            I.LG()[((int64_t)a * I.gwin + (b - I.off()[p + 1])) * 16 + x * 4 + yy] = lv;
        }
    }
    // typed values of this span were filled by k_gen_closed
    // branch value, S2 (eq. 7), P_S, S1 and the retention test, one cell per wave
    for (int ci = wave; ci < ncell; ci += nw) {
        const int a = a_lo + ci / wb, b = b_lo + ci % wb;
        const int64_t cell = I.rowoff()[a] + (b - I.off()[p + 1]);
        int64_t Bv = kINF;
        {
            const int64_t v = lane < 6 ? I.V()[cell * 6 + lane] : kINF;
            if (v < kINF) Bv = v + fx(S.ml_intern + au_pen(S, lane), s);
            Bv = wave_min(Bv);
        }
        const int keep = multiloop_cell(I, a, b, p, q, cell, Bv, lane, ctr);
        if (lane == 0) {
            G.keep[ci] = keep;
            G.cellB[ci] = Bv;
        }
    }
    __syncthreads();
    // appends in start-state order, one lane per right endpoint
    if (wave == 0) {
        append_candidates(I, a_lo, wa, b_lo, wb, G.keep, G.cellB, g, lane);
    }
    return ctr;
}

// typed closed values of span g on a generic lattice: every wave draws (job, part) tickets of the
// span's job list (host-built: cells and types that can close) and folds its part into V with an
// atomic minimum (V starts at infinity, set by k_init).  Occupancy is hinted to 3 waves per SIMD
// (168 VGPRs, a few spilled): 11 % faster on a 300-aa design than the unhinted 2 waves; 4 waves
// spill too much.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gen_closed(Inst I, const EnergyTables* __restrict__ E,
                                                    const int32_t* __restrict__ spec, int g) {
    __shared__ SmallE S;
    stage_tables(S, E);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t j0 = I.gjob_off()[g], total = (I.gjob_off()[g + 1] - j0) * kGenParts;
    for (;;) {
        unsigned k = 0;
        if (lane == 0) k = atomicAdd(&I.gtickets()[g], 1u);
        k = __shfl(k, 0, 64);
        if ((int64_t)k >= total) break;
        const int64_t j = j0 + k / kGenParts;
        const int a = I.gjobs()[2 * j], bt = I.gjobs()[2 * j + 1], b = bt >> 3, t = bt & 7;
        const int64_t v = gen_closed_part(I, S, E, spec, a, b, t, I.layer()[a], I.layer()[b], (int)(k % kGenParts), lane);
        if (lane == 0 && v < kINF)
            __hip_atomic_fetch_min(&I.V()[cell_of(I, a, b) * 6 + t], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// span step on a generic lattice: layer pair xcd_band(x) for block x < layer pairs, then the
// external column one layer behind
__global__ __launch_bounds__(256) void k_span_gen(Inst I, const EnergyTables* __restrict__ E,
                                                  const int32_t* __restrict__ spec, int g,
                                                  int ext_layer, int nblk_cells) {
    __shared__ SmallE S;
    __shared__ int64_t red[256];
    __shared__ GenShared G;
    stage_tables(S, E);
    __syncthreads();
    if ((int)blockIdx.x >= nblk_cells) {
        if (ext_layer >= 0) ext_column(I, S, ext_layer, red);
        return;
    }
    const int p = xcd_band(blockIdx.x, nblk_cells), q = p + g;
    GroupCounters c = gen_span_group<4>(I, S, E, spec, p, q, G);
    flush_counters(I, c, p, threadIdx.x & 63);
}

// ---- batched persistent kernel ------------------------------------------------------------------
// All instances advance one global span per grid barrier.  At step g the work items are the layer
// pairs of span g of every instance with n >= g, followed (per instance) by the external column
// of layer n - g + 1 (one layer behind).  The items of a step are cut into 8 contiguous bands, one
// per workgroup group (XCD); a group's workgroups draw its band's items from the group's ticket
// counter.  The barrier is two-level: the last arrival of a group counts the group at the top
// word, the last group bumps the generation (agent-scope release / acquire).
//
// Release: the cell values (S1, S2, B, V) and the candidate appends are stored by many waves,
// and a workgroup barrier alone does not wait for their stores (no vmcnt wait before
// s_barrier), while thread 0's agent-scope fence (L2 write-back, then its own vmcnt wait) only
// covers the stores that have reached this XCD's L2.  So every wave first waits until its own
// stores are acknowledged by L2 (vmcnt 0); after the workgroup barrier, thread 0's write-back
// then carries every wave's stores to memory before the arrival.  Without the per-wave wait a
// workgroup on another XCD could read a value of the previous span from memory before it was
// written back (a stale S1 makes P_S too large and the retention test then keeps extra
// non-strict candidates).  A full agent-scope fence in every wave is also correct but repeats
// the L2 write-back once per wave (8 s instead of 5 s for the 256-design batch).
__device__ __forceinline__ void wait_own_stores() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // keeps the compiler from sinking stores
    __builtin_amdgcn_s_waitcnt(0x0F70);                      // vmcnt(0), expcnt and lgkmcnt untouched
}

__device__ bool grid_barrier(BatchCtl* ctl, unsigned spin_cap, int* s_flag) {
    wait_own_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned grp = blockIdx.x & 7, ngrp = gridDim.x < 8 ? gridDim.x : 8;
        const unsigned members = (gridDim.x - grp + 7) >> 3;
        const unsigned g0 = __hip_atomic_load(&ctl->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int err = 0;
        bool last = false;
        const unsigned a = __hip_atomic_fetch_add(&ctl->arrive[grp].v, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (a == members) {
            __hip_atomic_store(&ctl->arrive[grp].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned t = __hip_atomic_fetch_add(&ctl->top.v, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
            if (t == ngrp) {
                __hip_atomic_store(&ctl->top.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&ctl->gen.v, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                last = true;
            }
        }
        if (!last) {
            // poll with relaxed loads: an acquire per poll would invalidate this XCD's caches
            // over and over under the feet of the workgroups still working; one acquire fence
            // follows the wait.  The pause between polls grows to about 1.7 us.
            unsigned spins = 0;
            int pause = 1;
            while (__hip_atomic_load(&ctl->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                if (__hip_atomic_load(&ctl->err.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || ++spins > spin_cap) {
                    __hip_atomic_store(&ctl->err.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    err = 1;
                    break;
                }
                for (int k = 0; k < pause; k++) __builtin_amdgcn_s_sleep(4);
                if (pause < 16) pause <<= 1;
            }
        }
        __threadfence();
        *s_flag = err;
    }
    __syncthreads();
    return *s_flag == 0;
}

// Work items per instance at its span g = g0 + step: the layer pairs of span g, then one external
// column (layer n - g + 1, one layer behind).  pref[i] is the exclusive prefix over instances and
// pref[ninst] the step's total; each thread takes a contiguous run of instances.  Ends with a
// workgroup barrier.
template <int NT>
__device__ void step_prefix(const Inst* __restrict__ insts, int ninst, int step, int* pref, int* wsum) {
    const int per = (ninst + NT - 1) / NT, lo = threadIdx.x * per, hi = min(lo + per, ninst);
    int sum = 0;
    for (int i = lo; i < hi; i++) {
        const int n = insts[i].n, g = insts[i].g0 + step;
        sum += (g <= n ? n - g + 1 : 0) + ((g >= 2 && g <= n + 1) ? 1 : 0);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int base_w = 0;
    for (int k = 0; k < w; k++) base_w += wsum[k];
    int acc = base_w + incl - sum;
    for (int i = lo; i < hi; i++) {
        pref[i] = acc;
        const int n = insts[i].n, g = insts[i].g0 + step;
        acc += (g <= n ? n - g + 1 : 0) + ((g >= 2 && g <= n + 1) ? 1 : 0);
    }
    if (threadIdx.x == NT - 1) {
        int tot = 0;
        for (int k = 0; k < NT / 64; k++) tot += wsum[k];
        pref[ninst] = tot;
    }
    __syncthreads();
}

// the last instance whose prefix is <= item
__device__ __forceinline__ int item_instance(const int* pref, int ninst, int item) {
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Persistent batched launch, the workgroup's waves sharing each work item (NT = 64: one wave).
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_persistent(
    const Inst* __restrict__ insts, int ninst, int nsteps, const EnergyTables* __restrict__ E,
    const int32_t* __restrict__ spec, BatchCtl* ctl, unsigned spin_cap) {
    __shared__ SmallE S;
    __shared__ int64_t red[NT];
    __shared__ GroupShared<NT / 64> G;
    __shared__ int pref[kMaxBatch + 1];
    __shared__ int wsum[NT / 64];
    __shared__ int s_flag;
    __shared__ unsigned s_ticket;
    stage_tables(S, E);
    // Work tickets of group grp number the items of its band of step 0, then of step 1, ...  A
    // workgroup that draws a ticket beyond the current step keeps it for the step it belongs to.
    const unsigned grp = blockIdx.x & 7, ngrp = gridDim.x < 8 ? gridDim.x : 8;
    if (threadIdx.x == 0) s_ticket = atomicAdd(&ctl->next[grp].v, 1u);
    __syncthreads();
    unsigned ticket = s_ticket, base = 0;
    for (int step = 0; step < nsteps; step++) {
        step_prefix<NT>(insts, ninst, step, pref, wsum);
        const unsigned total = (unsigned)pref[ninst];
        const unsigned lo_item = (unsigned)((uint64_t)total * grp / ngrp);
        const unsigned band = (unsigned)((uint64_t)total * (grp + 1) / ngrp) - lo_item;
        while (ticket < base + band) {
            // the next ticket is drawn by the last wave when the item starts (in four-wave
            // workgroups that wave rarely has a typed-value part) and published when it ends,
            // so the atomic's latency overlaps the item instead of following it
            const bool drawer = threadIdx.x == NT - 64;
            unsigned nxt = 0;
            if (drawer) nxt = atomicAdd(&ctl->next[grp].v, 1u);
            const int item = (int)(lo_item + (ticket - base));
            // the instance index is block-uniform
            const int inst = __builtin_amdgcn_readfirstlane(item_instance(pref, ninst, item));
            const Inst I = insts[inst];  // a few scalar registers: bases and sizes
            const int local = item - pref[inst], g = I.g0 + step;
            const int n = I.n, ncell_items = g <= n ? n - g + 1 : 0;
            if (local < ncell_items) {
                GroupCounters c = span_group(I, S, E, spec, local, local + g, G);
                flush_counters(I, c, local, threadIdx.x & 63);
            } else {
                ext_column(I, S, n - g + 1, red);
            }
            if (drawer) s_ticket = nxt;
            __syncthreads();  // the item is done and the next ticket is published
            ticket = s_ticket;
            __syncthreads();  // every thread has read it before the next item's drawer writes
        }
        base += band;
        if (!grid_barrier(ctl, spin_cap, &s_flag)) return;
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl->steps_done.v = step + 1;
    }
}

// Persistent batched launch, every wave of the workgroup on its own work items: the waves share
// the staged energy tables and the step's prefix, and each draws its own tickets and works on its
// own layer pair with wave-level ordering only.  Between a step's prefix and the grid barrier no
// workgroup barrier is executed, since the waves run different numbers of items.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_persistent_waves(
    const Inst* __restrict__ insts, int ninst, int nsteps, const EnergyTables* __restrict__ E,
    const int32_t* __restrict__ spec, BatchCtl* ctl, unsigned spin_cap) {
    __shared__ SmallE S;
    __shared__ GroupShared<1> G[NT / 64];
    __shared__ int pref[kMaxBatch + 1];
    __shared__ int wsum[NT / 64];
    __shared__ int s_flag;
    stage_tables(S, E);
    const unsigned grp = blockIdx.x & 7, ngrp = gridDim.x < 8 ? gridDim.x : 8;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WaveTeam T;
    unsigned ticket = 0, base = 0;
    if (lane == 0) ticket = atomicAdd(&ctl->next[grp].v, 1u);
    ticket = __builtin_amdgcn_readfirstlane(ticket);
    for (int step = 0; step < nsteps; step++) {
        step_prefix<NT>(insts, ninst, step, pref, wsum);
        const unsigned total = (unsigned)pref[ninst];
        const unsigned lo_item = (unsigned)((uint64_t)total * grp / ngrp);
        const unsigned band = (unsigned)((uint64_t)total * (grp + 1) / ngrp) - lo_item;
        while (ticket < base + band) {
            unsigned nxt = 0;
            if (lane == 0) nxt = atomicAdd(&ctl->next[grp].v, 1u);  // drawn now, used after the item
            const int item = (int)(lo_item + (ticket - base));
            const int inst = __builtin_amdgcn_readfirstlane(item_instance(pref, ninst, item));
            const Inst I = insts[inst];
            const int local = item - pref[inst], g = I.g0 + step;
            const int n = I.n, ncell_items = g <= n ? n - g + 1 : 0;
            if (local < ncell_items) {
                GroupCounters c = span_group(I, S, E, spec, local, local + g, G[wave], T);
                flush_counters(I, c, local, lane);
            } else {
                ext_column(I, S, n - g + 1, nullptr, T);
            }
            ticket = __builtin_amdgcn_readfirstlane(nxt);
        }
        base += band;
        if (!grid_barrier(ctl, spin_cap, &s_flag)) return;
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl->steps_done.v = step + 1;
    }
}

// Resets the barrier state and initialises every instance whose g0 is 1 (new instances).
__global__ void k_batch_init(const Inst* __restrict__ insts, int ninst, BatchCtl* ctl) {
    const Inst& I = insts[blockIdx.x];
    const int tid = threadIdx.x, nt = blockDim.x;
    if (blockIdx.x == 0 && tid < 8) {
        ctl->arrive[tid].v = 0;
        ctl->next[tid].v = 0;
        if (tid == 0) {
            ctl->top.v = 0;
            ctl->gen.v = 0;
            ctl->err.v = 0;
            ctl->steps_done.v = 0;
        }
    }
    if (I.g0 != 1) return;
    for (int i = tid; i < I.N; i += nt) {
        I.ccnt()[i] = 0;
        I.X()[i] = I.layer()[i] == I.n ? 0 : kINF;  // every state of the last layer is a sink
    }
    for (size_t i = tid; i < (size_t)(I.n + 1) * 2 * kLMRing; i += nt) I.LM()[i] = kINF;
    for (size_t i = tid; i < (size_t)I.N * kLMRing * 12; i += nt) {
        I.IDL()[i] = kINF;
        I.JDL()[i] = kINF;
    }
    for (size_t i = tid; i < (size_t)I.N * kLMRing; i += nt) {
        I.BI()[i] = kINF;
        I.BJ()[i] = kINF;
    }
    for (size_t i = tid; i < (size_t)I.N * kLMRing * 16; i += nt) {
        I.RS()[i] = kINF;
        I.LS()[i] = kINF;
    }
    if (tid < 4) I.stats()[tid] = tid == 2 ? ~0ull : 0ull;
    for (int i = tid; i <= I.n; i += nt) {
        I.visits()[i] = 0;
        I.feasible()[i] = 0;
    }
}

}  // namespace sd

// ---- host launch wrappers ----------------------------------------------------------------------
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
    e = hipMemcpyToSymbol(HIP_SYMBOL(kL2), l2, sizeof(l2));
    if (e != hipSuccess) return e;
    // categorised pair lists per phase (p mod 3, q mod 3)
    static unsigned short list[5][9][kNumPairs];
    static unsigned short cnt[5][9][31];
    memset(list, 0, sizeof(list));
    memset(cnt, 0, sizeof(cnt));
    for (int pm = 0; pm < 3; pm++)
        for (int qm = 0; qm < 3; qm++) {
            const int ph = pm * 3 + qm, p = 3 + pm, q = 300 + qm;  // representatives of the phases
            int len[5] = {0, 0, 0, 0, 0};
            for (int sum = 0; sum <= kMaxLoop; sum++) {
                for (int a = 0; a <= sum; a++) {
                    const int b = sum - a;
                    const bool sl = a >= 2 && (p + 2) / 3 != (p + a) / 3;
                    const bool sr = b >= 2 && (q - b) / 3 != (q - 2) / 3;
                    int lst;
                    unsigned short code = (unsigned short)(a | b << 5);
                    if ((a == 0 || b == 0) && a + b >= 3) lst = kListBulgeSep;
                    else if (a == 0 || b == 0) lst = kListBulge;  // (0,0) (0,1) (1,0) (0,2) (2,0), enumerated directly by bulge_lanes
                    else if (sl && sr) lst = kListFast;
                    else if (!sl && !sr) lst = kListLab;
                    else {
                        lst = kListOne;
                        if (sl) code |= 1 << 10;
                    }
                    list[lst][ph][len[lst]++] = code;
                }
                for (int l = 0; l < 5; l++) cnt[l][ph][sum] = (unsigned short)len[l];
            }
        }
    e = hipMemcpyToSymbol(HIP_SYMBOL(kPairList), list, sizeof(list));
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(kPairCnt), cnt, sizeof(cnt));
}

hipError_t launch_init(const Inst& I, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3(64), dim3(256), 0, st, I);
    return hipGetLastError();
}

// one span step: cells of span g plus the external column of layer ext_layer (or -1)
hipError_t launch_span(const Inst& I, const EnergyTables* E, const int32_t* spec, int g,
                       int ext_layer, int threads, int item_waves, hipStream_t st) {
    const int layers = I.n - g + 1;
    const int nblk = layers > 0 ? layers : 0;
    const int total = nblk + (ext_layer >= 0 ? 1 : 0);
    if (total == 0) return hipSuccess;
    if (item_waves == 1 && threads == 256) {  // every wave on its own pair, four per workgroup
        hipLaunchKernelGGL(k_span_waves<256>, dim3((total + 3) / 4), dim3(256), 0, st, I, E, spec, g, ext_layer, nblk);
        return hipGetLastError();
    }
    if (item_waves != threads / 64) return hipErrorInvalidValue;
    switch (threads) {
    case 64: hipLaunchKernelGGL(k_span<64>, dim3(total), dim3(64), 0, st, I, E, spec, g, ext_layer, nblk); break;
    case 256: hipLaunchKernelGGL(k_span<256>, dim3(total), dim3(256), 0, st, I, E, spec, g, ext_layer, nblk); break;
    case 512: hipLaunchKernelGGL(k_span<512>, dim3(total), dim3(512), 0, st, I, E, spec, g, ext_layer, nblk); break;
    case 1024: hipLaunchKernelGGL(k_span<1024>, dim3(total), dim3(1024), 0, st, I, E, spec, g, ext_layer, nblk); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// one span step on a generic lattice (same grid as launch_span)
hipError_t launch_span_gen(const Inst& I, const EnergyTables* E, const int32_t* spec, int g,
                           int ext_layer, int num_cu, hipStream_t st) {
    const int layers = I.n - g + 1;
    const int nblk = layers > 0 ? layers : 0;
    const int total = nblk + (ext_layer >= 0 ? 1 : 0);
    if (total == 0) return hipSuccess;
    if (g >= 5 && nblk > 0) {
        hipLaunchKernelGGL(k_gen_closed, dim3(4 * num_cu), dim3(256), 0, st, I, E, spec, g);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_span_gen, dim3(total), dim3(256), 0, st, I, E, spec, g, ext_layer, nblk);
    return hipGetLastError();
}

hipError_t launch_batch_init(const Inst* insts_dev, int ninst, BatchCtl* ctl, hipStream_t st) {
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_init, dim3(ninst), dim3(256), 0, st, insts_dev, ninst, ctl);
    return hipGetLastError();
}

// Schedule of the persistent launch: threads per workgroup and waves per work item.  64 threads:
// one wave per item; 256 or 512 threads with item_waves = threads / 64: the waves share each
// item; 256 threads with item_waves = 1: every wave on its own items.
bool persistent_schedule_valid(int threads, int item_waves) {
    return (threads == 64 && item_waves == 1) || (threads == 256 && (item_waves == 4 || item_waves == 1)) ||
           (threads == 512 && item_waves == 8);
}

hipError_t persistent_occupancy(int threads, int item_waves, int* blocks_per_cu) {
    if (!persistent_schedule_valid(threads, item_waves)) return hipErrorInvalidValue;
    if (threads == 64) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent<64>, 64, 0);
    if (threads == 512) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent<512>, 512, 0);
    if (item_waves == 1)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent_waves<256>, 256, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent<256>, 256, 0);
}

hipError_t launch_persistent(const Inst* insts_dev, int ninst, int nsteps, const EnergyTables* E,
                             const int32_t* spec, BatchCtl* ctl, int grid, int threads, int item_waves,
                             unsigned spin_cap, hipStream_t st) {
    if (!persistent_schedule_valid(threads, item_waves)) return hipErrorInvalidValue;
    if (threads == 64)
        hipLaunchKernelGGL(k_persistent<64>, dim3(grid), dim3(64), 0, st, insts_dev, ninst, nsteps, E, spec, ctl, spin_cap);
    else if (threads == 512)
        hipLaunchKernelGGL(k_persistent<512>, dim3(grid), dim3(512), 0, st, insts_dev, ninst, nsteps, E, spec, ctl, spin_cap);
    else if (item_waves == 1)
        hipLaunchKernelGGL(k_persistent_waves<256>, dim3(grid), dim3(256), 0, st, insts_dev, ninst, nsteps, E, spec,
                           ctl, spin_cap);
    else
        hipLaunchKernelGGL(k_persistent<256>, dim3(grid), dim3(256), 0, st, insts_dev, ninst, nsteps, E, spec, ctl, spin_cap);
    return hipGetLastError();
}

hipError_t launch_ml_abstract(const Inst& I, int g, hipStream_t st) {
    if (I.n - g + 1 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ml_abstract, dim3(I.n - g + 1), dim3(64), 0, st, I, g);
    return hipGetLastError();
}

hipError_t launch_checksum(const Inst& I, int g, unsigned long long* out, hipStream_t st) {
    hipError_t e = hipMemsetAsync(out, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_checksum, dim3(256), dim3(256), 0, st, I, g, out);
    return hipGetLastError();
}

hipError_t launch_ext(const Inst& I, const EnergyTables* E, int L, hipStream_t st) {
    hipLaunchKernelGGL(k_ext, dim3(1), dim3(256), 0, st, I, E, L);
    return hipGetLastError();
}

}  // namespace sd
