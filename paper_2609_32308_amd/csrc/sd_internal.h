// Internal layout shared by the host side of the library and its gfx950 kernels.
//
// Device data of one design instance (all int64 values are fixed point: energy * 2^s plus
// rounded codon costs; kINF = 2^62 marks infeasible):
//   automaton   layer[N], off[n+2] (first state of each layer), out_dst/out_U[N*4] (edge by
//               label, DFA so at most one per label), in-edge CSR sorted by (source, label).
//   gap         closed form for the codon trie: G(a,b) = tail(a) + P[k(b)] - P[k(a)+1] across
//               codons, 0 / unreachable inside one codon (prefix test on pfx).
//   cells       row layout over state pairs: cell(a,b) = rowoff[a] + b - off[layer(a)+1], i.e.
//               row a holds every b of a later layer, contiguous in state order.  Per cell:
//               V[6] (typed closed values), B (branch), S1, S2 (multiloop fragments).
//   candidates  per right endpoint b a packed segment [coff[b], coff[b]+ccap[b]) of
//               (cc = start state, cB = B(c,b)); ccnt[b] entries committed so far, appended in
//               span order (each span's entries in start-state order).
#pragma once
#include <stdint.h>

namespace sd {

constexpr int64_t kINF = int64_t(1) << 62;
constexpr int64_t kHalfINF = int64_t(1) << 61;  // anything above is infeasible
constexpr int kMaxLoop = 30;                    // bulge / interior unpaired cap (Sec. 3)
constexpr int kNumPairs = 496;                  // (l1,l2) with l1 + l2 <= 30

// Energy tables in 0.01 kcal/mol; two-loop tables index the inner pair from inside the loop.
struct EnergyTables {
    int32_t stack[6][6];
    int32_t mmH[6][4][4], mmI[6][4][4], mm1n[6][4][4], mm23[6][4][4];
    int32_t int11[6][6][4][4];
    int32_t int21[6][6][4][4][4];
    int32_t int22[6][6][4][4][4][4];
    int32_t hairpin[31], bulge[31], interior[31];
    int32_t ml_closing, ml_intern, ml_base, terminal_au, ninio, ninio_max;
    int32_t pad[2];
};

// Special hairpin lookup: key = base-4 number of the loop sequence (closing pair included),
// value = listed total energy or kNoSpecial.
constexpr int32_t kNoSpecial = 0x7fffffff;
constexpr int kSpecOff5 = 0, kSpecOff6 = 1024, kSpecOff8 = 1024 + 4096, kSpecSize = 1024 + 4096 + 65536;

struct Inst {
    int n, N, A, shift;
    int64_t mlbase_fx;  // ML_base * 2^s
    const int *layer, *off;
    const int *out_dst;
    const int64_t *out_U;
    const int *in_start, *in_src, *in_lab;
    const int64_t *in_U;
    const int64_t *tail;  // cheapest completion of the current codon from a state
    const int *pfx;       // 2-base prefix code of a phase-2 state (4x+y), base x of phase 1
    const int64_t *P;     // prefix sums of per-codon minimum cost, A+1 entries
    const int *hp_init;   // hairpin initiation per size m (extrapolated above 30), n+1 entries
    const int64_t *rowoff;
    int64_t *V, *Bt, *S1, *S2;
    const int64_t *coff;
    const int *ccap;
    int *ccnt;
    int *cc;
    int64_t *cB;
    int64_t *X;
    unsigned long long *stats;  // [0] visits [1] appends [2] overflow flag [3] feasible B
    unsigned long long *span_appends;  // per span appended candidates (n+1), may be null
    // separable interior-loop data (see the two-loop notes in sd_kernels.hip)
    const int64_t *alphaU;  // [N*4] U(d -x-> d2) + tail(d2), INF if no edge
    const int64_t *betaU;   // [N*4] min U over in-edges of c labelled x, INF if none
    int64_t *LM;            // [kLMRing][n+1][2] per layer-pair inner minima, ring over spans
    int64_t *IDL;           // [N][kLMRing][3][4] inner minima per left inner state, class, x_{k-1}
    int64_t *JDL;           // [N][kLMRing][3][4] inner minima per right inner state, class, x_{l+1}
    // label paths of 1..4 edges: forward from a state / backward into a state (CSR by state*4+l-1)
    // meta = other_end << 4 | first_label << 2 | last_label, cost = sum of edge costs
    const int *fwd_off, *fwd_meta, *bwd_off, *bwd_meta;
    const int64_t *fwd_cost, *bwd_cost;
    // generic hairpins: HB[b*16 + y*4 + z] = min over b2 -z-> b1 -y-> b of U(b2->b1) + U(b1->b)
    const int64_t *hpB;
    const int64_t *OB, *OA;  // [state][t][X][label] outer minima of one-sided interior loops
    // bulges of >= 3 bases, per state and span (span innermost):
    //   BI[c][g] = min over d at layer(c)+g, type t' of V_t'(c,d) + tail(d) + AU(t')
    //   BJ[d][g] = min over c at layer(d)-g, type t' of V_t'(c,d) + AU(t')
    int64_t *BI, *BJ;
    // one-sided interior loops, minimised over the separable side's length, per state and span:
    //   RS[c][s][l1-1][x_{k-1}]: explicit left segment of l1 <= 4 bases ending in c, right side
    //                            separable, s = layer(b1) - layer(c)
    //   LS[d][s][l2-1][x_{l+1}]: explicit right segment of l2 <= 4 bases starting at d, left side
    //                            separable, s = layer(d) - layer(a1)
    int64_t *RS, *LS;
    int retain_all;
    int g0;  // persistent launches: first span this launch processes for the instance
};

constexpr int kLMRing = 64;
constexpr int kMaxWaves = 16;  // waves per workgroup of the span-step kernels (1024 threads)  // > 32 spans of two-loop reach
static_assert(sizeof(Inst) % 8 == 0, "instance descriptors are copied as 8-byte words");

// Batched persistent launch: barrier state shared by all workgroups.
struct BatchCtl {
    unsigned int count;  // arrivals at the current barrier
    unsigned int gen;    // barrier generation
    int err;             // set when a barrier wait exceeds its spin limit (every group then exits)
    int steps_done;      // spans completed (diagnostics)
};
constexpr int kMaxBatch = 1024;  // instances per persistent launch

}  // namespace sd
