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
    // 16-bit copies of int21 / int22 (the parser requires entries in [-32768, 32767]) that the
    // kernels stage into LDS with 16-byte copies
    alignas(16) int16_t int21h[6][6][4][4][4];
    alignas(16) int16_t int22h[6][6][4][4][4][4];
};

// Special hairpin lookup: key = base-4 number of the loop sequence (closing pair included),
// value = listed total energy or kNoSpecial.
constexpr int32_t kNoSpecial = 0x7fffffff;
constexpr int kSpecOff5 = 0, kSpecOff6 = 1024, kSpecOff8 = 1024 + 4096, kSpecSize = 1024 + 4096 + 65536;

// A pending decision of the traceback: kind (external column, closed value, S1, S2, branch),
// the cell (a, b) and, for closed values, the pair type.
struct TFrame {
    int kind, a, b, t;
};

// Instance descriptor.  All arrays of one design live in two device regions whose layout is a
// function of a few sizes, so the descriptor holds two base pointers plus sizes and every array
// address is recomputed arithmetically where it is used (cheap scalar ALU, few live registers,
// also when the descriptor is read from memory by the batched kernel).
//
// Region A (inputs and small mutable state) is cut into units of U bytes, U >= 8 * (N + 2),
// >= 8 * (n + 2) and >= 8 * (A + 1), a multiple of 256; unit k starts at ra + k * U:
//   0 layer[N]  1 off[n+2]  2 in_start[N+1]  3 tail[N]  4 pfx[N]  5 P[A+1]  6 hp_init[n+1]
//   7 rowoff[N]  8 coff[N]  9 ccap[N]  10 ccnt[N]  11 X[N]  12-13 out_dst[4N]  14-17 out_U[4N]
//   18-21 alphaU[4N]  22-25 betaU[4N]  26-28 fwd_off[4N+1]  29-31 bwd_off[4N+1]
//   32-47 hpB[16N]  48-119 OB[72N]  120-191 OA[72N]  192 stats[4], trace results [8..11]
//   193 visits[n+1]  194 feasible[n+1]  195 inmask[N]  196 tr_seq[n]  197 tr_pair[n]
//   198-199 tr_stack[n+2] (16-byte frames)  200 cstrict[N]
//   201.. in_src[nE], in_lab[nE], in_U[nE], fwd_meta[nF], fwd_cost[nF], bwd_meta[nB],
//         bwd_cost[nB], fwd_crow[nF] (each start 8-byte aligned)
// Region B (DP tables) is cut into ring units of R = 512 * N bytes (N states x 64 spans x 8 B):
//   0-1 LM  2-13 IDL  14-25 JDL  26 BI  27 BJ  28-43 RS  44-59 LS  60-61 MINI, then from 62 R:
//   V[cells][6], Bt[cells], S1[cells], S2[cells], cc[slots], cB[slots], and for generic lattices
//   G[cells] (minimum path cost a -> b) and LG[state][gwin][4][4] (minimum cost of a path u -> v
//   of 1..30 edges with first label x and last label y; v indexed from the first state of the
//   layer after u's).
// Meaning of the arrays:
//   layer/off: layer of a state, first state of a layer; out_dst/out_U: out-edge by label
//   (-1 / cost); in_start/in_src/in_lab/in_U: in-edges (CSR, sorted by source and label);
//   inmask: bit y set if the state has an in-edge labelled y; tail: cheapest completion of the
//   current codon from a state; pfx: 2-base prefix code of a
//   phase-2 state (4x+y), base x of phase 1; P: prefix sums of per-codon minimum cost;
//   hp_init: hairpin initiation per size (extrapolated above 30); rowoff: cell row offsets,
//   cell(a,b) = rowoff[a] + b - off[layer(a)+1]; V/Bt/S1/S2: typed closed values, branch value,
//   multiloop prefixes; coff/ccap/ccnt/cc/cB: candidate segment per right endpoint (offset,
//   capacity, committed count, start states with the non-strict flag in bit 31, B values);
//   X: external column; stats: [2] earliest overflow span, [8..11] traceback results (energy,
//   path cost, status, X(s)); tr_seq / tr_pair: the traceback's base label per position and
//   pairing partner per position (-1 unpaired); tr_stack: its pending decisions; cstrict:
//   strict candidates per right endpoint (retain-all control only); visits / feasible:
//   candidate visits and cells with finite B, summed per left layer (one adder per layer pair
//   and step, so the counters see no contention).
//   alphaU[d*4+x] = U(d -x-> d2) + tail(d2); betaU[c*4+x] = min U over in-edges of c labelled x.
//   LM[layer][class 2][span]: layer-pair minima of the both-separable interior form.
//   MINI[layer p][span][class 2]: both-separable interior minimum of layer pair (p, p + span),
//   prepared one step ahead.
//   IDL/JDL[state][class 3][label 4][span]: inner minima per left / right inner state.
//   fwd_*/bwd_*: label paths of 1..4 edges out of / into a state (CSR by state*4+l-1);
//   meta = other_end << 4 | first_label << 2 | last_label, cost = sum of edge costs; fwd_crow =
//   the cell-row base of the path's end state c (cell(c, d) = fwd_crow + d).
//   hpB[b*16 + y*4 + z] = min over b2 -z-> b1 -y-> b of U(b2->b1) + U(b1->b).
//   OB/OA[state][t][X][label]: outer minima of one-sided interior loops.
//   BI[c][span] = min over d, t' of V_t'(c,d) + tail(d) + AU(t');  BJ[d][span] likewise without
//   the tail.  RS[c][span][l-1][label], LS[d][span][l-1][label]: one-sided loops minimised over
//   the separable side's length (explicit side of l <= 4 bases).
struct Inst {
    char *ra, *rb;         // region bases
    int64_t U;             // region-A unit in bytes
    int64_t nE, nF, nB;    // in-edges, forward and backward path entries
    int64_t cells, slots;  // DP cells, candidate slots
    int64_t mlbase_fx;     // ML_base * 2^s
    int64_t njobs;         // generic lattices: typed-value jobs over all spans
    int n, N, A, shift;
    int retain_all;
    int g0;  // persistent launches: first span this launch processes for the instance
    int gwin;  // generic lattices: states in the 30 layers after any layer (0 for the codon trie)
    int wmax;  // widest layer

    __host__ __device__ static int64_t al8(int64_t x) { return (x + 7) & ~(int64_t)7; }
    __host__ __device__ char* ua(int k) const { return ra + (int64_t)k * U; }
    __host__ __device__ int64_t R() const { return (int64_t)512 * N; }
    __host__ __device__ char* ub(int k) const { return rb + (int64_t)k * R(); }

    __host__ __device__ const int* layer() const { return (const int*)ua(0); }
    __host__ __device__ const int* off() const { return (const int*)ua(1); }
    __host__ __device__ const int* in_start() const { return (const int*)ua(2); }
    __host__ __device__ const int64_t* tail() const { return (const int64_t*)ua(3); }
    __host__ __device__ const int* pfx() const { return (const int*)ua(4); }
    __host__ __device__ const int64_t* P() const { return (const int64_t*)ua(5); }
    __host__ __device__ const int* hp_init() const { return (const int*)ua(6); }
    __host__ __device__ const int64_t* rowoff() const { return (const int64_t*)ua(7); }
    __host__ __device__ const int64_t* coff() const { return (const int64_t*)ua(8); }
    __host__ __device__ const int* ccap() const { return (const int*)ua(9); }
    __host__ __device__ int* ccnt() const { return (int*)ua(10); }
    __host__ __device__ int64_t* X() const { return (int64_t*)ua(11); }
    __host__ __device__ const int* out_dst() const { return (const int*)ua(12); }
    __host__ __device__ const int64_t* out_U() const { return (const int64_t*)ua(14); }
    __host__ __device__ const int64_t* alphaU() const { return (const int64_t*)ua(18); }
    __host__ __device__ const int64_t* betaU() const { return (const int64_t*)ua(22); }
    __host__ __device__ const int* fwd_off() const { return (const int*)ua(26); }
    __host__ __device__ const int* bwd_off() const { return (const int*)ua(29); }
    __host__ __device__ const int64_t* hpB() const { return (const int64_t*)ua(32); }
    __host__ __device__ const int64_t* OB() const { return (const int64_t*)ua(48); }
    __host__ __device__ const int64_t* OA() const { return (const int64_t*)ua(120); }
    __host__ __device__ unsigned long long* stats() const { return (unsigned long long*)ua(192); }
    __host__ __device__ unsigned long long* visits() const { return (unsigned long long*)ua(193); }
    __host__ __device__ unsigned long long* feasible() const { return (unsigned long long*)ua(194); }
    __host__ __device__ const int* inmask() const { return (const int*)ua(195); }
    __host__ __device__ int* tr_seq() const { return (int*)ua(196); }
    __host__ __device__ int* tr_pair() const { return (int*)ua(197); }
    __host__ __device__ TFrame* tr_stack() const { return (TFrame*)ua(198); }
    __host__ __device__ int* cstrict() const { return (int*)ua(200); }
    __host__ __device__ long long* tr_res() const { return (long long*)ua(192) + 8; }
    __host__ __device__ const int* in_src() const { return (const int*)ua(201); }
    __host__ __device__ const int* in_lab() const { return (const int*)(ua(201) + al8(4 * nE)); }
    __host__ __device__ const int64_t* in_U() const { return (const int64_t*)(ua(201) + 2 * al8(4 * nE)); }
    __host__ __device__ char* paths() const { return ua(201) + 2 * al8(4 * nE) + 8 * nE; }
    __host__ __device__ const int* fwd_meta() const { return (const int*)paths(); }
    __host__ __device__ const int64_t* fwd_cost() const { return (const int64_t*)(paths() + al8(4 * nF)); }
    __host__ __device__ const int* bwd_meta() const { return (const int*)(paths() + al8(4 * nF) + 8 * nF); }
    __host__ __device__ const int64_t* bwd_cost() const {
        return (const int64_t*)(paths() + al8(4 * nF) + 8 * nF + al8(4 * nB));
    }
    __host__ __device__ const int64_t* fwd_crow() const {
        return (const int64_t*)(paths() + al8(4 * nF) + 8 * nF + al8(4 * nB) + 8 * nB);
    }
    // generic lattices: per span g the typed-value jobs [gjob_off[g], gjob_off[g+1]) of gjobs
    // (pairs a, b * 8 + type), and one work-ticket counter per span
    __host__ __device__ int64_t* gjob_off() const {
        return (int64_t*)(paths() + al8(4 * nF) + 8 * nF + al8(4 * nB) + 8 * nB + 8 * nF);
    }
    __host__ __device__ int* gjobs() const { return (int*)(gjob_off() + (gwin ? n + 2 : 0)); }
    __host__ __device__ unsigned* gtickets() const { return (unsigned*)(gjobs() + 2 * njobs); }
    __host__ __device__ int64_t a_bytes() const {
        return (int64_t)((char*)gtickets() - ra) + (gwin ? al8(4 * ((int64_t)n + 1)) : 0);
    }

    __host__ __device__ int64_t* LM() const { return (int64_t*)ub(0); }
    __host__ __device__ int64_t* IDL() const { return (int64_t*)ub(2); }
    __host__ __device__ int64_t* JDL() const { return (int64_t*)ub(14); }
    __host__ __device__ int64_t* BI() const { return (int64_t*)ub(26); }
    __host__ __device__ int64_t* BJ() const { return (int64_t*)ub(27); }
    __host__ __device__ int64_t* RS() const { return (int64_t*)ub(28); }
    __host__ __device__ int64_t* LS() const { return (int64_t*)ub(44); }
    __host__ __device__ int64_t* MINI() const { return (int64_t*)ub(60); }
    __host__ __device__ int64_t* V() const { return (int64_t*)ub(62); }
    __host__ __device__ int64_t* Bt() const { return (int64_t*)(ub(62) + 48 * cells); }
    __host__ __device__ int64_t* S1() const { return (int64_t*)(ub(62) + 56 * cells); }
    __host__ __device__ int64_t* S2() const { return (int64_t*)(ub(62) + 64 * cells); }
    __host__ __device__ int* cc() const { return (int*)(ub(62) + 72 * cells); }
    __host__ __device__ int64_t* cB() const { return (int64_t*)(ub(62) + 72 * cells + al8(4 * slots)); }
    // generic lattices only: gap table G[cells] and labelled gap table LG[N][gwin][16]
    __host__ __device__ int64_t* Gt() const { return (int64_t*)(ub(62) + 72 * cells + al8(4 * slots) + 8 * slots); }
    __host__ __device__ int64_t* LG() const { return Gt() + cells; }
    __host__ __device__ int64_t b_bytes() const {
        return 62 * R() + 72 * cells + al8(4 * slots) + 8 * slots + (gwin ? 8 * cells + 128 * (int64_t)N * gwin : 0);
    }
};

constexpr int kLMRing = 64;
constexpr int kMaxWidth = 4;  // states per layer (the lattice build rejects wider layers)
constexpr int kGenMaxWidth = 16;  // states per layer of a generic (motif-constrained) lattice
constexpr int kGenLoopWin = 30;   // layer distances covered by the labelled gap table
constexpr int kMaxWaves = 16;  // waves per workgroup of the span-step kernels (1024 threads)
static_assert(sizeof(Inst) % 8 == 0, "instance descriptors are copied as 8-byte words");

// Batched persistent launch: barrier and work-ticket state shared by all workgroups.  Workgroup
// i belongs to group i mod 8 (the XCD it is dispatched to); every contended word sits on its own
// 128-byte line.
struct alignas(128) CtlWord {
    unsigned int v;
    unsigned int pad[31];
};
struct BatchCtl {
    CtlWord arrive[8];  // arrivals of each group at the current barrier
    CtlWord top;        // groups complete at the current barrier
    CtlWord gen;        // barrier generation
    CtlWord next[8];    // work tickets handed out per group (its band of every step, in order)
    CtlWord err;        // set when a barrier wait exceeds its spin limit (every group then exits)
    CtlWord steps_done; // spans completed (diagnostics)
};
constexpr int kMaxBatch = 1024;  // instances per persistent launch

}  // namespace sd
