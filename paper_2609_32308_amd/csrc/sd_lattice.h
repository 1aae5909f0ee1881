// Host-side lattice model of one design: the codon trie automaton, fixed-point costs, the
// closed-form gap data, the row layout of the cell tables and the candidate segments.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "sd_internal.h"

namespace sd {

struct Params {
    EnergyTables E;
    double lxc = 0.0;
    std::vector<std::string> special[3];  // triloop, tetraloop, hexaloop sequences
    std::vector<int32_t> special_e[3];
    int32_t maxabs = 0;
    std::string sha256;
    std::vector<int32_t> spec_table;  // kSpecSize entries (see sd_internal.h)
};

struct CodonTable {
    double w[64];
};

struct Lattice {
    int A = 0, n = 0, N = 0, shift = 0;
    double lambda = 0.0;
    std::string protein;
    std::vector<int> layer, off;
    std::vector<int> out_dst, out_cod;  // [N*4]
    std::vector<int64_t> out_U;
    std::vector<double> out_q;          // -ln w on third edges
    std::vector<int> in_start, in_src, in_lab, in_cod;
    std::vector<int64_t> in_U;
    std::vector<int64_t> tail, P;
    std::vector<int64_t> alphaU, betaU;  // [N*4] separable segment ends (see sd_kernels.hip)
    std::vector<int> fwd_off, fwd_meta, bwd_off, bwd_meta;  // label paths of 1..4 edges
    std::vector<int64_t> fwd_cost, bwd_cost;
    std::vector<int64_t> fwd_crow;  // per forward path: rowoff[end] - off[layer(end) + 1]
    std::vector<int64_t> hpB;  // [N*16] hairpin closing-side minima (see sd_internal.h)
    std::vector<int64_t> OB, OA;  // [N*72] one-sided loop outer minima, [state][t][X][label]
    std::vector<int> pfx, hp_init;
    std::vector<int> inmask;  // [N] bit y: the state has an in-edge labelled y
    std::vector<int64_t> rowoff, coff;
    std::vector<int> ccap;
    int64_t cells = 0, cand_slots = 0;
    int64_t mlbase_fx = 0;
    // generic lattice (codon automaton x forbidden-motif matcher): the kernels use gap tables
    // instead of the trie's closed form
    bool generic = false;
    int gwin = 0, wmax = 0;
    std::vector<std::string> motifs;
    std::vector<int64_t> gjob_off;  // [n+2]: jobs of span g are [gjob_off[g], gjob_off[g+1])
    std::vector<int32_t> gjobs;     // pairs (a, b*8 + type) of typed-value jobs
};

// validation and construction; return sd_status values
int check_protein(const char* p);
// Candidate capacity per right endpoint: override > 0 wins; else with K bin fractions each b
// gets min(worst, ceil(worst * min(1, frac[bin] * (1 + margin))) + slack); else worst case.
struct CapPolicy {
    int override_slots = 0;
    const float* frac = nullptr;
    int K = 0;
    float margin = 0.f;
    int slack = 0;
};
int position_bin(int layer, int n, int K);
int build_lattice(const char* protein, const CodonTable& T, const Params& P, double lambda,
                  const CapPolicy& cap, Lattice& L, std::string& err);

// Design under forbidden motifs: the codon trie of `protein` intersected with a deterministic
// matcher of the motifs (1..kMaxMotifLen bases over ACGU, at most kMaxMotifs of them).  The
// fixed-point shift is the unconstrained design's.  SD_E_INFEASIBLE if no coding sequence avoids
// every motif, SD_E_RANGE if a layer is wider than kGenMaxWidth states.
constexpr int kMaxMotifLen = 32;
constexpr int kMaxMotifs = 256;
int build_motif_lattice(const char* protein, const CodonTable& T, const Params& P, double lambda,
                        const CapPolicy& cap, const std::vector<std::string>& motifs, Lattice& L,
                        std::string& err);


std::string sha256_hex(const std::string& data);
int parse_params(const std::string& text, Params& P, std::string& err);

}  // namespace sd
