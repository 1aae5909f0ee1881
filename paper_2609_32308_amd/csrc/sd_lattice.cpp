// Host preparation of a design: parameter parsing, input validation, the codon trie automaton
// (Sec. 3), fixed-point edge costs and the table layouts used by the kernels.
#include "sd_lattice.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <sstream>

#include "../../include/sparsedesign.h"

namespace sd {

namespace {
// standard genetic code, codon index 16*b1 + 4*b2 + b3 with A<C<G<U
const char kCode[65] = "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";
const char* kAmino = "ACDEFGHIKLMNPQRSTVWY";

int nuc_code(char c) {
    switch (c) {
        case 'A': return 0;
        case 'C': return 1;
        case 'G': return 2;
        case 'U': return 3;
    }
    return -1;
}
}  // namespace

// ------------------------------------------------------------------------------------------------
// parameter file: "SPARSEDESIGN-PARAMS 1", then [section] headers with counts
// ------------------------------------------------------------------------------------------------
int parse_params(const std::string& text, Params& P, std::string& err) {
    std::istringstream in(text);
    std::vector<std::string> tok;
    std::string line;
    while (std::getline(in, line)) {
        size_t h = line.find('#');
        if (h != std::string::npos) line = line.substr(0, h);
        std::istringstream ls(line);
        std::string t;
        while (ls >> t) tok.push_back(t);
    }
    size_t i = 0;
    auto need = [&](const char* what) -> const std::string* {
        if (i >= tok.size()) {
            err = std::string("parameter file ends inside ") + what;
            return nullptr;
        }
        return &tok[i++];
    };
    auto as_int = [&](const std::string& s, int32_t& v, bool allow_inf) -> bool {
        if (allow_inf && s == "INF") {
            v = kNoSpecial;
            return true;
        }
        char* end = nullptr;
        long x = strtol(s.c_str(), &end, 10);
        if (*end || x < -100000 || x > 100000) {
            err = "bad integer '" + s + "'";
            return false;
        }
        v = (int32_t)x;
        return true;
    };
    if (tok.size() < 2 || tok[0] != "SPARSEDESIGN-PARAMS" || tok[1] != "1") {
        err = "missing 'SPARSEDESIGN-PARAMS 1' header";
        return SD_E_PARAMS;
    }
    i = 2;
    memset(&P.E, 0, sizeof(P.E));
    unsigned seen = 0;
    struct Arr {
        const char* name;
        int32_t* dst;
        int count;
        bool inf;
    } arrs[] = {
        {"[stack]", &P.E.stack[0][0], 36, false},
        {"[mismatch_hairpin]", &P.E.mmH[0][0][0], 96, false},
        {"[mismatch_interior]", &P.E.mmI[0][0][0], 96, false},
        {"[mismatch_interior_1n]", &P.E.mm1n[0][0][0], 96, false},
        {"[mismatch_interior_23]", &P.E.mm23[0][0][0], 96, false},
        {"[int11]", &P.E.int11[0][0][0][0], 576, false},
        {"[int21]", &P.E.int21[0][0][0][0][0], 2304, false},
        {"[int22]", &P.E.int22[0][0][0][0][0][0], 9216, false},
        {"[hairpin]", P.E.hairpin, 31, true},
        {"[bulge]", P.E.bulge, 31, true},
        {"[interior]", P.E.interior, 31, true},
    };
    const char* specials[3] = {"[triloop]", "[tetraloop]", "[hexaloop]"};
    while (i < tok.size()) {
        const std::string sec = tok[i++];
        if (sec == "[end]") break;
        if (sec == "[name]") {
            if (!need("[name]")) return SD_E_PARAMS;
            continue;
        }
        if (sec == "[scalars]") {
            for (int k = 0; k < 7; k++) {
                const std::string* key = need("[scalars]");
                const std::string* val = need("[scalars]");
                if (!key || !val) return SD_E_PARAMS;
                if (*key == "lxc") {
                    char* end = nullptr;
                    P.lxc = strtod(val->c_str(), &end);
                    if (*end || !(P.lxc >= 0.0 && P.lxc < 1000.0)) {
                        err = "bad lxc";
                        return SD_E_PARAMS;
                    }
                    continue;
                }
                int32_t v;
                if (!as_int(*val, v, false)) return SD_E_PARAMS;
                if (*key == "ML_closing") P.E.ml_closing = v;
                else if (*key == "ML_intern") P.E.ml_intern = v;
                else if (*key == "ML_base") P.E.ml_base = v;
                else if (*key == "TerminalAU") P.E.terminal_au = v;
                else if (*key == "Ninio") P.E.ninio = v;
                else if (*key == "NinioMax") P.E.ninio_max = v;
                else {
                    err = "unknown scalar " + *key;
                    return SD_E_PARAMS;
                }
            }
            seen |= 1u << 0;
            continue;
        }
        const std::string* cnt = need(sec.c_str());
        if (!cnt) return SD_E_PARAMS;
        int count = atoi(cnt->c_str());
        bool done = false;
        for (int k = 0; k < 11 && !done; k++) {
            if (sec != arrs[k].name) continue;
            if (count != arrs[k].count) {
                err = sec + " has the wrong entry count";
                return SD_E_PARAMS;
            }
            for (int j = 0; j < count; j++) {
                const std::string* s = need(sec.c_str());
                if (!s || !as_int(*s, arrs[k].dst[j], arrs[k].inf)) return SD_E_PARAMS;
            }
            seen |= 1u << (1 + k);
            done = true;
        }
        for (int k = 0; k < 3 && !done; k++) {
            if (sec != specials[k]) continue;
            const size_t len = k == 0 ? 5 : k == 1 ? 6 : 8;
            if (count < 0 || count > 4096) {
                err = sec + " count out of range";
                return SD_E_PARAMS;
            }
            for (int j = 0; j < count; j++) {
                const std::string* s = need(sec.c_str());
                const std::string* v = need(sec.c_str());
                int32_t e;
                if (!s || !v || !as_int(*v, e, false)) return SD_E_PARAMS;
                if (s->size() != len) {
                    err = "special loop of wrong length in " + sec;
                    return SD_E_PARAMS;
                }
                for (char c : *s)
                    if (nuc_code(c) < 0) {
                        err = "bad base in special loop";
                        return SD_E_PARAMS;
                    }
                P.special[k].push_back(*s);
                P.special_e[k].push_back(e);
            }
            seen |= 1u << (12 + k);
            done = true;
        }
        if (!done) {
            err = "unknown section " + sec;
            return SD_E_PARAMS;
        }
    }
    if (seen != (1u << 15) - 1) {
        err = "parameter file misses a section";
        return SD_E_PARAMS;
    }
    for (int m = 3; m <= 30; m++)
        if (P.E.hairpin[m] == kNoSpecial) { err = "hairpin sizes 3..30 must be finite"; return SD_E_PARAMS; }
    for (int m = 1; m <= 30; m++)
        if (P.E.bulge[m] == kNoSpecial) { err = "bulge sizes 1..30 must be finite"; return SD_E_PARAMS; }
    for (int m = 2; m <= 30; m++)
        if (P.E.interior[m] == kNoSpecial) { err = "interior sizes 2..30 must be finite"; return SD_E_PARAMS; }
    // largest magnitude of any finite entry (input to the fixed-point range rule)
    int32_t mx = 0;
    auto upd = [&](int32_t v) {
        if (v == kNoSpecial) return;
        int32_t a = v < 0 ? -v : v;
        if (a > mx) mx = a;
    };
    for (auto& a : arrs)
        for (int j = 0; j < a.count; j++) upd(a.dst[j]);
    for (int k = 0; k < 3; k++)
        for (int32_t e : P.special_e[k]) upd(e);
    for (int32_t v : {P.E.ml_closing, P.E.ml_intern, P.E.ml_base, P.E.terminal_au, P.E.ninio, P.E.ninio_max}) upd(v);
    P.maxabs = mx;
    // 16-bit copies of the 1x2 and 2x2 tables for the kernels
    for (int j = 0; j < 2304; j++) {
        const int32_t v = (&P.E.int21[0][0][0][0][0])[j];
        if (v < -32768 || v > 32767) {
            err = "[int21] entry outside the 16-bit range the kernels stage";
            return SD_E_PARAMS;
        }
        (&P.E.int21h[0][0][0][0][0])[j] = (int16_t)v;
    }
    for (int j = 0; j < 9216; j++) {
        const int32_t v = (&P.E.int22[0][0][0][0][0][0])[j];
        if (v < -32768 || v > 32767) {
            err = "[int22] entry outside the 16-bit range the kernels stage";
            return SD_E_PARAMS;
        }
        (&P.E.int22h[0][0][0][0][0][0])[j] = (int16_t)v;
    }
    // special-loop lookup table keyed by the base-4 value of the loop sequence
    P.spec_table.assign(kSpecSize, kNoSpecial);
    const int offs[3] = {kSpecOff5, kSpecOff6, kSpecOff8};
    for (int k = 0; k < 3; k++)
        for (size_t j = 0; j < P.special[k].size(); j++) {
            int key = 0;
            for (char c : P.special[k][j]) key = key * 4 + nuc_code(c);
            if (P.spec_table[offs[k] + key] == kNoSpecial) P.spec_table[offs[k] + key] = P.special_e[k][j];
        }
    return SD_OK;
}

// ------------------------------------------------------------------------------------------------
int check_protein(const char* p) {
    if (!p) return SD_E_ARG;
    size_t A = strlen(p);
    if (A == 0) return SD_E_PROTEIN;
    for (size_t k = 0; k < A; k++) {
        if (p[k] == '*') {
            if (k + 1 != A) return SD_E_PROTEIN;
        } else if (!strchr(kAmino, p[k])) {
            return SD_E_PROTEIN;
        }
    }
    return SD_OK;
}

int position_bin(int layer, int n, int K) {
    const int k = n > 0 ? (int)(((int64_t)layer * K) / (n + 1)) : 0;
    return k < K ? k : K - 1;
}

namespace {
// in-edges sorted by (source, label), and the in-label mask of every state
void index_in_edges(Lattice& L) {
    const int N = L.N;
    L.in_start.assign(N + 1, 0);
    for (int u = 0; u < N; u++)
        for (int x = 0; x < 4; x++)
            if (L.out_dst[4 * u + x] >= 0) L.in_start[L.out_dst[4 * u + x] + 1]++;
    for (int v = 0; v < N; v++) L.in_start[v + 1] += L.in_start[v];
    const int nE = L.in_start[N];
    L.in_src.assign(nE, 0);
    L.in_lab.assign(nE, 0);
    L.in_cod.assign(nE, -1);
    L.in_U.assign(nE, 0);
    std::vector<int> fill(N, 0);
    for (int u = 0; u < N; u++)
        for (int x = 0; x < 4; x++) {
            int v = L.out_dst[4 * u + x];
            if (v < 0) continue;
            int j = L.in_start[v] + fill[v]++;
            L.in_src[j] = u;
            L.in_lab[j] = x;
            L.in_cod[j] = L.out_cod[4 * u + x];
            L.in_U[j] = L.out_U[4 * u + x];
        }
    L.inmask.assign(N, 0);
    for (int v = 0; v < N; v++)
        for (int j = L.in_start[v]; j < L.in_start[v + 1]; j++) L.inmask[v] |= 1 << L.in_lab[j];
}

// hairpin initiation per size, extrapolated above 30 (rounded half away from zero)
void hairpin_init(Lattice& L, const Params& P) {
    L.hp_init.assign(L.n + 1, kNoSpecial);
    for (int m = 3; m <= L.n; m++)
        L.hp_init[m] = m <= 30 ? P.E.hairpin[m]
                               : P.E.hairpin[30] + (int32_t)lround(P.lxc * log((double)m / 30.0));
}

// row layout of the cell tables and the candidate segments (capacity per right endpoint)
void layout_rows(Lattice& L, const CapPolicy& cp) {
    const int N = L.N, n = L.n;
    L.rowoff.assign(N, 0);
    int64_t acc = 0;
    for (int a = 0; a < N; a++) {
        L.rowoff[a] = acc;
        acc += N - L.off[L.layer[a] + 1];
    }
    L.cells = acc;
    L.coff.assign(N, 0);
    L.ccap.assign(N, 0);
    acc = 0;
    for (int b = 0; b < N; b++) {
        int lb = L.layer[b];
        int worst = lb >= 5 ? L.off[lb - 4] : 0;
        int cap = worst;
        if (cp.override_slots > 0) {
            cap = std::min(worst, cp.override_slots);
        } else if (cp.frac && cp.K > 0) {
            const double f = std::min(1.0, (double)cp.frac[position_bin(lb, n, cp.K)] * (1.0 + cp.margin));
            cap = std::min<int64_t>(worst, (int64_t)ceil(worst * f) + cp.slack);
        }
        L.coff[b] = acc;
        L.ccap[b] = cap;
        acc += cap;
    }
    L.cand_slots = acc;
}
}  // namespace

// Bound on |E| of any partial structure on n nucleotides, the energy side of the fixed-point
// range rule.  A DP value is E * 2^s plus the rounded costs of some codons of the path.  Every
// pair of the partial structure closes one loop and is at most one branch (multiloop:
// ML_intern + AU, exterior loop: AU); the other multiloop terms are ML_base per unpaired base.
// So with at most n/2 pairs and one loop's energy in [lo, hi], one branch term in [blo, bhi]:
//     n/2 * (min(0, lo) + blo) + n * min(0, ML_base)  <=  E  <=  n/2 * (max(0, hi) + bhi) + n * max(0, ML_base).
// The loop range covers hairpins of every size up to n (initiation plus a terminal AU or a
// mismatch, or a listed special loop), stacks, bulges, the interior-loop tables and generic
// interior loops (initiation, Ninio asymmetry, two mismatches), and the multiloop closing pair.
static int64_t energy_bound(const Params& P, int n) {
    const EnergyTables& E = P.E;
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    auto cover = [&](int64_t a, int64_t b) { lo = std::min(lo, a); hi = std::max(hi, b); };
    auto range = [](const int32_t* t, int cnt, int64_t z) {  // [min, max] of t and z
        int64_t a = z, b = z;
        for (int i = 0; i < cnt; i++) a = std::min<int64_t>(a, t[i]), b = std::max<int64_t>(b, t[i]);
        return std::make_pair(a, b);
    };
    const int64_t tau = E.terminal_au, au0 = std::min<int64_t>(0, tau), au1 = std::max<int64_t>(0, tau);
    // hairpins
    const auto mh = range(&E.mmH[0][0][0], 96, 0);
    int64_t i0 = INT64_MAX, i1 = INT64_MIN;
    for (int m = 3; m <= std::max(n, 3); m++) {
        const int64_t e = m <= 30 ? E.hairpin[m] : E.hairpin[30] + (int64_t)lround(P.lxc * log((double)m / 30.0));
        i0 = std::min(i0, e);
        i1 = std::max(i1, e);
    }
    cover(i0 + std::min(au0, mh.first), i1 + std::max(au1, mh.second));
    for (int k = 0; k < 3; k++)
        for (int32_t e : P.special_e[k]) cover(e, e);
    // stacks, bulges
    const auto st = range(&E.stack[0][0], 36, E.stack[0][0]);
    cover(st.first, st.second);
    cover(E.bulge[1] + st.first, E.bulge[1] + st.second);
    for (int l = 2; l <= 30; l++) cover(E.bulge[l] + 2 * au0, E.bulge[l] + 2 * au1);
    // interior loops
    for (auto t : {range(&E.int11[0][0][0][0], 576, E.int11[0][0][0][0]),
                   range(&E.int21[0][0][0][0][0], 2304, E.int21[0][0][0][0][0]),
                   range(&E.int22[0][0][0][0][0][0], 9216, E.int22[0][0][0][0][0][0])})
        cover(t.first, t.second);
    const auto mI = range(&E.mmI[0][0][0], 96, 0), m1 = range(&E.mm1n[0][0][0], 96, 0),
               m23 = range(&E.mm23[0][0][0], 96, 0);
    const int64_t mm0 = std::min({mI.first, m1.first, m23.first}), mm1 = std::max({mI.second, m1.second, m23.second});
    const int64_t as0 = std::min<int64_t>({0, E.ninio_max, 28 * (int64_t)E.ninio}), as1 = std::max<int64_t>(0, E.ninio_max);
    for (int l = 2; l <= 30; l++) cover(E.interior[l] + as0 + 2 * mm0, E.interior[l] + as1 + 2 * mm1);
    // multiloop closing pair
    cover((int64_t)E.ml_closing + E.ml_intern + au0, (int64_t)E.ml_closing + E.ml_intern + au1);
    const int64_t blo = std::min<int64_t>({0, E.ml_intern + au0, au0}), bhi = std::max<int64_t>({0, E.ml_intern + au1, au1});
    const int64_t pairs = n / 2;
    const int64_t elo = pairs * (std::min<int64_t>(0, lo) + blo) + (int64_t)n * std::min<int64_t>(0, E.ml_base);
    const int64_t ehi = pairs * (std::max<int64_t>(0, hi) + bhi) + (int64_t)n * std::max<int64_t>(0, E.ml_base);
    return std::max(-elo, ehi);
}

int build_lattice(const char* protein, const CodonTable& T, const Params& P, double lambda,
                  const CapPolicy& cp, Lattice& L, std::string& err) {
    int rc = check_protein(protein);
    if (rc) {
        err = "protein must use ACDEFGHIKLMNPQRSTVWY with an optional final '*'";
        return rc;
    }
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) {
        err = "lambda must be finite and >= 0";
        return SD_E_LAMBDA;
    }
    L = Lattice();
    L.protein = protein;
    L.lambda = lambda;
    const int A = (int)strlen(protein), n = 3 * A;
    L.A = A;
    L.n = n;
    // codon families used by the protein must be normalised (max w = 1)
    for (int k = 0; k < A; k++) {
        double mx = 0.0;
        for (int c = 0; c < 64; c++)
            if (kCode[c] == protein[k]) mx = std::max(mx, T.w[c]);
        if (mx != 1.0) {
            err = std::string("codon family of '") + protein[k] + "' has no weight equal to 1";
            return SD_E_CODON_TABLE;
        }
    }
    // trie states: layer 3k = codon boundary, 3k+1 = first base, 3k+2 = two-base prefix
    L.off.assign(n + 2, 0);
    L.layer.clear();
    L.pfx.clear();
    std::vector<int> first(4 * (A + 1), -1), pre(16 * (A + 1), -1), beta(A + 1, -1);
    auto add_state = [&](int lay, int code) {
        L.layer.push_back(lay);
        L.pfx.push_back(code);
        return (int)L.layer.size() - 1;
    };
    beta[0] = add_state(0, 0);
    for (int k = 0; k < A; k++) {
        bool hasx[4] = {false, false, false, false}, hasxy[16] = {};
        for (int c = 0; c < 64; c++)
            if (kCode[c] == protein[k]) {
                hasx[c >> 4] = true;
                hasxy[c >> 2] = true;
            }
        L.off[3 * k + 1] = (int)L.layer.size();
        for (int x = 0; x < 4; x++)
            if (hasx[x]) first[4 * k + x] = add_state(3 * k + 1, x);
        L.off[3 * k + 2] = (int)L.layer.size();
        for (int xy = 0; xy < 16; xy++)
            if (hasxy[xy]) pre[16 * k + xy] = add_state(3 * k + 2, xy);
        L.off[3 * k + 3] = (int)L.layer.size();
        beta[k + 1] = add_state(3 * k + 3, 0);
    }
    L.off[n + 1] = (int)L.layer.size();
    const int N = L.N = (int)L.layer.size();
    for (int p = 0; p <= n; p++) {
        if (L.off[p + 1] - L.off[p] > 4) {  // kernels buffer at most 4 x 4 cells per layer pair
            err = "automaton layer wider than 4 states";
            return SD_E_INTERNAL;
        }
        L.wmax = std::max(L.wmax, L.off[p + 1] - L.off[p]);
    }
    L.out_dst.assign((size_t)4 * N, -1);
    L.out_cod.assign((size_t)4 * N, -1);
    L.out_q.assign((size_t)4 * N, 0.0);
    for (int k = 0; k < A; k++)
        for (int c = 0; c < 64; c++) {
            if (kCode[c] != protein[k]) continue;
            int x = c >> 4, y = (c >> 2) & 3, z = c & 3;
            L.out_dst[4 * beta[k] + x] = first[4 * k + x];
            L.out_dst[4 * first[4 * k + x] + y] = pre[16 * k + (c >> 2)];
            int e = 4 * pre[16 * k + (c >> 2)] + z;
            L.out_dst[e] = beta[k + 1];
            L.out_cod[e] = c;
            L.out_q[e] = -log(T.w[c]);
        }
    // fixed point: largest shift s in [16, 40] meeting the range rule (energy_bound)
    const double lam100 = 100.0 * lambda;
    const __int128 ebound = energy_bound(P, n);
    int shift = -1;
    for (int s = 40; s >= 16 && shift < 0; s--) {
        __int128 tot = 0;
        for (int k = 0; k < A && tot < ((__int128)1 << 60); k++) {
            int64_t mx = 0;
            for (int c = 0; c < 64; c++) {
                if (kCode[c] != protein[k]) continue;
                const double x = ldexp(lam100 * -log(T.w[c]), s);
                if (!(x < 0x1p60)) {  // this codon alone breaks the rule (and would overflow llround)
                    mx = (int64_t)1 << 60;
                    break;
                }
                mx = std::max<int64_t>(mx, llround(x));
            }
            tot += mx;
        }
        tot += ebound << s;
        if (tot < ((__int128)1 << 60)) shift = s;
    }
    if (shift < 0) {
        err = "fixed-point range rule cannot be met for this length / lambda";
        return SD_E_RANGE;
    }
    L.shift = shift;
    L.mlbase_fx = (int64_t)P.E.ml_base * ((int64_t)1 << shift);
    L.out_U.assign((size_t)4 * N, 0);
    for (size_t e = 0; e < L.out_U.size(); e++)
        if (L.out_cod[e] >= 0) L.out_U[e] = llround(ldexp(lam100 * L.out_q[e], shift));
    index_in_edges(L);
    // gap closed form: cheapest completion of the current codon, per-codon minima, prefix sums
    L.tail.assign(N, 0);
    L.P.assign(A + 1, 0);
    // tail: phase 0 -> codon minimum, phase 1 -> min over its completions, phase 2 -> min over
    // its third edges; cmin = per-codon minimum for the prefix sums P
    std::vector<int64_t> cmin(A, kINF);
    for (int v = 0; v < N; v++) L.tail[v] = kINF;
    for (int k = 0; k < A; k++)
        for (int c = 0; c < 64; c++)
            if (kCode[c] == protein[k]) {
                int64_t u = L.out_U[4 * pre[16 * k + (c >> 2)] + (c & 3)];
                int sb = beta[k], sx = first[4 * k + (c >> 4)], sxy = pre[16 * k + (c >> 2)];
                cmin[k] = std::min(cmin[k], u);
                L.tail[sb] = std::min(L.tail[sb], u);
                L.tail[sx] = std::min(L.tail[sx], u);
                L.tail[sxy] = std::min(L.tail[sxy], u);
            }
    L.tail[beta[A]] = 0;
    for (int k = 0; k < A; k++) L.P[k + 1] = L.P[k] + cmin[k];
    // segment ends: alpha(d,x) = U(d -x-> d2) + tail(d2); beta(c,x) = min U over in-edges labelled x
    L.alphaU.assign((size_t)4 * N, kINF);
    L.betaU.assign((size_t)4 * N, kINF);
    for (int v = 0; v < N; v++)
        for (int x = 0; x < 4; x++) {
            int d = L.out_dst[4 * v + x];
            if (d >= 0) L.alphaU[4 * v + x] = L.out_U[4 * v + x] + L.tail[d];
        }
    for (int v = 0; v < N; v++)
        for (int j = L.in_start[v]; j < L.in_start[v + 1]; j++)
            L.betaU[4 * v + L.in_lab[j]] = std::min(L.betaU[4 * v + L.in_lab[j]], L.in_U[j]);
    // hairpin closing side: min over b2 -z-> b1 -y-> b of the two edge costs
    L.hpB.assign((size_t)16 * N, kINF);
    for (int v = 0; v < N; v++)
        for (int j = L.in_start[v]; j < L.in_start[v + 1]; j++) {
            const int b1 = L.in_src[j], y = L.in_lab[j];
            for (int j2 = L.in_start[b1]; j2 < L.in_start[b1 + 1]; j2++) {
                const int z = L.in_lab[j2];
                int64_t& h = L.hpB[16 * v + 4 * y + z];
                h = std::min(h, L.in_U[j] + L.in_U[j2]);
            }
        }
    // outer minima of one-sided interior loops, per state, closing type t, mismatch class X
    // (0 generic, 1 2x3, 2 1xn) and boundary label x:
    //   OB(b1, t, X, x) = min_o beta(b1, o) + mm_X[t][x][o]    (x = x_{i+1}, o = x_{j-1})
    //   OA(a1, t, X, x) = min_o alpha(a1, o) + mm_X[t][o][x]   (o = x_{i+1}, x = x_{j-1})
    L.OB.assign((size_t)72 * N, kINF);
    L.OA.assign((size_t)72 * N, kINF);
    {
        const int32_t(*mm[3])[4][4] = {P.E.mmI, P.E.mm23, P.E.mm1n};
        const int64_t unit = (int64_t)1 << shift;
        for (int v = 0; v < N; v++)
            for (int t = 0; t < 6; t++)
                for (int X = 0; X < 3; X++)
                    for (int x = 0; x < 4; x++) {
                        int64_t rb = kINF, ra = kINF;
                        for (int o = 0; o < 4; o++) {
                            const int64_t be = L.betaU[4 * v + o], al = L.alphaU[4 * v + o];
                            if (be < kINF) rb = std::min(rb, be + (int64_t)mm[X][t][x][o] * unit);
                            if (al < kINF) ra = std::min(ra, al + (int64_t)mm[X][t][o][x] * unit);
                        }
                        L.OB[(size_t)72 * v + (t * 3 + X) * 4 + x] = rb;
                        L.OA[(size_t)72 * v + (t * 3 + X) * 4 + x] = ra;
                    }
    }
    // label paths of 1..4 edges out of / into every state (explicit short loop segments)
    L.fwd_off.assign((size_t)4 * N + 1, 0);
    L.bwd_off.assign((size_t)4 * N + 1, 0);
    L.fwd_meta.clear(); L.fwd_cost.clear(); L.bwd_meta.clear(); L.bwd_cost.clear();
    for (int u = 0; u < N; u++)
        for (int len = 1; len <= 4; len++) {
            L.fwd_off[4 * u + len - 1] = (int)L.fwd_meta.size();
            struct Fr { int state, first_lab, last_lab; int64_t cost; int depth; };
            std::vector<Fr> stack{{u, -1, -1, 0, 0}};
            while (!stack.empty()) {
                Fr f = stack.back();
                stack.pop_back();
                if (f.depth == len) {
                    L.fwd_meta.push_back(f.state << 4 | f.first_lab << 2 | f.last_lab);
                    L.fwd_cost.push_back(f.cost);
                    continue;
                }
                for (int x = 0; x < 4; x++) {
                    int e = 4 * f.state + x, d = L.out_dst[e];
                    if (d < 0) continue;
                    stack.push_back({d, f.depth == 0 ? x : f.first_lab, x, f.cost + L.out_U[e], f.depth + 1});
                }
            }
        }
    L.fwd_off[4 * N] = (int)L.fwd_meta.size();
    for (int v = 0; v < N; v++)
        for (int len = 1; len <= 4; len++) {
            L.bwd_off[4 * v + len - 1] = (int)L.bwd_meta.size();
            // backward walk over in-edge sequences; record (start, first label, last label)
            struct Fr { int state, first_lab, last_lab; int64_t cost; int depth; };
            std::vector<Fr> stack{{v, -1, -1, 0, 0}};
            while (!stack.empty()) {
                Fr f = stack.back();
                stack.pop_back();
                if (f.depth == len) {
                    L.bwd_meta.push_back(f.state << 4 | f.first_lab << 2 | f.last_lab);
                    L.bwd_cost.push_back(f.cost);
                    continue;
                }
                for (int j = L.in_start[f.state]; j < L.in_start[f.state + 1]; j++)
                    stack.push_back({L.in_src[j], L.in_lab[j], f.depth == 0 ? L.in_lab[j] : f.last_lab,
                                     f.cost + L.in_U[j], f.depth + 1});
            }
        }
    L.bwd_off[4 * N] = (int)L.bwd_meta.size();
    hairpin_init(L, P);
    layout_rows(L, cp);
    L.fwd_crow.resize(L.fwd_meta.size());
    for (size_t e = 0; e < L.fwd_meta.size(); e++) {
        const int c = L.fwd_meta[e] >> 4;
        L.fwd_crow[e] = L.rowoff[c] - L.off[L.layer[c] + 1];
    }
    return SD_OK;
}

// ------------------------------------------------------------------------------------------------
// Forbidden motifs (Sec. 3): the codon trie intersected with a deterministic motif matcher.
// Matcher states are the distinct motif prefixes (the empty one included), ranked by length and
// then lexicographically in A<C<G<U order; reading base x in prefix m goes to the longest suffix
// of m.x that is a prefix, and is not allowed when a suffix of m.x is a whole motif.  Product
// states are the (trie state, matcher state) pairs reachable from (source, empty prefix) that can
// still reach the last layer, ordered by layer, then trie state, then matcher rank.
// ------------------------------------------------------------------------------------------------
int build_motif_lattice(const char* protein, const CodonTable& T, const Params& P, double lambda,
                        const CapPolicy& cp, const std::vector<std::string>& motifs, Lattice& L,
                        std::string& err) {
    if (motifs.empty() || (int)motifs.size() > kMaxMotifs) {
        err = "need 1 to 256 motifs";
        return SD_E_ARG;
    }
    for (const std::string& m : motifs) {
        if (m.empty() || (int)m.size() > kMaxMotifLen || m.find_first_not_of("ACGU") != std::string::npos) {
            err = "motifs are 1 to 32 bases over A, C, G, U";
            return SD_E_ARG;
        }
    }
    Lattice Tr;
    int rc = build_lattice(protein, T, P, lambda, CapPolicy(), Tr, err);
    if (rc) return rc;
    // matcher
    std::vector<std::string> pre{std::string()};
    for (const std::string& m : motifs)
        for (size_t l = 1; l <= m.size(); l++) pre.push_back(m.substr(0, l));
    std::sort(pre.begin(), pre.end(), [](const std::string& a, const std::string& b) {
        return a.size() != b.size() ? a.size() < b.size() : a < b;
    });
    pre.erase(std::unique(pre.begin(), pre.end()), pre.end());
    const int K = (int)pre.size();
    std::map<std::string, int> rank;
    for (int i = 0; i < K; i++) rank[pre[i]] = i;
    std::vector<int> step((size_t)4 * K, -1);
    for (int m = 0; m < K; m++)
        for (int x = 0; x < 4; x++) {
            const std::string t = pre[m] + "ACGU"[x];
            bool banned = false;
            for (const std::string& w : motifs)
                if (w.size() <= t.size() && t.compare(t.size() - w.size(), w.size(), w) == 0) banned = true;
            if (banned) continue;
            for (size_t k = 0; k <= t.size(); k++) {  // longest suffix first
                auto it = rank.find(t.substr(k));
                if (it != rank.end()) {
                    step[(size_t)4 * m + x] = it->second;
                    break;
                }
            }
        }
    // forward: reachable pairs per layer, sorted by (trie state, matcher rank)
    const int n = Tr.n;
    typedef std::pair<int, int> QM;
    std::vector<std::vector<QM>> lay(n + 1);
    lay[0].push_back(QM(0, 0));
    for (int p = 0; p < n; p++) {
        std::vector<QM>& nx = lay[p + 1];
        for (const QM& s : lay[p])
            for (int x = 0; x < 4; x++) {
                const int d = Tr.out_dst[(size_t)4 * s.first + x], m2 = step[(size_t)4 * s.second + x];
                if (d >= 0 && m2 >= 0) nx.push_back(QM(d, m2));
            }
        std::sort(nx.begin(), nx.end());
        nx.erase(std::unique(nx.begin(), nx.end()), nx.end());
    }
    // backward: keep the pairs with a path to the last layer
    auto succ = [&](int p, const QM& s, int x) -> int {  // index in lay[p+1] or -1
        const int d = Tr.out_dst[(size_t)4 * s.first + x], m2 = step[(size_t)4 * s.second + x];
        if (d < 0 || m2 < 0) return -1;
        auto it = std::lower_bound(lay[p + 1].begin(), lay[p + 1].end(), QM(d, m2));
        return (it != lay[p + 1].end() && *it == QM(d, m2)) ? (int)(it - lay[p + 1].begin()) : -1;
    };
    std::vector<std::vector<char>> live(n + 1);
    live[n].assign(lay[n].size(), 1);
    for (int p = n - 1; p >= 0; p--) {
        live[p].assign(lay[p].size(), 0);
        for (size_t i = 0; i < lay[p].size(); i++)
            for (int x = 0; x < 4 && !live[p][i]; x++) {
                const int j = succ(p, lay[p][i], x);
                if (j >= 0 && live[p + 1][j]) live[p][i] = 1;
            }
    }
    if (!live[0][0]) {
        err = "no synonymous mRNA avoids every motif";
        return SD_E_INFEASIBLE;
    }
    std::vector<std::vector<int>> id(n + 1);
    L = Lattice();
    L.protein = protein;
    L.lambda = lambda;
    L.A = Tr.A;
    L.n = n;
    L.shift = Tr.shift;
    L.mlbase_fx = Tr.mlbase_fx;
    L.off.assign(n + 2, 0);
    int N = 0;
    for (int p = 0; p <= n; p++) {
        L.off[p] = N;
        id[p].assign(lay[p].size(), -1);
        for (size_t i = 0; i < lay[p].size(); i++)
            if (live[p][i]) {
                id[p][i] = N++;
                L.layer.push_back(p);
            }
        if (N - L.off[p] > kGenMaxWidth) {
            err = "motif automaton layer wider than 16 states";
            return SD_E_RANGE;
        }
        L.wmax = std::max(L.wmax, N - L.off[p]);
    }
    L.off[n + 1] = N;
    L.N = N;
    L.out_dst.assign((size_t)4 * N, -1);
    L.out_cod.assign((size_t)4 * N, -1);
    L.out_q.assign((size_t)4 * N, 0.0);
    L.out_U.assign((size_t)4 * N, 0);
    for (int p = 0; p < n; p++)
        for (size_t i = 0; i < lay[p].size(); i++) {
            if (id[p][i] < 0) continue;
            const int u = id[p][i], q = lay[p][i].first;
            for (int x = 0; x < 4; x++) {
                const int j = succ(p, lay[p][i], x);
                if (j < 0 || id[p + 1][j] < 0) continue;
                L.out_dst[(size_t)4 * u + x] = id[p + 1][j];
                L.out_cod[(size_t)4 * u + x] = Tr.out_cod[(size_t)4 * q + x];
                L.out_q[(size_t)4 * u + x] = Tr.out_q[(size_t)4 * q + x];
                L.out_U[(size_t)4 * u + x] = Tr.out_U[(size_t)4 * q + x];
            }
        }
    index_in_edges(L);
    hairpin_init(L, P);
    layout_rows(L, cp);
    // the trie's closed-form arrays are not used on a generic lattice: neutral fillers that keep
    // the device layout's extents
    L.tail.assign(N, 0);
    L.pfx.assign(N, 0);
    L.P.assign(L.A + 1, 0);
    L.alphaU.assign((size_t)4 * N, kINF);
    L.betaU.assign((size_t)4 * N, kINF);
    L.hpB.assign((size_t)16 * N, kINF);
    L.OB.assign((size_t)72 * N, kINF);
    L.OA.assign((size_t)72 * N, kINF);
    L.fwd_off.assign((size_t)4 * N + 1, 0);
    L.bwd_off.assign((size_t)4 * N + 1, 0);
    L.generic = true;
    L.motifs = motifs;
    for (int p = 0; p <= n; p++)
        L.gwin = std::max(L.gwin, L.off[std::min(p + 1 + kGenLoopWin, n + 1)] - L.off[std::min(p + 1, n + 1)]);
    L.gwin = std::max(L.gwin, 1);
    // typed-value jobs per span: (a, b, t) with an out-edge of a labelled t's 5' base, an in-edge
    // of b labelled its 3' base and span >= 5 (no other type can close the cell)
    L.gjob_off.assign(n + 2, 0);
    L.gjobs.clear();
    for (int g = 0; g <= n; g++) {
        L.gjob_off[g] = (int64_t)L.gjobs.size() / 2;
        if (g < 5) continue;
        for (int p = 0; p + g <= n; p++)
            for (int a = L.off[p]; a < L.off[p + 1]; a++)
                for (int b = L.off[p + g]; b < L.off[p + g + 1]; b++)
                    for (int t = 0; t < 6; t++) {
                        static const int tx[6] = {0, 1, 2, 2, 3, 3}, ty[6] = {3, 2, 1, 3, 0, 2};
                        if (L.out_dst[(size_t)4 * a + tx[t]] < 0 || !((L.inmask[b] >> ty[t]) & 1)) continue;
                        L.gjobs.push_back(a);
                        L.gjobs.push_back(b * 8 + t);
                    }
    }
    L.gjob_off[n + 1] = (int64_t)L.gjobs.size() / 2;
    return SD_OK;
}

}  // namespace sd
