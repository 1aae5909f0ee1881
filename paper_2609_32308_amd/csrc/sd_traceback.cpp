// Canonical first-match traceback over the completed fixed-point tables.
//
// At every decision the alternatives are enumerated in a fixed order and the first one whose
// value equals the cell value exactly is taken, so the emitted (mRNA, structure) does not depend
// on reduction order or on how the tables were filled (Sec. 5: traceback reconstructs decisions
// from completed costs; Sec. 7.2: optima are often tied, so a fixed rule is needed to compare
// sequences).  The order:
//   X(a):   unpaired out-edges by label; then branches b by state index, pair type AU,CG,GC,GU,UA,UG
//   V_t:    hairpin (sizes 3,4,6: paths in lexicographic base order; other sizes: x_{i+1} by
//           base, closing in-edge of b by (source, base), in-edge of b1 by (source, base)),
//           then two-loops (l1 asc, l2 asc, closing in-edge of b, inner c by index, d by index,
//           inner type, left segment, right segment), then multiloop (closing in-edge of b)
//   S1:     direct branch, S2, left unpaired edge (by label), right unpaired edge (in-edge order)
//   S2:     right unpaired edge (in-edge order), then candidates c of C_b by state index (eq. 7)
//   branch: pair type order
//   gaps:   minimum-cost path taking the smallest base that stays on a minimum path
#include <string.h>

#include <vector>

#include "../../include/sparsedesign.h"
#include "sd_lattice.h"
#include "sd_traceback.h"

namespace sd {

namespace {
const int TX[6] = {0, 1, 2, 2, 3, 3};
const int TY[6] = {3, 2, 1, 3, 0, 2};
int ptype(int x, int y) {
    static const int T[16] = {-1, -1, -1, 0, -1, -1, 1, -1, -1, 2, -1, 3, 4, -1, 5, -1};
    return T[x * 4 + y];
}
int32_t aupen(const EnergyTables& E, int t) { return (t == 1 || t == 2) ? 0 : E.terminal_au; }

int32_t two_loop(const EnergyTables& E, int t, int tr, int l1, int l2, int xi1, int xk1, int xl1, int xj1) {
    if (l1 == 0 && l2 == 0) return E.stack[t][tr];
    if (l1 == 0 || l2 == 0) {
        int l = l1 + l2;
        return l == 1 ? E.bulge[1] + E.stack[t][tr] : E.bulge[l] + aupen(E, t) + aupen(E, tr);
    }
    if (l1 == 1 && l2 == 1) return E.int11[t][tr][xi1][xj1];
    if (l1 == 1 && l2 == 2) return E.int21[t][tr][xi1][xl1][xj1];
    if (l1 == 2 && l2 == 1) return E.int21[tr][t][xl1][xi1][xk1];
    if (l1 == 2 && l2 == 2) return E.int22[t][tr][xi1][xk1][xl1][xj1];
    int d = l1 > l2 ? l1 - l2 : l2 - l1;
    int32_t asym = std::min(E.ninio * d, E.ninio_max);
    int32_t e = E.interior[l1 + l2] + asym;
    if (l1 == 1 || l2 == 1) return e + E.mm1n[t][xi1][xj1] + E.mm1n[tr][xl1][xk1];
    if (l1 + l2 == 5 && (l1 == 2 || l1 == 3)) return e + E.mm23[t][xi1][xj1] + E.mm23[tr][xl1][xk1];
    return e + E.mmI[t][xi1][xj1] + E.mmI[tr][xl1][xk1];
}

struct Seg {
    int e1;        // out-edge id (state*4+label) of the first base, -1 if none
    int e2;        // in-edge CSR index of the last base (length >= 2), -1 otherwise
    int gfrom, gto;
    int xa, xb;
    int64_t cost;
};

struct Tracer {
    const Lattice& L;
    const Params& P;
    const TraceTables& T;
    std::vector<int> seq, pr;
    int64_t E = 0, U = 0;
    bool ok = true;

    int segmax = 8;  // loop segments between two states: a segment of >= 2 bases is a first edge
                     // and an in-edge of its end state, so at most 4 x the largest in-degree

    Tracer(const Lattice& l, const Params& p, const TraceTables& t) : L(l), P(p), T(t) {
        seq.assign(L.n, -1);
        pr.assign(L.n, -1);
        for (int v = 0; v < L.N; v++) segmax = std::max(segmax, 4 * (L.in_start[v + 1] - L.in_start[v]) + 4);
    }
    int64_t fx(int64_t e) const { return e * ((int64_t)1 << L.shift); }
    int64_t cell(int a, int b) const { return L.rowoff[a] + (b - L.off[L.layer[a] + 1]); }
    bool fwd(int a, int b) const { return L.layer[a] < L.layer[b]; }
    int64_t V(int t, int a, int b) const { return fwd(a, b) ? T.V[cell(a, b) * 6 + t] : kINF; }
    int64_t B(int a, int b) const { return fwd(a, b) ? T.B[cell(a, b)] : kINF; }
    int64_t S1(int a, int b) const { return fwd(a, b) ? T.S1[cell(a, b)] : kINF; }
    int64_t S2(int a, int b) const { return fwd(a, b) ? T.S2[cell(a, b)] : kINF; }
    static int64_t add(int64_t a, int64_t b) { return (a >= kINF || b >= kINF) ? kINF : a + b; }

    void emit_out(int e) {  // out-edge id = state*4 + label
        int p = L.layer[e >> 2];
        if (seq[p] >= 0) ok = false;
        seq[p] = e & 3;
        U += L.out_U[e];
    }
    void emit_in(int j) {  // in-edge CSR index
        int p = L.layer[L.in_src[j]];
        if (seq[p] >= 0) ok = false;
        seq[p] = L.in_lab[j];
        U += L.in_U[j];
    }
    void emit_gap(int u, int v) {
        while (u != v) {
            int64_t g = host_gap(L, u, v);
            bool took = false;
            for (int x = 0; x < 4 && !took; x++) {
                int e = u * 4 + x, d = L.out_dst[e];
                if (d < 0) continue;
                if (add(L.out_U[e], host_gap(L, d, v)) == g) {
                    emit_out(e);
                    u = d;
                    took = true;
                }
            }
            if (!took) {
                ok = false;
                return;
            }
        }
    }

    // ---- hairpin
    bool hp_dfs(int pos, int len, int st, int b, int t, int64_t cost, int key, int* lab, int* edge, int64_t target) {
        if (pos == len) {
            if (st != b) return false;
            int m = len - 2;
            int off = m == 3 ? kSpecOff5 : m == 4 ? kSpecOff6 : kSpecOff8;
            int32_t en = P.spec_table[off + key];
            if (en == kNoSpecial) en = L.hp_init[m] + (m == 3 ? aupen(P.E, t) : P.E.mmH[t][lab[1]][lab[len - 2]]);
            if (cost + fx(en) != target) return false;
            for (int i = 0; i < len; i++) emit_out(edge[i]);
            E += en;
            return true;
        }
        for (int x = 0; x < 4; x++) {
            if (pos == 0 && x != TX[t]) continue;
            if (pos == len - 1 && x != TY[t]) continue;
            int e = st * 4 + x, d = L.out_dst[e];
            if (d < 0) continue;
            lab[pos] = x;
            edge[pos] = e;
            if (hp_dfs(pos + 1, len, d, b, t, cost + L.out_U[e], key * 4 + x, lab, edge, target)) return true;
        }
        return false;
    }

    bool hairpin(int a, int b, int t, int64_t v) {
        int g = L.layer[b] - L.layer[a], m = g - 2;
        if (m < 3) return false;
        int ea = a * 4 + TX[t];
        if (L.out_dst[ea] < 0) return false;
        if (m == 3 || m == 4 || m == 6) {
            int lab[8], edge[8];
            return hp_dfs(0, g, a, b, t, 0, 0, lab, edge, v);
        }
        int a1 = L.out_dst[ea];
        for (int x2 = 0; x2 < 4; x2++) {
            int e1 = a1 * 4 + x2, a2 = L.out_dst[e1];
            if (a2 < 0) continue;
            for (int j = L.in_start[b]; j < L.in_start[b + 1]; j++) {
                if (L.in_lab[j] != TY[t]) continue;
                int b1 = L.in_src[j];
                for (int j2 = L.in_start[b1]; j2 < L.in_start[b1 + 1]; j2++) {
                    int b2 = L.in_src[j2];
                    int64_t gg = host_gap(L, a2, b2);
                    if (gg >= kINF) continue;
                    int32_t en = L.hp_init[m] + P.E.mmH[t][x2][L.in_lab[j2]];
                    int64_t val = L.out_U[ea] + L.out_U[e1] + gg + L.in_U[j2] + L.in_U[j] + fx(en);
                    if (val != v) continue;
                    emit_out(ea);
                    emit_out(e1);
                    emit_gap(a2, b2);
                    emit_in(j2);
                    emit_in(j);
                    E += en;
                    return true;
                }
            }
        }
        return false;
    }

    // ---- two-loop
    int segs(int u, int v, int l, Seg* out) {
        int k = 0;
        if (l == 0) {
            if (u != v) return 0;
            out[0] = Seg{-1, -1, -1, -1, 0, 0, 0};
            return 1;
        }
        if (l == 1) {
            for (int x = 0; x < 4; x++) {
                int e = u * 4 + x;
                if (L.out_dst[e] == v) out[k++] = Seg{e, -1, -1, -1, x, x, L.out_U[e]};
            }
            return k;
        }
        for (int x = 0; x < 4; x++) {
            int e = u * 4 + x, u2 = L.out_dst[e];
            if (u2 < 0) continue;
            for (int j = L.in_start[v]; j < L.in_start[v + 1]; j++) {
                int64_t gg = host_gap(L, u2, L.in_src[j]);
                if (gg >= kINF) continue;
                out[k++] = Seg{e, j, u2, L.in_src[j], x, L.in_lab[j], L.out_U[e] + gg + L.in_U[j]};
            }
        }
        return k;
    }
    void emit_seg(const Seg& s) {
        if (s.e1 >= 0) emit_out(s.e1);
        if (s.e2 >= 0) {
            emit_gap(s.gfrom, s.gto);
            emit_in(s.e2);
        }
    }

    bool twoloop(int a, int b, int t, int64_t v, int& oc, int& od, int& otp) {
        int la = L.layer[a], lb = L.layer[b];
        int ea = a * 4 + TX[t], a1 = L.out_dst[ea];
        if (a1 < 0) return false;
        std::vector<Seg> Lv(segmax), Rv(segmax);
        Seg *Ls = Lv.data(), *Rs = Rv.data();
        for (int l1 = 0; l1 <= kMaxLoop; l1++)
            for (int l2 = 0; l1 + l2 <= kMaxLoop; l2++) {
                int cl = la + 1 + l1, dl = lb - 1 - l2;
                if (dl - cl < 5) continue;
                for (int j = L.in_start[b]; j < L.in_start[b + 1]; j++) {
                    if (L.in_lab[j] != TY[t]) continue;
                    int b1 = L.in_src[j];
                    for (int c = L.off[cl]; c < L.off[cl + 1]; c++) {
                        int nl = segs(a1, c, l1, Ls);
                        if (!nl) continue;
                        for (int d = L.off[dl]; d < L.off[dl + 1]; d++) {
                            int nr = -1;
                            for (int tp = 0; tp < 6; tp++) {
                                int64_t vin = V(tp, c, d);
                                if (vin >= kINF) continue;
                                if (nr < 0) nr = segs(d, b1, l2, Rs);
                                int tr = ptype(TY[tp], TX[tp]);
                                for (int p = 0; p < nl; p++)
                                    for (int q = 0; q < nr; q++) {
                                        int32_t e2 = two_loop(P.E, t, tr, l1, l2, Ls[p].xa, Ls[p].xb, Rs[q].xa, Rs[q].xb);
                                        int64_t val = L.out_U[ea] + Ls[p].cost + vin + Rs[q].cost + L.in_U[j] + fx(e2);
                                        if (val != v) continue;
                                        emit_out(ea);
                                        emit_seg(Ls[p]);
                                        emit_seg(Rs[q]);
                                        emit_in(j);
                                        E += e2;
                                        oc = c;
                                        od = d;
                                        otp = tp;
                                        return true;
                                    }
                            }
                        }
                    }
                }
            }
        return false;
    }

    bool multiloop(int a, int b, int t, int64_t v, int& oa1, int& ob1) {
        if (L.layer[b] - L.layer[a] < 12) return false;
        int ea = a * 4 + TX[t], a1 = L.out_dst[ea];
        if (a1 < 0) return false;
        int32_t mlc = P.E.ml_closing + P.E.ml_intern + aupen(P.E, t);
        for (int j = L.in_start[b]; j < L.in_start[b + 1]; j++) {
            if (L.in_lab[j] != TY[t]) continue;
            int b1 = L.in_src[j];
            if (L.layer[b1] - L.layer[a1] < 10) continue;
            if (add(L.out_U[ea] + L.in_U[j] + fx(mlc), S2(a1, b1)) != v) continue;
            emit_out(ea);
            emit_in(j);
            E += mlc;
            oa1 = a1;
            ob1 = b1;
            return true;
        }
        return false;
    }

    enum Kind { KX, KV, KS1, KS2, KBR };
    struct Frame {
        int kind, a, b, t;
    };

    void run() {
        std::vector<Frame> st;
        st.push_back({KX, 0, -1, -1});
        std::vector<int> cands;
        while (!st.empty() && ok) {
            Frame f = st.back();
            st.pop_back();
            const int a = f.a, b = f.b;
            if (f.kind == KX) {
                if (L.layer[a] == L.n) continue;
                int64_t x = T.X[a];
                bool done = false;
                for (int y = 0; y < 4 && !done; y++) {
                    int e = a * 4 + y, d = L.out_dst[e];
                    if (d < 0) continue;
                    if (add(L.out_U[e], T.X[d]) == x) {
                        emit_out(e);
                        st.push_back({KX, d, -1, -1});
                        done = true;
                    }
                }
                int b0 = L.layer[a] + 5 <= L.n ? L.off[L.layer[a] + 5] : L.N;
                for (int bb = b0; bb < L.N && !done; bb++)
                    for (int t = 0; t < 6 && !done; t++)
                        if (add(add(V(t, a, bb), fx(aupen(P.E, t))), T.X[bb]) == x) {
                            E += aupen(P.E, t);
                            st.push_back({KX, bb, -1, -1});
                            st.push_back({KV, a, bb, t});
                            done = true;
                        }
                if (!done) ok = false;
            } else if (f.kind == KV) {
                int64_t v = V(f.t, a, b);
                int i = L.layer[a], j = L.layer[b] - 1;
                pr[i] = j;
                pr[j] = i;
                if (hairpin(a, b, f.t, v)) continue;
                int c, d, tp;
                if (twoloop(a, b, f.t, v, c, d, tp)) {
                    st.push_back({KV, c, d, tp});
                    continue;
                }
                int a1, b1;
                if (multiloop(a, b, f.t, v, a1, b1)) {
                    st.push_back({KS2, a1, b1, -1});
                    continue;
                }
                ok = false;
            } else if (f.kind == KBR) {
                int64_t v = B(a, b);
                bool done = false;
                for (int t = 0; t < 6 && !done; t++) {
                    int32_t beta = P.E.ml_intern + aupen(P.E, t);
                    if (add(V(t, a, b), fx(beta)) == v) {
                        E += beta;
                        st.push_back({KV, a, b, t});
                        done = true;
                    }
                }
                if (!done) ok = false;
            } else if (f.kind == KS1) {
                int64_t v = S1(a, b);
                if (B(a, b) == v) {
                    st.push_back({KBR, a, b, -1});
                    continue;
                }
                if (S2(a, b) == v) {
                    st.push_back({KS2, a, b, -1});
                    continue;
                }
                bool done = false;
                for (int y = 0; y < 4 && !done; y++) {
                    int e = a * 4 + y, ap = L.out_dst[e];
                    if (ap < 0 || L.layer[ap] >= L.layer[b]) continue;
                    if (add(L.out_U[e] + L.mlbase_fx, S1(ap, b)) == v) {
                        emit_out(e);
                        E += P.E.ml_base;
                        st.push_back({KS1, ap, b, -1});
                        done = true;
                    }
                }
                for (int j = L.in_start[b]; j < L.in_start[b + 1] && !done; j++) {
                    int bp = L.in_src[j];
                    if (L.layer[bp] <= L.layer[a]) continue;
                    if (add(S1(a, bp), L.in_U[j] + L.mlbase_fx) == v) {
                        emit_in(j);
                        E += P.E.ml_base;
                        st.push_back({KS1, a, bp, -1});
                        done = true;
                    }
                }
                if (!done) ok = false;
            } else {  // KS2
                int64_t v = S2(a, b);
                bool done = false;
                for (int j = L.in_start[b]; j < L.in_start[b + 1] && !done; j++) {
                    int bp = L.in_src[j];
                    if (L.layer[bp] <= L.layer[a]) continue;
                    if (add(S2(a, bp), L.in_U[j] + L.mlbase_fx) == v) {
                        emit_in(j);
                        E += P.E.ml_base;
                        st.push_back({KS2, a, bp, -1});
                        done = true;
                    }
                }
                if (!done) {
                    // strict candidates of C_b with rho(c) > rho(a), increasing state index
                    cands.clear();
                    int64_t base = L.coff[b];
                    for (int k = 0; k < T.ccnt[b]; k++) {
                        int raw = T.cc[base + k];
                        if (raw < 0) continue;  // non-strict entry (retain-all control)
                        if (L.layer[raw] > L.layer[a]) cands.push_back(raw);
                    }
                    std::sort(cands.begin(), cands.end());
                    for (int c : cands) {
                        if (add(S1(a, c), B(c, b)) == v) {
                            st.push_back({KS1, a, c, -1});
                            st.push_back({KBR, c, b, -1});
                            done = true;
                            break;
                        }
                    }
                }
                if (!done) ok = false;
            }
        }
    }
};
}  // namespace

int trace_design(const Lattice& L, const Params& P, const TraceTables& T, TraceResult& R) {
    Tracer tr(L, P, T);
    if (T.X[0] >= kINF) return SD_E_INTERNAL;
    tr.run();
    // self-check: a complete path s -> t, E*2^s + U == X(s)
    int st = 0;
    int64_t Uw = 0;
    double C = 0.0;
    bool ok = tr.ok;
    for (int i = 0; i < L.n && ok; i++) {
        if (tr.seq[i] < 0) { ok = false; break; }
        int e = st * 4 + tr.seq[i];
        if (L.out_dst[e] < 0) { ok = false; break; }
        Uw += L.out_U[e];
        if (L.out_cod[e] >= 0) C += L.out_q[e];
        st = L.out_dst[e];
    }
    if (L.layer[st] != L.n) ok = false;
    if (ok && (Uw != tr.U || tr.fx(tr.E) + tr.U != T.X[0])) ok = false;
    R.mrna.assign(L.n, 'N');
    R.structure.assign(L.n, '.');
    for (int i = 0; i < L.n; i++) {
        if (tr.seq[i] >= 0) R.mrna[i] = "ACGU"[tr.seq[i]];
        if (tr.pr[i] >= 0) R.structure[i] = tr.pr[i] > i ? '(' : ')';
    }
    R.energy = (int32_t)tr.E;
    R.path_u = tr.U;
    R.codon_cost = C;
    R.ok = ok;
    return ok ? SD_OK : SD_E_INTERNAL;
}

}  // namespace sd
