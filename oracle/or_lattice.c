/* Oracle: the plain dense lattice DP (test infrastructure only; shares nothing with the GPU
 * library).
 *
 * Follows the paper section by section:
 *   Sec. 3   -- problem (eq. 1), codon weights w = f / max_syn f, C(r) = -sum ln w; the layered
 *               codon DFA with the whole -ln w on each codon's third edge; lambda in kcal/mol is
 *               multiplied by 100 (internal units are 0.01 kcal/mol).
 *   Sec. 4.1 -- typed closed values V_tau(a,b) (hairpin, two-loop, multiloop closure), scalar
 *               branch B = min_tau V_tau + beta_tau (eq. 2), dense right-normal multiloop
 *               recurrences D2 (eq. 3), P_D (eq. 4), D1 (eq. 5); candidates C_b (eq. 6) are
 *               derived from the dense tables and used only by the traceback and the counters.
 *   Sec. 5   -- span order (all cells of span g after every smaller span); final-column
 *               external values X(a) for fragments a -> t.
 * Fixed point: U(e) = llround(ldexp(100*lambda*q(e), s)), energies enter as E*2^s, the
 * sentinel OR_INF saturates.  The shift s is the largest value in [16,40] for which the range
 * rule holds (see choose_shift: a bound on every partial value from the parameter tables).
 *
 * DFA: the prefix trie of each codon family; layer 3k holds one state per codon boundary,
 * layer 3k+1 one state per distinct first base, layer 3k+2 one per distinct two-base prefix.
 * States are numbered layer by layer, within a layer by prefix (A<C<G<U).
 */
#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* amino acid of codon index 16*b1 + 4*b2 + b3 (A<C<G<U), standard genetic code */
static const char CODE[65] = "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";
static const char *AMINO = "ACDEFGHIKLMNPQRSTVWY";
static const int TX[6] = {0, 1, 2, 2, 3, 3}; /* 5' base of pair type AU CG GC GU UA UG */
static const int TY[6] = {3, 2, 1, 3, 0, 2}; /* 3' base */

static inline int64_t sat(int64_t a, int64_t b) { return (a >= OR_INF || b >= OR_INF) ? OR_INF : a + b; }
static inline int64_t mn(int64_t a, int64_t b) { return a < b ? a : b; }

typedef struct {
    int A, n, N, nE;
    int *layer, *off;                  /* off[p] = first state of layer p, off[n+1] = N */
    int *esrc, *edst, *elab, *ecod;    /* ecod: codon index on third edges, else -1 */
    double *eq;                        /* -ln w on third edges, else 0 */
    int64_t *eU;                       /* fixed-point codon cost */
    int64_t *eu_ml;                    /* U(e) + ML_base*2^s */
    int *out;                          /* [N*4] edge id by label, -1 if none */
    int *in_start, *in_e;              /* edges into a state, sorted by (source, label) */
    int *out_start, *out_e;            /* edges out of a state, sorted by label */
} dfa_t;

static void dfa_free(dfa_t *D) {
    free(D->layer); free(D->off); free(D->esrc); free(D->edst); free(D->elab); free(D->ecod);
    free(D->eq); free(D->eU); free(D->eu_ml); free(D->out); free(D->in_start); free(D->in_e);
    free(D->out_start); free(D->out_e);
    memset(D, 0, sizeof(*D));
}

static int check_protein(const char *p) {
    if (!p) return OR_E_ARG;
    int A = (int)strlen(p);
    if (A < 1) return OR_E_PROTEIN;
    for (int k = 0; k < A; k++) {
        if (p[k] == '*') {
            if (k != A - 1) return OR_E_PROTEIN;
        } else if (!strchr(AMINO, p[k]) || p[k] == 0) {
            return OR_E_PROTEIN;
        }
    }
    return OR_OK;
}

static int check_codons(const char *p, const double *w) {
    if (!w) return OR_E_ARG;
    for (const char *c = p; *c; c++) {
        double mx = 0.0;
        for (int i = 0; i < 64; i++) {
            if (CODE[i] != *c) continue;
            double v = w[i];
            if (!(v > 0.0 && v <= 1.0)) return OR_E_CODON;
            if (v > mx) mx = v;
        }
        if (mx != 1.0) return OR_E_CODON;
    }
    return OR_OK;
}

static int finish_dfa(dfa_t *D);

/* prefix-trie codon DFA of Sec. 3 (Fig. 1 state-join rule holds by construction) */
static int build_dfa(const char *prot, const double *w, dfa_t *D) {
    memset(D, 0, sizeof(*D));
    int A = (int)strlen(prot), n = 3 * A;
    int maxS = 1 + A * 21, maxE = A * 84;
    D->A = A;
    D->n = n;
    D->layer = malloc(sizeof(int) * maxS);
    D->off = malloc(sizeof(int) * (n + 2));
    D->esrc = malloc(sizeof(int) * maxE);
    D->edst = malloc(sizeof(int) * maxE);
    D->elab = malloc(sizeof(int) * maxE);
    D->ecod = malloc(sizeof(int) * maxE);
    D->eq = malloc(sizeof(double) * maxE);
    if (!D->layer || !D->off || !D->esrc || !D->edst || !D->elab || !D->ecod || !D->eq) return OR_E_NOMEM;
    int N = 0, E = 0;
    D->off[0] = 0;
    D->layer[N++] = 0; /* beta_0 = s */
    int beta = 0;
    for (int k = 0; k < A; k++) {
        int cods[6], nc = 0;
        for (int i = 0; i < 64; i++)
            if (CODE[i] == prot[k]) cods[nc++] = i;
        int first_state[4], pre_state[16];
        for (int i = 0; i < 4; i++) first_state[i] = -1;
        for (int i = 0; i < 16; i++) pre_state[i] = -1;
        D->off[3 * k + 1] = N;
        for (int x = 0; x < 4; x++)
            for (int i = 0; i < nc; i++)
                if (cods[i] / 16 == x && first_state[x] < 0) {
                    first_state[x] = N;
                    D->layer[N++] = 3 * k + 1;
                }
        D->off[3 * k + 2] = N;
        for (int xy = 0; xy < 16; xy++)
            for (int i = 0; i < nc; i++)
                if (cods[i] / 4 == xy && pre_state[xy] < 0) {
                    pre_state[xy] = N;
                    D->layer[N++] = 3 * k + 2;
                }
        D->off[3 * k + 3] = N;
        int nb = N;
        D->layer[N++] = 3 * k + 3;
        for (int x = 0; x < 4; x++)
            if (first_state[x] >= 0) {
                D->esrc[E] = beta; D->edst[E] = first_state[x]; D->elab[E] = x;
                D->ecod[E] = -1; D->eq[E] = 0.0; E++;
            }
        for (int xy = 0; xy < 16; xy++)
            if (pre_state[xy] >= 0) {
                D->esrc[E] = first_state[xy / 4]; D->edst[E] = pre_state[xy]; D->elab[E] = xy % 4;
                D->ecod[E] = -1; D->eq[E] = 0.0; E++;
            }
        for (int i = 0; i < nc; i++) {
            int c = cods[i];
            D->esrc[E] = pre_state[c / 4]; D->edst[E] = nb; D->elab[E] = c % 4;
            D->ecod[E] = c; D->eq[E] = -log(w[c]); E++;
        }
        beta = nb;
    }
    D->off[n + 1] = N;
    D->N = N;
    D->nE = E;
    return finish_dfa(D);
}

/* out-edge table by label, in-edges sorted by (source, label), out-edges sorted by label */
static int finish_dfa(dfa_t *D) {
    int N = D->N, E = D->nE;
    D->out = malloc(sizeof(int) * 4 * N);
    D->in_start = calloc(N + 1, sizeof(int));
    D->in_e = malloc(sizeof(int) * (E + 1));
    D->out_start = calloc(N + 1, sizeof(int));
    D->out_e = malloc(sizeof(int) * (E + 1));
    D->eU = calloc(E + 1, sizeof(int64_t));
    D->eu_ml = calloc(E + 1, sizeof(int64_t));
    if (!D->out || !D->in_start || !D->in_e || !D->out_start || !D->out_e || !D->eU || !D->eu_ml)
        return OR_E_NOMEM;
    for (int i = 0; i < 4 * N; i++) D->out[i] = -1;
    for (int e = 0; e < E; e++) {
        D->out[D->esrc[e] * 4 + D->elab[e]] = e;
        D->in_start[D->edst[e] + 1]++;
        D->out_start[D->esrc[e] + 1]++;
    }
    for (int v = 0; v < N; v++) {
        D->in_start[v + 1] += D->in_start[v];
        D->out_start[v + 1] += D->out_start[v];
    }
    int *fill = calloc(N, sizeof(int));
    if (!fill) return OR_E_NOMEM;
    /* in-edges sorted by (source, label): scan sources in index order, labels ascending */
    for (int u = 0; u < N; u++)
        for (int x = 0; x < 4; x++) {
            int e = D->out[u * 4 + x];
            if (e < 0) continue;
            int v = D->edst[e];
            D->in_e[D->in_start[v] + fill[v]++] = e;
        }
    for (int u = 0; u < N; u++) {
        int k = D->out_start[u];
        for (int x = 0; x < 4; x++)
            if (D->out[u * 4 + x] >= 0) D->out_e[k++] = D->out[u * 4 + x];
    }
    free(fill);
    return OR_OK;
}

/* --- forbidden motifs (Sec. 3: the codon DFA intersected with a deterministic motif matcher) ---
 * Matcher states are the distinct prefixes of the motifs (the empty prefix included), ranked by
 * length and then in A<C<G<U order.  Reading base x in state m leads to the longest suffix of
 * m.x that is again a prefix; the step is forbidden when some suffix of m.x is a whole motif
 * (such transitions are removed).  The product keeps the pairs (codon state, matcher state)
 * reachable from (source, empty prefix) by allowed steps, then drops every pair from which no
 * path reaches the last layer.  Within a layer, states are ordered by codon state, then by
 * matcher rank.  An empty language (no synonymous mRNA avoids the motifs) is OR_E_INFEASIBLE. */
typedef struct {
    int K;
    char (*str)[OR_MAX_MOTIF + 1];
    int *delta; /* [K*4] next matcher state, -1 if the step completes a motif */
} matcher_t;

static int pref_cmp(const void *x, const void *y) {
    const char *a = x, *b = y;
    size_t la = strlen(a), lb = strlen(b);
    if (la != lb) return la < lb ? -1 : 1;
    return strcmp(a, b);
}

static int pref_find(const matcher_t *M, const char *t) {
    for (int i = 0; i < M->K; i++)
        if (strcmp(M->str[i], t) == 0) return i;
    return -1;
}

static int build_matcher(const char *const *motifs, int nm, matcher_t *M) {
    memset(M, 0, sizeof(*M));
    int cap = 1;
    for (int i = 0; i < nm; i++) {
        if (!motifs[i]) return OR_E_ARG;
        size_t L = strlen(motifs[i]);
        if (L < 1 || L > OR_MAX_MOTIF) return OR_E_ARG;
        for (size_t k = 0; k < L; k++)
            if (or_nuc(motifs[i][k]) < 0) return OR_E_ARG;
        cap += (int)L;
    }
    M->str = calloc(cap, sizeof(*M->str));
    if (!M->str) return OR_E_NOMEM;
    int K = 0;
    M->str[K++][0] = 0;
    for (int i = 0; i < nm; i++) {
        size_t L = strlen(motifs[i]);
        for (size_t l = 1; l <= L; l++) {
            memcpy(M->str[K], motifs[i], l);
            M->str[K][l] = 0;
            K++;
        }
    }
    qsort(M->str, K, sizeof(*M->str), pref_cmp);
    int u = 0;
    for (int i = 0; i < K; i++)
        if (u == 0 || strcmp(M->str[u - 1], M->str[i]) != 0) memcpy(M->str[u++], M->str[i], sizeof(*M->str));
    M->K = K = u;
    M->delta = malloc(sizeof(int) * 4 * K);
    if (!M->delta) return OR_E_NOMEM;
    char t[OR_MAX_MOTIF + 2];
    for (int m = 0; m < K; m++)
        for (int x = 0; x < 4; x++) {
            size_t L = strlen(M->str[m]);
            memcpy(t, M->str[m], L);
            t[L] = "ACGU"[x];
            t[L + 1] = 0;
            int forbidden = 0, next = -1;
            for (size_t k = 0; k <= L + 1; k++) { /* suffixes, longest first */
                for (int i = 0; i < nm && !forbidden; i++)
                    if (strcmp(t + k, motifs[i]) == 0) forbidden = 1;
                if (next < 0 && k <= L + 1 && (L + 1 - k) <= OR_MAX_MOTIF) next = pref_find(M, t + k);
            }
            M->delta[m * 4 + x] = forbidden ? -1 : next;
        }
    return OR_OK;
}

static void matcher_free(matcher_t *M) {
    free(M->str);
    free(M->delta);
    memset(M, 0, sizeof(*M));
}

typedef struct {
    int q, m;
} pq_t;

static int pq_cmp(const void *x, const void *y) {
    const pq_t *a = x, *b = y;
    if (a->q != b->q) return a->q < b->q ? -1 : 1;
    return (a->m > b->m) - (a->m < b->m);
}

/* product of the codon DFA T with the matcher of the motifs; T's costs are copied per edge */
static int build_product(const dfa_t *T, const char *const *motifs, int nm, dfa_t *D) {
    memset(D, 0, sizeof(*D));
    matcher_t M;
    int rc = build_matcher(motifs, nm, &M);
    if (rc) {
        matcher_free(&M);
        return rc;
    }
    const int n = T->n, K = M.K;
    /* forward pass, layer by layer: states as (codon state, matcher state) pairs */
    int cap = 64, S = 0;
    pq_t *st = malloc(sizeof(pq_t) * cap);
    int *loff = malloc(sizeof(int) * (n + 2));
    if (!st || !loff) {
        free(st); free(loff); matcher_free(&M);
        return OR_E_NOMEM;
    }
    loff[0] = 0;
    st[S++] = (pq_t){0, 0};
    for (int p = 0; p < n; p++) {
        loff[p + 1] = S;
        for (int i = loff[p]; i < loff[p + 1]; i++)
            for (int x = 0; x < 4; x++) {
                int e = T->out[st[i].q * 4 + x];
                if (e < 0) continue;
                int m2 = M.delta[st[i].m * 4 + x];
                if (m2 < 0) continue;
                if (S == cap) {
                    cap *= 2;
                    pq_t *ns = realloc(st, sizeof(pq_t) * cap);
                    if (!ns) { free(st); free(loff); matcher_free(&M); return OR_E_NOMEM; }
                    st = ns;
                }
                st[S++] = (pq_t){T->edst[e], m2};
            }
        /* sort and deduplicate the new layer */
        qsort(st + loff[p + 1], S - loff[p + 1], sizeof(pq_t), pq_cmp);
        int u = loff[p + 1];
        for (int i = loff[p + 1]; i < S; i++)
            if (u == loff[p + 1] || pq_cmp(&st[u - 1], &st[i]) != 0) st[u++] = st[i];
        S = u;
    }
    loff[n + 1] = S;
    /* backward pass: live = some path reaches the last layer */
    char *live = calloc(S, 1);
    int *id = malloc(sizeof(int) * S);
    if (!live || !id) { free(st); free(loff); free(live); free(id); matcher_free(&M); return OR_E_NOMEM; }
    for (int i = loff[n]; i < S; i++) live[i] = 1;
    for (int p = n - 1; p >= 0; p--)
        for (int i = loff[p]; i < loff[p + 1]; i++)
            for (int x = 0; x < 4 && !live[i]; x++) {
                int e = T->out[st[i].q * 4 + x];
                if (e < 0) continue;
                int m2 = M.delta[st[i].m * 4 + x];
                if (m2 < 0) continue;
                pq_t key = {T->edst[e], m2};
                pq_t *hit = bsearch(&key, st + loff[p + 1], loff[p + 2] - loff[p + 1], sizeof(pq_t), pq_cmp);
                if (hit && live[hit - st]) live[i] = 1;
            }
    if (!live[0]) {
        free(st); free(loff); free(live); free(id); matcher_free(&M);
        return OR_E_INFEASIBLE;
    }
    int N = 0;
    for (int i = 0; i < S; i++) id[i] = live[i] ? N++ : -1;
    D->A = T->A;
    D->n = n;
    D->N = N;
    D->layer = malloc(sizeof(int) * N);
    D->off = malloc(sizeof(int) * (n + 2));
    int maxE = 4 * N;
    D->esrc = malloc(sizeof(int) * maxE);
    D->edst = malloc(sizeof(int) * maxE);
    D->elab = malloc(sizeof(int) * maxE);
    D->ecod = malloc(sizeof(int) * maxE);
    D->eq = malloc(sizeof(double) * maxE);
    if (!D->layer || !D->off || !D->esrc || !D->edst || !D->elab || !D->ecod || !D->eq) {
        free(st); free(loff); free(live); free(id); matcher_free(&M);
        return OR_E_NOMEM;
    }
    int E = 0;
    for (int p = 0; p <= n; p++) {
        D->off[p] = N;
        for (int i = loff[p]; i < loff[p + 1]; i++)
            if (live[i]) {
                if (D->off[p] == N) D->off[p] = id[i];
                D->layer[id[i]] = p;
            }
    }
    D->off[n + 1] = N;
    for (int p = n; p >= 0; p--) /* empty layers cannot occur, but keep off monotone anyway */
        if (D->off[p] > D->off[p + 1]) D->off[p] = D->off[p + 1];
    for (int p = 0; p < n; p++)
        for (int i = loff[p]; i < loff[p + 1]; i++) {
            if (!live[i]) continue;
            for (int x = 0; x < 4; x++) {
                int e = T->out[st[i].q * 4 + x];
                if (e < 0) continue;
                int m2 = M.delta[st[i].m * 4 + x];
                if (m2 < 0) continue;
                pq_t key = {T->edst[e], m2};
                pq_t *hit = bsearch(&key, st + loff[p + 1], loff[p + 2] - loff[p + 1], sizeof(pq_t), pq_cmp);
                if (!hit || !live[hit - st]) continue;
                D->esrc[E] = id[i];
                D->edst[E] = id[hit - st];
                D->elab[E] = x;
                D->ecod[E] = T->ecod[e];
                D->eq[E] = T->eq[e];
                E++;
            }
        }
    D->nE = E;
    (void)K;
    free(st); free(loff); free(live); free(id);
    matcher_free(&M);
    return finish_dfa(D);
}

/* Range rule for the fixed-point shift.  Every finite DP value is E*2^s + U for a partial design:
 * U is the rounded cost of some of the path's codons (0 <= U <= sum_k max_c U_k) and E is the
 * energy of a partial structure on at most n nucleotides.  Each pair of such a structure closes
 * exactly one loop (hairpin, stack / bulge / interior loop, or a multiloop with its closing
 * terms) and is at most one branch (of a multiloop: ML_intern + AU; of the exterior loop: AU);
 * every other multiloop term is ML_base per unpaired base.  With at most floor(n/2) pairs,
 *     floor(n/2) * (min(0, Lmin) + Bmin) + n * min(0, ML_base)  <=  E
 *     E  <=  floor(n/2) * (max(0, Lmax) + Bmax) + n * max(0, ML_base)
 * where [Lmin, Lmax] bounds the energy of one loop and [Bmin, Bmax] one branch term, both read
 * off the parameter tables (loop_bounds below).  The shift is the largest s in [16, 40] with
 *     sum_k max_c U_k(s) + max(|E lower bound|, E upper bound) * 2^s  <  2^60,
 * so every finite value lies in (-2^60, 2^60), far from OR_INF = 2^62. */
static int64_t mn64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t mx64(int64_t a, int64_t b) { return a > b ? a : b; }

static void tab_range(const int32_t *t, int cnt, int64_t *lo, int64_t *hi) {
    for (int i = 0; i < cnt; i++) {
        *lo = mn64(*lo, t[i]);
        *hi = mx64(*hi, t[i]);
    }
}

/* [Lmin, Lmax]: energy of one loop closed by a pair, on a design of n nucleotides */
static void loop_bounds(const or_params *P, int n, int64_t *Lmin, int64_t *Lmax) {
    const int64_t au_lo = mn64(0, P->terminal_au), au_hi = mx64(0, P->terminal_au);
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    /* hairpins of every size 3..n: initiation plus a terminal AU (size 3) or a mismatch */
    int64_t mh_lo = 0, mh_hi = 0, init_lo = INT64_MAX, init_hi = INT64_MIN;
    tab_range(&P->mmH[0][0][0], 96, &mh_lo, &mh_hi);
    for (int m = 3; m <= (n > 3 ? n : 3); m++) {
        int64_t e = or_loop_init(P->hairpin, P->lxc, m);
        init_lo = mn64(init_lo, e);
        init_hi = mx64(init_hi, e);
    }
    lo = mn64(lo, init_lo + mn64(au_lo, mh_lo));
    hi = mx64(hi, init_hi + mx64(au_hi, mh_hi));
    for (int k = 0; k < 3; k++) tab_range(P->spec_e[k], P->nspec[k], &lo, &hi); /* listed totals */
    /* stacks and bulges */
    int64_t st_lo = INT64_MAX, st_hi = INT64_MIN;
    tab_range(&P->stack[0][0], 36, &st_lo, &st_hi);
    lo = mn64(lo, st_lo);
    hi = mx64(hi, st_hi);
    lo = mn64(lo, P->bulge[1] + st_lo);
    hi = mx64(hi, P->bulge[1] + st_hi);
    for (int l = 2; l <= 30; l++) {
        lo = mn64(lo, P->bulge[l] + 2 * au_lo);
        hi = mx64(hi, P->bulge[l] + 2 * au_hi);
    }
    /* interior loops: full tables, and initiation + asymmetry + two mismatches */
    tab_range(&P->int11[0][0][0][0], 576, &lo, &hi);
    tab_range(&P->int21[0][0][0][0][0], 2304, &lo, &hi);
    tab_range(&P->int22[0][0][0][0][0][0], 9216, &lo, &hi);
    int64_t mi_lo = 0, mi_hi = 0;
    tab_range(&P->mmI[0][0][0], 96, &mi_lo, &mi_hi);
    tab_range(&P->mm1n[0][0][0], 96, &mi_lo, &mi_hi);
    tab_range(&P->mm23[0][0][0], 96, &mi_lo, &mi_hi);
    const int64_t asym_lo = mn64(0, mn64(P->ninio_max, 28 * (int64_t)P->ninio));
    const int64_t asym_hi = mx64(0, P->ninio_max);
    for (int l = 2; l <= 30; l++) {
        lo = mn64(lo, P->interior[l] + asym_lo + 2 * mi_lo);
        hi = mx64(hi, P->interior[l] + asym_hi + 2 * mi_hi);
    }
    /* multiloop closing pair */
    lo = mn64(lo, (int64_t)P->ml_closing + P->ml_intern + au_lo);
    hi = mx64(hi, (int64_t)P->ml_closing + P->ml_intern + au_hi);
    *Lmin = lo;
    *Lmax = hi;
}

/* Energy bound of the range rule: max(|E lower bound|, E upper bound) for n nucleotides. */
static int64_t energy_bound(const or_params *P, int n) {
    int64_t Lmin, Lmax;
    loop_bounds(P, n, &Lmin, &Lmax);
    const int64_t au_lo = mn64(0, P->terminal_au), au_hi = mx64(0, P->terminal_au);
    const int64_t br_lo = mn64(0, mn64(P->ml_intern + au_lo, au_lo));
    const int64_t br_hi = mx64(0, mx64(P->ml_intern + au_hi, au_hi));
    const int64_t pairs = n / 2;
    const int64_t e_lo = pairs * (mn64(0, Lmin) + br_lo) + (int64_t)n * mn64(0, P->ml_base);
    const int64_t e_hi = pairs * (mx64(0, Lmax) + br_hi) + (int64_t)n * mx64(0, P->ml_base);
    return mx64(-e_lo, e_hi);
}

static int choose_shift(const dfa_t *D, const or_params *P, double lam100) {
    const int64_t ebound = energy_bound(P, D->n);
    int64_t *mx = calloc(D->A + 1, sizeof(int64_t));
    if (!mx) return OR_E_NOMEM;
    int chosen = OR_E_RANGE;
    for (int s = 40; s >= 16; s--) {
        memset(mx, 0, sizeof(int64_t) * (D->A + 1));
        int too_big = 0;
        for (int e = 0; e < D->nE; e++) {
            if (D->ecod[e] < 0) continue;
            double x = ldexp(lam100 * D->eq[e], s);
            if (!(x < 0x1p60)) { /* one codon alone breaks the rule (llround would overflow) */
                too_big = 1;
                break;
            }
            int64_t u = llround(x);
            int k = D->layer[D->esrc[e]] / 3;
            if (u > mx[k]) mx[k] = u;
        }
        if (too_big) continue;
        __int128 tot = 0;
        for (int k = 0; k < D->A; k++) tot += mx[k];
        tot += (__int128)ebound * ((__int128)1 << s);
        if (tot < ((__int128)1 << 60)) {
            chosen = s;
            break;
        }
    }
    free(mx);
    return chosen;
}

static void set_costs(dfa_t *D, const or_params *P, double lam100, int s) {
    for (int e = 0; e < D->nE; e++) {
        D->eU[e] = D->ecod[e] >= 0 ? llround(ldexp(lam100 * D->eq[e], s)) : 0;
        D->eu_ml[e] = D->eU[e] + ((int64_t)P->ml_base << s);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Dense multiloop recurrences, one cell (eqs. 3-5).  Shared by the design DP and the abstract  */
/* DAG entry point so that the same code is pinned by brute-force path enumeration.             */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int N;
    const int *layer;
    const int *esrc, *edst;
    const int64_t *eu;
    const int *in_start, *in_e, *out_start, *out_e;
} mlg_t;

static void ml_cell(const mlg_t *G, int a, int b, const int64_t *B, int64_t *D1, int64_t *D2,
                    int64_t *PD) {
    size_t N = (size_t)G->N;
    int la = G->layer[a], lb = G->layer[b];
    int64_t d2 = OR_INF;
    for (int i = G->in_start[b]; i < G->in_start[b + 1]; i++) {
        int e = G->in_e[i], bp = G->esrc[e];
        if (G->layer[bp] > la) d2 = mn(d2, sat(D2[a * N + bp], G->eu[e]));
    }
    for (int c = 0; c < G->N; c++) {
        int lc = G->layer[c];
        if (lc <= la || lc >= lb) continue;
        d2 = mn(d2, sat(D1[a * N + c], B[c * N + b]));
    }
    D2[a * N + b] = d2;
    int64_t pd = d2;
    for (int i = G->out_start[a]; i < G->out_start[a + 1]; i++) {
        int e = G->out_e[i], ap = G->edst[e];
        if (G->layer[ap] < lb) pd = mn(pd, sat(G->eu[e], D1[ap * N + b]));
    }
    for (int i = G->in_start[b]; i < G->in_start[b + 1]; i++) {
        int e = G->in_e[i], bp = G->esrc[e];
        if (G->layer[bp] > la) pd = mn(pd, sat(D1[a * N + bp], G->eu[e]));
    }
    PD[a * N + b] = pd;
    D1[a * N + b] = mn(B[a * N + b], pd);
}

int or_multiloop_dense(int N, const int *layer, int nE, const int *esrc, const int *edst,
                       const int64_t *eu, const int64_t *B, int64_t *D1, int64_t *D2, int64_t *PD) {
    if (N <= 0 || !layer || !B || !D1 || !D2 || !PD || nE < 0) return OR_E_ARG;
    for (int e = 0; e < nE; e++)
        if (layer[edst[e]] != layer[esrc[e]] + 1) return OR_E_ARG;
    int *in_start = calloc(N + 1, sizeof(int)), *out_start = calloc(N + 1, sizeof(int));
    int *in_e = malloc(sizeof(int) * (nE + 1)), *out_e = malloc(sizeof(int) * (nE + 1));
    int *fi = calloc(N, sizeof(int)), *fo = calloc(N, sizeof(int));
    for (int e = 0; e < nE; e++) {
        in_start[edst[e] + 1]++;
        out_start[esrc[e] + 1]++;
    }
    for (int v = 0; v < N; v++) {
        in_start[v + 1] += in_start[v];
        out_start[v + 1] += out_start[v];
    }
    for (int e = 0; e < nE; e++) {
        in_e[in_start[edst[e]] + fi[edst[e]]++] = e;
        out_e[out_start[esrc[e]] + fo[esrc[e]]++] = e;
    }
    mlg_t G = {N, layer, esrc, edst, eu, in_start, in_e, out_start, out_e};
    size_t NN = (size_t)N * N;
    for (size_t i = 0; i < NN; i++) D1[i] = D2[i] = PD[i] = OR_INF;
    int maxl = 0;
    for (int v = 0; v < N; v++) maxl = layer[v] > maxl ? layer[v] : maxl;
    for (int g = 1; g <= maxl; g++)
        for (int a = 0; a < N; a++)
            for (int b = 0; b < N; b++)
                if (layer[b] - layer[a] == g) ml_cell(&G, a, b, B, D1, D2, PD);
    free(in_start); free(out_start); free(in_e); free(out_e); free(fi); free(fo);
    return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* DP context                                                                                  */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    const or_params *P;
    dfa_t D;
    int s;
    size_t N;
    int64_t *G;                /* min path cost between states, N*N */
    int64_t *V;                /* 6*N*N typed closed values */
    int64_t *B, *D1, *D2, *PD; /* N*N */
    int64_t *X;                /* N */
    mlg_t mg;
    int wmax;                  /* widest layer */
    int segmax;                /* bound on the loop segments between two states (4 x in-degree) */
} dp_t;

#define IDX(a, b) ((size_t)(a) * C->N + (size_t)(b))
#define VV(t, a, b) C->V[(size_t)(t) * C->N * C->N + IDX(a, b)]
#define EN(x) ((int64_t)(x) * ((int64_t)1 << C->s))

static void fill_gap(dp_t *C) {
    const dfa_t *D = &C->D;
    for (size_t i = 0; i < C->N * C->N; i++) C->G[i] = OR_INF;
#pragma omp parallel for schedule(dynamic, 16)
    for (int a = 0; a < D->N; a++) {
        C->G[IDX(a, a)] = 0;
        for (int u = a; u < D->N; u++) {
            int64_t gu = C->G[IDX(a, u)];
            if (gu >= OR_INF) continue;
            for (int i = D->out_start[u]; i < D->out_start[u + 1]; i++) {
                int e = D->out_e[i];
                int64_t v = gu + D->eU[e];
                if (v < C->G[IDX(a, D->edst[e])]) C->G[IDX(a, D->edst[e])] = v;
            }
        }
    }
}

/* --- traceback record ------------------------------------------------------------------- */
typedef struct {
    int *seq, *pair;
    int64_t E, U;
    int ok;
} tb_t;

static void emit_edge(const dp_t *C, tb_t *T, int e) {
    int p = C->D.layer[C->D.esrc[e]];
    if (T->seq[p] >= 0) T->ok = 0; /* every position is emitted exactly once */
    T->seq[p] = C->D.elab[e];
    T->U += C->D.eU[e];
}

/* canonical minimum-cost path u -> v: smallest label whose edge stays on a minimum path */
static void emit_gpath(const dp_t *C, tb_t *T, int u, int v) {
    const dfa_t *D = &C->D;
    while (u != v) {
        int64_t g = C->G[IDX(u, v)];
        int took = 0;
        for (int x = 0; x < 4 && !took; x++) {
            int e = D->out[u * 4 + x];
            if (e < 0) continue;
            if (sat(D->eU[e], C->G[IDX(D->edst[e], v)]) == g) {
                emit_edge(C, T, e);
                u = D->edst[e];
                took = 1;
            }
        }
        if (!took) {
            T->ok = 0;
            return;
        }
    }
}

/* --- hairpin closure ---------------------------------------------------------------------- */
typedef struct {
    const dp_t *C;
    int a, b, len, t;
    int lab[10], edge[10];
    int64_t best, target;
    int trace, found;
    int fe[10];
    int32_t fE;
} hp_enum_t;

static void hp_dfs(hp_enum_t *H, int pos, int state, int64_t cost) {
    const dfa_t *D = &H->C->D;
    if (H->found) return;
    if (pos == H->len) {
        if (state != H->b) return;
        int32_t e = or_hairpin_energy(H->C->P, H->lab, H->len);
        if (e >= OR_EINF) return;
        int64_t v = cost + (int64_t)e * ((int64_t)1 << H->C->s);
        if (!H->trace) {
            if (v < H->best) H->best = v;
        } else if (v == H->target) {
            H->found = 1;
            memcpy(H->fe, H->edge, sizeof(H->edge));
            H->fE = e;
        }
        return;
    }
    for (int x = 0; x < 4; x++) {
        if (pos == 0 && x != TX[H->t]) continue;
        if (pos == H->len - 1 && x != TY[H->t]) continue;
        int e = D->out[state * 4 + x];
        if (e < 0) continue;
        H->lab[pos] = x;
        H->edge[pos] = e;
        hp_dfs(H, pos + 1, D->edst[e], cost + D->eU[e]);
        if (H->found) return;
    }
}

/* Hairpin alternatives in canonical order.  T == NULL: return the minimum.  Otherwise stop at
 * the first alternative equal to target, emit it into T and return target (OR_INF if none). */
static int64_t hairpin_scan(const dp_t *C, int a, int b, int t, int64_t target, tb_t *T) {
    const dfa_t *D = &C->D;
    int g = D->layer[b] - D->layer[a], m = g - 2;
    if (m < 3) return OR_INF;
    int ea = D->out[a * 4 + TX[t]];
    if (ea < 0) return OR_INF;
    if (m == 3 || m == 4 || m == 6) {
        hp_enum_t H;
        memset(&H, 0, sizeof(H));
        H.C = C; H.a = a; H.b = b; H.len = g; H.t = t; H.best = OR_INF; H.target = target;
        H.trace = T != NULL;
        hp_dfs(&H, 0, a, 0);
        if (!T) return H.best;
        if (!H.found) return OR_INF;
        for (int i = 0; i < g; i++) emit_edge(C, T, H.fe[i]);
        T->E += H.fE;
        return target;
    }
    int a1 = D->edst[ea];
    int64_t best = OR_INF;
    for (int x2 = 0; x2 < 4; x2++) {
        int e1 = D->out[a1 * 4 + x2];
        if (e1 < 0) continue;
        int a2 = D->edst[e1];
        for (int i = D->in_start[b]; i < D->in_start[b + 1]; i++) {
            int eb = D->in_e[i];
            if (D->elab[eb] != TY[t]) continue;
            int b1 = D->esrc[eb];
            for (int j = D->in_start[b1]; j < D->in_start[b1 + 1]; j++) {
                int eb2 = D->in_e[j], b2 = D->esrc[eb2];
                int64_t gg = C->G[IDX(a2, b2)];
                if (gg >= OR_INF) continue;
                int32_t en = or_hairpin_generic(C->P, t, m, x2, D->elab[eb2]);
                if (en >= OR_EINF) continue;
                int64_t v = D->eU[ea] + D->eU[e1] + gg + D->eU[eb2] + D->eU[eb] + EN(en);
                if (!T) {
                    best = mn(best, v);
                } else if (v == target) {
                    emit_edge(C, T, ea);
                    emit_edge(C, T, e1);
                    emit_gpath(C, T, a2, b2);
                    emit_edge(C, T, eb2);
                    emit_edge(C, T, eb);
                    T->E += en;
                    return target;
                }
            }
        }
    }
    return !T ? best : OR_INF;
}

/* --- two-loop closure (stack, bulge, interior; l1 + l2 <= 30) ----------------------------- */
typedef struct {
    int e1, e2;     /* edges of the segment (-1 if unused) */
    int mid_from, mid_to; /* G path endpoints for length >= 2 */
    int xa, xb;     /* boundary labels */
    int64_t cost;
} seg_t;

/* left segment a1 ~> c with l unpaired bases; labels (x_{i+1}, x_{k-1}) */
static int left_segs(const dp_t *C, int a1, int c, int l, seg_t *out) {
    const dfa_t *D = &C->D;
    int k = 0;
    if (l == 0) {
        if (c != a1) return 0;
        out[0] = (seg_t){-1, -1, -1, -1, -1, -1, 0};
        return 1;
    }
    if (l == 1) {
        for (int x = 0; x < 4; x++) {
            int e = D->out[a1 * 4 + x];
            if (e >= 0 && D->edst[e] == c) out[k++] = (seg_t){e, -1, -1, -1, x, x, D->eU[e]};
        }
        return k;
    }
    for (int x = 0; x < 4; x++) {
        int e1 = D->out[a1 * 4 + x];
        if (e1 < 0) continue;
        int a2 = D->edst[e1];
        for (int i = D->in_start[c]; i < D->in_start[c + 1]; i++) {
            int e2 = D->in_e[i], c1 = D->esrc[e2];
            int64_t gg = C->G[IDX(a2, c1)];
            if (gg >= OR_INF) continue;
            out[k++] = (seg_t){e1, e2, a2, c1, x, D->elab[e2], D->eU[e1] + gg + D->eU[e2]};
        }
    }
    return k;
}

/* right segment d ~> b1 with l unpaired bases; labels (x_{l+1}, x_{j-1}) */
static int right_segs(const dp_t *C, int d, int b1, int l, seg_t *out) {
    return left_segs(C, d, b1, l, out);
}

static void emit_seg(const dp_t *C, tb_t *T, const seg_t *s) {
    if (s->e1 >= 0) emit_edge(C, T, s->e1);
    if (s->e2 >= 0) {
        emit_gpath(C, T, s->mid_from, s->mid_to);
        emit_edge(C, T, s->e2);
    }
}

typedef struct {
    int c, d, tp;
} tl_pick_t;

static int64_t twoloop_scan(const dp_t *C, int a, int b, int t, int64_t target, tb_t *T,
                            tl_pick_t *pick) {
    const dfa_t *D = &C->D;
    int la = D->layer[a], lb = D->layer[b];
    int ea = D->out[a * 4 + TX[t]];
    if (ea < 0) return OR_INF;
    int a1 = D->edst[ea];
    int64_t best = OR_INF;
    seg_t Ls[C->segmax], Rs[C->segmax];
    for (int l1 = 0; l1 <= 30; l1++)
        for (int l2 = 0; l1 + l2 <= 30; l2++) {
            int lc = la + 1 + l1, ld = lb - 1 - l2;
            if (ld - lc < 5) continue;
            for (int i = D->in_start[b]; i < D->in_start[b + 1]; i++) {
                int eb = D->in_e[i];
                if (D->elab[eb] != TY[t]) continue;
                int b1 = D->esrc[eb];
                for (int c = D->off[lc]; c < D->off[lc + 1]; c++) {
                    int nl = left_segs(C, a1, c, l1, Ls);
                    if (!nl) continue;
                    for (int d = D->off[ld]; d < D->off[ld + 1]; d++) {
                        int nr = -1;
                        for (int tp = 0; tp < 6; tp++) {
                            int64_t vin = VV(tp, c, d);
                            if (vin >= OR_INF) continue;
                            int tr = or_pair_type(TY[tp], TX[tp]);
                            if (nr < 0) nr = right_segs(C, d, b1, l2, Rs);
                            for (int p = 0; p < nl; p++)
                                for (int q = 0; q < nr; q++) {
                                    int32_t e2 = or_two_loop_energy(C->P, t, tr, l1, l2, Ls[p].xa,
                                                                    Ls[p].xb, Rs[q].xa, Rs[q].xb);
                                    if (e2 >= OR_EINF) continue;
                                    int64_t v = D->eU[ea] + Ls[p].cost + vin + Rs[q].cost +
                                                D->eU[eb] + EN(e2);
                                    if (!T) {
                                        best = mn(best, v);
                                    } else if (v == target) {
                                        emit_edge(C, T, ea);
                                        emit_seg(C, T, &Ls[p]);
                                        emit_seg(C, T, &Rs[q]);
                                        emit_edge(C, T, eb);
                                        T->E += e2;
                                        pick->c = c; pick->d = d; pick->tp = tp;
                                        return target;
                                    }
                                }
                        }
                    }
                }
            }
        }
    return !T ? best : OR_INF;
}

/* --- multiloop closure: (ML_closing + ML_intern + AU(t)) + D2 of the interior ------------- */
static int64_t multiloop_scan(const dp_t *C, int a, int b, int t, int64_t target, tb_t *T,
                              int *pa1, int *pb1) {
    const dfa_t *D = &C->D;
    int ea = D->out[a * 4 + TX[t]];
    if (ea < 0) return OR_INF;
    int a1 = D->edst[ea];
    int32_t mlc = C->P->ml_closing + C->P->ml_intern + or_au(C->P, t);
    int64_t best = OR_INF;
    for (int i = D->in_start[b]; i < D->in_start[b + 1]; i++) {
        int eb = D->in_e[i];
        if (D->elab[eb] != TY[t]) continue;
        int b1 = D->esrc[eb];
        if (D->layer[b1] - D->layer[a1] < 10) continue;
        int64_t v = sat(D->eU[ea] + D->eU[eb] + EN(mlc), C->D2[IDX(a1, b1)]);
        if (!T) {
            best = mn(best, v);
        } else if (v == target) {
            emit_edge(C, T, ea);
            emit_edge(C, T, eb);
            T->E += mlc;
            *pa1 = a1;
            *pb1 = b1;
            return target;
        }
    }
    return !T ? best : OR_INF;
}

static void fill_cell(dp_t *C, int a, int b) {
    const dfa_t *D = &C->D;
    int g = D->layer[b] - D->layer[a];
    int64_t bb = OR_INF;
    if (g >= 5) {
        for (int t = 0; t < 6; t++) {
            int64_t v = hairpin_scan(C, a, b, t, -1, NULL);
            v = mn(v, twoloop_scan(C, a, b, t, -1, NULL, NULL));
            if (g >= 12) v = mn(v, multiloop_scan(C, a, b, t, -1, NULL, NULL, NULL));
            VV(t, a, b) = v;
            bb = mn(bb, sat(v, EN(C->P->ml_intern + or_au(C->P, t))));
        }
    }
    C->B[IDX(a, b)] = bb;
    ml_cell(&C->mg, a, b, C->B, C->D1, C->D2, C->PD);
}

/* --- traceback ---------------------------------------------------------------------------- */
enum { F_X, F_V, F_S1, F_S2, F_BR };
typedef struct {
    int kind, a, b, t;
} frame_t;

static int cand(const dp_t *C, int c, int b) { return C->B[IDX(c, b)] < C->PD[IDX(c, b)]; }

static int traceback(dp_t *C, tb_t *T) {
    const dfa_t *D = &C->D;
    const or_params *P = C->P;
    int cap = 4 * D->n + 64, sp = 0;
    frame_t *st = malloc(sizeof(frame_t) * cap);
    if (!st) return OR_E_NOMEM;
    st[sp++] = (frame_t){F_X, 0, -1, -1};
    while (sp > 0) {
        frame_t f = st[--sp];
        if (sp + 4 >= cap) {
            cap *= 2;
            st = realloc(st, sizeof(frame_t) * cap);
        }
        int a = f.a, b = f.b;
        if (f.kind == F_X) {
            if (D->layer[a] == D->n) continue;
            int64_t x = C->X[a];
            int done = 0;
            for (int i = D->out_start[a]; i < D->out_start[a + 1] && !done; i++) {
                int e = D->out_e[i];
                if (sat(D->eU[e], C->X[D->edst[e]]) == x) {
                    emit_edge(C, T, e);
                    st[sp++] = (frame_t){F_X, D->edst[e], -1, -1};
                    done = 1;
                }
            }
            int b0 = D->layer[a] + 5 <= D->n ? D->off[D->layer[a] + 5] : D->N;
            for (int bb = b0; bb < D->N && !done; bb++)
                for (int t = 0; t < 6 && !done; t++)
                    if (sat(sat(VV(t, a, bb), EN(or_au(P, t))), C->X[bb]) == x) {
                        T->E += or_au(P, t);
                        st[sp++] = (frame_t){F_X, bb, -1, -1};
                        st[sp++] = (frame_t){F_V, a, bb, t};
                        done = 1;
                    }
            if (!done) T->ok = 0;
        } else if (f.kind == F_V) {
            int64_t v = VV(f.t, a, b);
            int i = D->layer[a], j = D->layer[b] - 1;
            T->pair[i] = j;
            T->pair[j] = i;
            if (hairpin_scan(C, a, b, f.t, v, T) == v) continue;
            tl_pick_t pk;
            if (twoloop_scan(C, a, b, f.t, v, T, &pk) == v) {
                st[sp++] = (frame_t){F_V, pk.c, pk.d, pk.tp};
                continue;
            }
            int a1, b1;
            if (D->layer[b] - D->layer[a] >= 12 && multiloop_scan(C, a, b, f.t, v, T, &a1, &b1) == v) {
                st[sp++] = (frame_t){F_S2, a1, b1, -1};
                continue;
            }
            T->ok = 0;
        } else if (f.kind == F_BR) {
            int64_t v = C->B[IDX(a, b)];
            int done = 0;
            for (int t = 0; t < 6 && !done; t++) {
                int32_t beta = P->ml_intern + or_au(P, t);
                if (sat(VV(t, a, b), EN(beta)) == v) {
                    T->E += beta;
                    st[sp++] = (frame_t){F_V, a, b, t};
                    done = 1;
                }
            }
            if (!done) T->ok = 0;
        } else if (f.kind == F_S1) {
            int64_t v = C->D1[IDX(a, b)];
            if (C->B[IDX(a, b)] == v) {
                st[sp++] = (frame_t){F_BR, a, b, -1};
                continue;
            }
            if (C->D2[IDX(a, b)] == v) {
                st[sp++] = (frame_t){F_S2, a, b, -1};
                continue;
            }
            int done = 0;
            for (int i = D->out_start[a]; i < D->out_start[a + 1] && !done; i++) {
                int e = D->out_e[i], ap = D->edst[e];
                if (D->layer[ap] < D->layer[b] && sat(D->eu_ml[e], C->D1[IDX(ap, b)]) == v) {
                    emit_edge(C, T, e);
                    T->E += P->ml_base;
                    st[sp++] = (frame_t){F_S1, ap, b, -1};
                    done = 1;
                }
            }
            for (int i = D->in_start[b]; i < D->in_start[b + 1] && !done; i++) {
                int e = D->in_e[i], bp = D->esrc[e];
                if (D->layer[bp] > D->layer[a] && sat(C->D1[IDX(a, bp)], D->eu_ml[e]) == v) {
                    emit_edge(C, T, e);
                    T->E += P->ml_base;
                    st[sp++] = (frame_t){F_S1, a, bp, -1};
                    done = 1;
                }
            }
            if (!done) T->ok = 0;
        } else { /* F_S2 */
            int64_t v = C->D2[IDX(a, b)];
            int done = 0;
            for (int i = D->in_start[b]; i < D->in_start[b + 1] && !done; i++) {
                int e = D->in_e[i], bp = D->esrc[e];
                if (D->layer[bp] > D->layer[a] && sat(C->D2[IDX(a, bp)], D->eu_ml[e]) == v) {
                    emit_edge(C, T, e);
                    T->E += P->ml_base;
                    st[sp++] = (frame_t){F_S2, a, bp, -1};
                    done = 1;
                }
            }
            /* candidates c in C_b with rho(c) > rho(a), by state index (eq. 7 alternatives) */
            for (int c = D->off[D->layer[a] + 1]; c < D->off[D->layer[b]] && !done; c++) {
                if (!cand(C, c, b)) continue;
                if (sat(C->D1[IDX(a, c)], C->B[IDX(c, b)]) == v) {
                    st[sp++] = (frame_t){F_S1, a, c, -1};
                    st[sp++] = (frame_t){F_BR, c, b, -1};
                    done = 1;
                }
            }
            if (!done) T->ok = 0;
        }
    }
    free(st);
    return OR_OK;
}

static int setup(dp_t *C, const char *protein, const double *w, const or_params *P, double lambda,
                 const char *const *motifs, int nm) {
    memset(C, 0, sizeof(*C));
    int rc = check_protein(protein);
    if (rc) return rc;
    if (!P) return OR_E_ARG;
    if (!(lambda >= 0.0) || !isfinite(lambda)) return OR_E_LAMBDA;
    rc = check_codons(protein, w);
    if (rc) return rc;
    C->P = P;
    rc = build_dfa(protein, w, &C->D);
    if (rc) return rc;
    double lam100 = 100.0 * lambda;
    C->s = choose_shift(&C->D, P, lam100);
    if (C->s < 0) return OR_E_RANGE;
    if (nm > 0) {
        if (!motifs || nm > OR_MAX_MOTIFS) return OR_E_ARG;
        dfa_t prod;
        rc = build_product(&C->D, motifs, nm, &prod);
        dfa_free(&C->D);
        C->D = prod;
        if (rc) return rc;
    } else if (nm < 0) {
        return OR_E_ARG;
    }
    set_costs(&C->D, P, lam100, C->s);
    C->wmax = 1;
    for (int p = 0; p <= C->D.n; p++)
        if (C->D.off[p + 1] - C->D.off[p] > C->wmax) C->wmax = C->D.off[p + 1] - C->D.off[p];
    int maxin = 1;
    for (int v = 0; v < C->D.N; v++)
        if (C->D.in_start[v + 1] - C->D.in_start[v] > maxin) maxin = C->D.in_start[v + 1] - C->D.in_start[v];
    C->segmax = 4 * maxin + 4;
    C->N = (size_t)C->D.N;
    C->mg = (mlg_t){C->D.N, C->D.layer, C->D.esrc, C->D.edst, C->D.eu_ml,
                    C->D.in_start, C->D.in_e, C->D.out_start, C->D.out_e};
    return OR_OK;
}

static void teardown(dp_t *C) {
    free(C->G); free(C->V); free(C->B); free(C->D1); free(C->D2); free(C->PD); free(C->X);
    dfa_free(&C->D);
}

int or_fixed_shift(const char *protein, const double w[64], const or_params *P, double lambda) {
    dp_t C;
    int rc = setup(&C, protein, w, P, lambda, NULL, 0);
    int s = rc ? rc : C.s;
    teardown(&C);
    return s;
}

int or_lattice_stats(const char *protein, int64_t *n_states, int64_t *n_edges, int64_t *n_cells,
                     int64_t *n_feasible) {
    int rc = check_protein(protein);
    if (rc) return rc;
    double w[64];
    for (int i = 0; i < 64; i++) w[i] = 1.0;
    dfa_t D;
    rc = build_dfa(protein, w, &D);
    if (rc) {
        dfa_free(&D);
        return rc;
    }
    int64_t cells = 0, feas = 0;
    for (int a = 0; a < D.N; a++) {
        cells += D.N - D.off[D.layer[a] + 1];
        for (int b = D.off[D.layer[a] + 1]; b < D.N; b++) {
            if (D.layer[b] - D.layer[a] < 5) continue;
            int ok = 0;
            for (int i = D.out_start[a]; i < D.out_start[a + 1] && !ok; i++)
                for (int j = D.in_start[b]; j < D.in_start[b + 1] && !ok; j++)
                    if (or_pair_type(D.elab[D.out_e[i]], D.elab[D.in_e[j]]) >= 0) ok = 1;
            feas += ok;
        }
    }
    if (n_states) *n_states = D.N;
    if (n_edges) *n_edges = D.nE;
    if (n_cells) *n_cells = cells;
    if (n_feasible) *n_feasible = feas;
    dfa_free(&D);
    return OR_OK;
}

static int design_impl(const char *protein, const double w[64], const or_params *P, double lambda,
                       const char *const *motifs, int nm, int nthreads, char *mrna, char *structure,
                       or_result *res, int64_t *dbg_V, int64_t *dbg_B, int64_t *dbg_D1,
                       int64_t *dbg_D2, int64_t *dbg_X) {
    if (!mrna || !structure || !res) return OR_E_ARG;
    memset(res, 0, sizeof(*res));
    dp_t Cx, *C = &Cx;
    int rc = setup(C, protein, w, P, lambda, motifs, nm);
    if (rc) {
        teardown(C);
        return rc;
    }
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const dfa_t *D = &C->D;
    size_t NN = C->N * C->N;
    C->G = malloc(sizeof(int64_t) * NN);
    C->V = malloc(sizeof(int64_t) * NN * 6);
    C->B = malloc(sizeof(int64_t) * NN);
    C->D1 = malloc(sizeof(int64_t) * NN);
    C->D2 = malloc(sizeof(int64_t) * NN);
    C->PD = malloc(sizeof(int64_t) * NN);
    C->X = malloc(sizeof(int64_t) * C->N);
    if (!C->G || !C->V || !C->B || !C->D1 || !C->D2 || !C->PD || !C->X) {
        teardown(C);
        return OR_E_NOMEM;
    }
    for (size_t i = 0; i < NN; i++) C->B[i] = C->D1[i] = C->D2[i] = C->PD[i] = OR_INF;
    for (size_t i = 0; i < 6 * NN; i++) C->V[i] = OR_INF;
    fill_gap(C);
    /* span wavefront: every cell of span g depends only on smaller spans */
    int *ca = malloc(sizeof(int) * C->N * C->wmax), *cb = malloc(sizeof(int) * C->N * C->wmax);
    for (int g = 1; g <= D->n; g++) {
        int nc = 0;
        for (int p = 0; p + g <= D->n; p++)
            for (int a = D->off[p]; a < D->off[p + 1]; a++)
                for (int b = D->off[p + g]; b < D->off[p + g + 1]; b++) {
                    ca[nc] = a;
                    cb[nc++] = b;
                }
#pragma omp parallel for schedule(dynamic, 4)
        for (int i = 0; i < nc; i++) fill_cell(C, ca[i], cb[i]);
    }
    free(ca);
    free(cb);
    /* external column X(a) for fragments a -> t */
    for (int i = 0; i < D->N; i++) C->X[i] = D->layer[i] == D->n ? 0 : OR_INF;
    for (int p = D->n - 1; p >= 0; p--)
        for (int a = D->off[p]; a < D->off[p + 1]; a++) {
            int64_t x = OR_INF;
            for (int i = D->out_start[a]; i < D->out_start[a + 1]; i++) {
                int e = D->out_e[i];
                x = mn(x, sat(D->eU[e], C->X[D->edst[e]]));
            }
            if (p + 5 <= D->n)
                for (int b = D->off[p + 5]; b < D->N; b++)
                    for (int t = 0; t < 6; t++)
                        x = mn(x, sat(sat(VV(t, a, b), EN(or_au(P, t))), C->X[b]));
            C->X[a] = x;
        }
    /* statistics */
    int64_t cells = 0, feas = 0, Z = 0, vd = 0, vs = 0;
    int *cnt = calloc(D->n + 2, sizeof(int));
    for (int b = 0; b < D->N; b++) {
        memset(cnt, 0, sizeof(int) * (D->n + 2));
        for (int c = 0; c < D->off[D->layer[b]]; c++)
            if (cand(C, c, b)) {
                cnt[D->layer[c]]++;
                Z++;
            }
        /* suffix sums: candidates strictly right of layer p */
        int64_t suf = 0;
        for (int p = D->layer[b] - 1; p >= 0; p--) {
            for (int a = D->off[p]; a < D->off[p + 1]; a++) {
                vs += suf;
                vd += D->off[D->layer[b]] - D->off[p + 1];
            }
            suf += cnt[p];
        }
    }
    free(cnt);
    for (int a = 0; a < D->N; a++) {
        cells += D->N - D->off[D->layer[a] + 1];
        for (int b = D->off[D->layer[a] + 1]; b < D->N; b++) feas += C->B[IDX(a, b)] < OR_INF;
    }
    res->n_states = D->N;
    res->n_edges = D->nE;
    res->n_cells = cells;
    res->n_feasible_direct = feas;
    res->n_candidates = Z;
    res->visits_dense = vd;
    res->visits_sparse = vs;
    res->fixed_shift = C->s;
    res->objective_fixed = C->X[0];
    /* canonical traceback */
    tb_t T;
    T.seq = malloc(sizeof(int) * (D->n + 1));
    T.pair = malloc(sizeof(int) * (D->n + 1));
    for (int i = 0; i < D->n; i++) T.seq[i] = T.pair[i] = -1;
    T.E = 0;
    T.U = 0;
    T.ok = C->X[0] < OR_INF;
    if (T.ok) traceback(C, &T);
    /* self-check: full path from s to t, and E*2^s + U == X(s) */
    int state = 0;
    int64_t Uwalk = 0;
    double ccost = 0.0;
    for (int i = 0; i < D->n && T.ok; i++) {
        if (T.seq[i] < 0) {
            T.ok = 0;
            break;
        }
        int e = D->out[state * 4 + T.seq[i]];
        if (e < 0) {
            T.ok = 0;
            break;
        }
        Uwalk += D->eU[e];
        if (D->ecod[e] >= 0) ccost += D->eq[e];
        state = D->edst[e];
    }
    if (D->layer[state] != D->n) T.ok = 0;
    if (T.ok && (Uwalk != T.U || EN(T.E) + T.U != C->X[0])) T.ok = 0;
    for (int i = 0; i < D->n; i++) {
        mrna[i] = T.seq[i] >= 0 ? "ACGU"[T.seq[i]] : 'N';
        structure[i] = T.pair[i] < 0 ? '.' : (T.pair[i] > i ? '(' : ')');
    }
    mrna[D->n] = 0;
    structure[D->n] = 0;
    res->energy = (int32_t)T.E;
    res->path_u = T.U;
    res->codon_cost = ccost;
    res->objective_kcal = (double)T.E / 100.0 + lambda * ccost;
    res->selfcheck_ok = T.ok;
    if (dbg_V) memcpy(dbg_V, C->V, sizeof(int64_t) * NN * 6);
    if (dbg_B) memcpy(dbg_B, C->B, sizeof(int64_t) * NN);
    if (dbg_D1) memcpy(dbg_D1, C->D1, sizeof(int64_t) * NN);
    if (dbg_D2) memcpy(dbg_D2, C->D2, sizeof(int64_t) * NN);
    if (dbg_X) memcpy(dbg_X, C->X, sizeof(int64_t) * C->N);
    free(T.seq);
    free(T.pair);
    teardown(C);
    return T.ok ? OR_OK : OR_E_INTERNAL;
}

int or_design(const char *protein, const double w[64], const or_params *P, double lambda,
              int nthreads, char *mrna, char *structure, or_result *res,
              int64_t *dbg_V, int64_t *dbg_B, int64_t *dbg_D1, int64_t *dbg_D2, int64_t *dbg_X) {
    return design_impl(protein, w, P, lambda, NULL, 0, nthreads, mrna, structure, res, dbg_V, dbg_B,
                       dbg_D1, dbg_D2, dbg_X);
}

int or_design_motifs(const char *protein, const double w[64], const or_params *P, double lambda,
                     const char *const *motifs, int nm, int nthreads, char *mrna, char *structure,
                     or_result *res) {
    if (nm < 1) return OR_E_ARG;
    return design_impl(protein, w, P, lambda, motifs, nm, nthreads, mrna, structure, res, NULL, NULL,
                       NULL, NULL, NULL);
}

int or_design_motifs_tables(const char *protein, const double w[64], const or_params *P, double lambda,
                            const char *const *motifs, int nm, int nthreads, char *mrna, char *structure,
                            or_result *res, int64_t *dbg_V, int64_t *dbg_B, int64_t *dbg_D1,
                            int64_t *dbg_D2, int64_t *dbg_X) {
    if (nm < 1) return OR_E_ARG;
    return design_impl(protein, w, P, lambda, motifs, nm, nthreads, mrna, structure, res, dbg_V, dbg_B,
                       dbg_D1, dbg_D2, dbg_X);
}

int or_motif_lattice(const char *protein, const char *const *motifs, int nm, int64_t *n_states,
                     int64_t *n_edges, int64_t *width, int64_t *n_paths) {
    int rc = check_protein(protein);
    if (rc) return rc;
    if (nm < 1 || nm > OR_MAX_MOTIFS || !motifs) return OR_E_ARG;
    double w[64];
    for (int i = 0; i < 64; i++) w[i] = 1.0;
    dfa_t T, D;
    rc = build_dfa(protein, w, &T);
    if (rc) {
        dfa_free(&T);
        return rc;
    }
    rc = build_product(&T, motifs, nm, &D);
    dfa_free(&T);
    if (rc) {
        dfa_free(&D);
        return rc;
    }
    /* paths from the source, layer by layer (saturating) */
    int64_t *cnt = calloc(D.N, sizeof(int64_t));
    if (!cnt) {
        dfa_free(&D);
        return OR_E_NOMEM;
    }
    cnt[0] = 1;
    int64_t wmax = 0, total = 0;
    for (int p = 0; p <= D.n; p++) {
        if (D.off[p + 1] - D.off[p] > wmax) wmax = D.off[p + 1] - D.off[p];
        for (int u = D.off[p]; u < D.off[p + 1]; u++)
            for (int i = D.out_start[u]; i < D.out_start[u + 1]; i++) {
                int v = D.edst[D.out_e[i]];
                cnt[v] = cnt[v] > INT64_MAX - cnt[u] ? INT64_MAX : cnt[v] + cnt[u];
            }
    }
    for (int u = D.off[D.n]; u < D.N; u++) total = total > INT64_MAX - cnt[u] ? INT64_MAX : total + cnt[u];
    if (n_states) *n_states = D.N;
    if (n_edges) *n_edges = D.nE;
    if (width) *width = wmax;
    if (n_paths) *n_paths = total;
    free(cnt);
    dfa_free(&D);
    return OR_OK;
}
