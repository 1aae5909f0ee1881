/* Oracle: parameter-file loader and loop energies (test infrastructure only).
 *
 * Energy model (Sec. 3): Turner-2004 at 37 C, dangle-0; pairs AU/CG/GU both orientations;
 * hairpins of at least three unpaired bases with special tri/tetra/hexaloops (listed loops take
 * their total listed energy); stacks, bulges and interior loops with full 1x1, 1x2 and 2x2 loop
 * tables; affine multiloops with terminal-pair penalties; no dangles or coaxial stacking.
 *
 * Pair-type order: AU, CG, GC, GU, UA, UG.  Nucleotides A, C, G, U = 0..3.
 * Two-loop convention for outer pair (i,j) of type t and inner pair (k,l): the inner pair is
 * indexed from inside the loop, tr = type(x_l, x_k).
 */
#include <ctype.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

int or_nuc(char c) {
    switch (c) {
        case 'A': return 0;
        case 'C': return 1;
        case 'G': return 2;
        case 'U': return 3;
        default: return -1;
    }
}

int or_pair_type(int x, int y) {
    static const int T[4][4] = {{-1, -1, -1, 0}, {-1, -1, 1, -1}, {-1, 2, -1, 3}, {4, -1, 5, -1}};
    if (x < 0 || y < 0) return -1;
    return T[x][y];
}

/* terminal AU/GU penalty applies to every pair that is not CG or GC */
int32_t or_au(const or_params *P, int t) { return (t == 1 || t == 2) ? 0 : P->terminal_au; }

/* loop initiation for size m; sizes above 30 extrapolate with lxc*ln(m/30), rounded half away
 * from zero (only hairpins reach that range inside the optimisation domain). */
int32_t or_loop_init(const int32_t tab[31], double lxc, int m) {
    if (m < 0) return OR_EINF;
    if (m <= 30) return tab[m];
    if (tab[30] >= OR_EINF) return OR_EINF;
    return tab[30] + (int32_t)lround(lxc * log((double)m / 30.0));
}

static int special_lookup(const or_params *P, const int *seq, int len, int32_t *e) {
    int kind = len == 5 ? 0 : len == 6 ? 1 : len == 8 ? 2 : -1;
    if (kind < 0) return 0;
    char s[10];
    for (int i = 0; i < len; i++) s[i] = "ACGU"[seq[i]];
    s[len] = 0;
    for (int i = 0; i < P->nspec[kind]; i++)
        if (strcmp(P->spec_seq[kind][i], s) == 0) {
            *e = P->spec_e[kind][i];
            return 1;
        }
    return 0;
}

/* hairpin closed by (i,j) with m = len-2 unpaired bases, generic (non-special) part */
int32_t or_hairpin_generic(const or_params *P, int t, int m, int xi1, int xj1) {
    if (m < 3 || t < 0) return OR_EINF;
    int32_t e = or_loop_init(P->hairpin, P->lxc, m);
    if (e >= OR_EINF) return OR_EINF;
    if (m == 3) return e + or_au(P, t);
    return e + P->mmH[t][xi1][xj1];
}

/* hairpin energy of the loop sequence seq[0..len-1] (closing pair included) */
int32_t or_hairpin_energy(const or_params *P, const int *seq, int len) {
    int t = or_pair_type(seq[0], seq[len - 1]);
    int m = len - 2;
    if (t < 0 || m < 3) return OR_EINF;
    int32_t e;
    if ((m == 3 || m == 4 || m == 6) && special_lookup(P, seq, len, &e)) return e;
    return or_hairpin_generic(P, t, m, seq[1], seq[len - 2]);
}

/* stack / bulge / interior loop between outer pair type t and inner type tr (seen from inside),
 * l1 unpaired on the 5' side, l2 on the 3' side.  xi1 = x_{i+1}, xk1 = x_{k-1},
 * xl1 = x_{l+1}, xj1 = x_{j-1} (ignored where the side is empty). */
int32_t or_two_loop_energy(const or_params *P, int t, int tr, int l1, int l2,
                           int xi1, int xk1, int xl1, int xj1) {
    if (t < 0 || tr < 0) return OR_EINF;
    if (l1 == 0 && l2 == 0) return P->stack[t][tr];
    if (l1 == 0 || l2 == 0) {
        int l = l1 + l2;
        int32_t e = or_loop_init(P->bulge, P->lxc, l);
        if (e >= OR_EINF) return OR_EINF;
        if (l == 1) return e + P->stack[t][tr];
        return e + or_au(P, t) + or_au(P, tr);
    }
    if (l1 == 1 && l2 == 1) return P->int11[t][tr][xi1][xj1];
    if (l1 == 1 && l2 == 2) return P->int21[t][tr][xi1][xl1][xj1];
    if (l1 == 2 && l2 == 1) return P->int21[tr][t][xl1][xi1][xk1];
    if (l1 == 2 && l2 == 2) return P->int22[t][tr][xi1][xk1][xl1][xj1];
    int l = l1 + l2;
    int32_t e = or_loop_init(P->interior, P->lxc, l);
    if (e >= OR_EINF) return OR_EINF;
    int d = l1 > l2 ? l1 - l2 : l2 - l1;
    int32_t asym = P->ninio * d;
    if (asym > P->ninio_max) asym = P->ninio_max;
    e += asym;
    if (l1 == 1 || l2 == 1) return e + P->mm1n[t][xi1][xj1] + P->mm1n[tr][xl1][xk1];
    if ((l1 == 2 && l2 == 3) || (l1 == 3 && l2 == 2))
        return e + P->mm23[t][xi1][xj1] + P->mm23[tr][xl1][xk1];
    return e + P->mmI[t][xi1][xj1] + P->mmI[tr][xl1][xk1];
}

/* ------------------------------------------------------------------------------------------ */
/* loader: whitespace-separated tokens; "[section] count" headers                           */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    char *buf;
    char *p;
} tok_t;

static char *next_tok(tok_t *t) {
    for (;;) {
        while (*t->p && isspace((unsigned char)*t->p)) t->p++;
        if (*t->p == '#') { /* comment to end of line */
            while (*t->p && *t->p != '\n') t->p++;
            continue;
        }
        break;
    }
    if (!*t->p) return NULL;
    char *s = t->p;
    while (*t->p && !isspace((unsigned char)*t->p)) t->p++;
    if (*t->p) *t->p++ = 0;
    return s;
}

static int read_ints(tok_t *t, int32_t *dst, int count, int allow_inf) {
    for (int i = 0; i < count; i++) {
        char *s = next_tok(t);
        if (!s) return -1;
        if (allow_inf && strcmp(s, "INF") == 0) {
            dst[i] = OR_EINF;
            continue;
        }
        char *end;
        long v = strtol(s, &end, 10);
        if (*end || v < -100000 || v > 100000) return -1;
        dst[i] = (int32_t)v;
    }
    return 0;
}

static void upd_max(int32_t *m, int32_t v) {
    if (v >= OR_EINF) return;
    int32_t a = v < 0 ? -v : v;
    if (a > *m) *m = a;
}

int or_params_load(const char *path, or_params **out) {
    if (!path || !out) return OR_E_ARG;
    *out = NULL;
    FILE *f = fopen(path, "rb");
    if (!f) return OR_E_PARAMS;
    fseek(f, 0, SEEK_END);
    long sz = ftell(f);
    fseek(f, 0, SEEK_SET);
    if (sz <= 0 || sz > (1 << 24)) {
        fclose(f);
        return OR_E_PARAMS;
    }
    char *buf = (char *)malloc((size_t)sz + 1);
    if (!buf) {
        fclose(f);
        return OR_E_NOMEM;
    }
    size_t got = fread(buf, 1, (size_t)sz, f);
    fclose(f);
    buf[got] = 0;
    or_params *P = (or_params *)calloc(1, sizeof(or_params));
    if (!P) {
        free(buf);
        return OR_E_NOMEM;
    }
    tok_t t = {buf, buf};
    int rc = OR_E_PARAMS, seen = 0;
    char *s = next_tok(&t);
    if (!s || strcmp(s, "SPARSEDESIGN-PARAMS") != 0) goto done;
    s = next_tok(&t);
    if (!s || strcmp(s, "1") != 0) goto done;
    while ((s = next_tok(&t)) != NULL) {
        if (strcmp(s, "[end]") == 0) break;
        if (strcmp(s, "[name]") == 0) {
            if (!next_tok(&t)) goto done;
            continue;
        }
        if (strcmp(s, "[scalars]") == 0) {
            for (int i = 0; i < 7; i++) {
                char *k = next_tok(&t), *v = next_tok(&t);
                if (!k || !v) goto done;
                char *end;
                if (strcmp(k, "lxc") == 0) {
                    P->lxc = strtod(v, &end);
                    if (*end || !(P->lxc >= 0.0 && P->lxc < 1000.0)) goto done;
                    continue;
                }
                long x = strtol(v, &end, 10);
                if (*end || x < -100000 || x > 100000) goto done;
                if (!strcmp(k, "ML_closing")) P->ml_closing = (int32_t)x;
                else if (!strcmp(k, "ML_intern")) P->ml_intern = (int32_t)x;
                else if (!strcmp(k, "ML_base")) P->ml_base = (int32_t)x;
                else if (!strcmp(k, "TerminalAU")) P->terminal_au = (int32_t)x;
                else if (!strcmp(k, "Ninio")) P->ninio = (int32_t)x;
                else if (!strcmp(k, "NinioMax")) P->ninio_max = (int32_t)x;
                else goto done;
            }
            seen |= 1;
            continue;
        }
        char *cnt = next_tok(&t);
        if (!cnt) goto done;
        int n = atoi(cnt);
        struct {
            const char *name;
            int32_t *dst;
            int count, inf, bit;
        } arr[] = {
            {"[stack]", &P->stack[0][0], 36, 0, 2},
            {"[mismatch_hairpin]", &P->mmH[0][0][0], 96, 0, 3},
            {"[mismatch_interior]", &P->mmI[0][0][0], 96, 0, 4},
            {"[mismatch_interior_1n]", &P->mm1n[0][0][0], 96, 0, 5},
            {"[mismatch_interior_23]", &P->mm23[0][0][0], 96, 0, 6},
            {"[int11]", &P->int11[0][0][0][0], 576, 0, 7},
            {"[int21]", &P->int21[0][0][0][0][0], 2304, 0, 8},
            {"[int22]", &P->int22[0][0][0][0][0][0], 9216, 0, 9},
            {"[hairpin]", P->hairpin, 31, 1, 10},
            {"[bulge]", P->bulge, 31, 1, 11},
            {"[interior]", P->interior, 31, 1, 12},
        };
        int handled = 0;
        for (size_t i = 0; i < sizeof(arr) / sizeof(arr[0]); i++)
            if (strcmp(s, arr[i].name) == 0) {
                if (n != arr[i].count || read_ints(&t, arr[i].dst, n, arr[i].inf)) goto done;
                seen |= 1 << arr[i].bit;
                handled = 1;
            }
        if (handled) continue;
        int kind = !strcmp(s, "[triloop]") ? 0 : !strcmp(s, "[tetraloop]") ? 1
                 : !strcmp(s, "[hexaloop]") ? 2 : -1;
        if (kind < 0 || n < 0 || n > OR_MAX_SPECIAL) goto done;
        int need = kind == 0 ? 5 : kind == 1 ? 6 : 8;
        for (int i = 0; i < n; i++) {
            char *q = next_tok(&t), *v = next_tok(&t);
            if (!q || !v || (int)strlen(q) != need) goto done;
            for (int j = 0; j < need; j++)
                if (or_nuc(q[j]) < 0) goto done;
            strcpy(P->spec_seq[kind][i], q);
            char *end;
            long x = strtol(v, &end, 10);
            if (*end || x < -100000 || x > 100000) goto done;
            P->spec_e[kind][i] = (int32_t)x;
        }
        P->nspec[kind] = n;
        seen |= 1 << (13 + kind);
    }
    if (seen != (1 << 16) - 1 - 2) goto done; /* bits 0, 2..15 */
    /* hairpins need finite sizes 3..30, bulges 1..30, interior 2..30 */
    for (int m = 3; m <= 30; m++)
        if (P->hairpin[m] >= OR_EINF) goto done;
    for (int m = 1; m <= 30; m++)
        if (P->bulge[m] >= OR_EINF) goto done;
    for (int m = 2; m <= 30; m++)
        if (P->interior[m] >= OR_EINF) goto done;
    {
        int32_t mx = 0;
        const int32_t *all[] = {&P->stack[0][0], &P->mmH[0][0][0], &P->mmI[0][0][0],
                                &P->mm1n[0][0][0], &P->mm23[0][0][0], &P->int11[0][0][0][0],
                                &P->int21[0][0][0][0][0], &P->int22[0][0][0][0][0][0],
                                P->hairpin, P->bulge, P->interior};
        const int cnts[] = {36, 96, 96, 96, 96, 576, 2304, 9216, 31, 31, 31};
        for (int i = 0; i < 11; i++)
            for (int j = 0; j < cnts[i]; j++) upd_max(&mx, all[i][j]);
        for (int k = 0; k < 3; k++)
            for (int i = 0; i < P->nspec[k]; i++) upd_max(&mx, P->spec_e[k][i]);
        upd_max(&mx, P->ml_closing);
        upd_max(&mx, P->ml_intern);
        upd_max(&mx, P->ml_base);
        upd_max(&mx, P->terminal_au);
        upd_max(&mx, P->ninio);
        upd_max(&mx, P->ninio_max);
        P->maxabs = mx;
    }
    rc = OR_OK;
done:
    free(buf);
    if (rc == OR_OK)
        *out = P;
    else
        free(P);
    return rc;
}

void or_params_free(or_params *p) { free(p); }
