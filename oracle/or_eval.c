/* Oracle: loop-decomposition structure evaluator (test infrastructure only).
 *
 * Scores a given (sequence, dot-bracket) pair under the dangle-0 nearest-neighbour model of
 * Sec. 3 by walking the loops of the structure.  It deliberately does NOT call the loop-energy
 * helpers used by the DPs: each loop class is scored here from the parameter tables directly,
 * so that a mistake in the DPs' energy code shows up as a disagreement.  Loops of any size are
 * scored (the 30-unpaired cap restricts the optimisation domain only, Sec. 3 and Sec. 7.1);
 * sizes above 30 extrapolate with lxc*ln(size/30), rounded half away from zero.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int ptype(char a, char b) {
    const char *pairs[6] = {"AU", "CG", "GC", "GU", "UA", "UG"};
    for (int t = 0; t < 6; t++)
        if (pairs[t][0] == a && pairs[t][1] == b) return t;
    return -1;
}

static int nuc(char c) { return c == 'A' ? 0 : c == 'C' ? 1 : c == 'G' ? 2 : c == 'U' ? 3 : -1; }

static int32_t terminal(const or_params *P, int t) { return (t == 0 || t >= 3) ? P->terminal_au : 0; }

static int32_t init_len(const int32_t *tab, double lxc, int size) {
    if (size <= 30) return tab[size];
    return tab[30] + (int32_t)lround(lxc * log(size / 30.0));
}

static int32_t eval_hairpin(const or_params *P, const char *s, int i, int j) {
    int m = j - i - 1, t = ptype(s[i], s[j]);
    int kind = m == 3 ? 0 : m == 4 ? 1 : m == 6 ? 2 : -1;
    if (kind >= 0)
        for (int q = 0; q < P->nspec[kind]; q++)
            if (strncmp(P->spec_seq[kind][q], s + i, (size_t)(m + 2)) == 0) return P->spec_e[kind][q];
    int32_t e = init_len(P->hairpin, P->lxc, m);
    if (m == 3) return e + terminal(P, t);
    return e + P->mmH[t][nuc(s[i + 1])][nuc(s[j - 1])];
}

/* closing pair (i,j), single inner pair (k,l) */
static int32_t eval_twoloop(const or_params *P, const char *s, int i, int j, int k, int l) {
    int t_out = ptype(s[i], s[j]);
    int t_in = ptype(s[l], s[k]); /* inner pair read from inside the loop */
    int u5 = k - i - 1, u3 = j - l - 1;
    int a = nuc(s[i + 1]), b = nuc(s[k - 1]), c = nuc(s[l + 1]), d = nuc(s[j - 1]);
    if (u5 + u3 == 0) return P->stack[t_out][t_in];
    if (u5 == 0 || u3 == 0) {
        int sz = u5 + u3;
        int32_t e = init_len(P->bulge, P->lxc, sz);
        return sz == 1 ? e + P->stack[t_out][t_in] : e + terminal(P, t_out) + terminal(P, t_in);
    }
    switch (u5 * 10 + u3) {
        case 11: return P->int11[t_out][t_in][a][d];
        case 12: return P->int21[t_out][t_in][a][c][d];
        case 21: return P->int21[t_in][t_out][c][a][b];
        case 22: return P->int22[t_out][t_in][a][b][c][d];
        default: break;
    }
    int sz = u5 + u3;
    int32_t e = init_len(P->interior, P->lxc, sz);
    int32_t asym = P->ninio * abs(u5 - u3);
    e += asym < P->ninio_max ? asym : P->ninio_max;
    const int32_t(*mm)[4][4] = P->mmI;
    if (u5 == 1 || u3 == 1) mm = P->mm1n;
    else if (u5 * u3 == 6) mm = P->mm23;
    return e + mm[t_out][a][d] + mm[t_in][c][b];
}

int or_eval(const char *seq, const char *structure, const or_params *P, int32_t *energy) {
    if (!seq || !structure || !P || !energy) return OR_E_ARG;
    int n = (int)strlen(seq);
    if ((int)strlen(structure) != n) return OR_E_ARG;
    int *pt = malloc(sizeof(int) * (n + 1)), *stk = malloc(sizeof(int) * (n + 1)), sp = 0;
    int rc = OR_OK;
    for (int i = 0; i < n; i++) {
        pt[i] = -1;
        if (nuc(seq[i]) < 0) rc = OR_E_ARG;
    }
    for (int i = 0; i < n && rc == OR_OK; i++) {
        if (structure[i] == '(') stk[sp++] = i;
        else if (structure[i] == ')') {
            if (!sp) { rc = OR_E_ARG; break; }
            int j = stk[--sp];
            pt[i] = j;
            pt[j] = i;
        } else if (structure[i] != '.') rc = OR_E_ARG;
    }
    if (sp) rc = OR_E_ARG;
    for (int i = 0; i < n && rc == OR_OK; i++)
        if (pt[i] > i && (ptype(seq[i], seq[pt[i]]) < 0 || pt[i] - i - 1 < 3)) rc = OR_E_ARG;
    int64_t E = 0;
    /* exterior loop: terminal penalty per top-level helix */
    for (int i = 0; i < n && rc == OR_OK;) {
        if (pt[i] > i) {
            E += terminal(P, ptype(seq[i], seq[pt[i]]));
            i = pt[i] + 1;
        } else {
            i++;
        }
    }
    /* every pair closes exactly one loop */
    for (int i = 0; i < n && rc == OR_OK; i++) {
        if (pt[i] <= i) continue;
        int j = pt[i], branches = 0, unpaired = 0, bk = -1;
        int64_t stems = 0;
        for (int k = i + 1; k < j;) {
            if (pt[k] > k) {
                branches++;
                bk = k;
                stems += P->ml_intern + terminal(P, ptype(seq[k], seq[pt[k]]));
                k = pt[k] + 1;
            } else {
                unpaired++;
                k++;
            }
        }
        if (branches == 0) E += eval_hairpin(P, seq, i, j);
        else if (branches == 1) E += eval_twoloop(P, seq, i, j, bk, pt[bk]);
        else E += P->ml_closing + P->ml_intern + terminal(P, ptype(seq[j], seq[i])) + stems +
                  (int64_t)P->ml_base * unpaired;
    }
    free(pt);
    free(stk);
    if (rc == OR_OK) *energy = (int32_t)E;
    return rc;
}
