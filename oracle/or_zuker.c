/* Oracle: fixed-sequence Zuker MFE over S_{3,30} (test infrastructure only).
 *
 * A textbook O(n^3) minimum-free-energy recursion on one fixed sequence, written with the
 * classic left/right multiloop table WM (at least one branch) rather than the right-normal
 * D1/D2 form of the lattice DP, so that it checks the lattice recurrences independently:
 *   V(i,j)  = min{hairpin, stack/bulge/interior with l1+l2 <= 30, multiloop closure}
 *   WM(i,j) = min{V(i,j)+stem, WM(i+1,j)+base, WM(i,j-1)+base, WM(i,u-1)+V(u,j)+stem}
 *   closure = ML_closing + ML_intern + AU(i,j) + min_u WM(i+1,u-1) + WM(u,j-1)
 *   W(j)    = min{W(j-1), W(i-1) + V(i,j) + AU(i,j)}   (exterior loop, dangle-0)
 * Brute force over synonymous sequences uses it as the per-sequence MFE (Sec. 7.1 describes the
 * same kind of independent enumeration).
 */
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define ZI OR_EINF

typedef struct {
    int n;
    const int *s;
    const or_params *P;
    int32_t *V, *WM, *W;
} zk_t;

#define ZV(i, j) Z->V[(size_t)(i) * Z->n + (j)]
#define ZM(i, j) Z->WM[(size_t)(i) * Z->n + (j)]

static int32_t add2(int32_t a, int32_t b) { return (a >= ZI || b >= ZI) ? ZI : a + b; }

static int32_t wm(const zk_t *Z, int i, int j) { return (i < 0 || j >= Z->n || j - i < 4) ? ZI : ZM(i, j); }

static int32_t stem(const zk_t *Z, int i, int j) {
    return Z->P->ml_intern + or_au(Z->P, or_pair_type(Z->s[i], Z->s[j]));
}

static int32_t hp(const zk_t *Z, int i, int j) { return or_hairpin_energy(Z->P, Z->s + i, j - i + 1); }

static int32_t two(const zk_t *Z, int i, int j, int k, int l) {
    const int *s = Z->s;
    int t = or_pair_type(s[i], s[j]), tr = or_pair_type(s[l], s[k]);
    return or_two_loop_energy(Z->P, t, tr, k - i - 1, j - l - 1, s[i + 1], s[k - 1], s[l + 1], s[j - 1]);
}

static int32_t closing(const zk_t *Z, int i, int j) {
    return Z->P->ml_closing + Z->P->ml_intern + or_au(Z->P, or_pair_type(Z->s[i], Z->s[j]));
}

static void fill(zk_t *Z) {
    int n = Z->n;
    for (size_t q = 0; q < (size_t)n * n; q++) Z->V[q] = Z->WM[q] = ZI;
    for (int d = 4; d < n; d++)
        for (int i = 0; i + d < n; i++) {
            int j = i + d;
            int32_t v = ZI;
            if (or_pair_type(Z->s[i], Z->s[j]) >= 0) {
                v = hp(Z, i, j);
                for (int k = i + 1; k < j && k - i - 1 <= 30; k++)
                    for (int l = j - 1; l > k && (k - i - 1) + (j - l - 1) <= 30; l--) {
                        if (l - k < 4 || ZV(k, l) >= ZI) continue;
                        int32_t e = two(Z, i, j, k, l);
                        if (e < ZI && e + ZV(k, l) < v) v = e + ZV(k, l);
                    }
                for (int u = i + 2; u <= j - 1; u++) {
                    int32_t m = add2(wm(Z, i + 1, u - 1), wm(Z, u, j - 1));
                    if (m < ZI && m + closing(Z, i, j) < v) v = m + closing(Z, i, j);
                }
            }
            ZV(i, j) = v;
            int32_t w = ZI;
            if (v < ZI) w = v + stem(Z, i, j);
            int32_t t = add2(wm(Z, i + 1, j), Z->P->ml_base);
            if (t < w) w = t;
            t = add2(wm(Z, i, j - 1), Z->P->ml_base);
            if (t < w) w = t;
            for (int u = i + 1; u <= j - 4; u++) {
                if (ZV(u, j) >= ZI) continue;
                t = add2(wm(Z, i, u - 1), ZV(u, j) + stem(Z, u, j));
                if (t < w) w = t;
            }
            ZM(i, j) = w;
        }
    Z->W[0] = 0;
    for (int j = 0; j < n; j++) {
        int32_t w = Z->W[j];
        for (int i = 0; i + 4 <= j; i++) {
            if (ZV(i, j) >= ZI) continue;
            int32_t t = Z->W[i] + ZV(i, j) + or_au(Z->P, or_pair_type(Z->s[i], Z->s[j]));
            if (t < w) w = t;
        }
        Z->W[j + 1] = w;
    }
}

/* traceback (first match, any fixed order) used only to hand the structure to the evaluator */
static void tb_wm(const zk_t *Z, int i, int j, char *st);
static void tb_v(const zk_t *Z, int i, int j, char *st) {
    st[i] = '(';
    st[j] = ')';
    int32_t v = ZV(i, j);
    if (hp(Z, i, j) == v) return;
    for (int k = i + 1; k < j && k - i - 1 <= 30; k++)
        for (int l = j - 1; l > k && (k - i - 1) + (j - l - 1) <= 30; l--) {
            if (l - k < 4 || ZV(k, l) >= ZI) continue;
            int32_t e = two(Z, i, j, k, l);
            if (e < ZI && e + ZV(k, l) == v) {
                tb_v(Z, k, l, st);
                return;
            }
        }
    for (int u = i + 2; u <= j - 1; u++) {
        int32_t m = add2(wm(Z, i + 1, u - 1), wm(Z, u, j - 1));
        if (m < ZI && m + closing(Z, i, j) == v) {
            tb_wm(Z, i + 1, u - 1, st);
            tb_wm(Z, u, j - 1, st);
            return;
        }
    }
}

static void tb_wm(const zk_t *Z, int i, int j, char *st) {
    int32_t w = ZM(i, j);
    if (ZV(i, j) < ZI && ZV(i, j) + stem(Z, i, j) == w) {
        tb_v(Z, i, j, st);
        return;
    }
    if (add2(wm(Z, i + 1, j), Z->P->ml_base) == w) {
        tb_wm(Z, i + 1, j, st);
        return;
    }
    if (add2(wm(Z, i, j - 1), Z->P->ml_base) == w) {
        tb_wm(Z, i, j - 1, st);
        return;
    }
    for (int u = i + 1; u <= j - 4; u++) {
        if (ZV(u, j) >= ZI) continue;
        if (add2(wm(Z, i, u - 1), ZV(u, j) + stem(Z, u, j)) == w) {
            tb_wm(Z, i, u - 1, st);
            tb_v(Z, u, j, st);
            return;
        }
    }
}

int or_zuker(const char *seq, const or_params *P, int32_t *energy, char *structure) {
    if (!seq || !P || !energy) return OR_E_ARG;
    int n = (int)strlen(seq);
    int *s = malloc(sizeof(int) * (n + 1));
    for (int i = 0; i < n; i++) {
        s[i] = or_nuc(seq[i]);
        if (s[i] < 0) {
            free(s);
            return OR_E_ARG;
        }
    }
    zk_t Z = {n, s, P, NULL, NULL, NULL};
    if (n > 0) {
        Z.V = malloc(sizeof(int32_t) * (size_t)n * n);
        Z.WM = malloc(sizeof(int32_t) * (size_t)n * n);
    }
    Z.W = malloc(sizeof(int32_t) * (n + 1));
    if ((n > 0 && (!Z.V || !Z.WM)) || !Z.W) {
        free(s); free(Z.V); free(Z.WM); free(Z.W);
        return OR_E_NOMEM;
    }
    if (n > 0) fill(&Z);
    else Z.W[0] = 0;
    *energy = Z.W[n];
    if (structure) {
        for (int i = 0; i < n; i++) structure[i] = '.';
        structure[n] = 0;
        int j = n;
        while (j > 0) {
            if (Z.W[j] == Z.W[j - 1]) {
                j--;
                continue;
            }
            int found = 0;
            for (int i = 0; i + 4 <= j - 1 && !found; i++) {
                int32_t v = Z.V[(size_t)i * n + (j - 1)];
                if (v >= ZI) continue;
                if (Z.W[i] + v + or_au(P, or_pair_type(s[i], s[j - 1])) == Z.W[j]) {
                    tb_v(&Z, i, j - 1, structure);
                    j = i;
                    found = 1;
                }
            }
            if (!found) break;
        }
    }
    free(s); free(Z.V); free(Z.WM); free(Z.W);
    return OR_OK;
}
