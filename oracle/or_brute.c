/* Oracle: brute force over every synonymous mRNA (test infrastructure only).
 *
 * For each r in Syn(p) (Sec. 3): MFE(r) by the fixed-sequence Zuker recursion, the rounded
 * codon costs U(r) and the FP64 codon penalty C(r).  Returns min_r MFE(r)*2^s + U(r) in the
 * fixed point of the lattice DP (same shift rule and rounding), and min_r MFE(r)/100 +
 * lambda*C(r) in FP64 (the objective of eq. 1).  Sec. 7.1 reports the same kind of independent
 * synonymous enumeration as a correctness check.  With forbidden motifs, mRNAs containing any
 * motif as a substring are skipped (the constrained language of Sec. 3).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static const char CODE64[65] = "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";

int or_bruteforce_motifs(const char *protein, const double w[64], const or_params *P, double lambda,
                         const char *const *motifs, int nm, int64_t *best_fixed, double *best_kcal,
                         int64_t *n_seqs, int32_t *shift) {
    if (!protein || !w || !P || !best_fixed || !best_kcal || !n_seqs || !shift) return OR_E_ARG;
    if (nm < 0 || (nm > 0 && !motifs)) return OR_E_ARG;
    int s = or_fixed_shift(protein, w, P, lambda);
    if (s < 0) return s;
    int A = (int)strlen(protein);
    int fam[64][6], nf[64], idx[64];
    for (int k = 0; k < A; k++) {
        nf[k] = 0;
        for (int c = 0; c < 64; c++)
            if (CODE64[c] == protein[k]) fam[k][nf[k]++] = c;
        idx[k] = 0;
    }
    double lam100 = 100.0 * lambda;
    char *seq = malloc((size_t)3 * A + 1);
    int64_t best = OR_INF, count = 0;
    double bestk = INFINITY;
    for (;;) {
        int64_t U = 0;
        double Cr = 0.0;
        for (int k = 0; k < A; k++) {
            int c = fam[k][idx[k]];
            seq[3 * k] = "ACGU"[c / 16];
            seq[3 * k + 1] = "ACGU"[(c / 4) % 4];
            seq[3 * k + 2] = "ACGU"[c % 4];
            double q = -log(w[c]);
            U += llround(ldexp(lam100 * q, s));
            Cr += q;
        }
        seq[3 * A] = 0;
        int banned = 0;
        for (int i = 0; i < nm && !banned; i++) banned = strstr(seq, motifs[i]) != NULL;
        if (banned) {
            int k = A - 1;
            while (k >= 0 && ++idx[k] == nf[k]) idx[k--] = 0;
            if (k < 0) break;
            continue;
        }
        int32_t e;
        int rc = or_zuker(seq, P, &e, NULL);
        if (rc) {
            free(seq);
            return rc;
        }
        int64_t f = (int64_t)e * ((int64_t)1 << s) + U;
        if (f < best) best = f;
        double fk = (double)e / 100.0 + lambda * Cr;
        if (fk < bestk) bestk = fk;
        count++;
        int k = A - 1;
        while (k >= 0 && ++idx[k] == nf[k]) idx[k--] = 0;
        if (k < 0) break;
    }
    free(seq);
    *best_fixed = best;
    *best_kcal = bestk;
    *n_seqs = count;
    *shift = s;
    return OR_OK;
}

int or_bruteforce(const char *protein, const double w[64], const or_params *P, double lambda,
                  int64_t *best_fixed, double *best_kcal, int64_t *n_seqs, int32_t *shift) {
    return or_bruteforce_motifs(protein, w, P, lambda, NULL, 0, best_fixed, best_kcal, n_seqs, shift);
}
