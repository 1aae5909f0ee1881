/*
 * oracle.h -- plain, slow CPU oracle for exact coding-sequence design.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link, load or run this
 * code: only the tests, the smoke check and the benchmark's CPU-baseline leg use it.  It shares
 * no code with the GPU library (no headers, helpers, tables or generators).
 *
 * What it computes (the paper, "SparseDesign: Scaling Exact Coding-Sequence Design"):
 *   F*(p, lambda) = min over synonymous mRNAs r and structures S in S_{3,30}(r) of
 *                   E_T04,d0(r, S) + lambda * C(r),  C(r) = -sum_codons ln w(c)   (Sec. 3, eq. 1)
 * as the PLAIN DENSE lattice DP: typed closed values V_tau (Sec. 4.1), the scalar branch B
 * (eq. 2) and the right-normal dense multiloop recurrences D2, P_D, D1 (eqs. 3-5) over all
 * split states, followed by the external column and a canonical first-match traceback.
 * Arithmetic is int64 fixed point (energies times 2^s plus rounded codon costs), so the
 * result is exact and independent of summation order.
 *
 * Independent checkers in this directory: a fixed-sequence Zuker MFE (or_zuker.c), a loop-
 * decomposition structure evaluator (or_eval.c) with its own loop-energy code, and a brute-force
 * synonymous enumerator (or_brute.c).
 */
#ifndef SD_ORACLE_H
#define SD_ORACLE_H
#include <stdint.h>

#define OR_INF ((int64_t)1 << 62)   /* fixed-point infeasibility sentinel */
#define OR_EINF 1000000000          /* integer energy of an infeasible / unlisted loop size */
#define OR_MAX_SPECIAL 256
#define OR_MAX_MOTIF 32            /* longest forbidden motif */
#define OR_MAX_MOTIFS 256          /* motifs per design */

/* Energy parameters in 0.01 kcal/mol (Turner-2004 d0 array shapes, Sec. 3). */
typedef struct or_params {
    int32_t stack[6][6];
    int32_t mmH[6][4][4], mmI[6][4][4], mm1n[6][4][4], mm23[6][4][4];
    int32_t int11[6][6][4][4];
    int32_t int21[6][6][4][4][4];
    int32_t int22[6][6][4][4][4][4];
    int32_t hairpin[31], bulge[31], interior[31];
    int32_t ml_closing, ml_intern, ml_base, terminal_au, ninio, ninio_max;
    double lxc;
    int nspec[3];                         /* triloop, tetraloop, hexaloop */
    char spec_seq[3][OR_MAX_SPECIAL][9];  /* loop sequence including the closing pair */
    int32_t spec_e[3][OR_MAX_SPECIAL];    /* total loop energy */
    int32_t maxabs;                       /* largest |finite entry|, for the range rule */
} or_params;

typedef struct or_result {
    int32_t energy;          /* E(r,S) in 0.01 kcal/mol                          */
    int64_t objective_fixed; /* X(s) = E*2^s + sum of rounded codon costs          */
    int64_t path_u;          /* sum of rounded codon costs along the design        */
    int32_t fixed_shift;     /* s                                                   */
    double codon_cost;       /* C(r) in nats, FP64, summed in codon order          */
    double objective_kcal;   /* E/100 + lambda*C(r)                                 */
    int64_t n_states, n_edges, n_cells, n_feasible_direct, n_candidates;
    int64_t visits_dense, visits_sparse;
    int32_t selfcheck_ok;    /* E*2^s + sum U == X(s) and the path spells a valid design */
} or_result;

/* status codes shared by the oracle entry points (same meaning as the library's, own copy) */
enum { OR_OK = 0, OR_E_ARG = -1, OR_E_PROTEIN = -2, OR_E_CODON = -3, OR_E_PARAMS = -4,
       OR_E_LAMBDA = -5, OR_E_RANGE = -6, OR_E_NOMEM = -7, OR_E_INTERNAL = -11,
       OR_E_INFEASIBLE = -12 };

int or_params_load(const char *path, or_params **out);
void or_params_free(or_params *p);

/* Full dense design.  mrna/structure must hold 3*A+1 chars.  Optional debug tables (may be
 * NULL) are N*N row-major over state indices [a*N+b]: V has 6*N*N entries ([tau][a][b]). */
int or_design(const char *protein, const double w[64], const or_params *P, double lambda,
              int nthreads, char *mrna, char *structure, or_result *res,
              int64_t *dbg_V, int64_t *dbg_B, int64_t *dbg_D1, int64_t *dbg_D2, int64_t *dbg_X);
/* Design under forbidden motifs: the same DP over the product of the codon DFA with the motif
 * matcher (Sec. 3).  motifs: nm strings over ACGU (1..OR_MAX_MOTIF bases, nm <= OR_MAX_MOTIFS);
 * the returned mRNA contains none of them.  The fixed-point shift is the one of the
 * unconstrained design (range rule over the codon families).  OR_E_INFEASIBLE if no
 * synonymous mRNA avoids every motif. */
int or_design_motifs(const char *protein, const double w[64], const or_params *P, double lambda,
                     const char *const *motifs, int nm, int nthreads, char *mrna, char *structure,
                     or_result *res);
/* The same with the dense debug tables of or_design (N = states of the product automaton). */
int or_design_motifs_tables(const char *protein, const double w[64], const or_params *P, double lambda,
                            const char *const *motifs, int nm, int nthreads, char *mrna, char *structure,
                            or_result *res, int64_t *dbg_V, int64_t *dbg_B, int64_t *dbg_D1,
                            int64_t *dbg_D2, int64_t *dbg_X);
/* Product automaton statistics: states, edges, widest layer and the number of source-to-sink
 * paths (saturating at INT64_MAX); every state lies on such a path (dead states are removed). */
int or_motif_lattice(const char *protein, const char *const *motifs, int nm, int64_t *n_states,
                     int64_t *n_edges, int64_t *width, int64_t *n_paths);
/* Lattice statistics only (no DP): states, edges, cells, feasible direct intervals. */
int or_lattice_stats(const char *protein, int64_t *n_states, int64_t *n_edges, int64_t *n_cells,
                     int64_t *n_feasible);
/* Fixed-point shift chosen by the range rule, or OR_E_RANGE. */
int or_fixed_shift(const char *protein, const double w[64], const or_params *P, double lambda);

/* Fixed-sequence Zuker MFE in S_{3,30}; structure (len+1 chars) may be NULL. */
int or_zuker(const char *seq, const or_params *P, int32_t *energy, char *structure);
/* Independent evaluator of E(r,S) for any pseudoknot-free structure (no loop-size cap). */
int or_eval(const char *seq, const char *structure, const or_params *P, int32_t *energy);
/* Brute force over every synonymous mRNA: min of zuker(r)*2^s + U(r) (fixed point) and the
 * min of the FP64 objective E/100 + lambda*C(r). */
int or_bruteforce(const char *protein, const double w[64], const or_params *P, double lambda,
                  int64_t *best_fixed, double *best_kcal, int64_t *n_seqs, int32_t *shift);
/* The same over the synonymous mRNAs that contain none of the motifs (n_seqs counts those;
 * best_fixed is OR_INF and best_kcal +inf if there is none). */
int or_bruteforce_motifs(const char *protein, const double w[64], const or_params *P, double lambda,
                         const char *const *motifs, int nm, int64_t *best_fixed, double *best_kcal,
                         int64_t *n_seqs, int32_t *shift);

/* Abstract multiloop recurrences (eqs. 3-5) on a layered DAG with given direct costs B
 * (N*N, OR_INF = absent) and unpaired-edge costs u; fills D1, D2, PD (N*N). */
int or_multiloop_dense(int N, const int *layer, int nE, const int *esrc, const int *edst,
                       const int64_t *eu, const int64_t *B, int64_t *D1, int64_t *D2, int64_t *PD);

/* internal helpers shared inside the oracle */
int or_pair_type(int x, int y);
int32_t or_au(const or_params *P, int t);
int32_t or_loop_init(const int32_t tab[31], double lxc, int m);
int32_t or_hairpin_energy(const or_params *P, const int *seq, int len);
int32_t or_hairpin_generic(const or_params *P, int t, int m, int xi1, int xj1);
int32_t or_two_loop_energy(const or_params *P, int t, int tr, int l1, int l2,
                           int xi1, int xk1, int xl1, int xj1);
int or_nuc(char c);

#endif
