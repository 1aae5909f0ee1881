/*
 * sparsedesign.h -- C ABI of the MI355X (gfx950) exact coding-sequence design library.
 *
 * The library computes, for a protein p, a codon relative-adaptiveness table w and a weight
 * lambda >= 0 (kcal/mol), the optimum of
 *
 *     F*(p, lambda) = min over synonymous mRNAs r, structures S in S_{3,30}(r) of
 *                     E_T04,d0(r, S) + lambda * C(r),   C(r) = -sum_{codons c of r} ln w(c)
 *
 * (paper "SparseDesign: Scaling Exact Coding-Sequence Design", Sec. 3, eq. 1) with the
 * candidate-sparsified lattice-parsing DP (Sec. 4.1, eqs. 2-7), evaluated on the GPU one span
 * per step with every cell of the span in parallel (Sec. 5, Algorithm 1, re-designed for the
 * GPU).  Energies are int32 in 0.01 kcal/mol; the DP runs in int64 fixed point (energies times
 * 2^s plus rounded codon costs), so the optimum, the candidate sets and the canonical traceback
 * are exact and independent of reduction order.
 *
 * Conventions shared by every entry point:
 *  - Every function returns sd_status (SD_OK = 0, negative on error) unless noted; no C++
 *    exception crosses the ABI.  A failed call leaves its outputs untouched except where noted
 *    and stores a message retrievable with sd_last_error (per calling thread).
 *  - Input pointers are borrowed for the duration of the call only.  Handles (sd_params,
 *    sd_codon_table, sd_context, sd_server) are owned by the caller and released with their
 *    *_free / *_destroy function; a handle must outlive every call that uses it.
 *  - Strings inside sd_result are allocated by the library and released by sd_result_free.
 *  - A context is thread-compatible, not thread-safe: calls on one context must not overlap.
 *  - There is no CPU fallback: every DP step runs in the library's HIP kernels on the
 *    context's device; without a usable gfx950 device sd_context_create fails with
 *    SD_E_DEVICE.
 */
#ifndef SPARSEDESIGN_H
#define SPARSEDESIGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sd_status {
    SD_OK = 0,
    SD_E_ARG = -1,          /* null pointer, bad size or option                         */
    SD_E_PROTEIN = -2,      /* empty, symbol outside ACDEFGHIKLMNPQRSTVWY*, '*' not last  */
    SD_E_CODON_TABLE = -3,  /* w outside (0,1] / NaN, or a needed family without w = 1   */
    SD_E_PARAMS = -4,       /* unreadable / malformed parameter file, SHA-256 mismatch   */
    SD_E_LAMBDA = -5,       /* lambda < 0 or not finite (eq. 1 requires lambda >= 0)     */
    SD_E_RANGE = -6,        /* fixed-point range rule cannot be met                      */
    SD_E_NOMEM = -7,        /* host or device allocation failed / pool exhausted         */
    SD_E_DEVICE = -8,       /* HIP error or no gfx950 device                             */
    SD_E_BUSY = -9,         /* server: request still running                             */
    SD_E_CANCELLED = -10,   /* server: request cancelled or server stopped               */
    SD_E_INTERNAL = -11     /* self-check failed (should never happen)                   */
} sd_status;

typedef struct sd_params sd_params;           /* opaque int32 energy tables (0.01 kcal/mol) */
typedef struct sd_codon_table sd_codon_table; /* opaque, 64 codons -> w in (0,1]            */
typedef struct sd_context sd_context;         /* device, stream, scratch memory             */

typedef struct sd_options {
    int retain_all;        /* 1: scalar dense control -- retain every finite direct interval
                              instead of the strict test B < P_S (Sec. 8.1); same optimum     */
    int capacity_override; /* >0: candidate slots per right endpoint (forces the overflow
                              fallback when small; results are unchanged); 0: worst case      */
    int kernel_timing;     /* 1: bracket every span-step launch with HIP events on the
                              context's stream and report the summed kernel time            */
    int reserved[5];
} sd_options;

typedef struct sd_result {
    char *mrna;              /* 3A bases A/C/G/U (library-owned, see sd_result_free)          */
    char *structure;         /* dot-bracket of the same length                                */
    int32_t energy_centi;    /* E(r,S) in 0.01 kcal/mol                                       */
    double codon_cost;       /* C(r) = -sum ln w in nats, FP64, summed in codon order          */
    double objective_kcal;   /* E/100 + lambda*C(r)                                            */
    int64_t objective_fixed; /* DP optimum in fixed point: E*2^s + sum of rounded codon costs */
    int32_t fixed_shift;     /* s                                                              */
    double cai;              /* exp(-C(r)/A)                                                   */
    int64_t n_states;        /* automaton states N                                             */
    int64_t n_cells;         /* state pairs (a,b) with rho(a) < rho(b)                         */
    int64_t n_candidates;    /* Z = sum_b |C_b| (eq. 6)                                        */
    int64_t n_visits;        /* candidate entries scanned by the multiloop split (eq. 7)       */
    int64_t n_feasible;      /* cells with finite direct branch cost B                        */
    double t_fill_s;         /* cost-only time: allocation + forward fill (Sec. 6)             */
    double t_total_s;        /* complete time: input -> strings                                */
    double t_span_kernels_s; /* with kernel_timing: summed duration of the span-step kernels  */
    int64_t n_span_launches; /* span-step kernel launches of the forward fill                  */
} sd_result;

/* Parameter file (project text format "SPARSEDESIGN-PARAMS 1"; Turner-2004 d0 array shapes,
 * Sec. 3).  expect_sha256 (64 hex chars) may be NULL; a mismatch gives SD_E_PARAMS. */
sd_status sd_params_load(const char *path, const char *expect_sha256, sd_params **out);
/* Writes the 64-hex-char SHA-256 of the loaded file plus a terminating NUL into out[65]. */
sd_status sd_params_sha256(const sd_params *p, char out[65]);
void sd_params_free(sd_params *p);

/* Codon table from relative adaptiveness w (index 16*b1 + 4*b2 + b3, A<C<G<U); every entry
 * must lie in (0,1].  Families used by a design must contain w = 1 (Sec. 3). */
sd_status sd_codon_table_from_weights(const double w[64], sd_codon_table **out);
/* Codon table from usage frequencies f > 0: w = f / max over the synonymous family. */
sd_status sd_codon_table_from_freqs(const double f[64], sd_codon_table **out);
void sd_codon_table_free(sd_codon_table *t);

/* Context on HIP device `device` (options may be NULL for defaults). */
sd_status sd_context_create(int device, const sd_options *opt, sd_context **out);
void sd_context_destroy(sd_context *ctx);

/* One design, plain mode: one span-step kernel launch per span length (Algorithm 1 order),
 * canonical traceback on the device.  On success *out owns two strings. */
sd_status sd_design(sd_context *ctx, const char *protein, const sd_codon_table *table,
                    const sd_params *params, double lambda_kcal, sd_result *out);

/* n designs in one persistent launch (all instances advance one span per grid barrier).
 * proteins[i] with lambdas[i]; outs[i] receives each result.  On error no output owns memory. */
sd_status sd_design_batch(sd_context *ctx, int n, const char *const *proteins,
                          const double *lambdas, const sd_codon_table *table,
                          const sd_params *params, sd_result *outs);

/* Test hook: the plain design plus its tables copied into caller buffers in a dense
 * state-pair layout [a*N + b] (V: [tau][a][b] with tau in AU,CG,GC,GU,UA,UG; entries with
 * rho(a) >= rho(b) are set to 2^62).  Any table pointer may be NULL.  N = out->n_states. */
sd_status sd_design_tables(sd_context *ctx, const char *protein, const sd_codon_table *table,
                           const sd_params *params, double lambda_kcal, sd_result *out,
                           int64_t *V, int64_t *B, int64_t *S1, int64_t *S2, int64_t *X);

/* Number of automaton states of a protein (to size the sd_design_tables buffers). */
sd_status sd_lattice_size(const char *protein, int64_t *n_states, int64_t *n_cells);

void sd_result_free(sd_result *r);
const char *sd_status_str(sd_status s);
const char *sd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
