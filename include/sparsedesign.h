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
    SD_E_INTERNAL = -11,    /* self-check failed (should never happen)                   */
    SD_E_INFEASIBLE = -12   /* no coding sequence meets the constraints (forbidden motifs) */
} sd_status;

typedef struct sd_params sd_params;           /* opaque int32 energy tables (0.01 kcal/mol) */
typedef struct sd_codon_table sd_codon_table; /* opaque, 64 codons -> w in (0,1]            */
typedef struct sd_context sd_context;         /* device, stream, scratch memory             */

typedef struct sd_options {
    int retain_all;        /* 1: scalar dense control -- retain every finite direct interval
                              instead of the strict test B < P_S (Sec. 8.1); same optimum     */
    int capacity_override; /* >0: candidate slots per right endpoint (forces the overflow
                              fallback when small; results are unchanged); 0: worst case      */
    int kernel_timing;     /* k > 0: bracket every k-th span-step launch (spans 1, 1+k, ...)
                              with HIP events on the context's stream and report their summed
                              duration and count; an event between two launches adds a gap,
                              so k > 1 keeps the fill close to an untimed one              */
    int span_threads;      /* workgroup size of the plain-mode span step: 0 (library choice per
                              span, autotuned per span band; see span_item_waves), 64, 256, 512
                              or 1024 for every span; anything else gives SD_E_ARG at create */
    int span_item_waves;   /* with span_threads set: 0 (the workgroup's waves share each layer
                              pair) or 1 with span_threads 256 (every wave on its own pair, four
                              pairs per workgroup); must be 0 when span_threads is 0          */
    int batch_threads;     /* persistent (batched / served) launch: threads per workgroup, 64,
                              256 or 512, with batch_per_cu workgroups per CU; both 0: autotuned */
    int batch_per_cu;
    int batch_item_waves;  /* with batch_threads set: waves per work item (layer pair) of the
                              persistent launch -- 0 or threads / 64 (the workgroup's waves
                              share each item), or 1 with 64 or 256 threads (every wave works on
                              its own items); must be 0 when batch_threads is 0; anything else
                              gives SD_E_ARG at create                                        */
    int span_check;        /* debug mode (race detection): 1 = plain designs run every span step
                              twice, the second time with another workgroup size after restoring
                              the committed candidate counts and the counters, and compare digests
                              of everything the step wrote; batched designs re-run the whole
                              persistent launch under another schedule and compare a digest of
                              each member's tables.  A difference fails the call with
                              SD_E_INTERNAL naming the span or member.  2 = the same, but the
                              visit counters are deliberately not restored before the re-run, so
                              the comparison must fail (a self-test of the check).  0 = off   */
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
    double t_span_kernels_s; /* with kernel_timing: summed duration of the timed span-step
                                launches (batched: this member's share of the persistent one) */
    int64_t n_span_launches; /* span-step kernel launches of the forward fill                  */
    int64_t cand_slots;      /* candidate slots reserved for the fill that produced the result */
    int64_t cand_slots_first;/* slots reserved by the first attempt (before any fallback)      */
    int32_t cand_overflow;   /* 1 if the first attempt's reservation overflowed (then exact
                                worst-case segments were used; the result is unchanged)       */
    int64_t n_timed_launches;/* span-step launches timed with kernel_timing (plain mode)       */
    int32_t path;            /* which forward fill produced the result (sd_path below)         */
    int32_t graph_captured;  /* 1 if that fill was a persistent launch replayed from a captured
                                hipGraph, else 0                                               */
    int32_t sched_threads;   /* persistent launch behind the result: threads per workgroup
                                (0 for the plain paths)                                        */
    int32_t sched_grid;      /* ... and its workgroup count (resident workgroups per CU times
                                the CU count; 0 for the plain paths)                           */
    int32_t sched_item_waves;/* ... and its waves per work item (0 for the plain paths)        */
    int32_t sched_tuned;     /* 1 if that schedule was fixed by the caller or is the autotuner's
                                settled choice for the batch's size class; 0 while the tuner
                                still explores (it runs one candidate per call).  Plain results:
                                the same for the per-span-band tile choice of the span step   */
} sd_result;

/* sd_result.path: the fill behind a result.  Batched and served results come from the persistent
 * launch unless its grid barrier gave up (then the member is recomputed in plain mode) or, in a
 * batch, the member's learned candidate reservation overflowed (recomputed in plain mode with
 * worst-case segments).  A served request whose reservation overflows is re-run inside the mix
 * with worst-case segments and stays SD_PATH_PERSISTENT with cand_overflow = 1.  Every path
 * gives the same design. */
typedef enum sd_path {
    SD_PATH_PLAIN = 0,                /* sd_design: one span-step launch per span              */
    SD_PATH_PERSISTENT = 1,           /* batched or served persistent launch                   */
    SD_PATH_PLAIN_AFTER_BARRIER = 2,  /* batch or server member redone after a barrier timeout */
    SD_PATH_PLAIN_AFTER_OVERFLOW = 3  /* batch member redone after a candidate overflow        */
} sd_path;

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
/* Context on memory and a stream the caller owns (e.g. a framework's caching allocator and
 * current stream): every design of the context runs on `hip_stream` (a hipStream_t; NULL is the
 * device's null stream, on which batched launches run without graph capture) and places its
 * per-design device tables in [dev_pool, dev_pool + pool_bytes) (device memory, 256-byte aligned,
 * at least 4 KiB) instead of a library allocation; the device is the pool's.  A design whose
 * tables do not fit gives SD_E_NOMEM (sd_lattice_size / sd_motif_lattice_size give N and the cell
 * count; about 72 B per cell plus per-state rings).  The energy tables, pinned host staging
 * buffers and design servers are still allocated by the library.  sd_context_destroy
 * synchronises the stream and frees neither the pool nor the stream; both must outlive the
 * context.  Calls on one context must not overlap, as for sd_context_create. */
sd_status sd_context_create_external(void *hip_stream, void *dev_pool, size_t pool_bytes,
                                     const sd_options *opt, sd_context **out);
void sd_context_destroy(sd_context *ctx);

/* Tuning cache for processes that should not re-explore schedules a previous process measured.
 * sd_tuning_save writes the context's settled choices to the text file `path` (overwritten): a
 * header line "sparsedesign-tuning 1", a line "device gfx950 <compute units>", then one line
 * "batch <class> <grid> <threads> <item_waves>" per settled batched-launch class (the class of
 * the batch tuner: floor log2 of the members' mean length times 8 plus min(4, floor log2 of the
 * member count)) and one line "span <class> <band> <threads> <item_waves>" per tuned span band
 * of the plain path (class floor log2 of the mRNA length in nucleotides, band floor log2 of the
 * span's layer pairs).  Classes still exploring are not written.  SD_E_ARG if the file cannot be written.
 * sd_tuning_load installs such a file's entries as settled choices of `ctx` (replacing those of
 * the same classes), so their first designs run the saved schedules without exploring.  The whole
 * file is checked first and nothing is installed if any part fails: SD_E_ARG for a missing or
 * malformed file, a device line of another architecture or compute-unit count, a batched
 * schedule this device cannot keep resident, or a span tile the library does not have.
 * Schedules fixed in the context's options still take precedence. */
sd_status sd_tuning_save(const sd_context *ctx, const char *path);
sd_status sd_tuning_load(sd_context *ctx, const char *path);

/* One design, plain mode (Sec. 4.1 recurrences in the span order of Sec. 5, Algorithm 1): the
 * automaton of `protein` (NUL-terminated one-letter string, optional final '*') is built on the
 * host and uploaded, the forward fill runs as one span-step kernel launch per span length on
 * the context's stream, and the canonical first-match traceback (deferred traceback, Sec. 5)
 * runs on the device over the resident tables; only the chosen path (one base and pair partner
 * per nucleotide, the energy, the path cost) is copied back, and the host builds the strings and
 * checks the design exactly (the bases spell a path of the automaton whose costs add up to the
 * optimum's).  lambda_kcal >= 0 weights
 * the codon cost (eq. 1).  On success *out is filled and owns two strings (sd_result_free); on
 * error *out is untouched: SD_E_PROTEIN / SD_E_CODON_TABLE / SD_E_LAMBDA / SD_E_RANGE for bad
 * inputs (no kernel launched), SD_E_NOMEM / SD_E_DEVICE for allocation or HIP failures,
 * SD_E_INTERNAL if the self-check fails. */
sd_status sd_design(sd_context *ctx, const char *protein, const sd_codon_table *table,
                    const sd_params *params, double lambda_kcal, sd_result *out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): sd_design with no allocation.  The design's device
 * state (energy tables, automaton inputs, DP tables, rings and candidate segments) is placed in
 * one static device array of 256 MiB that the library holds on each GPU it runs on until the
 * process ends (its address is taken once per device when a context is created there); no
 * hipMalloc, hipFree or other allocating device routine is called.  Inputs and outputs are as
 * for sd_design (plain mode; result strings are host allocations owned by the caller, freed
 * with sd_result_free); the context's kernel_timing option is ignored.  A design whose state
 * does not fit the array gives SD_E_NOMEM with the bytes it needs (about 72 B per cell plus
 * 31 KiB per automaton state: a 300-aa design takes about 75 MiB, 500 aa is near the limit;
 * sd_design has no such limit).  Every call on a GPU shares that GPU's array, which keeps the
 * last call's contents: calls that overlap on one GPU (from any contexts or threads) race and
 * must be serialised by the caller.  SD_E_DEVICE if the array has no address on the device. */
sd_status sd_design_noalloc(sd_context *ctx, const char *protein, const sd_codon_table *table,
                            const sd_params *params, double lambda_kcal, sd_result *out);

/* n designs in one persistent, graph-captured launch (all instances advance one span per grid
 * barrier; the schedule is fixed by sd_options or autotuned: the first calls of a size class
 * each run one candidate schedule, later calls the fastest, reported in sd_result.sched_*).
 * proteins[i] (as for sd_design) with lambdas[i]; outs[i] (array of n) receives each result,
 * identical to sd_design's.  Members whose learned reservation overflows, or a launch whose
 * barrier gives up, are recomputed exactly in plain mode.  On error no output owns memory and
 * the status names the first invalid member (SD_E_PROTEIN, ...) or the failure. */
sd_status sd_design_batch(sd_context *ctx, int n, const char *const *proteins,
                          const double *lambdas, const sd_codon_table *table,
                          const sd_params *params, sd_result *outs);

/* Supported lambda envelope of one protein on [lambda_lo, lambda_hi] (the supported-envelope /
 * inverse-lambda tools of Sec. 10; eq. 1 is a lower envelope of lines E/100 + lambda * C).
 * Exact dichotomic search: the designs optimal at the interval ends, then at every crossing of
 * two consecutive supported lines the optimum is computed (all crossings of one level in one
 * batched call) and kept if it lies strictly below both lines (relative tolerance 1e-9).
 * On success outs[0..*n_out-1] (caller array of max_designs >= 2 entries) hold the supported
 * designs in increasing lambda (decreasing codon cost), each owning its strings; design i is
 * optimal for lambda in [breaks[i], breaks[i+1]] (breaks: caller array of max_designs + 1).
 * If the search would exceed max_designs it stops with the designs found so far (then a
 * breakpoint interval may hide further supported designs).  Errors as for sd_design_batch, plus
 * SD_E_LAMBDA unless 0 <= lambda_lo < lambda_hi < inf. */
sd_status sd_lambda_envelope(sd_context *ctx, const char *protein, double lambda_lo, double lambda_hi,
                             int max_designs, const sd_codon_table *table, const sd_params *params,
                             sd_result *outs, double *breaks, int *n_out);

/* One design under forbidden-motif constraints (Sec. 3: the codon automaton intersected with a
 * deterministic matcher of the motifs keeps the layered path model; transitions that complete a
 * motif are removed; the finite-state constraint experiments report the state growth).
 * motifs: n_motifs (1..256) NUL-terminated strings of 1..32 bases over A, C, G, U; the returned
 * mRNA contains none of them as a substring, in any frame and across codon boundaries.
 * The product automaton keeps the pairs (codon state, matcher state) that lie on a path from
 * the source to the last layer; layers may hold up to 16 states.  The fill runs in plain mode
 * with a generic span kernel that reads minimum path costs from gap tables built on the device
 * (the codon trie's closed form does not hold on the product).  The fixed-point shift is the
 * unconstrained design's, so objectives of constrained and unconstrained designs compare
 * exactly.  Errors as for sd_design, plus SD_E_ARG for a malformed motif list,
 * SD_E_INFEASIBLE if every synonymous mRNA contains a motif, SD_E_RANGE if a layer of the
 * product is wider than 16 states.  Candidate segments are sized for the worst case (the
 * learned sizer is trained on unconstrained designs); sd_options.capacity_override applies. */
sd_status sd_design_motifs(sd_context *ctx, const char *protein, const char *const *motifs,
                           int n_motifs, const sd_codon_table *table, const sd_params *params,
                           double lambda_kcal, sd_result *out);

/* Inverse lambda (the inverse-lambda tool of Sec. 10): the smallest lambda in [0, lambda_hi] at
 * which a supported design of `protein` has CAI >= target_cai (relative tolerance 1e-12), found
 * on the supported envelope of [0, lambda_hi] (sd_lambda_envelope with max_designs).  The optimal
 * CAI is a non-decreasing step function of lambda, so *lambda_out is the left breakpoint of the
 * first supported line that meets the target (0 if the lambda = 0 optimum already does); *out
 * receives that design (owning its strings).  SD_E_ARG unless 0 < target_cai <= 1,
 * SD_E_INFEASIBLE if no supported design on the interval reaches it; otherwise errors as for
 * sd_lambda_envelope. */
sd_status sd_inverse_lambda(sd_context *ctx, const char *protein, double target_cai, double lambda_hi,
                            int max_designs, const sd_codon_table *table, const sd_params *params,
                            sd_result *out, double *lambda_out);

/* Test hook: the plain design plus its tables copied into caller buffers in a dense
 * state-pair layout [a*N + b] (V: [tau][a][b] with tau in AU,CG,GC,GU,UA,UG; entries with
 * rho(a) >= rho(b) are set to 2^62).  Any table pointer may be NULL.  N = out->n_states. */
sd_status sd_design_tables(sd_context *ctx, const char *protein, const sd_codon_table *table,
                           const sd_params *params, double lambda_kcal, sd_result *out,
                           int64_t *V, int64_t *B, int64_t *S1, int64_t *S2, int64_t *X);
/* Test hook: sd_design_batch plus the tables of batch member `member` (0 <= member < n) in the
 * dense layout of sd_design_tables, N = outs[member].n_states.  The tables are the ones that
 * produced that member's result (the persistent launch's, or the plain fill's when the member
 * fell back; outs[member].path says which).  SD_E_ARG for a member index outside the batch. */
sd_status sd_design_batch_tables(sd_context *ctx, int n, const char *const *proteins, const double *lambdas,
                                 const sd_codon_table *table, const sd_params *params, sd_result *outs,
                                 int member, int64_t *V, int64_t *B, int64_t *S1, int64_t *S2, int64_t *X);
/* Test hook: sd_design_motifs plus its tables, in the same dense layout over the product
 * automaton's states (N = out->n_states; the states are ordered by layer, codon state, matcher
 * rank). */
sd_status sd_design_motifs_tables(sd_context *ctx, const char *protein, const char *const *motifs,
                                  int n_motifs, const sd_codon_table *table, const sd_params *params,
                                  double lambda_kcal, sd_result *out, int64_t *V, int64_t *B,
                                  int64_t *S1, int64_t *S2, int64_t *X);

/* Fixed-point shift s that sd_design uses for these inputs (host only, no device work).  The DP
 * runs in int64 fixed point: energies times 2^s plus codon costs rounded to the nearest multiple
 * of 2^-s (the paper's real-valued objective of Sec. 3, eq. 1, read exactly; each codon's
 * rounding is at most 2^-(s+1) internal units).  s is the largest value in [16, 40] with
 *     sum over codon positions of the largest rounded cost of a synonymous codon
 *     + Ebound(n) * 2^s  <  2^60,
 * where Ebound(n) bounds |energy| of any partial structure on n = 3A nucleotides: at most n/2
 * pairs, each closing one loop (energy range read off the parameter tables: hairpins of every
 * size up to n, special loops, stacks, bulges, interior tables and generic interior loops, the
 * multiloop closing pair) and being at most one branch (ML_intern + AU, or AU), plus ML_base
 * per unpaired base.  Every finite DP value then lies in (-2^60, 2^60).  SD_E_RANGE if no s in
 * [16, 40] qualifies (a very large lambda); SD_E_PROTEIN, SD_E_LAMBDA, SD_E_ARG for bad inputs. */
sd_status sd_fixed_shift(const char *protein, const sd_codon_table *table, const sd_params *params,
                         double lambda_kcal, int32_t *shift);
/* Test hook: the multiloop recurrences alone (eqs. 6-7 with the online retention test) on an
 * abstract layered DAG, the exact-integer abstract test of Sec. 7.1, run by the span step's own
 * device code with the direct costs given instead of computed from loop energies.  States
 * 0..N-1 in layer order (layer[0] = 0, consecutive non-empty layers of at most 4 states);
 * n_edges edges esrc[k] -> edst[k] between consecutive layers (at most 4 out of a state) with
 * unpaired-edge costs eu[k]; B[a*N + b] the direct cost of the arc (a, b) (>= 2^61: none).
 * Costs must lie in [-2^40, 2^40] (SD_E_RANGE).  Outputs, dense [a*N + b]: S1 and S2 (2^62 for
 * rho(a) >= rho(b) or infeasible), cand[a*N + b] = 1 if a was retained in C_b, and Z = sum |C_b|.
 * SD_E_ARG for a malformed DAG. */
sd_status sd_multiloop_abstract(sd_context *ctx, int N, const int32_t *layer, int n_edges, const int32_t *esrc,
                                const int32_t *edst, const int64_t *eu, const int64_t *B, int64_t *S1,
                                int64_t *S2, int8_t *cand, int64_t *Z);
/* Number of automaton states of a protein (to size the sd_design_tables buffers). */
sd_status sd_lattice_size(const char *protein, int64_t *n_states, int64_t *n_cells);
/* Size of the product automaton of sd_design_motifs (host only, no device work): states N and
 * cells.  Errors as for sd_design_motifs' input checks (SD_E_PROTEIN, SD_E_ARG, SD_E_INFEASIBLE,
 * SD_E_RANGE). */
sd_status sd_motif_lattice_size(const char *protein, const char *const *motifs, int n_motifs,
                                int64_t *n_states, int64_t *n_cells);

/* ---- learned candidate-buffer sizing ------------------------------------------------------
 * A small FP32 MLP (22 -> hidden -> hidden -> K, ReLU, sigmoid outputs) trained on the GPU by the
 * library's own kernels.  Input features of a request (sd_sizer_features): log(A)/log(2000),
 * the 20 amino-acid fractions, lambda/4.  Output k: the largest fraction of its worst-case
 * candidate slots that the exact DP retains for any right endpoint b in position bin k
 * (layer(b)/n in [k/K, (k+1)/K); endpoints with fewer than 64 worst-case slots excluded), as
 * logged by sd_occupancy.  Sizing only changes how much memory is reserved: an overflowing
 * reservation falls back to exact worst-case segments, results are unchanged. */
typedef struct sd_sizer sd_sizer;
sd_status sd_sizer_create(sd_context *ctx, int hidden, int n_out, uint64_t seed, sd_sizer **out);
void sd_sizer_free(sd_sizer *z);
int64_t sd_sizer_num_params(const sd_sizer *z);
/* parameters as one flat FP32 array: W1[hidden][22], b1, W2[hidden][hidden], b2, W3[K][hidden], b3 */
sd_status sd_sizer_get_params(const sd_sizer *z, float *flat);
sd_status sd_sizer_set_params(sd_sizer *z, const float *flat);
/* MSE loss and its gradient (flat layout above) on n samples X[n][22], Y[n][K] */
sd_status sd_sizer_gradient(sd_sizer *z, int n, const float *X, const float *Y, float *loss, float *grad);
/* full-batch Adam on the device; final_loss (may be NULL) = loss before the last update */
sd_status sd_sizer_train(sd_sizer *z, int n, const float *X, const float *Y, int steps, float lr,
                         float *final_loss);
sd_status sd_sizer_predict(sd_sizer *z, int n, const float *X, float *Yhat);
/* The same forward pass on the host (FP32, no device work): the predictor that sizing and server
 * admission use for each request, from the parameters as of the last train / set_params. */
sd_status sd_sizer_predict_host(const sd_sizer *z, int n, const float *X, float *Yhat);
sd_status sd_sizer_features(const char *protein, double lambda_kcal, float out[22]);
/* Sizing policy of a context: NULL restores worst-case segments.  A right endpoint in bin k gets
 * min(worst, ceil(worst * min(1, yhat_k * (1 + margin))) + slack) slots.  The sizer must outlive
 * the context's use of it. */
sd_status sd_context_set_sizer(sd_context *ctx, const sd_sizer *z, float margin, int slack);
/* The candidate reservation one request gets under sizer z with (margin, slack) as in
 * sd_context_set_sizer (host only): *cand_slots slots of 12 bytes (*cand_bytes), beside the
 * worst case *worst_slots.  This is what a sized context or server reserves for the request
 * before any overflow (sd_result.cand_slots_first).  SD_E_PROTEIN for a bad protein, SD_E_ARG
 * for null pointers or negative margin / slack. */
sd_status sd_sizer_request_bytes(const sd_sizer *z, const char *protein, double lambda_kcal, float margin,
                                 int slack, int64_t *cand_slots, int64_t *cand_bytes,
                                 int64_t *worst_slots);
/* Exact occupancy log: designs n requests (batched, worst-case segments) and writes Y[n][K], the
 * per-bin largest retained fraction of the worst-case slots (see above), plus the results (may
 * be NULL). */
sd_status sd_occupancy(sd_context *ctx, int n, const char *const *proteins, const double *lambdas,
                       const sd_codon_table *table, const sd_params *params, int K, float *Y,
                       sd_result *outs);

/* ---- design server (continuous batching) ---------------------------------------------------
 * A server thread admits queued requests FIFO while a slot is free and the request's device
 * state fits the pool (tables sized exactly from the automaton, candidate segments from the
 * context's sizing policy), runs one persistent launch of steps_per_round span steps over all
 * active requests (each at its own span), and retires finished ones (their tracebacks in one
 * device launch), freeing their memory for the next admissions.  A launch's schedule is the one
 * fixed in the context's sd_options, else chosen per round from the mix: every wave on its own
 * layer pairs when the round starts with at least 12 pairs per resident wave, else four waves
 * per pair.  While a server runs, its context must not be used by other calls.  Results are
 * identical to sd_design; t_total_s is the latency from submission to completion. */
typedef struct sd_server sd_server;
typedef struct sd_server_cfg {
    size_t pool_bytes;   /* device memory for the DP state of admitted requests (>= 1 MiB)  */
    int max_active;      /* concurrent requests on the device (1..1024)                     */
    int steps_per_round; /* span steps per persistent launch between admission points (>0) */
    int reserved[6];
} sd_server_cfg;
typedef struct sd_server_stats {
    int64_t submitted, admitted, completed, fallbacks, rounds, peak_active, active, queued;
    int64_t pool_in_use, pool_high_water, reserved_bytes, reserved_cand_bytes;
    double gpu_seconds;
} sd_server_stats;
sd_status sd_server_start(sd_context *ctx, const sd_codon_table *table, const sd_params *params,
                          const sd_server_cfg *cfg, sd_server **out);
sd_status sd_server_submit(sd_server *s, const char *protein, double lambda_kcal, uint64_t *ticket);
/* SD_E_BUSY while pending; on completion *out owns its strings (sd_result_free) */
sd_status sd_server_poll(sd_server *s, uint64_t ticket, sd_result *out);
sd_status sd_server_wait(sd_server *s, uint64_t ticket, sd_result *out);
sd_status sd_server_get_stats(sd_server *s, sd_server_stats *out);
/* cancels queued requests (SD_E_CANCELLED), finishes active ones, frees the server */
sd_status sd_server_stop(sd_server *s);

void sd_result_free(sd_result *r);
const char *sd_status_str(sd_status s);
const char *sd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
