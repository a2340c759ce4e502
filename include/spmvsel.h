/*
 * spmvsel — selected CSR SpMV on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libspmvsel.so.  Every entry point returns an spmv_status_t; no C++
 * exception crosses the boundary.  After a non-zero status,
 * spmv_last_error() returns a message for the calling thread.
 *
 * Method: Elafrou, Goumas, Koziris, "A lightweight optimization selection
 * method for Sparse Matrix-Vector Multiplication" (arXiv 1511.02494).  The
 * library computes y = A x for A in CSR (Section 2, Algorithm 1), extracts
 * structural features of A (Table 1), classifies A with the profiling-based
 * classifier (Section 3.2.1) or with a learned selector over the features
 * (Section 3.2.2, here an MLP), and runs the optimisation chosen for it from
 * a pool of six GPU variants (Table 2, remapped to the GPU).
 *
 * Conventions
 *   - Pointers named d_* are device pointers (hipMalloc'd or from any
 *     allocator of the current HIP device); others are host pointers.
 *   - A stream argument is a hipStream_t passed as void* (NULL = the
 *     default stream).
 *   - CSR input: 0-based int32 indices (the paper's listing is 1-based);
 *     rowptr[0] = 0, rowptr[N] = NNZ, rowptr non-decreasing; columns in
 *     [0, M) and strictly increasing inside each row; N < 2^31 - 1,
 *     M < 2^31 and NNZ < 2^31 - 2^16 (the kernels step int32 nonzero
 *     indices up to 2048 past a row's end).  Empty rows are allowed
 *     (y_i = 0); N = 0 and NNZ = 0 are valid.
 *   - Value dtypes: SPMV_F64 values use double x and y; SPMV_F32 and
 *     SPMV_BF16 values (bfloat16 bit patterns in uint16) use float x and y
 *     with FP32 accumulation, Kahan-compensated on rows of more than 256
 *     nonzeros.
 */
#ifndef SPMVSEL_H
#define SPMVSEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spmv_plan *spmv_plan_t;

typedef enum {
    SPMV_OK = 0,
    SPMV_ERR_ARG = 1,          /* bad argument (NULL, negative size, ...) */
    SPMV_ERR_CSR_ROWPTR = 2,   /* rowptr[0] != 0, rowptr[N] != NNZ, decreasing, out of [0, NNZ] */
    SPMV_ERR_CSR_COL_RANGE = 3,/* a column index outside [0, M) */
    SPMV_ERR_CSR_UNSORTED = 4, /* columns not strictly increasing in a row (includes duplicates) */
    SPMV_ERR_OOM = 5,          /* device allocation failed; nothing is leaked */
    SPMV_ERR_HIP = 6,          /* any other HIP runtime error */
    SPMV_ERR_INFEASIBLE = 7,   /* the variant cannot represent this matrix */
    SPMV_ERR_NO_MODEL = 8      /* no MLP parameters loaded, or the file is corrupt */
} spmv_status_t;

typedef enum { SPMV_F64 = 0, SPMV_F32 = 1, SPMV_BF16 = 2 } spmv_dtype_t;

/* The optimisation pool (Table 2, remapped to the GPU).
 *  CSR_SCALAR  one lane per row: the unoptimised baseline of Section 4.3.
 *  CSR_VECTOR  a sub-wavefront of 2..64 lanes per row, DPP/swizzle reduction
 *              (vectorisation, class CMP; the architecture-centric default).
 *  MERGE_PATH  nonzero-balanced merge-path tiles (class IMB; replaces the
 *              OpenMP dynamic/auto schedules).
 *  DELTA16     16-bit column offsets from one reference column per group of
 *              rows (column-index compression, class MB; Section 3.3), in one
 *              of two layouts (spmv_set_delta16_layout): rows streamed
 *              through LDS with one reference per block of 256 x R rows, or
 *              sliced: slices of 64 rows, one row per lane of a wavefront,
 *              the nonzeros stored column-major in pairs with one reference
 *              per slice, taken when padding to the slice's longest row
 *              costs at most 1.35 slots per nonzero, or 1.5 when rows
 *              average 16 nonzeros or more (stencils, rows of nearly equal
 *              length); a slice whose rows use at most 32 diagonals c - r
 *              stores those diagonals once and a bit mask per row, and no
 *              column data at all.  The sliced layout's other slices store
 *              16-bit offsets from the slice's reference column or 8-bit
 *              deltas from the row's previous column, code 255 escaping to
 *              the full column: one width per matrix, never both
 *              (Section 3.3; spmv_set_delta16_offset_bits).  An offset
 *              slice whose columns span fewer than 512 reads x from a copy
 *              of that window in LDS.
 *  XBLOCK_LDS  x blocking (class CML; replaces software prefetching of x):
 *              the columns are cut into S <= 8 slices (spmv_set_xblock_slices),
 *              each stored as its own CSR and run on the XCDs that take that
 *              slice, so the slice of x it gathers stays in their L2; rows
 *              are streamed through LDS per slice, rows with a slice segment
 *              over 128 nonzeros are summed from the CSR in chunks instead
 *              (merge-path tiles per slice when such rows hold over a
 *              quarter of the nonzeros); S partial y vectors are summed in
 *              slice order.  When no row leaves the slices, a workgroup
 *              instead owns a few row blocks and walks the slices in order
 *              (all workgroups resident, so all gather from about one slice
 *              at a time), each row's sum kept by its thread: no partial y,
 *              and FP64 rows summed in column order.  (The name is kept from
 *              an earlier design that staged x windows in LDS.)
 *  SHORT_ROW   rows streamed through LDS in chunks of 2048 nonzeros with one
 *              thread summing each row (short rows: inner-loop overhead). */
typedef enum {
    V_CSR_SCALAR = 0, V_CSR_VECTOR = 1, V_MERGE_PATH = 2,
    V_DELTA16 = 3, V_XBLOCK_LDS = 4, V_SHORT_ROW = 5, SPMV_N_VARIANTS = 6
} spmv_variant_t;

/* Bottleneck classes of Section 3.1. */
typedef enum { K_CML = 0, K_MB = 1, K_IMB = 2, K_CMP = 3 } spmv_class_t;

typedef enum {
    SEL_PROFILING = 0,  /* micro-benchmarks + threshold cascade (Section 3.2.1) */
    SEL_MLP = 1,        /* features + MLP; falls back to SEL_PROFILING */
    SEL_EXHAUSTIVE = 2, /* time every feasible variant, keep the fastest */
    SEL_DTREE = 3,      /* features + CART decision tree; falls back to SEL_PROFILING */
    SEL_GNB = 4         /* features + Gaussian naive Bayes; falls back to SEL_PROFILING */
} spmv_selector_t;

/* plan_create flags */
#define SPMV_COPY_INPUTS   1u  /* copy the CSR arrays instead of borrowing them */
#define SPMV_SKIP_VALIDATE 2u  /* trust the caller's CSR (no validation pass) */

#define SPMV_N_FEATURES 12
#define SPMV_N_ACCUM 12

/* Result of spmv_select. */
typedef struct {
    int32_t variant;        /* chosen spmv_variant_t */
    int32_t klass;          /* spmv_class_t from the profiling cascade or from a
                               class-labelled feature classifier, or -1 */
    int32_t selector;       /* selector actually used (after any fallback) */
    int32_t fell_back;      /* 1 if SEL_MLP / SEL_DTREE / SEL_GNB fell back to SEL_PROFILING */
    uint32_t feasible;      /* bit v set if variant v can run this matrix */
    float margin;           /* MLP top1 - top2 logit (0 if not run) */
    float logits[6];        /* MLP logits (0 if not run) */
    double meas[5];         /* profiling: t_base, t_nox, t_inf (s, median),
                               d_max, d_mean (per-partition device-clock ticks) */
    double scores[3];       /* s_nox, s_inf, s_bal */
    double features[12];    /* spmv_features output */
    double t_features_s;    /* host wall-clock of the feature extraction and
                               feasibility test; for a learned selector on a
                               plan with no features yet (automatic index
                               coding) these, the device finalisation of the
                               features and the selector run as one pass on
                               the plan's stream with one wait, all counted
                               here */
    double t_decide_s;      /* the learned selector's inference (0 when it
                               ran in that one pass), or the cascade */
    double t_profile_s;     /* micro-benchmarks (0 unless they ran) */
    double t_total_s;       /* whole selection, excluding format preparation */
    double t_prepare_s;     /* format preparation of the chosen variant */
    double variant_times_s[6]; /* SEL_EXHAUSTIVE: median time per variant (0 = infeasible) */
} spmv_select_info_t;

/* ----------------------------------------------------------------------- */
/* Plan life cycle                                                          */

/* Create a plan for the CSR matrix A (N x M, NNZ nonzeros).  Validates the
 * CSR invariants listed above on the device unless SPMV_SKIP_VALIDATE is set
 * (CSR, Section 2) and returns the first violated one as a status.  The plan
 * borrows d_rowptr[N+1], d_colind[NNZ] and d_val[NNZ] (dtype val_dtype)
 * until spmv_plan_destroy, unless SPMV_COPY_INPUTS is set.  Derived formats
 * are built lazily and owned by the plan.  Synchronises `stream`.
 * Arrays must be 16-byte aligned.  Sizes outside the limits above, an
 * unknown dtype, a NULL or misaligned array return SPMV_ERR_ARG before any
 * device work.  *out is NULL on failure. */
spmv_status_t spmv_plan_create(spmv_plan_t *out, int64_t n_rows, int64_t n_cols,
                               int64_t nnz, const int32_t *d_rowptr,
                               const int32_t *d_colind, const void *d_val,
                               int32_t val_dtype, void *stream, uint32_t flags);

/* Release the plan and everything it owns.  NULL is a no-op (SPMV_OK). */
spmv_status_t spmv_plan_destroy(spmv_plan_t plan);

/* ----------------------------------------------------------------------- */
/* The selected-SpMV path                                                   */

/* The twelve structural features of Table 1 used by the selectors, in
 * order: N, NNZ, nnz_avg, nnz_sd, nnz_max, nnz_min, bw_avg, bw_sd,
 * dispersion_avg, dispersion_sd, miss_per_nnz, size.  bw_i is the column
 * distance of a row's first and last nonzero; dispersion_i = nnz_i /
 * (bw_i + 1) in Q31 fixed point; a miss is a gap of more than 128 bytes of
 * x between consecutive nonzeros of a row; size is 1 if the CSR working set
 * fits a 256 MiB last-level cache.  Standard deviations are population ones.
 * Computed from exact integer sums (one pass over rowptr and colind on the
 * device) and one fixed FP64 finalisation (on the host, or on the device
 * by the same IEEE operations in the one-pass MLP selection of spmv_select),
 * so the result is bit-reproducible.  out_acc (nullable) receives the exact sums:
 * nnz_min, nnz_max, bw_max, S_L2, S_bw, S_bw2 (lo, hi), S_q, S_q2 (lo, hi),
 * S_miss, NNZ.  Synchronous on the plan stream. */
spmv_status_t spmv_features(spmv_plan_t plan, double out_features[12],
                            uint64_t out_acc[12]);

/* Choose a variant with `selector` (spmv_selector_t), set it on the plan and
 * build its format: the online step of the method (Section 3.2): the
 * profiling selector's micro-benchmarks and bottleneck cascade (Section
 * 3.2.1, Table 2's class-to-optimisation map), or a classifier on the
 * structural features of Table 1 (Section 3.2.2).  info (nullable) receives the decision record.
 * Synchronous.  The learned selectors (SPMV_SEL_MLP, SPMV_SEL_DTREE,
 * SPMV_SEL_GNB) on a plan with no features yet, under automatic index
 * coding, take one pass (feature sums and delta16 spans, device
 * finalisation, the selector; one wait); the result is the same as that of
 * the step-by-step path taken otherwise. */
spmv_status_t spmv_select(spmv_plan_t plan, int32_t selector,
                          spmv_select_info_t *info);

/* y = A x (Algorithm 1, the CSR product) with the plan's current variant
 * (CSR_SCALAR before any select or set_variant), on `stream`,
 * asynchronously.  y is fully overwritten.
 * d_x has M elements and d_y N elements, of type double for F64 plans and
 * float otherwise.  Calls on one plan must not overlap in time (the merge
 * path variant keeps per-tile carries in plan scratch). */
spmv_status_t spmv_execute(spmv_plan_t plan, const void *d_x, void *d_y,
                           void *stream);

/* ----------------------------------------------------------------------- */
/* Control and inspection                                                   */

/* Force a variant; builds its format (synchronous).  SPMV_ERR_INFEASIBLE if
 * the matrix cannot use it (DELTA16: a block of rows (256 x R, else 256)
 * spans more than 65536 columns). */
spmv_status_t spmv_set_variant(spmv_plan_t plan, int32_t variant);
spmv_status_t spmv_get_variant(spmv_plan_t plan, int32_t *variant);

/* Index coding of the column indices the variant kernels read (Section 3.3:
 * column-index compression as an optimisation of its own, Table 2 class MB,
 * applied on top of the other variants - the multi-level combinations of
 * the Conclusions).  coding:
 *   -1 (default) each variant's own: DELTA16 reads 16-bit codes, the others
 *      the caller's int32 columns;
 *    0 int32 columns everywhere (DELTA16 is then infeasible);
 *    1 16-bit column codes everywhere they exist:
 *      SHORT_ROW  the rows-streamed DELTA16 layout (offsets from one reference
 *                 column per block of rows);
 *      MERGE_PATH offsets from each merge-path tile's smallest column,
 *                 feasible when every tile spans < 65536 columns;
 *      XBLOCK_LDS offsets from the smallest column of each row block of each
 *                 column slice (the slice kernel's block: 256 rows in the
 *                 phased walk), feasible when every such segment spans
 *                 < 65536 columns and the slices are row-streamed;
 *      DELTA16    unchanged;
 *      CSR_SCALAR, CSR_VECTOR have no coded form (infeasible).
 * The request applies to spmv_set_variant, spmv_variant_mask, spmv_bytes,
 * spmv_time_variant and spmv_select from then on (the selectors choose among
 * the variants feasible under it); the current variant is rebuilt under it
 * when it has a form there, else spmv_execute reports SPMV_ERR_ARG (no
 * prepared format) until a variant is set.  A variant that cannot run under
 * the request gives SPMV_ERR_INFEASIBLE from spmv_set_variant.  Results
 * equal those of the int32 form of the same variant bit for bit (the codes
 * decode to the same columns; the order of operations is unchanged).
 * SPMV_ERR_ARG for any other value. */
typedef enum { SPMV_IDX_AUTO = -1, SPMV_IDX_I32 = 0, SPMV_IDX_CODED = 1 } spmv_index_t;
spmv_status_t spmv_set_index_coding(spmv_plan_t plan, int32_t coding);

/* FP32/BF16 plans: rows of at least `len` nonzeros accumulate with Kahan's
 * compensated sum (default 257, i.e. rows longer than 256; the merge-path
 * variant compensates every FP32 sum that crosses its threads or tiles);
 * INT32_MAX turns compensation off everywhere, to measure what it buys on
 * the same kernels (Section 3's precision path; tests).  FP64 plans ignore
 * it.  SPMV_ERR_ARG for len < 1. */
spmv_status_t spmv_set_kahan_min_len(spmv_plan_t plan, int32_t len);

/* Column slices of the XBLOCK_LDS format: 0 (default) picks the smallest of
 * 1, 2, 4, 8 that cuts x into slices of at most 256 Ki entries (2 MiB in
 * FP64), doubling only while a slice row keeps at least 0.9 nonzeros on
 * average (10 NNZ >= 9 (2 S) N; the row pointers and partial y vectors grow
 * with the count), so that each XCD's 4 MB L2 mostly holds the slice it
 * gathers from; 1, 2, 4 or 8 force that count (tests,
 * tuning).  If the format is built with another count it is rebuilt
 * (synchronous).  SPMV_ERR_ARG for any other value. */
spmv_status_t spmv_set_xblock_slices(spmv_plan_t plan, int32_t slices);

/* Layout of the DELTA16 format: -1 (default) picks the sliced layout when
 * its slots (each slice padded to its longest row, rounded up to even; with
 * the row order of spmv_set_delta16_sort) are at most 1.35 per nonzero, or
 * 1.6 when 2 NNZ >= 15 N and no offset slice spans 8192 columns or more,
 * else rows streamed
 * (sliced layouts also need NNZ < 2^30); 0 forces rows streamed, 1
 * forces sliced (tests, tuning).  A built format is dropped and, if DELTA16
 * is the plan's variant, rebuilt (synchronous).  SPMV_ERR_ARG for any other
 * value; building reports SPMV_ERR_INFEASIBLE as for the variant. */
spmv_status_t spmv_set_delta16_layout(spmv_plan_t plan, int32_t layout);

/* Row order of the sliced DELTA16 layout.  Sorted (as in SELL-C-sigma): the
 * rows of each window of 256 are placed by length, longest first (ties in
 * row order), so that a 64-row slice holds rows of similar lengths and pads
 * less; the kernel then reads the row index of each slice position (4 bytes
 * per row) and writes y through it.  Only offset slices are formed (no
 * diagonal slices), and a window lies inside one block of the streamed
 * layout, so the 16-bit feasibility is unchanged.  A sorted slice spans
 * its window's columns, so fewer slices stage x in LDS (an offset slice
 * does when its span is under 512 columns and at most 32 w - 1 for width
 * w).  -1 (default) sorts when at most 1% of the plain layout's slices are
 * diagonal and its slots exceed 1.05 per nonzero, sorting saves at least 5%
 * of its slots, and either under half of the plain layout's offset-slice
 * nonzeros are in staging slices and sorting saves at least 4 slots per
 * row, or sorting keeps at least half of the nonzeros in staging slices and
 * saves at least 8 slots per row; 0 never sorts, 1 always does (with the
 * sliced layout).
 * A built format is dropped and, if DELTA16 is the plan's variant, rebuilt
 * (synchronous).  SPMV_ERR_ARG for any other value. */
spmv_status_t spmv_set_delta16_sort(spmv_plan_t plan, int32_t mode);

/* Column-code width of the sliced DELTA16 layout's offset slices, the same
 * for the whole matrix (Section 3.3 uses 8- or 16-bit deltas, never both).
 * 16: offsets c - ref from the slice's reference column (its smallest).
 * 8: the code of a row's k-th nonzero is c_k - c_(k-1), with c_(-1) = ref,
 * when that is at most 254, else 255 (escape) and c_k itself is stored: the
 * e-th escape of lane l of slice s is escape entry 64 (eunits[s] + e) + l,
 * eunits being the exclusive prefix sums over slices of the largest number
 * of escapes of one of the slice's rows (E).  A slice spanning at most 255
 * columns has no escapes.  0 (default) takes 8 bits when the matrix has
 * offset slices and 256 sum E <= (nonzeros of offset slices) / 2 (the escape
 * entries cost at most half of the byte per nonzero the codes save), else
 * 16; 8 or 16 force the width (tests, tuning).  The rows-streamed layout
 * always stores 16 bits.  A built format is dropped and, if DELTA16 is the
 * plan's variant, rebuilt (synchronous).  SPMV_ERR_ARG for any other
 * value. */
spmv_status_t spmv_set_delta16_offset_bits(spmv_plan_t plan, int32_t bits);

/* Bit v set if variant v can run this matrix (computes features if needed). */
spmv_status_t spmv_variant_mask(spmv_plan_t plan, uint32_t *feasible_bits);

/* Algorithmic (compulsory) bytes of one SpMV with `variant`: 4(N+1) +
 * ib NNZ + vb NNZ + xb M + yb N, plus for DELTA16 (ib = 2 there, else 4)
 * 4 bytes per block reference column in the streamed layout; in the sliced
 * one, 16 bytes per 64-row slice (width, unit offset, reference column,
 * kind), 4 per offset slice (its column span) and 128 per diagonal slice
 * (its diagonals), with 1 or 2 index bytes (the code width) only for the
 * nonzeros of offset slices, plus with 8-bit codes 4 bytes per escaped
 * column and 4 per offset slice (its eunits entry), and with sorted rows
 * 4 per row (its index) (a row's mask in a diagonal slice takes the place
 * of its row pointer).  The layout is
 * decided here if needed; the streamed form is counted where DELTA16 is
 * infeasible.  Traffic a variant adds on top (the XBLOCK_LDS slice row
 * pointers and partial y vectors, the sliced layout's padding slots, the
 * x windows a sliced offset slice stages in LDS) is overhead and is not
 * counted. */
spmv_status_t spmv_bytes(spmv_plan_t plan, int32_t variant, int64_t *bytes);

/* Median and minimum time of `reps` executions of `variant` (hipEvents on
 * the plan stream, after 2 warm-ups).  cold != 0 evicts the 256 MiB
 * Infinity Cache before each timed run by streaming a 512 MiB buffer.
 * Uses internal x and y buffers.  SPMV_ERR_INFEASIBLE if not runnable. */
spmv_status_t spmv_time_variant(spmv_plan_t plan, int32_t variant, int32_t reps,
                                int32_t cold, double *t_median_s, double *t_min_s);

/* Back-to-back form of the above (the solver-loop rate): each of `reps`
 * timed runs is `launches` executions between one event pair, and the times
 * are per execution (median and minimum over the runs), which spreads the
 * event overhead and launch jitter of microsecond-scale kernels over the
 * batch.  Warm only.  launches in [1, 100000]. */
spmv_status_t spmv_time_variant_batch(spmv_plan_t plan, int32_t variant, int32_t launches,
                                      int32_t reps, double *t_median_s, double *t_min_s);

/* Plan parameters and derived arrays, for tests and tools.
 * Keys: 0 variant, 1 csr_vector width, 2 short_row/delta16 rows per block,
 * 3 merge-path items per tile, 4 merge-path tiles, 5 x-block columns per
 * slice, 6 x-block tiles (all slices), 7 x-block slices, 8 profiling
 * partitions, 9 delta16 feasible, 10 x-block feasible (always 1),
 * 11 delta16 rows per block, 12 x-block per-slice kernel (rows per block of
 * row streaming, or 0 for merge-path tiles), 13 x-block long rows (rows
 * with a slice segment longer than 128 nonzeros, summed from the original
 * CSR in chunks of 256 instead of in the slices; 0 when they would hold
 * more than a quarter of the nonzeros, in which case nothing is split and
 * the slices use merge-path tiles), 14 delta16 layout (-1 infeasible,
 * 0 rows streamed, 1 sliced), 15 delta16 sliced slots (64 x the sum of the
 * slice widths, padding included), 16 x-block row blocks per workgroup of
 * the phased slice kernel, at most (0 when the slices use merge-path tiles),
 * 17 delta16 code bits (8 or 16; -1 infeasible), 18 delta16 largest
 * offset of an offset slice (its columns minus its reference column; 0 with
 * no offset slices; -1 infeasible), 19 delta16 escape units (sum E; 0 with
 * 16-bit codes), 20 delta16 escaped nonzeros (0 with 16-bit codes),
 * 21 1 if the current variant (its format built by this call if needed)
 * sums every row from +0 in increasing column order, one product at a time
 * (Algorithm 1's order: FP64 results equal the sequential sum bit for bit),
 * else 0, 22 1 if the current variant reads 16-bit column codes under the
 * index-coding request, 23 1 if the merge-path tiles' codes fit 16 bits,
 * 24 1 if the x-block slices' codes fit 16 bits, 25 rows per x-block code
 * block, 26 1 if the sliced delta16 layout sorts rows by length (0 when it
 * does not or the layout is streamed; -1 infeasible). */
spmv_status_t spmv_plan_query(spmv_plan_t plan, int32_t key, int64_t *value);

/* Copy a derived array to host memory (builds it if needed).  which:
 * 0 delta16 block reference columns int32[ceil(N / rows per block)],
 * 1 delta16 offsets uint16[NNZ], 2 merge-path split rows int32[tiles+1],
 * 3 merge-path split nonzeros int32[tiles+1], 4 x-block slice row
 * pointers int32[S (N+1)] (S = key 7), 5 x-block slice-major column
 * indices int32[NNZ minus the long rows' nonzeros],
 * 6 profiling partition bounds int32[parts+1], 7 x-block long rows
 * int32[key 13] (ascending; their slice segments are empty in 4 and 5).
 * Sliced delta16 layout (SPMV_ERR_ARG in the streamed layout, as 0 and 1
 * are in the sliced one), S = ceil(N / 64) slices: 8 widths int32[S] (the
 * slice's longest row rounded up to even), 9 units int32[S] (exclusive
 * prefix sums of width / 2), 10 reference columns int32[S] (the slice's
 * smallest column, 0 if it has none), 11 column codes: uint16 offsets
 * [key 15] at the slots below, or uint8 delta codes [key 15 + 128 S] with
 * code k of lane l of slice s at byte 128 (units[s] + s) + 256 (k / 4) +
 * 4 l + k % 4 (0 in diagonal slices and padding),
 * 16 escaped columns int32[64 x key 19] (0 where unused), 17 eunits
 * int32[S] (8-bit codes only, else empty),
 * 12 values [key 15] of the plan's value type, 13 kinds int32[S] (0 for an
 * offset slice, 1 + D for a diagonal slice of D diagonals), 14 diagonals
 * int32[32 S] (slice s's sorted diagonals c - r from 32 s, zero-padded;
 * zeros for offset slices), 15 masks uint32[N] (bit k: the row has a
 * nonzero on diagonal k of its slice; 0 in offset slices), 22 with sorted
 * rows (key 26) the row at each slice position int32[N], else empty.
 * Position k of the row at slice position 64 s + l (that row itself, or
 * array 22's entry with sorted rows) is at slot 128 units[s] + 128 (k / 2) +
 * 2 l + (k % 2), where k counts the row's nonzeros in an offset slice and
 * is the diagonal's index in a diagonal slice; offsets are 0 in diagonal
 * slices and every other slot holds zero.
 * Coded forms (spmv_set_index_coding): 18 merge-path tile reference columns
 * int32[tiles] (key 4), 19 merge-path codes uint16[NNZ] (column minus the
 * reference of the nonzero's tile), 20 x-block reference columns
 * int32[S x ceil(N / H)] (slice-major, H = key 25), 21 x-block codes
 * uint16[NNZ minus the long rows' nonzeros] at the positions of array 5.
 * These are built (and their feasibility required) by the copy itself.
 * `bytes` must equal the array size. */
spmv_status_t spmv_plan_copy_format(spmv_plan_t plan, int32_t which,
                                    void *host_dst, int64_t bytes);

/* ----------------------------------------------------------------------- */
/* Profiling-based classifier (Section 3.2.1)                               */

/* Run the three micro-benchmarks against baseline CSR on the plan:
 * baseline, `noxmiss` (irregular x accesses removed: every column index of
 * row i replaced by i mod M; all-zero indices, as printed in the paper,
 * would make every wavefront hit one cache line on a GPU) and `inflate`
 * (int64 rowptr and colind), each the median of `reps` runs on a static partition of
 * 256 x (CUs) row ranges with equal nonzeros, one per wavefront; `balance`
 * from the per-partition device-clock durations of the baseline runs.
 * meas = {t_base, t_nox, t_inf, d_max, d_mean}.  Temporary copies are
 * freed before returning.  Synchronous. */
spmv_status_t spmv_profile_measure(spmv_plan_t plan, int32_t reps, double meas[5]);

/* The cascade as a pure host function: scores s_nox = t_base/t_nox,
 * s_inf = t_inf/t_base, s_bal = d_max/d_mean (0 when a denominator is not
 * positive); taken from the highest down (ties keep noxmiss, inflate,
 * balance), the first exceeding its threshold theta[0..2] gives CML, MB or
 * IMB; otherwise CMP.  Class -> variant: CML -> XBLOCK_LDS if feasible else
 * CSR_VECTOR; MB -> DELTA16 if feasible else CSR_VECTOR; IMB -> MERGE_PATH;
 * CMP -> SHORT_ROW if nnz_avg (features[2]) <= theta[3] else CSR_VECTOR. */
spmv_status_t spmv_profile_decide(const double meas[5], const double features[12],
                                  const double theta[4], uint32_t feasible_bits,
                                  int32_t *variant, int32_t *klass);

/* Process-wide thresholds used by spmv_select (default 2.0, 1.2, 1.5, 4.0). */
spmv_status_t spmv_set_thresholds(const double theta[4]);
spmv_status_t spmv_get_thresholds(double theta[4]);

/* ----------------------------------------------------------------------- */
/* Learned selector: MLP 12 -> 64 -> 64 -> 6, FP32                          */

/* Load parameters for the current process (all devices) from a file:
 * "SPMVMLP1", u32 version=1, u32 n_params=5382, f32 mu[12], f32 rho[12],
 * f32 tau, f32 params[5382] (W1[64][12], b1, W2[64][64], b2, W3[6][64], b3),
 * u32 CRC-32 (IEEE 802.3) of everything before it.  SPMV_ERR_NO_MODEL if the
 * file is missing or corrupt (no model is then loaded). */
spmv_status_t spmv_model_load(const char *path);
spmv_status_t spmv_model_unload(void);

/* Device inference for one feature vector: z_k = fl32(fl32(fl32(g_k) -
 * mu_k) * rho_k) with g_k = plog2(1 + f_k) (k < 8) or f_k, where
 * plog2(v) = (e - 1) + (2m - 1) for (m, e) = frexp(v); three dense layers
 * with acc = 0; acc = fl32(acc + fl32(w * in)) in input order, then + bias,
 * ReLU on the hidden layers; infeasible variants skipped; first maximal
 * logit wins; margin = top1 - top2; fallback = margin < tau or some
 * |z_k| > 8.  Outputs are nullable.  SPMV_ERR_NO_MODEL without a model. */
spmv_status_t spmv_mlp_predict(const double features[12], uint32_t feasible_bits,
                               int32_t *variant, float *margin, int32_t *fallback,
                               float logits[6], float z[12]);

/* One training minibatch on the device: mean softmax cross-entropy over
 * the feasible logits (d_mask[B*6], 1 = feasible) of d_Z[B*12] against
 * d_labels[B]; writes the loss to d_loss[0] and the gradient of every
 * parameter to d_grads[5382].  B <= 1024. */
spmv_status_t spmv_mlp_forward_backward(const float *d_params, const float *d_Z,
                                        const int32_t *d_labels, const uint8_t *d_mask,
                                        int32_t B, float *d_grads, float *d_loss,
                                        void *stream);

/* The same minibatch step with set-valued targets: d_accept[B*6] marks, per
 * sample, every variant that counts as a correct pick (labelling: those
 * within 5% of the fastest timed variant).  The loss is the mean of
 * -log(sum over the feasible marked variants of softmax p_j), whose gradient
 * with respect to logit j is p_j - p_j [j marked] / sum_marked p; a single
 * mark per sample is exactly the cross-entropy above.  Every sample needs at
 * least one feasible mark.  B <= 1024. */
spmv_status_t spmv_mlp_forward_backward_sets(const float *d_params, const float *d_Z,
                                             const uint8_t *d_accept, const uint8_t *d_mask,
                                             int32_t B, float *d_grads, float *d_loss,
                                             void *stream);

/* Adam (Kingma and Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
spmv_status_t spmv_mlp_adam_step(float *d_params, const float *d_grads, float *d_m,
                                 float *d_v, int32_t n, int32_t step, float lr,
                                 float b1, float b2, float eps, void *stream);

/* ----------------------------------------------------------------------- */
/* The paper's feature classifiers (Section 3.2.2, Tables 4 and 5)          */
/*
 * A CART decision tree (Gini criterion) and Gaussian naive Bayes over the
 * twelve features of spmv_features.  Labels are either variants
 * (SPMV_LABEL_VARIANT, 6 classes, the label kind of the MLP) or bottleneck
 * classes (SPMV_LABEL_CLASS, 4 classes CML/MB/IMB/CMP as the profiling
 * cascade assigns them, mapped to a variant through Table 2 with the current
 * thresholds).  Fitting is host code; prediction for selection runs on the
 * device.  Arrays are host memory, row-major, owned by the caller.
 *
 * CART: a node splits on feature j at t (left x_j <= t); thresholds lie
 * between consecutive distinct values a < b (t = a/2 + b/2, or a if that
 * rounds out of [a, b)); children keep >= min_leaf samples; the split with
 * the lowest weighted Gini impurity wins (compared exactly; first in
 * (feature, threshold) order on ties) and must lower the impurity strictly.
 * Leaves: depth max_depth (root 0), pure, < 2 min_leaf samples, no split.
 * Nodes are in pre-order; feature[i] = -1 marks a leaf; counts[i][k] are
 * the training samples of class k under node i.  A prediction is the
 * feasible class with the largest leaf count (lowest on ties).
 *
 * Naive Bayes on g_k = plog2(1 + f_k) (k < 8; plog2 as for the MLP) or f_k:
 * mu, var per class (population, sums in sample order) + 1e-9 times the
 * largest feature variance; stored w = 0.5 / var, c = log(n_k / n) -
 * 0.5 sum_j log(2 pi var).  Score c_k - sum_j w_kj (g_j - mu_kj)^2. */
typedef enum { SPMV_CLF_DTREE = 0, SPMV_CLF_GNB = 1 } spmv_classifier_t;
typedef enum { SPMV_LABEL_VARIANT = 0, SPMV_LABEL_CLASS = 1 } spmv_label_kind_t;

/* Fit a tree on X[n][12] with labels y[n] in [0, n_classes) (n_classes <= 8,
 * max_depth <= 64, min_leaf >= 1).  Outputs have room for max_nodes nodes
 * (counts: max_nodes x n_classes); *n_nodes receives the node count.
 * SPMV_ERR_ARG if the tree would need more nodes, or on bad input. */
spmv_status_t spmv_dtree_fit(const double *X, const int32_t *y, int64_t n, int32_t n_classes,
                             int32_t max_depth, int32_t min_leaf, int32_t max_nodes,
                             int32_t *feature, double *threshold, int32_t *left, int32_t *right,
                             int32_t *counts, int32_t *n_nodes);

/* Fit naive Bayes on raw features F[n][12]: mu[n_classes][12],
 * w[n_classes][12], c[n_classes], count[n_classes] (classes without
 * samples have count 0 and are never predicted). */
spmv_status_t spmv_gnb_fit(const double *F, const int32_t *y, int64_t n, int32_t n_classes,
                           double *mu, double *w, double *c, int32_t *count);

/* Install the process-wide models used by SEL_DTREE / SEL_GNB (copied; the
 * tree's structure is checked: pre-order children, features in range).
 * n_classes must be 6 for SPMV_LABEL_VARIANT and 4 for SPMV_LABEL_CLASS. */
spmv_status_t spmv_dtree_load(int32_t n_nodes, int32_t n_classes, int32_t label_kind,
                              const int32_t *feature, const double *threshold, const int32_t *left,
                              const int32_t *right, const int32_t *counts);
spmv_status_t spmv_gnb_load(int32_t n_classes, int32_t label_kind, const double *mu,
                            const double *w, const double *c, const int32_t *count);
spmv_status_t spmv_classifier_unload(int32_t which);

/* Device inference of a loaded classifier (synchronous).  variant: the
 * selected variant; label: the predicted class index (variant or bottleneck
 * class); fallback: 1 if no feasible class has support (the selector then
 * falls back to profiling); leaf: the tree leaf (-1 for naive Bayes);
 * scores: the naive Bayes scores s_k (8 slots; zeros for the tree).  Output
 * pointers may be NULL.  SPMV_ERR_NO_MODEL if the classifier is not loaded. */
spmv_status_t spmv_classifier_predict(int32_t which, const double features[12], uint32_t feasible,
                                      int32_t *variant, int32_t *label, int32_t *fallback,
                                      int32_t *leaf, double scores[8]);

/* ----------------------------------------------------------------------- */
/* Solver loop                                                              */

/* Conjugate gradients (Hestenes and Stiefel 1952) with the plan's current
 * variant: the iterative method whose SpMVs repay the selection.  The plan
 * must be FP64 and square, its matrix symmetric positive definite.  d_b
 * (N doubles) is read; d_x (N doubles) holds the start and receives the
 * result.  Stops when ||r|| <= rtol ||b|| (r the updated residual) or after
 * max_iters iterations; *iters and *rel_resid (||r|| / ||b||) may be NULL.
 * Synchronous on `stream`; deterministic (fixed-order dot products);
 * allocates 3 N doubles of workspace per call (kept blocks are reused). */
spmv_status_t spmv_cg(spmv_plan_t plan, const double *d_b, double *d_x, int32_t max_iters,
                      double rtol, void *stream, int32_t *iters, double *rel_resid);

/* ----------------------------------------------------------------------- */
/* Allocation-free SpMV                                                     */

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  y = A x
 * with the MERGE_PATH variant's kernels (merge-path splits, then tiles and
 * their carry fix-up), without a plan: the splits and carries live in a
 * static device array of 8 MiB that each GPU holds from the first call on it
 * until the process ends.  Nothing is allocated (no hipMalloc, hipFree or
 * allocating library call) and nothing needs clearing (every split and carry
 * is written before it is read).  Arguments as for spmv_plan_create and
 * spmv_execute; the CSR is not validated (the caller guarantees the
 * invariants listed at the top of this file).  N + NNZ above 8 MiB / 20 B
 * times 2048 items (about 858 million) returns SPMV_ERR_ARG before any
 * device work.  Asynchronous on `stream`.  Calls that overlap in time on
 * one GPU share its array and race: serialise them (one stream, or events).
 * The result equals spmv_execute's with MERGE_PATH on the same data, bit for
 * bit. */
spmv_status_t spmv_merge_path_noalloc(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                      const int32_t *d_rowptr, const int32_t *d_colind,
                                      const void *d_val, int32_t val_dtype, const void *d_x,
                                      void *d_y, void *stream);

/* ----------------------------------------------------------------------- */
/* Utilities                                                                */

/* FP64 -> FP32 (to_dtype SPMV_F32) or bfloat16 bits (SPMV_BF16), one
 * round-to-nearest-even from FP64.  d_out has n elements of 4 or 2 bytes. */
spmv_status_t spmv_quantize(const double *d_in, void *d_out, int64_t n,
                            int32_t to_dtype, void *stream);

/* Seeded synthetic CSR on the device.  family: 0 5-point 2D Laplacian,
 * 1 9-point 2D box, 2 7-point 3D star, 3 27-point 3D box (p[0] = grid side;
 * p[1] = 1 for random values else constant 2d/2d-1 stencil values),
 * 4 uniform random (p = n_rows, n_cols, per_row), 5 banded (p = n, d16,
 * half_width), 6 random rows (p = n, d16), 7 power law (p = n, p16, cap,
 * force_long), 8 short rows (p = n).  Counter-based SplitMix64 draws.
 * Call with d_rowptr only (others NULL) to get *nnz_out and rowptr; then
 * again with d_colind and d_val of nnz_out elements. */
spmv_status_t spmv_generate(int32_t family, const int64_t *params, int32_t n_params,
                            uint64_t seed, int32_t *d_rowptr, int32_t *d_colind,
                            double *d_val, int64_t *nnz_out, void *stream);

/* x_j = 2 u_j - 1 with u_j = (h(seed, 1, j) >> 11) 2^-53 (double, n elements). */
spmv_status_t spmv_generate_vector(int64_t n, uint64_t seed, double *d_x, void *stream);

/* Device memory the library releases (derived formats, temporaries) is kept
 * per device for reuse, up to 2 GiB in all and 1 GiB per block, because plans
 * are typically created and destroyed around every solve.  Other allocators
 * (PyTorch's caching allocator) cannot see these blocks: call this before
 * large allocations elsewhere if memory is tight.  It frees every kept block
 * on every device.  A failed allocation of the library also frees the kept
 * blocks of its device and retries once.  Destroying a plan waits for its
 * stream once (for the whole device if spmv_execute ran it on other streams)
 * before its buffers join the kept blocks. */
spmv_status_t spmv_release_cached_blocks(void);

/* Evict the Infinity Cache: read and write a 512 MiB scratch buffer. */
spmv_status_t spmv_cache_flush(void *stream);

/* Attainable HBM bandwidth over a `bytes` buffer: streaming read and copy,
 * median of 5 runs, in GB/s (1e9 B/s). */
spmv_status_t spmv_hbm_probe(int64_t bytes, double *read_gbs, double *copy_gbs);

/* Ceiling of an x-gather-bound SpMV: median time (s, hipEvents on the
 * default stream, 5 runs after 2 warm-ups) of `gathers` random reads of
 * elem_bytes (4 or 8) from `windows` (1, 2, 4 or 8) windows of window_elems
 * elements, workgroup b reading window (b mod 8) mod windows as the x-block
 * kernels map XCDs to column slices; eight reads per thread, four in
 * flight, indices from a per-thread linear congruential sequence (no index
 * loads).  The windows live in the cache-flush buffer (512 MiB). */
spmv_status_t spmv_gather_probe(int64_t window_elems, int32_t elem_bytes, int32_t windows,
                                int64_t gathers, double *t_median_s);

/* The same ceiling with the indices streamed (indexed != 0): every thread
 * also reads, coalesced, a 4-byte column and an elem_bytes value per gather
 * from arrays of `gathers` elements (uniform random columns in the window),
 * which is all a CSR kernel must do per nonzero besides summing rows and
 * writing y.  indexed = 0 is spmv_gather_probe.  Allocates the two arrays
 * (12 or 8 bytes per gather) for the call. */
spmv_status_t spmv_gather_probe2(int64_t window_elems, int32_t elem_bytes, int32_t windows,
                                 int64_t gathers, int32_t indexed, double *t_median_s);

/* Message of the calling thread's last error ("" if none). */
const char *spmv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPMVSEL_H */
