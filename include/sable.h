/* libsable: hybrid VDIA + VBR + CSR sparse matrix-vector and matrix-matrix products on an
 * AMD Instinct MI355X (gfx950).
 *
 * The library follows the plan / extract / dispatch method of "Bring Your Own Formats and
 * Kernels: Composable Abstractions for Sparse Matrix Computation" (SABLE):
 *   - a plan holds a residual matrix and an ordered list of extractions (Sec. 3 "Initialize",
 *     "Extract"); each extractor claims the nonzeros that fit its structure into a format and
 *     leaves the rest, and the list must end with a catch-all CSR extractor (Sec. 3 "Dispatch",
 *     Sec. 4.3 "Format Composition");
 *   - the band extractor (Sec. 4.2, Alg. 3 and Alg. 4) produces the VDIA format (Sec. 4.2.1);
 *   - the block extractor (Sec. 4.1, Alg. 1 and Alg. 2) produces variable-size delta-dense
 *     blocks (VBR, App. B);
 *   - every region accumulates into one output (Sec. 3.4), which is valid because the
 *     operations are sums (Sec. 5 "Kernels").
 * Extraction runs as GPU scans; every region of a product runs in one fused kernel launch.
 *
 * Conventions for every function:
 *   - All matrix and vector pointers are DEVICE pointers unless a parameter says "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Products are
 *     asynchronous on that stream and never synchronise; errors of an asynchronous kernel
 *     surface at a later call or at hipStreamSynchronize. sable_plan synchronises internally.
 *   - Dense operands are row-major: x[ncols], y[nrows]; X[ncols * n] with X[j*n + c];
 *     Y[nrows * n] with Y[i*n + c] (App. A.2). Operands must not alias; X and Y must be
 *     16-byte aligned.
 *   - y / Y are OVERWRITTEN with A x / A X; rows without entries get 0.
 *   - Argument checks happen before any GPU work. On failure an out-handle is set to NULL
 *     and nothing leaks. No C++ exception crosses this interface. sable_last_error()
 *     returns a thread-local message describing the last failure of the calling thread.
 */
#ifndef SABLE_H
#define SABLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SABLE_OK = 0,
  SABLE_ERR_INVALID_ARG = 1,  /* NULL pointer, bad size, bad threshold, misaligned operand */
  SABLE_ERR_INVALID_CSR = 2,  /* indptr not monotone / not 0..nnz, column out of range or
                                 columns not strictly increasing within a row */
  SABLE_ERR_INCOMPLETE = 3,   /* extractor list does not end with the CSR catch-all (Sec. 3) */
  SABLE_ERR_TOO_LARGE = 4,    /* nnz >= 2^31, or literal block search over budget */
  SABLE_ERR_OOM = 5,          /* device or host allocation failed */
  SABLE_ERR_HIP = 6,          /* a HIP runtime call failed */
  SABLE_ERR_INTERNAL = 7
} sable_status;

/* Extractor kinds (Sec. 3.2): band -> VDIA, block -> VBR, catch-all -> CSR. */
enum { SABLE_X_VDIA = 1, SABLE_X_VBR = 2, SABLE_X_CSR = 3 };

/* Block search variants: the literal recursive search of Alg. 1/2 ("paper"), allowed when
 * nrows * ncols * max(nrows, ncols) <= 2^37 or when its sparse window scan's work on the VBR
 * extractor's input is <= 2^37 (one step per outer span (o0, o1) of length >= ceil(sqrt(
 * amin_block)) of the row and column passes, plus min(inner length, entries of the span));
 * a tiled delta-dense detection ("tiled") that scales to any size; "auto" picks paper when
 * it is allowed, else tiled. A paper request for dimensions where even one step per span is
 * over budget fails before any GPU work; otherwise the work is counted on the residual. */
enum { SABLE_VBR_AUTO = 0, SABLE_VBR_PAPER = 1, SABLE_VBR_TILED = 2 };

typedef struct {
  int32_t kind;     /* SABLE_X_* */
  int32_t vbr_mode; /* SABLE_VBR_*; ignored for other kinds */
} sable_extractor;

/* Input matrix in canonical CSR (device arrays, borrowed only during sable_plan):
 * indptr[nrows+1] with indptr[0] = 0 and indptr[nrows] = nnz, indices[nnz] strictly
 * increasing within each row, values[nnz]. Explicitly stored zeros are structural. */
typedef struct {
  int32_t nrows, ncols;
  int64_t nnz;
  const int32_t* indptr;
  const int32_t* indices;
  const float* values;
} sable_csr;

/* Extraction thresholds. Densities are per-mille integers p (delta = p/1000) and every
 * density test is the exact integer test 1000*nnz >= p*area.
 *   delta_block_pm  block density floor delta (Sec. 4.1, default 500; must be >= 500
 *                   because the block score uses (density - 0.5)^1.5)
 *   delta_band_pm   band density floor (Sec. 4.2; default 750, the band evaluation value)
 *   amin_block      minimum block area A_min (Sec. 4.1, default 2500)
 *   amin_band       minimum total area of an accepted band region (Alg. 3, default 2500)
 *   lseg            minimum segment length l_seg (Alg. 4; default 64) - also the count
 *                   threshold for candidate diagonals (Alg. 3)
 *   wmax            cap on ribbon extent below / above the candidate diagonal (default 32,
 *                   at most 63)
 *   dmax            largest |offset| considered (Alg. 3; -1 = all)
 *   coverage_pm     block coverage cutoff (Alg. 1; default 80 = 8%)
 *   tile_set_mask   tiled search: bit t selects tile size {4,6,8,16,32}[t]; 0 = all
 *   flags           SABLE_F_SPLIT_BF16 (default on): keep bf16 hi/lo copies of block values
 *                   for split-precision matrix-core SpMM; SABLE_F_SPARSE_SEARCH: run the
 *                   literal block search's window scans over non-empty inner lines only (the
 *                   same blocks; used anyway where the dense scan's tables would not fit). */
typedef struct {
  int32_t delta_band_pm, delta_block_pm;
  int64_t amin_band, amin_block;
  int32_t lseg, wmax, dmax, coverage_pm, tile_set_mask;
  uint32_t flags;
} sable_thresholds;

#define SABLE_F_SPLIT_BF16 1u
#define SABLE_F_SPARSE_SEARCH 2u

typedef struct sable_plan_s* sable_plan_t;   /* opaque, library-owned */
typedef struct sable_batch_s* sable_batch_t; /* opaque, library-owned */

/* Plan statistics (counts of the exported formats and of one product's compulsory bytes). */
typedef struct {
  int32_t nrows, ncols;
  int64_t nnz;             /* structural nonzeros of A */
  int32_t nseg;            /* VDIA segments */
  int64_t nidiag;          /* total stored diagonals over all segments */
  int64_t vdia_cells;      /* stored VDIA values (fill included) */
  int64_t vdia_nnz;        /* A's entries held by VDIA */
  int32_t nblk;            /* VBR blocks */
  int32_t vbr_mode_used;   /* SABLE_VBR_PAPER or SABLE_VBR_TILED (0 if no VBR extractor) */
  int32_t vbr_tile;        /* chosen tile size in tiled mode, else 0 */
  int32_t pad0;
  int64_t vbr_cells;       /* stored VBR values (fill included) */
  int64_t vbr_nnz;
  int64_t csr_nnz;
  int64_t bytes_matrix;    /* algorithmic matrix bytes of one product (formats only) */
  int64_t device_bytes;    /* device memory held by the plan */
  double plan_ms;          /* wall time of sable_plan */
  int32_t spmv_variant, spmm_variant, plain_variant; /* kernel variants in use */
  int32_t far_split;       /* 1 if the streamed SpMV variants gather far-column CSR entries
                              in a separate pass (see sable_spmv) */
  int64_t far_nnz;         /* CSR entries handled by that pass */
  double spec_ms;          /* wall time of sable_plan_specialize (0 if not specialized) */
  uint64_t structure_hash; /* hash of A's sparsity pattern, the extractor list and the
                              thresholds: plans with equal hashes have the same formats and
                              schedules (the key of the autotuning cache) */
  uint64_t partition_hash; /* hash of the partition itself: the format and slot of every
                              entry and the VDIA segments and VBR blocks. Equal hashes mean
                              the same formats with the same layout, whatever the extractor
                              list or thresholds that produced them */
  int64_t mm_panels;       /* SpMM operand panels (64 rows x 32 block columns) */
  int64_t mm_units;        /* their occupied units (one row x 8 columns, 32 bytes each) */
} sable_plan_stats;

/* Host buffers for sable_plan_export, sized from sable_plan_info:
 *   vdia_val[vdia_cells] (diagonal-major within a segment: value of row r0+r on diagonal t
 *   of segment s at seg_val_ptr[s] + t*seg_nrows[s] + r), idiag[nidiag], seg_*[nseg];
 *   blk[4*nblk] = (r0, r1, c0, c1) sorted by (r0, c0), blk_val_ptr[nblk], vbr_val[vbr_cells]
 *   (column-major within a block); csr_ptr[nrows+1], csr_col[csr_nnz], csr_val[csr_nnz];
 *   owner[nnz] (0 VDIA, 1 VBR, 2 CSR for every input entry) and slot[nnz] (its index in
 *   that format's value array); vbr_bf16[vbr_cells]: the split-bf16 copy that the
 *   matrix-core SpMM multiplies, one 32-bit word hi | lo << 16 per block cell in the order of
 *   vbr_val (hi = bf16 round-to-nearest-even of the value a, lo = the same rounding of
 *   a - hi; all zero when the plan keeps no bf16 copies). Any pointer may be NULL to skip
 *   that array. */
typedef struct {
  float* vdia_val;
  int32_t* idiag;
  int32_t* seg_row_start;
  int32_t* seg_nrows;
  int32_t* seg_ndiags;
  int64_t* seg_val_ptr;
  int32_t* seg_idiag_ptr;
  int32_t* blk;
  int64_t* blk_val_ptr;
  float* vbr_val;
  int64_t* csr_ptr;
  int32_t* csr_col;
  float* csr_val;
  int8_t* owner;
  int64_t* slot;
  uint32_t* vbr_bf16;
} sable_partition_host;

/* Fill *out with the defaults listed at sable_thresholds. */
sable_status sable_thresholds_default(sable_thresholds* out);

/* Build a plan (Sec. 3): validate A, run the extractors of list[0..nlist-1] in order on the
 * residual (each kind at most once; SABLE_X_CSR must be last, else SABLE_ERR_INCOMPLETE),
 * pack the formats and the execution schedule. A's arrays are only read during the call;
 * the plan owns copies of everything it needs. th may be NULL (defaults). Synchronises
 * `stream`. Errors: INVALID_ARG, INVALID_CSR, INCOMPLETE, TOO_LARGE (nnz >= 2^31 or
 * SABLE_VBR_PAPER over budget), OOM, HIP. */
sable_status sable_plan(const sable_csr* A, const sable_extractor* list, int32_t nlist,
                        const sable_thresholds* th, void* stream, sable_plan_t* out);

/* Release every resource of a plan. NULL is accepted. */
sable_status sable_plan_destroy(sable_plan_t p);

/* Host copy of the plan statistics. */
sable_status sable_plan_info(sable_plan_t p, sable_plan_stats* out);

/* Copy the formats into caller-owned host buffers (layout at sable_partition_host).
 * Synchronous. */
sable_status sable_plan_export(sable_plan_t p, const sable_partition_host* out);

/* y = A x over all regions in one fused launch (Sec. 3.4 shared output): per row
 * (sum over VDIA segments + sum over VBR blocks) + sum over CSR entries, in a fixed order,
 * so results are bitwise reproducible. x[ncols], y[nrows] device fp32.
 * Far-column split: for wide matrices (more than 2^20 columns) whose CSR part has at least
 * 2^16 entries more than 2^17 columns away from their row, the streamed variants first run
 * a gather pass over those entries (grouped by 8192-column slices of x, each staged in
 * LDS) into a product buffer owned by the plan, then the fused launch adds the products
 * in the same order as without the pass. Two calls with the same plan must therefore not
 * run concurrently on different streams. A plan that is its CSR part alone (no band
 * segment, no block) runs as sable_csr_spmv: its CSR part is the input in the input's order,
 * and the plain kernels (the plan's plain variant) are the hybrid launch's CSR-only case. */
sable_status sable_spmv(sable_plan_t p, const float* x, float* y, void* stream);

/* Y = A X with n >= 1 right-hand sides (row-major, App. A.2). VBR blocks run on matrix
 * cores as split-bf16 products (hi*hi + hi*lo + lo*hi, fp32 accumulate) when the plan kept
 * bf16 copies (SABLE_F_SPLIT_BF16) and the selected SpMM variant uses them (0, 3 or 4, see
 * sable_plan_set_variant), otherwise in fp32 on the vector units; VDIA and CSR run in fp32.
 * X and Y must be 16-byte aligned (SABLE_ERR_INVALID_ARG otherwise). */
sable_status sable_spmm(sable_plan_t p, const float* X, float* Y, int32_t n, void* stream);

/* Plain CSR SpMV of the whole input matrix: the baseline kernel family (wave / sub-wave per
 * row) applied to A. Equivalent to a plan with list {CSR}; provided for comparisons. */
sable_status sable_csr_spmv(sable_plan_t p, const float* x, float* y, void* stream);

/* ---- FP64 executor (the paper's precision, Sec. 5 / App. A) -------------------------
 * The partition depends only on the structure, so an fp32 plan also serves fp64 products:
 * sable_update_values_f64 stores fp64 values (device values[nnz], input order, same
 * structure as at planning time) in fp64 copies of every format (allocated on the first
 * call, asynchronous on `stream`). sable_spmv_f64 / sable_spmm_f64 then run the same fused
 * tile bodies in fp64 (VBR blocks on the fp64 VALU: gfx950's fp64 matrix-core peak equals
 * its fp64 vector peak); x[ncols], y[nrows], X[ncols x n], Y[nrows x n] device fp64,
 * row-major. Summation orders are fixed as in the fp32 executor (bitwise reproducible).
 * The far-column split (op 3 of sable_plan_set_variant) applies to sable_spmv_f64 as well,
 * with fp64 copies of the far entries' values and products (the same result bit for bit).
 * Both return SABLE_ERR_INVALID_ARG until fp64 values have been set. */
sable_status sable_update_values_f64(sable_plan_t p, const double* values, void* stream);
sable_status sable_spmv_f64(sable_plan_t p, const double* x, double* y, void* stream);
sable_status sable_spmm_f64(sable_plan_t p, const double* X, double* Y, int32_t n, void* stream);

/* ||y - yref||_2 / ||yref||_2 (or ||y - yref||_2 if yref = 0) reduced in FP64 on the GPU:
 * y[len] fp32 device, yref[len] fp64 device, *out host. Synchronises `stream`. */
sable_status sable_error_norm_f64(const float* y, const double* yref, int64_t len,
                                  void* stream, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): the same relative error as sable_error_norm_f64,
 * from the same kernels, written to a DEVICE double *out_dev; asynchronous on `stream` (no
 * synchronisation, no host copy, no allocation of any kind). The partial sums live in a
 * library-owned static device array of 1024 pairs of doubles (16 KiB, one copy per GPU,
 * held until the process ends); the reduction grid is capped at 1024 workgroups, so every
 * len >= 0 fits. Each call overwrites that GPU's array: calls that overlap on one GPU (on
 * different streams, or from several threads) race and must be serialised by the caller.
 * Errors: SABLE_ERR_INVALID_ARG (out_dev NULL, len < 0, NULL y / yref with len > 0),
 * SABLE_ERR_HIP. */
sable_status sable_error_norm_f64_noalloc(const float* y, const double* yref, int64_t len,
                                          void* stream, double* out_dev);

/* Replace the values of A (same structure as at planning time, device values[nnz]) in every
 * format without re-extracting: the inspector-executor reuse of Sec. 5 "Evaluation
 * scenario". Asynchronous on `stream`. */
sable_status sable_update_values(sable_plan_t p, const float* values, void* stream);

/* ---- Autotuning ---------------------------------------------------------------------
 * Time a small grid of launch parameters for the plan's fused kernel on `stream` (op 0 =
 * SpMV, 1 = SpMM with n columns) and keep the fastest. The SpMM choice is kept per n: later
 * sable_spmm calls with that n use it, other n use the most recent choice. x/X, y/Y are
 * scratch operands of the right sizes. Synchronises `stream`.
 * The grid: SpMV tile kernels (streamed tiles of 256/512/1024 rows, W lanes per CSR row,
 * row-length bins mapped to subwave widths, non-temporal loads, the far-column split, the
 * specialized kernel when present), the plain CSR baseline's kernels, and for SpMM the block
 * path (matrix cores from registers or from LDS-staged panels, fp32 VALU) and the work split.
 * Results are cached process-wide by (structure_hash, specialized or not, op, n, device): a
 * plan with a pattern, extractor list and thresholds tuned before takes the stored choice at
 * once, without timing anything. */
sable_status sable_autotune(sable_plan_t p, int32_t op, int32_t n, const float* x, float* y,
                            void* stream);

/* Forget every cached autotuning result (the next sable_autotune times again). */
sable_status sable_autotune_cache_clear(void);

/* Select a fused-kernel variant explicitly (the set sable_autotune chooses from).
 * op 0 = hybrid SpMV: 0..2 streamed tiles of 256/512/1024 rows, 3..7 with 1/2/4/8/16 lanes
 *        per row on tiles of 256/W rows (bands lane per row; for W > 1 a row's lanes share its
 *        block columns and CSR entries), 8..10 = 0..2 with non-temporal matrix loads,
 *        11 = the run-time specialized kernel (after sable_plan_specialize), 12..14 = CSR
 *        rows binned by length (0, 1-4, 5-8, 9-16, 17-32, 33-64, > 64 entries) within tiles of
 *        up to 256 rows, each bin's rows taken by subwaves whose width gives about 1, 2 or 4
 *        entries per lane (a wave for rows over 64 entries), bands and blocks lane per row;
 *        15, 16 = 0 and 8 as a persistent launch (a few workgroups per CU each run many tiles
 *        in turn, loading the next tile's record, row pointers and first entries while the
 *        current tile computes; the same results bit for bit);
 * op 1 = SpMM: 0 tiled with matrix-core blocks (for n <= 32 the four waves split the tile's
 *        row slices, otherwise its column chunks), 1 tiled fp32, 2 one wave per row, 3 tiled
 *        with matrix-core blocks and the column-chunk split at every n, 4 tiled with the
 *        blocks on matrix cores from operands staged in LDS: per 64-row tile, the distinct
 *        rows of X its blocks read are loaded once, 32 at a time, and multiplied in
 *        16x16x32 bf16 steps;
 * op 2 = plain CSR baseline: 0..2 streamed, 3..9 with 1..64 lanes per row, 10..12 = 0..2
 *        with non-temporal matrix loads, 13..15 = row-length bins as SpMV 12..14, 16, 17 = 0
 *        and 10 as persistent launches (as SpMV 15, 16);
 * op 3 = far-column split of the streamed SpMV variants: 0 off, 1 on (when the plan has one).
 * For a plan with neither bands nor blocks, op 0 selects nothing but the specialized kernel
 * (11): its SpMV runs the plain kernels of op 2.
 * Every variant computes the same product; each is bitwise reproducible on its own. An
 * explicit SpMM variant applies to every n (it clears the per-n autotuned choices). */
sable_status sable_plan_set_variant(sable_plan_t p, int32_t op, int32_t variant);

/* ---- Run-time specialization (Sec. 3.3 - 3.4 code generation, on the GPU) ------------
 * Generate HIP source for this plan's SpMV with every band segment (rows, diagonal offsets,
 * value offset) and every VBR block (rectangle, value offset) as literal constants, compile it
 * with hipRTC for the current device and keep it in the plan as SpMV variant 11 (the
 * autotuner then considers it). Work is one thread per row, one workgroup per 256-row tile,
 * the tile's CSR entries streamed through LDS; per row (bands, diagonals ascending, then
 * blocks in block order) + CSR in index order.
 * Meant for small matrices: SABLE_ERR_TOO_LARGE if the plan has more than 4096 tiles,
 * more than 16384 (tile, segment or block) pairs or a segment wider than 128 diagonals;
 * SABLE_ERR_HIP with the compiler log in sable_last_error if compilation fails.
 * Synchronous; a second call is a no-op. */
sable_status sable_plan_specialize(sable_plan_t p, void* stream);

/* ---- Learned planner (matrix features -> MLP -> extractor list and delta) ------------- */
#define SABLE_NFEAT 140
#define SABLE_NCLASS 15

/* 140 fp32 features of A computed on the GPU: 64-bin histogram of diagonal run lengths,
 * 64-bin histogram of 16x16 tile densities, row-length mean/var/max and 9 extras.
 * out is a host array of SABLE_NFEAT floats. Synchronises `stream`. */
sable_status sable_features(const sable_csr* A, void* stream, float* out);

/* Class c of the planner's label space: list kind (c / 3) in {CSR, VDIA+CSR, VBR+CSR,
 * VDIA+VBR+CSR, VBR+VDIA+CSR}, delta = {500, 700, 900}[c % 3] for bands and blocks.
 * Writes up to 3 extractors to list and returns their count in *nlist. */
sable_status sable_class_plan(int32_t c, sable_extractor* list, int32_t* nlist,
                              sable_thresholds* th);

/* MLP 140-128-128-15 with ReLU (weights row-major W1[128][140], b1, W2[128][128], b2,
 * W3[15][128], b3, all device fp32, in one contiguous parameter array of
 * SABLE_MLP_NPARAM floats in that order). */
#define SABLE_MLP_NPARAM (128 * 140 + 128 + 128 * 128 + 128 + 15 * 128 + 15)

/* Forward pass for a batch: feats[B][140] (device, already normalised) -> logits[B][15]. */
sable_status sable_mlp_forward(const float* params, const float* feats, int32_t batch,
                               float* logits, void* stream);

/* One training step of softmax cross-entropy with Adam (lr, beta1, beta2, eps; step t >= 1)
 * on a batch: feats[B][140], labels[B] (int32 class ids) -> params updated in place; grads
 * (SABLE_MLP_NPARAM) receives the batch-mean gradient; m, v Adam moments; *loss (host) the
 * batch-mean loss. t = 0 computes the loss and the gradient only (no update; m, v unused).
 * Synchronises `stream`. */
sable_status sable_mlp_train_step(float* params, float* grads, float* m, float* v,
                                  const float* feats, const int32_t* labels, int32_t batch,
                                  float lr, float beta1, float beta2, float eps, int32_t t,
                                  void* stream, float* loss);

/* Exhaustive timed search over the 15 classes (the fallback and yardstick of the learned
 * planner): plans A with every class, autotunes each plan's SpMV kernels (sable_autotune),
 * times the chosen kernel on `stream` (after one warm-up, three rounds of `reps`
 * back-to-back launches; the median per-launch average) and returns the fastest plan.
 * x[ncols], y[nrows] are scratch device vectors; times_ms (host, SABLE_NCLASS entries, may be
 * NULL) receives every class's time. Classes whose plans have the same partition_hash (for
 * one, classes 0..2, CSR only) are timed once and share that time; ties go to the lower class
 * index. ref_ms (host, 2 entries, may be NULL) receives, tuned and timed the same
 * way, the plain CSR baseline (sable_csr_spmv) and the default extractor list [VDIA, VBR,
 * CSR] with the default thresholds. */
sable_status sable_plan_exhaustive(const sable_csr* A, const float* x, float* y, int32_t reps,
                                   void* stream, sable_plan_t* out, int32_t* best_class,
                                   float* times_ms, float* ref_ms);

/* Learned plan choice: features of A, normalised as (f - feat_mean) / feat_std (host arrays
 * of SABLE_NFEAT), MLP forward with params (device, SABLE_MLP_NPARAM), softmax. If the top
 * probability is >= tau_conf the top class is planned; otherwise the exhaustive search runs
 * (x, y scratch as above). Outputs: the plan, the class used, the top probability and
 * whether the fallback ran. */
sable_status sable_plan_auto(const sable_csr* A, const float* params, const float* feat_mean,
                             const float* feat_std, float tau_conf, const float* x, float* y,
                             void* stream, sable_plan_t* out, int32_t* chosen_class,
                             float* confidence, int32_t* fell_back);

/* ---- Batched persistent execution ---------------------------------------------------- */
typedef struct {
  int32_t op;      /* 0 SpMV, 1 SpMM */
  int32_t n;       /* right-hand sides for SpMM (1 for SpMV) */
  const float* x;  /* x or X (device) */
  float* y;        /* y or Y (device) */
} sable_batch_item;

/* Concatenate the work of count plans into persistent kernels captured in one hipGraph:
 * SpMV items run the 256-row streamed tile (the plan's SpMV variant 0, whatever variant it
 * holds), SpMM items the fused SpMM tile in the plan's mode; each item's result is bitwise
 * equal to that standalone launch. Items without rows do nothing and complete at the start.
 * The plans and operands must outlive the batch. Errors: SABLE_ERR_INVALID_ARG for a bad
 * item (op, n, NULL or misaligned operands), SABLE_ERR_TOO_LARGE past 2^31 work units. */
sable_status sable_batch_create(const sable_plan_t* plans, const sable_batch_item* items,
                                int32_t count, void* stream, sable_batch_t* out);
/* Launch the captured graph on `stream` (asynchronous). */
sable_status sable_batch_run(sable_batch_t b, void* stream);
/* Per-item completion time in GPU clock ticks since the batch start, of the last run
 * (host array of count). Synchronises the batch's last stream. *tick_hz receives the
 * counter frequency. */
sable_status sable_batch_latencies(sable_batch_t b, uint64_t* ticks, double* tick_hz);
sable_status sable_batch_destroy(sable_batch_t b);

/* Thread-local description of the last failure on the calling thread ("" if none). */
const char* sable_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SABLE_H */
