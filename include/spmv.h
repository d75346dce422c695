/*
 * libspmv -- CRS sparse matrix-vector multiplication for AMD MI355X (gfx950).
 *
 * The operation is the Compressed Row Storage product of the paper's
 * Sect. 1.2: the nonzeros of A are held row by row in `val`, their column
 * indices in `col_idx` and the start offset of every row in `row_ptr`, and
 *
 *     C(i) = sum_{j = row_ptr(i)}^{row_ptr(i+1)-1} val(j) * B(col_idx(j))
 *
 * with C overwritten (the listing accumulates into a C that starts at zero).
 *
 * Conventions for every entry point:
 *  - Indices are 0-based. row_ptr and col_idx are int32 (the paper's 4-byte
 *    index). n_rows, n_cols and nnz may each be at most 2^31 - 4097 (the
 *    kernels step through rows and nonzeros in int32 with strides of up to
 *    4096); larger inputs return SPMV_ERR_UNSUPPORTED.
 *  - Every array argument is a DEVICE pointer owned by the caller unless the
 *    comment says "host". A handle BORROWS the matrix arrays and the
 *    workspace: they must stay alive and unchanged until the handle is
 *    destroyed. The library never allocates device memory for a matrix; all
 *    per-matrix device state lives in the caller's workspace.
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *    Apply calls are asynchronous on that stream, never synchronise, never
 *    allocate, and may be captured into a HIP graph. They are const on the
 *    handle: concurrent applies on different streams with disjoint C are
 *    safe. B and C must not overlap.
 *  - Results are deterministic run to run: no floating-point atomics; each
 *    output element is reduced by one thread group in a fixed order.
 *  - Errors are returned as negative status codes; nothing is thrown across
 *    the ABI. spmv_last_error() gives a thread-local description of the last
 *    failure on the calling thread.
 *  - Accuracy: each row is a sum of the products val(j)*B(col_idx(j)) in
 *    float64 (fused multiply-add allowed), so |C - C_exact| is at most about
 *    nnz_row * 2^-53 * sum_j |val(j) B(col_idx(j))|. Float32-stored val and B
 *    are widened exactly; their products are exact in float64, so only the
 *    float64 summation error remains.
 */
#ifndef SPMV_H
#define SPMV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ types */

typedef struct spmv_plan* spmv_handle;        /* one analysed matrix */
typedef struct spmv_batch* spmv_batch_handle; /* an uneven batch of matrices */
typedef struct spmv_graph* spmv_graph_handle; /* an instantiated HIP graph */
typedef struct spmv_split* spmv_split_handle; /* a local/remote split plan */

typedef enum { SPMV_F64 = 0, SPMV_F32 = 1 } spmv_dtype;

typedef enum {
  SPMV_OK = 0,
  SPMV_ERR_INVALID_ARG = -1, /* null pointer, negative size, bad enum, ldb < k ... */
  SPMV_ERR_BAD_CRS = -2,     /* row_ptr/col_idx violate the CRS definition */
  SPMV_ERR_UNSUPPORTED = -3, /* size or dtype combination not supported */
  SPMV_ERR_WORKSPACE = -4,   /* workspace missing, too small or misaligned */
  SPMV_ERR_HIP = -5,         /* a HIP runtime call failed */
  SPMV_ERR_STATE = -6        /* call not valid in the current state */
} spmv_status;

/* Kernel variants: the same product with different thread-to-work maps. */
typedef enum {
  SPMV_V0_THREAD_ROW = 0, /* one lane per row */
  SPMV_V1_LANES4 = 1,     /* 4 lanes per row, DPP reduction */
  SPMV_V2_LANES16 = 2,    /* 16 lanes per row, DPP reduction */
  SPMV_V3_WAVE_ROW = 3,   /* one 64-lane wavefront per row */
  SPMV_V4_LDS_BLOCK = 4,  /* nnz-balanced row blocks staged through LDS */
  SPMV_V5_BINNED = 5,     /* row-length bins, one launch per non-empty bin */
  SPMV_V6_SELL64 = 6,     /* chunked copy: 64 rows per chunk stored column by column
                             (sliced ELLPACK, built at create; needs SPMV_FLAG_SELL) */
  SPMV_NUM_VARIANTS = 7
} spmv_variant;

/* The MLP selector ranks V0..V6; its V6 output is ignored for a plan without
 * the V6 copy (no SPMV_FLAG_SELL, or the copy did not fit its reserve). */
#define SPMV_NUM_SELECTOR_OUTPUTS 7

/* spmv_create flags. The low byte selects how the variant is chosen. */
/* Default: V4 where the plan takes its window form, V6 where the plan holds
 * the chunked copy, else the MLP selector's pick if weights are loaded, else
 * V4. */
#define SPMV_SELECT_DEFAULT 0x0u
#define SPMV_SELECT_MLP 0x1u      /* MLP selector; fall back to autotune when unsure */
#define SPMV_SELECT_AUTOTUNE 0x2u /* time every variant, keep the fastest */
#define SPMV_SELECT_FIXED 0x3u    /* use the variant in bits 8..11 */
#define SPMV_FLAG_VARIANT(v) (SPMV_SELECT_FIXED | ((uint32_t)(v) << 8))
#define SPMV_FLAG_SKIP_VALIDATE 0x10000u /* trust the CRS arrays (no device check) */
/* Reserve workspace for the V6 copy and build it at create. The copy holds
 * 64 * (sum over chunks of the longest row in the chunk) slots of 4-byte
 * column index + value, plus a 2-byte column delta per slot and a 4-byte base
 * per 64 slots; the reserve is 1.5 nnz + 4096 slots (rounded up to 64) at 14
 * bytes each whatever val_dtype is, plus the bases. A chunk whose every slot
 * has its 64 columns within 254 of each other is read through 8-bit deltas (9
 * instead of 12 bytes per float64 slot), else within 65534 through 16-bit
 * deltas (10 bytes); other chunks read the 4-byte columns. All give the same
 * products in the same order. A pattern whose padded size
 * exceeds it still gets a plan, without V6 (spmv_get_sell_slots reports
 * SPMV_ERR_STATE); asking for V6 by name then fails with UNSUPPORTED. With
 * a built copy the selector's V6 output is a candidate (without one it is
 * ignored), and autotune times V6 with the others. */
#define SPMV_FLAG_SELL 0x20000u
/* V4 in its B-staging form: each row block copies a range of B into LDS (its
 * exact column span when that fits 2048 entries, 4096 for float32 plans, else
 * that many columns around its rows) and gathers from it where it can. By default a plan stages when at
 * least a quarter of its blocks fit exactly, and autotune times both forms;
 * these flags force one form (setting both is SPMV_ERR_INVALID_ARG). */
#define SPMV_FLAG_V4_STAGE_ON 0x40000u
#define SPMV_FLAG_V4_STAGE_OFF 0x80000u
/* V4 in its window form: super-blocks of 4096 rows, one 512-lane workgroup
 * each, that copy the two (float32 plans: three) most used aligned 4096-column
 * windows of B into LDS and gather from them where they can; each wavefront
 * streams its 512 rows' nonzeros on its own, and each lane adds one row's
 * products in CRS order, so every row equals the Sect. 1.2 loop bit for bit.
 * The windows are chosen at create from the columns of each super-block. By
 * default a plan takes this form when fewer than a quarter of its row blocks
 * fit the staging form exactly, the windows hold at least 65% of the
 * nonzeros and there are at least 512 super-blocks. Exclusive with the two
 * flags above. */
#define SPMV_FLAG_V4_WINDOWS 0x200000u
/* With SPMV_FLAG_SELL: read every chunk of the V6 copy through its 4-byte
 * columns (the deltas are not built). Without SPMV_FLAG_SELL it is
 * SPMV_ERR_INVALID_ARG. */
#define SPMV_FLAG_SELL_WIDE 0x100000u

#define SPMV_NUM_FEATURES 16
#define SPMV_MLP_PARAMS 5703 /* 16->64->64->7: W1 b1 W2 b2 W3 b3, [out,in] row-major */

/* ---------------------------------------------------------- single matrix */

/*
 * Bytes of device workspace spmv_create needs for this shape (host call, no
 * device work). The workspace holds the row-block table, the row-length bin
 * lists, the analysis counters, the selector scratch and, with
 * SPMV_FLAG_SELL, the reserve of the V6 copy. It depends only on
 * (n_rows, n_cols, nnz, flags) and is stable across calls. `bytes` is a host
 * pointer.
 */
int spmv_workspace_size(int64_t n_rows, int64_t n_cols, int64_t nnz, uint32_t flags,
                        size_t* bytes);

/*
 * Analyse a CRS matrix and build a plan (the paper's point that the
 * bookkeeping of a sparsity pattern is done once and reused, Sect. 3.1).
 *  h        host out: the new handle
 *  n_rows, n_cols >= 0; nnz = row_ptr[n_rows] >= 0; each at most 2^31 - 4097
 *  row_ptr  int32[n_rows+1], col_idx int32[nnz], val float64 or float32 [nnz]
 *  val_dtype SPMV_F64 or SPMV_F32
 *  workspace device, >= spmv_workspace_size() bytes, 256-byte aligned
 *  flags    SPMV_SELECT_* | SPMV_FLAG_SKIP_VALIDATE | SPMV_FLAG_SELL
 *  stream   the stream for the analysis kernels
 * Unless SPMV_FLAG_SKIP_VALIDATE is set, the CRS arrays are checked on the
 * device (row_ptr[0]=0, nondecreasing, row_ptr[n_rows]=nnz, 0<=col<n_cols)
 * and SPMV_ERR_BAD_CRS is returned on violation. This call synchronises the
 * stream: once to read back the analysis, and again for every timed launch
 * of autotune (also when SPMV_SELECT_MLP falls back to it). Apply calls never
 * do.
 */
int spmv_create(spmv_handle* h, int64_t n_rows, int64_t n_cols, int64_t nnz,
                const int32_t* row_ptr, const int32_t* col_idx, const void* val,
                int val_dtype, void* workspace, size_t ws_bytes, uint32_t flags, void* stream);

/*
 * C = A*B (Sect. 1.2). B: n_cols entries of b_dtype; C: float64[n_rows].
 * b_dtype must equal the handle's val_dtype (float64 with float64, or
 * float32 val with float32 B: float64 accumulation and output either way).
 */
int spmv_apply(spmv_handle h, const void* B, int b_dtype, double* C, void* stream);

/*
 * Multi-RHS form, row-major blocks: C[i*ldc + c] = sum_j val(j) B[col_idx(j)*ldb + c]
 * for 0 <= c < k. Requires k >= 1, ldb >= k, ldc >= k. The matrix stream is
 * read once for all k columns: from the V6 copy when the plan runs V6, k <= 8
 * and the rows average at least 8 entries, else from the CRS arrays. k = 1
 * with ldb = ldc = 1 is spmv_apply (the plan's variant and form, same results)
 * unless the plan runs V6 with rows averaging fewer than 8 entries.
 */
int spmm_apply(spmv_handle h, int32_t k, const void* B, int64_t ldb, int b_dtype, double* C,
               int64_t ldc, void* stream);

/* Variant in use (host out). */
int spmv_get_variant(spmv_handle h, int* variant);
/* Switch the variant of an existing plan (every table is built at create);
 * SPMV_ERR_STATE for V6 on a plan without the V6 copy. */
int spmv_set_variant(spmv_handle h, int variant);
/* The 16 row-statistics features computed at create (host out, float64[16]). */
int spmv_get_features(spmv_handle h, double* features);
/* The selector's predicted relative log2 times of V0..V6 from create (host
 * out, float[SPMV_NUM_SELECTOR_OUTPUTS]); SPMV_ERR_STATE if no selector ran. */
int spmv_get_predictions(spmv_handle h, float* pred);
/* Per-variant times in microseconds measured by SPMV_SELECT_AUTOTUNE (host
 * out, double[SPMV_NUM_VARIANTS]): the median of five timed launches for a
 * variant within 1.5x of the best time seen before it, else its single timed
 * launch; +infinity for a variant the plan does not have. SPMV_ERR_STATE if
 * autotune did not run. */
int spmv_get_autotune_times(spmv_handle h, double* us);
/* Slots of the V6 copy (host out): 64 * sum of chunk widths, >= nnz; the
 * padding is slots - nnz. SPMV_ERR_STATE if the plan has no V6 copy. */
int spmv_get_sell_slots(spmv_handle h, int64_t* slots);
/* Bytes one V6 product reads from the copy (host out): per chunk its offset
 * and delta flag, its slot bases where it has deltas, and per slot the value
 * and the column (1- or 2-byte delta or 4-byte index). B and C come on top.
 * Copies the chunk widths and flags to the host (blocking). SPMV_ERR_STATE if
 * the plan has no V6 copy. */
int spmv_get_sell_stream_bytes(spmv_handle h, int64_t* bytes);
/* Chunks of the V6 copy read through 8-bit and through 16-bit column deltas,
 * and all chunks (host out). Copies the per-chunk flags to the host (a
 * blocking copy after the device work of create, which has completed when
 * create returns). SPMV_ERR_STATE if the plan has no V6 copy. */
int spmv_get_sell_deltas(spmv_handle h, int64_t* chunks8, int64_t* chunks16, int64_t* chunks);
/* Whether V4 runs in its B-staging form (host out: 1 or 0; see
 * SPMV_FLAG_V4_STAGE_ON). */
int spmv_get_v4_staged(spmv_handle h, int* staged);
/* The three forms of V4: the same row blocks and sums, different B access. */
typedef enum { SPMV_V4_PLAIN = 0, SPMV_V4_STAGED = 1, SPMV_V4_WINDOWS = 2 } spmv_v4_form;
/* The V4 form in use (host out), and the nonzeros whose column lies in their
 * super-block's windows (host out, may be null). */
int spmv_get_v4_form(spmv_handle h, int* form, int64_t* win_covered);
/* Switch the V4 form of a plan (every table is built at create). */
int spmv_set_v4_form(spmv_handle h, int form);
/* Number of row blocks of the LDS-block variant (host out). */
int spmv_get_num_blocks(spmv_handle h, int64_t* nblocks);
int spmv_destroy(spmv_handle h);

/* ----------------------------------------------------------------- solvers */

/*
 * Conjugate gradients for a symmetric positive definite plan (square): solves
 * A x = b, x holding the initial guess on entry (device float64 arrays of n).
 * Every vector operation and scalar stays on the device; an iteration is one
 * product with the plan's variant (an FP32-storage plan gets a float32 copy of
 * the search direction; the iteration itself is float64), two fixed-order dot
 * products and three vector updates, in four launches. For a plan running V0
 * or V1 the search-direction update, the product (a lane per row, products
 * added in CRS order: V0's arithmetic) and the first dot are one launch, so an
 * iteration is two; with V0 its values equal the four-launch iteration's bit
 * for bit. use_graph != 0 captures the iterations between two residual
 * checks (the largest divisor of check_every up to 64) in one HIP graph and
 * replays it, the same kernels in the same order (needs a non-null stream).
 * The recurrence residual ||r||/||b|| is read back every check_every
 * iterations (one sync each); stops when it is <= tol or after maxit
 * iterations. iters, relres:
 * host out. workspace: spmv_cg_workspace_size(n) bytes, 256-byte aligned.
 * Results are bitwise reproducible for a given plan, b and x0.
 */
int spmv_cg_workspace_size(int64_t n, size_t* bytes);
int spmv_cg_solve(spmv_handle h, const double* b, double* x, double tol, int32_t maxit,
                  int32_t check_every, int32_t use_graph, void* workspace, size_t ws_bytes,
                  int32_t* iters, double* relres, void* stream);

/*
 * spmv_cg_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * solver scratch (residual, search direction, A p, the float32 copy for
 * FP32-storage plans, the reduction partials and arrival counters) lives in
 * a file-scope device array of the library, 32 MiB per GPU, held from the
 * first call on that GPU until the process ends. No call allocates, frees or
 * calls an allocating routine. Iterations run as separate launches (no graph
 * mode). Arguments, results and synchronisation as spmv_cg_solve; the plan's
 * device must be current (else SPMV_ERR_STATE).
 * Limit: n <= 931,680 (36 bytes per row plus 13 KB), else
 * SPMV_ERR_UNSUPPORTED. Every call on a GPU shares that GPU's array and the
 * array keeps the last call's contents (each call initialises what it reads):
 * calls that overlap in time on one GPU race, from any host thread or stream.
 */
int spmv_cg_solve_noalloc(spmv_handle h, const double* b, double* x, double tol, int32_t maxit,
                          int32_t check_every, int32_t* iters, double* relres, void* stream);

/*
 * k steps of the Lanczos recurrence (no reorthogonalisation) from the device
 * start vector v0 (float64[n], not modified, must be nonzero). Host out:
 * alpha[0..k-1] (diagonal of T_k) and beta[0..k-1] with beta[j] = beta_{j+1}
 * (beta[0..k-2] are the off-diagonals of T_k; beta[k-1] is the norm of the
 * last residual vector). The eigenvalues of T_k approximate the extreme
 * eigenvalues of a symmetric A. A zero beta (invariant subspace) makes the
 * following values non-finite. A step is four launches (the product with the
 * plan's variant, two fused reductions, the scaling of the next vector); for
 * a plan running V0 or V1 it is two (the next vector formed where the product
 * gathers it, the product a lane per row in CRS order, alpha; then beta),
 * with V0 equal to the four-launch step bit for bit. workspace:
 * spmv_lanczos_workspace_size bytes.
 */
int spmv_lanczos_workspace_size(int64_t n, int32_t k, size_t* bytes);
int spmv_lanczos(spmv_handle h, const double* v0, int32_t k, double* alpha, double* beta,
                 void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------- local/remote split */

/*
 * The split product of the paper's Sect. 3.1 ("vector mode with naive
 * overlap"): entries whose column lies in [col_lo, col_hi) are "local", the
 * others "remote". Pass 0 writes C = A_local*B, pass 1 adds C += A_remote*B,
 * so C is written twice -- the extra traffic of eq. (2). In a distributed run
 * pass 0 overlaps the exchange of the remote B entries.
 * create copies the two parts (original column indices, original order
 * inside each row) into the caller's workspace; spmv_split_workspace_size
 * gives the bytes (depends only on n_rows, n_cols, nnz). create validates the
 * CRS arrays (SPMV_ERR_BAD_CRS) and synchronises `stream`.
 * apply: pass 0, 1, or -1 for both in order; asynchronous on `stream`.
 */
int spmv_split_workspace_size(int64_t n_rows, int64_t n_cols, int64_t nnz, size_t* bytes);
int spmv_split_create(spmv_split_handle* h, int64_t n_rows, int64_t n_cols, int64_t nnz,
                      const int32_t* row_ptr, const int32_t* col_idx, const void* val,
                      int val_dtype, int64_t col_lo, int64_t col_hi, void* workspace,
                      size_t ws_bytes, void* stream);
int spmv_split_apply(spmv_split_handle h, int pass, const void* B, int b_dtype, double* C,
                     void* stream);
/* Nonzeros in the local and remote parts (host out). */
int spmv_split_get_nnz(spmv_split_handle h, int64_t* nnz_local, int64_t* nnz_remote);
int spmv_split_destroy(spmv_split_handle h);

/* ----------------------------------------------------------- uneven batch */

/*
 * Many independent small matrices, multiplied by one persistent launch.
 * All array-of-pointer arguments are DEVICE arrays (of device pointers);
 * `n_rows`, `n_cols` and `nnz` are HOST arrays of length `count`.
 * The matrices are split into nnz-balanced row tiles whose (matrix, rows)
 * list is built on the device at create. All matrices share val_dtype.
 */
int spmv_batch_workspace_size(int32_t count, int64_t total_rows, int64_t total_nnz,
                              size_t* bytes);
int spmv_batch_create(spmv_batch_handle* h, int32_t count, const int64_t* n_rows,
                      const int64_t* n_cols, const int64_t* nnz,
                      const int32_t* const* row_ptrs, const int32_t* const* col_idxs,
                      const void* const* vals, int val_dtype, void* workspace, size_t ws_bytes,
                      void* stream);
/* C^m = A^m B^m for every m, one launch. Bs / Cs: device arrays of `count`
 * device pointers. */
int spmv_batch_apply(spmv_batch_handle h, const void* const* Bs, double* const* Cs,
                     int b_dtype, void* stream);
/* The same product as `count` separate launches (host arrays of device
 * pointers), for comparison with the persistent launch. */
int spmv_batch_apply_each(spmv_batch_handle h, const void* const* Bs_host,
                          double* const* Cs_host, int b_dtype, void* stream);
int spmv_batch_get_num_tiles(spmv_batch_handle h, int64_t* ntiles);
/* Launch shape of spmv_batch_apply (one kernel launch in every mode):
 *  SPMV_BATCH_TILE_GRID (default) one workgroup per tile; the hardware
 *                       dispatcher balances the uneven tiles
 *  SPMV_BATCH_DYNAMIC   persistent grid sized to the device; workgroups
 *                       claim tiles from a counter in the workspace that
 *                       the last workgroup resets, so applies of one batch
 *                       must not overlap in time
 *  SPMV_BATCH_STATIC    persistent grid; each workgroup owns a contiguous
 *                       range of tiles (no counters)
 * All three give bitwise-identical results. */
typedef enum { SPMV_BATCH_DYNAMIC = 0, SPMV_BATCH_STATIC = 1, SPMV_BATCH_TILE_GRID = 2 } spmv_batch_mode;
int spmv_batch_set_mode(spmv_batch_handle h, int mode);
/* Bytes one spmv_batch_apply reads for the matrices' nonzeros (host out): per
 * tile its record, the values, the chunk's columns (1- or 2-byte deltas where
 * the tile has them, else 4-byte indices) and a long last row's columns past
 * the chunk. row_ptr, B and C come on top. Copies the tile list to the host
 * (blocking). */
int spmv_batch_get_stream_bytes(spmv_batch_handle h, int64_t* bytes);
int spmv_batch_destroy(spmv_batch_handle h);

/* -------------------------------------------------------------- reordering */

/*
 * Reverse Cuthill-McKee ordering of a square CRS pattern (HOST arrays; no
 * device work): perm[new] = old, a permutation of 0..n-1. The graph is the
 * pattern of A + A^T (symmetric_part = 0) or only the entries present in
 * both A and A^T (symmetric_part = 1: one-sided long-range entries, such as
 * random extras, are ignored so they cannot collapse the level structure).
 * Self loops and columns >= n are ignored. Applying it as A' = P A P^T
 * narrows the band of A, which improves the locality of the B gathers (the
 * paper's Sect. 1.3.1 use of RCM). O(nnz log d) time, O(nnz) host memory.
 * SPMV_ERR_BAD_CRS if row_ptr does not start at 0 or decreases.
 */
int spmv_rcm_order(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int symmetric_part,
                   int32_t* perm);

/*
 * Symmetric permutation on the HOST: (row_ptr_out, col_idx_out, val_out) =
 * P A P^T with perm[new] = old; the entries of each new row are sorted by
 * their new column (stable for duplicates). Output arrays are caller-owned
 * host arrays of sizes n+1, nnz, nnz. SPMV_ERR_INVALID_ARG if perm is not a
 * permutation, SPMV_ERR_BAD_CRS if a column is outside [0, n).
 */
int spmv_permute_crs(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const void* val,
                     int val_dtype, const int32_t* perm, int32_t* row_ptr_out,
                     int32_t* col_idx_out, void* val_out);

/* ------------------------------------------------------------- HIP graphs */

/* Start capturing the calls issued on `stream` (thread-local capture mode).
 * Only apply-type calls may be issued until spmv_graph_end. */
int spmv_graph_begin(void* stream);
/* End the capture and instantiate it into *g. */
int spmv_graph_end(void* stream, spmv_graph_handle* g);
int spmv_graph_launch(spmv_graph_handle g, void* stream);
int spmv_graph_destroy(spmv_graph_handle g);

/* ---------------------------------------------------------------- selector */

/*
 * Load the selector network on the current device (host arrays):
 *  params   float[SPMV_MLP_PARAMS] in the layout above
 *  feat_mu, feat_sigma  float[16]: inputs are (feature - mu) / sigma
 *  feat_lo, feat_hi     float[16]: training range; a feature outside
 *                       [lo, hi] makes SPMV_SELECT_MLP fall back to autotune
 *  margin   minimum predicted gap (log2 units) between the best two variants
 *           below which SPMV_SELECT_MLP falls back to autotune
 */
int spmv_selector_load(const float* params, const float* feat_mu, const float* feat_sigma,
                       const float* feat_lo, const float* feat_hi, float margin);
int spmv_selector_loaded(int* loaded);
/* Load a packed weights file (host path): 8-byte magic "SPMVSEL2", then
 * little-endian float32 params[SPMV_MLP_PARAMS], mu[16], sigma[16], lo[16],
 * hi[16], margin[1]. SPMV_ERR_INVALID_ARG if the file is missing or malformed. */
int spmv_selector_load_file(const char* path);

/*
 * Selector network kernels (device arrays, float32), used by the trainer.
 *  forward:  X[nb,16] -> Y[nb,7]; Z1, Z2 [nb,64] keep pre-activations
 *  backward: squared-error loss against T[nb,7], summed over the targets
 *            that are not NaN (a NaN target is a variant without a time, such
 *            as V6 where the copy did not fit) and divided by nb*7
 *            -> grad[SPMV_MLP_PARAMS]; dz scratch: float[nb*(64+64+7)]
 *  adam:     one Adam step t>=1 on theta with moments m, v (all [SPMV_MLP_PARAMS])
 */
int spmv_mlp_forward(const float* theta, const float* X, int32_t nb, float* Y, float* Z1,
                     float* Z2, void* stream);
int spmv_mlp_backward(const float* theta, const float* X, const float* Z1, const float* Z2,
                      const float* Y, const float* T, int32_t nb, float* dz_scratch,
                      float* grad, void* stream);
int spmv_mlp_adam(float* theta, const float* grad, float* m, float* v, int32_t t, float lr,
                  float beta1, float beta2, float eps, void* stream);

/* ------------------------------------------------------------ measurement */

/* STREAM-style triad a[i] = b[i] + s*c[i] over float64[n] (the paper's
 * practical bandwidth ceiling, Sect. 2), for the roofline denominator. */
int spmv_stream_triad(double* a, const double* b, const double* c, double s, int64_t n,
                      void* stream);
/* Plain copy dst[i] = src[i] over float64[n] (counter calibration). */
int spmv_stream_copy(double* dst, const double* src, int64_t n, void* stream);

/* ------------------------------------------------------------------- misc */

const char* spmv_status_string(int status);
const char* spmv_last_error(void);
/* Library version, e.g. "1.0.0". */
const char* spmv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPMV_H */
