/*
 * spmm.h - C ABI of the MI355X (gfx950) CSR sparse x dense matrix multiply.
 *
 * Operation (paper Sec. 1; input/output statement of Algorithm 1):
 *   A is m-by-k in CSR: A_rowptr[m+1] (int32 offsets, A_rowptr[0] = 0,
 *   non-decreasing), A_colind[nnz] (int32, 0 <= c < k; need not be sorted;
 *   duplicates are summed), A_vals[nnz].
 *   B is k-by-n dense, row-major, row stride ld elements.
 *   C is m-by-n dense, row-major, row stride ld elements, float32.
 *   C = A * B, i.e. C[i,c] = sum over p in [rowptr[i], rowptr[i+1]) of
 *   vals[p] * B[colind[p], c]. C is overwritten (never accumulated into);
 *   rows of A without entries give exact zeros. Sums run in float32 in an
 *   order fixed by the plan, so repeated calls give bitwise equal results.
 *
 * Storage types: vals and B share one type - float32, bfloat16 or float16
 * (16-bit types as their bit patterns); they are widened exactly to float32
 * and accumulated in float32. C, dC and dB are always float32. Where the
 * forward kernels take bfloat16 entries two at a time (v_dot2_f32_bf16),
 * bfloat16 values below 2^-126 in magnitude (float32's denormal range) count
 * as zero.
 *
 * Pointers: every pointer argument is a DEVICE pointer unless its name ends
 * in _host. The caller owns A, B, C and every other array it passes; the
 * library owns plans and batches and the device workspace inside them
 * (allocated at create time, freed at destroy). C must not alias A, B or a
 * plan's workspace.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 * stream). Execute calls only enqueue kernels on it: they allocate nothing
 * and never synchronise the host, so they may be captured into a hipGraph.
 * Create/build calls may allocate and synchronise.
 *
 * Sizes: m, k, n and ld fit int32; nnz is at most 2^31 - 4097 (entry
 * indices are int32 in the kernels); larger sizes give SPMM_ERR_UNSUPPORTED.
 *
 * Errors: every call returns an int status (spmm_status). Nothing aborts or
 * throws across the ABI. spmm_last_error() returns a thread-local message
 * for the last failing call on this thread. Argument checks happen on the
 * host before any launch; kernel launch failures are reported as
 * SPMM_ERR_HIP. The CSR structure itself (monotone rowptr, colind in range)
 * is the caller's contract and is not checked by execute calls;
 * spmm_csr_validate() checks it on request.
 *
 * Alignment: for 16-byte vector access the library checks B, C, dC, dB and
 * ld; when they are not aligned it falls back to element access on its own
 * (no error).
 */
#ifndef SPMM_MI355X_H
#define SPMM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spmm_status {
    SPMM_OK = 0,
    SPMM_ERR_INVALID = -1,     /* bad argument (null pointer, negative size, ld < n, ...) */
    SPMM_ERR_UNSUPPORTED = -2, /* valid but not supported (dtype, config) */
    SPMM_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
    SPMM_ERR_NOMEM = -4,       /* device or host allocation failed */
    SPMM_ERR_STATE = -5        /* destroyed/foreign handle, or call not allowed now */
} spmm_status;

typedef enum spmm_dtype { SPMM_F32 = 0, SPMM_BF16 = 1, SPMM_F16 = 2 } spmm_dtype;

/* How a plan chooses its kernel.
 *   PAPER    : the mean-row-length rule of Sec. 5.4 - merge-based when
 *              nnz / m < 9.35, row split otherwise (compared exactly as
 *              100 * nnz < 935 * m).
 *   AUTOTUNE : time the candidate kernels and shapes on scratch buffers of
 *              the plan's sizes and keep the fastest. Column panels
 *              (spmm_config.col_panels) are candidates when the rows are
 *              sorted, B is larger than 4 MB and rows hold 64 or more entries
 *              on average.
 *   ROWSPLIT / MERGE : force that kernel with default shapes.
 *   RULE     : the rule re-derived on MI355X from the kernel-choice
 *              sweep (the Sec. 5.4 procedure on this GPU): merge-based when
 *              the mean row length is below 4 or the longest row has 4096
 *              or more entries (row split cannot spread one row over
 *              several workgroups); otherwise row blocks of 2 rows when
 *              n >= 32, the rows are sorted, k < 2^24 and blocks of 2 rows
 *              hold at most 0.9 distinct columns per entry (from the
 *              row-block sweep; costs a row-order check and one union
 *              count on the device); row split otherwise.
 *   NZSPLIT  : force the nonzero split (Sec. 4, scheme (a): the 1-D
 *              partition the paper's merge-based kernel implements) with
 *              default shapes.
 *   ROWBLOCK : force the row-block kernel (2 rows per block, default
 *              shapes); SPMM_ERR_UNSUPPORTED unless every row's column
 *              indices strictly increase and k < 2^24. AUTOTUNE also times
 *              it (2 and 4 rows per block) when those hold, the longest row
 *              has at most 4096 entries and blocks of 2 rows hold at most
 *              0.9 distinct columns per entry. */
typedef enum spmm_mode {
    SPMM_MODE_PAPER = 0,
    SPMM_MODE_AUTOTUNE = 1,
    SPMM_MODE_ROWSPLIT = 2,
    SPMM_MODE_MERGE = 3,
    SPMM_MODE_RULE = 4,
    SPMM_MODE_NZSPLIT = 5,
    SPMM_MODE_ROWBLOCK = 6
} spmm_mode;

/* ROWSPLIT: Sec. 4.1. MERGE: merge-based, pieces cut on the diagonals of
 * the merge path (2-D search; each piece holds items_per_wg rows plus
 * nonzeros). NZSPLIT: merge-based, pieces cut by nonzero count (each piece
 * holds items_per_wg nonzeros and however many row ends fall among them,
 * found by a 1-D search on the row offsets): cheaper to partition, but a run
 * of empty rows lands in one piece and is written by one lane group.
 * ROWBLOCK (not in the paper; for matrices whose neighbouring rows share
 * columns, such as stencils): row split over blocks of rows_per_block
 * consecutive rows. The plan stores, per block, the sorted union of the
 * block's columns (one 32-bit word per distinct column: the column and the
 * set of the block's rows holding it, k * 4 bytes at most per row), and the
 * kernel gathers each B row of the union once per block instead of once per
 * entry. Only for the ordinary product: spmm_execute_semiring on such a plan
 * runs row split with the same lane shape. */
typedef enum spmm_kernel {
    SPMM_KERNEL_ROWSPLIT = 0,
    SPMM_KERNEL_MERGE = 1,
    SPMM_KERNEL_NZSPLIT = 2,
    SPMM_KERNEL_ROWBLOCK = 3
} spmm_kernel;

/* Semirings of spmm_execute_semiring: (add, multiply, identity). */
typedef enum spmm_semiring {
    SPMM_PLUS_TIMES = 0, /* (+, *, 0): the ordinary product */
    SPMM_MIN_PLUS = 1,   /* (min, +, +inf): shortest-path relaxation */
    SPMM_MAX_PLUS = 2,   /* (max, +, -inf) */
    SPMM_MAX_TIMES = 3   /* (max, *, -inf) */
} spmm_semiring;

/* Kernel shape. A zero field means "choose automatically". */
typedef struct spmm_config {
    int32_t kernel;        /* spmm_kernel */
    int32_t vec;           /* elements per lane per B-row access: 1, or the 16-byte width
                              (4 for float32, 8 for 16-bit types) */
    int32_t lanes_per_row; /* row split (Sec. 4.1): lanes of a wavefront sharing one row of A
                              (ROWBLOCK: one block of rows), a power of two from the lanes one
                              B row needs up to 64 */
    int32_t unroll;        /* B-row gathers in flight per lane group: 1, 2, 4 or 8 */
    int32_t items_per_wg;  /* merge-based (Sec. 4.2): merge items (rows + nonzeros) per
                              workgroup, 64 .. 8192; NZSPLIT: nonzeros per workgroup */
    int32_t tile_cols;     /* columns per column tile (Fig. 3(a)'s 2-D grid): a multiple of
                              vec; the product runs over ceil(n / tile_cols) tiles, each
                              re-reading A but touching only its columns of B. 0 = as wide as
                              one wavefront covers (64 * vec columns) */
    int32_t rows_per_block;/* ROWBLOCK: rows per block, 2, 4 or 8 (0 = 2); other kernels
                              ignore it */
    int32_t tile_order;    /* ROWSPLIT / ROWBLOCK: order in which workgroups take their rows.
                              0 = automatic: strips across planes (see below) when the plan
                              finds plane structure and one plane of B rows is larger than an
                              XCD's 4 MB L2, else row order; 1 = row order; 2 = strips across
                              planes whenever plane structure is found. Plane structure: the
                              offsets colind - row form a near cluster (|offset| <= h) and a
                              far one around +-D no wider than it, with D >= 16 h - the
                              neighbour planes of a 3-D stencil, D rows apart. Rows are then
                              taken in strips of S consecutive rows (S a power of two dividing
                              D, the largest whose B rows for three planes fill at most 2 MB)
                              through every plane before the next strip, so each B row is
                              reused from L2 by the three planes that need it. Only the order
                              of the workgroups changes: results are bitwise the same. */
    int32_t col_panels;    /* ROWSPLIT: 0 or 1 = none; P = 2 .. 64 = column panels (the 2-D
                              tiling Sec. 6 discusses, with one row tile): A's columns are cut
                              into P panels of ceil(k / P) columns and the product runs as P
                              row-split passes, pass p taking from every row the entries whose
                              column lies in panel p and adding their sum into C (pass 0
                              overwrites C), so each pass gathers from a slice of B that can
                              stay in an XCD's L2. The plan stores each row's panel starts
                              ((P + 1) * m ints). Needs column indices that strictly increase
                              in every row (SPMM_ERR_UNSUPPORTED otherwise). Each element of C
                              is summed panel by panel: a different order from P = 1. */
} spmm_config;

typedef struct spmm_plan_info {
    int64_t m, k, nnz, n, ld;
    int32_t dtype;         /* spmm_dtype */
    int32_t mode;          /* spmm_mode the plan was created with */
    int32_t paper_choice;  /* kernel the Sec. 5.4 rule picks for this matrix */
    spmm_config config;    /* the shape that execute calls use */
    int32_t lanes_per_slot;/* lanes that cover one B row (or one 64*vec column tile) */
    int32_t col_tiles;     /* column tiles (grid y) */
    int64_t num_parts;     /* MERGE / NZSPLIT: workgroups P (coordinates hold P + 1 pairs) */
    int64_t max_row_len;   /* longest row (from the device row statistics) */
    double mean_row_len;   /* nnz / m */
    double tuned_ms;       /* AUTOTUNE: median time of the chosen candidate, else 0 */
    int32_t has_transpose; /* spmm_transpose_build has run */
    int64_t long_rows;     /* rows with 1024 or more entries (device row statistics) */
    int64_t plane_rows;    /* row split / row blocks taken in strips: the plane distance D in
                              rows, else 0 */
    int64_t strip_rows;    /* ... and the strip S in rows, else 0 */
} spmm_plan_info;

typedef struct spmm_plan_s* spmm_plan_t;
typedef struct spmm_batch_s* spmm_batch_t;

/* ---------------------------------------------------------------- one call
 * C = A * B in float32 (Sec. 1), with an internal plan cache keyed by
 * (A_rowptr, A_colind, m, k, n, ld, device, stream); safe to call from
 * several host threads.
 *
 * Kernel choice: mode RULE restricted to the paper's two kernels - the
 * procedure of Sec. 5.4 (a threshold on row statistics, fitted by timing
 * both kernels) re-derived on MI355X: merge-based when the mean row length
 * is below 4 or the longest row has 4096 or more entries, row split
 * otherwise. This departs from the paper's own threshold (merge-based iff
 * nnz / m < 9.35; SPMM_MODE_PAPER of spmm_plan_create), which picks row
 * split for every matrix with mean row length >= 9.35 however long its
 * longest row - on a 1M x 1M power-law matrix with mean 16 and rows of up to
 * 100,000 entries, 6x slower than merge-based. Row blocks are not used here.
 *
 * Synchronisation: on a miss the call reads A_rowptr[m] (nnz) and the device
 * row statistics back to the host together - one stream synchronisation, so
 * a miss is not capture-safe - then plans without further synchronisation.
 * A hit only enqueues work.
 *
 * Structure changes: a cached row-split plan depends on the structure only
 * through m. A cached merge-based plan keeps the merge-path partition of the
 * row offsets it was made for, so each call first re-checks that partition
 * against A_rowptr on the device (one small kernel): coordinates that no
 * longer lie on the merge path of the current row offsets are searched
 * again, so a different structure with the same nnz (for instance a new
 * matrix placed at a freed matrix's addresses) is computed correctly. If
 * A_rowptr[m] differs from the cached nnz, that call writes NaN into all of
 * C and reads nothing else of A, and the next call with the same arguments
 * returns SPMM_ERR_STATE and drops the plan (the one after plans afresh);
 * call spmm_cache_clear() after freeing or changing a structure to avoid
 * this. Rows with invalid offsets (A_rowptr[0] != 0, decreasing) are refused
 * with SPMM_ERR_INVALID on a miss.
 *
 * Returns SPMM_OK for m == 0 or n == 0 without touching memory. */
int spmm_csr(const int32_t* A_rowptr, const int32_t* A_colind, const float* A_vals,
             const float* B, float* C, int64_t m, int64_t k, int64_t n, int64_t ld,
             void* stream);

/* ---------------------------------------------------------------- no allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): C = A * B
 * in float32 like spmm_csr, with no allocation of any kind, no host
 * synchronisation and no plan cache.
 *
 * Differences from spmm_csr: the caller passes nnz (it must equal
 * A_rowptr[m]; nothing is read back), and the kernel is the Sec. 5.4 choice
 * of the paper - merge-based iff 100 * nnz < 935 * m, row split otherwise -
 * with that kernel's default shape, rows in row order. The merge-based
 * kernel's workspace (P + 1 merge-path coordinates, P carry-out row ids and
 * P carry-out rows of n floats, P = ceil((m + nnz) / W) pieces of W items)
 * lives in one static device array of SPMM_NOALLOC_SCRATCH_BYTES per GPU,
 * held from the library's first use on that GPU until the process ends.
 * Sizes whose workspace exceeds it return SPMM_ERR_UNSUPPORTED before any
 * launch (use spmm_csr or a plan then). Row split uses no workspace.
 *
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap in time on one GPU (two streams, two host
 * threads) race and give wrong results; serialise them. Results equal
 * spmm_csr's within the float32 tolerance of summation order (bitwise when
 * both pick the same kernel and shape). */
#define SPMM_NOALLOC_SCRATCH_BYTES (64 << 20)
int spmm_csr_noalloc(const int32_t* A_rowptr, const int32_t* A_colind, const float* A_vals,
                     const float* B, float* C, int64_t m, int64_t k, int64_t nnz, int64_t n,
                     int64_t ld, void* stream);

/* Facts of the plan spmm_csr holds for these arguments (the same key; the
 * current device): kernel, shape, row statistics. SPMM_ERR_STATE when no
 * such plan is cached. */
int spmm_csr_plan_info(const int32_t* A_rowptr, const int32_t* A_colind, int64_t m, int64_t k,
                       int64_t n, int64_t ld, void* stream, spmm_plan_info* info_host);

/* Drop every cached plan of spmm_csr (frees their workspace). */
int spmm_cache_clear(void);

/* Autotuner results kept across processes. The autotuner remembers, per
 * process, the shape it chose for each key (device, m, k, nnz, n, ld,
 * longest row, rows of >= 1024 entries, dtype, unroll, largest merge piece,
 * row blocks allowed, column panels allowed); a plan with a known key takes
 * that shape without timing trials. spmm_tune_cache_save writes every
 * remembered choice to the text file path_host (format version 2: a header
 * line, then one line per key - 13 key fields, the 9 fields of spmm_config,
 * the tuned time in ms); spmm_tune_cache_load adds a file's choices (a later
 * entry for one key replaces an earlier one). A loaded shape is checked like
 * a forced config when a plan would use it and ignored (tuned afresh) if it
 * does not fit. Returns SPMM_ERR_INVALID for an unreadable, unwritable or
 * malformed file (nothing is loaded then). */
int spmm_tune_cache_save(const char* path_host);
int spmm_tune_cache_load(const char* path_host);

/* ---------------------------------------------------------------- plans
 * Create a plan for the structure (A_rowptr, A_colind) with nnz nonzeros
 * (nnz must equal A_rowptr[m]; given by the caller so no read-back is
 * needed), output width n, row stride ld (shared by B and C), storage type
 * dtype and kernel choice mode. The plan keeps the two structure pointers;
 * they must stay valid and unchanged while the plan lives. Creation runs a
 * device row-statistics pass and, for merge-based plans, the Phase 1
 * partition of Algorithm 1 (the merge-path coordinates of Sec. 4); it
 * synchronises `stream`. AUTOTUNE additionally allocates scratch B/C/vals of
 * the plan's sizes, times the candidates and frees the scratch. */
int spmm_plan_create(spmm_plan_t* out_plan, const int32_t* A_rowptr, const int32_t* A_colind,
                     int64_t m, int64_t k, int64_t nnz, int64_t n, int64_t ld,
                     int32_t dtype, int32_t mode, void* stream);

/* Same, with an explicit kernel shape (zero fields are filled in). */
int spmm_plan_create_config(spmm_plan_t* out_plan, const int32_t* A_rowptr,
                            const int32_t* A_colind, int64_t m, int64_t k, int64_t nnz,
                            int64_t n, int64_t ld, int32_t dtype, const spmm_config* config_host,
                            void* stream);

/* C = A * B with the plan's kernel: row split (Sec. 4.1) or merge-based
 * Phases 2-3 of Algorithm 1 (Sec. 4.2). A_vals and B are of the plan's
 * dtype; C is float32. Enqueue only. The carry-out workspace of a
 * merge-based plan belongs to the plan: products (and SDDMM or A^T calls)
 * with one plan must not overlap on different streams; use one plan per
 * stream. */
int spmm_execute(spmm_plan_t plan, const void* A_vals, const void* B, float* C, void* stream);

/* The same as spmm_execute, for measurement: records the caller's events
 * ev_before / ev_after (hipEvent_t as void*, may be NULL) on `stream`
 * immediately before and after the launch of the main kernel (row split,
 * or Phase 2 of the merge-based kernel; the merge fix-up pass follows
 * ev_after), so their elapsed time is that kernel's duration. */
int spmm_execute_events(spmm_plan_t plan, const void* A_vals, const void* B, float* C,
                        void* ev_before, void* ev_after, void* stream);

/* C[i,c] = (add) over the entries p of row i of (A_vals[p] (multiply)
 * B[colind[p], c]) for one of the semirings above - SpMM as an instance of
 * the GraphBLAS product on a semiring (Sec. 1). Same plan, kernels and
 * launch shape as spmm_execute; rows without entries give the identity.
 * min and max are exact, so results do not depend on the summation order:
 * each element is the float32 rounding of the exact result whenever every
 * product or sum of two stored values is exact in float64. Enqueue only. */
int spmm_execute_semiring(spmm_plan_t plan, int32_t semiring, const void* A_vals, const void* B,
                          float* C, void* stream);

/* Plan facts for the host (sizes, the chosen config, Sec. 5.4 choice). */
int spmm_plan_info_get(spmm_plan_t plan, spmm_plan_info* info_host);

/* Merge-based plans: copy the P + 1 merge-path coordinates (i_p, j_p) that
 * start the pieces into coords_host (2 * (P + 1) int32, interleaved i, j).
 * MERGE: the states on diagonals min(p * W, m + nnz). NZSPLIT: (0, 0), then
 * j_p = min(p * W, nnz) with i_p the number of rows whose end is <= j_p,
 * and (m, nnz) last. cap is the capacity in pairs. Synchronous.
 * SPMM_ERR_STATE for row-split and row-block plans. */
int spmm_plan_partition(spmm_plan_t plan, int32_t* coords_host, int64_t cap);

/* Free the plan and its workspace (after the work queued with it is done:
 * the call synchronises the device). */
int spmm_plan_destroy(spmm_plan_t plan);

/* ---------------------------------------------------------------- backward
 * Gradients of L = <dC, A B> (not in the paper; A^T products are named as
 * future work in Sec. 6): dB = A^T dC and dvals = SDDMM(dC, B) on A's
 * pattern.
 *
 * spmm_transpose_build: build, once per structure, the CSR of A^T
 * (k rows, m columns): AT_rowptr[k+1], AT_colind[nnz] holding the row ids of
 * A in increasing order within each row of A^T, and perm[nnz] with
 * AT_vals[q] = A_vals[perm[q]]. Stored in the plan; allocates; synchronises.
 * The product with A^T gets a plan of its own, made with the plan's mode
 * (RULE for a plan made from a forced config or in mode ROWBLOCK). */
int spmm_transpose_build(spmm_plan_t plan, void* stream);

/* Copy the transpose into caller buffers (device pointers: k + 1, nnz, nnz
 * int32). Enqueue only. SPMM_ERR_STATE before spmm_transpose_build. */
int spmm_transpose_get(spmm_plan_t plan, int32_t* AT_rowptr, int32_t* AT_colind, int32_t* perm,
                       void* stream);

/* dB (k-by-n, stride ld, float32) = A^T * dC (m-by-n, stride ld, float32):
 * gathers AT_vals = A_vals[perm] into plan workspace and runs the forward
 * kernels on (A^T, dC). Requires spmm_transpose_build. Enqueue only. */
int spmm_execute_t(spmm_plan_t plan, const void* A_vals, const float* dC, float* dB,
                   void* stream);

/* The same dB = A^T * dC without a transpose (the SpMM_T of Sec. 6 on the
 * CSR of A alone): dB is zeroed (columns < n of its k rows), then every
 * entry p of row i adds A_vals[p] * dC[i, :] into row colind[p] of dB with
 * float atomic adds, the work split on the merge pieces the plan holds for
 * SDDMM. Needs no spmm_transpose_build and allocates nothing. The order of
 * the additions into an element depends on timing, so results are not
 * bitwise repeatable (they meet the same float32 tolerance; integer-valued
 * data is exact). dB must not alias dC. Enqueue only. */
int spmm_execute_t_scatter(spmm_plan_t plan, const void* A_vals, const float* dC, float* dB,
                           void* stream);

/* dvals[p] = sum_c dC[row(p), c] * B[colind[p], c] for every stored entry
 * p of A (float32 out, nnz entries). dC is float32, B of the plan's dtype.
 * The work is split on diagonal merge pieces of 1024 items that the plan
 * builds at creation (a merge plan with pieces of that size uses its own).
 * Enqueue only. */
int spmm_sddmm(spmm_plan_t plan, const float* dC, const void* B, float* dvals, void* stream);

/* ---------------------------------------------------------------- batches
 * Many independent products C_b = A_b * B_b of uneven sizes in one
 * persistent kernel launch (plus one fix-up launch for merge-based
 * problems), captured once into a hipGraph and replayed by spmm_batch_run.
 * Each problem's kernel and shape comes from its own plan (mode as in
 * spmm_plan_create; AUTOTUNE times each problem on its own buffers, which
 * overwrites C_b). All problems share dtype. The problem array is copied;
 * the device buffers it names must stay valid while the batch lives. */
typedef struct spmm_problem {
    const int32_t* A_rowptr;
    const int32_t* A_colind;
    const void* A_vals;
    const void* B;
    float* C;
    int64_t m, k, nnz, n, ld;
} spmm_problem;

int spmm_batch_plan(spmm_batch_t* out_batch, const spmm_problem* problems_host, int64_t count,
                    int32_t dtype, int32_t mode, void* stream);

/* Launch the captured graph on `stream`: all products of the batch. The
 * batch's work queues live in the batch object, so runs of one batch must
 * not overlap (queue them on one stream, or wait between streams); runs of
 * different batches may. Enqueue only. */
int spmm_batch_run(spmm_batch_t batch, void* stream);

/* The same work without the graph: direct kernel launches on `stream`
 * (same rule on overlapping runs). */
int spmm_batch_run_direct(spmm_batch_t batch, void* stream);

/* Per-problem chosen config (problem index b). */
int spmm_batch_problem_config(spmm_batch_t batch, int64_t b, spmm_config* config_host);

/* Free the batch, its plans and its graph (synchronises the device first). */
int spmm_batch_destroy(spmm_batch_t batch);

/* ---------------------------------------------------------------- misc */
/* Check CSR validity on the device: rowptr[0] == 0, non-decreasing,
 * rowptr[m] == nnz, 0 <= colind < k. Synchronous. SPMM_OK or
 * SPMM_ERR_INVALID (message in spmm_last_error). */
int spmm_csr_validate(const int32_t* A_rowptr, const int32_t* A_colind, int64_t m, int64_t k,
                      int64_t nnz, void* stream);

/* Measurement aid for the roofline of the gather kernels (no product uses
 * it): `threads` lanes (a multiple of 256) read rows of `row_bytes` bytes
 * (32, 64, 128, 256 or 512; 16 bytes per lane, row_bytes / 16 lanes per row) at
 * pseudo-random row indices of `table` (device, 16-byte aligned, table_rows
 * rows of row_bytes bytes, table_rows a power of two up to 2^31), `steps`
 * rows per lane group
 * (a multiple of 8, eight in flight), and write one float per lane to `out`
 * (device, `threads` floats) - the access the products make to B, without
 * their reads of A and writes of C. Bytes read: threads * steps * 16.
 * Enqueue only: time it with events on `stream`. SPMM_ERR_INVALID on a bad
 * argument. */
int spmm_calibrate_gather(const void* table, int64_t table_rows, int32_t row_bytes,
                          int32_t steps, float* out, int64_t threads, void* stream);

const char* spmm_status_string(int status);
const char* spmm_last_error(void);
/* Library version, e.g. "0.1.0". */
const char* spmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPMM_MI355X_H */
