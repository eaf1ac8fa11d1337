/*
 * smash.h -- C ABI of libsmash, a row-wise (Gustavson) sparse matrix-matrix
 * multiply C = A * B for AMD Instinct MI355X (gfx950).
 *
 * The operation is the row-wise product of the SMASH thesis (arXiv
 * 2105.14156), Background chapter, eq. "row_wise":
 *     C[i,:] = sum_k A[i,k] * B[k,:],
 * i.e. c_ij = sum_k a_ik * b_kj (eq. "inner_product"), with every output
 * row's partial products merged in an on-chip hash table by atomic
 * compare-and-swap on keys and atomic add on values (SMASH Kernels chapter,
 * section "Hashing Phase"; algorithms "SMASH HASHING" even/odd sections).
 * Output sizing follows the Window Distribution Phase: per-row product
 * counts from the row pointers, then an exact symbolic count.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Matrices are CSR with int32 row pointers and int32 column indices, values
 * FP32 or FP64 (smash_dtype).  All matrix arrays live in device memory and
 * are owned by the caller; the library never frees caller memory.
 * Preconditions on A and B: row_ptr[0] = 0, row_ptr nondecreasing,
 * row_ptr[rows] = nnz, 0 <= col_idx < cols, columns strictly ascending in each
 * row.  With SMASH_OPT_VALIDATE set (the default) these are checked on the
 * device and a violation returns SMASH_ERR_INVALID_CSR.
 * C is returned canonical: int64 row pointer, columns ascending and unique
 * in each row, and every structural product kept, even where the products
 * cancel to 0.0.
 * All work is ordered on the caller's HIP stream.  A context is not
 * thread-safe: use one context per host thread.
 * Every function returns a status; nothing aborts or throws across the ABI.
 * After an error the output buffers hold unspecified values, but nothing
 * outside them is written.  smash_last_error() returns the message of the
 * last failing call on the context.
 *
 * Device memory.  The multiply's calls allocate no device memory: besides
 * its inputs and outputs, a call uses one caller-owned workspace (ws,
 * ws_bytes; device memory, 256-byte aligned, e.g. a torch tensor) whose
 * size smash_workspace_size() reports, and output buffers come from the
 * caller's allocation callback.  A workspace that is too small is never
 * written beyond ws_bytes: the call returns SMASH_ERR_CAPACITY and
 * smash_get_stats() reports the bytes it needs (workspace_bytes).  The
 * context itself holds only a small device header, and the weights of an
 * installed predictor.
 *
 * Host synchronisation.  smash_spgemm_symbolic (and so smash_spgemm)
 * synchronises the stream once, to read nnz(C) back (in global heavy-row
 * mode twice more, to plan the table waves; smash_spgemm_fused once more,
 * to size its staging area).  smash_spgemm_numeric does not synchronise:
 * inconsistencies its kernels detect (a C_row_ptr that does not match the
 * product) are reported by smash_sync() or, failing that, by the next
 * symbolic call on the context.
 */
#ifndef SMASH_H
#define SMASH_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SMASH_OK = 0,
    SMASH_ERR_INVALID_ARG = 1,     /* null pointer, bad shape, bad option */
    SMASH_ERR_INVALID_CSR = 2,     /* validation found a precondition violated */
    SMASH_ERR_INDEX_OVERFLOW = 3,  /* a count does not fit the requested index type */
    SMASH_ERR_CAPACITY = 4,        /* a caller buffer or the C_row_ptr given is too small */
    SMASH_ERR_OUT_OF_MEMORY = 5,   /* device or pinned host allocation failed */
    SMASH_ERR_HIP = 6,             /* a HIP runtime call failed */
    SMASH_ERR_NO_PLAN = 7          /* numeric phase without a matching symbolic phase */
} smash_status;

typedef enum { SMASH_F32 = 0, SMASH_F64 = 1 } smash_dtype;

/* Opaque per-device context: the plan of the last symbolic call (its
 * arrays live in the caller's workspace), options, an installed predictor
 * and per-kernel timing. */
typedef struct smash_ctx_s *smash_ctx;

/* A CSR matrix in device memory (see the conventions above).  val may be
 * NULL for the symbolic phase. */
typedef struct {
    int64_t rows, cols, nnz;
    const int32_t *row_ptr;   /* rows + 1 entries */
    const int32_t *col_idx;   /* nnz entries */
    const void *val;          /* nnz entries of the call's dtype */
} smash_csr;

/* Options (smash_set_option / smash_get_option).  Setting an option drops
 * the plan of the last symbolic call. */
typedef enum {
    /* 1 = check the CSR preconditions of A and B on the device (default 1). */
    SMASH_OPT_VALIDATE = 0,
    /* Rows whose output bound min(products, cols) exceeds this many
     * entries leave the LDS row tables for the heavy-row path.  Range
     * 32..1024, default 1024. */
    SMASH_OPT_LDS_ROW_MAX = 1,
    /* Heavy-row path: 0 = column segments merged in LDS, hashed or, for
     * chunks with more than 1024 of their 8192 columns, accumulated by column (default);
     * 1 = one hash table per row in global memory (the paper's third
     * version, "Fragmenting Memory", moves the table to DRAM). */
    SMASH_OPT_HEAVY_MODE = 2,
    /* 1 = record HIP events around every kernel launch and accumulate the
     * elapsed time per kernel (smash_kernel_time).  Default 0. */
    SMASH_OPT_TIMING = 3,
    /* Row capacities of smash_spgemm_fused: 0 = the installed predictor
     * (default); 1 = the exact upper bound min(products, cols), without the
     * network (the baseline that shows what the network gains). */
    SMASH_OPT_FUSED_SIZING = 4,
    /* Global mode (SMASH_OPT_HEAVY_MODE = 1): the most hash-table slots the
     * heavy rows may hold at once; 0 = no limit (default).  Every heavy row
     * has a table of next_pow2(2 x its bound) slots; when the tables of all
     * heavy rows exceed the limit, the rows are processed in waves of
     * consecutive rows whose tables fit, and the pool is reused from wave
     * to wave (a row whose own table exceeds the limit forms a wave alone,
     * with a pool of its size).  The pool is the workspace's: a workspace
     * smaller than all tables limits it the same way. */
    SMASH_OPT_GLOBAL_POOL = 5,
    /* Hash of the LDS row tables of light rows: 0 = multiplicative
     * (Fibonacci) hash, entries then ordered by bitmap ranks or a bitonic
     * sort (default); 1 = the order-preserving hash of the paper's first
     * version (slot = column scaled to the table: High-Bit Hashing), whose
     * table is nearly sorted, entries then put in order by an insertion
     * pass bounded by the longest probe (Write-back Phase, Algorithm
     * "SMASH WRITEBACK").  Also a candidate of smash_batch_autotune. */
    SMASH_OPT_ROW_HASH = 6,
    SMASH_OPT_COUNT = 7
} smash_option;

/* Counters of the last symbolic/numeric call (smash_get_stats). */
typedef struct {
    int64_t rows;               /* A.rows */
    int64_t products;           /* sum over rows of the products (multiply-adds) */
    int64_t nnz_c;              /* nnz(C) */
    int64_t rows_empty;         /* rows with no product */
    int64_t rows_lds;           /* rows merged in an LDS row table */
    int64_t rows_heavy;         /* rows on the heavy-row path */
    int64_t heavy_segments;     /* hashed column segments of heavy rows */
    int64_t heavy_dense_chunks; /* column chunks of heavy rows accumulated by column */
    int64_t global_slots;       /* global hash table slots (global mode) */
    int64_t nnz_heavy;          /* entries of C in heavy rows */
    int64_t nnz_dense;          /* entries of C in dense chunks of heavy rows */
    int64_t fused_rows;         /* rows completed by the fused pass (smash_spgemm_fused) */
    int64_t fused_overflow;     /* rows the fused pass handed back (prediction too small) */
    int64_t fused_capacity;     /* sum of the capacities the fused pass reserved (staging slots) */
    int64_t global_waves;       /* launches of global-mode row waves (symbolic + numeric) */
    int64_t global_pool;        /* slots of the global table pool used (the largest wave) */
    int64_t fused_entries;      /* entries of the rows the fused pass completed */
    int64_t workspace_bytes;    /* workspace bytes the last symbolic call needed (also after CAPACITY) */
} smash_stats;

/* Allocation callback of smash_spgemm: return device memory of at least
 * `bytes` bytes (256-byte aligned) or NULL.  The caller owns it. */
typedef void *(*smash_alloc_fn)(size_t bytes, void *user);

/* Create a context on HIP device `device`.  *out is NULL on failure. */
smash_status smash_create(smash_ctx *out, int device);

/* Destroy a context and free its scratch memory.  NULL is ignored.  Work
 * queued on streams by this context must have completed. */
void smash_destroy(smash_ctx ctx);

/* Message of the last failing call on ctx ("" if none).  Owned by ctx. */
const char *smash_last_error(smash_ctx ctx);

/* Static name of a status code. */
const char *smash_status_string(smash_status s);

smash_status smash_set_option(smash_ctx ctx, smash_option opt, int64_t value);
smash_status smash_get_option(smash_ctx ctx, smash_option opt, int64_t *value);

/* Workspace bytes that smash_spgemm_symbolic / _numeric / smash_spgemm /
 * smash_spgemm_fused need for C = A * B under the context's current options
 * (and installed predictor).  The plan arrays are sized from the shapes; the
 * heavy-row tables (rows whose output bound exceeds the LDS row limit: the
 * paper's rows that overflow a scratchpad window, Window Distribution Phase)
 * from a device pass that counts them, after a memory-safety check of the
 * operands (row pointers and column ranges; INVALID_CSR if it fails).
 * Synchronises the stream.  A, B values are not read.
 * Errors: INVALID_ARG, INVALID_CSR, HIP. */
smash_status smash_workspace_size(smash_ctx ctx, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                  size_t *bytes, hipStream_t stream);

/* Symbolic phase: the exact nnz of every row of C = A * B.
 * Writes C_row_ptr[0..A.rows] (device, int64, exclusive prefix of the row
 * counts) and *C_nnz (host).  A.val and B.val are not read.  The plan built
 * here (row bins, heavy-row column counts, in ws) is kept for the next
 * smash_spgemm_numeric call with the same A, B, C_row_ptr and ws, whose
 * contents the caller must leave untouched in between.
 * Synchronizes the stream once (to read nnz(C) back).
 * Errors: INVALID_ARG (null pointer, A.cols != B.rows, negative sizes),
 * INVALID_CSR, CAPACITY (ws too small: smash_get_stats().workspace_bytes
 * holds the bytes needed), HIP, and errors of an earlier numeric call not
 * yet reported. */
smash_status smash_spgemm_symbolic(smash_ctx ctx, const smash_csr *A, const smash_csr *B,
                                   int64_t *C_row_ptr, int64_t *C_nnz, void *ws, size_t ws_bytes,
                                   hipStream_t stream);

/* Numeric phase: the columns and values of C = A * B, written at
 * C_col_idx[C_row_ptr[i] .. C_row_ptr[i+1]) and the same range of C_val
 * (device; nnz(C) entries each; C_val of dtype).  Requires the plan of a
 * preceding smash_spgemm_symbolic call on ctx with the same A and B
 * descriptors, C_row_ptr pointer and ws (else SMASH_ERR_NO_PLAN); the plan
 * stays valid, so numeric may be repeated after A.val or B.val change.
 * Does not synchronise: a C_row_ptr found inconsistent with the product on
 * the device is reported as CAPACITY by smash_sync() (or the next symbolic
 * call).  Errors: INVALID_ARG, NO_PLAN, HIP. */
smash_status smash_spgemm_numeric(smash_ctx ctx, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                  const int64_t *C_row_ptr, int32_t *C_col_idx, void *C_val,
                                  void *ws, size_t ws_bytes, hipStream_t stream);

/* Both phases: symbolic, then C_col_idx and C_val allocated through
 * alloc(nnz * 4, user) and alloc(nnz * value_bytes, user), then numeric.
 * C_row_ptr (device, A.rows + 1 int64) and ws are the caller's.  On success
 * *C_col_idx, *C_val (never NULL, also when nnz(C) = 0) and *C_nnz are set.
 * One host synchronisation (the nnz readback).
 * Errors: those of the two phases, OUT_OF_MEMORY if alloc returns NULL. */
smash_status smash_spgemm(smash_ctx ctx, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                          smash_alloc_fn alloc, void *user, int64_t *C_row_ptr,
                          int32_t **C_col_idx, void **C_val, int64_t *C_nnz, void *ws, size_t ws_bytes,
                          hipStream_t stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): smash_spgemm with neither a workspace
 * nor an allocation callback.  The workspace is a 64 MiB device array of the
 * library (SMASH_NOALLOC_SCRATCH_BYTES, one per GPU, held until the process
 * ends); C goes to the caller's buffers: C_row_ptr (A.rows + 1 int64),
 * C_col_idx and C_val (C_capacity entries each, C_val of dtype).  The call
 * allocates no device memory (with SMASH_OPT_TIMING off: timing events
 * aside) and synchronises the stream once, like smash_spgemm.  *C_nnz
 * receives nnz(C), also when it exceeds C_capacity (then CAPACITY, and
 * nothing is written to C_col_idx / C_val).  Errors: CAPACITY (C_capacity too
 * small, or the product needs more workspace than the array holds:
 * smash_get_stats().workspace_bytes then says how much), INVALID_ARG (also
 * for SMASH_OPT_HEAVY_MODE = 1, which is not supported here), INVALID_CSR,
 * HIP.  Every call on one GPU uses the same array: calls that overlap on one
 * GPU (from several contexts or streams) race and must be serialised by the
 * caller; each call initialises the parts of the array it reads. */
#define SMASH_NOALLOC_SCRATCH_BYTES (64ull << 20)
smash_status smash_spgemm_noalloc(smash_ctx ctx, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                  int64_t *C_row_ptr, int32_t *C_col_idx, void *C_val, int64_t C_capacity,
                                  int64_t *C_nnz, hipStream_t stream);

/* Waits for `stream` and reports what the numeric calls enqueued on ctx
 * since the last report found wrong on the device (CAPACITY: a C_row_ptr
 * inconsistent with the product); clears it.  Errors: CAPACITY, HIP. */
smash_status smash_sync(smash_ctx ctx, hipStream_t stream);

/* Counters of the last symbolic (and numeric) call on ctx. */
smash_status smash_get_stats(smash_ctx ctx, smash_stats *out);

/* ------------------------------------------------- learned row-size predictor
 *
 * A small MLP (6 -> 64 -> 64 -> 1, ReLU, FP32) maps six per-row features of
 * C = A * B to log2(1 + nnz(C_i)); the fused pass (smash_spgemm_fused) sizes
 * its LDS tables from it instead of running a symbolic phase.  Parameters
 * are packed floats: W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3
 * (SMASH_MLP_PARAMS floats).  Features are standardized as (f - mean) / std
 * with mean_std = {mean[6], std[6]}.  This predictor is the library's
 * addition; the paper sizes output from per-row product counts (Window
 * Distribution Phase) and names flop-estimate-based distribution as future
 * work (Conclusions, Future Work). */
#define SMASH_MLP_FEATURES 6
#define SMASH_MLP_PARAMS 4673

/* Features of every row i of C = A * B (device float[A.rows * 6], row-major):
 * log2(1 + x) of nnz(A_i), ub_i = sum_k nnz(B_k), max_k nnz(B_k),
 * min_k nnz(B_k), min(ub_i, B.cols) and sum_k nnz(B_k)^2 / ub_i; zeros for
 * empty rows. */
smash_status smash_features(smash_ctx ctx, const smash_csr *A, const smash_csr *B, float *feats, hipStream_t stream);

/* yhat[i] = network output for feats[i] (all device pointers; m rows). */
smash_status smash_mlp_predict(smash_ctx ctx, int64_t m, const float *feats, const float *params,
                               const float *mean_std, float *yhat, hipStream_t stream);

/* Mean squared error of the network over the n samples feats[idx[s]] with
 * targets targets[idx[s]], and its gradient with respect to params (device
 * float[SMASH_MLP_PARAMS]).  *loss is written on the host (synchronizes). */
smash_status smash_mlp_loss_grad(smash_ctx ctx, const float *feats, const float *targets, const int32_t *idx,
                                 int64_t n, const float *mean_std, const float *params, float *grad, double *loss,
                                 hipStream_t stream);

typedef struct {
    int32_t epochs;   /* passes over the data */
    int32_t batch;    /* samples per Adam step (the last step of an epoch may be smaller) */
    float lr, beta1, beta2, eps;   /* Adam hyper-parameters */
} smash_train_args;

/* Mini-batch Adam training of params (device, in/out) on n samples.  orders
 * (device int32[epochs * n]) holds one permutation of 0..n-1 per epoch; the
 * steps of epoch e take consecutive batches of orders[e*n ...].
 * epoch_loss (host, epochs entries) receives the mean batch loss of every
 * epoch.  Synchronizes once at the end. */
smash_status smash_mlp_train(smash_ctx ctx, const float *feats, const float *targets, int64_t n,
                             const float *mean_std, float *params, const int32_t *orders,
                             const smash_train_args *args, double *epoch_loss, hipStream_t stream);

/* Installs a predictor in ctx: host params (SMASH_MLP_PARAMS floats), host
 * mean_std (12 floats) and the capacity margin delta (log2 units): a row's
 * capacity is clamp(ceil(2^(yhat + delta) - 1), max(max_k nnz(B_k), 1),
 * min(ub_i, B.cols)). */
smash_status smash_predictor_set(smash_ctx ctx, const float *params, const float *mean_std, float delta);

/* Fused single pass: C = A * B like smash_spgemm, without a symbolic phase
 * for the rows the installed predictor sizes into LDS (predicted capacity
 * <= SMASH_OPT_LDS_ROW_MAX): those rows are hashed, counted, sorted and
 * staged in one kernel; rows whose columns exceed their capacity, and rows
 * predicted above the LDS limit, go through the exact two-phase path (a row
 * is never lost to a bad prediction; only time is).  Staged rows are copied
 * to their final offsets after the row-pointer scan.  The result is the same
 * canonical C as smash_spgemm.  Errors: NO_PLAN if no predictor is
 * installed while SMASH_OPT_FUSED_SIZING is 0, and those of smash_spgemm. */
smash_status smash_spgemm_fused(smash_ctx ctx, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                smash_alloc_fn alloc, void *user, int64_t *C_row_ptr,
                                int32_t **C_col_idx, void **C_val, int64_t *C_nnz, void *ws, size_t ws_bytes,
                                hipStream_t stream);

/* Loads a predictor file: 8 bytes "SMASHMLP", int32 version (1), int32
 * SMASH_MLP_PARAMS, float delta, float mean_std[12], float params[...],
 * little-endian.  Errors: INVALID_ARG (unreadable or malformed file). */
smash_status smash_predictor_load(smash_ctx ctx, const char *path);

/* ---------------------------------------------------------------- batches
 * Many independent products C_p = A_p * B_p (p = 0 .. count-1) computed by
 * one pipeline over the concatenated rows of all problems, so that uneven
 * problem sizes share the machine and the whole batch costs one fixed
 * sequence of kernel launches with no host synchronisation: it can be
 * captured once as a HIP graph and replayed.  The pipeline is the same as
 * smash_spgemm's (per-row product bounds, binning, symbolic, row-pointer
 * scan, numeric: the steps of the SMASH Kernels chapter), with rows above the
 * LDS limit hashed in per-row global-memory tables (its version 3).  Work is
 * spread like the paper's tokenised row distribution (SMASH Version 2) and
 * oversubscribed windows (Window Distribution Phase): persistent workgroups
 * take row blocks of each bin from device-side counts.
 *
 * Output layout: one pool.  Global row g = row0[p] + i is row i of problem
 * p (row0 = exclusive prefix of the problems' row counts).  C_row_ptr holds
 * total_rows + 1 int64 offsets into the pool; problem p's C is rows
 * row0[p] .. row0[p+1]-1 of that CSR (its row pointers are absolute pool
 * offsets; its column indices are in B_p's column space).
 */
typedef struct smash_batch_plan_s *smash_batch_plan;

/* Tunables of the batched launch (the autotuner chooses them):
 *  lds_row_max   rows with min(products, cols) above this use global tables
 *                (bin threshold): 32 .. 1024, and at most 2048 >> table_shift;
 *  table_shift   LDS table slots = next_pow2(bound << table_shift): 1 or 2
 *                (load factor at most 1/2 or 1/4);
 *  wide_groups   0: one wavefront per row up to 1024 slots, 4 for 2048;
 *                1: rows with 512 or more slots use 2, 4, 8 wavefronts;
 *  blocks_per_cu persistent workgroups per compute unit: 1 .. 32;
 *  row_hash      hash of the LDS row tables in the numeric pass: 0 or 1, as
 *                SMASH_OPT_ROW_HASH. */
typedef struct {
    int32_t lds_row_max;
    int32_t table_shift;
    int32_t wide_groups;
    int32_t blocks_per_cu;
    int32_t row_hash;
} smash_batch_config;

/* Creates a plan for the `count` problems A[p] * B[p] (arrays of descriptors,
 * read during the call only; the matrices they point to must stay alive and
 * unmoved while the plan is used; values must be non-NULL, of `dtype`).  cfg
 * NULL takes the defaults {1024, 1, 0, 8, 0}.  Every device buffer of the plan
 * comes from `alloc` (the library allocates no device memory): first the
 * plan's workspace (per-row arrays, descriptors, header), then, after the
 * per-row analysis (which synchronises `stream`) has sized it, the output
 * pool: C_row_ptr (int64[total_rows + 1]) and col/val pools of capacity sum
 * over rows of min(products_i, cols_p), an exact upper bound on the entries
 * of any replay with the same structure; then the global hash tables of
 * problems wider than 2^20 columns (keys, FP64 values, touched-slot lists;
 * smash_batch_plan_configure may ask for larger ones).  `alloc` and `user`
 * must stay valid while the plan lives.  The caller owns all of these
 * buffers (free them after the plan).
 * With SMASH_OPT_VALIDATE set every operand is checked here (once; replays
 * do not validate).
 * Errors: INVALID_ARG (count < 0, a NULL pointer, A[p].cols != B[p].rows,
 * bad cfg), INVALID_CSR, INDEX_OVERFLOW (total rows >= 2^31),
 * OUT_OF_MEMORY, HIP. */
smash_status smash_batch_plan_create(smash_ctx ctx, smash_dtype dtype, int32_t count, const smash_csr *A,
                                     const smash_csr *B, const smash_batch_config *cfg, smash_alloc_fn alloc,
                                     void *user, smash_batch_plan *out, hipStream_t stream);

/* Changes the tunables of a plan (grows its workspace if needed; drops a
 * captured graph).  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP. */
smash_status smash_batch_plan_configure(smash_batch_plan plan, const smash_batch_config *cfg, hipStream_t stream);
smash_status smash_batch_plan_get_config(smash_batch_plan plan, smash_batch_config *cfg);

/* Output pool of the plan (device pointers owned by the caller), its
 * capacity in entries, the total row count, and row0 (host, count + 1
 * entries, valid while the plan lives).  Any pointer argument may be NULL. */
smash_status smash_batch_plan_outputs(smash_batch_plan plan, int64_t **C_row_ptr, int32_t **C_col_idx,
                                      void **C_val, int64_t *capacity, int64_t *total_rows, const int64_t **row0);

/* Enqueues the whole batch on `stream` (no host synchronisation, no
 * allocation).  Results are complete when the stream reaches that point;
 * errors detected on the device are reported by smash_batch_plan_result. */
smash_status smash_batch_plan_run(smash_batch_plan plan, hipStream_t stream);

/* Captures smash_batch_plan_run on `stream` into a graph owned by the plan
 * (replacing a previous one); smash_batch_plan_launch replays it on any
 * stream of the plan's device.  Errors: HIP (capture failed), NO_PLAN
 * (launch before capture). */
smash_status smash_batch_plan_capture(smash_batch_plan plan, hipStream_t stream);
smash_status smash_batch_plan_launch(smash_batch_plan plan, hipStream_t stream);

/* Synchronises `stream` and reports the last run: total entries, and per
 * problem entries into nnz_per_problem (host, `count` entries) if non-NULL.
 * Returns CAPACITY if the entries exceeded the pool (the structure changed
 * since create; C is then incomplete), HIP on an internal inconsistency. */
smash_status smash_batch_plan_result(smash_batch_plan plan, hipStream_t stream, int64_t *nnz_total,
                                     int64_t *nnz_per_problem);

void smash_batch_plan_destroy(smash_batch_plan plan);

/* Autotuner: times smash_batch_plan_run on this plan for each candidate
 * configuration (bin threshold, table multiplier, workgroup width,
 * persistent grid), `reps` timed runs each after one warm-up, and
 * configures the plan with the fastest.  With cache_path non-NULL the
 * result is looked up first in, and afterwards appended to, a text file of
 * lines "key lds_row_max table_shift wide_groups blocks_per_cu row_hash ms", where
 * key describes the batch (dtype, count, rows, nnz of A and B, products);
 * a hit configures the plan without timing.  *best (if non-NULL) receives
 * the chosen configuration and *best_ms (if non-NULL) its mean time (0 on
 * a cache hit).  Errors: those of run/configure; an unreadable cache is
 * ignored, an unwritable one is INVALID_ARG. */
smash_status smash_batch_autotune(smash_batch_plan plan, hipStream_t stream, int32_t reps, const char *cache_path,
                                  smash_batch_config *best, double *best_ms);

/* Per-kernel timing (SMASH_OPT_TIMING = 1).  For kernel index `index`
 * (0 .. smash_kernel_count()-1) returns its static name, the number of
 * launches and the summed elapsed milliseconds since the last reset.
 * Returns INVALID_ARG for an index out of range. */
int smash_kernel_count(void);
smash_status smash_kernel_time(smash_ctx ctx, int index, const char **name, int64_t *launches, double *ms);
smash_status smash_kernel_time_reset(smash_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* SMASH_H */
