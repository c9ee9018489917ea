/*
 * lorax.h - C ABI of liblorax.so: hierarchical factorization of a sparse matrix
 * with low-rank compression of well-separated fill-in (extended sparsification),
 * its forward/backward solve, and GMRES preconditioned by that solve, on one
 * AMD MI355X (gfx950).
 *
 * The operations follow Pouransari, Coulier, Darve, "Fast hierarchical solvers
 * for sparse matrices using extended sparsification and low-rank approximation":
 *   lrx_factor  Algorithm 1 (Sec. 4): level-by-level MergeRedNodes, Compress,
 *               Eliminate(super-node), Eliminate(black node) on the H-tree of
 *               Def. "hierarchical tree"; truncated SVD with the cut-off of
 *               eqn. cutOff1, or rank-revealing QR (Sec. 7 lists both).
 *   lrx_solve   Algorithms 2-4 (Sec. 4.5): SetRHS, forward SolveL, backward
 *               SolveU and SplitVar; x ~ A^{-1} b.
 *   lrx_gmres   Sec. 6.2: GMRES with the solve as preconditioner.
 *
 * Conventions for every call
 *   - Every call returns an lrx_status; nothing throws or aborts across the ABI.
 *     On an error the outputs are left untouched (except where stated) and
 *     lrx_last_error() returns a message for the calling thread.
 *   - Host pointers are plain CPU memory owned by the caller; the caller may free
 *     them as soon as the call returns.  Device pointers (the *_dev calls) are
 *     HBM allocations of the caller on the current HIP device.
 *   - A handle owns all device memory it allocates and releases it in lrx_free.
 *     Released blocks (up to 8 GiB per device, and 1 GiB of pinned host
 *     memory) stay with the library for reuse by later handles until the
 *     process ends; a failed allocation returns them to HIP and retries.
 *     A release waits for all work queued on the device, as hipFree does.
 *     Solves on one handle may run concurrently on different streams only if
 *     each stream has its own handle; calls on one handle are not thread-safe.
 *   - Matrices are CSR, 0-based, int64 row pointers, int32 column indices,
 *     columns sorted and unique within each row, FP64 values, all finite.
 */
#ifndef LORAX_H
#define LORAX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LRX_OK = 0,
    LRX_EINVAL = 1,     /* malformed argument: CSR, tree, options, sizes, NaN/Inf, stale handle */
    LRX_ENOMEM = 2,     /* device allocation failed or the factor exceeds hbm_budget_bytes */
    LRX_ESINGULAR = 3,  /* a pivot block is exactly singular after partial pivoting */
    LRX_ENOCONV = 4,    /* GMRES reached maxit before tol (best x, iters, relres returned) */
    LRX_EDEVICE = 5,    /* HIP runtime error or no usable gfx950 device */
    LRX_EBUSY = 6       /* reserved */
} lrx_status;

/* LRX_FP64: every step in FP64 (products on FP64 matrix cores).
 * LRX_MIXED: when epsilon >= 1e-5 (FP32 resolves the cut-off), the compression's
 * reduced QRs and Jacobi SVD run in FP32, and the Schur-complement GEMMs and
 * the projection B V of the compression take FP32 operands with FP32
 * accumulation on the matrix cores (their results update FP64 blocks); the
 * solve reads FP32 copies of the stored off-diagonal blocks (the FP64 factor is
 * released after factorization).  Pivot inverses (computed and stored in
 * FP64), W_k = S^-1 Mat(k->s), vectors, accumulation in the solve and GMRES stay
 * FP64, so GMRES refines the result to its FP64 tolerance.  Below 1e-5 the
 * factorization runs as in LRX_FP64 and only the solve reads FP32 copies.
 * LRX_MIXED_BF16: the BF16 trial of the compression GEMMs: as LRX_MIXED, with
 * the projection B V of every compression on BF16 operands (FP32
 * accumulation).  V stays accurate, but [R; Q] = B V carries BF16 input
 * rounding (about 2^-9 relative), so ||B - [R; Q] V^T||_2 <= epsilon ||B||_2
 * no longer holds for epsilon below that level; GMRES still refines the result
 * to its tolerance, with more iterations. */
typedef enum { LRX_FP64 = 0, LRX_MIXED = 1, LRX_MIXED_BF16 = 2 } lrx_precision;
typedef enum { LRX_COLORED = 0, LRX_NATURAL = 1 } lrx_order;
typedef enum { LRX_SVD = 0, LRX_RRQR = 1, LRX_RAND = 2 } lrx_compress;
/* Truncation rule of Compress.  LRX_RULE_CUTOFF1 (eqn. cutOff1): keep sigma_k >=
 * epsilon sigma_0 of each stacked block (RRQR: stop at ||R22||_F <= epsilon |R11|).
 * LRX_RULE_FROB, the paper's variant of eqn. curOff6: keep the fewest singular
 * values whose discarded tail has Frobenius norm < epsilon N_i, where N_i^2 sums
 * the squared Frobenius norms of all blocks of level i and of every level below,
 * each level's blocks taken when the level starts (after MergeRedNodes; at the
 * leaf level they are the entries of A, so N_l = ||A||_F); RRQR: stop at the
 * first k with ||R22||_F < epsilon N_i.  The threshold is absolute per level, so
 * blocks that are small against the whole take lower ranks (Sec. 6.2). */
typedef enum { LRX_RULE_CUTOFF1 = 0, LRX_RULE_FROB = 1 } lrx_rule;

typedef struct lrx_handle_s* lrx_handle;     /* opaque */

/* Sparse matrix A (n x n) in CSR form, host memory. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int64_t* row_ptr;   /* n+1 entries, row_ptr[0] = 0, row_ptr[n] = nnz */
    const int32_t* col_idx;   /* nnz entries, sorted and unique within a row */
    const double* val;        /* nnz entries */
} lrx_csr;

/* Nested binary partitionings P_0..P_depth (Def. "nested partitionings"):
 * perm[t] is the original row/column at tree position t; leaf c holds tree
 * positions [leaf_ptr[c], leaf_ptr[c+1]); cluster j of level i is the union of
 * leaves [j*2^(depth-i), (j+1)*2^(depth-i)).  Leaves must be non-empty,
 * depth >= 1, 2^depth + 1 entries in leaf_ptr. */
typedef struct {
    int32_t depth;
    const int32_t* perm;
    const int32_t* leaf_ptr;
} lrx_tree;

typedef struct {
    double epsilon;            /* truncation tolerance, 0 <= epsilon < 1; 0 keeps everything (exact).
                                  LRX_SVD: keep sigma_k >= epsilon * sigma_0 of the stacked block B
                                  (eqn. cutOff1), so ||B - B V V^T||_2 < epsilon ||B||_2.
                                  LRX_RRQR: row-pivoted QR of B stopped at the first k with
                                  ||R22||_F <= epsilon |R11|, so ||B - B V V^T||_2 <= epsilon ||B||_2.
                                  LRX_RAND (randomized SVD, one of the low-rank methods Sec. 7
                                  lists): blocks of at most 64 columns by an adaptive randomized
                                  range finder on the nonzero rows and columns of B: sketch
                                  Y = B^T Omega with l = min(16, c_nz) Rademacher columns drawn
                                  from SplitMix64 of (((level << 24) | j) << 34) + (row << 6) + col
                                  (row counted among the nonzero rows of B, stacking order),
                                  Q = Householder QR of Y, C = B Q = U S W^T; rank = fewest k with
                                  sqrt(||B||_F^2 - sum S^2 + sum_{t>=k} S_t^2) <= epsilon S_0
                                  (uncaptured energy 0 when l = c_nz), accepted when k < l or
                                  l = c_nz, else l doubles; V = Q W_k.  Then again
                                  ||B - B V V^T||_2 <= epsilon ||B||_2.  Wider blocks take the SVD.
                                  Needs rule LRX_RULE_CUTOFF1. */
    int32_t precision;         /* lrx_precision */
    int32_t compress;          /* lrx_compress: low-rank method of Compress (Sec. 4.3) */
    int32_t order;             /* lrx_order: order of the super-nodes inside a level */
    int64_t hbm_budget_bytes;  /* 0 = no limit; otherwise LRX_ENOMEM when exceeded */
    void* stream;              /* hipStream_t used by the handle, or NULL for the null stream */
    int32_t rule;              /* lrx_rule (appended field) */
    int32_t symmetric;         /* 1: A is symmetric (checked entry for entry, LRX_EINVAL otherwise) and
                                  Compress stacks only A_k = Mat(s->p_k), since B_k = A_k, with
                                  Q_k = R_k: half the stacked rows (Sec. 4.3, last paragraph) */
} lrx_opts;

/* Counters of a factorization (sizes in elements/bytes, times in ms). */
typedef struct {
    int32_t depth;
    int32_t n_compressions;
    int32_t n_colour_steps;        /* sum over levels of colours */
    int32_t max_rank;
    double mean_rank;
    int32_t rank_max_by_level[32]; /* index = level, 0..depth */
    double rank_mean_by_level[32];
    double mean_node_size_by_level[32];
    int64_t extended_size;         /* n + auxiliary variables */
    double max_compression_error;  /* max over compressions of ||B - B V V^T||_2 / ||B||_2
                                      (SVD: sigma_r / sigma_0) or of its bound ||R22||_F / |R11|
                                      (RRQR); at most epsilon */
    int64_t factor_bytes;          /* device bytes of stored blocks */
    int64_t solve_bytes;           /* bytes one solve reads from stored blocks */
    int64_t factor_flops;          /* algorithmic flops of the factorization */
    double t_plan_ms;              /* host symbolic planning */
    double t_factor_ms;            /* whole lrx_factor call */
    double t_sync_ms;              /* host time blocked on the stream inside lrx_factor */
    double t_solve_prog_ms;        /* host compilation of the solve sweeps */
    /* appended fields */
    int64_t device_bytes;          /* device memory the handle holds now: factor storage (arena chunk
                                      capacities), solve programs, resident A, and the solve / GMRES
                                      workspaces it has grown to (they grow with nrhs and restart) */
    double flops_compress;         /* factor_flops by operation: stacked QRs + truncated SVD / RRQR */
    double flops_pivot;            /* pivot inverses of super-nodes and black nodes */
    double flops_schur;            /* Schur-complement products, W_k = S^-1 Mat(k->v) included */
    double flops_project;          /* projection [R; Q] = B V */
    double level_norm_by_level[32];/* LRX_RULE_FROB: N_i of eqn. curOff6 by level (0 otherwise) */
    int64_t sweep_stages;          /* LDS stages of both sweeps' node programs, summed over the nodes */
    int64_t sweep_launches;        /* launches of one solve application (one per colour step and sweep) */
    double t_host_compress_ms;     /* host time building and launching the compress steps (no waits) */
    double t_host_node_ms;         /* host time from each rank read-back to the last node launch */
} lrx_stats_t;

/* Symbolic counts, computed on the host without any device call. */
typedef struct {
    int32_t depth;
    int32_t n_supernodes;          /* super-nodes over all levels (= 2^depth - 1) */
    int32_t n_colour_steps;
    int32_t colours_by_level[32];
    int64_t n_candidates;          /* well-separated neighbours over all compressions */
    int64_t n_schur_pairs;         /* (in-neighbour, out-neighbour) updates over all eliminations */
    int64_t n_edges_created;
    int64_t candidates_by_level[32];
} lrx_plan_info;

/* Algorithm 1.  Copies A and T; runs the symbolic plan on the host and the
 * numeric factorization on the device.  On success *out is a new handle.
 * Errors: LRX_EINVAL (bad CSR/tree/options, non-finite values), LRX_ESINGULAR,
 * LRX_ENOMEM, LRX_EDEVICE. */
lrx_status lrx_factor(const lrx_csr* A, const lrx_tree* T, const lrx_opts* o, lrx_handle* out);

/* Same as lrx_factor with the values already in HBM: A supplies the pattern
 * (row_ptr, col_idx on the host, used by the symbolic plan; A->val is ignored)
 * and val_dev holds the nnz values in device memory (read-only, in CSR order).
 * Non-finite values give LRX_EINVAL. */
lrx_status lrx_factor_dev(const lrx_csr* A, const double* val_dev, const lrx_tree* T,
                          const lrx_opts* o, lrx_handle* out);

/* Batched form of lrx_factor (Algorithm 1 for k independent systems at once).
 * A[i], T[i] (arrays of k structs, host memory, copied) describe system i;
 * val_dev is NULL (values in A[i].val on the host) or an array of k device
 * pointers, val_dev[i] holding the nnz_i values of system i in HBM as in
 * lrx_factor_dev (A[i].val is then ignored).  All systems share the options o (epsilon, precision, rule, order, per-handle HBM budget
 * and stream).  The symbolic plans run on host threads; the numeric level loops
 * of all systems advance in lock-step over (height above the leaves, colour):
 * each kernel of a step is one launch over the nodes of every system with a
 * step there (super-nodes of one colour are independent by Thm. "preservation of sparsity",
 * Sec. 5, and distinct
 * systems share nothing).  On success out[i] is the handle of system i and
 * equals the handle lrx_factor gives for that system alone (the solve results
 * are bitwise the same).  The batch succeeds or fails as a whole: on any error
 * no handle is created and every out[i] is set to NULL; the message of
 * lrx_last_error names the system.  1 <= k <= 65536. */
lrx_status lrx_factor_batch(int32_t k, const lrx_csr* A, const double* const* val_dev, const lrx_tree* T,
                            const lrx_opts* o, lrx_handle* out);

/* Algorithms 2-4 for nrhs right-hand sides, host memory, column-major:
 * b[k*ldb + i] is entry i of right-hand side k (ldb >= n); x likewise (ldx >= n).
 * Synchronous. */
lrx_status lrx_solve(lrx_handle h, int32_t nrhs, const double* b, int64_t ldb,
                     double* x, int64_t ldx);

/* Same on device memory, enqueued on the handle's stream, no host sync.
 * b and x are n x nrhs with leading dimension n, column-major, may not alias. */
lrx_status lrx_solve_dev(lrx_handle h, int32_t nrhs, const double* b_dev, double* x_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): lrx_solve_dev
 * with the extended vector (n + auxiliary variables, times nrhs doubles) in a
 * static device array of the library, 32 MiB per device, held until the
 * process ends, instead of the handle's workspace.  It allocates nothing and
 * records no timing events.  The array's device address is looked up on the
 * first call on each device (the handle's device must be current).  Every call
 * on one device shares that array: calls that overlap on one device (other
 * streams or threads) race and give wrong results; calls queued on one stream
 * are ordered and safe.  Results equal lrx_solve_dev's bit for bit.
 * Errors: LRX_EINVAL when n_ext * nrhs * 8 exceeds 32 MiB (lrx_stats gives
 * n_ext as extended_size), for bad pointers or nrhs, or when the handle's
 * device is not current. */
lrx_status lrx_solve_dev_noalloc(lrx_handle h, int32_t nrhs, const double* b_dev, double* x_dev);

/* Batched form of lrx_solve_dev: k distinct handles on the same device, nrhs
 * right-hand sides each; b_dev[i], x_dev[i] are n_i x nrhs
 * column-major in HBM.  Every (level, colour) step of the sweeps is one launch
 * over the nodes of all k factorizations (their steps are independent), on the
 * stream of hs[0]; FP64 and mixed-precision handles may share a batch.
 * Synchronous: returns when every x_dev[i] is written.  Each result equals the
 * one lrx_solve_dev gives for that handle alone. */
lrx_status lrx_solve_batch_dev(int32_t k, const lrx_handle* hs, int32_t nrhs, const double* const* b_dev,
                               double* const* x_dev);

/* GMRES(restart) with the solve as right preconditioner, x_0 = 0, for nrhs
 * right-hand sides (host, column-major, leading dimension n).  A must be the
 * matrix the handle was factored from: its pattern and values are compared
 * entry for entry with the handle's resident copy (read back from the device),
 * and any difference gives LRX_EINVAL (the products use that copy).  Stops each
 * right-hand side when its true relative residual ||b - A x|| / ||b|| <= tol.
 * iters[k] and relres[k] (nrhs entries each, may be NULL) receive the
 * iteration count and final true relative residual.  Returns LRX_ENOCONV if any
 * right-hand side reached maxit; x, iters and relres are then still filled. */
lrx_status lrx_gmres(const lrx_csr* A, lrx_handle h, int32_t nrhs, const double* b,
                     double* x, double tol, int32_t restart, int32_t maxit,
                     int32_t* iters, double* relres);

/* Same on device memory (b, x: n x nrhs column-major in HBM) on the handle's
 * stream; uses the handle's resident copy of A.  Synchronises the stream once
 * per Arnoldi step (the Hessenberg column goes to the host). */
lrx_status lrx_gmres_dev(lrx_handle h, int32_t nrhs, const double* b_dev, double* x_dev,
                         double tol, int32_t restart, int32_t maxit,
                         int32_t* iters, double* relres);

/* Batched form of lrx_gmres_dev: k distinct handles on one device, nrhs
 * right-hand sides each, b_dev[i] and x_dev[i] n_i x nrhs column-major in HBM.
 * The k FGMRES iterations (Sec. 6.2) run in lock-step on the stream of hs[0]:
 * each vector operation is one launch over the rows of every system still
 * iterating, the preconditioner one sweep launch per (level, colour) step over
 * the nodes of all of them, and the Hessenberg columns of all systems cross to
 * the host in one copy per Arnoldi step.  Every right-hand side of every system
 * stops on its own true relative residual (tol); a system whose right-hand
 * sides have all stopped leaves the launches.  iters and relres (may be NULL)
 * receive k * nrhs entries, system-major: entry i * nrhs + j is right-hand side
 * j of system i.  Synchronous.  Returns LRX_ENOCONV if any right-hand side
 * reached maxit (all outputs are still written).  1 <= k <= 65535; a handle may
 * appear once; concurrent calls that share a handle race. */
lrx_status lrx_gmres_batch_dev(int32_t k, const lrx_handle* hs, int32_t nrhs, const double* const* b_dev,
                               double* const* x_dev, double tol, int32_t restart, int32_t maxit,
                               int32_t* iters, double* relres);

/* lrx_gmres_batch_dev from an initial guess: on entry x_dev[i] holds x_0 of
 * every right-hand side of system i (column-major, as on exit).  The relative
 * residual is still ||b - A x|| / ||b||; a right-hand side with b = 0 returns
 * x = 0.  A caller can so run a few restart cycles per call (maxit = one cycle)
 * and continue unconverged right-hand sides in a later call, next to new ones
 * (the serving loop admits requests at cycle boundaries this way).  Other
 * arguments, results and errors as lrx_gmres_batch_dev. */
lrx_status lrx_gmres_batch_dev_x0(int32_t k, const lrx_handle* hs, int32_t nrhs, const double* const* b_dev,
                                  double* const* x_dev, double tol, int32_t restart, int32_t maxit,
                                  int32_t* iters, double* relres);

/* Moves the handle to another HIP stream (NULL: the null stream): solves and
 * GMRES calls on it are enqueued there from now on, so a server can factor on
 * one stream while it solves on another.  The caller orders the switch with any
 * work still running on the old stream.  Errors: LRX_EINVAL (bad handle). */
lrx_status lrx_set_stream(lrx_handle h, void* stream);

/* Releases every resource of the handle (its device blocks go to the library's
 * reuse cache after a device-wide synchronization).  NULL is accepted.  A
 * handle that was already freed gives LRX_EINVAL. */
lrx_status lrx_free(lrx_handle h);

/* Releases the handle's solve and GMRES workspaces (extended vectors, Krylov
 * basis, batch tables); the next solve or GMRES call grows them again.  The
 * factorization stays resident.  Waits for the handle's stream.  A server
 * trims idle handles to keep their device footprint (lrx_stats device_bytes)
 * at the factor itself.  Errors: LRX_EINVAL (bad handle). */
lrx_status lrx_trim(lrx_handle h);

/* Fills *s with the counters of the factorization. */
lrx_status lrx_stats(lrx_handle h, lrx_stats_t* s);

/* Ranks of all compressions in processing order (level l..1, then the order
 * inside the level); ranks must hold n_compressions entries; levels and js
 * (same length, may be NULL) receive the level i and super-node index j. */
lrx_status lrx_ranks(lrx_handle h, int32_t* ranks, int32_t* levels, int32_t* js);

/* Truncation data of compression idx (same order as lrx_ranks).
 * LRX_SVD:  out[0] = sigma_0, out[1..c] = all singular values of the stacked
 *           block in descending order (c = its number of non-zero columns);
 *           *len = c + 1.
 * LRX_RRQR: out[0] = |R11| (largest row norm of B), out[1 + k] = ||R22||_F before
 *           pivot step k, k = 0..rank; *len = rank + 2.
 * LRX_RAND: as LRX_SVD, with the singular values of the sketched block C = B Q
 *           (l of them, then zeros) for the blocks of at most 64 columns.
 * At most cap values are written. */
lrx_status lrx_compression_tails(lrx_handle h, int32_t idx, double* out, int32_t cap, int32_t* len);

/* Shape of the stacked block B of compression idx (same order as lrx_ranks, Sec.
 * 4.3): *rows = the rows stored (the non-zero rows of the pieces of
 * well-separated neighbours), *cols = its columns c (the super-node's variables
 * that couple to them).  The variant that compressed it follows from the
 * shape: c <= 64, 64 < c <= 192 (tall when rows c >= 3e5), and the split form
 * beyond (or rows c >= 1e6).  LRX_EINVAL for a bad index or NULL outputs. */
lrx_status lrx_compression_shape(lrx_handle h, int32_t idx, int32_t* rows, int32_t* cols);

/* Residual history of the last lrx_gmres / lrx_gmres_dev / batched GMRES call on
 * this handle for right-hand side rhs (Sec. 6.2, FGMRES with the solve as
 * preconditioner): in order, the true relative residual ||b - A x|| / ||b|| at
 * the start of each restart cycle, then the estimate |g_{j+1}| / ||b|| after
 * each Arnoldi step j of that cycle.  *len = the number of values (0 before any
 * GMRES call); at most cap are written to out (host memory, may be NULL).
 * LRX_EINVAL for rhs outside the last call's right-hand sides. */
lrx_status lrx_gmres_history(lrx_handle h, int32_t rhs, double* out, int32_t cap, int32_t* len);

/* Host-only symbolic plan of Algorithm 1 for (A, T, order): no device call. */
lrx_status lrx_plan_inspect(const lrx_csr* A, const lrx_tree* T, int32_t order,
                            lrx_plan_info* info);

/* Optional event timing of kernel launches, accumulated by kernel class over
 * all handles until read with reset.  lrx_timing_enable takes a bit mask of
 * classes (1 << LRX_K_...; 0 turns timing off, the default); every timed launch
 * adds two event records to its stream. */
typedef enum {
    LRX_K_COMPRESS = 0,       /* stacked-block assembly + truncated SVD / RRQR (Sec. 4.3) */
    LRX_K_FACTOR_NODE = 1,    /* projection, rewiring and pivot inverses of the nodes (Sec. 4.3, 4.4) */
    LRX_K_SOLVE_FWD = 2,      /* SolveL sweep of one colour step (Algorithm 3) */
    LRX_K_SOLVE_BWD = 3,      /* SolveU sweep of one colour step (Algorithm 4) */
    LRX_K_SPMV = 4,           /* A times the preconditioned vectors (GMRES) */
    LRX_K_SCHUR = 5,          /* Schur-complement products of Eliminate(s), Eliminate(b) (Sec. 2.2) */
    LRX_K_PROJECT = 6,        /* projection [R; Q] = B V of the compressed blocks (Sec. 4.3) */
    LRX_K_COMPRESS_GRAM = 7,  /* Compress through the FP64 Gram matrix (lrx_tune.compress_gram) */
    LRX_K_CLASSES = 8
} lrx_kernel_class;

typedef struct {
    int64_t launches;
    double total_ms;          /* sum of event-measured durations */
    double bytes;             /* algorithmic bytes (stored blocks / matrix read), summed */
    double flops;             /* algorithmic flops, summed */
} lrx_kernel_time;

typedef struct {
    lrx_kernel_time k[LRX_K_CLASSES];
} lrx_timing_t;

void lrx_timing_enable(int32_t class_mask);
lrx_status lrx_timing_read(lrx_timing_t* t, int32_t reset);

/* Launch shapes of the hot kernels, process-wide.  The library starts with
 * defaults; a tuner measures the alternatives on the device and a caller sets
 * the winners once, before factorizations and solves (setting them while calls
 * run on other threads races).  Results depend on these shapes only through
 * rounding order (gemm_kc: K blocking of the products; compress_nt_*: row
 * segments of the compression's QRs).  Errors: LRX_EINVAL for values out of
 * range. */
typedef struct {
    int32_t gemm_kc;          /* K chunk staged in LDS by the MFMA products: 16..256, multiple of 16 */
    int32_t gemm_f64_valu;    /* 1: FP64 products on the VALU tile kernel instead of the matrix cores */
    int32_t sweep_nk_max;     /* right-hand sides per solve-sweep work-group (at most; the library also
                                 splits them into slices that run side by side): 1, 2 or 4 */
    int32_t compress_nt_small;  /* threads per stacked block of <= 32 columns in Compress: 256, 512, 1024 */
    int32_t compress_nt_mid;    /* the same for 33..64 columns */
    int32_t gemm_grid;        /* 0: one work-group per 32 x 32 product tile; n > 0: a persistent grid of at
                                 most n work-groups walks the tile list (0..65536) */
    int32_t solve_graph;      /* 1: GMRES captures its preconditioner (the sweep launches of one
                                 application) into a HIP graph after the first application and
                                 replays it at every later Arnoldi step (not on the null stream,
                                 nor while solve sweeps are event-timed); 0: direct launches */
    int32_t compress_gram;    /* SVD compression at epsilon >= 1e-5 under the cut-off of eqn. cutOff1
                                 with R1 and the column order from the FP64 Gram matrix G = B^T B and a
                                 Cholesky factorization with diagonal pivoting, instead of the QR of B
                                 and the QRCP of R (the LQ and the one-sided Jacobi follow as usual):
                                 sigma_k is off by about c u sigma_0^2 / sigma_k and values below about
                                 sqrt(c u trace(G)) are not resolved.  Blocks of more than 64 columns
                                 form G on the matrix cores and factor it in panels.  0 never, 1 in mixed
                                 precision (default), 2 in mixed and FP64 precision */
    int32_t large_split_c;    /* stacked blocks with more columns than this (65..65536; default 128), or
                                 with rows x columns >= 1e6, finish their compression in launches over
                                 many work-groups (panel LQ and block-Jacobi rounds); narrower ones
                                 above 64 columns in one work-group per block */
} lrx_tune;

lrx_status lrx_tune_get(lrx_tune* t);
lrx_status lrx_tune_set(const lrx_tune* t);

/* Message of the last error on this thread ("" if none). */
const char* lrx_last_error(void);

/* Library version string. */
const char* lrx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LORAX_H */
