// Host-side launchers of the HIP kernels (kernels.hip).  All launches are
// asynchronous on `st`; every pointer is device memory.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dev.hpp"

namespace lrx {

constexpr int kFactorThreads = 256;

// dst_base[idx[e]] = val[e], e < nnz
hipError_t launch_scatter(double* dst_base, const int64_t* idx, const double* val, int64_t nnz,
                          hipStream_t st);
hipError_t launch_merge(const DMerge* t, int n, hipStream_t st);
// Frobenius rule (eqn. curOff6): adds the squared Frobenius norms of the nv
// values v (v != nullptr) or of the source blocks of npieces merge pieces
// (npieces may be 0) to state[0], then state[1] = eps sqrt(state[0]) and
// state[2 + level] = sqrt(state[0]); partial holds level_norm_groups(npieces,
// nv) doubles.
hipError_t launch_level_norm(const DMerge* pieces, int npieces, const double* v, int64_t nv, double* state,
                             double* partial, double eps, int level, hipStream_t st);
int level_norm_groups(int npieces, int64_t nv);
// dst[e] = src[idx[e]]
hipError_t launch_gather_idx(double* dst, const double* src, const int64_t* idx, int64_t n,
                             hipStream_t st);
// *cnt = number of non-finite entries of v
hipError_t launch_count_nonfinite(const double* v, int64_t n, int64_t* cnt, hipStream_t st);
// lds_bytes: dynamic LDS per work-group
hipError_t launch_compress(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap,
                           int max_c, hipStream_t st);
// fp32: reduced QRs and Jacobi in FP32 when every task has c <= 64 (mixed
// precision); nt: threads per task (256, 512 or 1024) when every task has c <= 64
// gram (max_c <= 64): R1 and the column order from the FP64 Gram matrix and a
// pivoted Cholesky instead of the QR and QRCP of B.
hipError_t launch_compress_svd(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap,
                               int max_c, int max_M, bool fp32, int nt, hipStream_t st, bool gram = false);
// Truncated SVD of stacked blocks with c > 64 columns (FP64, matrices in the
// workspace: hv needs 4 c^2 + c + 8 doubles, Bw M c).  Trailing QRCP rows below
// trunc_rel * epsilon * |R1[0,0]| (Frobenius) are dropped (0: only exact
// zeros).  Fits when compress_large_fits(M, c).
// mode 0: the whole pipeline per work-group; launch_assemble_large(copy =
// true) + launch_qr_blocked(0) + mode 5 + launch_qr_blocked(1, 2) + mode 6: the
// QRs over many work-groups and the state (Jacobi only for L taller than the
// block rounds hold), then launch_large_round for rounds
// 0..large_rounds(max_c)-1 per sweep and launch_large_flags (out[i] = 1: task i
// goes on) until no task goes on; mode 2: singular values, rank and V; mode 7:
// after launch_assemble_large(copy = true) and launch_qr_blocked(0), the rest in
// one work-group; launch_assemble_large(copy = false) + launch_gram_chol + mode
// 8 leave what mode 5 leaves through the Gram matrix, and mode 9 then does the
// rest in one work-group.
// jac_f32: the one-sided Jacobi stops at the FP32 level (rotation threshold
// 3.6 u_32 kk instead of 3.6 u_64 kk), for mixed precision.
hipError_t launch_compress_large(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap, int max_c,
                                 int max_M, double trunc_rel, int mode, hipStream_t st, bool jac_f32 = false);
hipError_t launch_large_round(const DCompress* t, int n, int max_c, int round, hipStream_t st);
// Assembly of the stacked blocks B of large tasks over many work-groups (zero,
// scatter of the pieces, largest |entry|); copy: also Bw = B / 2^e and the
// scale in the header, for the QR route.
hipError_t launch_assemble_large(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap,
                                 int64_t max_mc, int max_pieces, bool copy, hipStream_t st);
// FP64 Gram matrix of every task's B / 2^e (matrix cores) and its Cholesky
// factorization with diagonal pivoting in panels, truncated like the QRCP of
// mode 5 (trunc_rel; and below c u trace(G)): between
// launch_assemble_large(copy = false) and mode 8.
hipError_t launch_gram_chol(const DCompress* t, int n, int max_c, double trunc_rel, hipStream_t st);
// Randomized compression of stacked blocks with at most 64 columns (see
// k_rand_sketch): the sketch launch (first = 1 also assembles B, ||B||_F^2 and
// the nonzero column count; it writes the width l and the full-sketch flag
// into ctasks), then launch_compress_svd(fp32 = false) on ctasks, then the
// finish launch (flags[i]: bit 0 = task i needs a wider sketch, bits 1..7 the
// Jacobi sweeps, bits 8.. the width).
hipError_t launch_rand_sketch(const DCompress* t, const DRand* rt, DCompress* ctasks, int n, const DPiece* pieces,
                              const int32_t* imap, int first, int bf16, hipStream_t st);
// Each column of V of every task gets its entry of largest magnitude positive.
hipError_t launch_v_sign(const DCompress* t, int n, hipStream_t st);
hipError_t launch_rand_finish(const DCompress* t, const DRand* rt, const DCompress* ctasks, int n, int32_t* flags,
                              hipStream_t st);
// Blocked Householder QR in panels of 16 columns over many work-groups:
// which 0: tall QR of every task's Bw (between launch_compress_large modes 4
// and 5); which 1: QR of A2 (the LQ step) and which 2: W = Q2 E (between modes 5
// and 6).
hipError_t launch_qr_blocked(const DCompress* t, int n, int max_c, int max_M, int which, hipStream_t st);
int large_rounds(int max_c);
hipError_t launch_large_flags(const DCompress* t, int n, int32_t* out, hipStream_t st);
inline bool compress_large_fits(int M, int c) {
    const size_t vlen = (size_t)(M > c ? M : c) + 1;
    return (vlen + 4 * (size_t)c) * sizeof(double) + 2 * (size_t)c * sizeof(int) <= 152 * 1024;
}
// Projection, rewiring and pivot inverse per task (DPrep); info[slot] = 1 for an
// exactly singular pivot.  gj_perm (kGjPermInts ints per task; required when
// max_m > 128): pivots of 129..1024 rows are inverted by panel and update
// launches over many work-groups.
constexpr int kGjPermInts = 1024;
hipError_t launch_node_prep(const DPrep* t, int n, int max_m, const DProj* proj, const int32_t* imap,
                            int32_t* info, hipStream_t st, int* gj_perm = nullptr);
// ntile 32 x 32 tiles of the products g (DGemm, DTile); kmax = largest K.
hipError_t launch_gemm_tiles(const DGemm* g, const DTile* tiles, int ntile, int kmax, const int32_t* imap,
                             hipStream_t st);
// The same products on the matrix cores (gemm.hip): operands staged as FP64,
// FP32 or BF16 (prec: GP_*), FP64 or FP32 accumulation; K staged in chunks of
// at most kc_cap (<= 256) columns; grid_cap > 0: a persistent grid of at most
// grid_cap work-groups walks the tile list (0: one work-group per tile).
enum { GP_F64 = 0, GP_F32 = 1, GP_BF16 = 2 };
hipError_t launch_gemm_mfma(const DGemm* g, const DTile* tiles, int ntile, int kmax, const int32_t* imap, int prec,
                            int kc_cap, int grid_cap, hipStream_t st);

// One sweep launch (forward or backward program) over n super-nodes of a
// colour step and ns slices of nk right-hand sides, [k0, k0 + ns nk) of x (ldx
// per row), nk in {1,2,4,8}; a work-group per (node, slice).
// Nodes with x == nullptr use x; each node's program is its own device pointer
// and each run states its blocks' storage type, so nodes of several
// factorizations (FP64 or mixed precision) can share one launch.
hipError_t launch_sweep(const SwNode* nodes, int n, double* x, int ldx, int k0, int nk, int ns, hipStream_t st);
// Device address of the static scratch array of the allocation-free entry
// points on device dev (which must be current at the first call per device);
// kNoallocScratchBytes per device, shared by every such call on that device.
constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
hipError_t noalloc_scratch(int dev, void** ptr);

// Copies of stored blocks (DConv: to FP32, or FP64 as is), one work-group per block.
hipError_t launch_to_f32(const DConv* segs, int n, hipStream_t st);

// ---- vectors: layout v[i * nrhs + k] ("row-interleaved") -------------------
// xt[t*nrhs + k] = b[perm[t] + k*ldb]   (t < n)      and zero xt[n*nrhs .. ntot*nrhs)
hipError_t launch_gather_perm(const double* b, int64_t ldb, const int32_t* perm, int n, int nrhs,
                              double* xt, int64_t ntot, hipStream_t st);
// x[perm[t] + k*ldx] = xt[t*nrhs + k]
hipError_t launch_scatter_perm(const double* xt, const int32_t* perm, int n, int nrhs, double* x,
                               int64_t ldx, hipStream_t st);
// ---- batched FGMRES vector operations (DKry systems, DKryChunk chunks) ------
// Rows per chunk for nrhs right-hand sides (about 2048 elements per work-group).
inline int kry_rows(int nrhs) { return nrhs >= 2048 ? 1 : 2048 / nrhs; }
struct KryLaunch {
    const DKry* sys;
    const DKryChunk* ch;
    const int32_t* act;     // per system: 0 = skip
    int nchunk, nsys, nrhs, rc;
    hipStream_t st;
};
// mode 0: b = bin in tree order, x = 0;  mode 1: xout = x in the original order;
// mode 2: x = xout in tree order (an initial guess), 0 for right-hand side k
// when sm[off + k] (its ||b||^2) is 0
hipError_t kry_perm(const KryLaunch& L, int mode, int off = 0);
// residual: r = b - A x;  otherwise w = A Z_j
hipError_t kry_spmv(const KryLaunch& L, bool residual, int j);
// sm[out_off + j*nrhs + k] = (mode 0) <V_j, w>_k for j < J, (1) ||w||_k^2, (2) ||r||_k^2;
// part holds nchunk * J * nrhs doubles
hipError_t kry_dots(const KryLaunch& L, int mode, int J, double* part, int out_off);
// op 0: w -= sum_{j<J} V_j h_j (h at sm[off]);  op 1: x += sum_{j<Js} Z_j y_j (y at
// sm[off], Js = sm[off2]);  op 2: V_j = (J == 0 ? r : w) / sqrt(sm[off + k]);
// op 3: xe = [V_j; 0];  op 4: Z_j = xe[0:n]
hipError_t kry_axpy(const KryLaunch& L, int op, int J, int j, int off, int off2);

}  // namespace lrx
