// Device-side task descriptors shared by the host driver and the HIP kernels.
//
// Blocks Mat(u -> v) are dense, column-major, leading dimension = rows.  A
// "map" is an offset into an int32 index table in device memory, or -1 for the
// identity.  Every descriptor is built on the host (all sizes are known when a
// kernel is launched) and uploaded before the launch.
#pragma once

#include <cstdint>

namespace lrx {

struct DBlk {
    double* p;
    int32_t nr, nc;
};

// ---- Compress: one work-group per super-node ---------------------------------
// The stacked block B (eqn. lra) is assembled in workspace, row-major M x c
// (a row of B is contiguous), from pieces:
//   trans == 0: rows [row0, row0 + blk.nr) of B are the rows of blk (A_k = Mat(s->p_k));
//               column t of blk goes to column map[t] of B
//   trans == 1: rows [row0, row0 + blk.nc) of B are the columns of blk (B_k = Mat(p_k->s)^T);
//               row t of blk goes to column map[t] of B
struct DPiece {
    DBlk blk;
    int32_t trans, row0, map, pad_;
};

// Two truncation rules share the descriptor:
//   SVD  (eqn. cutOff1): B is assembled column-major (ld M) and kept; a copy is
//        reduced by Householder QR to the c x c triangle R, whose one-sided
//        Jacobi SVD gives sigma and V; rank = #{sigma_k >= eps * sigma_0}.
//   RRQR: B is assembled row-major and overwritten by the row-pivoted QR.
struct DCompress {
    int32_t piece0, npieces;   // npieces < 0 (small-block SVD only): B is already in place
    int32_t M, c;
    double* B;          // SVD: M x c column-major (kept); RRQR: M x c row-major (overwritten)
    double* Bw;         // SVD: working copy of B (M x c column-major)
    double* V;          // c x c column-major: first r columns = V on exit
    double* hv;         // SVD: c x c R / Jacobi matrix; RRQR: Householder vectors
    int32_t* rank_out;  // one int
    double* tails;      // SVD: sigma_0 then the c singular values in descending order;
                        // RRQR: |R11|, then ||R22||_F before each step and at the stop
    double eps;
    const double* tau;  // nullptr: cut-off of eqn. cutOff1 (eps relative to sigma_0); else the
                        // absolute threshold of eqn. curOff6: the smallest k whose discarded
                        // tail has Frobenius norm < *tau (RRQR: ||R22||_F < *tau)
    const double* nb2;  // randomized compression (the sketched block C = B Q is this task):
                        // ||B||_F^2 of the original stacked block, for the rank rule of the
                        // sketch (nullptr otherwise)
    int32_t rand_full;  // the sketch spans every column of B (nothing uncaptured)
    int32_t rand_pad_;
};

// Randomized compression of one stacked block with at most 64 columns: the
// requested sketch width l and the task key of its counter-based sketch (the
// sketched block C = B Q, M x l, is compressed by a task of its own at the same
// index, whose width and full-sketch flag the sketch kernel fills in).
struct DRand {
    int32_t l, active;
    int64_t key;
};

// ---- Node factorization: projection, rewiring, Eliminate(s), Eliminate(b) ---
// After the pivoted QR, the first r columns of the transformed B equal B V, so
// the blocks R_k (trans 0) and Q_k^T (trans 1) are copies of rows of B.
struct DProj {
    DBlk dst;
    int32_t row0, nrows, trans;
    int32_t map;         // position of each piece row inside dst's rows (trans 0) or
                         // columns (trans 1): later fill may widen dst's support
};

// One launch per colour step prepares every super-node (projection and
// rewiring, then the inverse of its pivot); a second kind of launch covers the
// pivot of the black node only (do_proj == 0).
struct DPrep {
    int32_t r, c, nproj, proj0;
    int32_t M, svd;      // svd: R_k / Q_k = B V computed from the kept B (column-major, ld M)
    const double* B;     // SVD: stacked block (column-major); RRQR: transformed block (row-major)
    const double* V;     // c x r column-major
    DBlk sb, bs, bP, Pb; // Mat(s->b) = V^T, Mat(b->s) = V, Mat(b->P) = Mat(P->b) = -I_r
    DBlk piv;            // pivot block Mat(v->v), inverted in place (nr == 0: none)
    int32_t info_slot, do_proj;
};

// ---- Block elimination as batched gather/scatter products (Sec. 2.2) --------
//   C[crow(i), ccol(j)] (-)= sum_t A[i + acol(t) lda] B[brow(t) + j ldb]
// i < M, j < N, t < K; every map is an imap offset or -1 (identity).  For the
// pivot v with inverse S: W_k = S[:, rows of Mat(k->v)] Mat(k->v) (sub = 0),
// then Mat(k->q)[rpos, cpos] -= Mat(v->q) W_k[cols of Mat(v->q), :] (sub = 1).
struct DGemm {
    const double* A;
    const double* B;
    double* C;
    int32_t M, N, K;
    int32_t lda, ldb, ldc;
    int32_t amap, bmap, crmap, ccmap;
    int32_t sub;
    int32_t tr;          // 1: element (i, j) of the product goes to C[ccol(j) + crow(i) ldc]
};

struct DTile {           // one 32 x 32 block of C of product g
    int32_t g, i0, j0, pad_;
};

// ---- MergeRedNodes: copy a red block into its super-node block --------------
struct DMerge {
    DBlk src, dst;
    int32_t r0, c0;
};

// ---- Solve sweeps (Algorithms 3 and 4): staged node programs ---------------
// One work-group runs the program of one super-node of a colour step (its
// pivot s, then its black node b in the forward sweep; b, then s backward).
// A program is a sequence of stages.  Each stage first copies "runs" of global
// data (rows of stored blocks, gathered rows of the extended vector x) into
// LDS with every load of the stage in flight at once, then executes its groups
// of row computations, with a barrier after each group.  The descriptor block
// of stage k+1 is fetched together with the data of stage k.
//
// Descriptor blocks are int32 words: a header, then groups, runs, comps and the
// index lists ("maps") they use; a map is a word offset inside the same block,
// or -1 for the identity.  LDS data offsets are in doubles.
constexpr int kSwThreads = 1024;       // work-group size of the sweep kernel
constexpr int kSwDescWords = 2048;     // largest descriptor block (two are resident)
constexpr int kSwData = 17408;         // doubles of LDS for buffers and staged data
constexpr int kSwKS = 4;               // row stride of vector buffers in LDS (max RHS per work-group)

struct SwNode {
    const int32_t* desc; // stage 0's descriptor block (device)
    double* x;           // extended vector of this node's system (nullptr: the launch's)
    const int32_t* live; // nullptr, or a flag of the node's system: 0 = skip the node
    int32_t words0;      // size of stage 0's block in words
    int32_t nstage;
};

struct SwHeader {        // 8 words
    int32_t words_next;  // size of the next stage's block (0 for the last stage)
    int32_t nrun;
    int32_t elems_mat;   // elements of the matrix runs of this stage
    int32_t ngroup;
    int32_t groups, runs, comps;   // word offsets of the sections
    int32_t xrows;       // rows of x copied by the vector runs of this stage
};

struct SwGroup {         // 4 words: comps [comp0, comp0 + ncomp), rows summed
    int32_t comp0, ncomp, rows;
    int32_t lglanes;     // log2 of the lanes that share one row's dot products
};

// Matrix run set: nrun runs of len elements, run t at src + t * ld (elements of
// es bytes: FP64, or FP32 for the off-diagonal blocks in mixed precision),
// stored in LDS as doubles at lds + t * dld.  Vector run set (src == nullptr): nrun rows of x, row t is x row (map < 0
// ? ld + t : map[t]), the launch's right-hand sides, stored in the LDS row that
// starts at lds + t * kSwKS (elements of a row in a bank-spreading order).
struct SwRun {           // 10 words
    const void* src;
    int32_t ld, len, nrun, map, lds, dld;
    float rlen;          // 1 / len (index split without integer division)
    int32_t es;          // bytes per element of src: 8 (FP64) or 4 (FP32)
};

// One row computation: for each row a < nr of the block at LDS `mat`
// (column-major, leading dimension ld), with acc[k] = sum_t mat[a + t ld] *
// in[(in_map ? in_map[t] : t) * kSwKS + k]:
//   out value = init < 0 ? acc : init_row(a)[k] - acc
// written to LDS (out >= 0) and/or to x (gbase >= 0 or gmap >= 0).
struct SwComp {          // 12 words
    int32_t mat, ld, nr, nc;
    int32_t in, in_map;
    int32_t init, init_map;
    int32_t out, out_map;
    int32_t gbase, gmap;
};

// Copy of one stored block for the solve (mixed precision): to FP32 (f64 == 0)
// or as FP64 (f64 == 1, pivot inverses)
struct DConv {
    const double* src;
    void* dst;
    int64_t n;
    int32_t f64, pad_;
};

// ---- Batched FGMRES vectors (preconditioned by the solve, Sec. 6.2) ---------
// Vectors of a system are n x nrhs, row-interleaved (v[i*nrhs + k]), in tree
// order.  One work-group per chunk of rows of one system (DKryChunk); systems
// whose act flag is 0 are skipped.
struct DKry {
    int32_t n, chunk0;          // rows; first chunk of the system in the chunk table
    int32_t nchunk, pad_;
    int64_t nv, n_ext;          // n * nrhs; rows of the extended vector
    const int64_t* rp;          // A in tree order (CSR)
    const int32_t* ci;
    const double* av;
    const int32_t* perm;        // tree position -> original index
    double* V;                  // basis V_0..V_m, each nv
    double* Z;                  // preconditioned vectors Z_0..Z_{m-1}
    double* w;
    double* r;
    double* b;                  // right-hand sides in tree order
    double* x;                  // iterate in tree order
    double* xe;                 // extended vector of the solve (n_ext x nrhs)
    double* sm;                 // scalars, see kry_sm_* offsets
    const double* bin;          // caller's b and x: n x nrhs column-major
    double* xout;
};
struct DKryChunk {
    int32_t sys, row0;
};

}  // namespace lrx
