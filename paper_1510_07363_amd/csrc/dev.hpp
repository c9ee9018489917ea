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
    int32_t piece0, npieces;
    int32_t M, c;
    double* B;          // SVD: M x c column-major (kept); RRQR: M x c row-major (overwritten)
    double* Bw;         // SVD: working copy of B (M x c column-major)
    double* V;          // c x c column-major: first r columns = V on exit
    double* hv;         // SVD: c x c R / Jacobi matrix; RRQR: Householder vectors
    int32_t* rank_out;  // one int
    double* tails;      // SVD: sigma_0 then the c singular values in descending order;
                        // RRQR: |R11|, then ||R22||_F before each step and at the stop
    double eps;
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

struct DIn {             // in-edge Mat(k -> v); its rows are vars of v
    DBlk blk;
    int32_t rmap, pad_;  // rows -> pivot-local index (map or identity)
    double* W;           // workspace m x blk.nc: Mat(v->v)^{-1} Mat(k->v)
};

struct DOut {            // out-edge Mat(v -> q); its columns are vars of v
    DBlk blk;
    int32_t cmap, pad_;  // columns -> pivot-local index
};

struct DPair {           // Mat(k->q)[rpos, cpos] -= Mat(v->q) W_k
    DBlk tgt;
    int32_t in_i, out_i;
    int32_t rpos, cpos;  // row positions (len out.nr) and column positions (len in.nc) in tgt
};

struct DPivot {
    DBlk piv;            // Mat(v->v), inverted in place
    int32_t in0, nin, out0, nout, pair0, npair;
    int32_t info_slot, pad_;
};

struct DNode {
    int32_t r, c, nproj, proj0;
    int32_t M, svd;      // svd: R_k / Q_k = B V computed from the kept B (column-major, ld M)
    const double* B;     // SVD: stacked block (column-major); RRQR: transformed block (row-major)
    const double* V;     // c x r column-major
    DBlk sb, bs, bP, Pb; // Mat(s->b) = V^T, Mat(b->s) = V, Mat(b->P) = Mat(P->b) = -I_r
    DPivot ps, pb;
};

// ---- MergeRedNodes: copy a red block into its super-node block --------------
struct DMerge {
    DBlk src, dst;
    int32_t r0, c0;
};

// ---- Solve sweeps ------------------------------------------------------------
// Row a of an edge maps to rbase + a (rmap < 0) or imap[rmap + a]; columns
// likewise.  Out-edges (forward) carry absolute rows / pivot-local columns;
// in-edges (backward) pivot-local rows / absolute columns.
struct DSEdge {
    const double* E;
    int32_t nr, nc;
    int32_t rbase, rmap, cbase, cmap;
};

struct DSPiv {
    const double* Sinv;  // m x m column-major
    int32_t m, off;      // variables [off, off + m) of the extended vector
    int32_t out0, nout, in0, nin;
};

struct DSNode {
    DSPiv s, b;
};

}  // namespace lrx
