// Symbolic plan of the hierarchical factorization (host only, no device calls).
//
// The plan replays Algorithm 1 of the paper on the *structure* of the H-tree:
// which edges exist, which neighbours of a super-node are well-separated, which
// Schur-complement updates an elimination performs, and the row/column support
// of every block.  Nothing here depends on numerical values or on the ranks the
// compressions will find, so the whole structure is known before the first
// kernel runs; only block dimensions along auxiliary (rank-sized) variables are
// resolved at run time.
//
// Exact zero rows/columns: blocks that touch a leaf super-node are stored
// compactly.  A leaf block Mat(u -> v) only has non-zero rows at the degrees of
// freedom of v that couple to u, and the Schur update
//   Mat(k->q) -= Mat(s->q) Mat(s->s)^{-1} Mat(k->s)
// only has non-zero rows where Mat(s->q) has rows and non-zero columns where
// Mat(k->s) has columns.  The plan propagates these supports (index sets of
// local variables) structurally; they are exact, so compaction does not change
// any result.  Dimensions along auxiliary variables are always full.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace lrx {

struct Support {
    bool all = true;
    std::vector<int32_t> idx;   // sorted, unique local indices (when !all)
    void unite(const Support& o);
    int32_t count(int32_t full) const { return all ? full : (int32_t)idx.size(); }
};

enum NodeKind : int8_t { NK_RED = 0, NK_SUPER = 1, NK_BLACK = 2 };

struct PNode {
    NodeKind kind;
    int32_t level = 0, idx = 0;
    int32_t static_size = -1;   // leaf super-nodes: number of degrees of freedom
    bool leaf = false;          // leaf super-node (supports index its dofs)
    int32_t comp0 = -1, comp1 = -1;  // super-node above the leaves: its two red nodes
    int32_t dof0 = 0;           // leaf super-node: first tree position
    int32_t elim = -1;          // elimination position (Order)
};

enum EdgeOrigin : int8_t { EO_INIT, EO_MERGE, EO_R, EO_QT, EO_VT, EO_V, EO_NEGI, EO_FILL };

struct PEdge {
    int32_t src, dst;           // Mat(src -> dst): rows = vars of dst, cols = vars of src
    Support rows, cols;
    EdgeOrigin origin;
};

struct CandRef {
    int32_t p;                  // well-separated neighbour
    int32_t e_sp, e_ps;         // Mat(s->p), Mat(p->s) (-1 if absent)
    int32_t e_Pp, e_pP;         // new edges P(b)->p (R_k) and p->P(b) (Q_k^T)
};

struct PivotPlan {
    int32_t node = -1, e_self = -1;
    std::vector<int32_t> in_nodes, in_edges;     // k, Mat(k->v)
    std::vector<int32_t> out_nodes, out_edges;   // q, Mat(v->q)
    std::vector<int32_t> pair_in, pair_out, pair_edge;   // Schur pairs -> Mat(k->q)
};

struct NodeStep {
    int32_t j = 0, s = -1, b = -1, P = -1;
    std::vector<CandRef> cands;   // order: red nodes by index, then super-nodes by index
    Support gamma;                // columns of the stacked block (vars of s)
    int32_t e_sb = -1, e_bs = -1, e_bP = -1, e_Pb = -1;
    PivotPlan ps, pb;
};

struct ColourStep {
    int32_t level = 0, colour = 0;
    std::vector<NodeStep> nodes;
    std::vector<int32_t> new_edges;   // edges first created in this step
};

struct MergePiece {
    int32_t src_edge, dst_edge;
    int8_t row_hi, col_hi;            // 1: the piece sits after the first red node
};

struct LevelPlan {
    int32_t level = 0;
    std::vector<int32_t> supers;      // node ids, index j
    std::vector<MergePiece> merges;
    std::vector<int32_t> merge_edges;
    int32_t step0 = 0, nsteps = 0;
    int32_t colours = 0;
    int64_t candidates = 0;
};

struct Plan {
    int32_t n = 0, depth = 0, order = 0;
    std::vector<int32_t> leaf_ptr, perm, pos;
    std::vector<PNode> nodes;
    std::vector<PEdge> edges;
    std::vector<LevelPlan> levels;    // levels[0] is the leaf level (depth), last is level 1
    std::vector<ColourStep> steps;
    std::vector<int32_t> init_edges;  // leaf super-node edges taken from A
    std::vector<int32_t> elim_nodes;  // nodes in elimination order
    int32_t root_red = -1;
    int64_t n_candidates = 0, n_pairs = 0;
};

// Checks the CSR and tree and builds the plan; returns "" or an error message.
// nthreads > 1: the CSR checks, the leaf-cluster adjacency and the leaf blocks
// are computed on that many host threads (same plan).
std::string build_plan(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                       int32_t depth, const int32_t* perm, const int32_t* leaf_ptr,
                       int32_t order, Plan& out, int nthreads = 1);

// Position of every element of `sub` inside `sup` (both supports of the same
// node); empty vector when both are full; the single value -1 when sub is not
// a subset of sup (a planning error).
std::vector<int32_t> positions(const Support& sub, const Support& sup, int32_t full);

}  // namespace lrx
