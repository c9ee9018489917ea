// Host-side compiler of the solve sweeps (Algorithms 3 and 4) into the staged
// node programs run by k_sweep (descriptor formats in dev.hpp).  Pure C++: no
// device calls; the caller uploads the result.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "dev.hpp"

namespace lrx {

// A stored block Mat(u -> v): column-major nr x nc, rows are variables of v and
// columns variables of u, given as local indices of those nodes (an empty list
// is the identity 0..n-1).  Blocks hold elements of es bytes (8: FP64, 4: FP32).
struct SwEdgeIR {
    const void* E = nullptr;
    int32_t nr = 0, nc = 0;
    int32_t other = -1;              // target node (out-edge) or source node (in-edge)
    int64_t other_off = 0;           // first variable of that node in the extended vector
    std::vector<int32_t> rows, cols; // local indices (rows of dst, cols of src)
};

struct SwPivIR {
    const void* inv = nullptr;       // explicit inverse of the pivot block, m x m column-major
    int32_t m = 0;
    int64_t off = 0;                 // first variable of the node
    int32_t node = -1;
    std::vector<SwEdgeIR> out, in;   // frozen out-edges (forward) and in-edges (backward)
};

struct SwNodeIR {
    SwPivIR s, b;                    // super-node pivot, then its black node
    int32_t es = 8;                  // bytes per element of the edge blocks
    int32_t es_piv = 8;              // bytes per element of the pivot inverses
};

// A node program before upload: its first block as a word offset.
struct SwNodeRel {
    int64_t desc = 0;
    int32_t words0 = 0, nstage = 0;
};

struct SwProgram {
    std::vector<int32_t> words;      // all descriptor blocks
    std::vector<SwNodeRel> fwd, bwd; // one per super-node, grouped by colour step
    std::vector<int32_t> step0;      // first node of each colour step (same in fwd and bwd)
    int64_t max_stages = 0, total_stages = 0;
};

// Compiles both sweeps.  Returns false with a message when a node cannot be
// staged within the LDS budget.
bool build_sweep_program(const std::vector<std::vector<SwNodeIR>>& steps, SwProgram& out,
                         std::string& err);

// Compiles the forward and backward programs of one super-node, appending their
// descriptor blocks to words (descriptors relative to the start of words).
bool build_node_programs(const SwNodeIR& N, std::vector<int32_t>& words, SwNodeRel& fwd, SwNodeRel& bwd,
                         std::string& err);

}  // namespace lrx
