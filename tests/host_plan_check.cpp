// Host-only check of the symbolic planner, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py: for a problem file
// (n, nnz, depth, row_ptr, col_idx, perm, leaf_ptr) it builds the plan on one
// and on four host threads, checks that both are the same plan, and that
// corrupted inputs are refused with a message instead of being read out of
// bounds.  Prints "ok" on success.
#include "plan.hpp"

#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

using namespace lrx;

static bool same(const Plan& a, const Plan& b) {
    if (a.edges.size() != b.edges.size() || a.nodes.size() != b.nodes.size() || a.steps.size() != b.steps.size() ||
        a.n_pairs != b.n_pairs || a.n_candidates != b.n_candidates)
        return false;
    for (size_t e = 0; e < a.edges.size(); ++e) {
        const PEdge &x = a.edges[e], &y = b.edges[e];
        if (x.src != y.src || x.dst != y.dst || x.origin != y.origin || x.rows.all != y.rows.all ||
            x.cols.all != y.cols.all || x.rows.idx != y.rows.idx || x.cols.idx != y.cols.idx)
            return false;
    }
    return true;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hd[3];
    if (fread(hd, 8, 3, f) != 3) return 2;
    const int32_t n = (int32_t)hd[0], depth = (int32_t)hd[2];
    const int64_t nnz = hd[1];
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> ci(nnz), perm(n), lp(((size_t)1 << depth) + 1);
    if (fread(rp.data(), 8, rp.size(), f) != rp.size() || fread(ci.data(), 4, ci.size(), f) != ci.size() ||
        fread(perm.data(), 4, perm.size(), f) != perm.size() || fread(lp.data(), 4, lp.size(), f) != lp.size())
        return 2;
    fclose(f);
    Plan p1, p4;
    std::string e1 = build_plan(n, nnz, rp.data(), ci.data(), depth, perm.data(), lp.data(), 0, p1, 1);
    std::string e4 = build_plan(n, nnz, rp.data(), ci.data(), depth, perm.data(), lp.data(), 0, p4, 4);
    if (!e1.empty() || !e4.empty()) { printf("unexpected error: %s %s\n", e1.c_str(), e4.c_str()); return 1; }
    if (!same(p1, p4)) { printf("plans differ between 1 and 4 threads\n"); return 1; }
    Plan pn;
    if (!build_plan(n, nnz, rp.data(), ci.data(), depth, perm.data(), lp.data(), 1, pn, 4).empty()) return 1;
    // corrupted inputs: each must be refused with a message
    int refused = 0, cases = 0;
    auto expect_error = [&](const std::vector<int64_t>& r, const std::vector<int32_t>& c, const std::vector<int32_t>& pm,
                            const std::vector<int32_t>& l, int32_t d) {
        Plan q;
        ++cases;
        if (!build_plan(n, (int64_t)c.size(), r.data(), c.data(), d, pm.data(), l.data(), 0, q, 4).empty()) ++refused;
    };
    { auto c = ci; c[nnz / 2] = n; expect_error(rp, c, perm, lp, depth); }                 // column out of range
    { auto c = ci; c[nnz - 1] = -1; expect_error(rp, c, perm, lp, depth); }               // negative column
    { auto c = ci; std::swap(c[rp[n / 2]], c[rp[n / 2] + 1]); expect_error(rp, c, perm, lp, depth); }   // unsorted row
    { auto r = rp; r[n / 3] = r[n / 3 + 1] + 1; expect_error(r, ci, perm, lp, depth); }   // decreasing row_ptr
    { auto pm = perm; pm[0] = pm[1]; expect_error(rp, ci, pm, lp, depth); }               // repeated index in perm
    { auto pm = perm; pm[n - 1] = n; expect_error(rp, ci, pm, lp, depth); }               // perm out of range
    { auto l = lp; l[1] = l[0]; expect_error(rp, ci, perm, l, depth); }                   // empty leaf
    { auto l = lp; l.back() = n + 1; expect_error(rp, ci, perm, l, depth); }              // leaves beyond n
    if (refused != cases) { printf("%d of %d corrupted inputs accepted\n", cases - refused, cases); return 1; }
    printf("ok %zu edges %lld pairs\n", p1.edges.size(), (long long)p1.n_pairs);
    return 0;
}
