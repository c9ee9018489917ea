// Symbolic plan of Algorithm 1 (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <numeric>
#include <thread>
#include <utility>

namespace lrx {

void Support::unite(const Support& o) {
    if (all) return;
    if (o.all) { all = true; idx.clear(); return; }
    if (std::includes(idx.begin(), idx.end(), o.idx.begin(), o.idx.end())) return;   // no change
    thread_local std::vector<int32_t> u;
    u.clear();
    u.reserve(idx.size() + o.idx.size());
    std::set_union(idx.begin(), idx.end(), o.idx.begin(), o.idx.end(), std::back_inserter(u));
    idx.assign(u.begin(), u.end());
}

std::vector<int32_t> positions(const Support& sub, const Support& sup, int32_t full) {
    std::vector<int32_t> p;
    if (sup.all) {
        if (sub.all) return p;                 // identity
        p = sub.idx;                           // positions inside the full set
        return p;
    }
    // sub must be a subset of sup
    if (sub.all) { p.clear(); p.push_back(-1); return p; }
    p.resize(sub.idx.size());
    size_t k = 0;
    for (size_t a = 0; a < sub.idx.size(); ++a) {
        while (k < sup.idx.size() && sup.idx[k] < sub.idx[a]) ++k;
        if (k == sup.idx.size() || sup.idx[k] != sub.idx[a]) { p.clear(); p.push_back(-1); return p; }
        p[a] = (int32_t)k;
    }
    (void)full;
    return p;
}

namespace {

struct Adj {                                   // active interaction edges of one node
    std::vector<std::pair<int32_t, int32_t>> v;   // (neighbour, edge)
    int32_t find(int32_t nb) const {
        for (auto& e : v) if (e.first == nb) return e.second;
        return -1;
    }
    void erase(int32_t nb) {
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i].first == nb) { v[i] = v.back(); v.pop_back(); return; }
    }
};

struct Builder {
    Plan& P;
    std::vector<Adj> out, in;
    std::vector<std::vector<std::vector<int32_t>>> cadj;   // [level][cluster] sorted neighbours
    std::vector<char> empty;       // node is known to have no variables (rank 0 for sure)
    int32_t elim_counter = 0;

    explicit Builder(Plan& p) : P(p) {}

    int32_t add_node(NodeKind k, int32_t level, int32_t idx) {
        PNode nd;
        nd.kind = k; nd.level = level; nd.idx = idx;
        P.nodes.push_back(nd);
        out.emplace_back();
        in.emplace_back();
        out.back().v.reserve(8);
        in.back().v.reserve(8);
        empty.push_back(0);
        return (int32_t)P.nodes.size() - 1;
    }
    int32_t add_edge(int32_t src, int32_t dst, Support rows, Support cols, EdgeOrigin o) {
        PEdge e;
        e.src = src; e.dst = dst; e.rows = std::move(rows); e.cols = std::move(cols); e.origin = o;
        P.edges.push_back(std::move(e));
        int32_t id = (int32_t)P.edges.size() - 1;
        out[src].v.push_back({dst, id});
        in[dst].v.push_back({src, id});
        return id;
    }
    void drop_edge(int32_t e) {
        const PEdge& E = P.edges[e];
        out[E.src].erase(E.dst);
        in[E.dst].erase(E.src);
    }
    Support full_or_empty(int32_t node) const {
        Support s;
        if (P.nodes[node].leaf) { s.all = false; }
        return s;
    }
    bool adjacent_or_equal(int32_t k, int32_t a, int32_t b) const {
        if (a == b) return true;
        const auto& nb = cadj[k][a];
        return std::binary_search(nb.begin(), nb.end(), b);
    }
    int32_t cluster_of(int32_t node) const { return P.nodes[node].idx; }

    // Block Gauss elimination of v: structural part (Sec. 2.2).
    void eliminate(int32_t v, PivotPlan& pp, ColourStep& cs) {
        pp.node = v;
        pp.e_self = out[v].find(v);
        pp.in_nodes.reserve(in[v].v.size());
        pp.in_edges.reserve(in[v].v.size());
        pp.out_nodes.reserve(out[v].v.size());
        pp.out_edges.reserve(out[v].v.size());
        for (auto& e : in[v].v) if (e.first != v) { pp.in_nodes.push_back(e.first); pp.in_edges.push_back(e.second); }
        for (auto& e : out[v].v) if (e.first != v) { pp.out_nodes.push_back(e.first); pp.out_edges.push_back(e.second); }
        // deterministic order: by node id
        auto sort_pair = [](std::vector<int32_t>& a, std::vector<int32_t>& b) {
            thread_local std::vector<std::pair<int32_t, int32_t>> ab;
            ab.clear();
            for (size_t i = 0; i < a.size(); ++i) ab.push_back({a[i], b[i]});
            std::sort(ab.begin(), ab.end());          // node ids are distinct
            for (size_t i = 0; i < ab.size(); ++i) { a[i] = ab[i].first; b[i] = ab[i].second; }
        };
        sort_pair(pp.in_nodes, pp.in_edges);
        sort_pair(pp.out_nodes, pp.out_edges);
        if (!empty[v]) {
            const size_t np = pp.in_nodes.size() * pp.out_nodes.size();
            pp.pair_in.reserve(np);
            pp.pair_out.reserve(np);
            pp.pair_edge.reserve(np);
        }
        // a pivot without variables creates no fill
        for (size_t qi = 0; !empty[v] && qi < pp.out_nodes.size(); ++qi) {
            int32_t q = pp.out_nodes[qi];
            const int32_t e_vq = pp.out_edges[qi];
            for (size_t ki = 0; ki < pp.in_nodes.size(); ++ki) {
                int32_t k = pp.in_nodes[ki];
                const int32_t e_kv = pp.in_edges[ki];
                int32_t e_kq = out[k].find(q);
                if (e_kq < 0) {
                    Support r = P.edges[e_vq].rows, c = P.edges[e_kv].cols;
                    e_kq = add_edge(k, q, std::move(r), std::move(c), EO_FILL);
                    cs.new_edges.push_back(e_kq);
                } else {                       // no edge is added here: references stay valid
                    PEdge& T = P.edges[e_kq];
                    T.rows.unite(P.edges[e_vq].rows);
                    T.cols.unite(P.edges[e_kv].cols);
                }
                pp.pair_in.push_back((int32_t)ki);
                pp.pair_out.push_back((int32_t)qi);
                pp.pair_edge.push_back(e_kq);
            }
        }
        P.n_pairs += (int64_t)pp.pair_edge.size();
        // freeze: remove v from the active graph
        std::vector<int32_t> es;
        for (auto& e : out[v].v) es.push_back(e.second);
        for (auto& e : in[v].v) if (e.first != v) es.push_back(e.second);
        for (int32_t e : es) drop_edge(e);
        P.nodes[v].elim = elim_counter++;
        P.elim_nodes.push_back(v);
    }
};

// fn(t, nt) on nt host threads (t = 0 on the calling thread)
template <class Fn>
void on_threads(int nt, Fn&& fn) {
    if (nt <= 1) { fn(0, 1); return; }
    std::vector<std::thread> th;
    th.reserve((size_t)nt - 1);
    for (int t = 1; t < nt; ++t) th.emplace_back([&fn, t, nt]() { fn(t, nt); });
    fn(0, nt);
    for (auto& x : th) x.join();
}

}  // namespace

std::string build_plan(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                       int32_t depth, const int32_t* perm, const int32_t* leaf_ptr,
                       int32_t order, Plan& P, int nthreads) {
    char msg[256];
    if (n < 1) return "n must be >= 1";
    if (depth < 1 || depth > 30) return "depth must be in [1, 30]";
    const int64_t nleaf = (int64_t)1 << depth;
    if (nleaf > n) return "more leaves than rows (2^depth > n)";
    if (!row_ptr || !col_idx || !perm || !leaf_ptr) return "null CSR or tree array";
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return "row_ptr[0] must be 0 and row_ptr[n] = nnz";
    // the rows in nt ranges; the error of the lowest row is reported
    const int nt = n >= 8192 ? std::max(1, nthreads) : 1;
    {
        std::vector<int32_t> bad_row(nt, -1);
        std::vector<int> bad_kind(nt, 0);
        on_threads(nt, [&](int t, int T) {
            const int32_t r0 = (int32_t)((int64_t)n * t / T), r1 = (int32_t)((int64_t)n * (t + 1) / T);
            for (int32_t r = r0; r < r1; ++r) {
                int kind = 0;
                if (row_ptr[r + 1] < row_ptr[r]) kind = 1;
                else
                    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
                        const int32_t c = col_idx[e];
                        if (c < 0 || c >= n) { kind = 2; break; }
                        if (e > row_ptr[r] && col_idx[e - 1] >= c) { kind = 3; break; }
                    }
                if (kind) { bad_row[t] = r; bad_kind[t] = kind; return; }
            }
        });
        for (int t = 0; t < nt; ++t) {
            if (bad_row[t] < 0) continue;
            if (bad_kind[t] == 1) return "row_ptr is not non-decreasing";
            snprintf(msg, sizeof msg, bad_kind[t] == 2 ? "column index out of range in row %d"
                                                       : "columns not sorted/unique in row %d", bad_row[t]);
            return msg;
        }
    }
    if (order != 0 && order != 1) return "order must be LRX_COLORED or LRX_NATURAL";
    P = Plan();
    P.n = n; P.depth = depth; P.order = order;
    P.perm.assign(perm, perm + n);
    P.leaf_ptr.assign(leaf_ptr, leaf_ptr + nleaf + 1);
    P.pos.assign(n, -1);
    for (int32_t t = 0; t < n; ++t) {
        int32_t r = perm[t];
        if (r < 0 || r >= n || P.pos[r] >= 0) return "perm is not a permutation";
        P.pos[r] = t;
    }
    if (leaf_ptr[0] != 0 || leaf_ptr[nleaf] != n) return "leaf_ptr must start at 0 and end at n";
    for (int64_t c = 0; c < nleaf; ++c)
        if (leaf_ptr[c + 1] <= leaf_ptr[c]) return "leaf clusters must be non-empty";

    Builder B(P);
    // room for the edges and nodes the method creates (about 40 edges and 8
    // nodes per leaf cluster on the workloads here), so the tables are not moved
    P.edges.reserve((size_t)nleaf * 40);
    P.nodes.reserve((size_t)nleaf * 8);
    B.out.reserve((size_t)nleaf * 8);
    B.in.reserve((size_t)nleaf * 8);
    const int32_t l = depth;
    // leaf cluster of each tree position
    std::vector<int32_t> leaf_of(n);
    for (int32_t c = 0; c < nleaf; ++c)
        for (int32_t t = leaf_ptr[c]; t < leaf_ptr[c + 1]; ++t) leaf_of[t] = c;

    // ---- cluster adjacency at every level (Def. "adjacent clusters"), pattern of A and A^T
    {
        // distinct pairs of leaf clusters joined by an entry of A, found cluster
        // by cluster (rows of a cluster are consecutive tree positions)
        std::vector<std::vector<std::pair<int32_t, int32_t>>> lpt(nt);
        on_threads(nt, [&](int th, int T) {
            std::vector<int32_t> seen((size_t)nleaf, -1);
            auto& lp = lpt[th];
            const int32_t a0 = (int32_t)(nleaf * th / T), a1 = (int32_t)(nleaf * (th + 1) / T);
            for (int32_t a = a0; a < a1; ++a) {
                for (int32_t t = leaf_ptr[a]; t < leaf_ptr[a + 1]; ++t) {
                    const int32_t r = perm[t];
                    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
                        const int32_t b = leaf_of[P.pos[col_idx[e]]];
                        if (b == a || seen[b] == a) continue;
                        seen[b] = a;
                        lp.push_back({std::min(a, b), std::max(a, b)});
                    }
                }
            }
        });
        std::vector<std::pair<int32_t, int32_t>> lp;
        for (auto& v : lpt) lp.insert(lp.end(), v.begin(), v.end());
        std::sort(lp.begin(), lp.end());
        lp.erase(std::unique(lp.begin(), lp.end()), lp.end());
        B.cadj.assign(l + 1, {});
        for (int32_t k = 0; k <= l; ++k) {
            int32_t sh = l - k;
            auto& A = B.cadj[k];
            A.assign((size_t)1 << k, {});
            for (auto& pr : lp) {
                int32_t a = pr.first >> sh, b = pr.second >> sh;
                if (a != b) { A[a].push_back(b); A[b].push_back(a); }
            }
            for (auto& v : A) { std::sort(v.begin(), v.end()); v.erase(std::unique(v.begin(), v.end()), v.end()); }
        }
    }

    // ---- leaf super-nodes and their edges from A (Initialize + merge of the leaves)
    const int32_t nsl = (int32_t)(nleaf / 2);
    LevelPlan L0;
    L0.level = l;
    for (int32_t j = 0; j < nsl; ++j) {
        int32_t id = B.add_node(NK_SUPER, l, j);
        PNode& nd = P.nodes[id];
        nd.leaf = true;
        nd.dof0 = leaf_ptr[2 * j];
        nd.static_size = leaf_ptr[2 * j + 2] - leaf_ptr[2 * j];
        L0.supers.push_back(id);
    }
    {
        // blocks of A between leaf super-nodes: for every destination super-node
        // (its rows are consecutive tree positions) the entries of its rows are
        // bucketed by source super-node; rows come out sorted and unique, columns
        // are sorted and deduplicated per block; edges are then created in
        // (source, destination) order
        struct Grp { int32_t src, dst; std::vector<int32_t> rows, cols; };
        std::vector<std::vector<Grp>> grpt(nt);
        on_threads(nt, [&](int th, int T) {
            std::vector<Grp>& grps = grpt[th];
            const int32_t sd0 = (int32_t)((int64_t)nsl * th / T), sd1 = (int32_t)((int64_t)nsl * (th + 1) / T);
            grps.reserve((size_t)(sd1 - sd0) * 12);
            std::vector<int32_t> slot(nsl, -1);           // group of a source for the current destination
            std::vector<int32_t> touched;
            for (int32_t sd = sd0; sd < sd1; ++sd) {
                const PNode& dn = P.nodes[L0.supers[sd]];
                touched.clear();
                for (int32_t lr = 0; lr < dn.static_size; ++lr) {
                    const int32_t r = perm[dn.dof0 + lr];
                    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
                        const int32_t tc = P.pos[col_idx[e]];
                        const int32_t ss = leaf_of[tc] >> 1;
                        int32_t g = slot[ss];
                        if (g < 0) {
                            g = slot[ss] = (int32_t)grps.size();
                            grps.push_back(Grp{ss, sd, {}, {}});
                            touched.push_back(ss);
                        }
                        if (ss == sd) continue;                // the pivot block is full
                        Grp& G = grps[g];
                        if (G.rows.empty() || G.rows.back() != lr) G.rows.push_back(lr);
                        G.cols.push_back(tc - P.nodes[L0.supers[ss]].dof0);
                    }
                }
                for (int32_t ss : touched) {
                    Grp& G = grps[slot[ss]];
                    std::sort(G.cols.begin(), G.cols.end());
                    G.cols.erase(std::unique(G.cols.begin(), G.cols.end()), G.cols.end());
                    slot[ss] = -1;
                }
            }
        });
        std::vector<Grp> grps;
        {
            size_t tot = 0;
            for (auto& v : grpt) tot += v.size();
            grps.reserve(tot);
            for (auto& v : grpt)
                for (auto& g : v) grps.push_back(std::move(g));
        }
        std::vector<int32_t> order_g(grps.size());
        for (size_t g = 0; g < grps.size(); ++g) order_g[g] = (int32_t)g;
        std::sort(order_g.begin(), order_g.end(), [&](int32_t x, int32_t y) {
            return grps[x].src != grps[y].src ? grps[x].src < grps[y].src : grps[x].dst < grps[y].dst;
        });
        for (int32_t g : order_g) {
            Grp& G = grps[g];
            Support rows, cols;
            if (G.src != G.dst) {
                rows.all = false; cols.all = false;
                rows.idx = std::move(G.rows);
                cols.idx = std::move(G.cols);
            }
            int32_t e = B.add_edge(L0.supers[G.src], L0.supers[G.dst], std::move(rows), std::move(cols), EO_INIT);
            P.init_edges.push_back(e);
        }
        // every super-node carries a pivot block even if A has no diagonal there
        for (int32_t j = 0; j < nsl; ++j) {
            int32_t s = L0.supers[j];
            if (B.out[s].find(s) < 0) {
                int32_t e = B.add_edge(s, s, Support(), Support(), EO_INIT);
                P.init_edges.push_back(e);
            }
        }
    }

    std::vector<int32_t> reds_next;      // red nodes of level i-1 created at level i (index = cluster)
    for (int32_t i = l; i >= 1; --i) {
        LevelPlan Lv;
        if (i == l) {
            Lv = std::move(L0);
        } else {
            Lv.level = i;
            const int32_t ns = 1 << (i - 1);
            std::vector<int32_t> owner(P.nodes.size(), -1), half(P.nodes.size(), 0);
            for (int32_t j = 0; j < ns; ++j) {
                int32_t id = B.add_node(NK_SUPER, i, j);
                P.nodes[id].comp0 = reds_next[2 * j];
                P.nodes[id].comp1 = reds_next[2 * j + 1];
                B.empty[id] = B.empty[reds_next[2 * j]] && B.empty[reds_next[2 * j + 1]];
                Lv.supers.push_back(id);
            }
            owner.resize(P.nodes.size(), -1);
            half.resize(P.nodes.size(), 0);
            for (int32_t j = 0; j < ns; ++j) {
                owner[reds_next[2 * j]] = Lv.supers[j];
                owner[reds_next[2 * j + 1]] = Lv.supers[j];
                half[reds_next[2 * j + 1]] = 1;
            }
            // MergeRedNodes (Sec. 4.2): every active edge is between red nodes of level i
            std::vector<int32_t> red_edges;
            for (int32_t r : reds_next)
                for (auto& e : B.out[r].v) red_edges.push_back(e.second);
            for (size_t u = 0; u < P.nodes.size(); ++u) {
                if (owner[u] >= 0) continue;
                if (!B.out[u].v.empty() || !B.in[u].v.empty()) {
                    snprintf(msg, sizeof msg, "internal: unexpected active node at level %d", i);
                    return msg;
                }
            }
            std::sort(red_edges.begin(), red_edges.end());
            for (int32_t e : red_edges) {
                const int32_t esrc = P.edges[e].src, edst = P.edges[e].dst;   // add_edge may move P.edges
                int32_t su = owner[esrc], sv = owner[edst];
                int32_t me = B.out[su].find(sv);
                if (me < 0) {
                    me = B.add_edge(su, sv, Support(), Support(), EO_MERGE);
                    Lv.merge_edges.push_back(me);
                }
                Lv.merges.push_back({e, me, (int8_t)half[edst], (int8_t)half[esrc]});
            }
            for (int32_t e : red_edges) B.drop_edge(e);
            // pivot blocks for super-nodes with no merged self edge
            for (int32_t j = 0; j < ns; ++j) {
                int32_t s = Lv.supers[j];
                if (B.out[s].find(s) < 0) {
                    int32_t me = B.add_edge(s, s, Support(), Support(), EO_MERGE);
                    Lv.merge_edges.push_back(me);
                }
            }
        }
        // order inside the level
        const int32_t ns = 1 << (i - 1);
        std::vector<int32_t> colour(ns, 0);
        int32_t ncol = 0;
        if (order == 0) {
            const auto& A = B.cadj[i - 1];
            std::vector<int32_t> mark(ns, -1);
            for (int32_t j = 0; j < ns; ++j) {
                // colours used within distance 2
                std::vector<int32_t> used;
                for (int32_t a : A[j]) {
                    if (a < j) used.push_back(colour[a]);
                    for (int32_t b : A[a]) if (b != j && b < j) used.push_back(colour[b]);
                }
                std::sort(used.begin(), used.end());
                int32_t c = 0;
                for (int32_t u : used) { if (u == c) ++c; else if (u > c) break; }
                colour[j] = c;
                ncol = std::max(ncol, c + 1);
            }
        } else {
            for (int32_t j = 0; j < ns; ++j) colour[j] = j;
            ncol = ns;
        }
        Lv.colours = ncol;
        Lv.step0 = (int32_t)P.steps.size();
        Lv.nsteps = ncol;
        reds_next.assign((size_t)ns, -1);
        for (int32_t c = 0; c < ncol; ++c) {
            ColourStep cs;
            cs.level = i; cs.colour = c;
            cs.nodes.reserve((size_t)std::count(colour.begin(), colour.end(), c));
            for (int32_t j = 0; j < ns; ++j) {
                if (colour[j] != c) continue;
                NodeStep st;
                st.j = j;
                st.s = Lv.supers[j];
                st.b = B.add_node(NK_BLACK, i, j);
                st.P = B.add_node(NK_RED, i - 1, j);
                reds_next[j] = st.P;
                const int32_t s = st.s;
                // ---- Compress (Sec. 4.3): well-separated neighbours of s
                std::vector<int32_t> nb;
                for (auto& e : B.out[s].v) if (e.first != s) nb.push_back(e.first);
                for (auto& e : B.in[s].v) if (e.first != s) nb.push_back(e.first);
                std::sort(nb.begin(), nb.end());
                nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
                std::vector<int32_t> cand;
                for (int32_t p : nb) {
                    const PNode& pn = P.nodes[p];
                    if (pn.kind == NK_BLACK || pn.elim >= 0) return "internal: black or eliminated neighbour at compression";
                    if (!B.adjacent_or_equal(i - 1, B.cluster_of(p), j)) cand.push_back(p);
                }
                std::sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
                    const PNode& x = P.nodes[a];
                    const PNode& y = P.nodes[b];
                    if (x.kind != y.kind) return x.kind < y.kind;       // red before super
                    return x.idx < y.idx;
                });
                st.gamma = B.full_or_empty(s);
                for (int32_t p : cand) {
                    CandRef cr;
                    cr.p = p;
                    cr.e_sp = B.out[s].find(p);
                    cr.e_ps = B.in[s].find(p);
                    if (cr.e_sp >= 0) st.gamma.unite(P.edges[cr.e_sp].cols);
                    if (cr.e_ps >= 0) st.gamma.unite(P.edges[cr.e_ps].rows);
                    st.cands.push_back(cr);
                }
                if (cand.empty() || B.empty[s]) { B.empty[st.b] = 1; B.empty[st.P] = 1; }
                Lv.candidates += (int64_t)cand.size();
                P.n_candidates += (int64_t)cand.size();
                for (auto& cr : st.cands) {
                    if (cr.e_sp >= 0) B.drop_edge(cr.e_sp);
                    if (cr.e_ps >= 0) B.drop_edge(cr.e_ps);
                }
                for (auto& cr : st.cands) {
                    Support rows = cr.e_sp >= 0 ? P.edges[cr.e_sp].rows : B.full_or_empty(cr.p);
                    cr.e_Pp = B.add_edge(st.P, cr.p, rows, Support(), EO_R);
                    Support cols = cr.e_ps >= 0 ? P.edges[cr.e_ps].cols : B.full_or_empty(cr.p);
                    cr.e_pP = B.add_edge(cr.p, st.P, Support(), cols, EO_QT);
                    cs.new_edges.push_back(cr.e_Pp);
                    cs.new_edges.push_back(cr.e_pP);
                }
                st.e_sb = B.add_edge(s, st.b, Support(), st.gamma, EO_VT);
                st.e_bs = B.add_edge(st.b, s, st.gamma, Support(), EO_V);
                st.e_bP = B.add_edge(st.b, st.P, Support(), Support(), EO_NEGI);
                st.e_Pb = B.add_edge(st.P, st.b, Support(), Support(), EO_NEGI);
                cs.new_edges.push_back(st.e_sb);
                cs.new_edges.push_back(st.e_bs);
                cs.new_edges.push_back(st.e_bP);
                cs.new_edges.push_back(st.e_Pb);
                // ---- Eliminate(s), Eliminate(b) (Sec. 4.4)
                B.eliminate(s, st.ps, cs);
                B.eliminate(st.b, st.pb, cs);
                cs.nodes.push_back(std::move(st));
            }
            P.steps.push_back(std::move(cs));
        }
        P.levels.push_back(std::move(Lv));
    }
    P.root_red = reds_next.empty() ? -1 : reds_next[0];
    // the root red node is never merged; it must carry no edge
    return "";
}

}  // namespace lrx
