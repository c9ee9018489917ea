// Compiler of the solve sweeps into staged node programs (see dev.hpp).
//
// Forward sweep of one super-node (Algorithm 3, SolveL):
//   F_s = S^-1 R_s                    R_s = x[s], the right-hand side after the
//                                     updates of earlier nodes
//   R_b = x[b] - Mat(s->b) F_s        the black node's right-hand side
//   F_b = B^-1 R_b,  x[b] = R_b
//   x[q] -= Mat(s->q) F_s + Mat(b->q) F_b   for every later node q
// Backward sweep (Algorithm 4, SolveU), using the final x of later nodes:
//   Y_b = x[b] - sum_q Mat(q->b) x[q],  x[b] = B^-1 Y_b
//   Y_s = x[s] - sum_q Mat(q->s) x[q] - Mat(b->s) x[b],  x[s] = S^-1 Y_s
// R, F, Y and x[b] of the node live in reserved LDS buffers for the whole
// program; stored blocks and the rows x[q] of other nodes are staged per unit.
#include "sweep.hpp"

#include <algorithm>
#include <cstring>

namespace lrx {
namespace {

constexpr int kHeaderWords = 8, kGroupWords = 4, kRunWords = 10, kCompWords = 12;
constexpr int kGroupReserve = 32;          // groups per stage at most

static_assert(sizeof(SwHeader) == 4 * kHeaderWords, "header layout");
static_assert(sizeof(SwGroup) == 4 * kGroupWords, "group layout");
static_assert(sizeof(SwRun) == 4 * kRunWords, "run layout");
static_assert(sizeof(SwComp) == 4 * kCompWords, "comp layout");

// An LDS offset that is either absolute (reserved buffers) or relative to the
// unit's place in the stage area; v < 0 and !rel means "none".
struct Off {
    int32_t v = -1;
    bool rel = false;
    static Off none() { return {}; }
    static Off abs(int32_t x) { return {x, false}; }
    static Off rel_(int32_t x) { return {x, true}; }
};

struct URun {
    const void* src = nullptr;       // nullptr: rows of x
    int32_t ld = 0, len = 0, nrun = 0, dld = 0, es = 8;
    int map = -1;                    // unit map id
    Off dst;
};

struct UComp {
    int seq = 0;
    Off mat;
    int32_t ld = 0, nr = 0, nc = 0;
    Off in;  int in_map = -1;
    Off init; int init_map = -1;
    Off out; int out_map = -1;
    int32_t gbase = -1; int gmap = -1;
};

struct Unit {
    std::vector<URun> runs;
    std::vector<UComp> comps;
    std::vector<std::vector<int32_t>> maps;
    int32_t area = 0;
    int add_map(std::vector<int32_t> m) {
        if (m.empty()) return -1;
        maps.push_back(std::move(m));
        return (int)maps.size() - 1;
    }
    int32_t words() const {
        int32_t w = (int32_t)(runs.size() * kRunWords + comps.size() * kCompWords);
        for (auto& m : maps) w += (int32_t)m.size();
        return w;
    }
};

inline int32_t odd(int32_t r) { return r | 1; }

// Identity lists are empty; these return explicit lists where needed.
std::vector<int32_t> expand(const std::vector<int32_t>& v, int32_t n) {
    if (!v.empty()) return v;
    std::vector<int32_t> r(n);
    for (int32_t i = 0; i < n; ++i) r[i] = i;
    return r;
}

std::vector<int32_t> slice(const std::vector<int32_t>& v, int32_t a0, int32_t a1) {
    if (v.empty()) {               // identity slice: explicit offsets a0..a1-1
        std::vector<int32_t> r(a1 - a0);
        for (int32_t i = a0; i < a1; ++i) r[i - a0] = i;
        return r;
    }
    return std::vector<int32_t>(v.begin() + a0, v.begin() + a1);
}

bool is_identity(const std::vector<int32_t>& v) {
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i] != (int32_t)i) return false;
    return true;
}

// ------------------------------------------------------------------ stages
struct StageB {
    std::vector<SwRun> runs;
    std::vector<std::pair<int, SwComp>> comps;   // (seq, comp)
    std::vector<int32_t> maps;                   // map section (offsets fixed at close)
    int32_t area = 0;                            // stage-area doubles used
    int32_t elems_mat = 0;
    int32_t words() const {
        return kHeaderWords + kGroupWords * kGroupReserve + (int32_t)runs.size() * kRunWords +
               (int32_t)comps.size() * kCompWords + (int32_t)maps.size();
    }
};

struct NodePacker {
    int32_t base;                    // first double of the stage area
    int32_t cap_area;
    std::vector<StageB> stages;

    bool fits(const StageB& s, const Unit& u) const {
        return s.area + u.area <= cap_area && s.words() + u.words() <= kSwDescWords;
    }

    void place(StageB& s, const Unit& u) {
        const int32_t ub = base + s.area;
        auto resolve = [&](Off o) -> int32_t { return o.v < 0 && !o.rel ? -1 : (o.rel ? ub + o.v : o.v); };
        std::vector<int32_t> moff(u.maps.size());
        for (size_t i = 0; i < u.maps.size(); ++i) {
            moff[i] = (int32_t)s.maps.size();
            s.maps.insert(s.maps.end(), u.maps[i].begin(), u.maps[i].end());
        }
        auto mres = [&](int id) -> int32_t { return id < 0 ? -1 : moff[id]; };
        for (const URun& r : u.runs) {
            SwRun w{};
            w.src = r.src;
            w.ld = r.ld;
            w.len = r.len;
            w.nrun = r.nrun;
            w.map = mres(r.map);
            w.lds = resolve(r.dst);
            w.dld = r.dld;
            w.rlen = r.len > 0 ? 1.0f / (float)r.len : 0.0f;
            w.es = r.es;
            s.runs.push_back(w);
            if (r.src) s.elems_mat += r.len * r.nrun;
        }
        for (const UComp& c : u.comps) {
            SwComp w{};
            w.mat = resolve(c.mat);
            w.ld = c.ld;
            w.nr = c.nr;
            w.nc = c.nc;
            w.in = resolve(c.in);
            w.in_map = mres(c.in_map);
            w.init = resolve(c.init);
            w.init_map = mres(c.init_map);
            w.out = resolve(c.out);
            w.out_map = mres(c.out_map);
            w.gbase = c.gbase;
            w.gmap = mres(c.gmap);
            s.comps.push_back({c.seq, w});
        }
        s.area += u.area;
    }

    bool add(const Unit& u, std::string& err) {
        if (stages.empty()) stages.emplace_back();
        if (!fits(stages.back(), u)) {
            StageB fresh;
            if (!fits(fresh, u)) {
                err = "solve sweep: a unit needs " + std::to_string(u.area) + " doubles / " +
                      std::to_string(u.words()) + " words, more than one stage holds";
                return false;
            }
            stages.push_back(std::move(fresh));
        }
        place(stages.back(), u);
        return true;
    }

    // Serialises the stages into words; returns the node descriptor.  Sets
    // ok = false if a block exceeds the descriptor budget.
    SwNodeRel emit(std::vector<int32_t>& words, bool& ok) const {
        SwNodeRel nd{};
        nd.nstage = (int32_t)stages.size();
        std::vector<std::vector<int32_t>> blocks;
        for (const StageB& s : stages) {
            auto comps = s.comps;
            std::stable_sort(comps.begin(), comps.end(),
                             [](const std::pair<int, SwComp>& a, const std::pair<int, SwComp>& b) {
                                 return a.first < b.first;
                             });
            std::vector<SwGroup> groups;
            for (size_t i = 0; i < comps.size();) {
                size_t j = i;
                SwGroup g{};
                g.comp0 = (int32_t)i;
                while (j < comps.size() && comps[j].first == comps[i].first) {
                    g.rows += comps[j].second.nr;
                    ++j;
                }
                g.ncomp = (int32_t)(j - i);
                int lg = 0;
                while (lg < 4 && (int64_t)g.rows << (lg + 1) <= kSwThreads) ++lg;
                g.lglanes = lg;
                groups.push_back(g);
                i = j;
            }
            SwHeader h{};
            h.nrun = (int32_t)s.runs.size();
            h.elems_mat = s.elems_mat;
            for (const SwRun& r : s.runs)
                if (!r.src) h.xrows += r.nrun;
            h.ngroup = (int32_t)groups.size();
            h.groups = kHeaderWords;
            h.runs = h.groups + kGroupWords * h.ngroup;
            h.comps = h.runs + kRunWords * h.nrun;
            const int32_t maps0 = h.comps + kCompWords * (int32_t)comps.size();
            std::vector<int32_t> blk(maps0 + s.maps.size() + ((maps0 + s.maps.size()) & 1), 0);
            std::memcpy(blk.data() + h.groups, groups.data(), groups.size() * sizeof(SwGroup));
            for (size_t i = 0; i < s.runs.size(); ++i) {
                SwRun r = s.runs[i];
                if (r.map >= 0) r.map += maps0;
                std::memcpy(blk.data() + h.runs + kRunWords * i, &r, sizeof(SwRun));
            }
            for (size_t i = 0; i < comps.size(); ++i) {
                SwComp c = comps[i].second;
                for (int32_t* f : {&c.in_map, &c.init_map, &c.out_map, &c.gmap})
                    if (*f >= 0) *f += maps0;
                std::memcpy(blk.data() + h.comps + kCompWords * i, &c, sizeof(SwComp));
            }
            std::copy(s.maps.begin(), s.maps.end(), blk.begin() + maps0);
            std::memcpy(blk.data(), &h, sizeof(SwHeader));
            if ((int32_t)blk.size() > kSwDescWords) ok = false;
            blocks.push_back(std::move(blk));
        }
        for (size_t i = 0; i + 1 < blocks.size(); ++i) {
            SwHeader h;
            std::memcpy(&h, blocks[i].data(), sizeof h);
            h.words_next = (int32_t)blocks[i + 1].size();
            std::memcpy(blocks[i].data(), &h, sizeof h);
        }
        if (words.size() & 1) words.push_back(0);
        nd.desc = (int64_t)words.size();
        nd.words0 = blocks.empty() ? 0 : (int32_t)blocks[0].size();
        for (auto& b : blocks) words.insert(words.end(), b.begin(), b.end());
        return nd;
    }
};

// ------------------------------------------------------------------ units
inline const void* at(const void* base, int64_t elems, int32_t es) {
    return (const char*)base + elems * es;
}

// Rows [r0, r0 + rc) of a pivot inverse: out = inv[rows, :] * in.
void pivot_units(const SwPivIR& P, int32_t in_abs, int32_t out_abs, bool to_x, int seq, int32_t cap,
                 int32_t es, std::vector<Unit>& units) {
    const int32_t m = P.m;
    int32_t rc = m;
    while (rc > 1 && (int64_t)odd(rc) * m > cap) rc = (rc + 1) / 2;
    for (int32_t r0 = 0; r0 < m; r0 += rc) {
        const int32_t n = std::min(rc, m - r0);
        Unit u;
        URun r;
        r.src = at(P.inv, r0, es);
        r.es = es;
        r.ld = m; r.len = n; r.nrun = m; r.dld = odd(n);
        r.dst = Off::rel_(0);
        u.runs.push_back(r);
        UComp c;
        c.seq = seq;
        c.mat = Off::rel_(0);
        c.ld = odd(n); c.nr = n; c.nc = m;
        c.in = Off::abs(in_abs);
        c.out = out_abs >= 0 ? Off::abs(out_abs + r0 * kSwKS) : Off::none();
        c.gbase = to_x ? (int32_t)(P.off + r0) : -1;
        u.comps.push_back(c);
        u.area = odd(n) * m;
        units.push_back(std::move(u));
    }
}

// An edge whose input and output both live in reserved buffers:
// buf[rows] = buf[rows] - E * in[cols].
void local_edge_units(const SwEdgeIR& E, int32_t in_abs, int32_t buf_abs, int seq, int32_t cap,
                      int32_t es, std::vector<Unit>& units) {
    int32_t rc = E.nr;
    while (rc > 1 && (int64_t)odd(rc) * E.nc > cap) rc = (rc + 1) / 2;
    for (int32_t a0 = 0; a0 < E.nr; a0 += rc) {
        const int32_t n = std::min(rc, E.nr - a0);
        Unit u;
        URun r;
        r.src = at(E.E, a0, es);
        r.es = es;
        r.ld = E.nr; r.len = n; r.nrun = E.nc; r.dld = odd(n);
        r.dst = Off::rel_(0);
        u.runs.push_back(r);
        UComp c;
        c.seq = seq;
        c.mat = Off::rel_(0);
        c.ld = odd(n); c.nr = n; c.nc = E.nc;
        c.in = Off::abs(in_abs);
        c.in_map = E.cols.empty() || is_identity(E.cols) ? -1 : u.add_map(E.cols);
        std::vector<int32_t> rows = slice(E.rows, a0, a0 + n);
        const bool ident = (a0 == 0 && (E.rows.empty() || is_identity(rows)));
        c.init = Off::abs(buf_abs);
        c.out = Off::abs(buf_abs);
        if (ident) {
            c.init_map = c.out_map = -1;
        } else {
            c.init_map = c.out_map = u.add_map(rows);
        }
        u.comps.push_back(c);
        u.area = odd(n) * E.nc;
        units.push_back(std::move(u));
    }
}

// Forward: the later node q receives Mat(s->q) F_s and Mat(b->q) F_b.
void target_units(const SwEdgeIR* Es, const SwEdgeIR* Eb, int32_t fs_abs, int32_t fb_abs,
                  int32_t cap, int32_t es, std::vector<Unit>& units) {
    std::vector<int32_t> U;
    std::vector<int32_t> abs_s, abs_b;
    if (Es) {
        for (int32_t a : expand(Es->rows, Es->nr)) abs_s.push_back((int32_t)(Es->other_off + a));
        U.insert(U.end(), abs_s.begin(), abs_s.end());
    }
    if (Eb) {
        for (int32_t a : expand(Eb->rows, Eb->nr)) abs_b.push_back((int32_t)(Eb->other_off + a));
        U.insert(U.end(), abs_b.begin(), abs_b.end());
    }
    std::sort(U.begin(), U.end());
    U.erase(std::unique(U.begin(), U.end()), U.end());
    auto pos = [&](const std::vector<int32_t>& a) {
        std::vector<int32_t> p(a.size());
        for (size_t i = 0; i < a.size(); ++i)
            p[i] = (int32_t)(std::lower_bound(U.begin(), U.end(), a[i]) - U.begin());
        return p;
    };
    const std::vector<int32_t> ps = pos(abs_s), pb = pos(abs_b);
    const int32_t nU = (int32_t)U.size();
    // row ranges of each edge inside a U-range (positions are increasing)
    auto erange = [](const std::vector<int32_t>& p, int32_t u0, int32_t u1) {
        int32_t e0 = (int32_t)(std::lower_bound(p.begin(), p.end(), u0) - p.begin());
        int32_t e1 = (int32_t)(std::lower_bound(p.begin(), p.end(), u1) - p.begin());
        return std::make_pair(e0, e1);
    };
    auto area_of = [&](int32_t u0, int32_t u1) {
        int64_t a = (int64_t)(u1 - u0) * kSwKS;
        if (Es) { auto r = erange(ps, u0, u1); if (r.second > r.first) a += (int64_t)odd(r.second - r.first) * Es->nc; }
        if (Eb) { auto r = erange(pb, u0, u1); if (r.second > r.first) a += (int64_t)odd(r.second - r.first) * Eb->nc; }
        return a;
    };
    int32_t nchunk = 1;
    for (;; ++nchunk) {
        bool ok = true;
        const int32_t cs = (nU + nchunk - 1) / nchunk;
        for (int32_t u0 = 0; u0 < nU && ok; u0 += cs) ok = area_of(u0, std::min(nU, u0 + cs)) <= cap;
        if (ok || cs == 1) break;
    }
    const int32_t cs = (nU + nchunk - 1) / nchunk;
    for (int32_t u0 = 0; u0 < nU; u0 += cs) {
        const int32_t u1 = std::min(nU, u0 + cs);
        Unit u;
        int32_t fill = 0;
        URun xr;
        xr.len = 0; xr.nrun = u1 - u0; xr.dld = kSwKS;
        xr.map = u.add_map(std::vector<int32_t>(U.begin() + u0, U.begin() + u1));
        xr.dst = Off::rel_(0);
        u.runs.push_back(xr);
        const int gmap = xr.map;
        fill += (u1 - u0) * kSwKS;
        auto edge = [&](const SwEdgeIR* E, const std::vector<int32_t>& p, int32_t f_abs, int seq) {
            if (!E) return;
            auto rg = erange(p, u0, u1);
            const int32_t n = rg.second - rg.first;
            if (n <= 0) return;
            URun r;
            r.src = at(E->E, rg.first, es);
            r.es = es;
            r.ld = E->nr; r.len = n; r.nrun = E->nc; r.dld = odd(n);
            r.dst = Off::rel_(fill);
            u.runs.push_back(r);
            UComp c;
            c.seq = seq;
            c.mat = Off::rel_(fill);
            c.ld = odd(n); c.nr = n; c.nc = E->nc;
            c.in = Off::abs(f_abs);
            c.in_map = E->cols.empty() || is_identity(E->cols) ? -1 : u.add_map(E->cols);
            std::vector<int32_t> loc(n);
            for (int32_t i = 0; i < n; ++i) loc[i] = p[rg.first + i] - u0;
            c.init = Off::rel_(0);
            c.out = Off::rel_(0);
            c.init_map = c.out_map = is_identity(loc) && n == u1 - u0 ? -1 : u.add_map(loc);
            u.comps.push_back(c);
            fill += odd(n) * E->nc;
        };
        edge(Es, ps, fs_abs, 3);
        edge(Eb, pb, fb_abs, 4);
        UComp st;                       // x[U] = T
        st.seq = 5;
        st.nr = u1 - u0; st.nc = 0; st.ld = 1;
        st.in = Off::none();
        st.init = Off::rel_(0);
        st.gmap = gmap;
        u.comps.push_back(st);
        u.area = fill;
        units.push_back(std::move(u));
    }
}

// Backward: rows of the pivot's buffer receive -Mat(q->v) x[q] for one source q.
struct RoundSet {
    std::vector<std::vector<char>> used;   // per round, per buffer row
    int32_t n;
    explicit RoundSet(int32_t rows) : n(rows) {}
    int assign(const std::vector<int32_t>& rows) {
        for (size_t r = 0;; ++r) {
            if (r == used.size()) used.emplace_back(n, 0);
            bool ok = true;
            for (int32_t a : rows) if (used[r][a]) { ok = false; break; }
            if (ok) {
                for (int32_t a : rows) used[r][a] = 1;
                return (int)r;
            }
        }
    }
};

struct SrcEdge {
    const SwEdgeIR* E;
    int32_t buf_abs;
    int seq;
};

void source_units(const std::vector<SrcEdge>& es, int32_t cap, int32_t esz, std::vector<Unit>& units) {
    // columns of all edges of this source, as absolute rows of x
    std::vector<int32_t> U;
    std::vector<std::vector<int32_t>> absc(es.size());
    for (size_t i = 0; i < es.size(); ++i) {
        for (int32_t t : expand(es[i].E->cols, es[i].E->nc)) absc[i].push_back((int32_t)(es[i].E->other_off + t));
        U.insert(U.end(), absc[i].begin(), absc[i].end());
    }
    std::sort(U.begin(), U.end());
    U.erase(std::unique(U.begin(), U.end()), U.end());
    int64_t total = (int64_t)U.size() * kSwKS;
    for (auto& e : es) total += (int64_t)odd(e.E->nr) * e.E->nc;
    auto make = [&](const std::vector<int32_t>& Uu, const std::vector<std::pair<size_t, std::pair<int32_t, int32_t>>>& parts) {
        Unit u;
        URun xr;
        xr.len = 0; xr.nrun = (int32_t)Uu.size(); xr.dld = kSwKS;
        xr.map = u.add_map(Uu);
        xr.dst = Off::rel_(0);
        u.runs.push_back(xr);
        int32_t fill = (int32_t)Uu.size() * kSwKS;
        for (auto& pr : parts) {
            const SrcEdge& se = es[pr.first];
            const SwEdgeIR& E = *se.E;
            const int32_t a0 = pr.second.first, n = pr.second.second - a0;
            URun r;
            r.src = at(E.E, a0, esz);
            r.es = esz;
            r.ld = E.nr; r.len = n; r.nrun = E.nc; r.dld = odd(n);
            r.dst = Off::rel_(fill);
            u.runs.push_back(r);
            UComp c;
            c.seq = se.seq;
            c.mat = Off::rel_(fill);
            c.ld = odd(n); c.nr = n; c.nc = E.nc;
            c.in = Off::rel_(0);
            std::vector<int32_t> cp(E.nc);
            for (int32_t t = 0; t < E.nc; ++t)
                cp[t] = (int32_t)(std::lower_bound(Uu.begin(), Uu.end(), absc[pr.first][t]) - Uu.begin());
            c.in_map = is_identity(cp) ? -1 : u.add_map(cp);
            std::vector<int32_t> rows = slice(E.rows, a0, a0 + n);
            c.init = Off::abs(se.buf_abs);
            c.out = Off::abs(se.buf_abs);
            c.init_map = c.out_map = (a0 == 0 && is_identity(rows)) ? -1 : u.add_map(rows);
            u.comps.push_back(c);
            fill += odd(n) * E.nc;
        }
        u.area = fill;
        units.push_back(std::move(u));
    };
    if (total <= cap) {
        std::vector<std::pair<size_t, std::pair<int32_t, int32_t>>> parts;
        for (size_t i = 0; i < es.size(); ++i) parts.push_back({i, {0, es[i].E->nr}});
        make(U, parts);
        return;
    }
    for (size_t i = 0; i < es.size(); ++i) {       // one unit per edge, rows split as needed
        std::vector<int32_t> Ui = absc[i];
        std::sort(Ui.begin(), Ui.end());
        Ui.erase(std::unique(Ui.begin(), Ui.end()), Ui.end());
        const SwEdgeIR& E = *es[i].E;
        const int64_t xa = (int64_t)Ui.size() * kSwKS;
        int32_t rc = E.nr;
        while (rc > 1 && xa + (int64_t)odd(rc) * E.nc > cap) rc = (rc + 1) / 2;
        for (int32_t a0 = 0; a0 < E.nr; a0 += rc)
            make(Ui, {{i, {a0, std::min(E.nr, a0 + rc)}}});
    }
}

bool edge_nonempty(const SwEdgeIR& e) { return e.E && e.nr > 0 && e.nc > 0; }

bool build_fwd(const SwNodeIR& N, std::vector<int32_t>& words, SwNodeRel& out, std::string& err) {
    const SwPivIR& S = N.s;
    const SwPivIR& B = N.b;
    const int32_t ms = S.m, r = B.m;
    // reserved: R_s, F_s, R_b, F_b
    const int32_t oRs = 0, oFs = oRs + ms * kSwKS, oRb = oFs + ms * kSwKS, oFb = oRb + r * kSwKS;
    const int32_t res = oFb + r * kSwKS;
    NodePacker pk{res, kSwData - res, {}};
    bool ok = true;
    if (ms == 0) { out = pk.emit(words, ok); return true; }
    if (pk.cap_area < 1024) { err = "solve sweep: pivot too large for LDS"; return false; }
    std::vector<Unit> units;
    {
        Unit u;                                     // R_s = x[s], R_b = x[b]
        URun a;
        a.len = 0; a.nrun = ms; a.ld = (int32_t)S.off; a.dld = kSwKS; a.dst = Off::abs(oRs);
        u.runs.push_back(a);
        if (r > 0) {
            URun b;
            b.len = 0; b.nrun = r; b.ld = (int32_t)B.off; b.dld = kSwKS; b.dst = Off::abs(oRb);
            u.runs.push_back(b);
        }
        units.push_back(std::move(u));
    }
    pivot_units(S, oRs, oFs, false, 0, pk.cap_area, N.es_piv, units);
    const SwEdgeIR* sb = nullptr;
    for (const SwEdgeIR& e : S.out)
        if (e.other == B.node && edge_nonempty(e)) sb = &e;
    if (r > 0) {
        if (sb) local_edge_units(*sb, oFs, oRb, 1, pk.cap_area, N.es, units);
        pivot_units(B, oRb, oFb, false, 2, pk.cap_area, N.es_piv, units);
        Unit u;                                     // x[b] = R_b
        UComp st;
        st.seq = 2; st.nr = r; st.nc = 0; st.ld = 1;
        st.init = Off::abs(oRb);
        st.gbase = (int32_t)B.off;
        u.comps.push_back(st);
        units.push_back(std::move(u));
    }
    // targets: pair the out-edges of s and b by target node
    std::vector<int32_t> tg;
    for (const SwEdgeIR& e : S.out) if (edge_nonempty(e) && e.other != B.node) tg.push_back(e.other);
    if (r > 0) for (const SwEdgeIR& e : B.out) if (edge_nonempty(e)) tg.push_back(e.other);
    std::sort(tg.begin(), tg.end());
    tg.erase(std::unique(tg.begin(), tg.end()), tg.end());
    for (int32_t q : tg) {
        const SwEdgeIR* es = nullptr;
        const SwEdgeIR* eb = nullptr;
        for (const SwEdgeIR& e : S.out) if (e.other == q && edge_nonempty(e)) es = &e;
        if (r > 0) for (const SwEdgeIR& e : B.out) if (e.other == q && edge_nonempty(e)) eb = &e;
        target_units(es, eb, oFs, oFb, pk.cap_area, N.es, units);
    }
    for (const Unit& u : units)
        if (!pk.add(u, err)) return false;
    out = pk.emit(words, ok);
    if (!ok) err = "solve sweep: descriptor block too large";
    return ok;
}

bool build_bwd(const SwNodeIR& N, std::vector<int32_t>& words, SwNodeRel& out, std::string& err) {
    const SwPivIR& S = N.s;
    const SwPivIR& B = N.b;
    const int32_t ms = S.m, r = B.m;
    // reserved: Y_b, Y_s, X_b
    const int32_t oYb = 0, oYs = oYb + r * kSwKS, oXb = oYs + ms * kSwKS;
    const int32_t res = oXb + r * kSwKS;
    NodePacker pk{res, kSwData - res, {}};
    bool ok = true;
    if (ms == 0) { out = pk.emit(words, ok); return true; }
    if (pk.cap_area < 1024) { err = "solve sweep: pivot too large for LDS"; return false; }
    std::vector<Unit> units;
    {
        Unit u;                                     // Y_b = x[b], Y_s = x[s]
        if (r > 0) {
            URun b;
            b.len = 0; b.nrun = r; b.ld = (int32_t)B.off; b.dld = kSwKS; b.dst = Off::abs(oYb);
            u.runs.push_back(b);
        }
        URun a;
        a.len = 0; a.nrun = ms; a.ld = (int32_t)S.off; a.dld = kSwKS; a.dst = Off::abs(oYs);
        u.runs.push_back(a);
        units.push_back(std::move(u));
    }
    // in-edges from later nodes, grouped by source; rounds keep the rows that
    // one group updates disjoint
    RoundSet rb(std::max(r, 1)), rs(ms);
    const SwEdgeIR* bs = nullptr;
    std::vector<int32_t> srcs;
    for (const SwEdgeIR& e : S.in) {
        if (!edge_nonempty(e)) continue;
        if (e.other == B.node) { bs = &e; continue; }
        srcs.push_back(e.other);
    }
    if (r > 0) for (const SwEdgeIR& e : B.in) if (edge_nonempty(e)) srcs.push_back(e.other);
    std::sort(srcs.begin(), srcs.end());
    srcs.erase(std::unique(srcs.begin(), srcs.end()), srcs.end());
    struct Pending { std::vector<SrcEdge> es; };
    std::vector<Pending> pend;
    int nround = 0;
    for (int32_t q : srcs) {
        Pending p;
        if (r > 0)
            for (const SwEdgeIR& e : B.in)
                if (e.other == q && edge_nonempty(e)) {
                    const int rd = rb.assign(expand(e.rows, e.nr));
                    p.es.push_back({&e, oYb, rd});
                    nround = std::max(nround, rd + 1);
                }
        for (const SwEdgeIR& e : S.in)
            if (e.other == q && edge_nonempty(e)) {
                const int rd = rs.assign(expand(e.rows, e.nr));
                p.es.push_back({&e, oYs, rd});
                nround = std::max(nround, rd + 1);
            }
        pend.push_back(std::move(p));
    }
    for (auto& p : pend) source_units(p.es, pk.cap_area, N.es, units);
    if (r > 0) {
        pivot_units(B, oYb, oXb, true, nround, pk.cap_area, N.es_piv, units);
        if (bs) local_edge_units(*bs, oXb, oYs, nround + 1, pk.cap_area, N.es, units);
    }
    pivot_units(S, oYs, -1, true, nround + 2, pk.cap_area, N.es_piv, units);
    for (const Unit& u : units)
        if (!pk.add(u, err)) return false;
    out = pk.emit(words, ok);
    if (!ok) err = "solve sweep: descriptor block too large";
    return ok;
}

}  // namespace

bool build_node_programs(const SwNodeIR& N, std::vector<int32_t>& words, SwNodeRel& fwd, SwNodeRel& bwd,
                         std::string& err) {
    return build_fwd(N, words, fwd, err) && build_bwd(N, words, bwd, err);
}

bool build_sweep_program(const std::vector<std::vector<SwNodeIR>>& steps, SwProgram& out,
                         std::string& err) {
    out = SwProgram{};
    for (const auto& st : steps) {
        out.step0.push_back((int32_t)out.fwd.size());
        for (const SwNodeIR& N : st) {
            SwNodeRel f{}, b{};
            if (!build_fwd(N, out.words, f, err)) return false;
            if (!build_bwd(N, out.words, b, err)) return false;
            out.fwd.push_back(f);
            out.bwd.push_back(b);
            out.max_stages = std::max<int64_t>(out.max_stages, std::max(f.nstage, b.nstage));
            out.total_stages += f.nstage + b.nstage;
        }
    }
    out.step0.push_back((int32_t)out.fwd.size());
    return true;
}

}  // namespace lrx
