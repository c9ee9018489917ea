// C ABI of liblorax.so: validation, handle registry, numeric driver of the
// factorization (Algorithm 1), solve program (Algorithms 2-4) and GMRES.
#include "lorax.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <thread>
#include <set>
#include <string>
#include <vector>

#include "dev.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "sweep.hpp"

using namespace lrx;

namespace {

thread_local std::string g_err;

struct Fail {
    lrx_status st;
    std::string msg;
};

[[noreturn]] void fail(lrx_status st, const std::string& m) { throw Fail{st, m}; }

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            fail(e_ == hipErrorOutOfMemory ? LRX_ENOMEM : LRX_EDEVICE,                    \
                 std::string(#expr) + ": " + hipGetErrorString(e_));                      \
    } while (0)

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Device-wide synchronizations and frees (which synchronize) wait while a
// thread captures a HIP graph on one of its streams: a synchronization that
// reached a capturing stream would break the capture.
std::shared_mutex g_capture_mu;
bool device_sync() {
    std::shared_lock<std::shared_mutex> lk(g_capture_mu);
    return hipDeviceSynchronize() == hipSuccess;
}
void free_dev(void* q) {
    std::shared_lock<std::shared_mutex> lk(g_capture_mu);
    (void)hipFree(q);
}
void free_pin(void* q) {
    std::shared_lock<std::shared_mutex> lk(g_capture_mu);
    (void)hipHostFree(q);
}
// Synchronous copies run on the null stream, which the runtime refuses while a
// blocking stream captures (the serving scheduler factors in one thread while
// another captures its solve graph): they wait for the capture as well.
hipError_t copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    std::shared_lock<std::shared_mutex> lk(g_capture_mu);
    return hipMemcpy(dst, src, bytes, kind);
}

// --------------------------------------------------------------- device memory
// Device and pinned host blocks the library releases are kept for reuse: one
// factorization with its solve takes and releases a few dozen blocks, and
// hipMalloc / hipFree of large blocks cost tens of microseconds each.  A
// released block enters the cache only after a device-wide synchronization (as
// hipFree synchronizes), so no queued kernel or copy still uses it when it is
// handed out again.  Sizes are rounded up (64 KiB steps to 1 MiB, then eighths
// of an octave) so that blocks fit again; at most kCacheBytes per device and
// kPinCacheBytes of pinned host memory are kept, and a device's cache is
// emptied when hipMalloc reports out of memory.
constexpr size_t kCacheBytes = (size_t)8 << 30;
constexpr size_t kPinCacheBytes = (size_t)1 << 30;
std::mutex g_cache_mu;
std::map<std::pair<int, size_t>, std::vector<void*>> g_dev_cache;   // (device, bytes) -> blocks
std::map<int, size_t> g_dev_cached;
std::map<size_t, std::vector<void*>> g_pin_cache;
size_t g_pin_cached = 0;

size_t block_class(size_t b) {
    const size_t step = (size_t)1 << 16;
    if (b <= ((size_t)1 << 20)) return std::max(step, (b + step - 1) & ~(step - 1));
    const int k = 63 - __builtin_clzll((unsigned long long)b);
    const size_t q = (size_t)1 << (k - 3);
    return (b + q - 1) / q * q;
}

void cache_flush_device(int dev) {
    std::vector<void*> ps;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (auto it = g_dev_cache.begin(); it != g_dev_cache.end();) {
            if (it->first.first != dev) { ++it; continue; }
            ps.insert(ps.end(), it->second.begin(), it->second.end());
            it = g_dev_cache.erase(it);
        }
        g_dev_cached[dev] = 0;
    }
    for (void* q : ps) free_dev(q);
}

void* dev_alloc(size_t b, size_t& got, int& dev) {
    HIPCHK(hipGetDevice(&dev));
    const size_t c = block_class(b);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_dev_cache.find({dev, c});
        if (it != g_dev_cache.end() && !it->second.empty()) {
            void* q = it->second.back();
            it->second.pop_back();
            g_dev_cached[dev] -= c;
            got = c;
            return q;
        }
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, c);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        cache_flush_device(dev);
        e = hipMalloc(&q, c);
    }
    if (e != hipSuccess)
        fail(e == hipErrorOutOfMemory ? LRX_ENOMEM : LRX_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    got = c;
    return q;
}

// Inside an IdleScope this thread has synchronized the device once and
// releases only blocks that no queued work uses, so releases skip their own
// synchronization.
thread_local int t_idle = 0;
struct IdleScope {
    bool ok;
    IdleScope() : ok(device_sync()) { if (ok) ++t_idle; }
    ~IdleScope() { if (ok) --t_idle; }
    IdleScope(const IdleScope&) = delete;
    IdleScope& operator=(const IdleScope&) = delete;
};

void dev_release(void* q, size_t c, int dev) {
    if (!q) return;
    int cur = dev;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    bool keep = false;
    if ((t_idle > 0 && cur == dev) || device_sync()) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (g_dev_cached[dev] + c <= kCacheBytes) {
            g_dev_cache[{dev, c}].push_back(q);
            g_dev_cached[dev] += c;
            keep = true;
        }
    }
    if (!keep) free_dev(q);
    if (cur != dev) (void)hipSetDevice(cur);
}

void* pin_alloc(size_t b, size_t& got) {
    const size_t c = block_class(b);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_pin_cache.find(c);
        if (it != g_pin_cache.end() && !it->second.empty()) {
            void* q = it->second.back();
            it->second.pop_back();
            g_pin_cached -= c;
            got = c;
            return q;
        }
    }
    void* q = nullptr;
    HIPCHK(hipHostMalloc(&q, c, hipHostMallocDefault));
    got = c;
    return q;
}

void pin_release(void* q, size_t c) {          // copies from or to it may be queued on the current device
    if (!q) return;
    bool keep = false;
    if (t_idle > 0 || device_sync()) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (g_pin_cached + c <= kPinCacheBytes) {
            g_pin_cache[c].push_back(q);
            g_pin_cached += c;
            keep = true;
        }
    }
    if (!keep) free_pin(q);
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int dev = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) dev_release(p, bytes, dev);
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t b) {          // grows; contents are not preserved
        if (b <= bytes) return;
        release();
        size_t got = 0;
        p = dev_alloc(std::max(b, (size_t)4096), got, dev);
        bytes = got;
    }
    template <class T> T* as() const { return (T*)p; }
};

struct PinBuf {
    void* p = nullptr;
    size_t bytes = 0;
    PinBuf() = default;
    PinBuf(const PinBuf&) = delete;
    PinBuf& operator=(const PinBuf&) = delete;
    ~PinBuf() { release(); }
    void release() {
        pin_release(p, bytes);
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t b) {          // caller guarantees no copy from it is in flight
        if (b <= bytes) return;
        release();
        size_t got = 0;
        p = pin_alloc(std::max(b * 2, (size_t)1 << 16), got);
        bytes = got;
    }
};

// Chunked bump allocator for the stored blocks of the factorization.
struct Arena {
    std::vector<std::pair<double*, size_t>> chunks;   // pointer, capacity (doubles)
    size_t used = 0;                                  // in the last chunk
    int64_t total = 0;                                // doubles handed out
    int64_t budget_bytes = 0;
    int dev = 0;
    ~Arena() { release(); }
    void release() {
        for (auto& c : chunks) dev_release(c.first, c.second * sizeof(double), dev);
        chunks.clear();
        used = 0;
        total = 0;
    }
    double* alloc(size_t n) {
        n = (n + 31) & ~(size_t)31;                   // 256-byte aligned blocks
        if (chunks.empty() || used + n > chunks.back().second) {
            // chunks grow with the storage so far (4 MiB .. 256 MiB), so a small
            // factorization holds little more than it uses
            const size_t grow = std::min(std::max((size_t)total, (size_t)1 << 19), (size_t)32 << 20);
            size_t cap = std::max(n, grow);
            size_t got = 0;
            double* p = (double*)dev_alloc(cap * sizeof(double), got, dev);
            chunks.push_back({p, got / sizeof(double)});
            used = 0;
        }
        double* p = chunks.back().first + used;
        used += n;
        total += (int64_t)n;
        if (budget_bytes > 0 && total * 8 > budget_bytes)
            fail(LRX_ENOMEM, "factor storage exceeds hbm_budget_bytes");
        return p;
    }
};

template <class T> size_t append_bytes(std::vector<char>& buf, const std::vector<T>& v) {
    size_t off = (buf.size() + 255) & ~(size_t)255;
    buf.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

// per-pivot static maps (offsets into the factor's int table)
struct PivMaps {
    std::vector<int32_t> in_rmap, out_cmap, pair_rpos, pair_cpos;
};
struct NodeMaps {
    std::vector<int32_t> a_map, b_map;   // stack pieces: A_k columns, B_k rows -> gamma
    std::vector<int32_t> ra_map, qb_map; // R_k rows / Q_k^T columns -> their final blocks
    PivMaps ps, pb;
};

struct SolveStep {
    int32_t node0 = 0, nnode = 0;
    int32_t height = 0, colour = 0;         // level above the leaves, colour inside the level
    int64_t bytes_fwd = 0, bytes_bwd = 0;   // algorithmic bytes of one launch (one right-hand side)
};

// Two library streams (with a fork and two join events) per host thread and
// device, on which independent compress variants of one colour step run beside
// the caller's stream; they are kept until the process ends.  Null if they
// cannot be made (then all runs on one stream).
struct AuxStreams {
    bool made = false;
    hipStream_t s[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
};
thread_local std::vector<AuxStreams> t_aux;

AuxStreams* aux_streams() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    if ((int)t_aux.size() <= dev) t_aux.resize(dev + 1);
    AuxStreams& a = t_aux[dev];
    if (!a.made) {
        for (int k = 0; k < 2; ++k) {
            if (!a.s[k] && hipStreamCreateWithFlags(&a.s[k], hipStreamNonBlocking) != hipSuccess) {
                a.s[k] = nullptr;
                return nullptr;
            }
            if (!a.join[k] && hipEventCreateWithFlags(&a.join[k], hipEventDisableTiming) != hipSuccess) {
                a.join[k] = nullptr;
                return nullptr;
            }
        }
        if (!a.fork && hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) != hipSuccess) {
            a.fork = nullptr;
            return nullptr;
        }
        a.made = true;
    }
    return &a;
}

// Optional event timing of every launch, by kernel class (lrx_timing_*).
struct TimedLaunch {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
};
std::mutex g_tmu;
uint32_t g_timing = 0;                 // bit mask of timed kernel classes
std::vector<TimedLaunch> g_pending;
std::vector<hipEvent_t> g_event_pool;
lrx_timing_t g_acc{};

hipEvent_t take_event() {
    if (!g_event_pool.empty()) { hipEvent_t e = g_event_pool.back(); g_event_pool.pop_back(); return e; }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events when timing is on.
struct LaunchTimer {
    TimedLaunch t{};
    bool on = false;
    hipStream_t st;
    LaunchTimer(int cls, hipStream_t s, double bytes, double flops) : st(s) {
        if (cls < 0) return;                     // untimed launch
        std::lock_guard<std::mutex> lk(g_tmu);
        if (!(g_timing & (1u << cls))) return;
        t.cls = cls; t.bytes = bytes; t.flops = flops;
        t.a = take_event(); t.b = take_event();
        if (!t.a || !t.b) return;
        on = hipEventRecord(t.a, st) == hipSuccess;
    }
    ~LaunchTimer() {
        if (!on) return;
        (void)hipEventRecord(t.b, st);
        std::lock_guard<std::mutex> lk(g_tmu);
        g_pending.push_back(t);
    }
};

void resolve_timing() {                  // caller holds g_tmu
    for (auto& t : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            lrx_kernel_time& k = g_acc.k[t.cls];
            k.launches += 1;
            k.total_ms += ms;
            k.bytes += t.bytes;
            k.flops += t.flops;
        }
        g_event_pool.push_back(t.a);
        g_event_pool.push_back(t.b);
    }
    g_pending.clear();
}

}  // namespace

namespace {
// Tunable launch shapes (lrx_tune_set; defaults measured on MI355X).
struct Tune {
    int32_t gemm_kc = 128;          // K chunk of the MFMA products (multiple of 16, <= 256)
    int32_t gemm_f64_valu = 0;      // 1: FP64 products on the VALU tile kernel instead of MFMA
    int32_t sweep_nk_max = 4;       // right-hand sides per sweep work-group (1, 2 or 4)
    int32_t compress_nt_small = 1024;   // threads per stacked block of at most 32 columns
    int32_t compress_nt_mid = 1024;     // threads per stacked block of 33..64 columns
    int32_t gemm_grid = 0;          // persistent grid of the MFMA products (0: a work-group per tile)
    int32_t solve_graph = 1;        // 1: GMRES replays its preconditioner as a captured HIP graph
    int32_t compress_gram = 1;      // 1: mixed-precision compression through the FP64 Gram matrix
    int32_t large_split_c = 128;    // wider blocks take the split (multi-work-group) back end
};
Tune g_tune;
}  // namespace

struct lrx_handle_s {
    uint64_t magic = 0x6c72786861646c65ull;
    Plan plan;
    hipStream_t stream = nullptr;
    int device = 0;
    double epsilon = 0;
    int32_t compress = LRX_SVD;
    int32_t rule = LRX_RULE_CUTOFF1;
    bool symmetric = false;        // half stack of the symmetric case (Sec. 4.3)
    std::vector<int32_t> size;     // per node
    std::vector<double*> eptr;     // per edge
    std::vector<int64_t> var_off;  // per node
    int64_t n_ext = 0;
    Arena arena;
    // solve program (staged node programs of both sweeps)
    DevBuf d_swnodes, d_swprog;
    std::vector<SwNode> sw_host;   // host copy of d_swnodes (forward nodes, then backward)
    DevBuf batch_nodes;            // node lists of batched solves led by this handle
    int32_t sw_nnode = 0;
    int64_t sw_stages = 0, sw_words = 0;
    std::vector<SolveStep> ssteps;
    DevBuf d_perm;
    DevBuf d_rp, d_ci, d_val;      // A in tree order
    int64_t nnz = 0;
    // scratch
    DevBuf x_ext, ws_b, ws_w;      // solve vector; factor workspaces (released after the factorization)
    DevBuf g_basis, g_z, g_w, g_r, g_b, g_x;
    DevBuf kry_tab, kry_small, kry_part;   // batched GMRES led by this handle
    PinBuf kry_pin;
    // stats
    lrx_stats_t stats{};
    std::vector<int32_t> ranks, rank_level, rank_j;
    std::vector<int32_t> comp_rows, comp_cols;   // stored stacked rows M and columns c per compression
    // last GMRES call: per right-hand side, the relative residual at each restart
    // (true residual) and after each Arnoldi step (estimate |g_{j+1}| / ||b||)
    std::vector<std::vector<double>> gmres_hist;
    std::vector<double> tails;          // per compression: |R11|, ||R22||_F for k = 0..r
    std::vector<int64_t> tail_off;
    double max_tail_ratio = 0.0;
    double t_sync_ms = 0.0, t_solve_prog_ms = 0.0;
    int32_t precision = LRX_FP64;
    bool solve_fp32 = false;       // the solve reads FP32 copies of the stored blocks
    Arena arena32;                 // those copies (mixed precision)
};

namespace {

std::mutex g_reg_mu;
std::set<lrx_handle> g_live;

void check_handle(lrx_handle h) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    if (!h || !g_live.count(h)) fail(LRX_EINVAL, "invalid or freed handle");
}

int32_t dim_of(const Support& s, int32_t full) { return s.count(full); }

void check_csr(const lrx_csr* A) {
    if (!A) fail(LRX_EINVAL, "A is NULL");
    if (A->n < 1 || A->nnz < 0) fail(LRX_EINVAL, "bad n or nnz");
    if (!A->row_ptr || !A->col_idx || (!A->val && A->nnz > 0)) fail(LRX_EINVAL, "null CSR array");
    for (int64_t e = 0; e < A->nnz; ++e)
        if (!std::isfinite(A->val[e])) fail(LRX_EINVAL, "non-finite value in A");
}

void ensure_gfx950(int dev) {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        fail(LRX_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
}

// ------------------------------------------------------------------ work accounting
// Algorithmic flops of one compression (counted from the actual sizes, ranks and
// Jacobi sweeps): Householder QR of the M x c stacked block, 2 M c^2 - 2/3 c^3
// (or 2 c M^2 - 2/3 M^3 when M < c); for the SVD the QR-preconditioned Jacobi of
// the c x c triangle: a column-pivoted QR, an LQ and the explicit Q2 (4/3 c^3
// each), then per sweep c (c - 1) / 2 pairs of 3 dot products and 2 rotations
// of length c (18 c flops a pair); for RRQR the row-pivoted QR stopped at rank
// r, 4 M c r.  The projection B V (2 M c r) is counted with its own launches.
double qr_flops(double M, double c) {
    return M >= c ? 2.0 * M * c * c - 2.0 / 3.0 * c * c * c : 2.0 * c * M * M - 2.0 / 3.0 * M * M * M;
}
double svd_pre_flops(double c) { return 4.0 * c * c * c; }
double jacobi_flops(double c, double sweeps) { return sweeps * 9.0 * c * c * (c - 1.0); }

// Adds work to a kernel class's timing totals without a launch (work known only
// after the kernels ran, such as Jacobi sweeps and ranks).
void timing_add(int cls, double bytes, double flops) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (g_timing & (1u << cls)) {
        g_acc.k[cls].bytes += bytes;
        g_acc.k[cls].flops += flops;
    }
}

// ------------------------------------------------------------------ factor driver
// State of one factorization in the level loop.  The driver below advances one
// or several factorizations in lock-step over (height above the leaves,
// colour): super-nodes of one colour are independent (Thm. "preservation of sparsity",
// Sec. 5) and distinct
// systems share nothing, so every participating factorization's tasks of a step
// go into one launch per kernel.  Each task's arithmetic depends on its own
// operands only, so a factorization in a batch equals the same factorization
// alone.
struct NodeBatch {
    std::vector<DPrep> prep_s, prep_b;
    std::vector<DProj> projs;                 // RRQR: copies of rows of the transformed block
    std::vector<DGemm> gp;                    // SVD: the pieces of B V as products
    std::vector<DGemm> g1s, g2s, g1b, g2b;
    int max_ms = 1, max_mb = 1;
    int64_t pf_s = 0, pf_b = 0, gf_p = 0, gf_s = 0, gf_b = 0;
};

struct FactorRun {
    lrx_handle h;
    Plan& P;
    std::vector<int32_t> imap;             // static index maps of this factorization
    int32_t imap_base = 0;                 // its offset in the batch table
    std::vector<std::vector<NodeMaps>> maps;
    std::vector<int32_t> level_at_height;  // plan level index per height (-1: none)
    int32_t info_base = 0, info_count = 0, info_next = 0;
    bool fp32_compress = false;
    bool frob = false;                     // truncation by eqn. curOff6
    DevBuf d_norm;                         // curOff6: N^2, tau, N per level (33), partial sums
    size_t merge0 = 0, merge1 = 0;         // this run's pieces in the height's merge list
    int64_t flops = 0;
    double fl_compress = 0, fl_pivot = 0, fl_schur = 0, fl_project = 0;   // by operation class
    double jac_flops = 0.0, jac_sweeps = 0.0;   // Jacobi work of the current step (timing)
    double v_bytes = 0.0;                       // bytes of V written in the current step (timing)
    double jac_flops_g = 0.0, v_bytes_g = 0.0;  // the same for the Gram-path tasks (their own class)
    DevBuf d_idx, d_val;                   // temporaries of the initial scatter
    // current colour step
    int32_t si = -1;
    std::vector<DCompress> ct;
    std::vector<DPiece> pieces;
    std::vector<std::vector<int32_t>> a_row0, b_row0;
    std::vector<size_t> wsB, wsV, wsH, tail_at;
    std::vector<size_t> wsR;               // randomized compression: sketch task workspace (0: none)
    std::vector<double*> rand_ws;
    std::vector<double> rand_fl;           // flops of the randomized compressions of the step
    std::vector<int> rand_l;               // their accepted sketch widths
    std::vector<char> gram_task;           // R1 from the Gram matrix (k_compress_svd64 GRAM variant)
    size_t ws_need = 0, tails_total = 0;
    int64_t task0 = 0, tails0 = 0;         // first task / tail value in the batch arrays

    explicit FactorRun(lrx_handle h_) : h(h_), P(h_->plan) {}

    // the SVD-shaped descriptor (B column-major and kept, V from an SVD):
    // the SVD and the randomized range finder
    bool svd_like() const { return h->compress != LRX_RRQR; }
    // stacked blocks that take the randomized path (at most 64 columns)
    bool rand_task(const DCompress& T) const {
        return h->compress == LRX_RAND && T.M > 0 && T.c > 0 && T.c <= 64;
    }

    int32_t mo(int32_t m) const { return m >= 0 ? m + imap_base : m; }
    int32_t nr_of(int32_t e) const { const PEdge& E = P.edges[e]; return dim_of(E.rows, h->size[E.dst]); }
    int32_t nc_of(int32_t e) const { const PEdge& E = P.edges[e]; return dim_of(E.cols, h->size[E.src]); }
    DBlk blk(int32_t e) const {
        DBlk b;
        if (e < 0) { b.p = nullptr; b.nr = 0; b.nc = 0; return b; }   // empty pivot
        b.p = h->eptr[e]; b.nr = nr_of(e); b.nc = nc_of(e);
        return b;
    }
    // one contiguous, zeroed region for a group of new blocks (one memset)
    void alloc_group(const std::vector<int32_t>& es, hipStream_t st) {
        if (es.empty()) return;
        std::vector<size_t> off(es.size());
        size_t tot = 0;
        for (size_t q = 0; q < es.size(); ++q) {
            off[q] = tot;
            tot += (((size_t)nr_of(es[q]) * nc_of(es[q])) + 31) & ~(size_t)31;
        }
        double* base = h->arena.alloc(std::max<size_t>(tot, 1));
        for (size_t q = 0; q < es.size(); ++q) h->eptr[es[q]] = base + off[q];
        HIPCHK(hipMemsetAsync(base, 0, std::max<size_t>(tot, 1) * 8, st));
    }

    void setup(const lrx_csr* A, const double* val_dev, hipStream_t st);
    void merge_tasks(const LevelPlan& L, hipStream_t st, std::vector<DMerge>& mt);
    size_t compress_tasks();
    void bind_compress(double* wsp, int32_t* ranks_dev, double* tails_dev, int32_t piece_base);
    void take_ranks(const int32_t* rk, const double* tails_h, hipStream_t st);
    void node_tasks(const int32_t* rk, NodeBatch& nb);
};

void FactorRun::setup(const lrx_csr* A, const double* val_dev, hipStream_t st) {
    const int32_t n = P.n;
    h->size.assign(P.nodes.size(), -1);
    h->eptr.assign(P.edges.size(), nullptr);
    for (size_t v = 0; v < P.nodes.size(); ++v)
        if (P.nodes[v].leaf) h->size[v] = P.nodes[v].static_size;
    // mixed precision: the reduced QRs and Jacobi of the compression in FP32
    // when FP32 resolves the cut-off (sigma_k / sigma_0 >= epsilon >= 1e-5)
    fp32_compress = h->precision != LRX_FP64 && h->epsilon >= 1e-5;
    for (size_t li = 0; li < P.levels.size(); ++li) {
        const int32_t hgt = P.depth - P.levels[li].level;
        if (hgt < 0) fail(LRX_EDEVICE, "internal: level above the depth");
        if ((size_t)hgt >= level_at_height.size()) level_at_height.resize(hgt + 1, -1);
        level_at_height[hgt] = (int32_t)li;
    }

    // ---------------- static index maps (depend on supports only)
    auto put_map = [&](const std::vector<int32_t>& v) -> int32_t {
        int32_t off = (int32_t)imap.size();
        imap.insert(imap.end(), v.begin(), v.end());
        return off;
    };
    auto put_pos = [&](const Support& sub, const Support& sup) -> int32_t {
        if (sub.all && sup.all) return -1;
        std::vector<int32_t> v = positions(sub, sup, 0);
        if (!sub.all && !sub.idx.empty() && (v.size() != sub.idx.size() || v[0] < 0))
            fail(LRX_EDEVICE, "internal: support is not contained in its target");
        if (sub.all) fail(LRX_EDEVICE, "internal: full support with a compact target");
        return put_map(v);
    };
    maps.assign(P.steps.size(), {});
    auto piv_maps = [&](const PivotPlan& pp, PivMaps& pm) {
        for (int32_t e : pp.in_edges) {
            const Support& r = P.edges[e].rows;
            pm.in_rmap.push_back(r.all ? -1 : put_map(r.idx));
        }
        for (int32_t e : pp.out_edges) {
            const Support& c = P.edges[e].cols;
            pm.out_cmap.push_back(c.all ? -1 : put_map(c.idx));
        }
        for (size_t q = 0; q < pp.pair_edge.size(); ++q) {
            const PEdge& T = P.edges[pp.pair_edge[q]];
            const PEdge& O = P.edges[pp.out_edges[pp.pair_out[q]]];
            const PEdge& I = P.edges[pp.in_edges[pp.pair_in[q]]];
            // a compact source may land in a full target (e.g. a self block)
            if ((!T.rows.all && O.rows.all) || (!T.cols.all && I.cols.all))
                fail(LRX_EDEVICE, "internal: full source with a compact target in a Schur pair");
            pm.pair_rpos.push_back(put_pos(O.rows, T.rows));
            pm.pair_cpos.push_back(put_pos(I.cols, T.cols));
        }
    };
    for (size_t s = 0; s < P.steps.size(); ++s) {
        const ColourStep& cs = P.steps[s];
        maps[s].resize(cs.nodes.size());
        info_count += 2 * (int32_t)cs.nodes.size();
        for (size_t ni = 0; ni < cs.nodes.size(); ++ni) {
            const NodeStep& ns = cs.nodes[ni];
            NodeMaps& nm = maps[s][ni];
            for (const CandRef& cr : ns.cands) {
                if (cr.e_sp >= 0) {
                    nm.a_map.push_back(put_pos(P.edges[cr.e_sp].cols, ns.gamma));
                    nm.ra_map.push_back(put_pos(P.edges[cr.e_sp].rows, P.edges[cr.e_Pp].rows));
                } else { nm.a_map.push_back(-2); nm.ra_map.push_back(-2); }
                if (cr.e_ps >= 0) {
                    nm.b_map.push_back(put_pos(P.edges[cr.e_ps].rows, ns.gamma));
                    nm.qb_map.push_back(put_pos(P.edges[cr.e_ps].cols, P.edges[cr.e_pP].cols));
                } else { nm.b_map.push_back(-2); nm.qb_map.push_back(-2); }
            }
            piv_maps(ns.ps, nm.ps);
            piv_maps(ns.pb, nm.pb);
        }
    }

    // ---------------- initial blocks: A gathered into the leaf super-node blocks
    int64_t tot = 0;
    std::vector<int64_t> eoff(P.init_edges.size());
    for (size_t q = 0; q < P.init_edges.size(); ++q) {
        int32_t e = P.init_edges[q];
        eoff[q] = tot;
        tot += (((int64_t)nr_of(e) * nc_of(e)) + 31) & ~(int64_t)31;
    }
    double* base = h->arena.alloc((size_t)std::max<int64_t>(tot, 1));
    std::vector<int32_t> slot(P.edges.size(), -1);
    for (size_t q = 0; q < P.init_edges.size(); ++q) {
        h->eptr[P.init_edges[q]] = base + eoff[q];
        slot[P.init_edges[q]] = (int32_t)q;
    }
    HIPCHK(hipMemsetAsync(base, 0, (size_t)std::max<int64_t>(tot, 1) * 8, st));
    // destination of every entry of A
    std::vector<int32_t> leaf_of(n);
    const int64_t nleaf = (int64_t)1 << P.depth;
    for (int64_t c = 0; c < nleaf; ++c)
        for (int32_t t = P.leaf_ptr[c]; t < P.leaf_ptr[c + 1]; ++t) leaf_of[t] = (int32_t)c;
    // edge lookup per (src, dst) super pair
    std::vector<std::vector<std::pair<int32_t, int32_t>>> out_init(P.nodes.size());
    for (int32_t e : P.init_edges) out_init[P.edges[e].src].push_back({P.edges[e].dst, e});
    std::vector<int64_t> idx((size_t)A->nnz);
    for (int32_t r = 0; r < n; ++r) {
        const int32_t tr = P.pos[r];
        const int32_t sd = leaf_of[tr] >> 1;
        const int32_t lr = tr - P.nodes[sd].dof0;
        for (int64_t q = A->row_ptr[r]; q < A->row_ptr[r + 1]; ++q) {
            const int32_t tc = P.pos[A->col_idx[q]];
            const int32_t ss = leaf_of[tc] >> 1;
            const int32_t lc = tc - P.nodes[ss].dof0;
            int32_t e = -1;
            for (auto& pr : out_init[ss]) if (pr.first == sd) { e = pr.second; break; }
            if (e < 0) fail(LRX_EDEVICE, "internal: missing initial edge");
            const PEdge& E = P.edges[e];
            int32_t pr_ = E.rows.all ? lr : (int32_t)(std::lower_bound(E.rows.idx.begin(), E.rows.idx.end(), lr) - E.rows.idx.begin());
            int32_t pc_ = E.cols.all ? lc : (int32_t)(std::lower_bound(E.cols.idx.begin(), E.cols.idx.end(), lc) - E.cols.idx.begin());
            idx[q] = eoff[slot[e]] + pr_ + (int64_t)pc_ * nr_of(e);
        }
    }
    if (A->nnz > 0) {
        // the driver synchronizes before these temporaries are released
        d_idx.ensure(idx.size() * 8);
        HIPCHK(copy_sync(d_idx.p, idx.data(), idx.size() * 8, hipMemcpyHostToDevice));
        const double* src = val_dev;
        if (!src) {
            d_val.ensure((size_t)A->nnz * 8);
            HIPCHK(copy_sync(d_val.p, A->val, (size_t)A->nnz * 8, hipMemcpyHostToDevice));
            src = d_val.as<double>();
        }
        HIPCHK(launch_scatter(base, d_idx.as<int64_t>(), src, A->nnz, st));
    }
    // Frobenius rule: the leaf level's blocks hold exactly the entries of A, so
    // N_l^2 = sum of the squared values
    frob = h->rule == LRX_RULE_FROB;
    if (frob) {
        size_t groups = (size_t)level_norm_groups(0, A->nnz);
        for (const LevelPlan& L : P.levels) groups = std::max(groups, L.merges.size());
        d_norm.ensure((35 + std::max<size_t>(groups, 1)) * sizeof(double));
        HIPCHK(hipMemsetAsync(d_norm.p, 0, 35 * sizeof(double), st));
        double* state = d_norm.as<double>();
        const double* src = val_dev ? val_dev : d_val.as<double>();
        HIPCHK(launch_level_norm(nullptr, 0, A->nnz ? src : nullptr, A->nnz, state, state + 35, h->epsilon,
                                 P.depth, st));
    }
}

void FactorRun::merge_tasks(const LevelPlan& L, hipStream_t st, std::vector<DMerge>& mt) {
    for (int32_t s : L.supers) {
        const PNode& nd = P.nodes[s];
        h->size[s] = h->size[nd.comp0] + h->size[nd.comp1];
    }
    alloc_group(L.merge_edges, st);
    for (const MergePiece& mp : L.merges) {
        DMerge d;
        d.src = blk(mp.src_edge);
        d.dst = blk(mp.dst_edge);
        const PEdge& D = P.edges[mp.dst_edge];
        d.r0 = mp.row_hi ? h->size[P.nodes[D.dst].comp0] : 0;
        d.c0 = mp.col_hi ? h->size[P.nodes[D.src].comp0] : 0;
        if (d.src.nr * d.src.nc > 0) mt.push_back(d);
    }
}

bool same_support(const Support& a, const Support& b) {
    return a.all == b.all && (a.all || a.idx == b.idx);
}

// Compress descriptors of the current step (Algorithm 1, stacked B of eqn.
// cutOff1); returns the workspace this step needs, in doubles.
size_t FactorRun::compress_tasks() {
    const ColourStep& cs = P.steps[si];
    const int nn = (int)cs.nodes.size();
    const bool svd = svd_like();
    ct.assign(nn, DCompress{});
    pieces.clear();
    a_row0.assign(nn, {});
    b_row0.assign(nn, {});
    wsB.assign(nn, 0); wsV.assign(nn, 0); wsH.assign(nn, 0); tail_at.assign(nn, 0);
    wsR.assign(nn, 0); rand_ws.assign(nn, nullptr); rand_fl.assign(nn, 0.0); rand_l.assign(nn, 0);
    gram_task.assign(nn, 0);
    ws_need = 0;
    tails_total = 0;
    for (int ni = 0; ni < nn; ++ni) {
        const NodeStep& ns = cs.nodes[ni];
        const NodeMaps& nm = maps[si][ni];
        const int32_t ms = h->size[ns.s];
        DCompress& T = ct[ni];
        T.piece0 = (int32_t)pieces.size();
        int32_t row = 0;
        for (size_t k = 0; k < ns.cands.size(); ++k) {
            const CandRef& cr = ns.cands[k];
            a_row0[ni].push_back(row);
            if (cr.e_sp >= 0) {
                DPiece pc{};
                pc.blk = blk(cr.e_sp); pc.trans = 0; pc.row0 = row; pc.map = mo(nm.a_map[k]);
                row += pc.blk.nr;
                if (pc.blk.nr * pc.blk.nc > 0) pieces.push_back(pc);
                // half stack (symmetric A): B_k = A_k, so Q_k = R_k takes the same rows;
                // that needs p's support in Mat(s->p) rows and Mat(p->s) columns to agree
                if (h->symmetric && cr.e_ps >= 0 && !same_support(P.edges[cr.e_sp].rows, P.edges[cr.e_ps].cols))
                    fail(LRX_EINVAL, "symmetric: the block pattern is not symmetric");
            } else if (h->symmetric && cr.e_ps >= 0) {
                DPiece pc{};
                pc.blk = blk(cr.e_ps); pc.trans = 1; pc.row0 = row; pc.map = mo(nm.b_map[k]);
                row += pc.blk.nc;
                if (pc.blk.nr * pc.blk.nc > 0) pieces.push_back(pc);
            }
        }
        for (size_t k = 0; k < ns.cands.size(); ++k) {
            const CandRef& cr = ns.cands[k];
            b_row0[ni].push_back(h->symmetric ? a_row0[ni][k] : row);
            if (h->symmetric) continue;                 // the half stack has no B_k rows
            if (cr.e_ps >= 0) {
                DPiece pc{};
                pc.blk = blk(cr.e_ps); pc.trans = 1; pc.row0 = row; pc.map = mo(nm.b_map[k]);
                row += pc.blk.nc;
                if (pc.blk.nr * pc.blk.nc > 0) pieces.push_back(pc);
            }
        }
        T.npieces = (int32_t)pieces.size() - T.piece0;
        T.M = row;
        T.c = ns.gamma.count(ms);
        T.eps = h->epsilon;
        T.tau = frob ? d_norm.as<double>() + 1 : nullptr;
        wsB[ni] = ws_need; ws_need += ((size_t)T.M * T.c * (svd ? 2 : 1) + 31) & ~(size_t)31;
        wsV[ni] = ws_need; ws_need += ((size_t)T.c * T.c + 31) & ~(size_t)31;
        // hv: c^2 + c, or 4 c^2 + c + 8 for the large-block SVD (c > 64)
        wsH[ni] = ws_need;
        ws_need += ((size_t)T.c * T.c * (svd && T.c > 64 ? 4 : 1) + T.c + 8 + 31) & ~(size_t)31;
        // randomized: V_C (l x l), tails and rank of the sketched block
        if (rand_task(T)) {
            wsR[ni] = ws_need;
            ws_need += (((size_t)T.c * T.c + 31) & ~(size_t)31) + (((size_t)T.c + 2 + 31) & ~(size_t)31) + 32;
        }
        tail_at[ni] = tails_total;
        tails_total += (size_t)T.c + 2;
    }
    return ws_need;
}

void FactorRun::bind_compress(double* wsp, int32_t* ranks_dev, double* tails_dev, int32_t piece_base) {
    const bool svd = svd_like();
    for (size_t ni = 0; ni < ct.size(); ++ni) {
        DCompress& T = ct[ni];
        T.piece0 += piece_base;
        T.B = wsp + wsB[ni];
        T.Bw = svd ? wsp + wsB[ni] + (size_t)T.M * T.c : nullptr;
        T.V = wsp + wsV[ni];
        T.hv = wsp + wsH[ni];
        T.tails = tails_dev + tail_at[ni];
        T.rank_out = ranks_dev + ni;
        rand_ws[ni] = wsR[ni] ? wsp + wsR[ni] : nullptr;
    }
}

void FactorRun::take_ranks(const int32_t* rk, const double* tails_h, hipStream_t st) {
    const ColourStep& cs = P.steps[si];
    const bool svd = svd_like();
    for (size_t ni = 0; ni < cs.nodes.size(); ++ni) {
        const NodeStep& ns = cs.nodes[ni];
        const DCompress& T = ct[ni];
        h->size[ns.b] = rk[ni];
        h->size[ns.P] = rk[ni];
        h->ranks.push_back(rk[ni]);
        const double* tl = tails_h + tail_at[ni];
        const bool emptyB = T.M == 0 || T.c == 0;
        const int len = emptyB ? 1 : (svd ? T.c + 1 : rk[ni] + 2);
        h->tail_off.push_back((int64_t)h->tails.size());
        h->tails.insert(h->tails.end(), tl, tl + len);
        double ratio = 0.0;
        if (!emptyB && tl[0] > 0) {
            if (svd) ratio = rk[ni] < T.c ? tl[1 + rk[ni]] / tl[0] : 0.0;
            else ratio = tl[1 + rk[ni]] / tl[0];
        }
        h->max_tail_ratio = std::max(h->max_tail_ratio, ratio);
        h->rank_level.push_back(cs.level);
        h->comp_rows.push_back(T.M);
        h->comp_cols.push_back(T.c);
        h->rank_j.push_back(ns.j);
        // flops of the stacked QR and the Jacobi SVD (sweeps reported by the
        // kernel after the c + 1 singular-value slots), or of the pivoted QR
        if (!emptyB) {
            if (rand_ws[ni]) {
                // every sketch width tried (counted by the launches), then V = Q V_C
                const double fl = rand_fl[ni] + 2.0 * T.c * rand_l[ni] * rk[ni];
                flops += (int64_t)fl;
                fl_compress += fl;
                jac_flops += fl;
                v_bytes += 8.0 * T.c * rk[ni];
            } else if (gram_task[ni]) {
                // the Gram matrix (upper half, M c (c + 1) flops), its pivoted
                // Cholesky (c^3 / 3), the LQ and Q2 (8/3 c^3), then the Jacobi sweeps
                const double sw = tl[T.c + 1];
                const double jf = jacobi_flops(T.c, sw);
                const double cc = T.c;
                const double fg = (double)T.M * cc * (cc + 1.0) + cc * cc * cc / 3.0 + svd_pre_flops(cc) * 2.0 / 3.0;
                flops += (int64_t)(fg + jf);
                fl_compress += fg + jf;
                jac_flops_g += jf;
                jac_sweeps += sw;
                v_bytes_g += 8.0 * T.c * rk[ni];
            } else if (svd) {
                const double sw = tl[T.c + 1];
                const double jf = jacobi_flops(T.c, sw);
                flops += (int64_t)(qr_flops(T.M, T.c) + svd_pre_flops(T.c) + jf);
                fl_compress += qr_flops(T.M, T.c) + svd_pre_flops(T.c) + jf;
                jac_flops += jf;
                jac_sweeps += sw;
                v_bytes += 8.0 * T.c * rk[ni];
            } else {
                flops += 4ll * T.M * T.c * rk[ni];
                fl_compress += 4.0 * T.M * T.c * rk[ni];
            }
        }
    }
    // the blocks created in this step
    alloc_group(cs.new_edges, st);
}

// Preparation of every super-node (projection, rewiring, inverse of S), Schur
// products of s, inverse of the black pivot B = -V^T S^{-1} V, Schur products
// of b (Sec. 4.4 with the block elimination of Sec. 2.2).
void FactorRun::node_tasks(const int32_t* rk, NodeBatch& nb) {
    const ColourStep& cs = P.steps[si];
    const int nn = (int)cs.nodes.size();
    // W_k = S^{-1}[:, rows of Mat(k->v)] Mat(k->v) for every pivot of the step, in
    // a buffer of its own sized now that the ranks are known (the stream is idle
    // after the rank read-back, so growing it is safe)
    size_t wtot = 0;
    auto w_of = [&](const PivotPlan& pp) {
        const int32_t m = h->size[pp.node];
        if (m == 0 || pp.e_self < 0) return;
        for (int32_t e : pp.in_edges) wtot += (((size_t)m * nc_of(e)) + 31) & ~(size_t)31;
    };
    for (int ni = 0; ni < nn; ++ni) {
        w_of(cs.nodes[ni].ps);
        w_of(cs.nodes[ni].pb);
    }
    DevBuf& ws = h->ws_w;
    if (wtot * 8 > ws.bytes) ws.ensure(wtot * 8 + (wtot * 8) / 2);
    double* wsp = ws.as<double>();
    size_t wcur = 0;
    const int64_t gf_s0 = nb.gf_s, gf_b0 = nb.gf_b, pf_s0 = nb.pf_s, pf_b0 = nb.pf_b, gf_p0 = nb.gf_p;
    auto schur = [&](const PivotPlan& pp, const PivMaps& pm, std::vector<DGemm>& g1, std::vector<DGemm>& g2,
                     int64_t& gfl) {
        const int32_t m = h->size[pp.node];
        if (m == 0 || pp.e_self < 0) return;
        const double* Sinv = h->eptr[pp.e_self];
        std::vector<double*> W(pp.in_edges.size(), nullptr);
        std::vector<DBlk> ib(pp.in_edges.size());
        for (size_t i = 0; i < pp.in_edges.size(); ++i) {
            ib[i] = blk(pp.in_edges[i]);
            W[i] = wsp + wcur;
            wcur += (((size_t)m * ib[i].nc) + 31) & ~(size_t)31;
            if ((int64_t)ib[i].nr * ib[i].nc == 0) continue;
            DGemm G{};
            G.A = Sinv; G.lda = m; G.amap = mo(pm.in_rmap[i]);
            G.B = ib[i].p; G.ldb = ib[i].nr; G.bmap = -1;
            G.C = W[i]; G.ldc = m; G.crmap = -1; G.ccmap = -1;
            G.M = m; G.N = ib[i].nc; G.K = ib[i].nr; G.sub = 0;
            g1.push_back(G);
            gfl += 2ll * m * ib[i].nr * ib[i].nc;
        }
        for (size_t q = 0; q < pp.pair_edge.size(); ++q) {
            const int32_t qi = pp.pair_out[q], ki = pp.pair_in[q];
            const DBlk O = blk(pp.out_edges[qi]);
            const DBlk T = blk(pp.pair_edge[q]);
            if ((int64_t)O.nr * O.nc * ib[ki].nc == 0) continue;
            DGemm G{};
            G.A = O.p; G.lda = O.nr; G.amap = -1;
            G.B = W[ki]; G.ldb = m; G.bmap = mo(pm.out_cmap[qi]);
            G.C = T.p; G.ldc = T.nr; G.crmap = mo(pm.pair_rpos[q]); G.ccmap = mo(pm.pair_cpos[q]);
            G.M = O.nr; G.N = ib[ki].nc; G.K = O.nc; G.sub = 1;
            g2.push_back(G);
            gfl += 2ll * O.nr * O.nc * ib[ki].nc;
        }
    };
    for (int ni = 0; ni < nn; ++ni) {
        const NodeStep& ns = cs.nodes[ni];
        DPrep T{};
        const int32_t r = rk[ni];
        T.r = r;
        T.c = ct[ni].c;
        T.M = ct[ni].M;
        T.svd = svd_like() ? 1 : 0;
        T.B = ct[ni].B;
        T.V = ct[ni].V;
        T.do_proj = 1;
        T.proj0 = (int32_t)nb.projs.size();
        const bool svd = svd_like();
        // SVD: piece k of B V = B[rows of k, :] V (nrows x r) into R_k (trans 0) or,
        // transposed, into Q_k^T (trans 1), as tiled products; RRQR: row copies
        auto piece = [&](const DProj& pj) {
            if (pj.nrows <= 0 || r <= 0) return;
            if (!svd) { nb.projs.push_back(pj); return; }
            DGemm G{};
            G.A = ct[ni].B + pj.row0; G.lda = ct[ni].M; G.amap = -1;
            G.B = ct[ni].V; G.ldb = ct[ni].c; G.bmap = -1;
            G.C = pj.dst.p; G.ldc = pj.trans ? r : pj.dst.nr;
            G.crmap = pj.map; G.ccmap = -1; G.tr = pj.trans;
            G.M = pj.nrows; G.N = r; G.K = ct[ni].c; G.sub = 0;
            nb.gp.push_back(G);
            nb.gf_p += 2ll * pj.nrows * ct[ni].c * r;
        };
        for (size_t k = 0; k < ns.cands.size(); ++k) {
            const CandRef& cr = ns.cands[k];
            if (cr.e_sp >= 0) {
                DProj pj{};
                pj.dst = blk(cr.e_Pp);
                pj.row0 = a_row0[ni][k];
                pj.nrows = nr_of(cr.e_sp);
                pj.trans = 0;
                pj.map = mo(maps[si][ni].ra_map[k]);
                piece(pj);
            }
            if (cr.e_ps >= 0) {
                DProj pj{};
                pj.dst = blk(cr.e_pP);
                pj.row0 = b_row0[ni][k];                 // half stack: the rows of A_k (Q_k = R_k)
                pj.nrows = nc_of(cr.e_ps);
                pj.trans = 1;
                pj.map = mo(maps[si][ni].qb_map[k]);
                piece(pj);
            }
        }
        T.nproj = (int32_t)nb.projs.size() - T.proj0;
        T.sb = blk(ns.e_sb);
        T.bs = blk(ns.e_bs);
        T.bP = blk(ns.e_bP);
        T.Pb = blk(ns.e_Pb);
        T.piv = blk(ns.ps.e_self);
        T.info_slot = info_base + info_next++;
        nb.max_ms = std::max(nb.max_ms, (int)T.piv.nr);
        nb.pf_s += 2ll * T.piv.nr * T.piv.nr * T.piv.nr + (svd ? 0ll : 2ll * T.M * T.c * r);
        nb.prep_s.push_back(T);
        DPrep U{};
        U.piv = blk(ns.pb.e_self);
        U.info_slot = info_base + info_next++;
        U.do_proj = 0;
        nb.max_mb = std::max(nb.max_mb, (int)U.piv.nr);
        nb.pf_b += 2ll * U.piv.nr * U.piv.nr * U.piv.nr;
        nb.prep_b.push_back(U);
        schur(ns.ps, maps[si][ni].ps, nb.g1s, nb.g2s, nb.gf_s);
        schur(ns.pb, maps[si][ni].pb, nb.g1b, nb.g2b, nb.gf_b);
    }
    flops += (nb.pf_s - pf_s0) + (nb.pf_b - pf_b0) + (nb.gf_s - gf_s0) + (nb.gf_b - gf_b0) + (nb.gf_p - gf_p0);
    fl_pivot += (double)((nb.pf_s - pf_s0) + (nb.pf_b - pf_b0));
    fl_schur += (double)((nb.gf_s - gf_s0) + (nb.gf_b - gf_b0));
    fl_project += (double)(nb.gf_p - gf_p0);
    if (wcur != wtot) fail(LRX_EDEVICE, "internal: Schur workspace size mismatch");
}

// Products of a factorization step (Schur updates, projection): on the matrix
// cores (MFMA) with operand precision prec, K staged in chunks of
// g_tune.gemm_kc columns; FP64 products may instead run as the VALU tile kernel
// when the tuning table says it is faster for this device.
hipError_t gemm_products(const DGemm* g, const DTile* t, int ntile, int kmax, const int32_t* imap, int prec,
                         hipStream_t st) {
    if (prec == GP_F64 && g_tune.gemm_f64_valu) return launch_gemm_tiles(g, t, ntile, kmax, imap, st);
    return launch_gemm_mfma(g, t, ntile, kmax, imap, prec, g_tune.gemm_kc, g_tune.gemm_grid, st);
}

// The level loop over one or several factorizations sharing the stream st.
// Throws on failure; the caller frees the handles.
void run_factor(const std::vector<FactorRun*>& runs, hipStream_t st, const std::vector<const lrx_csr*>& A,
                const std::vector<const double*>& val_dev) {
    double t_sync = 0.0;
    double t_h_comp = 0.0, t_h_node = 0.0;   // host work of the compress and node phases
    int64_t epoch = 0;                   // number of stream synchronizations so far
    auto sync = [&]() {
        const double ts = now_ms();
        HIPCHK(hipStreamSynchronize(st));
        t_sync += now_ms() - ts;
        ++epoch;
    };
    std::vector<int32_t> imap;
    int32_t info_total = 0;
    size_t max_h = 0;
    for (size_t i = 0; i < runs.size(); ++i) {
        FactorRun& r = *runs[i];
        r.setup(A[i], val_dev[i], st);
        if ((int64_t)imap.size() + (int64_t)r.imap.size() > INT32_MAX) fail(LRX_ENOMEM, "index tables exceed 2^31 entries");
        r.imap_base = (int32_t)imap.size();
        imap.insert(imap.end(), r.imap.begin(), r.imap.end());
        std::vector<int32_t>().swap(r.imap);
        r.info_base = info_total;
        info_total += r.info_count;
        max_h = std::max(max_h, r.level_at_height.size());
    }
    DevBuf d_imap, d_info;
    d_imap.ensure(std::max<size_t>(imap.size(), 1) * sizeof(int32_t));
    if (!imap.empty())
        HIPCHK(hipMemcpyAsync(d_imap.p, imap.data(), imap.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    const int32_t* dmap = d_imap.as<int32_t>();
    d_info.ensure(std::max(info_total, 1) * sizeof(int32_t));
    HIPCHK(hipMemsetAsync(d_info.p, 0, std::max(info_total, 1) * sizeof(int32_t), st));
    sync();
    for (FactorRun* r : runs) { r->d_idx.release(); r->d_val.release(); }

    PinBuf stage_m, stage_c, stage_n, pin_rt, pin_flags;   // descriptor staging, rank read-back
    DevBuf d_desc_m, d_desc_c, d_desc_n, d_rt, d_flags, d_gjperm;
    PinBuf pin_rand, pin_rflags;               // randomized compression: attempt descriptors, flags
    DevBuf d_rand, d_rflags;
    int64_t m_epoch = -1;                       // epoch of the last merge upload
    for (size_t hgt = 0; hgt < max_h; ++hgt) {
        std::vector<FactorRun*> lv;
        std::vector<DMerge> mt;
        int32_t ncol = 0;
        for (FactorRun* r : runs) {
            if (hgt >= r->level_at_height.size() || r->level_at_height[hgt] < 0) continue;
            const LevelPlan& L = r->P.levels[r->level_at_height[hgt]];
            r->merge0 = r->merge1 = mt.size();
            if (L.level < r->P.depth) r->merge_tasks(L, st, mt);
            r->merge1 = mt.size();
            lv.push_back(r);
            ncol = std::max(ncol, L.nsteps);
        }
        if (!mt.empty()) {
            // the previous merge upload may still read stage_m, its kernel d_desc_m
            if (m_epoch == epoch) sync();
            std::vector<char> buf;
            const size_t o = append_bytes(buf, mt);
            stage_m.ensure(buf.size());
            std::memcpy(stage_m.p, buf.data(), buf.size());
            d_desc_m.ensure(buf.size());
            HIPCHK(hipMemcpyAsync(d_desc_m.p, stage_m.p, buf.size(), hipMemcpyHostToDevice, st));
            HIPCHK(launch_merge((const DMerge*)(d_desc_m.as<char>() + o), (int)mt.size(), st));
            m_epoch = epoch;
        }
        // Frobenius rule: this level's blocks are the merged red blocks (a level
        // whose reds are all empty adds nothing, N carries over)
        for (FactorRun* r : lv) {
            const LevelPlan& L = r->P.levels[r->level_at_height[hgt]];
            if (!r->frob || L.level >= r->P.depth) continue;
            double* state = r->d_norm.as<double>();
            const DMerge* pieces = r->merge1 > r->merge0 ? d_desc_m.as<DMerge>() + r->merge0 : nullptr;
            HIPCHK(launch_level_norm(pieces, (int)(r->merge1 - r->merge0), nullptr, 0, state, state + 35,
                                     r->h->epsilon, L.level, st));
        }
        for (int32_t c = 0; c < ncol; ++c) {
            std::vector<FactorRun*> part;
            for (FactorRun* r : lv) {
                const LevelPlan& L = r->P.levels[r->level_at_height[hgt]];
                if (c >= L.nsteps) continue;
                r->si = L.step0 + c;
                part.push_back(r);
            }
            // ---- compress: descriptors, workspace, one launch per kernel variant
            const double tc0 = now_ms();
            bool grow = false;
            std::vector<size_t> wst(part.size());
            for (size_t i = 0; i < part.size(); ++i) {
                wst[i] = part[i]->compress_tasks();
                grow |= wst[i] * 8 > part[i]->h->ws_b.bytes;
            }
            // the workspace is only touched by kernels on this stream; growing it
            // frees it, which needs the stream idle
            if (grow) {
                sync();
                for (size_t i = 0; i < part.size(); ++i)
                    if (wst[i] * 8 > part[i]->h->ws_b.bytes) part[i]->h->ws_b.ensure(wst[i] * 8 + (wst[i] * 8) / 2);
            }
            int64_t ntask = 0, ntail = 0;
            for (FactorRun* r : part) {
                r->task0 = ntask;
                r->tails0 = ntail;
                ntask += (int64_t)r->ct.size();
                ntail += (int64_t)r->tails_total;
            }
            const size_t tails_off = ((size_t)ntask * 4 + 255) & ~(size_t)255;
            const size_t rt_bytes = tails_off + (size_t)ntail * 8;
            d_rt.ensure(rt_bytes);    // its last reader, the previous read-back, has completed
            std::vector<DCompress> all;
            std::vector<DPiece> allp;
            std::vector<int32_t> fp32_of;
            std::vector<std::pair<FactorRun*, int>> owner;   // run and node of every task
            all.reserve(ntask);
            for (FactorRun* r : part) {
                r->bind_compress(r->h->ws_b.as<double>(), d_rt.as<int32_t>() + r->task0,
                                 (double*)(d_rt.as<char>() + tails_off) + r->tails0, (int32_t)allp.size());
                all.insert(all.end(), r->ct.begin(), r->ct.end());
                allp.insert(allp.end(), r->pieces.begin(), r->pieces.end());
                for (size_t q = 0; q < r->ct.size(); ++q) {
                    // bit 2: pivoted QR; bit 3: randomized, bit 1 with it: BF16 sketch
                    // bit 4: the Gram path may take it (SVD, epsilon >= 1e-5, mixed
                    // precision with compress_gram >= 1 or FP64 with compress_gram = 2)
                    int f = r->h->compress == LRX_RRQR ? 4 : r->fp32_compress ? 1 : 0;
                    const bool gram = r->h->compress == LRX_SVD && r->h->epsilon >= 1e-5 &&
                                      g_tune.compress_gram >= (r->h->precision == LRX_FP64 ? 2 : 1);
                    if (gram) f |= 16;
                    if (r->rand_task(r->ct[q])) f = 8 | (r->h->precision == LRX_MIXED_BF16 ? 2 : 0);
                    fp32_of.push_back(f);
                    owner.emplace_back(r, (int)q);
                }
            }
            // variants: SVD with c <= 64 (FP64 / FP32 arithmetic: keys 0 / 1; 16 / 17
            // for 33..64 columns; 24: mixed precision through the FP64 Gram matrix), SVD
            // with c > 64 (even keys: FP64 rows kept, odd: rows below epsilon / 100
            // dropped in mixed precision; 8 / 9: one work-group per task; 12 / 13
            // for tall blocks, M c >= 3e5: the tall QR in multi-work-group panels,
            // the rest in one work-group; 10 / 11 for c > large_split_c (tuning, 128 by
            // default) or M c >= 1e6: QRs in panels and the Jacobi in multi-work-group
            // block rounds; key 2 when the LDS of the large kernel does not fit; 26 / 27 and 28 / 29: R1 through
            // the FP64 Gram matrix and its pivoted Cholesky, then as 12 / 13 and
            // 10 / 11), pivoted QR (key 4), randomized range finder with c <= 64
            // (20: FP64 sketch, 21: BF16 sketch); each task takes its own variant
            // whatever the others are
            struct Group {
                int key; std::vector<DCompress> t; std::vector<int> q;
                int max_c = 1, max_M = 1, max_pieces = 0; int64_t max_mc = 1;
                double fl = 0, by = 0; size_t off = 0;
            };
            std::vector<Group> groups;
            for (size_t q = 0; q < all.size(); ++q) {
                int key;
                if (fp32_of[q] & 8) key = 20 | ((fp32_of[q] & 2) ? 1 : 0);
                else if (fp32_of[q] & 4) key = 4;
                else if (all[q].c <= 64 && (fp32_of[q] & 16)) {
                    key = 24 | (fp32_of[q] & 1);         // FP64 Gram matrix and pivoted Cholesky
                    owner[q].first->gram_task[owner[q].second] = 1;
                } else if (all[q].c <= 64) key = (fp32_of[q] & 1) | (all[q].c > 32 ? 16 : 0);
                else if (compress_large_fits(all[q].M, all[q].c)) {
                    const int64_t mc = (int64_t)all[q].M * all[q].c;
                    const bool split = all[q].c > g_tune.large_split_c || mc >= 1000000;
                    // (odd keys drop pivoted-QR rows below epsilon / 100 relative to
                    // sigma_0: not under the absolute threshold of the Frobenius rule)
                    const int drop = (fp32_of[q] & 1) && !all[q].tau ? 1 : 0;
                    if ((fp32_of[q] & 16) && !all[q].tau) {
                        key = (split ? 28 : 26) | drop;  // R1 from the Gram matrix
                        owner[q].first->gram_task[owner[q].second] = 1;
                    } else
                        key = (split ? 10 : mc >= 300000 ? 12 : 8) | drop;
                } else key = 2;
                size_t g = 0;
                while (g < groups.size() && groups[g].key != key) ++g;
                if (g == groups.size()) { groups.push_back(Group{}); groups[g].key = key; }
                Group& G = groups[g];
                G.t.push_back(all[q]);
                G.q.push_back((int)q);
                G.max_c = std::max(G.max_c, (int)all[q].c);
                G.max_M = std::max(G.max_M, (int)all[q].M);
                G.max_mc = std::max(G.max_mc, (int64_t)all[q].M * all[q].c);
                G.max_pieces = std::max(G.max_pieces, (int)all[q].npieces);
                // known before the launch: the QRs (RRQR: at full rank, an upper
                // bound); the Jacobi sweeps are added after the read-back
                const double M = all[q].M, cc = all[q].c;
                if (M > 0 && cc > 0 && key < 20)     // (randomized: counted per sketch width)
                    G.fl += key == 4 ? 4.0 * M * cc * cc : qr_flops(M, cc) + svd_pre_flops(cc);
                else if (M > 0 && cc > 0 && key >= 24 && key <= 29)
                    G.fl += M * cc * (cc + 1.0) + cc * cc * cc / 3.0 + svd_pre_flops(cc) * 2.0 / 3.0;
                G.by += 8.0 * M * cc;        // the stacked pieces, read once (V is added after the read-back)
            }
            {
                std::vector<char> buf;
                for (Group& G : groups) G.off = append_bytes(buf, G.t);
                const size_t op = append_bytes(buf, allp);
                // randomized mode: every task's V gets a fixed sign per column
                const bool canon = part[0]->h->compress == LRX_RAND;
                const size_t oall = canon ? append_bytes(buf, all) : 0;
                stage_c.ensure(buf.size());
                std::memcpy(stage_c.p, buf.data(), buf.size());
                d_desc_c.ensure(buf.size());
                HIPCHK(hipMemcpyAsync(d_desc_c.p, stage_c.p, buf.size(), hipMemcpyHostToDevice, st));
                const DPiece* dp = (const DPiece*)(d_desc_c.as<char>() + op);
                // independent variants run side by side: the split variant (its
                // sweeps are driven from the host) on the caller's stream, the
                // others on library streams forked from it and joined back after
                // randomized range finder: sketch widths min(16, c_nz), then doubled
                // for the tasks whose rank was not below the width, until c_nz; each
                // attempt is a sketch, the SVD of the sketched blocks and a finish
                // launch, then a read-back of the flags (host-driven, on st)
                auto run_rand = [&](const std::vector<DCompress>& tk, const std::vector<int>& qs, int bf16,
                                    hipStream_t gs) {
                    const int n = (int)tk.size();
                    std::vector<int> act(n), lreq(n, 16);
                    for (int i = 0; i < n; ++i) act[i] = i;
                    bool first = true;
                    while (!act.empty()) {
                        const int na = (int)act.size();
                        std::vector<DCompress> ta(na), ca(na);
                        std::vector<DRand> ra(na);
                        int max_l = 1, max_M = 1;
                        for (int k = 0; k < na; ++k) {
                            const int i = act[k];
                            const DCompress& T = tk[i];
                            FactorRun* r = owner[qs[i]].first;
                            const int ni = owner[qs[i]].second;
                            const size_t cc = (size_t)T.c;
                            ta[k] = T;
                            ra[k] = DRand{};
                            ra[k].l = std::min(lreq[i], (int)T.c);
                            ra[k].active = 1;
                            ra[k].key = ((int64_t)r->P.steps[r->si].level << 24) | r->P.steps[r->si].nodes[ni].j;
                            double* w = r->rand_ws[ni];
                            DCompress C{};
                            C.piece0 = 0; C.npieces = -1; C.M = T.M; C.c = ra[k].l;
                            C.B = T.Bw; C.V = w;
                            C.tails = w + ((cc * cc + 31) & ~(size_t)31);
                            C.rank_out = (int32_t*)(C.tails + ((cc + 2 + 31) & ~(size_t)31));
                            C.eps = T.eps; C.nb2 = T.hv + cc * cc;
                            ca[k] = C;
                            max_l = std::max(max_l, ra[k].l);
                            max_M = std::max(max_M, (int)T.M);
                        }
                        std::vector<char> buf;
                        const size_t ot = append_bytes(buf, ta), orr = append_bytes(buf, ra);
                        const size_t oc = append_bytes(buf, ca);
                        // the previous attempt's copies and kernels completed at its sync
                        pin_rand.ensure(buf.size());
                        std::memcpy(pin_rand.p, buf.data(), buf.size());
                        d_rand.ensure(buf.size());
                        d_rflags.ensure((size_t)na * sizeof(int32_t));
                        pin_rflags.ensure((size_t)na * sizeof(int32_t));
                        HIPCHK(hipMemcpyAsync(d_rand.p, pin_rand.p, buf.size(), hipMemcpyHostToDevice, gs));
                        const DCompress* dta = (const DCompress*)(d_rand.as<char>() + ot);
                        const DRand* dra = (const DRand*)(d_rand.as<char>() + orr);
                        DCompress* dca = (DCompress*)(d_rand.as<char>() + oc);
                        HIPCHK(launch_rand_sketch(dta, dra, dca, na, dp, dmap, first ? 1 : 0, bf16, gs));
                        HIPCHK(launch_compress_svd(dca, na, dp, dmap, max_l, max_M, false,
                                                   max_l > 32 ? g_tune.compress_nt_mid : g_tune.compress_nt_small,
                                                   gs));
                        HIPCHK(launch_rand_finish(dta, dra, dca, na, d_rflags.as<int32_t>(), gs));
                        HIPCHK(hipMemcpyAsync(pin_rflags.p, d_rflags.p, (size_t)na * sizeof(int32_t),
                                              hipMemcpyDeviceToHost, gs));
                        sync();
                        const int32_t* fl = (const int32_t*)pin_rflags.p;
                        std::vector<int> next;
                        for (int k = 0; k < na; ++k) {
                            const int i = act[k];
                            FactorRun* r = owner[qs[i]].first;
                            const int ni = owner[qs[i]].second;
                            const double M = tk[i].M, c = tk[i].c;
                            const int l = fl[k] >> 8;
                            const double sw = (fl[k] >> 1) & 127;
                            // sketch (M c l additions), QR of Y and its explicit Q, C = B Q,
                            // QR-preconditioned Jacobi SVD of C
                            double f = M * c * l + 2.0 * qr_flops(c, l) + 2.0 * M * c * l;
                            if (l > 0) f += qr_flops(M, l) + svd_pre_flops(l) + jacobi_flops(l, sw);
                            r->rand_fl[ni] += f;
                            r->rand_l[ni] = l;
                            if (fl[k] & 1) {
                                lreq[i] *= 2;
                                next.push_back(i);
                            }
                        }
                        act.swap(next);
                        first = false;
                    }
                };
                auto run_group = [&](Group& G, hipStream_t gs) {
                    const DCompress* dt = (const DCompress*)(d_desc_c.as<char>() + G.off);
                    LaunchTimer tm(G.key >= 24 && G.key <= 29 ? LRX_K_COMPRESS_GRAM : LRX_K_COMPRESS, gs, G.by, G.fl);
                    // after the state mode 5 (or 8) leaves: the LQ and Q2 in panels, then
                    // sweeps of block-Jacobi rounds over all tasks until none rotates,
                    // then the singular values and V
                    auto split_rest = [&](const DCompress* dt, int nt, double trunc) {
                        HIPCHK(launch_qr_blocked(dt, nt, G.max_c, G.max_M, 1, gs));
                        HIPCHK(launch_qr_blocked(dt, nt, G.max_c, G.max_M, 2, gs));
                        HIPCHK(launch_compress_large(dt, nt, dp, dmap, G.max_c, G.max_M, trunc, 6, gs, (G.key & 1) != 0));
                        d_flags.ensure((size_t)nt * sizeof(int32_t));
                        pin_flags.ensure((size_t)nt * sizeof(int32_t));
                        const int rounds = large_rounds(G.max_c);
                        for (int sweep = 0; sweep < 40; ++sweep) {
                            for (int t = 0; t < rounds; ++t)
                                HIPCHK(launch_large_round(dt, nt, G.max_c, t, gs));
                            HIPCHK(launch_large_flags(dt, nt, d_flags.as<int32_t>(), gs));
                            HIPCHK(hipMemcpyAsync(pin_flags.p, d_flags.p, (size_t)nt * sizeof(int32_t),
                                                  hipMemcpyDeviceToHost, gs));
                            sync();
                            const int32_t* fl = (const int32_t*)pin_flags.p;
                            bool go = false;
                            for (int q = 0; q < nt; ++q) go |= fl[q] != 0;
                            if (!go) break;
                        }
                        HIPCHK(launch_compress_large(dt, nt, dp, dmap, G.max_c, G.max_M, trunc, 2, gs));
                    };
                    if (G.key == 4)
                        HIPCHK(launch_compress(dt, (int)G.t.size(), dp, dmap, G.max_c, gs));
                    else if (G.key == 8 || G.key == 9) {
                        HIPCHK(launch_compress_large(dt, (int)G.t.size(), dp, dmap, G.max_c, G.max_M,
                                                     (G.key & 1) ? 0.01 : 0.0, 0, gs, (G.key & 1) != 0));
                    } else if (G.key == 12 || G.key == 13) {
                        const int nt = (int)G.t.size();
                        const double trunc = (G.key & 1) ? 0.01 : 0.0;
                        HIPCHK(launch_assemble_large(dt, nt, dp, dmap, G.max_mc, G.max_pieces, true, gs));
                        HIPCHK(launch_qr_blocked(dt, nt, G.max_c, G.max_M, 0, gs));
                        HIPCHK(launch_compress_large(dt, nt, dp, dmap, G.max_c, G.max_M, trunc, 7, gs, (G.key & 1) != 0));
                    } else if (G.key == 10 || G.key == 11) {
                        const int nt = (int)G.t.size();
                        const double trunc = (G.key & 1) ? 0.01 : 0.0;
                        HIPCHK(launch_assemble_large(dt, nt, dp, dmap, G.max_mc, G.max_pieces, true, gs));
                        HIPCHK(launch_qr_blocked(dt, nt, G.max_c, G.max_M, 0, gs));
                        HIPCHK(launch_compress_large(dt, nt, dp, dmap, G.max_c, G.max_M, trunc, 5, gs));
                        split_rest(dt, nt, trunc);
                    } else if (G.key >= 26 && G.key <= 29) {
                        // Gram matrix and pivoted Cholesky for R1; the rest in one
                        // work-group per task (26, 27) or split as above (28, 29)
                        const int nt = (int)G.t.size();
                        const double trunc = (G.key & 1) ? 0.01 : 0.0;
                        HIPCHK(launch_assemble_large(dt, nt, dp, dmap, G.max_mc, G.max_pieces, false, gs));
                        HIPCHK(launch_gram_chol(dt, nt, G.max_c, trunc, gs));
                        HIPCHK(launch_compress_large(dt, nt, dp, dmap, G.max_c, G.max_M, trunc, 8, gs));
                        if (G.key < 28)
                            HIPCHK(launch_compress_large(dt, nt, dp, dmap, G.max_c, G.max_M, trunc, 9, gs, (G.key & 1) != 0));
                        else
                            split_rest(dt, nt, trunc);
                    } else if (G.key == 20 || G.key == 21) {
                        run_rand(G.t, G.q, G.key & 1, gs);
                    } else if (G.key == 24 || G.key == 25) {
                        // Gram path (25: FP32 LQ and Jacobi in mixed precision)
                        HIPCHK(launch_compress_svd(dt, (int)G.t.size(), dp, dmap, G.max_c, G.max_M, G.key == 25,
                                                   G.max_c > 32 ? g_tune.compress_nt_mid : g_tune.compress_nt_small,
                                                   gs, true));
                    }
                    else
                        HIPCHK(launch_compress_svd(dt, (int)G.t.size(), dp, dmap, G.max_c, G.max_M,
                                                   (G.key & 1) != 0,
                                                   G.key >= 16 ? g_tune.compress_nt_mid : g_tune.compress_nt_small,
                                                   gs));
                };
                auto host_driven = [](int key) {
                    return key == 10 || key == 11 || key == 20 || key == 21 || key == 28 || key == 29;
                };
                std::vector<hipStream_t> gsv(groups.size(), st);
                AuxStreams* ax = groups.size() > 1 ? aux_streams() : nullptr;
                bool used[2] = {false, false};
                if (ax) {
                    bool split = false;
                    for (const Group& G : groups) split |= host_driven(G.key);
                    bool keep = !split;                  // without a host-driven variant one stays on st
                    int j = 0;
                    for (size_t g = 0; g < groups.size(); ++g) {
                        if (host_driven(groups[g].key)) continue;
                        if (keep) { keep = false; continue; }
                        gsv[g] = ax->s[j & 1];
                        used[j & 1] = true;
                        ++j;
                    }
                    if (used[0] || used[1]) {
                        HIPCHK(hipEventRecord(ax->fork, st));
                        for (int k = 0; k < 2; ++k)
                            if (used[k]) HIPCHK(hipStreamWaitEvent(ax->s[k], ax->fork, 0));
                    }
                }
                for (size_t g = 0; g < groups.size(); ++g)
                    if (gsv[g] != st) run_group(groups[g], gsv[g]);
                for (size_t g = 0; g < groups.size(); ++g)
                    if (gsv[g] == st) run_group(groups[g], st);
                for (int k = 0; k < 2; ++k)
                    if (used[k]) {
                        HIPCHK(hipEventRecord(ax->join[k], ax->s[k]));
                        HIPCHK(hipStreamWaitEvent(st, ax->join[k], 0));
                    }
                if (canon)
                    HIPCHK(launch_v_sign((const DCompress*)(d_desc_c.as<char>() + oall), (int)all.size(), st));
            }
            t_h_comp += now_ms() - tc0;
            pin_rt.ensure(rt_bytes);
            if (rt_bytes) HIPCHK(hipMemcpyAsync(pin_rt.p, d_rt.p, rt_bytes, hipMemcpyDeviceToHost, st));
            sync();
            const double tn0 = now_ms();
            const int32_t* rk = (const int32_t*)pin_rt.p;
            const double* tails_h = (const double*)((const char*)pin_rt.p + tails_off);
            for (FactorRun* r : part) {
                r->jac_flops = 0.0;
                r->v_bytes = 0.0;
                r->jac_flops_g = 0.0;
                r->v_bytes_g = 0.0;
                r->take_ranks(rk + r->task0, tails_h + r->tails0, st);
                timing_add(LRX_K_COMPRESS, r->v_bytes, r->jac_flops);
                timing_add(LRX_K_COMPRESS_GRAM, r->v_bytes_g, r->jac_flops_g);
            }
            // ---- node tasks of every participating factorization
            NodeBatch nb;
            for (FactorRun* r : part) r->node_tasks(rk + r->task0, nb);
            auto tiles_of = [](const std::vector<DGemm>& gs, int& kmax) {
                std::vector<DTile> t;
                kmax = 1;
                for (size_t g = 0; g < gs.size(); ++g) {
                    kmax = std::max(kmax, (int)gs[g].K);
                    for (int32_t i0 = 0; i0 < gs[g].M; i0 += 32)
                        for (int32_t j0 = 0; j0 < gs[g].N; j0 += 32) t.push_back(DTile{(int32_t)g, i0, j0, 0});
                }
                return t;
            };
            int kps, k1s, k2s, k1b, k2b;
            const std::vector<DTile> tps = tiles_of(nb.gp, kps);
            const std::vector<DTile> t1s = tiles_of(nb.g1s, k1s), t2s = tiles_of(nb.g2s, k2s);
            const std::vector<DTile> t1b = tiles_of(nb.g1b, k1b), t2b = tiles_of(nb.g2b, k2b);
            std::vector<char> buf;
            const size_t o_ps = append_bytes(buf, nb.prep_s), o_pj = append_bytes(buf, nb.projs);
            const size_t o_pb = append_bytes(buf, nb.prep_b);
            const size_t o_gp = append_bytes(buf, nb.gp), o_tp = append_bytes(buf, tps);
            const size_t o_g1s = append_bytes(buf, nb.g1s), o_t1s = append_bytes(buf, t1s);
            const size_t o_g2s = append_bytes(buf, nb.g2s), o_t2s = append_bytes(buf, t2s);
            const size_t o_g1b = append_bytes(buf, nb.g1b), o_t1b = append_bytes(buf, t1b);
            const size_t o_g2b = append_bytes(buf, nb.g2b), o_t2b = append_bytes(buf, t2b);
            // the previous step's node kernels completed before the read-back above
            stage_n.ensure(buf.size());
            std::memcpy(stage_n.p, buf.data(), buf.size());
            d_desc_n.ensure(buf.size());
            HIPCHK(hipMemcpyAsync(d_desc_n.p, stage_n.p, buf.size(), hipMemcpyHostToDevice, st));
            char* b = d_desc_n.as<char>();
            int32_t* inf = d_info.as<int32_t>();
            const int np = (int)nb.prep_s.size();
            // operand precision of the products on the matrix cores: W_k = S^-1 Mat(k->v)
            // applies the pivot and stays FP64; in mixed precision (when the
            // compression runs in FP32) the Schur GEMMs take FP32 operands with FP32
            // accumulation, and the projection B V FP32 operands, or BF16 ones in the
            // BF16 trial; the results are subtracted from / written to FP64 blocks
            const bool f32p = part[0]->fp32_compress;
            const int p_schur = f32p ? GP_F32 : GP_F64;
            const int p_proj = !f32p ? GP_F64 : (part[0]->h->precision == LRX_MIXED_BF16 ? GP_BF16 : GP_F32);
            auto gemm = [&](size_t og, size_t ot, const std::vector<DTile>& t, int kmax, int64_t fl, int prec) {
                if (t.empty()) return;
                LaunchTimer tm(LRX_K_SCHUR, st, 0.0, (double)fl);
                HIPCHK(gemm_products((const DGemm*)(b + og), (const DTile*)(b + ot), (int)t.size(), kmax, dmap, prec,
                                     st));
            };
            if (!tps.empty()) {                    // projection B V of every super-node (SVD)
                LaunchTimer tm(LRX_K_PROJECT, st, 0.0, (double)nb.gf_p);
                HIPCHK(gemm_products((const DGemm*)(b + o_gp), (const DTile*)(b + o_tp), (int)tps.size(), kps, dmap,
                                     p_proj, st));
            }
            // pivots above 128 rows: the blocked inverse over many work-groups,
            // its row order kept in d_gjperm (the previous step's use has completed
            // at the read-back)
            int* gjp = nullptr;
            if (std::max(nb.max_ms, nb.max_mb) > 128) {
                d_gjperm.ensure((size_t)np * kGjPermInts * sizeof(int32_t));
                gjp = d_gjperm.as<int32_t>();
            }
            {
                LaunchTimer tm(LRX_K_FACTOR_NODE, st, 0.0, (double)nb.pf_s);
                HIPCHK(launch_node_prep((const DPrep*)(b + o_ps), np, nb.max_ms, (const DProj*)(b + o_pj), dmap,
                                        inf, st, gjp));
            }
            gemm(o_g1s, o_t1s, t1s, k1s, 0, GP_F64);
            gemm(o_g2s, o_t2s, t2s, k2s, nb.gf_s, p_schur);
            {
                LaunchTimer tm(LRX_K_FACTOR_NODE, st, 0.0, (double)nb.pf_b);
                HIPCHK(launch_node_prep((const DPrep*)(b + o_pb), np, nb.max_mb, nullptr, dmap, inf, st, gjp));
            }
            gemm(o_g1b, o_t1b, t1b, k1b, 0, GP_F64);
            gemm(o_g2b, o_t2b, t2b, k2b, nb.gf_b, p_schur);
            t_h_node += now_ms() - tn0;
        }
    }
    sync();
    std::vector<int32_t> info(std::max(info_total, 1));
    HIPCHK(copy_sync(info.data(), d_info.p, info.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < runs.size(); ++i) {
        FactorRun& r = *runs[i];
        for (int32_t q = 0; q < r.info_count; ++q)
            if (info[r.info_base + q])
                fail(LRX_ESINGULAR, runs.size() > 1 ? "exactly singular pivot block in system " + std::to_string(i)
                                                    : std::string("exactly singular pivot block"));
        r.h->stats.factor_flops = r.flops;
        r.h->stats.flops_compress = r.fl_compress;
        r.h->stats.flops_pivot = r.fl_pivot;
        r.h->stats.flops_schur = r.fl_schur;
        r.h->stats.flops_project = r.fl_project;
        if (r.frob) {
            double st_h[35];
            HIPCHK(copy_sync(st_h, r.d_norm.p, sizeof(st_h), hipMemcpyDeviceToHost));
            for (int lv = 0; lv < 32 && lv <= r.P.depth; ++lv) r.h->stats.level_norm_by_level[lv] = st_h[2 + lv];
        }
        r.h->t_sync_ms += t_sync;
        r.h->stats.t_host_compress_ms = t_h_comp;
        r.h->stats.t_host_node_ms = t_h_node;
    }
    IdleScope idle;
    for (FactorRun* r : runs) {
        r->h->ws_b.release();
        r->h->ws_w.release();
    }
    for (DevBuf* d : {&d_imap, &d_info, &d_desc_m, &d_desc_c, &d_desc_n, &d_rt, &d_flags, &d_gjperm}) d->release();
    for (PinBuf* q : {&stage_m, &stage_c, &stage_n, &pin_rt, &pin_flags}) q->release();
}

// ------------------------------------------------------------------ solve program

void build_solve_program(lrx_handle h) {
    const double t_begin = now_ms();
    Plan& P = h->plan;
    const int32_t n = P.n;
    h->var_off.assign(P.nodes.size(), -1);
    for (size_t v = 0; v < P.nodes.size(); ++v)
        if (P.nodes[v].leaf) h->var_off[v] = P.nodes[v].dof0;
    int64_t off = n;
    // red nodes of each level in index order (siblings adjacent), black nodes after
    std::vector<std::vector<int32_t>> reds_by_level(P.depth + 1);
    for (size_t v = 0; v < P.nodes.size(); ++v)
        if (P.nodes[v].kind == NK_RED) reds_by_level[P.nodes[v].level].push_back((int32_t)v);
    for (int32_t lev = P.depth - 1; lev >= 0; --lev) {
        auto& R = reds_by_level[lev];
        std::sort(R.begin(), R.end(), [&](int32_t a, int32_t b) { return P.nodes[a].idx < P.nodes[b].idx; });
        for (int32_t v : R) { h->var_off[v] = off; off += std::max(h->size[v], 0); }
    }
    for (size_t v = 0; v < P.nodes.size(); ++v)
        if (P.nodes[v].kind == NK_BLACK) { h->var_off[v] = off; off += std::max(h->size[v], 0); }
    for (size_t v = 0; v < P.nodes.size(); ++v)
        if (P.nodes[v].kind == NK_SUPER && !P.nodes[v].leaf) {
            const PNode& nd = P.nodes[v];
            h->var_off[v] = h->var_off[nd.comp0];
            if (h->var_off[nd.comp1] != h->var_off[nd.comp0] + h->size[nd.comp0])
                fail(LRX_EDEVICE, "internal: sibling red nodes are not adjacent");
        }
    h->n_ext = off;

    // mixed precision: the solve reads FP32 copies of every block it uses (pivot
    // inverses and frozen edges); the FP64 factor is released afterwards
    const bool f32 = h->precision != LRX_FP64;
    const int32_t es = f32 ? 4 : 8;
    std::vector<const void*> sptr(P.edges.size(), nullptr);
    if (f32) {
        std::vector<char> usedf(P.edges.size(), 0), pivf(P.edges.size(), 0);
        for (const ColourStep& cs : P.steps)
            for (const NodeStep& ns : cs.nodes)
                for (const PivotPlan* pp : {&ns.ps, &ns.pb}) {
                    if (pp->e_self >= 0) pivf[pp->e_self] = 1;
                    for (int32_t e : pp->out_edges) usedf[e] = 1;
                    for (int32_t e : pp->in_edges) usedf[e] = 1;
                }
        std::vector<DConv> segs;
        for (size_t e = 0; e < P.edges.size(); ++e) {
            if ((!usedf[e] && !pivf[e]) || !h->eptr[e]) continue;
            const PEdge& E = P.edges[e];
            const int64_t cnt = (int64_t)dim_of(E.rows, h->size[E.dst]) * dim_of(E.cols, h->size[E.src]);
            if (cnt <= 0) continue;
            if (pivf[e]) {                 // pivot inverses stay FP64
                double* d = h->arena32.alloc((size_t)cnt);
                segs.push_back(DConv{h->eptr[e], d, cnt, 1, 0});
                sptr[e] = d;
                continue;
            }
            float* d = (float*)h->arena32.alloc((size_t)(cnt + 1) / 2);
            segs.push_back(DConv{h->eptr[e], d, cnt, 0, 0});
            sptr[e] = d;
        }
        DevBuf dsegs;
        dsegs.ensure(std::max<size_t>(segs.size(), 1) * sizeof(DConv));
        if (!segs.empty()) {
            HIPCHK(copy_sync(dsegs.p, segs.data(), segs.size() * sizeof(DConv), hipMemcpyHostToDevice));
            HIPCHK(launch_to_f32(dsegs.as<DConv>(), (int)segs.size(), h->stream));
        }
        HIPCHK(hipStreamSynchronize(h->stream));      // dsegs is released at scope end
        h->solve_fp32 = true;
    } else {
        for (size_t e = 0; e < P.edges.size(); ++e) sptr[e] = h->eptr[e];
    }

    // per super-node (in colour-step order): the intermediate form of both
    // pivots with their frozen out-edges (forward) and in-edges (backward), then
    // its two programs; nodes are independent, so host threads share them
    struct NodeRef { int32_t step, node; };
    std::vector<NodeRef> refs;
    h->ssteps.assign(P.steps.size(), SolveStep{});
    for (size_t si = 0; si < P.steps.size(); ++si) {
        h->ssteps[si].node0 = (int32_t)refs.size();
        for (size_t ni = 0; ni < P.steps[si].nodes.size(); ++ni) refs.push_back({(int32_t)si, (int32_t)ni});
        h->ssteps[si].nnode = (int32_t)refs.size() - h->ssteps[si].node0;
    }
    const size_t nn = refs.size();
    struct NodeOut {
        std::vector<int32_t> words;
        SwNodeRel f{}, b{};
        int64_t bytes_fwd = 0, bytes_bwd = 0, solve_bytes = 0;
        std::string err;
    };
    std::vector<NodeOut> outs(nn);
    auto local = [](const Support& s) { return s.all ? std::vector<int32_t>() : s.idx; };
    auto work = [&](size_t i) {
        NodeOut& o = outs[i];
        const NodeStep& ns = P.steps[refs[i].step].nodes[refs[i].node];
        auto piv = [&](const PivotPlan& pp) {
            SwPivIR D;
            const int32_t v = pp.node;
            D.node = v;
            D.m = pp.e_self >= 0 ? h->size[v] : 0;
            D.off = h->var_off[v];
            D.inv = pp.e_self >= 0 ? sptr[pp.e_self] : nullptr;
            o.solve_bytes += 2ll * D.m * D.m * 8;
            for (int pass = 0; pass < 2; ++pass) {
                const auto& list = pass == 0 ? pp.out_edges : pp.in_edges;
                for (int32_t e : list) {
                    const PEdge& E = P.edges[e];
                    SwEdgeIR s;
                    s.E = sptr[e];
                    s.nr = dim_of(E.rows, h->size[E.dst]);
                    s.nc = dim_of(E.cols, h->size[E.src]);
                    if ((int64_t)s.nr * s.nc == 0) continue;
                    s.other = pass == 0 ? E.dst : E.src;
                    s.other_off = h->var_off[s.other];
                    s.rows = local(E.rows);
                    s.cols = local(E.cols);
                    o.solve_bytes += (int64_t)s.nr * s.nc * es;
                    (pass == 0 ? D.out : D.in).push_back(std::move(s));
                }
            }
            return D;
        };
        SwNodeIR d;
        d.es = es;
        d.es_piv = 8;
        d.s = piv(ns.ps);
        d.b = piv(ns.pb);
        for (const SwPivIR* pv : {&d.s, &d.b}) {
            const int64_t pivb = (int64_t)pv->m * pv->m * 8;
            int64_t ob = 0, ib = 0;
            for (auto& e : pv->out) ob += (int64_t)e.nr * e.nc * es;
            for (auto& e : pv->in) ib += (int64_t)e.nr * e.nc * es;
            o.bytes_fwd += pivb + ob;
            o.bytes_bwd += pivb + ib;
        }
        if (!build_node_programs(d, o.words, o.f, o.b, o.err) && o.err.empty()) o.err = "solve sweep";
    };
    {
        const size_t nth = std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
        std::atomic<size_t> next{0};
        auto loop = [&]() {
            for (size_t i; (i = next.fetch_add(1)) < nn;) {
                try {
                    work(i);
                } catch (const std::exception& e) {
                    outs[i].err = std::string("solve sweep: ") + e.what();
                }
            }
        };
        std::vector<std::thread> pool;
        for (size_t t = 1; t < nth && t < nn; ++t) pool.emplace_back(loop);
        loop();
        for (auto& t : pool) t.join();
    }
    int64_t solve_bytes = 0;
    std::vector<int32_t> words;
    std::vector<SwNodeRel> both(2 * nn);
    h->sw_stages = 0;
    for (size_t i = 0; i < nn; ++i) {
        NodeOut& o = outs[i];
        if (!o.err.empty()) fail(LRX_EDEVICE, o.err);
        if (words.size() & 1) words.push_back(0);
        const int64_t base = (int64_t)words.size();
        words.insert(words.end(), o.words.begin(), o.words.end());
        both[i] = o.f;
        both[nn + i] = o.b;
        both[i].desc += base;
        both[nn + i].desc += base;
        solve_bytes += o.solve_bytes;
        SolveStep& ss = h->ssteps[refs[i].step];
        ss.bytes_fwd += o.bytes_fwd;
        ss.bytes_bwd += o.bytes_bwd;
        h->sw_stages += o.f.nstage + o.b.nstage;
    }
    h->d_swnodes.ensure(std::max<size_t>(2 * nn, 1) * sizeof(SwNode));
    h->d_swprog.ensure(std::max<size_t>(words.size(), 1) * sizeof(int32_t));
    if (!words.empty())
        HIPCHK(copy_sync(h->d_swprog.p, words.data(), words.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    h->sw_host.resize(2 * nn);
    for (size_t i = 0; i < 2 * nn; ++i)
        h->sw_host[i] = SwNode{h->d_swprog.as<int32_t>() + both[i].desc, nullptr, nullptr, both[i].words0,
                              both[i].nstage};
    if (nn)
        HIPCHK(copy_sync(h->d_swnodes.p, h->sw_host.data(), h->sw_host.size() * sizeof(SwNode),
                         hipMemcpyHostToDevice));
    for (size_t si = 0; si < P.steps.size(); ++si) {
        h->ssteps[si].height = P.depth - P.steps[si].level;
        h->ssteps[si].colour = P.steps[si].colour;
    }
    h->sw_words = (int64_t)words.size();
    h->sw_nnode = (int32_t)nn;
    h->stats.solve_bytes = solve_bytes;
    h->stats.sweep_stages = h->sw_stages;
    h->stats.sweep_launches = 2 * (int64_t)h->plan.steps.size();
    if (h->solve_fp32) {               // the FP64 blocks are no longer read
        HIPCHK(hipStreamSynchronize(h->stream));
        IdleScope idle;
        h->arena.release();
        std::fill(h->eptr.begin(), h->eptr.end(), nullptr);
    }
    h->t_solve_prog_ms = now_ms() - t_begin;
}

// Right-hand sides per sweep work-group for rem remaining: the largest of 8, 4,
// 2, 1 that fits, capped by the tuning table.
int sweep_nk(int rem) {
    const int cap = g_tune.sweep_nk_max;
    for (int nk = kSwKS; nk > 1; nk >>= 1)
        if (nk <= cap && rem >= nk) return nk;
    return 1;
}

constexpr int kDeviceCUs = 256;

// One colour step of a sweep over all nrhs right-hand sides: the right-hand
// sides are split into slices that run side by side (a work-group per node and
// slice), with smaller slices while the node count leaves compute units idle;
// f(k0, nk, ns) issues one launch of ns slices of nk from k0.  The arithmetic of
// each right-hand side does not depend on the slicing.
template <class Fn>
void sweep_step(int nnode, int nrhs, Fn&& f) {
    const int target = std::max(1, kDeviceCUs / std::max(nnode, 1));
    for (int c0 = 0; c0 < nrhs;) {
        const int rem = nrhs - c0;
        int nk = sweep_nk(rem);
        while (nk > 1 && rem / (nk / 2) <= target) nk /= 2;
        const int ns = rem / nk;
        f(c0, nk, ns);
        c0 += nk * ns;
    }
}

// x_ext (n_ext x nrhs interleaved) -> in place sweeps.  timed = false records
// no events (the allocation-free path creates nothing).
void sweeps(lrx_handle h, double* xe, int nrhs, bool timed = true) {
    const hipStream_t st = h->stream;
    const SwNode* fwd = h->d_swnodes.as<SwNode>();
    const SwNode* bwd = fwd + h->sw_nnode;
    for (const SolveStep& s : h->ssteps)
        sweep_step(s.nnode, nrhs, [&](int k0, int nk, int ns) {
            LaunchTimer tm(timed ? LRX_K_SOLVE_FWD : -1, st, (double)s.bytes_fwd, (double)s.bytes_fwd / 4.0 * nk * ns);
            HIPCHK(launch_sweep(fwd + s.node0, s.nnode, xe, nrhs, k0, nk, ns, st));
        });
    for (auto it = h->ssteps.rbegin(); it != h->ssteps.rend(); ++it)
        sweep_step(it->nnode, nrhs, [&](int k0, int nk, int ns) {
            LaunchTimer tm(timed ? LRX_K_SOLVE_BWD : -1, st, (double)it->bytes_bwd, (double)it->bytes_bwd / 4.0 * nk * ns);
            HIPCHK(launch_sweep(bwd + it->node0, it->nnode, xe, nrhs, k0, nk, ns, st));
        });
}

// Algorithms 2-4 with the extended vector in xe (n_ext x nrhs): SetRHS (b in
// tree order, auxiliary variables zeroed by the same kernel), SolveL, SolveU,
// SplitVar (nothing to do: a super-node's variables are its reds'), x.
void solve_into(lrx_handle h, int nrhs, const double* b, double* x, double* xe, bool timed) {
    const hipStream_t st = h->stream;
    const int32_t n = h->plan.n;
    HIPCHK(launch_gather_perm(b, n, h->d_perm.as<int32_t>(), n, nrhs, xe, h->n_ext, st));
    sweeps(h, xe, nrhs, timed);
    HIPCHK(launch_scatter_perm(xe, h->d_perm.as<int32_t>(), n, nrhs, x, n, st));
}

void solve_dev(lrx_handle h, int nrhs, const double* b, double* x) {
    h->x_ext.ensure((size_t)h->n_ext * nrhs * 8);
    solve_into(h, nrhs, b, x, h->x_ext.as<double>(), true);
}

// Algorithms 2-4 for k factorizations at once: one sweep launch per (height,
// colour) step covers the nodes of every factorization that has that step (the
// factorizations share nothing, so their steps commute).  Synchronous.
void solve_batch_dev(int k, const lrx_handle* hs, int nrhs, const double* const* b, double* const* x) {
    const lrx_handle h0 = hs[0];
    const hipStream_t st = h0->stream;
    std::vector<std::pair<int32_t, int32_t>> keys;
    for (int i = 0; i < k; ++i)
        for (const SolveStep& s : hs[i]->ssteps) keys.push_back({s.height, s.colour});
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    // extended vectors, then per step the nodes of every factorization
    std::vector<double*> xe(k);
    for (int i = 0; i < k; ++i) {
        const lrx_handle h = hs[i];
        h->x_ext.ensure((size_t)h->n_ext * nrhs * 8);
        xe[i] = h->x_ext.as<double>();
    }
    std::vector<SwNode> nf, nb;
    std::vector<int32_t> k0f, k0b;
    for (const auto& key : keys) {
        k0f.push_back((int32_t)nf.size());
        for (int i = 0; i < k; ++i) {
            const lrx_handle h = hs[i];
            for (const SolveStep& s : h->ssteps) {
                if (s.height != key.first || s.colour != key.second) continue;
                for (int32_t j = 0; j < s.nnode; ++j) {
                    SwNode a = h->sw_host[s.node0 + j];
                    SwNode c = h->sw_host[h->sw_nnode + s.node0 + j];
                    a.x = c.x = xe[i];
                    nf.push_back(a);
                    nb.push_back(c);
                }
            }
        }
    }
    k0f.push_back((int32_t)nf.size());
    h0->batch_nodes.ensure(std::max<size_t>(2 * nf.size(), 1) * sizeof(SwNode));
    SwNode* dn = h0->batch_nodes.as<SwNode>();
    if (!nf.empty()) {
        HIPCHK(copy_sync(dn, nf.data(), nf.size() * sizeof(SwNode), hipMemcpyHostToDevice));
        HIPCHK(copy_sync(dn + nf.size(), nb.data(), nb.size() * sizeof(SwNode), hipMemcpyHostToDevice));
    }
    for (int i = 0; i < k; ++i) {
        const lrx_handle h = hs[i];
        const int32_t n = h->plan.n;
        HIPCHK(launch_gather_perm(b[i], n, h->d_perm.as<int32_t>(), n, nrhs, xe[i], h->n_ext, st));
    }
    for (size_t q = 0; q + 1 < k0f.size(); ++q)
        sweep_step(k0f[q + 1] - k0f[q], nrhs, [&](int c0, int nk, int ns) {
            HIPCHK(launch_sweep(dn + k0f[q], k0f[q + 1] - k0f[q], nullptr, nrhs, c0, nk, ns, st));
        });
    for (size_t q = k0f.size() - 1; q-- > 0;)
        sweep_step(k0f[q + 1] - k0f[q], nrhs, [&](int c0, int nk, int ns) {
            HIPCHK(launch_sweep(dn + nf.size() + k0f[q], k0f[q + 1] - k0f[q], nullptr, nrhs, c0, nk, ns, st));
        });
    for (int i = 0; i < k; ++i) {
        const lrx_handle h = hs[i];
        const int32_t n = h->plan.n;
        HIPCHK(launch_scatter_perm(xe[i], h->d_perm.as<int32_t>(), n, nrhs, x[i], n, st));
    }
    HIPCHK(hipStreamSynchronize(st));
}

// ------------------------------------------------------------------ GMRES
bool timing_on(int cls) {
    std::lock_guard<std::mutex> lk(g_tmu);
    return (g_timing & (1u << cls)) != 0;
}

// A captured preconditioner: ends an unfinished capture and releases the graph
// once the stream has run every replay.
struct SolveGraph {
    hipStream_t st;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    bool capturing = false;
    explicit SolveGraph(hipStream_t s) : st(s) {}
    ~SolveGraph() {
        if (capturing) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(st, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
        }
        if (exec || g) (void)hipStreamSynchronize(st);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (g) (void)hipGraphDestroy(g);
    }
};
// FGMRES(restart) with the solve as right preconditioner (Sec. 6.2), x_0 = 0,
// for k factorizations at once, nrhs right-hand sides each.  Every vector
// operation is one launch over the row chunks of all systems still iterating
// (DKry/DKryChunk tables); the preconditioner is one sweep launch per
// (height, colour) step over the nodes of all of them; the Hessenberg columns of
// all systems cross to the host with one copy per Arnoldi step.  Each right-hand
// side stops on its own true relative residual; a system whose right-hand sides
// have all stopped drops out of the launches (its act flag).  k = 1 is the
// single-system solver.
lrx_status gmres_batch(int K, const lrx_handle* hs, int nrhs, const double* const* b, double* const* x,
                       double tol, int restart, int maxit, int32_t* iters_out, double* relres_out,
                       bool use_x0 = false) {
    const lrx_handle h0 = hs[0];
    const hipStream_t st = h0->stream;
    const int m = restart;
    const int rc = kry_rows(nrhs);
    // scalars of one system: h1 | h2 | n2 | y | J
    const int o_h1 = 0, o_h2 = (m + 1) * nrhs, o_n2 = 2 * (m + 1) * nrhs, o_y = o_n2 + nrhs;
    const int o_J = o_y + (m + 1) * nrhs;
    const int smsz = (o_J + 1 + 3) & ~3;
    std::vector<DKry> sys(K);
    std::vector<DKryChunk> chunks;
    double nnz_bytes = 0.0, spmv_flops = 0.0;
    h0->kry_small.ensure((size_t)K * smsz * 8);
    for (int s = 0; s < K; ++s) {
        const lrx_handle h = hs[s];
        const int32_t n = h->plan.n;
        const int64_t nv = (int64_t)n * nrhs;
        h->g_basis.ensure((size_t)(m + 1) * nv * 8);
        h->g_z.ensure((size_t)m * nv * 8);
        h->g_w.ensure((size_t)nv * 8);
        h->g_r.ensure((size_t)nv * 8);
        h->g_b.ensure((size_t)nv * 8);
        h->g_x.ensure((size_t)nv * 8);
        h->x_ext.ensure((size_t)h->n_ext * nrhs * 8);
        DKry& S = sys[s];
        S.n = n;
        S.nv = nv;
        S.n_ext = h->n_ext;
        S.rp = h->d_rp.as<int64_t>();
        S.ci = h->d_ci.as<int32_t>();
        S.av = h->d_val.as<double>();
        S.perm = h->d_perm.as<int32_t>();
        S.V = h->g_basis.as<double>();
        S.Z = h->g_z.as<double>();
        S.w = h->g_w.as<double>();
        S.r = h->g_r.as<double>();
        S.b = h->g_b.as<double>();
        S.x = h->g_x.as<double>();
        S.xe = h->x_ext.as<double>();
        S.sm = h0->kry_small.as<double>() + (size_t)s * smsz;
        S.bin = b[s];
        S.xout = x[s];
        S.chunk0 = (int32_t)chunks.size();
        for (int32_t r0 = 0; r0 < n; r0 += rc) chunks.push_back(DKryChunk{s, r0});
        S.nchunk = (int32_t)chunks.size() - S.chunk0;
        nnz_bytes += (double)h->nnz * 12 + (double)(n + 1) * 8 + 2.0 * nv * 8;
        spmv_flops += 2.0 * (double)h->nnz * nrhs;
    }
    if (chunks.size() > (size_t)INT32_MAX) fail(LRX_EINVAL, "too many rows in the batch");
    h0->kry_part.ensure(std::max<size_t>(chunks.size(), 1) * (size_t)(m + 1) * nrhs * 8);
    double* part = h0->kry_part.as<double>();
    // device tables: systems | chunks | act
    const size_t o_ch = ((size_t)K * sizeof(DKry) + 255) & ~(size_t)255;
    const size_t o_act = (o_ch + chunks.size() * sizeof(DKryChunk) + 255) & ~(size_t)255;
    h0->kry_tab.ensure(o_act + (size_t)K * 4);
    HIPCHK(copy_sync(h0->kry_tab.p, sys.data(), (size_t)K * sizeof(DKry), hipMemcpyHostToDevice));
    if (!chunks.empty())
        HIPCHK(copy_sync(h0->kry_tab.as<char>() + o_ch, chunks.data(), chunks.size() * sizeof(DKryChunk),
                         hipMemcpyHostToDevice));
    int32_t* act_dev = (int32_t*)(h0->kry_tab.as<char>() + o_act);
    // pinned mirror: scalars of every system, then act
    const size_t pin_act = (size_t)K * smsz * 8;
    h0->kry_pin.ensure(pin_act + (size_t)K * 4);
    double* hsm = (double*)h0->kry_pin.p;
    int32_t* act = (int32_t*)((char*)h0->kry_pin.p + pin_act);
    const KryLaunch L{(const DKry*)h0->kry_tab.p, (const DKryChunk*)(h0->kry_tab.as<char>() + o_ch), act_dev,
                      (int)chunks.size(), K, nrhs, rc, st};
    auto put_act = [&]() {
        HIPCHK(hipMemcpyAsync(act_dev, act, (size_t)K * 4, hipMemcpyHostToDevice, st));
    };
    auto get_small = [&]() {
        HIPCHK(hipMemcpyAsync(hsm, h0->kry_small.p, (size_t)K * smsz * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    };
    auto put_small = [&]() {
        HIPCHK(hipMemcpyAsync(h0->kry_small.p, hsm, (size_t)K * smsz * 8, hipMemcpyHostToDevice, st));
    };
    // preconditioner: node lists of both sweeps over all systems, each node
    // skipped when its system's act flag is 0
    std::vector<std::pair<int32_t, int32_t>> keys;
    for (int s = 0; s < K; ++s)
        for (const SolveStep& q : hs[s]->ssteps) keys.push_back({q.height, q.colour});
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    std::vector<SwNode> nf, nb;
    std::vector<int32_t> k0f;
    std::vector<double> step_bytes_f, step_bytes_b;
    for (const auto& key : keys) {
        k0f.push_back((int32_t)nf.size());
        double bf = 0, bb = 0;
        for (int s = 0; s < K; ++s) {
            const lrx_handle h = hs[s];
            for (const SolveStep& q : h->ssteps) {
                if (q.height != key.first || q.colour != key.second) continue;
                bf += (double)q.bytes_fwd;
                bb += (double)q.bytes_bwd;
                for (int32_t j = 0; j < q.nnode; ++j) {
                    SwNode a = h->sw_host[q.node0 + j];
                    SwNode c = h->sw_host[h->sw_nnode + q.node0 + j];
                    a.x = c.x = sys[s].xe;
                    a.live = c.live = act_dev + s;
                    nf.push_back(a);
                    nb.push_back(c);
                }
            }
        }
        step_bytes_f.push_back(bf);
        step_bytes_b.push_back(bb);
    }
    k0f.push_back((int32_t)nf.size());
    h0->batch_nodes.ensure(std::max<size_t>(2 * nf.size(), 1) * sizeof(SwNode));
    SwNode* dn = h0->batch_nodes.as<SwNode>();
    if (!nf.empty()) {
        HIPCHK(copy_sync(dn, nf.data(), nf.size() * sizeof(SwNode), hipMemcpyHostToDevice));
        HIPCHK(copy_sync(dn + nf.size(), nb.data(), nb.size() * sizeof(SwNode), hipMemcpyHostToDevice));
    }
    auto sweep_launches = [&](bool timed) {
        for (size_t q = 0; q + 1 < k0f.size(); ++q)
            sweep_step(k0f[q + 1] - k0f[q], nrhs, [&](int c0, int nk, int ns) {
                LaunchTimer tm(timed ? LRX_K_SOLVE_FWD : -1, st, step_bytes_f[q], step_bytes_f[q] / 4.0 * nk * ns);
                HIPCHK(launch_sweep(dn + k0f[q], k0f[q + 1] - k0f[q], nullptr, nrhs, c0, nk, ns, st));
            });
        for (size_t q = k0f.size() - 1; q-- > 0;)
            sweep_step(k0f[q + 1] - k0f[q], nrhs, [&](int c0, int nk, int ns) {
                LaunchTimer tm(timed ? LRX_K_SOLVE_BWD : -1, st, step_bytes_b[q], step_bytes_b[q] / 4.0 * nk * ns);
                HIPCHK(launch_sweep(dn + nf.size() + k0f[q], k0f[q + 1] - k0f[q], nullptr, nrhs, c0, nk, ns, st));
            });
    };
    // The preconditioner is the same launch sequence at every Arnoldi step (the
    // node tables, vectors and act flags it reads stay where they are), so after
    // one direct application it is captured once into a HIP graph and replayed.
    // Only on a non-blocking stream (the null stream cannot be captured, and
    // null-stream work of other threads would synchronize with a blocking one),
    // and not while its launches are being event-timed.
    SolveGraph graph(st);
    unsigned int sflags = 0;
    const bool use_graph = g_tune.solve_graph && st != nullptr && hipStreamGetFlags(st, &sflags) == hipSuccess &&
                           (sflags & hipStreamNonBlocking) && !timing_on(LRX_K_SOLVE_FWD) &&
                           !timing_on(LRX_K_SOLVE_BWD);
    int applications = 0;
    auto precondition = [&]() {
        if (!use_graph || applications++ == 0) {
            sweep_launches(true);
            return;
        }
        if (!graph.exec) {
            std::unique_lock<std::shared_mutex> lk(g_capture_mu);
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            graph.capturing = true;
            sweep_launches(false);
            graph.capturing = false;
            HIPCHK(hipStreamEndCapture(st, &graph.g));
            lk.unlock();
            HIPCHK(hipGraphInstantiate(&graph.exec, graph.g, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(graph.exec, st));
    };

    // host state per (system, right-hand side)
    const size_t KR = (size_t)K * nrhs;
    std::vector<double> bnorm(KR, 0.0), relres(KR, 0.0);
    std::vector<int32_t> its(KR, 0), kk(KR, 0);
    std::vector<char> active(KR, 0), conv(KR, 0), done(KR, 1);
    for (int s = 0; s < K; ++s) hs[s]->gmres_hist.assign((size_t)nrhs, {});
    std::vector<double> H(KR * (m + 1) * m), cs(KR * m), sn(KR * m), g(KR * (m + 1));
    std::vector<char> in_cycle(K, 1);
    for (int s = 0; s < K; ++s) act[s] = 1;
    put_act();
    HIPCHK(kry_perm(L, 0));                   // b in tree order, x = 0
    bool first = true;
    if (use_x0) {
        // ||b|| from the residual of x = 0, then x = the caller's initial guess
        HIPCHK(kry_spmv(L, true, 0));
        HIPCHK(kry_dots(L, 2, 1, part, o_n2));
        get_small();
        for (int s = 0; s < K; ++s)
            for (int k = 0; k < nrhs; ++k) {
                const size_t q = (size_t)s * nrhs + k;
                bnorm[q] = std::sqrt(hsm[(size_t)s * smsz + o_n2 + k]);
                active[q] = bnorm[q] > 0.0;
                conv[q] = !active[q];
            }
        HIPCHK(kry_perm(L, 2, o_n2));
        first = false;
    }
    while (true) {
        HIPCHK(kry_spmv(L, true, 0));          // r = b - A x
        HIPCHK(kry_dots(L, 2, 1, part, o_n2));
        get_small();
        bool any = false;
        for (int s = 0; s < K; ++s) {
            in_cycle[s] = 0;
            if (!act[s]) continue;
            const double* n2 = hsm + (size_t)s * smsz + o_n2;
            for (int k = 0; k < nrhs; ++k) {
                const size_t q = (size_t)s * nrhs + k;
                if (first) {
                    bnorm[q] = std::sqrt(n2[k]);
                    active[q] = bnorm[q] > 0.0;
                    conv[q] = !active[q];
                }
                if (bnorm[q] == 0.0) continue;
                relres[q] = std::sqrt(n2[k]) / bnorm[q];
                if (!active[q]) continue;
                hs[s]->gmres_hist[k].push_back(relres[q]);
                if (relres[q] <= tol) { active[q] = 0; conv[q] = 1; }
                else if (its[q] >= maxit) active[q] = 0;
                if (active[q]) in_cycle[s] = 1;
            }
            any |= in_cycle[s] != 0;
        }
        first = false;
        if (!any) break;
        // systems with an active right-hand side take part in this cycle;
        // V_0 = r / ||r|| for active right-hand sides, 0 otherwise
        for (int s = 0; s < K; ++s) {
            act[s] = in_cycle[s];
            if (!act[s]) continue;
            double* n2 = hsm + (size_t)s * smsz + o_n2;
            for (int k = 0; k < nrhs; ++k) {
                const size_t q = (size_t)s * nrhs + k;
                if (!active[q]) n2[k] = 0.0;
                double* gq = g.data() + q * (m + 1);
                std::fill(gq, gq + m + 1, 0.0);
                gq[0] = active[q] ? std::sqrt(n2[k]) : 0.0;
                kk[q] = 0;
                done[q] = !active[q];
            }
        }
        put_act();
        put_small();
        HIPCHK(kry_axpy(L, 2, 0, 0, o_n2, 0));
        for (int j = 0; j < m; ++j) {
            HIPCHK(kry_axpy(L, 3, 0, j, 0, 0));          // xe = [V_j; 0]
            precondition();
            HIPCHK(kry_axpy(L, 4, 0, j, 0, 0));          // Z_j = M^{-1} V_j
            {
                LaunchTimer tm(LRX_K_SPMV, st, nnz_bytes, spmv_flops);
                HIPCHK(kry_spmv(L, false, j));           // w = A Z_j
            }
            // classical Gram-Schmidt, twice
            HIPCHK(kry_dots(L, 0, j + 1, part, o_h1));
            HIPCHK(kry_axpy(L, 0, j + 1, 0, o_h1, 0));
            HIPCHK(kry_dots(L, 0, j + 1, part, o_h2));
            HIPCHK(kry_axpy(L, 0, j + 1, 0, o_h2, 0));
            HIPCHK(kry_dots(L, 1, 1, part, o_n2));
            HIPCHK(kry_axpy(L, 2, 1, j + 1, o_n2, 0));   // V_{j+1} = w / ||w||
            get_small();
            bool all_done = true, act_changed = false;
            for (int s = 0; s < K; ++s) {
                if (!act[s]) continue;
                const double* sm = hsm + (size_t)s * smsz;
                const double* h1 = sm + o_h1;
                const double* h2 = sm + o_h2;
                const double* n2 = sm + o_n2;
                bool sys_done = true;
                for (int k = 0; k < nrhs; ++k) {
                    const size_t q = (size_t)s * nrhs + k;
                    if (done[q]) continue;
                    double* Hk = H.data() + q * (m + 1) * m;   // Hk[i*m + j]
                    double* gk = g.data() + q * (m + 1);
                    double* ck = cs.data() + q * m;
                    double* sk = sn.data() + q * m;
                    for (int i = 0; i <= j; ++i) Hk[i * m + j] = h1[i * nrhs + k] + h2[i * nrhs + k];
                    Hk[(j + 1) * m + j] = std::sqrt(std::max(n2[k], 0.0));
                    for (int i = 0; i < j; ++i) {
                        const double t = ck[i] * Hk[i * m + j] + sk[i] * Hk[(i + 1) * m + j];
                        Hk[(i + 1) * m + j] = -sk[i] * Hk[i * m + j] + ck[i] * Hk[(i + 1) * m + j];
                        Hk[i * m + j] = t;
                    }
                    const double a = Hk[j * m + j], bb = Hk[(j + 1) * m + j];
                    const double den = std::hypot(a, bb);
                    ck[j] = den != 0.0 ? a / den : 1.0;
                    sk[j] = den != 0.0 ? bb / den : 0.0;
                    Hk[j * m + j] = den;
                    Hk[(j + 1) * m + j] = 0.0;
                    gk[j + 1] = -sk[j] * gk[j];
                    gk[j] = ck[j] * gk[j];
                    its[q] += 1;
                    kk[q] = j + 1;
                    hs[s]->gmres_hist[k].push_back(std::fabs(gk[j + 1]) / bnorm[q]);
                    if (std::fabs(gk[j + 1]) <= tol * bnorm[q] || its[q] >= maxit || den == 0.0) done[q] = 1;
                    else sys_done = false;
                }
                if (sys_done) { act[s] = 0; act_changed = true; }
                else all_done = false;
            }
            if (all_done) break;
            if (act_changed) put_act();
        }
        // y from the triangular systems, then x += Z y for the systems of this cycle
        for (int s = 0; s < K; ++s) {
            act[s] = in_cycle[s];
            if (!act[s]) continue;
            double* sm = hsm + (size_t)s * smsz;
            double* y = sm + o_y;
            std::fill(y, y + (size_t)(m + 1) * nrhs, 0.0);
            int J = 0;
            for (int k = 0; k < nrhs; ++k) {
                const size_t q = (size_t)s * nrhs + k;
                if (!active[q] || kk[q] == 0) continue;
                const double* Hk = H.data() + q * (m + 1) * m;
                const double* gk = g.data() + q * (m + 1);
                std::vector<double> yk(kk[q]);
                for (int i = kk[q] - 1; i >= 0; --i) {
                    double t = gk[i];
                    for (int c = i + 1; c < kk[q]; ++c) t -= Hk[i * m + c] * yk[c];
                    yk[i] = Hk[i * m + i] != 0.0 ? t / Hk[i * m + i] : 0.0;
                }
                for (int i = 0; i < kk[q]; ++i) y[(size_t)i * nrhs + k] = yk[i];
                J = std::max(J, kk[q]);
            }
            sm[o_J] = (double)J;
        }
        put_act();
        put_small();
        HIPCHK(kry_axpy(L, 1, 0, 0, o_y, o_J));
    }
    for (int s = 0; s < K; ++s) act[s] = 1;
    put_act();
    HIPCHK(kry_perm(L, 1));                   // x in the original order
    HIPCHK(hipStreamSynchronize(st));
    bool all_conv = true;
    for (size_t q = 0; q < KR; ++q) {
        if (iters_out) iters_out[q] = its[q];
        if (relres_out) relres_out[q] = relres[q];
        if (!conv[q]) all_conv = false;
    }
    return all_conv ? LRX_OK : LRX_ENOCONV;
}

lrx_status gmres_dev(lrx_handle h, int nrhs, const double* b, double* x, double tol, int restart, int maxit,
                     int32_t* iters_out, double* relres_out) {
    return gmres_batch(1, &h, nrhs, &b, &x, tol, restart, maxit, iters_out, relres_out);
}

template <class F> lrx_status guarded(F&& f) {
    try {
        g_err.clear();
        return f();
    } catch (const Fail& e) {
        g_err = e.msg;
        return e.st;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return LRX_ENOMEM;
    } catch (...) {
        g_err = "unexpected exception";
        return LRX_EDEVICE;
    }
}

}  // namespace

// ====================================================================== C ABI
namespace {

void check_factor_args(const lrx_csr* A, const double* val_dev, const lrx_tree* T, const lrx_opts* o) {
    if (!T || !o) fail(LRX_EINVAL, "null tree or options");
    if (val_dev) {
        if (!A || A->n < 1 || A->nnz < 0 || !A->row_ptr || !A->col_idx) fail(LRX_EINVAL, "bad CSR pattern");
    } else {
        check_csr(A);
    }
    if (!(o->epsilon >= 0.0 && o->epsilon < 1.0)) fail(LRX_EINVAL, "epsilon must be in [0, 1)");
    if (o->precision != LRX_FP64 && o->precision != LRX_MIXED && o->precision != LRX_MIXED_BF16)
        fail(LRX_EINVAL, "precision must be LRX_FP64, LRX_MIXED or LRX_MIXED_BF16");
    if (o->compress != LRX_SVD && o->compress != LRX_RRQR && o->compress != LRX_RAND)
        fail(LRX_EINVAL, "unknown compress method");
    if (o->rule != LRX_RULE_CUTOFF1 && o->rule != LRX_RULE_FROB) fail(LRX_EINVAL, "unknown truncation rule");
    if (o->rule == LRX_RULE_FROB && o->compress == LRX_RAND)
        fail(LRX_EINVAL, "the randomized range finder takes the relative rule only");
    if (o->symmetric != 0 && o->symmetric != 1) fail(LRX_EINVAL, "symmetric must be 0 or 1");
    if (o->hbm_budget_bytes < 0) fail(LRX_EINVAL, "negative hbm budget");
}

// The half stack needs A = A^T entry for entry (values on the host, or copied
// from the device).
void check_symmetric(const lrx_csr* A, const double* val_dev) {
    std::vector<double> vh;
    const double* v = A->val;
    if (val_dev) {
        vh.resize((size_t)A->nnz);
        if (A->nnz) HIPCHK(copy_sync(vh.data(), val_dev, (size_t)A->nnz * 8, hipMemcpyDeviceToHost));
        v = vh.data();
    }
    for (int32_t r = 0; r < A->n; ++r)
        for (int64_t e = A->row_ptr[r]; e < A->row_ptr[r + 1]; ++e) {
            const int32_t c = A->col_idx[e];
            if (c < 0 || c >= A->n) fail(LRX_EINVAL, "column index out of range");
            const int32_t* b = A->col_idx + A->row_ptr[c];
            const int32_t* en = A->col_idx + A->row_ptr[c + 1];
            const int32_t* it = std::lower_bound(b, en, r);
            if (it == en || *it != r || v[A->row_ptr[c] + (it - b)] != v[e])
                fail(LRX_EINVAL, "symmetric: A is not symmetric");
        }
}

// Options, device, and A in tree order (for the GMRES products) of a handle
// whose plan is built.
void init_handle(lrx_handle h, const lrx_csr* A, const double* val_dev, const lrx_opts* o) {
    HIPCHK(hipGetDevice(&h->device));
    ensure_gfx950(h->device);
    h->stream = (hipStream_t)o->stream;
    h->epsilon = o->epsilon;
    h->compress = o->compress;
    h->rule = o->rule;
    h->symmetric = o->symmetric != 0;
    if (h->symmetric) check_symmetric(A, val_dev);
    h->precision = o->precision;
    h->arena.budget_bytes = o->hbm_budget_bytes;
    const int32_t n = A->n;
    const Plan& P = h->plan;
    std::vector<int64_t> rp(n + 1, 0);
    std::vector<int32_t> ci((size_t)A->nnz);
    std::vector<int64_t> src_of((size_t)A->nnz);
    for (int32_t t = 0; t < n; ++t) {
        const int32_t r = P.perm[t];
        rp[t + 1] = rp[t] + (A->row_ptr[r + 1] - A->row_ptr[r]);
    }
    for (int32_t t = 0; t < n; ++t) {
        const int32_t r = P.perm[t];
        int64_t q = rp[t];
        for (int64_t e = A->row_ptr[r]; e < A->row_ptr[r + 1]; ++e, ++q) {
            ci[q] = P.pos[A->col_idx[e]];
            src_of[q] = e;
        }
    }
    h->nnz = A->nnz;
    h->d_rp.ensure(rp.size() * 8);
    h->d_ci.ensure(std::max<size_t>(ci.size(), 1) * 4);
    h->d_val.ensure(std::max<size_t>(ci.size(), 1) * 8);
    h->d_perm.ensure((size_t)n * 4);
    const hipStream_t s0 = h->stream;
    HIPCHK(hipMemcpyAsync(h->d_rp.p, rp.data(), rp.size() * 8, hipMemcpyHostToDevice, s0));
    HIPCHK(hipMemcpyAsync(h->d_perm.p, P.perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s0));
    if (A->nnz) {
        HIPCHK(hipMemcpyAsync(h->d_ci.p, ci.data(), ci.size() * 4, hipMemcpyHostToDevice, s0));
        DevBuf d_src, d_vh;
        d_src.ensure(src_of.size() * 8);
        HIPCHK(hipMemcpyAsync(d_src.p, src_of.data(), src_of.size() * 8, hipMemcpyHostToDevice, s0));
        const double* vsrc = val_dev;
        if (!vsrc) {
            d_vh.ensure((size_t)A->nnz * 8);
            HIPCHK(hipMemcpyAsync(d_vh.p, A->val, (size_t)A->nnz * 8, hipMemcpyHostToDevice, s0));
            vsrc = d_vh.as<double>();
        } else {
            DevBuf d_cnt;
            d_cnt.ensure(8);
            HIPCHK(launch_count_nonfinite(vsrc, A->nnz, d_cnt.as<int64_t>(), s0));
            int64_t bad = 0;
            HIPCHK(hipMemcpyAsync(&bad, d_cnt.p, 8, hipMemcpyDeviceToHost, s0));
            HIPCHK(hipStreamSynchronize(s0));
            if (bad) fail(LRX_EINVAL, "non-finite value in A");
        }
        HIPCHK(launch_gather_idx(h->d_val.as<double>(), vsrc, d_src.as<int64_t>(), A->nnz, s0));
        HIPCHK(hipStreamSynchronize(s0));     // d_src, d_vh go out of scope
    } else {
        HIPCHK(hipStreamSynchronize(s0));     // rp and the host vectors go out of scope
    }
}

// lrx_gmres multiplies by the handle's resident copy of A: the caller's A must
// be that matrix, pattern and values, entry for entry (compared in tree order
// with the copy read back from the device).
void check_same_matrix(lrx_handle h, const lrx_csr* A) {
    const Plan& P = h->plan;
    const int32_t n = A->n;
    std::vector<int64_t> rp((size_t)n + 1);
    std::vector<int32_t> ci((size_t)std::max<int64_t>(A->nnz, 1));
    std::vector<double> va((size_t)std::max<int64_t>(A->nnz, 1));
    HIPCHK(hipMemcpyAsync(rp.data(), h->d_rp.p, rp.size() * 8, hipMemcpyDeviceToHost, h->stream));
    if (A->nnz) {
        HIPCHK(hipMemcpyAsync(ci.data(), h->d_ci.p, (size_t)A->nnz * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(va.data(), h->d_val.p, (size_t)A->nnz * 8, hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int32_t t = 0; t < n; ++t) {
        const int32_t r = P.perm[t];
        if (A->row_ptr[r + 1] - A->row_ptr[r] != rp[t + 1] - rp[t])
            fail(LRX_EINVAL, "A's pattern differs from the matrix the handle was factored from");
        int64_t q = rp[t];
        for (int64_t e = A->row_ptr[r]; e < A->row_ptr[r + 1]; ++e, ++q) {
            if (A->col_idx[e] < 0 || A->col_idx[e] >= n || ci[q] != P.pos[A->col_idx[e]])
                fail(LRX_EINVAL, "A's pattern differs from the matrix the handle was factored from");
            if (va[q] != A->val[e])
                fail(LRX_EINVAL, "A's values differ from the matrix the handle was factored from");
        }
    }
}

void finish_stats(lrx_handle h, double t_plan_ms, double t_factor_ms) {
    const Plan& P = h->plan;
    lrx_stats_t& S = h->stats;
    S.depth = P.depth;
    S.n_compressions = (int32_t)h->ranks.size();
    S.n_colour_steps = (int32_t)P.steps.size();
    double rs = 0;
    int32_t rmax = 0;
    std::vector<double> lsum(33, 0), lcnt(33, 0);
    for (size_t i = 0; i < h->ranks.size(); ++i) {
        rs += h->ranks[i];
        rmax = std::max(rmax, h->ranks[i]);
        int lv = h->rank_level[i];
        if (lv < 32) {
            S.rank_max_by_level[lv] = std::max(S.rank_max_by_level[lv], h->ranks[i]);
            lsum[lv] += h->ranks[i];
            lcnt[lv] += 1;
        }
    }
    for (auto& L : P.levels)
        if (L.level < 32) {
            double ms = 0;
            for (int32_t s : L.supers) ms += h->size[s];
            S.mean_node_size_by_level[L.level] = L.supers.empty() ? 0 : ms / L.supers.size();
        }
    for (int lv = 0; lv < 32; ++lv) S.rank_mean_by_level[lv] = lcnt[lv] ? lsum[lv] / lcnt[lv] : 0.0;
    S.max_rank = rmax;
    S.mean_rank = h->ranks.empty() ? 0.0 : rs / h->ranks.size();
    S.extended_size = h->n_ext;
    S.max_compression_error = h->max_tail_ratio;
    S.factor_bytes = (h->solve_fp32 ? h->arena32.total : h->arena.total) * 8;
    S.t_plan_ms = t_plan_ms;
    S.t_factor_ms = t_factor_ms;
    S.t_sync_ms = h->t_sync_ms;
    S.t_solve_prog_ms = h->t_solve_prog_ms;
}

constexpr int kPlanThreads = 8;

// Factorization of k systems (k = 1: lrx_factor); see lrx_factor_batch.
void factor_many(int32_t k, const lrx_csr* A, const double* const* val_dev, const lrx_tree* T, const lrx_opts* o,
                 lrx_handle* out) {
    const double t0 = now_ms();
    std::vector<std::unique_ptr<lrx_handle_s>> hs(k);
    for (int32_t i = 0; i < k; ++i) {
        try {
            check_factor_args(&A[i], val_dev[i], &T[i], o);
        } catch (Fail& f) {
            if (k > 1) f.msg = "system " + std::to_string(i) + ": " + f.msg;
            throw;
        }
        hs[i].reset(new lrx_handle_s());
    }
    // symbolic plans on host threads
    std::vector<std::string> errs(k);
    std::vector<double> t_plan(k, 0.0);
    {
        std::atomic<int32_t> next{0};
        auto work = [&]() {
            for (int32_t i; (i = next.fetch_add(1)) < k;) {
                const double ta = now_ms();
                try {
                    // one system: its planner spreads the leaf phases over host threads
                    errs[i] = build_plan(A[i].n, A[i].nnz, A[i].row_ptr, A[i].col_idx, T[i].depth, T[i].perm,
                                         T[i].leaf_ptr, o->order, hs[i]->plan, k == 1 ? kPlanThreads : 1);
                } catch (const std::exception& e) {
                    errs[i] = std::string("planner: ") + e.what();
                }
                t_plan[i] = now_ms() - ta;
            }
        };
        const int nt = (int)std::min<int64_t>(k, std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
        if (nt <= 1) {
            work();
        } else {
            std::vector<std::thread> th;
            for (int t = 0; t < nt; ++t) th.emplace_back(work);
            for (auto& t : th) t.join();
        }
    }
    for (int32_t i = 0; i < k; ++i)
        if (!errs[i].empty()) fail(LRX_EINVAL, k > 1 ? "system " + std::to_string(i) + ": " + errs[i] : errs[i]);
    const double t1 = now_ms();
    std::vector<std::unique_ptr<FactorRun>> runs;
    std::vector<FactorRun*> rp;
    std::vector<const lrx_csr*> ap;
    std::vector<const double*> vp;
    for (int32_t i = 0; i < k; ++i) {
        init_handle(hs[i].get(), &A[i], val_dev[i], o);
        runs.emplace_back(new FactorRun(hs[i].get()));
        rp.push_back(runs.back().get());
        ap.push_back(&A[i]);
        vp.push_back(val_dev[i]);
    }
    run_factor(rp, (hipStream_t)o->stream, ap, vp);
    runs.clear();
    for (int32_t i = 0; i < k; ++i) build_solve_program(hs[i].get());
    HIPCHK(hipStreamSynchronize((hipStream_t)o->stream));
    const double t2 = now_ms();
    for (int32_t i = 0; i < k; ++i) finish_stats(hs[i].get(), k > 1 ? t_plan[i] : t1 - t0, t2 - t0);
    std::lock_guard<std::mutex> lk(g_reg_mu);
    for (int32_t i = 0; i < k; ++i) {
        out[i] = hs[i].release();
        g_live.insert(out[i]);
    }
}

// Arguments of the batched entry points: k distinct live handles on one device.
void check_batch(int32_t k, const lrx_handle* hs, int32_t nrhs, const double* const* b_dev,
                 double* const* x_dev) {
    if (k < 1 || k > 65535 || !hs || !b_dev || !x_dev) fail(LRX_EINVAL, "bad batch arguments");
    if (nrhs < 1 || nrhs > 256) fail(LRX_EINVAL, "nrhs must be in [1, 256]");
    std::set<lrx_handle> seen;
    for (int i = 0; i < k; ++i) {
        check_handle(hs[i]);
        if (!b_dev[i] || !x_dev[i] || b_dev[i] == x_dev[i]) fail(LRX_EINVAL, "bad b/x pointers");
        if (!seen.insert(hs[i]).second) fail(LRX_EINVAL, "a handle appears twice in the batch");
        if (hs[i]->device != hs[0]->device) fail(LRX_EINVAL, "handles of a batch must share one device");
    }
}

}  // namespace

extern "C" {

const char* lrx_last_error(void) { return g_err.c_str(); }

const char* lrx_version(void) { return "lorax 0.1 (gfx950)"; }

lrx_status lrx_plan_inspect(const lrx_csr* A, const lrx_tree* T, int32_t order, lrx_plan_info* info) {
    return guarded([&]() -> lrx_status {
        if (!A || !T || !info) fail(LRX_EINVAL, "null argument");
        if (A->n < 1 || A->nnz < 0 || !A->row_ptr || !A->col_idx) fail(LRX_EINVAL, "bad CSR");
        Plan P;
        std::string err = build_plan(A->n, A->nnz, A->row_ptr, A->col_idx, T->depth, T->perm,
                                     T->leaf_ptr, order, P, kPlanThreads);
        if (!err.empty()) fail(LRX_EINVAL, err);
        std::memset(info, 0, sizeof(*info));
        info->depth = P.depth;
        int32_t nsup = 0;
        for (auto& L : P.levels) {
            nsup += (int32_t)L.supers.size();
            if (L.level < 32) {
                info->colours_by_level[L.level] = L.colours;
                info->candidates_by_level[L.level] = L.candidates;
            }
        }
        info->n_supernodes = nsup;
        info->n_colour_steps = (int32_t)P.steps.size();
        info->n_candidates = P.n_candidates;
        info->n_schur_pairs = P.n_pairs;
        int64_t created = 0;
        for (auto& E : P.edges) if (E.origin != EO_INIT && E.origin != EO_MERGE) ++created;
        info->n_edges_created = created;
        return LRX_OK;
    });
}

lrx_status lrx_factor(const lrx_csr* A, const lrx_tree* T, const lrx_opts* o, lrx_handle* out) {
    return guarded([&]() -> lrx_status {
        if (!out) fail(LRX_EINVAL, "out is NULL");
        *out = nullptr;
        if (!A || !T) fail(LRX_EINVAL, "null matrix or tree");
        const double* none = nullptr;
        factor_many(1, A, &none, T, o, out);
        return LRX_OK;
    });
}

lrx_status lrx_factor_dev(const lrx_csr* A, const double* val_dev, const lrx_tree* T,
                          const lrx_opts* o, lrx_handle* out) {
    return guarded([&]() -> lrx_status {
        if (!out) fail(LRX_EINVAL, "out is NULL");
        *out = nullptr;
        if (!val_dev) fail(LRX_EINVAL, "val_dev is NULL");
        if (!A || !T) fail(LRX_EINVAL, "null matrix or tree");
        factor_many(1, A, &val_dev, T, o, out);
        return LRX_OK;
    });
}

lrx_status lrx_factor_batch(int32_t k, const lrx_csr* A, const double* const* val_dev, const lrx_tree* T,
                            const lrx_opts* o, lrx_handle* out) {
    return guarded([&]() -> lrx_status {
        if (!out) fail(LRX_EINVAL, "out is NULL");
        if (k < 1 || k > 65536) fail(LRX_EINVAL, "k must be in [1, 65536]");
        for (int32_t i = 0; i < k; ++i) out[i] = nullptr;
        if (!A || !T) fail(LRX_EINVAL, "null matrix or tree array");
        std::vector<const double*> vd(k, nullptr);
        if (val_dev)
            for (int32_t i = 0; i < k; ++i) {
                if (!val_dev[i]) fail(LRX_EINVAL, "system " + std::to_string(i) + ": val_dev is NULL");
                vd[i] = val_dev[i];
            }
        factor_many(k, A, vd.data(), T, o, out);
        return LRX_OK;
    });
}

void lrx_timing_enable(int32_t class_mask) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = (uint32_t)class_mask;
}

lrx_status lrx_tune_get(lrx_tune* t) {
    return guarded([&]() -> lrx_status {
        if (!t) fail(LRX_EINVAL, "null tuning table");
        *t = lrx_tune{};
        t->gemm_kc = g_tune.gemm_kc;
        t->gemm_f64_valu = g_tune.gemm_f64_valu;
        t->sweep_nk_max = g_tune.sweep_nk_max;
        t->compress_nt_small = g_tune.compress_nt_small;
        t->compress_nt_mid = g_tune.compress_nt_mid;
        t->gemm_grid = g_tune.gemm_grid;
        t->solve_graph = g_tune.solve_graph;
        t->compress_gram = g_tune.compress_gram;
        t->large_split_c = g_tune.large_split_c;
        return LRX_OK;
    });
}

lrx_status lrx_tune_set(const lrx_tune* t) {
    return guarded([&]() -> lrx_status {
        if (!t) fail(LRX_EINVAL, "null tuning table");
        if (t->gemm_kc < 16 || t->gemm_kc > 256 || t->gemm_kc % 16) fail(LRX_EINVAL, "gemm_kc must be 16..256, a multiple of 16");
        if (t->gemm_f64_valu != 0 && t->gemm_f64_valu != 1) fail(LRX_EINVAL, "gemm_f64_valu must be 0 or 1");
        if (t->sweep_nk_max != 1 && t->sweep_nk_max != 2 && t->sweep_nk_max != 4)
            fail(LRX_EINVAL, "sweep_nk_max must be 1, 2 or 4");
        for (int32_t v : {t->compress_nt_small, t->compress_nt_mid})
            if (v != 256 && v != 512 && v != 1024) fail(LRX_EINVAL, "compress_nt_* must be 256, 512 or 1024");
        if (t->gemm_grid < 0 || t->gemm_grid > 65536) fail(LRX_EINVAL, "gemm_grid must be 0..65536");
        if (t->solve_graph != 0 && t->solve_graph != 1) fail(LRX_EINVAL, "solve_graph must be 0 or 1");
        if (t->compress_gram < 0 || t->compress_gram > 2) fail(LRX_EINVAL, "compress_gram must be 0, 1 or 2");
        if (t->large_split_c < 65 || t->large_split_c > 65536) fail(LRX_EINVAL, "large_split_c must be 65..65536");
        g_tune.large_split_c = t->large_split_c;
        g_tune.solve_graph = t->solve_graph;
        g_tune.compress_gram = t->compress_gram;
        g_tune.gemm_kc = t->gemm_kc;
        g_tune.compress_nt_small = t->compress_nt_small;
        g_tune.compress_nt_mid = t->compress_nt_mid;
        g_tune.gemm_grid = t->gemm_grid;
        g_tune.gemm_f64_valu = t->gemm_f64_valu;
        g_tune.sweep_nk_max = t->sweep_nk_max;
        return LRX_OK;
    });
}

lrx_status lrx_timing_read(lrx_timing_t* t, int32_t reset) {
    return guarded([&]() -> lrx_status {
        if (!t) fail(LRX_EINVAL, "null timing");
        std::lock_guard<std::mutex> lk(g_tmu);
        resolve_timing();
        *t = g_acc;
        if (reset) g_acc = lrx_timing_t{};
        return LRX_OK;
    });
}


lrx_status lrx_solve_dev(lrx_handle h, int32_t nrhs, const double* b_dev, double* x_dev) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (nrhs < 1 || nrhs > 256) fail(LRX_EINVAL, "nrhs must be in [1, 256]");
        if (!b_dev || !x_dev || b_dev == x_dev) fail(LRX_EINVAL, "bad b/x pointers");
        solve_dev(h, nrhs, b_dev, x_dev);
        return LRX_OK;
    });
}

lrx_status lrx_solve_dev_noalloc(lrx_handle h, int32_t nrhs, const double* b_dev, double* x_dev) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (nrhs < 1 || nrhs > 256) fail(LRX_EINVAL, "nrhs must be in [1, 256]");
        if (!b_dev || !x_dev || b_dev == x_dev) fail(LRX_EINVAL, "bad b/x pointers");
        const size_t need = (size_t)h->n_ext * nrhs * sizeof(double);
        if (need > kNoallocScratchBytes)
            fail(LRX_EINVAL, "n_ext * nrhs * 8 = " + std::to_string(need) + " bytes exceeds the " +
                                 std::to_string(kNoallocScratchBytes) + "-byte scratch of lrx_solve_dev_noalloc");
        int cur = -1;
        HIPCHK(hipGetDevice(&cur));
        if (cur != h->device) fail(LRX_EINVAL, "the handle's device is not the current device");
        void* p = nullptr;
        HIPCHK(noalloc_scratch(h->device, &p));
        solve_into(h, nrhs, b_dev, x_dev, static_cast<double*>(p), false);
        return LRX_OK;
    });
}

lrx_status lrx_solve_batch_dev(int32_t k, const lrx_handle* hs, int32_t nrhs, const double* const* b_dev,
                               double* const* x_dev) {
    return guarded([&]() -> lrx_status {
        check_batch(k, hs, nrhs, b_dev, x_dev);
        solve_batch_dev(k, hs, nrhs, b_dev, x_dev);
        return LRX_OK;
    });
}

lrx_status lrx_gmres_batch_dev(int32_t k, const lrx_handle* hs, int32_t nrhs, const double* const* b_dev,
                               double* const* x_dev, double tol, int32_t restart, int32_t maxit, int32_t* iters,
                               double* relres) {
    return guarded([&]() -> lrx_status {
        check_batch(k, hs, nrhs, b_dev, x_dev);
        if (!(tol > 0.0) || restart < 1 || restart > 200 || maxit < 0) fail(LRX_EINVAL, "bad tol/restart/maxit");
        const lrx_status s = gmres_batch(k, hs, nrhs, b_dev, x_dev, tol, restart, maxit, iters, relres);
        if (s == LRX_ENOCONV) g_err = "GMRES reached maxit before tol";
        return s;
    });
}

lrx_status lrx_gmres_batch_dev_x0(int32_t k, const lrx_handle* hs, int32_t nrhs, const double* const* b_dev,
                                  double* const* x_dev, double tol, int32_t restart, int32_t maxit, int32_t* iters,
                                  double* relres) {
    return guarded([&]() -> lrx_status {
        check_batch(k, hs, nrhs, b_dev, x_dev);
        if (!(tol > 0.0) || restart < 1 || restart > 200 || maxit < 0) fail(LRX_EINVAL, "bad tol/restart/maxit");
        lrx_status s = gmres_batch(k, hs, nrhs, b_dev, x_dev, tol, restart, maxit, iters, relres, true);
        if (s == LRX_ENOCONV) g_err = "GMRES reached maxit before tol";
        return s;
    });
}

lrx_status lrx_solve(lrx_handle h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        const int32_t n = h->plan.n;
        if (nrhs < 1 || nrhs > 256) fail(LRX_EINVAL, "nrhs must be in [1, 256]");
        if (!b || !x || ldb < n || ldx < n) fail(LRX_EINVAL, "bad b/x or leading dimension");
        for (int k = 0; k < nrhs; ++k)
            for (int32_t i = 0; i < n; ++i)
                if (!std::isfinite(b[i + k * ldb])) fail(LRX_EINVAL, "non-finite value in b");
        DevBuf db, dx;
        db.ensure((size_t)n * nrhs * 8);
        dx.ensure((size_t)n * nrhs * 8);
        HIPCHK(hipMemcpy2DAsync(db.p, (size_t)n * 8, b, (size_t)ldb * 8, (size_t)n * 8, nrhs,
                                hipMemcpyHostToDevice, h->stream));
        solve_dev(h, nrhs, db.as<double>(), dx.as<double>());
        HIPCHK(hipMemcpy2DAsync(x, (size_t)ldx * 8, dx.p, (size_t)n * 8, (size_t)n * 8, nrhs,
                                hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        return LRX_OK;
    });
}

lrx_status lrx_gmres_dev(lrx_handle h, int32_t nrhs, const double* b_dev, double* x_dev, double tol,
                         int32_t restart, int32_t maxit, int32_t* iters, double* relres) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (nrhs < 1 || nrhs > 256) fail(LRX_EINVAL, "nrhs must be in [1, 256]");
        if (!b_dev || !x_dev || b_dev == x_dev) fail(LRX_EINVAL, "bad b/x pointers");
        if (!(tol > 0.0) || restart < 1 || restart > 200 || maxit < 0) fail(LRX_EINVAL, "bad tol/restart/maxit");
        return gmres_dev(h, nrhs, b_dev, x_dev, tol, restart, maxit, iters, relres);
    });
}

lrx_status lrx_gmres(const lrx_csr* A, lrx_handle h, int32_t nrhs, const double* b, double* x,
                     double tol, int32_t restart, int32_t maxit, int32_t* iters, double* relres) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (!A || A->n != h->plan.n || A->nnz != h->nnz) fail(LRX_EINVAL, "A does not match the handle");
        check_csr(A);
        check_same_matrix(h, A);
        const int32_t n = h->plan.n;
        if (nrhs < 1 || nrhs > 256) fail(LRX_EINVAL, "nrhs must be in [1, 256]");
        if (!b || !x) fail(LRX_EINVAL, "null b/x");
        if (!(tol > 0.0) || restart < 1 || restart > 200 || maxit < 0) fail(LRX_EINVAL, "bad tol/restart/maxit");
        for (int64_t i = 0; i < (int64_t)n * nrhs; ++i)
            if (!std::isfinite(b[i])) fail(LRX_EINVAL, "non-finite value in b");
        DevBuf db, dx;
        db.ensure((size_t)n * nrhs * 8);
        dx.ensure((size_t)n * nrhs * 8);
        HIPCHK(hipMemcpyAsync(db.p, b, (size_t)n * nrhs * 8, hipMemcpyHostToDevice, h->stream));
        lrx_status s = gmres_dev(h, nrhs, db.as<double>(), dx.as<double>(), tol, restart, maxit, iters, relres);
        HIPCHK(hipMemcpyAsync(x, dx.p, (size_t)n * nrhs * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (s == LRX_ENOCONV) g_err = "GMRES reached maxit before tol";
        return s;
    });
}

lrx_status lrx_set_stream(lrx_handle h, void* stream) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        h->stream = (hipStream_t)stream;
        return LRX_OK;
    });
}

lrx_status lrx_free(lrx_handle h) {
    return guarded([&]() -> lrx_status {
        if (!h) return LRX_OK;
        {
            std::lock_guard<std::mutex> lk(g_reg_mu);
            if (!g_live.count(h)) fail(LRX_EINVAL, "handle already freed or invalid");
            g_live.erase(h);
        }
        (void)hipStreamSynchronize(h->stream);
        IdleScope idle;
        delete h;
        return LRX_OK;
    });
}

// Device bytes a handle holds now: arena chunks (capacity) and every buffer.
int64_t handle_device_bytes(lrx_handle h) {
    int64_t b = 0;
    for (const Arena* a : {&h->arena, &h->arena32})
        for (const auto& c : a->chunks) b += (int64_t)(c.second * sizeof(double));
    for (const DevBuf* d : {&h->d_swnodes, &h->d_swprog, &h->batch_nodes, &h->d_perm, &h->d_rp, &h->d_ci, &h->d_val,
                            &h->x_ext, &h->ws_b, &h->ws_w, &h->g_basis, &h->g_z, &h->g_w, &h->g_r, &h->g_b, &h->g_x,
                            &h->kry_tab, &h->kry_small, &h->kry_part})
        b += (int64_t)d->bytes;
    return b;
}

lrx_status lrx_trim(lrx_handle h) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        HIPCHK(hipStreamSynchronize(h->stream));
        IdleScope idle;
        for (DevBuf* d : {&h->x_ext, &h->g_basis, &h->g_z, &h->g_w, &h->g_r, &h->g_b, &h->g_x, &h->kry_tab,
                          &h->kry_small, &h->kry_part, &h->batch_nodes})
            d->release();
        h->kry_pin.release();
        return LRX_OK;
    });
}

lrx_status lrx_stats(lrx_handle h, lrx_stats_t* s) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (!s) fail(LRX_EINVAL, "null stats");
        *s = h->stats;
        s->device_bytes = handle_device_bytes(h);
        return LRX_OK;
    });
}

lrx_status lrx_compression_tails(lrx_handle h, int32_t idx, double* out, int32_t cap, int32_t* len) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (idx < 0 || idx >= (int32_t)h->ranks.size() || !len) fail(LRX_EINVAL, "bad compression index");
        const int64_t a = h->tail_off[idx];
        const int64_t b = (idx + 1 < (int32_t)h->tail_off.size()) ? h->tail_off[idx + 1] : (int64_t)h->tails.size();
        *len = (int32_t)(b - a);
        if (out) for (int64_t i = a; i < b && i - a < cap; ++i) out[i - a] = h->tails[i];
        return LRX_OK;
    });
}

lrx_status lrx_gmres_history(lrx_handle h, int32_t rhs, double* out, int32_t cap, int32_t* len) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (!len) fail(LRX_EINVAL, "null length");
        if (rhs < 0 || rhs >= (int32_t)h->gmres_hist.size()) {
            if (h->gmres_hist.empty() && rhs >= 0) { *len = 0; return LRX_OK; }   // no GMRES call yet
            fail(LRX_EINVAL, "right-hand side index out of range");
        }
        const std::vector<double>& v = h->gmres_hist[rhs];
        *len = (int32_t)v.size();
        if (out) for (int32_t i = 0; i < *len && i < cap; ++i) out[i] = v[i];
        return LRX_OK;
    });
}

lrx_status lrx_compression_shape(lrx_handle h, int32_t idx, int32_t* rows, int32_t* cols) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (idx < 0 || idx >= (int32_t)h->ranks.size() || !rows || !cols) fail(LRX_EINVAL, "bad compression index");
        *rows = h->comp_rows[idx];
        *cols = h->comp_cols[idx];
        return LRX_OK;
    });
}

lrx_status lrx_ranks(lrx_handle h, int32_t* ranks, int32_t* levels, int32_t* js) {
    return guarded([&]() -> lrx_status {
        check_handle(h);
        if (!ranks) fail(LRX_EINVAL, "null ranks");
        for (size_t i = 0; i < h->ranks.size(); ++i) {
            ranks[i] = h->ranks[i];
            if (levels) levels[i] = h->rank_level[i];
            if (js) js[i] = h->rank_j[i];
        }
        return LRX_OK;
    });
}

}  // extern "C"
