// Batched gather/scatter products on the matrix cores of gfx950 (MFMA).
//
// The Schur-complement updates of Eliminate(s) and Eliminate(b) (block Gauss
// elimination, Sec. 2.2 and Sec. 4.4) and the projection [R; Q] = B V of
// Compress (Sec. 4.3) are many small dense products whose operands are
// gathered through index maps (compact supports) and whose results are
// scattered, optionally subtracted, into stored blocks (DGemm in dev.hpp).
//
// One work-group of 256 threads (4 wavefronts) computes one 32 x 32 tile of C:
// the A rows and B columns of the tile are staged through LDS in chunks of K
// (zero-padded to the MFMA K step), and each wavefront accumulates one 16 x 16
// quadrant with 16x16 MFMA instructions:
//   GP_F64   v_mfma_f64_16x16x4_f64      FP64 operands, FP64 accumulation
//   GP_F32   v_mfma_f32_16x16x4_f32      FP32 operands, FP32 accumulation
//   GP_BF16  v_mfma_f32_16x16x16_bf16    BF16 operands, FP32 accumulation
// The result (FP64 or FP32 accumulator) is written to, or subtracted in FP64
// from, the FP64 block C.
//
// Operand layouts of these instructions (wave64, lane l, row i, column j):
//   A (16 x K_step): lane l holds A[l % 16][k0 + (l / 16) * E + e], e < E
//   B (K_step x 16): lane l holds B[k0 + (l / 16) * E + e][l % 16],  e < E
//   D (16 x 16):     lane l holds D[row(l, v)][l % 16], v < 4, with
//                    row = 4 (l / 16) + v for the FP32-accumulating forms and
//                    row = l / 16 + 4 v for the FP64 form
// with E = 1 (FP64, FP32) or 4 (BF16) elements per lane (checked on the device
// against host products).  Panels are kept
// K-contiguous in LDS (A row-major, B column-major), so a lane's E elements are
// adjacent; the row stride LDK is odd in 4-byte words per lane step (FP64,
// FP32) or an odd multiple of 8 bytes (BF16), so the 16 lanes of a group hit
// distinct LDS banks.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "kernels.hpp"

namespace lrx {

namespace {

constexpr int GM_T = 256;        // threads per tile work-group
constexpr int GM_KC = 256;       // largest K chunk staged in LDS (the launch may ask for less)

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int gmap(const int32_t* imap, int32_t map, int t) {
    return map < 0 ? t : imap[map + t];
}

// FP32 -> BF16, rounding to nearest with ties to even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int P> struct GTr;
template <> struct GTr<GP_F64> {
    using S = double;            // LDS element
    using Acc = f64x4;
    static constexpr int E = 1;  // elements per lane per MFMA
    static constexpr int KS = 4; // K per MFMA
    __device__ static S cvt(double v) { return v; }
    __device__ static Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static Acc mma(const S* a, const S* b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    }
    static constexpr int ldk(int kc) { return kc + 1; }
    __device__ static int drow(int lane, int v) { return lane / 16 + 4 * v; }
};
template <> struct GTr<GP_F32> {
    using S = float;
    using Acc = f32x4;
    static constexpr int E = 1;
    static constexpr int KS = 4;
    __device__ static S cvt(double v) { return (float)v; }
    __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static Acc mma(const S* a, const S* b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
    }
    static constexpr int ldk(int kc) { return kc + 1; }
    __device__ static int drow(int lane, int v) { return 4 * (lane / 16) + v; }
};
template <> struct GTr<GP_BF16> {
    using S = uint16_t;
    using Acc = f32x4;
    static constexpr int E = 4;
    static constexpr int KS = 16;
    __device__ static S cvt(double v) { return to_bf16((float)v); }
    __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static Acc mma(const S* a, const S* b, Acc c) {
        const i16x4 av = *reinterpret_cast<const i16x4*>(a);
        const i16x4 bv = *reinterpret_cast<const i16x4*>(b);
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
    }
    // kc is a multiple of 16; kc + 4 is 4 (mod 16): 8-byte aligned rows whose
    // stride is an odd multiple of 8 bytes
    static constexpr int ldk(int kc) { return kc + 4; }
    __device__ static int drow(int lane, int v) { return 4 * (lane / 16) + v; }
};

// One 32 x 32 tile of C (see the file header).  The work-groups of a launch
// walk the tile list with a stride of the grid size: one tile each when the
// grid has a work-group per tile, or a persistent grid sized to the machine.
template <int P>
__device__ void gemm_tile(const DGemm* __restrict__ gs, const DTile& tl, const int32_t* __restrict__ imap,
                          int kc_max, typename GTr<P>::S* As, typename GTr<P>::S* Bs, int ldk) {
    using Tr = GTr<P>;
    const DGemm G = gs[tl.g];
    const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
    const int mt = min(32, G.M - tl.i0), nt = min(32, G.N - tl.j0);
    const int iq = w & 1, jq = w >> 1;
    typename Tr::Acc acc = Tr::zero();
    for (int k0 = 0; k0 < G.K; k0 += kc_max) {
        const int kc = min(kc_max, G.K - k0);
        const int kp = (kc + Tr::KS - 1) / Tr::KS * Tr::KS;     // zero-padded chunk
        __syncthreads();                  // the previous chunk (or tile) is consumed
        // A panel, rows i0 .. i0 + 31 of A (column-major, lda), columns amap(k0 + t):
        // lanes over rows (contiguous in HBM), 8 column slots
        {
            const int a = tid % 32;
            for (int t = tid / 32; t < kp; t += GM_T / 32) {
                double v = 0.0;
                if (a < mt && t < kc) v = G.A[(int64_t)(tl.i0 + a) + (int64_t)gmap(imap, G.amap, k0 + t) * G.lda];
                As[a * ldk + t] = Tr::cvt(v);
            }
        }
        // B panel, rows bmap(k0 + t), columns j0 .. j0 + 31 (column-major, ldb):
        // lanes over K (contiguous in HBM), 4 column slots
        {
            const int t0 = tid % 64;
            for (int b = tid / 64; b < 32; b += GM_T / 64)
                for (int t = t0; t < kp; t += 64) {
                    double v = 0.0;
                    if (b < nt && t < kc)
                        v = G.B[(int64_t)gmap(imap, G.bmap, k0 + t) + (int64_t)(tl.j0 + b) * G.ldb];
                    Bs[b * ldk + t] = Tr::cvt(v);
                }
        }
        __syncthreads();
        const typename Tr::S* ap = As + (iq * 16 + lane % 16) * ldk + (lane / 16) * Tr::E;
        const typename Tr::S* bp = Bs + (jq * 16 + lane % 16) * ldk + (lane / 16) * Tr::E;
        for (int k = 0; k < kp; k += Tr::KS) acc = Tr::mma(ap + k, bp + k, acc);
    }
    // D[row(l, v)][l % 16] of quadrant (iq, jq)
    const int col = jq * 16 + lane % 16;
    if (col >= nt) return;               // no barrier follows in this tile
    const int ccol = gmap(imap, G.ccmap, tl.j0 + col);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = iq * 16 + Tr::drow(lane, v);
        if (row >= mt) continue;
        const int crow = gmap(imap, G.crmap, tl.i0 + row);
        double* c = G.C + (G.tr ? (int64_t)ccol + (int64_t)crow * G.ldc : (int64_t)crow + (int64_t)ccol * G.ldc);
        const double d = (double)acc[v];
        *c = G.sub ? *c - d : d;
    }
}

template <int P>
__global__ __launch_bounds__(GM_T) void k_gemm_mfma(const DGemm* __restrict__ gs, const DTile* __restrict__ tiles,
                                                     int ntile, const int32_t* __restrict__ imap, int kc_max) {
    // kc_max: K chunk of this launch (a multiple of the K step, <= GM_KC)
    using S = typename GTr<P>::S;
    extern __shared__ double sm_raw[];
    S* As = reinterpret_cast<S*>(sm_raw);
    const int ldk = GTr<P>::ldk(kc_max);
    S* Bs = As + 32 * ldk;
    for (int t = blockIdx.x; t < ntile; t += gridDim.x) gemm_tile<P>(gs, tiles[t], imap, kc_max, As, Bs, ldk);
}

template <int P>
size_t gemm_lds(int kc) {
    return (size_t)2 * 32 * GTr<P>::ldk(kc) * sizeof(typename GTr<P>::S);
}

template <int P>
hipError_t launch_p(const DGemm* g, const DTile* tiles, int ntile, int kmax, const int32_t* imap, int kc_cap,
                    int grid_cap, hipStream_t st) {
    static std::atomic<bool> attr{false};
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_gemm_mfma<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)gemm_lds<P>(GM_KC));
        if (e != hipSuccess) return e;
        attr = true;
    }
    // chunk width: the largest K, at most kc_cap (itself at most GM_KC), rounded
    // up to the instruction's K step
    const int cap = kc_cap < GTr<P>::KS ? GTr<P>::KS : (kc_cap > GM_KC ? GM_KC : kc_cap);
    int kc = kmax < 1 ? 1 : (kmax > cap ? cap : kmax);
    kc = (kc + GTr<P>::KS - 1) / GTr<P>::KS * GTr<P>::KS;
    if (kc > GM_KC) kc = GM_KC;
    const int grid = grid_cap > 0 && grid_cap < ntile ? grid_cap : ntile;
    hipLaunchKernelGGL(k_gemm_mfma<P>, dim3(grid), dim3(GM_T), gemm_lds<P>(kc), st, g, tiles, ntile, imap, kc);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_mfma(const DGemm* g, const DTile* tiles, int ntile, int kmax, const int32_t* imap, int prec,
                            int kc_cap, int grid_cap, hipStream_t st) {
    if (ntile == 0) return hipSuccess;
    switch (prec) {
        case GP_F64: return launch_p<GP_F64>(g, tiles, ntile, kmax, imap, kc_cap, grid_cap, st);
        case GP_F32: return launch_p<GP_F32>(g, tiles, ntile, kmax, imap, kc_cap, grid_cap, st);
        case GP_BF16: return launch_p<GP_BF16>(g, tiles, ntile, kmax, imap, kc_cap, grid_cap, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lrx
