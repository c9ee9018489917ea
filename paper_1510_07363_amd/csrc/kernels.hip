// HIP kernels for gfx950 (CDNA4, 64-wide wavefronts).
//
// Factorization kernels run one work-group (256 threads = 4 wavefronts) per
// super-node of a colour step: nodes of one colour are at distance >= 3 in the
// cluster adjacency graph and share no block, so work-groups never touch the
// same memory and no atomics are needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include <climits>
#include <cmath>

#include "kernels.hpp"

namespace lrx {

namespace {

constexpr int NT = kFactorThreads;
constexpr int WAVE = 64;
constexpr int kLdsBudget = 152 * 1024;      // dynamic LDS a work-group may request (160 KiB per CU)

__device__ __forceinline__ int imap_at(const int32_t* imap, int32_t map, int t) {
    return map < 0 ? t : imap[map + t];
}

// Block-wide (max value, lowest index) and sum; every thread receives the result.
__device__ void block_argmax_sum(double& best, int& bi, double& sum, double* s_d, int* s_i,
                                 double* s_s) {
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        double ob = __shfl_down(best, o);
        int oi = __shfl_down(bi, o);
        double os = __shfl_down(sum, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        sum += os;
    }
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    if (lane == 0) { s_d[w] = best; s_i[w] = bi; s_s[w] = sum; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = s_d[0], s = s_s[0];
        int i = s_i[0];
        for (int k = 1; k < NT / WAVE; ++k) {
            if (s_d[k] > b || (s_d[k] == b && s_i[k] < i)) { b = s_d[k]; i = s_i[k]; }
            s += s_s[k];
        }
        s_d[NT / WAVE] = b; s_i[NT / WAVE] = i; s_s[NT / WAVE] = s;
    }
    __syncthreads();
    best = s_d[NT / WAVE]; bi = s_i[NT / WAVE]; sum = s_s[NT / WAVE];
    __syncthreads();
}

// ----------------------------------------------------------------- scatter / merge
__global__ void k_scatter(double* __restrict__ dst, const int64_t* __restrict__ idx,
                          const double* __restrict__ val, int64_t nnz) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) dst[idx[e]] = val[e];
}

__global__ void k_merge(const DMerge* __restrict__ t) {
    const DMerge M = t[blockIdx.x];
    const int nr = M.src.nr, nc = M.src.nc;
    for (int e = threadIdx.x; e < nr * nc; e += blockDim.x) {
        int a = e % nr, b = e / nr;
        M.dst.p[(M.r0 + a) + (int64_t)(M.c0 + b) * M.dst.nr] = M.src.p[e];
    }
}

// ------------------------------------------------------------------ compress
// Column-pivoted Householder QR of B^T (pivots are rows of B), truncated at the
// first k with ||R22||_F <= eps |R11| (|R11| = largest row norm of B <= ||B||_2),
// so that ||B - B V V^T||_2 <= ||R22||_F <= eps ||B||_2.  Norms of the remaining
// rows are recomputed at every step; ties go to the lowest row index.
__global__ __launch_bounds__(NT) void k_compress(const DCompress* __restrict__ tasks,
                                                 const DPiece* __restrict__ pieces,
                                                 const int32_t* __restrict__ imap) {
    const DCompress T = tasks[blockIdx.x];
    const int M = T.M, c = T.c, tid = threadIdx.x;
    double* __restrict__ B = T.B;
    __shared__ double s_d[NT / WAVE + 1], s_s[NT / WAVE + 1];
    __shared__ int s_i[NT / WAVE + 1];
    extern __shared__ double s_dyn[];
    double* s_v = s_dyn;          // c
    double* s_beta = s_dyn + c;   // c

    if (M == 0 || c == 0) {
        if (tid == 0) { *T.rank_out = 0; T.tails[0] = 0.0; T.tails[1] = 0.0; }
        return;
    }
    for (int64_t e = tid; e < (int64_t)M * c; e += NT) B[e] = 0.0;
    __syncthreads();
    for (int q = 0; q < T.npieces; ++q) {
        const DPiece pc = pieces[T.piece0 + q];
        const int nr = pc.blk.nr, nc = pc.blk.nc;
        for (int e = tid; e < nr * nc; e += NT) {
            const int a = e % nr, b = e / nr;
            const double v = pc.blk.p[e];
            if (!pc.trans) B[(int64_t)(pc.row0 + a) * c + imap_at(imap, pc.map, b)] = v;
            else           B[(int64_t)(pc.row0 + b) * c + imap_at(imap, pc.map, a)] = v;
        }
    }
    __syncthreads();

    const int kmax = M < c ? M : c;
    double r11 = 0.0;
    int k = 0;
    for (; k < kmax; ++k) {
        double best = -1.0, sum = 0.0;
        int bi = INT_MAX;
        for (int i = tid; i < M; i += NT) {
            const double* row = B + (int64_t)i * c;
            double s2 = 0.0;
            for (int j = k; j < c; ++j) s2 += row[j] * row[j];
            sum += s2;
            if (s2 > best) { best = s2; bi = i; }
        }
        block_argmax_sum(best, bi, sum, s_d, s_i, s_s);
        if (bi < 0 || bi >= M) break;              // no finite row left (non-finite data)
        const double tail = sqrt(sum);
        if (k == 0) r11 = sqrt(best);
        if (tid == 0) { T.tails[0] = r11; T.tails[1 + k] = tail; }
        if (T.tau ? tail < *T.tau : (tail == 0.0 || tail <= T.eps * r11)) break;
        const int p = bi;
        double* rowp = B + (int64_t)p * c;
        const double xnorm = sqrt(best);
        const double x0 = rowp[k];
        const double alpha = -copysign(xnorm, x0);
        for (int j = tid; j < c - k; j += NT) s_v[j] = rowp[k + j];
        __syncthreads();
        if (tid == 0) {
            s_v[0] = x0 - alpha;
            s_beta[k] = 2.0 * (xnorm * xnorm + fabs(x0) * xnorm);   // v.v
        }
        __syncthreads();
        const double beta = s_beta[k];
        for (int j = tid; j < c - k; j += NT) T.hv[(int64_t)k * c + j] = s_v[j];
        if (beta > 0.0) {
            const double tau = 2.0 / beta;
            for (int i = tid; i < M; i += NT) {
                if (i == p) continue;
                double* row = B + (int64_t)i * c + k;
                double w = 0.0;
                for (int j = 0; j < c - k; ++j) w += s_v[j] * row[j];
                w *= tau;
                for (int j = 0; j < c - k; ++j) row[j] -= w * s_v[j];
            }
        }
        __syncthreads();
        for (int j = tid; j < c - k; j += NT) rowp[k + j] = (j == 0) ? alpha : 0.0;
        __syncthreads();
    }
    const int r = k;
    if (tid == 0 && r == kmax) T.tails[1 + r] = 0.0;
    // V = H_0 ... H_{r-1} I[:, :r]  (c x r, column-major, ld c); one column per thread
    for (int col = tid; col < r; col += NT) {
        double* vc = T.V + (int64_t)col * c;
        for (int a = 0; a < c; ++a) vc[a] = (a == col) ? 1.0 : 0.0;
        for (int t = r - 1; t >= 0; --t) {
            const double beta = s_beta[t];
            if (!(beta > 0.0)) continue;
            const double* v = T.hv + (int64_t)t * c;
            double w = 0.0;
            for (int j = 0; j < c - t; ++j) w += v[j] * vc[t + j];
            w *= 2.0 / beta;
            for (int j = 0; j < c - t; ++j) vc[t + j] -= w * v[j];
        }
    }
    if (tid == 0) *T.rank_out = r;
}

// Truncated SVD of the stacked block (eqn. lra with the cut-off of eqn.
// cutOff1): Householder QR of B (M x c, column-major) to the c x c triangle R,
// one-sided Jacobi (Hestenes) SVD of R with the rotations accumulated in V,
// singular values sorted in descending order, rank = #{sigma_k >= eps sigma_0}.
// R and V live in LDS when `lds_mat` is set (2 c^2 doubles), otherwise in the
// task's workspace.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of a DPP row; every lane receives the same value.
template <class T>
__device__ __forceinline__ T row16_sum(T v) {
    v += dpp_mov<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);    // row_half_mirror
    v += dpp_mov<0x140>(v);    // row_mirror
    return v;
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
    if constexpr (G == 16) return row16_sum(v);
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// Sum over the wavefront (all 64 lanes active); every lane receives the sum.
// DPP sums inside the four 16-lane rows, then the rows' sums through readlane.
__device__ __forceinline__ double wave_sum(double v) {
    v = row16_sum(v);
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        t += __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16 * r),
                              __builtin_amdgcn_readlane(__double2loint(v), 16 * r));
    return t;
}

// position of value k in a descending order of sv[0..c) (ties: lower index first)
__device__ __forceinline__ int desc_pos(const double* sv, int c, int k) {
    const double x = sv[k];
    int pos = 0;
    for (int j = 0; j < c; ++j) pos += (sv[j] > x) || (sv[j] == x && j < k);
    return pos;
}

// Rank under the Frobenius rule (eqn. curOff6): desc holds kk singular values in
// descending order, extra2 the squared Frobenius norm of what was dropped before
// (rows of a truncated pivoted QR, 0 otherwise); the smallest k with
// sqrt(extra2 + sum_{t >= k} desc[t]^2) < tau, or kk when no k qualifies.  The
// tail is summed from the smallest value up.
__device__ int frob_rank(const double* desc, int kk, double extra2, double tau) {
    double t2 = extra2;
    if (!(sqrt(t2) < tau)) return kk;
    int r = kk;
    for (int k = kk - 1; k >= 0; --k) {
        t2 += desc[k] * desc[k];
        if (sqrt(t2) < tau) r = k;
        else break;
    }
    return r;
}

// Rank rule of the randomized compression: the smallest k with
// sqrt(unc + sum_{t >= k} desc[t]^2) <= eps desc[0], or n + 1 when even k = n
// does not qualify (desc: n values in descending order).
__device__ int rand_rank(const double* desc, int n, double unc, double eps) {
    if (n == 0 || desc[0] == 0.0) return unc == 0.0 ? 0 : n + 1;
    const double thr = eps * desc[0];
    double t2 = unc;
    if (!(sqrt(t2) <= thr)) return n + 1;
    int r = n;
    for (int k = n - 1; k >= 0; --k) {
        t2 += desc[k] * desc[k];
        if (sqrt(t2) <= thr) r = k;
        else break;
    }
    return r;
}

__device__ double block_sum(double v, double* s_s) {
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    __syncthreads();
    if (lane == 0) s_s[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NT / WAVE; ++k) t += s_s[k];
    return t;
}

template <int JG>   // lanes per Jacobi pair
__global__ __launch_bounds__(NT) void k_compress_svd(const DCompress* __restrict__ tasks,
                                                     const DPiece* __restrict__ pieces,
                                                     const int32_t* __restrict__ imap,
                                                     int cap) {
    // With cap doubles of dynamic LDS, R, V and a chunk of ch rows of B live in
    // LDS (2 c^2 + ch c doubles), ch taken from the task's own sizes so that its
    // arithmetic does not depend on the other tasks of the launch; below 16 rows
    // (ch == 0) everything stays in the task's workspace.
    const DCompress T = tasks[blockIdx.x];
    const int M = T.M, c = T.c, tid = threadIdx.x;
    int ch = 0;
    if (c > 0) {
        int64_t t = ((int64_t)cap - 2ll * c * c) / c;
        t = t > M ? M : t;
        t = t > 1024 ? 1024 : t;
        ch = t < 16 ? 0 : (int)t;
    }
    const int lane = tid % WAVE, wv = tid / WAVE;
    constexpr int NW = NT / WAVE;
    __shared__ double s_s[NT / WAVE + 1];
    __shared__ int s_rot;
    extern __shared__ double s_dyn[];
    if (M == 0 || c == 0) {
        if (tid == 0) { *T.rank_out = 0; T.tails[0] = 0.0; }
        return;
    }
    double* __restrict__ B = T.B;
    // ---- assemble B (column-major, ld M)
    for (int64_t e = tid; e < (int64_t)M * c; e += NT) B[e] = 0.0;
    __syncthreads();
    for (int q = 0; q < T.npieces; ++q) {
        const DPiece pc = pieces[T.piece0 + q];
        const int nr = pc.blk.nr, nc = pc.blk.nc;
        for (int e = tid; e < nr * nc; e += NT) {
            const int a = e % nr, b = e / nr;
            const double v = pc.blk.p[e];
            if (!pc.trans) B[(pc.row0 + a) + (int64_t)imap_at(imap, pc.map, b) * M] = v;
            else           B[(pc.row0 + b) + (int64_t)imap_at(imap, pc.map, a) * M] = v;
        }
    }
    __syncthreads();
    const bool lds = ch > 0;
    double* Rm = lds ? s_dyn : T.hv;                      // c x c
    double* Vm = lds ? s_dyn + (size_t)c * c : T.V;       // c x c
    for (int e = tid; e < c * c; e += NT) Rm[e] = 0.0;
    if (lds) {
        // ---- QR of B, chunk by chunk: the triangle R and ch rows of B in LDS.
        // Column j of [R; chunk] is annihilated by a reflector that touches row
        // j of R and the chunk only (R is upper triangular).
        double* Ch = s_dyn + (size_t)2 * c * c;           // ch x c, column-major
        __syncthreads();
        for (int i0 = 0; i0 < M; i0 += ch) {
            const int rows = min(ch, M - i0);
            for (int e = tid; e < rows * c; e += NT) {
                const int r = e % rows, k = e / rows;
                Ch[r + k * ch] = B[(i0 + r) + (int64_t)k * M];
            }
            __syncthreads();
            for (int j = 0; j < c; ++j) {
                double part = 0.0;
                for (int r = tid; r < rows; r += NT) { const double x = Ch[r + j * ch]; part += x * x; }
                const double s2c = block_sum(part, s_s);
                if (s2c == 0.0) continue;                 // nothing below R[j][j] in this chunk
                const double x0 = Rm[j + j * c];
                const double s2 = x0 * x0 + s2c;
                const double xn = sqrt(s2);
                const double alpha = -copysign(xn, x0);
                const double tau = 2.0 / (2.0 * (s2 + fabs(x0) * xn));
                const double v0 = x0 - alpha;
                const double* vj = Ch + j * ch;
                for (int k = j + 1 + wv; k < c; k += NW) {
                    double* ck = Ch + k * ch;
                    double w = 0.0;
                    for (int r = lane; r < rows; r += WAVE) w += vj[r] * ck[r];
                    w = (wave_sum(w) + v0 * Rm[j + k * c]) * tau;
                    for (int r = lane; r < rows; r += WAVE) ck[r] -= w * vj[r];
                    if (lane == 0) Rm[j + k * c] -= w * v0;
                }
                __syncthreads();
                if (tid == 0) Rm[j + j * c] = alpha;
            }
            __syncthreads();
        }
        for (int e = tid; e < c * c; e += NT) Vm[e] = (e % c == e / c) ? 1.0 : 0.0;
        __syncthreads();
    } else {
        // ---- Householder QR of a workspace copy of B, by columns
        double* __restrict__ W = T.Bw;
        for (int64_t e = tid; e < (int64_t)M * c; e += NT) W[e] = B[e];
        __syncthreads();
        const int kq = M < c ? M : c;
        for (int j = 0; j < kq; ++j) {
            double part = 0.0;
            for (int i = j + tid; i < M; i += NT) { const double x = W[i + (int64_t)j * M]; part += x * x; }
            const double s2 = block_sum(part, s_s);
            const double x0 = W[j + (int64_t)j * M];
            const double xn = sqrt(s2);
            const double alpha = xn == 0.0 ? 0.0 : -copysign(xn, x0);
            const double beta = 2.0 * (s2 + fabs(x0) * xn);          // v.v
            __syncthreads();
            if (tid == 0) {
                W[j + (int64_t)j * M] = x0 - alpha;
                Rm[j + (int64_t)j * c] = alpha;
            }
            __syncthreads();
            if (beta > 0.0) {
                const double tau = 2.0 / beta;
                const double* v = W + (int64_t)j * M;
                for (int k = j + 1 + wv; k < c; k += NW) {
                    double* col = W + (int64_t)k * M;
                    double w = 0.0;
#pragma unroll 4
                    for (int i = j + lane; i < M; i += WAVE) w += v[i] * col[i];
                    w = wave_sum(w) * tau;
#pragma unroll 4
                    for (int i = j + lane; i < M; i += WAVE) col[i] -= w * v[i];
                }
            }
            __syncthreads();
        }
        // R: strict upper part from W, diagonal already written; rows >= kq are zero
        for (int e = tid; e < c * c; e += NT) {
            const int a = e % c, k = e / c;
            if (a < k && a < kq) Rm[e] = W[a + (int64_t)k * M];
            Vm[e] = (a == k) ? 1.0 : 0.0;
        }
        __syncthreads();
    }
    // ---- one-sided Jacobi on the columns of R; V accumulates the rotations.
    // Columns whose norm is at the rounding level of R (1e-15 ||R||_F) carry no
    // information; pairs involving them are not rotated, which keeps rounding
    // noise from re-triggering sweeps.
    const int n2 = c + (c & 1);
    const int g = tid / JG, gl = tid % JG;
    const double tol = 4.0e-16 * (double)c;
    double fro = 0.0;
    for (int e = tid; e < c * c; e += NT) fro += Rm[e] * Rm[e];
    fro = block_sum(fro, s_s);
    const double tiny2 = 1e-30 * fro;
    int sweeps_run = 0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        ++sweeps_run;
        for (int t = 0; t < n2 - 1; ++t) {
            for (int i = g; i < n2 / 2; i += NT / JG) {
                int a = (t + i) % (n2 - 1);
                int b = i == 0 ? n2 - 1 : (t - i + n2 - 1) % (n2 - 1);
                const int p = a < b ? a : b, q = a < b ? b : a;
                if (q >= c) continue;
                double* cp = Rm + (size_t)p * c;
                double* cq = Rm + (size_t)q * c;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = gl; r < c; r += JG) {
                    const double x = cp[r], y = cq[r];
                    al += x * x; be += y * y; ga += x * y;
                }
                al = group_sum<JG>(al); be = group_sum<JG>(be); ga = group_sum<JG>(ga);
                if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al * be)) || al <= tiny2 || be <= tiny2) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
                for (int r = gl; r < c; r += JG) {
                    const double x = cp[r], y = cq[r];
                    cp[r] = cs * x - sn * y;
                    cq[r] = sn * x + cs * y;
                }
                double* vp = Vm + (size_t)p * c;
                double* vq = Vm + (size_t)q * c;
                for (int r = gl; r < c; r += JG) {
                    const double x = vp[r], y = vq[r];
                    vp[r] = cs * x - sn * y;
                    vq[r] = sn * x + cs * y;
                }
                if (gl == 0) s_rot = 1;
            }
            __syncthreads();
        }
        const int rot = s_rot;
        __syncthreads();
        if (!rot) break;
    }
    // ---- singular values = column norms of the rotated R (scratch after R in hv)
    double* sv = T.hv + (size_t)c * c;
    for (int k = wv; k < c; k += NT / WAVE) {
        double s2 = 0.0;
        for (int r = lane; r < c; r += WAVE) { const double x = Rm[r + (size_t)k * c]; s2 += x * x; }
        s2 = wave_sum(s2);
        if (lane == 0) sv[k] = sqrt(s2);
    }
    __syncthreads();
    // descending order, ties by column index
    for (int k = tid; k < c; k += NT) T.tails[1 + desc_pos(sv, c, k)] = sv[k];
    __syncthreads();
    const double smax = T.tails[1];
    int r = 0;
    if (T.tau) r = frob_rank(T.tails + 1, c, 0.0, *T.tau);
    else if (smax > 0.0)
        for (int k = 0; k < c; ++k) r += (T.tails[1 + k] >= T.eps * smax) ? 1 : 0;
    // V (c x r): output column pos(k) is column k of the accumulated rotations
    const double* Vsrc = Vm;
    if (!lds) {                           // Vm is T.V itself: stage it in hv (R is done)
        for (int e = tid; e < c * c; e += NT) T.hv[e] = Vm[e];
        __syncthreads();
        Vsrc = T.hv;
    }
    for (int e = tid; e < c * c; e += NT) {
        const int a = e % c, k = e / c;
        const int pos = desc_pos(sv, c, k);
        if (pos < r) T.V[a + (size_t)pos * c] = Vsrc[a + (size_t)k * c];
    }
    if (tid == 0) {
        T.tails[0] = smax;
        T.tails[c + 1] = (double)sweeps_run;     // Jacobi sweeps (work accounting)
        *T.rank_out = r;
    }
}

// ---- truncated SVD for stacked blocks of at most 64 columns ------------------
// Same result as k_compress_svd, reached in fewer synchronisation steps:
//   1. Householder QR of B (row chunks through LDS): B = Q0 R0;
//   2. QR of R0 with column pivoting: R0 P = Q1 R1;
//   3. QR of R1^T: R1^T = Q2 R2, L = R2^T;
//   4. one-sided Jacobi on the columns of L, the rotations J accumulated onto
//      W = Q2: L J = U Sigma, so B = (Q0 Q1 U) Sigma (P Q2 J)^T.
// The two extra triangular QRs make the columns of L graded and nearly
// orthogonal, which cuts the Jacobi sweeps by about half (the QR
// preconditioning of one-sided Jacobi described by Drmac and Veselic), while V
// = P W keeps orthonormal columns to rounding.  1024 threads: in the QRs lane =
// column and wavefront = rows i = seg (mod 16); in Jacobi 16 lanes per column
// pair, reduced with DPP row permutations.
// NTC threads per task (256, 512 or 1024, a tuning choice); SEGC = NTC / 64
// row segments in the QRs.

// Largest v over a wavefront (lowest i on ties); every lane receives (v, i).
// DPP within rows of 16 lanes, then the four row results through readlane.
__device__ __forceinline__ double lane_read(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ float lane_read(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <int CTRL, class T>
__device__ __forceinline__ void argmax_step(T& v, int& i) {
    const T ov = dpp_mov<CTRL>(v);
    const int oi = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xF, 0xF, false);
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}

template <class T>
__device__ __forceinline__ void wave_argmax(T& v, int& i) {
    argmax_step<0xB1>(v, i);
    argmax_step<0x4E>(v, i);
    argmax_step<0x141>(v, i);
    argmax_step<0x140>(v, i);
    T b = lane_read(v, 0);
    int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        const T o = lane_read(v, 16 * r);
        const int oi = __builtin_amdgcn_readlane(i, 16 * r);
        if (o > b || (o == b && oi < bi)) { b = o; bi = oi; }
    }
    v = b;
    i = bi;
}

// In-place Householder QR, optionally with column pivoting (largest remaining
// column norm, lowest index on ties), of the nr x c matrix A in LDS (column-
// major, leading dimension ld, c <= 64).  On exit R is the upper triangle;
// reflector j is H_j = I - tau_j v v^T with v = (v0_j, A[j+1.., j]) acting on
// rows j..nr-1; perm[j] is the original column now at position j (pivot only).
// P: SEGC x WAVE, NV: SEGC elements of LDS scratch.  T: arithmetic type.
template <class T, int NTC>
__device__ void qr64(T* A, int nr, int c, int ld, bool pivot, int* perm, T* hv0, T* htau, T* P, T* NV) {
    constexpr int SEGC = NTC / WAVE;
    const int tid = threadIdx.x, k = tid % WAVE, s = tid / WAVE;
    const int kmax = min(nr, c);
    if (pivot) {
        for (int j = tid; j < c; j += NTC) perm[j] = j;
        __syncthreads();
    }
    for (int j = 0; j < kmax; ++j) {
        // first row > j of this segment (rows i = s mod SEGC)
        const int i0 = j + 1 + ((s - (j + 1)) % SEGC + SEGC) % SEGC;
        if (pivot) {
            T q = 0.0;
            if (k >= j && k < c) {
                for (int i = j + ((s - j) % SEGC + SEGC) % SEGC; i < nr; i += SEGC) {   // rows >= j
                    const T x = A[i + k * ld];
                    q += x * x;
                }
            }
            P[s * WAVE + k] = q;
            __syncthreads();
            T nk = -1.0;
            if (k >= j && k < c) {
                nk = 0.0;
                for (int t = 0; t < SEGC; ++t) nk += P[t * WAVE + k];
            }
            int bi = k;
            T bv = nk;
            wave_argmax(bv, bi);
            __syncthreads();
            if (bi != j) {
                if (k == j)
                    for (int i = s; i < nr; i += SEGC) {
                        const T a = A[i + j * ld];
                        A[i + j * ld] = A[i + bi * ld];
                        A[i + bi * ld] = a;
                    }
                if (tid == 0) {
                    const int t = perm[j];
                    perm[j] = perm[bi];
                    perm[bi] = t;
                }
                __syncthreads();
            }
        }
        // phase 1: partial products of column j with the columns to its right
        const T ajj = A[j + j * ld];
        const T ajk = k < c ? A[j + k * ld] : 0.0;
        T p1 = 0.0, nv = 0.0;
        for (int i = i0; i < nr; i += SEGC) {
            const T vi = A[i + j * ld];
            nv += vi * vi;
            if (k > j && k < c) p1 += vi * A[i + k * ld];
        }
        P[s * WAVE + k] = p1;
        if (k == 0) NV[s] = nv;
        __syncthreads();
        // phase 2: reflector and update.  A column whose squared norm below the
        // diagonal is at the bottom of T's range (denormal in FP32) is taken as
        // zero: 1 / (s2 + |ajj| xn) would overflow.  Callers scale A to max |A| < 1.
        const T tiny_sq = sizeof(T) == 4 ? (T)1e-30 : (T)1e-280;
        T nvt = 0.0;
        for (int t = 0; t < SEGC; ++t) nvt += NV[t];
        T tau = 0.0, v0 = 0.0, alpha = ajj;
        if (nvt > tiny_sq) {
            const T s2 = ajj * ajj + nvt;
            const T xn = sqrt(s2);
            alpha = -copysign(xn, ajj);
            v0 = ajj - alpha;
            tau = 1.0 / (s2 + fabs(ajj) * xn);
        }
        if (tau != 0.0 && k > j && k < c) {
            T w = v0 * ajk;
            for (int t = 0; t < SEGC; ++t) w += P[t * WAVE + k];
            w *= tau;
            if (s == 0) A[j + k * ld] = ajk - w * v0;
            for (int i = i0; i < nr; i += SEGC) A[i + k * ld] -= w * A[i + j * ld];
        }
        if (tid == 0) {
            A[j + j * ld] = alpha;
            hv0[j] = v0;
            htau[j] = tau;
        }
        __syncthreads();
    }
}

// Rotation (cs, sn) that makes columns with squared norms al, be and product
// ga orthogonal (one-sided Jacobi): zeta = (be - al) / (2 ga),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), cs = 1 / sqrt(1 + t^2),
// sn = cs t.  FP64 uses correctly rounded division and square roots; FP32 the
// hardware reciprocal, square root and reciprocal square root (about 1 ulp,
// the size of the FP32 rounding of every other step of that path).
__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double& cs, double& sn) {
    const double zeta = (be - al) / (2.0 * ga);
    const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    cs = 1.0 / sqrt(1.0 + t * t);
    sn = cs * t;
}
__device__ __forceinline__ void jacobi_rotation(float al, float be, float ga, float& cs, float& sn) {
    const float zeta = (be - al) * __builtin_amdgcn_rcpf(2.0f * ga);
    const float t = copysignf(1.0f, zeta) * __builtin_amdgcn_rcpf(fabsf(zeta) + __builtin_amdgcn_sqrtf(1.0f + zeta * zeta));
    cs = __builtin_amdgcn_rsqf(1.0f + t * t);
    sn = cs * t;
}

// R1 (c x c upper triangular, into X as F, ld ldx) and perm (the original column
// at each position) of B (M x c, column-major in HBM, scaled by inv_scale):
// FP64 Gram matrix from LDS chunks of 64 rows (2 x 2 register blocks, upper
// half mirrored), then right-looking Cholesky with diagonal pivoting (largest
// remaining diagonal, lowest index on ties) in LDS.  work: at least
// 64 (65) + 64 (65) doubles of LDS.  NTC >= 1024 is not needed: blocks loop.
template <class F, int NTC>
__device__ void gram_chol_r1(const double* __restrict__ B, int M, int c, double inv_scale, double* work, F* X,
                             int ldx, int* perm) {
    constexpr int RCH = 64;
    const int tid = threadIdx.x, lane = tid % WAVE;
    const int ld = c | 1, ldb = c + 1;
    double* G = work;                        // c x c (ld)
    double* Bc = work + WAVE * (WAVE + 1);   // RCH x (c + 1), row-major
    __shared__ double s_d[2];
    __shared__ int s_p[2];
    const int nb = (c + 1) / 2, nblk = nb * nb;
    constexpr int BPT = (32 * 32 + NTC - 1) / NTC;    // 2 x 2 blocks per thread (c <= 64)
    double acc[BPT][4];
#pragma unroll
    for (int u = 0; u < BPT; ++u) acc[u][0] = acc[u][1] = acc[u][2] = acc[u][3] = 0.0;
    for (int a0 = 0; a0 < M; a0 += RCH) {
        const int nr = min(RCH, M - a0);
        for (int e = tid; e < nr * c; e += NTC) {
            const int r = e % nr, k = e / nr;
            Bc[r * ldb + k] = B[(a0 + r) + (int64_t)k * M] * inv_scale;
        }
        if (c & 1)
            for (int r = tid; r < nr; r += NTC) Bc[r * ldb + c] = 0.0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int blk = tid + u * NTC;
            const int bi = blk / max(nb, 1), bk = blk % max(nb, 1);
            if (blk < nblk && bi <= bk) {
                const int i0 = 2 * bi, k0 = 2 * bk;
                for (int r = 0; r < nr; ++r) {
                    const double* row = Bc + r * ldb;
                    const double x0 = row[i0], x1 = row[i0 + 1], y0 = row[k0], y1 = row[k0 + 1];
                    acc[u][0] = fma(x0, y0, acc[u][0]);
                    acc[u][1] = fma(x0, y1, acc[u][1]);
                    acc[u][2] = fma(x1, y0, acc[u][2]);
                    acc[u][3] = fma(x1, y1, acc[u][3]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int blk = tid + u * NTC;
        const int bi = blk / max(nb, 1), bk = blk % max(nb, 1);
        if (blk < nblk && bi <= bk) {
            const int i0 = 2 * bi, k0 = 2 * bk, i1 = i0 + 1, k1 = k0 + 1;
            G[i0 + k0 * ld] = acc[u][0]; G[k0 + i0 * ld] = acc[u][0];
            if (k1 < c) { G[i0 + k1 * ld] = acc[u][1]; G[k1 + i0 * ld] = acc[u][1]; }
            if (i1 < c) { G[i1 + k0 * ld] = acc[u][2]; G[k0 + i1 * ld] = acc[u][2]; }
            if (i1 < c && k1 < c) { G[i1 + k1 * ld] = acc[u][3]; G[k1 + i1 * ld] = acc[u][3]; }
        }
    }
    __shared__ int s_mark[WAVE];             // 1 once a column is pivoted
    for (int j = tid; j < WAVE; j += NTC) s_mark[j] = 0;
    __syncthreads();
    double trace = 0.0;
    for (int k = 0; k < c; ++k) trace += G[k + k * ld];
    const double stop = 1.1102230246251565e-16 * (double)c * trace;
    // G stays in the original order: step k pivots on the largest remaining
    // diagonal p_k and updates the remaining rows and columns only, so row p_k
    // keeps the values of step k (R1[k][l] = G[p_k][p_l] / sqrt(G[p_k][p_k]))
    int kk = c;
    for (int k = 0; k < c; ++k) {
        if (tid < WAVE) {
            double v = lane < c && !s_mark[lane] ? G[lane + lane * ld] : -1.0;
            int i = lane;
            for (int o = WAVE / 2; o > 0; o >>= 1) {
                const double ov = __shfl_xor(v, o);
                const int oi = __shfl_xor(i, o);
                if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
            }
            if (lane == 0) {
                s_d[0] = v;
                s_p[0] = i;
                if (v > stop) { s_mark[i] = 1; perm[k] = i; }
            }
        }
        __syncthreads();
        const double dk = s_d[0];
        const int pk = s_p[0];
        if (!(dk > stop)) { kk = k; break; }             // uniform: the rest is numerically zero
        const double inv = 1.0 / dk;
        for (int e = tid; e < c * c; e += NTC) {
            const int i = e % c, j = e / c;
            if (!s_mark[i] && !s_mark[j]) G[i + j * ld] -= G[i + pk * ld] * G[pk + j * ld] * inv;
        }
        __syncthreads();
    }
    if (tid == 0) {                                      // the unpivoted columns follow in order
        int q = kk;
        for (int j = 0; j < c; ++j)
            if (!s_mark[j]) perm[q++] = j;
    }
    __syncthreads();
    // X = R1 (rows >= kk zero)
    for (int e = tid; e < c * c; e += NTC) {
        const int i = e % c, j = e / c;
        F v = (F)0;
        if (i <= j && i < kk) {
            const int pi = perm[i], pj = perm[j];
            v = (F)(G[pi + pj * ld] / sqrt(G[pi + pi * ld]));
        }
        X[i + j * ldx] = v;
    }
    __syncthreads();
}

// T = float: the reduced QRs and Jacobi in FP32 (mixed precision); B, the
// projection B V and all outputs stay FP64.
template <class F, int NTC, bool GRAM>
__global__ __launch_bounds__(NTC) void k_compress_svd64(const DCompress* __restrict__ tasks,
                                                        const DPiece* __restrict__ pieces,
                                                        const int32_t* __restrict__ imap, int cap_d) {
    constexpr int SEGC = NTC / WAVE;
    const DCompress T = tasks[blockIdx.x];
    const int M = T.M, c = T.c, tid = threadIdx.x;
    extern __shared__ double sm_d[];
    F* sm = reinterpret_cast<F*>(sm_d);
    const int cap = cap_d * (int)(sizeof(double) / sizeof(F));
    __shared__ int s_perm[WAVE];
    if (M == 0 || c == 0) {
        if (tid == 0) { *T.rank_out = 0; T.tails[0] = 0.0; }
        return;
    }
    F* P = sm;                               // SEGC x WAVE
    F* NV = P + SEGC * WAVE;                 // SEGC
    F* hv0 = NV + SEGC;                      // WAVE
    F* htau = hv0 + WAVE;                    // WAVE
    F* sv = htau + WAVE;                     // WAVE
    F* region = sv + WAVE;
    const int reg = cap - (SEGC * WAVE + SEGC + 3 * WAVE);
    const int ldc = c | 1;
    F* X = region + reg - c * ldc;           // c x c, kept to the end
    // ---- assemble B (column-major, ld M) in global memory; it stays for the projection
    double* __restrict__ B = T.B;
    double amax = 0.0;
    if (T.npieces < 0)                       // B already in place (sketched block)
        for (int64_t e = tid; e < (int64_t)M * c; e += NTC) amax = fmax(amax, fabs(B[e]));
    else {
        for (int64_t e = tid; e < (int64_t)M * c; e += NTC) B[e] = 0.0;
        __syncthreads();
    }
    for (int q = 0; q < T.npieces; ++q) {
        const DPiece pc = pieces[T.piece0 + q];
        const int nr = pc.blk.nr, nc = pc.blk.nc;
        for (int e = tid; e < nr * nc; e += NTC) {
            const int a = e % nr, b = e / nr;
            const double v = pc.blk.p[e];
            amax = fmax(amax, fabs(v));
            if (!pc.trans) B[(pc.row0 + a) + (int64_t)imap_at(imap, pc.map, b) * M] = v;
            else           B[(pc.row0 + b) + (int64_t)imap_at(imap, pc.map, a) * M] = v;
        }
    }
    // the factorization works on B / 2^e with max |B / 2^e| in [0.5, 1), so squared
    // column norms and their products stay inside the range of F; singular values
    // are scaled back exactly, V does not change
    __shared__ double s_amax[SEGC];
    for (int o = WAVE / 2; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o));
    if (tid % WAVE == 0) s_amax[tid / WAVE] = amax;
    __syncthreads();
    amax = 0.0;
    for (int t = 0; t < SEGC; ++t) amax = fmax(amax, s_amax[t]);
    const int bexp = amax > 0.0 ? ilogb(amax) + 1 : 0;
    const double inv_scale = ldexp(1.0, -bexp), scale = ldexp(1.0, bexp);
    if constexpr (GRAM) {
        // ---- 1'-2'. R1 and its column order from the FP64 Gram matrix: G =
        // (B / 2^e)^T (B / 2^e), then Cholesky with diagonal pivoting, P^T G P =
        // R1^T R1: in exact arithmetic the R and the column order of the pivoted
        // QR of steps 1-2 (the largest remaining diagonal is the largest
        // remaining column norm).  It stops once the largest remaining diagonal
        // is below c u trace(G) (rows below are zero), so singular values under
        // about sqrt(c u) sigma_0 are not resolved.
        gram_chol_r1<F, NTC>(B, M, c, inv_scale, reinterpret_cast<double*>(region), X, ldc, s_perm);
    } else {
    // ---- 1. QR of B through LDS chunks: [R (c rows); next rows of B]
    {
        F* A = region;
        const int rows_cap = (reg - c * ldc) / c - 1;
        const int ldA = rows_cap | 1;
        int r0 = 0, nrA = 0;
        bool first = true;
        while (r0 < M) {
            const int top = first ? 0 : c;
            const int nnew = min(M - r0, rows_cap - top);
            if (!first) {                            // keep R, clear the reflectors below it
                for (int e = tid; e < c * c; e += NTC) {
                    const int i = e % c, j = e / c;
                    if (i > j) A[i + j * ldA] = 0.0;
                }
            }
            for (int e = tid; e < nnew * c; e += NTC) {
                const int k = e / nnew, i = e - k * nnew;
                A[top + i + k * ldA] = (F)(B[(r0 + i) + (int64_t)k * M] * inv_scale);
            }
            nrA = top + nnew;
            __syncthreads();
            qr64<F, NTC>(A, nrA, c, ldA, false, nullptr, hv0, htau, P, NV);
            r0 += nnew;
            first = false;
        }
        // R0 (upper, rows < min(nrA, c)) into X
        for (int e = tid; e < c * c; e += NTC) {
            const int i = e % c, k = e / c;
            X[i + k * ldc] = (i <= k && i < nrA) ? A[i + k * ldA] : 0.0;
        }
        __syncthreads();
    }
    // ---- 2. R0 P = Q1 R1
    qr64<F, NTC>(X, c, c, ldc, true, s_perm, hv0, htau, P, NV);
    }
    // ---- 3. R1^T = Q2 R2 (A2 after W in the region); L = R2^T into X
    F* W = region;
    F* A2 = region + c * ldc;
    for (int e = tid; e < c * c; e += NTC) {
        const int i = e % c, k = e / c;
        A2[i + k * ldc] = (k <= i) ? X[k + i * ldc] : 0.0;
    }
    __syncthreads();
    qr64<F, NTC>(A2, c, c, ldc, false, nullptr, hv0, htau, P, NV);
    for (int e = tid; e < c * c; e += NTC) {
        const int i = e % c, k = e / c;
        X[i + k * ldc] = (k <= i) ? A2[k + i * ldc] : 0.0;
        W[i + k * ldc] = (i == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    // W = Q2 = H_0 ... H_{c-1} I, applied right to left
    {
        const int k = tid % WAVE, sg = tid / WAVE;
        for (int j = c - 1; j >= 0; --j) {
            const F tau = htau[j];
            if (tau == (F)0) continue;               // uniform: H_j = I
            const int i0 = j + 1 + ((sg - (j + 1)) % SEGC + SEGC) % SEGC;
            const F v0 = hv0[j];
            F p1 = 0;
            const F wjk = k < c ? W[j + k * ldc] : (F)0;
            if (k < c)
                for (int i = i0; i < c; i += SEGC) p1 += A2[i + j * ldc] * W[i + k * ldc];
            P[sg * WAVE + k] = p1;
            __syncthreads();
            if (k < c) {
                F w = v0 * wjk;
                for (int t = 0; t < SEGC; ++t) w += P[t * WAVE + k];
                w *= tau;
                if (sg == 0) W[j + k * ldc] = wjk - w * v0;
                for (int i = i0; i < c; i += SEGC) W[i + k * ldc] -= w * A2[i + j * ldc];
            }
            __syncthreads();
        }
    }
    // ---- 4. one-sided Jacobi on the columns of L; W accumulates the rotations
    int sweeps_run = 0;
    {
        const int n2 = c + (c & 1), npair = n2 / 2;
        const int g = tid / 16, gl = tid % 16;
        // rotation threshold ~3.6 c u and rounding-level columns (u: unit roundoff of F)
        const F u = sizeof(F) == 8 ? (F)1.1102230246251565e-16 : (F)5.9604645e-8;
        const F tol = (F)3.6 * u * (F)c;
        double f = 0.0;
        for (int e = tid; e < c * c; e += NTC) {
            const int i = e % c, k = e / c;
            const double x = (double)X[i + k * ldc];
            f += x * x;
        }
        f = wave_sum(f);
        __shared__ double s_fro[SEGC];
        if (tid % WAVE == 0) s_fro[tid / WAVE] = f;
        __syncthreads();
        double fro = 0.0;
        for (int t = 0; t < SEGC; ++t) fro += s_fro[t];
        const F tiny2 = (F)(81.0 * (double)u * (double)u * fro);
        constexpr int EPL = WAVE / 16;             // elements per lane (c <= 64)
        // a sweep whose rotations all had |gamma| <= sqrt(tol) sqrt(alpha beta)
        // ends the iteration: by the quadratic convergence of the sweeps the
        // next one would only rotate below the tol level, so it is not run
        const F tol_hi = sqrt(tol);
        __shared__ int s_big;
        for (int sweep = 0; sweep < 40; ++sweep) {
            if (tid == 0) s_big = 0;
            __syncthreads();
            ++sweeps_run;
            for (int t = 0; t < n2 - 1; ++t) {
                // NTC / 16 groups of 16 lanes take the npair disjoint pairs of round t
                for (int gp = g; gp < npair; gp += NTC / 16) {
                    // round-robin pair of round t (t + gp < 2 (n2 - 1): no division)
                    int a = t + gp;
                    if (a >= n2 - 1) a -= n2 - 1;
                    const int b = gp == 0 ? n2 - 1 : (t >= gp ? t - gp : t - gp + n2 - 1);
                    const int p = a < b ? a : b, q = a < b ? b : a;
                    const bool act = q < c;
                    F xp[EPL], xq[EPL], wp[EPL], wq[EPL];
                    F al = 0, be = 0, ga = 0;
#pragma unroll
                    for (int u = 0; u < EPL; ++u) {
                        const int r = gl + 16 * u;
                        const bool in = act && r < c;
                        xp[u] = in ? X[r + p * ldc] : (F)0;
                        xq[u] = in ? X[r + q * ldc] : (F)0;
                        wp[u] = in ? W[r + p * ldc] : (F)0;          // issued with X, used after the rotation
                        wq[u] = in ? W[r + q * ldc] : (F)0;
                    }
#pragma unroll
                    for (int u = 0; u < EPL; ++u) {
                        al += xp[u] * xp[u];
                        be += xq[u] * xq[u];
                        ga += xp[u] * xq[u];
                    }
                    al = row16_sum(al);
                    be = row16_sum(be);
                    ga = row16_sum(ga);
                    const F d = sqrt(al * be);
                    if (act && ga != (F)0 && fabs(ga) > tol * d && al > tiny2 && be > tiny2) {
                        F cs, sn;
                        jacobi_rotation(al, be, ga, cs, sn);
#pragma unroll
                        for (int u = 0; u < EPL; ++u) {
                            const int r = gl + 16 * u;
                            if (r < c) {
                                X[r + p * ldc] = cs * xp[u] - sn * xq[u];
                                X[r + q * ldc] = sn * xp[u] + cs * xq[u];
                                W[r + p * ldc] = cs * wp[u] - sn * wq[u];
                                W[r + q * ldc] = sn * wp[u] + cs * wq[u];
                            }
                        }
                        if (gl == 0 && fabs(ga) > tol_hi * d) s_big = 1;
                    }
                }
                __syncthreads();
            }
            const int big = s_big;
            __syncthreads();
            if (!big) break;
        }
    }
    // ---- singular values, order, rank, V = P W
    __shared__ double s_sv[WAVE];
    for (int k = tid / WAVE; k < c; k += SEGC) {
        double s2 = 0.0;
        for (int r = tid % WAVE; r < c; r += WAVE) { const double x = (double)X[r + k * ldc]; s2 += x * x; }
        s2 = wave_sum(s2);
        if (tid % WAVE == 0) s_sv[k] = sqrt(s2) * scale;
    }
    __syncthreads();
    (void)sv;
    for (int k = tid; k < c; k += NTC) T.tails[1 + desc_pos(s_sv, c, k)] = s_sv[k];
    double smax = 0.0;
    for (int k = 0; k < c; ++k) smax = fmax(smax, s_sv[k]);
    int r = 0;
    if (T.nb2) {
        // sketched block of a randomized compression: the fewest directions whose
        // discarded part (tail of this block plus the energy of B outside the
        // sketch) has Frobenius norm <= eps sigma_0; c + 1 when none qualifies
        __syncthreads();                          // the sorted values above are written
        double cap2 = 0.0;
        for (int k = 0; k < c; ++k) cap2 += T.tails[1 + k] * T.tails[1 + k];
        const double unc = T.rand_full ? 0.0 : fmax(0.0, *T.nb2 - cap2);
        r = rand_rank(T.tails + 1, c, unc, T.eps);
    } else if (T.tau) {
        __syncthreads();                          // the sorted values above are written
        r = frob_rank(T.tails + 1, c, 0.0, *T.tau);
    } else if (smax > 0.0)
        for (int k = 0; k < c; ++k) r += (s_sv[k] >= T.eps * smax) ? 1 : 0;
    for (int e = tid; e < c * c; e += NTC) {
        const int a = e % c, k = e / c;
        const int pos = desc_pos(s_sv, c, k);
        if (pos < r) T.V[s_perm[a] + (size_t)pos * c] = (double)W[a + k * ldc];   // (r = c + 1: all)
    }
    if (tid == 0) {
        T.tails[0] = smax;
        T.tails[c + 1] = (double)sweeps_run;     // Jacobi sweeps (work accounting)
        *T.rank_out = r;
    }
}

// ---- randomized compression (stacked blocks of at most 64 columns) ------------
// Adaptive randomized range finder on the nonzero part of the stacked block B
// (M x c): rows and columns that are zero (structural padding of the stacked
// pieces) take no part in the draw.
//   k_rand_sketch: (first pass) assemble B as the SVD kernels do, ||B||_F^2 and
//     the number c_nz of nonzero columns; the sketch width is
//     l = min(requested, c_nz) (written into the sketch task).  Y = B^T Omega
//     (c x l): Omega(a', t) = -1 when the top bit of SplitMix64 of the counter
//     (key << 34) + (a' << 6) + t is set, a' the position of row a among the
//     nonzero rows of B (SplitMix64: Steele, Lea and Flood, 2014); Householder
//     QR of Y, the explicit Q (c x l, kept in hv); C = B Q (M x l) into Bw.
//   k_compress_svd64<double> on the sketch tasks (C in place, npieces < 0,
//     with the rank rule of the sketch, rand_rank);
//   k_rand_finish: accept when the rank is below l or the sketch spans all c_nz
//     columns, then V = Q V_C (c x r), tails and rank; else flag the task (the
//     host doubles the requested width and runs the three launches again).
// bf16: the sketch product takes B rounded to BF16 (the signs are exact in
// BF16) with FP32 accumulation; C and everything after stay FP64.
constexpr int NTR = 1024;
constexpr int SEGR = NTR / WAVE;

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float bf16_round(float f) {   // to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return f;
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// LDS of k_rand_sketch, in doubles: Y and Q (c x l, ld <= 65), P (SEGR x WAVE),
// NV (SEGR), hv0 and htau (WAVE each), then NTR sign masks and NTR row ids.
constexpr size_t kRandLds = (size_t)(2 * (WAVE + 1) * WAVE + SEGR * WAVE + SEGR + 2 * WAVE) * sizeof(double) +
                            (size_t)NTR * (sizeof(uint64_t) + sizeof(int32_t));

__global__ __launch_bounds__(NTR) void k_rand_sketch(const DCompress* __restrict__ tasks,
                                                     const DRand* __restrict__ rt,
                                                     DCompress* __restrict__ ctasks,
                                                     const DPiece* __restrict__ pieces,
                                                     const int32_t* __restrict__ imap, int first, int bf16) {
    const DCompress T = tasks[blockIdx.x];
    const DRand R = rt[blockIdx.x];
    const int M = T.M, c = T.c, tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    if (!R.active || M <= 0 || c <= 0 || c > WAVE) return;
    extern __shared__ double sm[];
    const int ldy = c | 1;
    double* Y = sm;                          // c x l
    double* Qs = Y + (WAVE + 1) * WAVE;      // c x l
    double* P = Qs + (WAVE + 1) * WAVE;      // SEGR x WAVE
    double* NV = P + SEGR * WAVE;            // SEGR
    double* hv0 = NV + SEGR;                 // WAVE
    double* htau = hv0 + WAVE;               // WAVE
    uint64_t* masks = reinterpret_cast<uint64_t*>(htau + WAVE);   // NTR
    int32_t* rowid = reinterpret_cast<int32_t*>(masks + NTR);     // NTR
    __shared__ double s_red[SEGR];
    __shared__ int s_cnt[SEGR];
    double* __restrict__ B = T.B;
    if (first) {
        for (int64_t e = tid; e < (int64_t)M * c; e += NTR) B[e] = 0.0;
        __syncthreads();
        double f = 0.0;
        for (int q = 0; q < T.npieces; ++q) {
            const DPiece pc = pieces[T.piece0 + q];
            const int nr = pc.blk.nr, nc = pc.blk.nc;
            for (int e = tid; e < nr * nc; e += NTR) {
                const int a = e % nr, b = e / nr;
                const double v = pc.blk.p[e];
                f += v * v;
                if (!pc.trans) B[(pc.row0 + a) + (int64_t)imap_at(imap, pc.map, b) * M] = v;
                else           B[(pc.row0 + b) + (int64_t)imap_at(imap, pc.map, a) * M] = v;
            }
        }
        f = wave_sum(f);
        if (lane == 0) s_red[w] = f;
        __syncthreads();                     // B assembled, partial sums written
        int nzc = 0;                         // nonzero columns, a wave per column
        for (int k = w; k < c; k += SEGR) {
            bool nz = false;
            for (int a = lane; a < M; a += WAVE) nz |= B[a + (int64_t)k * M] != 0.0;
            nzc += __ballot(nz) != 0ull ? 1 : 0;
        }
        if (lane == 0) s_cnt[w] = nzc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            int n = 0;
            for (int q = 0; q < SEGR; ++q) { t += s_red[q]; n += s_cnt[q]; }
            T.hv[(size_t)c * c] = t;         // ||B||_F^2
            T.hv[(size_t)c * c + 1] = (double)n;
        }
        __syncthreads();
    }
    const int cnz = (int)T.hv[(size_t)c * c + 1];
    const int l = min(R.l, cnz);
    if (tid == 0) {
        ctasks[blockIdx.x].c = l;
        ctasks[blockIdx.x].rand_full = l == cnz ? 1 : 0;
    }
    if (l <= 0) return;                      // B = 0: the sketch task has no columns
    for (int e = tid; e < ldy * l; e += NTR) Y[e] = 0.0;
    // ---- Y = B^T Omega over chunks of NTR rows
    int base = 0;                            // nonzero rows before the chunk
    for (int a0 = 0; a0 < M; a0 += NTR) {
        const int na = min(NTR, M - a0);
        bool nz = false;
        if (tid < na)
            for (int k = 0; k < c; ++k) nz |= B[(a0 + tid) + (int64_t)k * M] != 0.0;
        const uint64_t bm = __ballot(nz);
        if (lane == 0) s_cnt[w] = __popcll(bm);
        __syncthreads();
        int pre = base, tot = 0;
        for (int q = 0; q < SEGR; ++q) {
            const int t = s_cnt[q];
            pre += q < w ? t : 0;
            tot += t;
        }
        rowid[tid] = pre + __popcll(bm & ((1ull << lane) - 1ull));
        base += tot;
        __syncthreads();
        for (int a = w; a < na; a += SEGR) {
            const uint64_t cnt = ((uint64_t)R.key << 34) + ((uint64_t)rowid[a] << 6) + (uint64_t)lane;
            const bool neg = lane < l && (splitmix64(cnt) >> 63) != 0;
            const uint64_t m = __ballot(neg);
            if (lane == 0) masks[a] = m;
        }
        __syncthreads();
        for (int k = w; k < c; k += SEGR) {
            if (lane < l) {
                const double* bc = B + (int64_t)k * M + a0;
                if (bf16) {
                    float acc = 0.f;
                    for (int a = 0; a < na; ++a) {
                        const float b = bf16_round((float)bc[a]);
                        acc += ((masks[a] >> lane) & 1ull) ? -b : b;
                    }
                    Y[k + lane * ldy] += (double)acc;
                } else {
                    double acc = 0.0;
                    for (int a = 0; a < na; ++a) {
                        const double b = bc[a];
                        acc += ((masks[a] >> lane) & 1ull) ? -b : b;
                    }
                    Y[k + lane * ldy] += acc;
                }
            }
        }
        __syncthreads();                     // s_cnt, rowid and masks are reused
    }
    // ---- Householder QR of Y (c x l), then Q = H_0 ... H_{l-1} I[:, :l]
    qr64<double, NTR>(Y, c, l, ldy, false, nullptr, hv0, htau, P, NV);
    for (int e = tid; e < c * l; e += NTR) {
        const int i = e % c, t = e / c;
        Qs[i + t * ldy] = (i == t) ? 1.0 : 0.0;
    }
    __syncthreads();
    {
        const int k = lane, sg = w;
        for (int j = l - 1; j >= 0; --j) {
            const double tau = htau[j];
            if (tau == 0.0) continue;                    // uniform: H_j = I
            const int i0 = j + 1 + ((sg - (j + 1)) % SEGR + SEGR) % SEGR;
            const double v0 = hv0[j];
            double p1 = 0.0;
            const double qjk = k < l ? Qs[j + k * ldy] : 0.0;
            if (k < l)
                for (int i = i0; i < c; i += SEGR) p1 += Y[i + j * ldy] * Qs[i + k * ldy];
            P[sg * WAVE + k] = p1;
            __syncthreads();
            if (k < l) {
                double wv = v0 * qjk;
                for (int t = 0; t < SEGR; ++t) wv += P[t * WAVE + k];
                wv *= tau;
                if (sg == 0) Qs[j + k * ldy] = qjk - wv * v0;
                for (int i = i0; i < c; i += SEGR) Qs[i + k * ldy] -= wv * Y[i + j * ldy];
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < c * l; e += NTR) {
        const int i = e % c, t = e / c;
        T.hv[i + (size_t)t * c] = Qs[i + t * ldy];
    }
    // ---- C = B Q (M x l) into Bw
    for (int64_t e = tid; e < (int64_t)M * l; e += NTR) {
        const int a = (int)(e % M), t = (int)(e / M);
        double acc = 0.0;
        for (int k = 0; k < c; ++k) acc += B[a + (int64_t)k * M] * Qs[k + t * ldy];
        T.Bw[e] = acc;
    }
}

// flags[i]: bit 0 = the sketch was too narrow (rank not below l, l < c_nz); bits
// 1..7 the Jacobi sweeps of the sketched block's SVD; bits 8.. the width l.
__global__ __launch_bounds__(256) void k_rand_finish(const DCompress* __restrict__ tasks,
                                                     const DRand* __restrict__ rt,
                                                     const DCompress* __restrict__ ctasks,
                                                     int32_t* __restrict__ flags) {
    const DCompress T = tasks[blockIdx.x];
    const DRand R = rt[blockIdx.x];
    const int tid = threadIdx.x;
    if (!R.active || T.M <= 0 || T.c <= 0 || T.c > WAVE) {
        if (tid == 0) flags[blockIdx.x] = 0;
        return;
    }
    const DCompress C = ctasks[blockIdx.x];
    const int l = C.c, c = T.c;
    const int rc = l > 0 ? *C.rank_out : 0;
    const int sweeps = l > 0 ? (int)C.tails[l + 1] : 0;
    const bool accept = C.rand_full || rc < l;
    if (!accept) {
        if (tid == 0) flags[blockIdx.x] = 1 | (sweeps << 1) | (l << 8);
        return;
    }
    const int r = min(rc, l);
    for (int e = tid; e < c * r; e += 256) {
        const int a = e % c, p = e / c;
        double acc = 0.0;
        for (int t = 0; t < l; ++t) acc += T.hv[a + (size_t)t * c] * C.V[t + (size_t)p * l];
        T.V[a + (size_t)p * c] = acc;
    }
    for (int k = tid; k < c; k += 256) T.tails[1 + k] = k < l ? C.tails[1 + k] : 0.0;
    if (tid == 0) {
        T.tails[0] = l > 0 ? C.tails[0] : 0.0;
        T.tails[c + 1] = (double)sweeps;
        *T.rank_out = r;
        flags[blockIdx.x] = (sweeps << 1) | (l << 8);
    }
}

// Sign of the auxiliary variables: every column of V (c x r, r = *rank_out)
// gets its entry of largest magnitude positive (lowest row on exact ties).  The
// factorization does not depend on these signs; a randomized sketch of a later
// stacked block, whose rows include these variables, does.  One wavefront per task.
__global__ __launch_bounds__(WAVE) void k_v_sign(const DCompress* __restrict__ tasks) {
    const DCompress T = tasks[blockIdx.x];
    const int lane = threadIdx.x;
    if (T.M <= 0 || T.c <= 0) return;
    const int c = T.c, r = min(*T.rank_out, c);
    for (int p = 0; p < r; ++p) {
        double* col = T.V + (size_t)p * c;
        double bv = -1.0;
        int bi = c;
        for (int a = lane; a < c; a += WAVE) {
            const double v = fabs(col[a]);
            if (v > bv) { bv = v; bi = a; }             // rows ascending: first of equals kept
        }
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (bi >= c) continue;
        const bool neg = col[bi] < 0.0;
        if (neg)
            for (int a = lane; a < c; a += WAVE) col[a] = -col[a];
    }
}

// ---------------------------------------------------------------- large stacked blocks
// Compress for c > 64 columns (FP64, 1024 threads, matrices in the task's
// workspace): the pipeline of k_compress_svd64 with global-memory QRs.
//   1. B / 2^e = Q0 R0 (Householder on a copy of B; the reflector in LDS).
//   2. R0 P = Q1 R1 (column pivoting, norms recomputed each step).  With a
//      truncation level t = trunc_rel * epsilon > 0 the factorization stops at the first k whose
//      trailing block has ||R1[k:, k:]||_F <= t |R1[0, 0]| (<= t sigma_0); the
//      dropped rows move each sigma_i^2 by at most that squared norm, so at
//      t = epsilon / 100 the singular values near the cut move by about
//      1/20000 of it (used in mixed precision).  t = 0 keeps every row
//      that is not exactly zero.
//   3. R1[:k, :]^T = Q2 R2, L = R2^T (k x k, lower triangular and graded).
//   4. one-sided Jacobi on the columns of L with W = Q2 accumulating the
//      rotations: B P = Q0 Q1 L Q2^T, so V = P Q2 J and sigma = column norms.
// Singular values beyond k (t > 0) are reported as the bound of the dropped
// part.  Workspace: Bw (M x c) for step 1; hv holds X (c x c: R0, R1, then L),
// A2 (c x c), W (c x c) and c scratch doubles.  LDS: reflector (M doubles),
// column norms, perm and the singular values.
constexpr int NTL = 1024;
constexpr int NWL = NTL / WAVE;

__device__ double blk_sum_l(double v, double* s_red) {
    v = wave_sum(v);
    __syncthreads();
    if (threadIdx.x % WAVE == 0) s_red[threadIdx.x / WAVE] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NWL; ++k) t += s_red[k];
    return t;
}

// Householder QR step on column j of the nr x ncol matrix A (column-major, ld):
// rows j..nr-1 reduced, columns j+1..ncol-1 updated; the reflector v (v[0] =
// v0, v[i - j] = A[i, j] for i > j) is left in A below the diagonal and in
// s_v (LDS copy, length nr - j).  Returns tau (0: H = I).  Every thread calls it.
__device__ double hh_step(double* A, int64_t ld, int nr, int ncol, int j, double* s_v, double* s_red,
                          double* v0_out) {
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    double part = 0.0;
    for (int i = j + 1 + tid; i < nr; i += NTL) {
        const double x = A[i + j * ld];
        s_v[i - j] = x;
        part += x * x;
    }
    const double nvt = blk_sum_l(part, s_red);        // barrier inside: s_v visible
    const double ajj = A[j + j * ld];
    double tau = 0.0, v0 = 0.0, alpha = ajj;
    if (nvt > 1e-280) {
        const double s2 = ajj * ajj + nvt;
        const double xn = sqrt(s2);
        alpha = -copysign(xn, ajj);
        v0 = ajj - alpha;
        tau = 1.0 / (s2 + fabs(ajj) * xn);
    }
    if (tau != 0.0) {
        // each lane keeps its elements of the column in registers (8 per pass)
        constexpr int E = 8;
        for (int k = j + 1 + wv; k < ncol; k += NWL) {
            double* col = A + k * ld;
            const double cj = col[j];
            double w = 0.0;
            if (nr - (j + 1) <= WAVE * E) {
                double x[E];
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const int i = j + 1 + lane + WAVE * u;
                    x[u] = i < nr ? col[i] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const int i = j + 1 + lane + WAVE * u;
                    if (i < nr) w += s_v[i - j] * x[u];
                }
                w = (wave_sum(w) + v0 * cj) * tau;
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const int i = j + 1 + lane + WAVE * u;
                    if (i < nr) col[i] = x[u] - w * s_v[i - j];
                }
            } else {                                  // longer columns: two passes
                for (int i0 = j + 1; i0 < nr; i0 += WAVE * E) {
                    double x[E];
#pragma unroll
                    for (int u = 0; u < E; ++u) {
                        const int i = i0 + lane + WAVE * u;
                        x[u] = i < nr ? col[i] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < E; ++u) {
                        const int i = i0 + lane + WAVE * u;
                        if (i < nr) w += s_v[i - j] * x[u];
                    }
                }
                w = (wave_sum(w) + v0 * cj) * tau;
                for (int i0 = j + 1; i0 < nr; i0 += WAVE * E) {
                    double x[E];
#pragma unroll
                    for (int u = 0; u < E; ++u) {
                        const int i = i0 + lane + WAVE * u;
                        x[u] = i < nr ? col[i] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < E; ++u) {
                        const int i = i0 + lane + WAVE * u;
                        if (i < nr) col[i] = x[u] - w * s_v[i - j];
                    }
                }
            }
            if (lane == 0) col[j] = cj - w * v0;
        }
    }
    __syncthreads();
    if (tid == 0) A[j + j * ld] = alpha;
    *v0_out = v0;
    return tau;
}

// One Jacobi rotation of columns p, q of L (length kk) and of W (length c) by a
// group of GL lanes (GL = 16, 32 or 64, aligned inside a wavefront); each lane
// holds E elements of each L column in registers, so all loads of a pass are in
// flight together.  Columns longer than GL * E take two passes.
template <int GL>
__device__ __forceinline__ double grp_sum(double v) {
    v = row16_sum(v);
    if constexpr (GL >= 32) {          // the group's DPP rows combined through readlane
        const double lo = lane_read(v, 0) + lane_read(v, 16);
        const double hi = lane_read(v, 32) + lane_read(v, 48);
        if constexpr (GL >= 64) v = lo + hi;
        else v = (threadIdx.x % WAVE) < 32 ? lo : hi;
    }
    return v;
}

// Returns 0 (no rotation), 1 (a rotation with |gamma| <= tol_hi sqrt(alpha
// beta)) or 2 (a larger one).
template <int GL, int E>
__device__ int jac_pair(double* __restrict__ cp, double* __restrict__ cq, double* __restrict__ wp,
                        double* __restrict__ wq, int kk, int c, int gl, double tol, double tol_hi, double tiny2) {
    constexpr int SPAN = GL * E;
    double xp[E], xq[E];
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int r0 = 0; r0 < kk; r0 += SPAN) {
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int r = r0 + gl + GL * u;
            xp[u] = r < kk ? cp[r] : 0.0;
            xq[u] = r < kk ? cq[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < E; ++u) {
            al += xp[u] * xp[u];
            be += xq[u] * xq[u];
            ga += xp[u] * xq[u];
        }
    }
    al = grp_sum<GL>(al);
    be = grp_sum<GL>(be);
    ga = grp_sum<GL>(ga);
    if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al * be)) || al <= tiny2 || be <= tiny2) return 0;
    const int kind = fabs(ga) > tol_hi * sqrt(al * be) ? 2 : 1;
    const double zeta = (be - al) / (2.0 * ga);
    const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
    for (int r0 = 0; r0 < kk; r0 += SPAN) {
        if (kk > SPAN) {                         // reload the chunk (uniform)
#pragma unroll
            for (int u = 0; u < E; ++u) {
                const int r = r0 + gl + GL * u;
                xp[u] = r < kk ? cp[r] : 0.0;
                xq[u] = r < kk ? cq[r] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int r = r0 + gl + GL * u;
            if (r < kk) {
                cp[r] = cs * xp[u] - sn * xq[u];
                cq[r] = sn * xp[u] + cs * xq[u];
            }
        }
    }
    constexpr int EW = E > 8 ? 8 : E;            // W in passes of GL * 8 rows
    for (int r0 = 0; r0 < c; r0 += GL * EW) {
        double yp[EW], yq[EW];
#pragma unroll
        for (int u = 0; u < EW; ++u) {
            const int r = r0 + gl + GL * u;
            yp[u] = r < c ? wp[r] : 0.0;
            yq[u] = r < c ? wq[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < EW; ++u) {
            const int r = r0 + gl + GL * u;
            if (r < c) {
                wp[r] = cs * yp[u] - sn * yq[u];
                wq[r] = sn * yp[u] + cs * yq[u];
            }
        }
    }
    return kind;
}

// A sweep round of the parallel ordering: pair i of round t joins columns
// (t + i) mod (n2 - 1) and (t - i) mod (n2 - 1), pair 0 taking column n2 - 1.
template <int GL, int E>
__device__ void jac_round(double* X, double* W, int64_t ldc, int kk, int c, int n2, int t, double tol,
                          double tol_hi, double tiny2, int* s_big) {
    const int g = threadIdx.x / GL, gl = threadIdx.x % GL;
    for (int pi = g; pi < n2 / 2; pi += NTL / GL) {
        const int a = (t + pi) % (n2 - 1);
        const int b = pi == 0 ? n2 - 1 : (t - pi + n2 - 1) % (n2 - 1);
        const int pp = a < b ? a : b, qq = a < b ? b : a;
        if (qq >= kk) continue;                  // uniform over the group
        if (jac_pair<GL, E>(X + pp * ldc, X + qq * ldc, W + pp * ldc, W + qq * ldc, kk, c, gl, tol, tol_hi,
                            tiny2) == 2 &&
            gl == 0)
            *s_big = 1;
    }
}

// State kept in hv after X, A2, W and the panel scratch (c^2 each) between the
// launches of the split form: the pivot order (c values) and a header.
enum { LH_KK = 0, LH_SCALE, LH_REST2, LH_TOL, LH_TINY2, LH_ROT, LH_DONE, LH_BIG, LH_N };
static_assert(LH_N <= 8, "the header has 8 doubles");
constexpr int KK_BLK = 8;                    // columns per block of the multi-work-group Jacobi
constexpr int KK_LDS_MAX = 1150;             // rows of L a block pair may hold in LDS (16 x 1150 doubles)

// mode 0: the whole pipeline in this work-group; mode 5: after the assembly and
// the scaled copy Bw (launch_assemble_large) and the tall QR of Bw by the panel
// and update launches, the pivoted QR and A2 (the LQ and Q2 follow as
// launches); mode 6: from A2 factored and W = Q2 formed, L and the state for
// the block rounds; mode 2: singular values, rank and V after the block rounds;
// mode 7: mode 0 from the tall QR of Bw done by the panel and update launches;
// mode 8: after the Gram matrix and its pivoted Cholesky (launch_gram_chol), A2
// and the state, as mode 5 leaves them; mode 9: from there the LQ, Q2, Jacobi
// and finish in this work-group.
// (The mode is a template parameter: each stage compiles to its own kernel.)
template <int mode>
__global__ __launch_bounds__(NTL) void k_compress_large(const DCompress* __restrict__ tasks,
                                                        const DPiece* __restrict__ pieces,
                                                        const int32_t* __restrict__ imap, double trunc_rel,
                                                        double jac_u) {
    const DCompress T = tasks[blockIdx.x];
    const int M = T.M, c = T.c, tid = threadIdx.x;
    const int lane = tid % WAVE, wv = tid / WAVE;
    const double trunc = trunc_rel * T.eps;
    extern __shared__ double sl[];
    __shared__ double s_red[NWL];
    __shared__ int s_piv;
    __shared__ int s_rot;
    if (M == 0 || c == 0) {
        if (tid == 0 && mode != 2) { *T.rank_out = 0; T.tails[0] = 0.0; }
        return;
    }
    double* hst = T.hv + 4 * (size_t)c * c;                 // pivot order (c), then the header
    double* hdr = hst + c;
    // LDS: reflector (max(M, c) + 1), norms (c), sv (c), hv0 (c), htau (c), perm (c), pos (c)
    const int vlen = (M > c ? M : c) + 1;
    double* s_v = sl;
    double* s_nrm = s_v + vlen;
    double* s_sv = s_nrm + c;
    double* s_hv0 = s_sv + c;
    double* s_tau = s_hv0 + c;
    int* s_perm = reinterpret_cast<int*>(s_tau + c);
    int* s_pos = s_perm + c;
    double* X = T.hv;                                   // c x c, ld c
    double* A2 = X + (size_t)c * c;                     // c x c
    double* W = A2 + (size_t)c * c;                     // c x c
    const int64_t ldc = c;
    int kk = 0;
    double rest2 = 0.0, scale = 1.0;
    if (mode == 8) {
        // A2 = R1[:kk, :]^T in pivot order from the rows of R kept transposed in X
        // over the original columns (Rt[i + J c] = R(J, i)); W = E
        kk = (int)hdr[LH_KK];
        for (int k = tid; k < c; k += NTL) s_perm[k] = (int)hst[k];
        __syncthreads();
        for (int e = tid; e < c * kk; e += NTL) {
            const int q = e % c, J = e / c;
            A2[q + J * ldc] = q >= J ? X[s_perm[q] + (int64_t)J * ldc] : 0.0;
            W[q + J * ldc] = q == J ? 1.0 : 0.0;
        }
        if (tid == 0) hdr[LH_DONE] = 0.0;
        return;
    }
    if (mode == 2) {
        kk = (int)hdr[LH_KK];
        scale = hdr[LH_SCALE];
        rest2 = hdr[LH_REST2];
        for (int k = tid; k < c; k += NTL) s_perm[k] = (int)hst[k];
        __syncthreads();
    } else {
    double* Bw = T.Bw;
    if (mode != 6 && mode != 9) {
    if (mode == 5 || mode == 7) {
        scale = hdr[LH_SCALE];
    } else {
    // ---- assemble B (column-major, ld M; kept for the projection), max |B|
    double* __restrict__ B = T.B;
    for (int64_t e = tid; e < (int64_t)M * c; e += NTL) B[e] = 0.0;
    __syncthreads();
    double amax = 0.0;
    for (int q = 0; q < T.npieces; ++q) {
        const DPiece pc = pieces[T.piece0 + q];
        const int nr = pc.blk.nr, nc = pc.blk.nc;
        for (int e = tid; e < nr * nc; e += NTL) {
            const int a = e % nr, b = e / nr;
            const double v = pc.blk.p[e];
            amax = fmax(amax, fabs(v));
            if (!pc.trans) B[(pc.row0 + a) + (int64_t)imap_at(imap, pc.map, b) * M] = v;
            else           B[(pc.row0 + b) + (int64_t)imap_at(imap, pc.map, a) * M] = v;
        }
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o));
    __syncthreads();
    if (lane == 0) s_red[wv] = amax;
    __syncthreads();
    amax = 0.0;
    for (int t = 0; t < NWL; ++t) amax = fmax(amax, s_red[t]);
    const int bexp = amax > 0.0 ? ilogb(amax) + 1 : 0;
    const double inv_scale = ldexp(1.0, -bexp);
    scale = ldexp(1.0, bexp);
    // ---- 1. tall QR of B / 2^e on the copy Bw
    for (int64_t e = tid; e < (int64_t)M * c; e += NTL) Bw[e] = B[e] * inv_scale;
    __syncthreads();
    for (int j = 0; j < (M < c ? M : c); ++j) {
        double v0;
        hh_step(Bw, M, M, c, j, s_v, s_red, &v0);
        __syncthreads();
    }
    }                                                   // mode != 5
    const int kq = M < c ? M : c;
    for (int e = tid; e < c * c; e += NTL) {
        const int i = e % c, k = e / c;
        X[e] = (i <= k && i < kq) ? Bw[i + (int64_t)k * M] : 0.0;
    }
    for (int k = tid; k < c; k += NTL) s_perm[k] = k;
    __syncthreads();
    // ---- 2. QRCP of R0 (rows < kq are the only nonzero ones), truncated
    double r00 = 0.0;
    for (int j = 0; j < kq; ++j) {
        // squared norms of columns j..c-1 over rows j..kq-1
        for (int k = j + wv; k < c; k += NWL) {
            double q = 0.0;
            for (int i = j + lane; i < kq; i += WAVE) { const double x = X[i + k * ldc]; q += x * x; }
            q = wave_sum(q);
            if (lane == 0) s_nrm[k] = q;
        }
        __syncthreads();
        if (wv == 0) {
            double best = -1.0, tot = 0.0;
            int bi = INT_MAX;
            for (int k = j + lane; k < c; k += WAVE) {
                const double q = s_nrm[k];
                tot += q;
                if (q > best) { best = q; bi = k; }
            }
            tot = wave_sum(tot);
            wave_argmax(best, bi);
            if (lane == 0) { s_piv = bi; s_red[0] = tot; s_red[1] = best; }
        }
        __syncthreads();
        const int p = s_piv;
        const double tot = s_red[0], best = s_red[1];
        if (j == 0) r00 = sqrt(best);
        // stop: nothing left, or the trailing block is below the truncation level
        if (!(best > 0.0) || tot <= trunc * trunc * r00 * r00) { rest2 = tot; break; }
        __syncthreads();
        if (p != j) {
            for (int i = tid; i < c; i += NTL) {
                const double a = X[i + j * ldc];
                X[i + j * ldc] = X[i + p * ldc];
                X[i + p * ldc] = a;
            }
            if (tid == 0) { const int t = s_perm[j]; s_perm[j] = s_perm[p]; s_perm[p] = t; }
            __syncthreads();
        }
        double v0;
        hh_step(X, ldc, kq, c, j, s_v, s_red, &v0);
        kk = j + 1;
        __syncthreads();
    }
    // ---- 3. A2 = R1[:kk, :]^T (c x kk, lower trapezoidal), QR -> R2, L = R2^T
    for (int e = tid; e < c * kk; e += NTL) {
        const int i = e % c, k = e / c;
        A2[i + k * ldc] = (i >= k) ? X[k + i * ldc] : 0.0;
    }
    if (mode == 5) {
        // the LQ and Q2 then run as panel and update launches (W = E now)
        for (int e = tid; e < c * kk; e += NTL) {
            const int i = e % c, k = e / c;
            W[i + k * ldc] = (i == k) ? 1.0 : 0.0;
        }
        for (int k = tid; k < c; k += NTL) hst[k] = (double)s_perm[k];
        if (tid == 0) {
            hdr[LH_KK] = kk;
            hdr[LH_SCALE] = scale;
            hdr[LH_REST2] = rest2;
            hdr[LH_DONE] = 0.0;
        }
        return;
    }
    }                                                   // mode != 6, 9
    if (mode == 6 || mode == 9) {
        kk = (int)hdr[LH_KK];
        scale = hdr[LH_SCALE];
        rest2 = hdr[LH_REST2];
        for (int k = tid; k < c; k += NTL) s_perm[k] = (int)hst[k];
    }
    if (mode != 6) {
    __syncthreads();
    for (int j = 0; j < kk; ++j) {
        double v0;
        const double tau = hh_step(A2, ldc, c, kk, j, s_v, s_red, &v0);
        if (tid == 0) { s_hv0[j] = v0; s_tau[j] = tau; }
        __syncthreads();
    }
    }
    for (int e = tid; e < kk * kk; e += NTL) {
        const int i = e % kk, k = e / kk;
        X[i + k * ldc] = (k <= i) ? A2[k + i * ldc] : 0.0;   // L (kk x kk, ld c)
    }
    if (mode != 6)
    for (int e = tid; e < c * kk; e += NTL) {
        const int i = e % c, k = e / c;
        W[i + k * ldc] = (i == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    // W = Q2[:, :kk] = H_0 ... H_{kk-1} E, applied right to left; H_j changes
    // rows j.. of columns j.. only (mode 6: done by the update launches)
    for (int j = (mode == 6 ? -1 : kk - 1); j >= 0; --j) {
        const double tau = s_tau[j];
        if (tau == 0.0) continue;                        // uniform
        const double v0 = s_hv0[j];
        for (int i = j + 1 + tid; i < c; i += NTL) s_v[i - j] = A2[i + j * ldc];
        __syncthreads();
        for (int k = j + wv; k < kk; k += NWL) {
            double* col = W + k * ldc;
            double w = 0.0;
            for (int i = j + 1 + lane; i < c; i += WAVE) w += s_v[i - j] * col[i];
            w = (wave_sum(w) + v0 * col[j]) * tau;
            for (int i = j + 1 + lane; i < c; i += WAVE) col[i] -= w * s_v[i - j];
            if (lane == 0) col[j] -= w * v0;
        }
        __syncthreads();
    }
    // ---- 4. one-sided Jacobi on the kk columns of L; W follows.  Pairs run in
    // groups of 16 lanes (64 at once) up to 128 rows, then 32 up to 256 and 64
    // beyond (columns longer than 512 in several passes).
    // In mode 6 it runs here only when L is too tall for the block rounds.
    // rotation threshold 3.6 jac_u kk (jac_u: FP64 or, in mixed precision, FP32
    // unit roundoff); the zero-column guard stays at FP64 level
    const double u = 1.1102230246251565e-16;
    const double tol = 3.6 * jac_u * (double)kk, tol_hi = sqrt(tol);
    double f = 0.0;
    for (int e = tid; e < kk * kk; e += NTL) {
        const double x = X[(e % kk) + (e / kk) * ldc];
        f += x * x;
    }
    const double fro = blk_sum_l(f, s_red);
    const double tiny2 = 81.0 * u * u * fro;
    const bool inline_jacobi = mode == 0 || mode == 7 || mode == 9 || kk > KK_LDS_MAX;
    // Jacobi sweeps of this task (work accounting): counted here when the sweeps
    // run inline, else one per sweep of the block rounds by k_large_flags
    if (tid == 0) T.tails[c + 1] = 0.0;
    if (mode == 6) {
        for (int k = tid; k < c; k += NTL) hst[k] = (double)s_perm[k];
        if (tid == 0) {
            hdr[LH_KK] = kk;
            hdr[LH_SCALE] = scale;
            hdr[LH_REST2] = rest2;
            hdr[LH_TOL] = tol;
            hdr[LH_TINY2] = tiny2;
            hdr[LH_ROT] = 0.0;
            hdr[LH_BIG] = 0.0;
            hdr[LH_DONE] = (inline_jacobi || kk <= 1) ? 1.0 : 0.0;
        }
    }
    if (kk > 1 && inline_jacobi) {
        const int n2 = kk + (kk & 1);
        // a sweep without a rotation above sqrt(tol) sqrt(alpha beta) ends it
        // (the next would only rotate below the tol level); s_rot holds that flag
        int sweeps_run = 0;
        for (int sweep = 0; sweep < 40; ++sweep) {
            if (tid == 0) s_rot = 0;
            __syncthreads();
            ++sweeps_run;
            for (int t = 0; t < n2 - 1; ++t) {
                // at most 8 elements of a column per lane (more spill registers)
                if (kk <= 128) jac_round<16, 8>(X, W, ldc, kk, c, n2, t, tol, tol_hi, tiny2, &s_rot);
                else if (kk <= 256) jac_round<32, 8>(X, W, ldc, kk, c, n2, t, tol, tol_hi, tiny2, &s_rot);
                else jac_round<64, 8>(X, W, ldc, kk, c, n2, t, tol, tol_hi, tiny2, &s_rot);
                __syncthreads();
            }
            const int rot = s_rot;
            __syncthreads();
            if (!rot) break;
        }
        if (tid == 0) T.tails[c + 1] = (double)sweeps_run;
    }
    if (mode == 6) return;
    }                                                   // mode != 2
    // ---- singular values, order, rank, V = P W
    for (int k = wv; k < kk; k += NWL) {
        double s2 = 0.0;
        for (int r = lane; r < kk; r += WAVE) { const double x = X[r + k * ldc]; s2 += x * x; }
        s2 = wave_sum(s2);
        if (lane == 0) s_sv[k] = sqrt(s2) * scale;
    }
    __syncthreads();
    for (int k = tid; k < kk; k += NTL) s_pos[k] = desc_pos(s_sv, kk, k);
    __syncthreads();
    double smax = 0.0;
    for (int k = 0; k < kk; ++k) smax = fmax(smax, s_sv[k]);
    const double bound = sqrt(fmax(rest2, 0.0)) * scale;
    for (int k = tid; k < kk; k += NTL) T.tails[1 + s_pos[k]] = s_sv[k];
    for (int k = kk + tid; k < c; k += NTL) T.tails[1 + k] = bound;
    int r = 0;
    if (T.tau) {
        __syncthreads();                          // the sorted values above are written
        r = frob_rank(T.tails + 1, kk, bound * bound, *T.tau);
    } else if (smax > 0.0)
        for (int k = 0; k < kk; ++k) r += (s_sv[k] >= T.eps * smax) ? 1 : 0;
    for (int e = tid; e < c * kk; e += NTL) {
        const int a = e % c, k = e / c;
        const int pos = s_pos[k];
        if (pos < r) T.V[s_perm[a] + (size_t)pos * c] = W[a + k * ldc];
    }
    if (tid == 0) {
        T.tails[0] = smax;
        *T.rank_out = r;
    }
}

// Blocked Householder QR over many work-groups, for the large stacked blocks.
// A panel of QB columns is reduced by one work-group per task, which also forms
// T of the compact WY form H_j0 ... H_j0+nb-1 = I - V T V^T (column a of V is
// v0_a at row j0 + a and the matrix below it); the other columns then receive
// the panel's transformation from work-groups of QB columns, reading each
// element twice and writing it once per panel instead of once per column.
//   which 0: tall QR of Bw (M x c, ld M), C <- C - V T^T V^T C to the right;
//   which 1: QR of A2 (c x kk, ld c), the LQ step, likewise;
//   which 2: W <- H_j0 ... H_j0+nb-1 W = W - V T V^T W with the panels of the
//            LQ, applied last panel first: W = Q2 E from W = E.
// tau, v0 and T of panel p stay in the task's scratch area (hv + 3 c^2).
constexpr int QB = 16;
constexpr int QB_SCR = 2 * QB + QB * QB;     // scratch doubles per panel

struct QrView {
    double* A;                               // the matrix being factored (V lives in it)
    int64_t ld;
    int nr, ncol, kq;                        // rows, columns, reflectors
    double* C;                               // the matrix updated (which 2: W)
    int ccol;                                // its columns
    double* scr;                             // panel scratch base
};

template <int which>
__device__ inline bool qr_view(const DCompress& T, QrView& v) {
    const int M = T.M, c = T.c;
    if (M == 0 || c == 0) return false;
    v.scr = T.hv + 3 * (size_t)c * c;
    if (which == 0) {
        v.A = T.Bw; v.ld = M; v.nr = M; v.ncol = c; v.kq = M < c ? M : c;
        v.C = T.Bw; v.ccol = c;
    } else {
        const double* hdr = T.hv + 4 * (size_t)c * c + c;
        if (hdr[LH_DONE] != 0.0) return false;
        const int kk = (int)hdr[LH_KK];
        v.A = T.hv + (size_t)c * c; v.ld = c; v.nr = c; v.ncol = kk; v.kq = kk;
        v.C = which == 2 ? T.hv + 2 * (size_t)c * c : v.A; v.ccol = kk;
    }
    return true;
}

template <int which>
__global__ __launch_bounds__(NTL) void k_qr_panel(const DCompress* __restrict__ tasks, int j0) {
    const DCompress T = tasks[blockIdx.x];
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    QrView Q;
    if (!qr_view<which>(T, Q) || j0 >= Q.kq) return;
    const int nb = min(QB, Q.kq - j0);
    extern __shared__ double s_vp[];
    __shared__ double s_red[NWL];
    __shared__ double s_S[QB * QB];
    double* A = Q.A;
    const int64_t ld = Q.ld;
    double* scr = Q.scr + (size_t)(j0 / QB) * QB_SCR;        // tau (QB), v0 (QB), T (QB x QB)
    for (int j = j0; j < j0 + nb; ++j) {
        double v0;
        const double tau = hh_step(A, ld, Q.nr, j0 + nb, j, s_vp, s_red, &v0);
        if (tid == 0) { scr[j - j0] = tau; scr[QB + (j - j0)] = v0; }
        __syncthreads();
    }
    // S = V^T V (a <= b), a wavefront per pair
    for (int pr = wv; pr < nb * nb; pr += NWL) {
        const int a = pr % nb, b = pr / nb;
        if (a > b) continue;                                  // uniform over the wavefront
        const double* va = A + (int64_t)(j0 + a) * ld;
        const double* vb = A + (int64_t)(j0 + b) * ld;
        double d = 0.0;
        for (int r = j0 + b + 1 + lane; r < Q.nr; r += WAVE) d += va[r] * vb[r];
        d = wave_sum(d);
        if (lane == 0) {
            const double vab = (a == b) ? scr[QB + a] : va[j0 + b];     // V[j0+b, a]
            s_S[a + b * QB] = d + vab * scr[QB + b];
        }
    }
    __syncthreads();
    if (tid == 0) {
        double* Tm = scr + 2 * QB;                            // Tm[a + b QB] = T[a][b]
        for (int e = 0; e < QB * QB; ++e) Tm[e] = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double tb = scr[b];
            Tm[b + b * QB] = tb;
            for (int a = 0; a < b; ++a) {                     // T[0:b, b] = -tau_b T[0:b, 0:b] S[0:b, b]
                double z = 0.0;
                for (int k = a; k < b; ++k) z += Tm[a + k * QB] * s_S[k + b * QB];
                Tm[a + b * QB] = -tb * z;
            }
        }
    }
}

template <int which>
__global__ __launch_bounds__(NTL) void k_qr_update(const DCompress* __restrict__ tasks, int j0) {
    const DCompress T = tasks[blockIdx.y];
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    QrView Q;
    if (!qr_view<which>(T, Q) || j0 >= Q.kq) return;
    const int nb = min(QB, Q.kq - j0);
    const int cfirst = which == 2 ? j0 : j0 + nb;             // columns the panel changes
    const int c0 = cfirst + blockIdx.x * QB;
    if (c0 >= Q.ccol) return;
    const int ncc = min(QB, Q.ccol - c0);
    __shared__ double s_W[QB * QB], s_W2[QB * QB];
    const double* A = Q.A;
    const int64_t ld = Q.ld;
    const int nr = Q.nr;
    const double* scr = Q.scr + (size_t)(j0 / QB) * QB_SCR;
    const double* v0 = scr + QB;
    const double* Tm = scr + 2 * QB;
    double* col = Q.C + (int64_t)(c0 + wv) * ld;              // a wavefront per column
    auto vat = [&](int r, int a) -> double {                   // V[r, a]
        const int d = j0 + a;
        return r < d ? 0.0 : (r == d ? v0[a] : A[r + (int64_t)d * ld]);
    };
    if (wv < ncc) {
        double acc[QB];
#pragma unroll
        for (int a = 0; a < QB; ++a) acc[a] = 0.0;
        for (int r = j0 + lane; r < nr; r += WAVE) {
            const double x = col[r];
#pragma unroll
            for (int a = 0; a < QB; ++a)
                if (a < nb) acc[a] += vat(r, a) * x;
        }
#pragma unroll
        for (int a = 0; a < QB; ++a) {
            const double t = wave_sum(acc[a]);
            if (lane == 0) s_W[a + wv * QB] = t;
        }
    }
    __syncthreads();
    if (tid < QB * QB) {                                       // W2 = T^T W (which 0, 1) or T W (which 2)
        const int a = tid % QB, cc = tid / QB;
        double z = 0.0;
        if (a < nb && cc < ncc) {
            if (which == 2)
                for (int b = a; b < nb; ++b) z += Tm[a + b * QB] * s_W[b + cc * QB];
            else
                for (int b = 0; b <= a; ++b) z += Tm[b + a * QB] * s_W[b + cc * QB];
        }
        s_W2[a + cc * QB] = z;
    }
    __syncthreads();
    if (wv < ncc) {
        double w2[QB];
#pragma unroll
        for (int a = 0; a < QB; ++a) w2[a] = s_W2[a + wv * QB];
        for (int r = j0 + lane; r < nr; r += WAVE) {
            double x = col[r];
#pragma unroll
            for (int a = 0; a < QB; ++a)
                if (a < nb) x -= vat(r, a) * w2[a];
            col[r] = x;
        }
    }
}

// One round of the block one-sided Jacobi over the columns of L (split form):
// the kk columns form blocks of KK_BLK; round t pairs the blocks by the same
// parallel ordering as single columns, and one work-group per block pair (all
// tasks of the launch, blockIdx.y = task) copies its (up to) 16 columns of L
// to LDS, runs one sweep of rotations over all pairs among them (a wavefront
// per pair, Q accumulating the rotations), writes the columns back and
// updates the same 16 columns of W by W Q.  Every rotation obeys the rotation
// test of the single-column form, so the result is that of one-sided Jacobi with
// another pair order.
__global__ __launch_bounds__(NTL) void k_large_round(const DCompress* __restrict__ tasks, int t) {
    const DCompress T = tasks[blockIdx.y];
    const int c = T.c, tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    if (T.M == 0 || c == 0) return;
    const double* hdr = T.hv + 4 * (size_t)c * c + c;
    if (hdr[LH_DONE] != 0.0) return;
    const int kk = (int)hdr[LH_KK];
    const int nbk = (kk + KK_BLK - 1) / KK_BLK, nb2 = nbk + (nbk & 1);
    const int pi = blockIdx.x;
    if (t >= nb2 - 1 || pi >= nb2 / 2) return;
    const int a = (t + pi) % (nb2 - 1);
    const int b = pi == 0 ? nb2 - 1 : (t - pi + nb2 - 1) % (nb2 - 1);
    if (a >= nbk || b >= nbk) return;                           // the dummy block
    const double tol = hdr[LH_TOL], tiny2 = hdr[LH_TINY2], tol_hi = sqrt(tol);
    double* X = T.hv;
    double* W = T.hv + 2 * (size_t)c * c;
    const int64_t ldc = c;
    extern __shared__ double sx[];                              // 16 columns of L, ld kk
    __shared__ double sq[16 * 16];
    __shared__ int s_col[16];
    __shared__ int s_rot, s_big;
    const int na = min(KK_BLK, kk - a * KK_BLK), nbb = min(KK_BLK, kk - b * KK_BLK);
    const int ncol = na + nbb;
    if (tid < 16) s_col[tid] = tid < na ? a * KK_BLK + tid : (tid < ncol ? b * KK_BLK + (tid - na) : -1);
    if (tid < 256) sq[tid] = (tid % 16 == tid / 16) ? 1.0 : 0.0;
    if (tid == 0) { s_rot = 0; s_big = 0; }
    __syncthreads();
    for (int e = tid; e < ncol * kk; e += NTL) {
        const int sl_ = e / kk, r = e - sl_ * kk;
        sx[e] = X[r + s_col[sl_] * ldc];
    }
    __syncthreads();
    // one sweep over the 16 slots: 15 rounds of 8 disjoint pairs, a wavefront each
    for (int t2 = 0; t2 < 15; ++t2) {
        if (wv < 8) {
            const int i = wv;
            const int p0 = (t2 + i) % 15, q0 = i == 0 ? 15 : (t2 - i + 15) % 15;
            const int p = p0 < q0 ? p0 : q0, q = p0 < q0 ? q0 : p0;
            if (q < ncol) {
                double* xp = sx + (size_t)p * kk;
                double* xq = sx + (size_t)q * kk;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = lane; r < kk; r += WAVE) {
                    const double x = xp[r], y = xq[r];
                    al += x * x; be += y * y; ga += x * y;
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be) && al > tiny2 && be > tiny2) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
                    for (int r = lane; r < kk; r += WAVE) {
                        const double x = xp[r], y = xq[r];
                        xp[r] = cs * x - sn * y;
                        xq[r] = sn * x + cs * y;
                    }
                    if (lane < 16) {
                        const double x = sq[p * 16 + lane], y = sq[q * 16 + lane];
                        sq[p * 16 + lane] = cs * x - sn * y;
                        sq[q * 16 + lane] = sn * x + cs * y;
                    }
                    if (lane == 0) {
                        s_rot = 1;
                        if (fabs(ga) > tol_hi * sqrt(al * be)) s_big = 1;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!s_rot) return;                                         // uniform: nothing moved
    for (int e = tid; e < ncol * kk; e += NTL) {
        const int sl_ = e / kk, r = e - sl_ * kk;
        X[r + s_col[sl_] * ldc] = sx[e];
    }
    // W[:, cols] = W[:, cols] Q, one row per thread: the row in registers, Q read
    // from LDS one output column at a time (unrolling the column loop as well
    // keeps all of Q in registers and spills)
    for (int r = tid; r < c; r += NTL) {
        double w[16];
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) w[s2] = s2 < ncol ? W[r + s_col[s2] * ldc] : 0.0;
#pragma unroll 1
        for (int s2 = 0; s2 < ncol; ++s2) {
            double acc = 0.0;
#pragma unroll
            for (int s1 = 0; s1 < 16; ++s1) acc += w[s1] * sq[s2 * 16 + s1];
            W[r + s_col[s2] * ldc] = acc;
        }
    }
    if (tid == 0) {
        const_cast<double*>(hdr)[LH_ROT] = 1.0;
        if (s_big) const_cast<double*>(hdr)[LH_BIG] = 1.0;
    }
}

// End of a sweep of the block rounds: out[task] = 1 if the task made a rotation
// with |gamma| > sqrt(tol) sqrt(alpha beta) during the sweep (it goes on), else
// the task is marked done: by the quadratic convergence of the sweeps the next
// one would only rotate below the tol level.
__global__ void k_large_flags(const DCompress* __restrict__ tasks, int n, int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DCompress T = tasks[i];
    if (T.M == 0 || T.c == 0) { out[i] = 0; return; }
    double* hdr = T.hv + 4 * (size_t)T.c * T.c + T.c;
    if (hdr[LH_DONE] == 0.0) T.tails[T.c + 1] += 1.0;     // the task ran this sweep
    const int go = hdr[LH_DONE] == 0.0 && hdr[LH_BIG] != 0.0;
    hdr[LH_ROT] = 0.0;
    hdr[LH_BIG] = 0.0;
    if (!go) hdr[LH_DONE] = 1.0;
    out[i] = go;
}

// ---------------------------------------------------------------- assembly of large stacked blocks
// B (M x c, column-major, kept for the projection) over many work-groups:
// zero it, scatter the pieces (a work-group per piece) while the largest |entry|
// goes to an atomic maximum (non-negative doubles order as their bit patterns),
// then for the QR route the scaled copy Bw = B / 2^e and the scale in the header
// (what mode 0 does in one work-group).  The maximum sits in the Cholesky state
// area (CH_AMAX), which nothing else uses before the Gram matrix is formed.
constexpr int ASM_T = 256;
// the Cholesky state of the Gram route (d, then these) at hv + 3 c^2
enum { CH_J = 0, CH_DONE, CH_R00SQ, CH_STOP, CH_AMAX, CH_N };

__device__ inline unsigned long long* asm_amax(const DCompress& T) {
    return reinterpret_cast<unsigned long long*>(T.hv + 3 * (size_t)T.c * T.c + T.c + CH_AMAX);
}

__global__ __launch_bounds__(ASM_T) void k_asm_zero(const DCompress* __restrict__ tasks) {
    const DCompress T = tasks[blockIdx.y];
    if (T.M == 0 || T.c == 0) return;
    const int64_t n = (int64_t)T.M * T.c;
    if (blockIdx.x == 0 && threadIdx.x == 0) *asm_amax(T) = 0ull;
    for (int64_t e = (int64_t)blockIdx.x * ASM_T + threadIdx.x; e < n; e += (int64_t)gridDim.x * ASM_T)
        T.B[e] = 0.0;
}

__global__ __launch_bounds__(ASM_T) void k_asm_scatter(const DCompress* __restrict__ tasks,
                                                       const DPiece* __restrict__ pieces,
                                                       const int32_t* __restrict__ imap) {
    const DCompress T = tasks[blockIdx.y];
    if (T.M == 0 || T.c == 0 || (int)blockIdx.x >= T.npieces) return;
    const DPiece pc = pieces[T.piece0 + blockIdx.x];
    const int nr = pc.blk.nr, nc = pc.blk.nc, M = T.M;
    double* __restrict__ B = T.B;
    double amax = 0.0;
    for (int e = threadIdx.x; e < nr * nc; e += ASM_T) {
        const int a = e % nr, b = e / nr;
        const double v = pc.blk.p[e];
        amax = fmax(amax, fabs(v));
        if (!pc.trans) B[(pc.row0 + a) + (int64_t)imap_at(imap, pc.map, b) * M] = v;
        else           B[(pc.row0 + b) + (int64_t)imap_at(imap, pc.map, a) * M] = v;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o));
    __shared__ double s_m[ASM_T / WAVE];
    if (threadIdx.x % WAVE == 0) s_m[threadIdx.x / WAVE] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < ASM_T / WAVE; ++k) amax = fmax(amax, s_m[k]);
        if (amax > 0.0) atomicMax(asm_amax(T), (unsigned long long)__double_as_longlong(amax));
    }
}

__global__ __launch_bounds__(ASM_T) void k_asm_scale(const DCompress* __restrict__ tasks) {
    const DCompress T = tasks[blockIdx.y];
    if (T.M == 0 || T.c == 0) return;
    const double amax = __longlong_as_double((long long)*asm_amax(T));
    const int bexp = amax > 0.0 ? ilogb(amax) + 1 : 0;
    const double inv_scale = ldexp(1.0, -bexp);
    const int64_t n = (int64_t)T.M * T.c;
    for (int64_t e = (int64_t)blockIdx.x * ASM_T + threadIdx.x; e < n; e += (int64_t)gridDim.x * ASM_T)
        T.Bw[e] = T.B[e] * inv_scale;
    if (blockIdx.x == 0 && threadIdx.x == 0) T.hv[4 * (size_t)T.c * T.c + T.c + LH_SCALE] = ldexp(1.0, bexp);
}

// ---------------------------------------------------------------- large blocks via the Gram matrix
// R1 and the column order of a stacked block with c > 64 columns from its FP64
// Gram matrix, in place of the tall QR of Bw and the QRCP of R0 (the LQ, Q2,
// Jacobi and finish stages follow as on the QR route):
//   1. G = Bw^T Bw (c x c, both triangles; from B, scaled by 4^-e) in the W
//      area, on the matrix cores: a work-group per 32 x 32 tile of the upper
//      triangle, K (the rows of B) in LDS chunks of GT_KC.
//   2. panels of CHB pivots, a work-group per task: the pivot is the largest
//      remaining diagonal (lowest column on ties); row J of R over the original
//      columns is R(J, i) = (S(i, p) - sum of R(J', i) R(J', p) over the
//      panel's earlier rows J') / sqrt(d_p), kept transposed in the X area
//      (Rt[i + J c]), and the remaining diagonal d drops by R(J, i)^2 at once.
//      The factorization stops at the first J whose largest remaining diagonal
//      is at most c u trace(G) (the rest is rounding) or whose remaining
//      diagonals sum (the squared Frobenius norm of the trailing block of R1)
//      to at most (trunc_rel epsilon)^2 R1[0,0]^2, the QRCP's truncation.
//   3. after each panel, S -= Rp^T Rp over the panel's rows Rp (matrix cores);
//      rows and columns already pivoted change too but are not read again.
// State at hv + 3 c^2: d (c doubles), then CH_N doubles; the pivot order, kk
// and the dropped part go where the QR route's mode 5 leaves them.
constexpr int GT_T = 256;                    // threads per Gram tile work-group
constexpr int GT_KC = 64;                    // K chunk of a tile in LDS
constexpr int GT_LDK = GT_KC + 1;
constexpr int CHB = 16;                      // pivots per Cholesky panel
typedef double gt_f64x4 __attribute__((ext_vector_type(4)));

// t-th tile (ti, tj), ti <= tj, of the upper triangle, column of tiles by column
__device__ inline void upper_tile(int t, int& ti, int& tj) {
    int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    while (j * (j + 1) / 2 > t) --j;
    tj = j;
    ti = t - j * (j + 1) / 2;
}

// CHOL false: S = B^T B / 4^e (B / 2^e as the QR route's Bw); true: S -= Rp^T Rp
// for the panel of rows J0 .. CH_J
// of the task's transposed R.  Operand layout of v_mfma_f64_16x16x4f64 (lane l):
// A[l % 16][k + l / 16], B[k + l / 16][l % 16], D[l / 16 + 4 v][l % 16].
template <bool CHOL>
__global__ __launch_bounds__(GT_T) void k_gram_tile(const DCompress* __restrict__ tasks, int J0) {
    const DCompress T = tasks[blockIdx.y];
    const int M = T.M, c = T.c;
    if (M == 0 || c == 0) return;
    int ti, tj;
    upper_tile(blockIdx.x, ti, tj);
    if (tj * 32 >= c) return;
    double* S = T.hv + 2 * (size_t)c * c;
    const double* A;
    int64_t lda;
    int k0, k1;
    double gscale = 1.0;
    if (!CHOL) {
        // A(k, i) = B[k + i M]; G of B / 2^e, e from the largest |entry| (exact)
        A = T.B; lda = M; k0 = 0; k1 = M;
        const double amax = __longlong_as_double((long long)*asm_amax(T));
        const int bexp = amax > 0.0 ? ilogb(amax) + 1 : 0;
        gscale = ldexp(1.0, -2 * bexp);
    } else {
        const double* st = T.hv + 3 * (size_t)c * c + c;
        if (st[CH_DONE] != 0.0) return;               // stopped: S is not read again
        A = T.hv; lda = c; k0 = J0; k1 = (int)st[CH_J];   // A(k, i) = Rt[i + k c]
        if (k1 <= k0) return;
    }
    __shared__ double As[32 * GT_LDK], Bs[32 * GT_LDK];
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int iq = w & 1, jq = w >> 1;
    const int i0 = ti * 32, j0 = tj * 32;
    gt_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int kb = k0; kb < k1; kb += GT_KC) {
        const int kc = min(GT_KC, k1 - kb);
        const int kp = (kc + 3) & ~3;
        __syncthreads();                              // the previous chunk is consumed
        if (!CHOL) {                                  // lanes along K (contiguous)
            const int t = tid % WAVE;
            for (int a = tid / WAVE; a < 32; a += GT_T / WAVE) {
                const bool ok = t < kc;
                As[a * GT_LDK + t] = ok && i0 + a < c ? A[(kb + t) + (int64_t)(i0 + a) * lda] : 0.0;
                Bs[a * GT_LDK + t] = ok && j0 + a < c ? A[(kb + t) + (int64_t)(j0 + a) * lda] : 0.0;
            }
        } else {                                      // lanes along the columns (contiguous)
            const int a = tid % 32;
            for (int t = tid / 32; t < GT_KC; t += GT_T / 32) {
                const bool ok = t < kc;
                As[a * GT_LDK + t] = ok && i0 + a < c ? A[(i0 + a) + (int64_t)(kb + t) * lda] : 0.0;
                Bs[a * GT_LDK + t] = ok && j0 + a < c ? A[(j0 + a) + (int64_t)(kb + t) * lda] : 0.0;
            }
        }
        __syncthreads();
        const double* ap = As + (iq * 16 + lane % 16) * GT_LDK + lane / 16;
        const double* bp = Bs + (jq * 16 + lane % 16) * GT_LDK + lane / 16;
        for (int k = 0; k < kp; k += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[k], bp[k], acc, 0, 0, 0);
    }
    const int j = j0 + jq * 16 + lane % 16;
    if (j >= c) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + iq * 16 + lane / 16 + 4 * v;
        if (i >= c) continue;
        double* g = S + i + (int64_t)j * c;
        const double val = CHOL ? *g - acc[v] : acc[v] * gscale;
        *g = val;
        if (ti != tj) S[j + (int64_t)i * c] = val;
    }
}

// One panel of the pivoted Cholesky (step 2 above), a work-group per task.
__global__ __launch_bounds__(NTL) void k_chol_panel(const DCompress* __restrict__ tasks, int J0, double trunc_rel) {
    const DCompress T = tasks[blockIdx.x];
    const int M = T.M, c = T.c, tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    if (M == 0 || c == 0 || J0 >= c) return;
    double* Rt = T.hv;                                  // Rt[i + J c] = R(J, i)
    const double* S = T.hv + 2 * (size_t)c * c;
    double* d = T.hv + 3 * (size_t)c * c;
    double* st = d + c;
    double* hst = T.hv + 4 * (size_t)c * c;             // pivot order (c), then the header
    double* hdr = hst + c;
    extern __shared__ double sl[];
    double* s_d = sl;                                   // remaining diagonal, by original column
    int* s_perm = reinterpret_cast<int*>(s_d + c);      // position -> original column
    __shared__ double s_pv[NWL], s_pt[NWL];
    __shared__ int s_pi[NWL], s_pq[NWL];
    double stop, r00sq;
    if (J0 == 0) {
        double tr = 0.0;
        for (int i = tid; i < c; i += NTL) {
            const double g = S[i + (int64_t)i * c];
            s_d[i] = g;
            s_perm[i] = i;
            tr += g;
        }
        tr = blk_sum_l(tr, s_pv);                       // barriers inside
        stop = 1.1102230246251565e-16 * (double)c * tr;
        r00sq = 0.0;
        if (tid == 0) {                                 // the scale of B / 2^e
            const double amax = __longlong_as_double((long long)*asm_amax(T));
            hdr[LH_SCALE] = ldexp(1.0, amax > 0.0 ? ilogb(amax) + 1 : 0);
        }
    } else {
        if (st[CH_DONE] != 0.0) return;                 // uniform
        for (int i = tid; i < c; i += NTL) {
            s_d[i] = d[i];
            s_perm[i] = (int)hst[i];
        }
        stop = st[CH_STOP];
        r00sq = st[CH_R00SQ];
    }
    __syncthreads();
    const double trunc = trunc_rel * T.eps;
    bool done = false;
    double rest2 = 0.0;
    int J = J0;
    for (; J < J0 + CHB && J < c; ++J) {
        // largest remaining diagonal (lowest original column on ties), and the sum
        double bv = -1.0, tot = 0.0;
        int bi = INT_MAX, bq = 0;
        for (int q = J + tid; q < c; q += NTL) {
            const int i = s_perm[q];
            const double v = s_d[i];
            tot += v;
            if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; bq = q; }
        }
        tot = wave_sum(tot);
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o), oq = __shfl_xor(bq, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; bq = oq; }
        }
        if (lane == 0) { s_pv[wv] = bv; s_pi[wv] = bi; s_pq[wv] = bq; s_pt[wv] = tot; }
        __syncthreads();
        bv = -1.0; bi = INT_MAX; bq = 0; tot = 0.0;
        for (int k = 0; k < NWL; ++k) {                 // every thread, same order
            tot += s_pt[k];
            if (s_pv[k] > bv || (s_pv[k] == bv && s_pi[k] < bi)) { bv = s_pv[k]; bi = s_pi[k]; bq = s_pq[k]; }
        }
        if (J == 0) r00sq = bv;
        if (!(bv > stop) || tot <= trunc * trunc * r00sq) {   // uniform
            done = true;
            rest2 = tot;
            break;
        }
        __syncthreads();                                // the partials and s_perm are read
        if (tid == 0) { s_perm[bq] = s_perm[J]; s_perm[J] = bi; }
        __syncthreads();
        const int p = bi;
        const double rpp = sqrt(bv);
        for (int q = tid; q < c; q += NTL) {
            const int i = s_perm[q];
            double r;
            if (q < J) r = 0.0;
            else if (q == J) r = rpp;
            else {
                double v = S[i + (int64_t)p * c];
                for (int k = J0; k < J; ++k) v -= Rt[i + (int64_t)k * c] * Rt[p + (int64_t)k * c];
                r = v / rpp;
                s_d[i] -= r * r;
            }
            Rt[i + (int64_t)J * c] = r;
        }
        __syncthreads();                                // row J and d are complete
    }
    for (int i = tid; i < c; i += NTL) {
        d[i] = s_d[i];
        hst[i] = (double)s_perm[i];
    }
    if (tid == 0) {
        st[CH_J] = (double)J;
        if (J0 == 0) { st[CH_STOP] = stop; st[CH_R00SQ] = r00sq; }
        const bool fin = done || J >= c;
        st[CH_DONE] = fin ? 1.0 : 0.0;
        if (fin) {
            hdr[LH_KK] = (double)J;
            hdr[LH_REST2] = done ? rest2 : 0.0;
        }
    }
}

// LDS of k_compress_large in bytes, or 0 when the task does not fit
inline size_t compress_large_lds(int M, int c) {
    const size_t vlen = (size_t)(M > c ? M : c) + 1;
    return (vlen + 4 * (size_t)c) * sizeof(double) + 2 * (size_t)c * sizeof(int);
}

// ------------------------------------------------------------------ elimination
constexpr int NTP = 1024;                    // threads of the pivot-preparation kernel
constexpr int NWP = NTP / WAVE;

// In-place inverse of the m x m column-major block by Gauss-Jordan elimination
// with partial (row) pivoting inside the block (large blocks, global memory);
// returns false if a pivot is 0.  scol: m doubles, sperm: m ints of LDS.
__device__ bool gj_inverse_global(double* A, int m, double* scol, int* sperm, double* s_d) {
    const int tid = threadIdx.x;
    for (int k = 0; k < m; ++k) {
        if (tid < WAVE) {
            double best = -1.0;
            int bi = INT_MAX;
            for (int i = k + tid; i < m; i += WAVE) {
                const double v = fabs(A[i + (int64_t)k * m]);
                if (v > best) { best = v; bi = i; }
            }
            for (int o = WAVE / 2; o > 0; o >>= 1) {
                double ob = __shfl_down(best, o);
                int oi = __shfl_down(bi, o);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (tid == 0) { sperm[k] = bi; s_d[0] = best; }
        }
        __syncthreads();
        const int p = sperm[k];
        if (!(s_d[0] > 0.0)) return false;
        if (p != k)
            for (int j = tid; j < m; j += NTP) {
                double t = A[k + (int64_t)j * m];
                A[k + (int64_t)j * m] = A[p + (int64_t)j * m];
                A[p + (int64_t)j * m] = t;
            }
        __syncthreads();
        const double d = 1.0 / A[k + (int64_t)k * m];
        for (int i = tid; i < m; i += NTP) scol[i] = A[i + (int64_t)k * m];
        __syncthreads();
        for (int j = tid; j < m; j += NTP)
            A[k + (int64_t)j * m] = (j == k) ? d : A[k + (int64_t)j * m] * d;
        __syncthreads();
        for (int e = tid; e < m * m; e += NTP) {
            const int i = e % m, j = e / m;
            if (i == k) continue;
            const double f = scol[i];
            if (j == k) A[i + (int64_t)k * m] = -f * d;
            else A[i + (int64_t)j * m] -= f * A[k + (int64_t)j * m];
        }
        __syncthreads();
    }
    for (int i = tid; i < m; i += NTP)
        for (int k = m - 1; k >= 0; --k) {
            const int p = sperm[k];
            if (p != k) {
                double t = A[i + (int64_t)k * m];
                A[i + (int64_t)k * m] = A[i + (int64_t)p * m];
                A[i + (int64_t)p * m] = t;
            }
        }
    __syncthreads();
    return true;
}

// Blocked Gauss-Jordan inverse with partial pivoting (128 < m <= 1024): panels
// of GJB columns are reduced in LDS (pivot search over the panel column, row
// swap inside the panel, the Gauss-Jordan step on the panel columns only);
// then the panel's row swaps are applied to the other columns and they receive
// the panel's combined transformation as one rank-GJB update.  Correctness:
// each step is the elementary matrix E_k (identity but for column k) after the
// swap P_k; a swap by a later step of the panel only permutes rows of the
// earlier E columns, so the panel's product is M = I + (M[:, J] - I[:, J]) with
// M[:, J] the panel columns as stored, and every other column c becomes
// M (swapped c).  Each element of A is read and written once per panel instead
// of once per column.  LDS of a panel: gj_blocked_lds(m) bytes.
constexpr int GJB = 16;                      // panel width
constexpr int GJB_CW = 64;                   // columns of the trailing update staged at once
constexpr int GJB_MAX = 1024;                // rows: one per thread in the update

// Panel j0 of the blocked inverse (every thread of the work-group): pivot steps
// on the m x nb panel in LDS Pn, the panel written back, its row swaps applied to
// the other columns; the pivot rows go to perm[j0 .. j0 + nb).  False: a zero
// pivot column (singular).
__device__ bool gj_panel(double* A, int m, int j0, double* sm, int* perm) {
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    const int nb = min(GJB, m - j0);
    double* Pn = sm;                                         // m x GJB panel, ld m
    double* s_bv = Pn + (size_t)GJB * m + GJB * GJB_CW;      // NWP
    int* s_bi = reinterpret_cast<int*>(s_bv + NWP);          // NWP
    int* s_pp = s_bi + NWP;                                  // GJB pivot rows of this panel
    for (int e = tid; e < m * nb; e += NTP) {
        const int i = e % m, t = e / m;
        Pn[i + t * m] = A[i + (int64_t)(j0 + t) * m];
    }
    __syncthreads();
    for (int kk = 0; kk < nb; ++kk) {
        const int k = j0 + kk;
        double best = -1.0;
        int bi = INT_MAX;
        for (int i = k + tid; i < m; i += NTP) {
            const double v = fabs(Pn[i + kk * m]);
            if (v > best) { best = v; bi = i; }
        }
        wave_argmax(best, bi);
        if (lane == 0) { s_bv[wv] = best; s_bi[wv] = bi; }
        __syncthreads();
        best = s_bv[0];
        bi = s_bi[0];
        for (int w = 1; w < NWP; ++w)
            if (s_bv[w] > best || (s_bv[w] == best && s_bi[w] < bi)) { best = s_bv[w]; bi = s_bi[w]; }
        if (!(best > 0.0)) return false;                     // uniform
        const int p = bi;
        if (p != k && tid < nb) {
            const double a = Pn[k + tid * m];
            Pn[k + tid * m] = Pn[p + tid * m];
            Pn[p + tid * m] = a;
        }
        if (tid == 0) s_pp[kk] = p;
        __syncthreads();
        // the step on the panel columns: row k scaled by d = 1 / pivot, the
        // other rows minus their column-k entry times the new row k
        const double d = 1.0 / Pn[k + kk * m];
        double rowk[GJB];
#pragma unroll
        for (int t = 0; t < GJB; ++t) rowk[t] = t < nb ? (t == kk ? d : Pn[k + t * m] * d) : 0.0;
        __syncthreads();                                     // row k read by every thread
        for (int i = tid; i < m; i += NTP) {
            if (i == k) {
                for (int t = 0; t < nb; ++t) Pn[k + t * m] = rowk[t];
            } else {
                const double f = Pn[i + kk * m];
                for (int t = 0; t < nb; ++t)
                    Pn[i + t * m] = (t == kk) ? -f * d : Pn[i + t * m] - f * rowk[t];
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < m * nb; e += NTP) {
        const int i = e % m, t = e / m;
        A[i + (int64_t)(j0 + t) * m] = Pn[i + t * m];
    }
    if (tid < nb) perm[j0 + tid] = s_pp[tid];
    // the panel's swaps on the other columns, in order (one thread per column)
    for (int c = tid; c < m; c += NTP) {
        if (c >= j0 && c < j0 + nb) continue;
        double* col = A + (int64_t)c * m;
        for (int kk = 0; kk < nb; ++kk) {
            const int k = j0 + kk, p = s_pp[kk];
            if (p != k) {
                const double a = col[k];
                col[k] = col[p];
                col[p] = a;
            }
        }
    }
    __syncthreads();
    return true;
}

// The panel's transformation on columns c0 .. c0 + GJB_CW - 1 outside the panel
// J: A[:, c] = A[:, c] + (M[:, J] - I[:, J]) A[J, c], M[:, J] the panel columns
// as stored; thread i updates row i.  Each column is read (rows J first, into
// Tc) before any of its rows is written, so chunks may run in separate
// work-groups.
__device__ void gj_update_chunk(double* A, int m, int j0, int c0, double* Tc) {
    const int tid = threadIdx.x;
    const int nb = min(GJB, m - j0);
    for (int e = tid; e < GJB * GJB_CW; e += NTP) {
        const int t = e % GJB, cc = e / GJB, c = c0 + cc;
        Tc[t + cc * GJB] = (t < nb && c < m && (c < j0 || c >= j0 + nb)) ? A[(j0 + t) + (int64_t)c * m] : 0.0;
    }
    __syncthreads();
    const int i = tid;
    if (i < m) {
        double mh[GJB];
#pragma unroll
        for (int t = 0; t < GJB; ++t)
            mh[t] = t < nb ? A[i + (int64_t)(j0 + t) * m] - (i == j0 + t ? 1.0 : 0.0) : 0.0;
        const int cend = min(GJB_CW, m - c0);
        for (int cc = 0; cc < cend; ++cc) {
            const int c = c0 + cc;
            if (c >= j0 && c < j0 + nb) continue;
            double acc = A[i + (int64_t)c * m];
#pragma unroll
            for (int t = 0; t < GJB; ++t) acc += mh[t] * Tc[t + cc * GJB];
            A[i + (int64_t)c * m] = acc;
        }
    }
    __syncthreads();
}

// The stored matrix is the inverse of A with rows permuted: undo by columns
// (rows i0 + tid).
__device__ void gj_unperm(double* A, int m, const int* perm, int i0) {
    for (int i = i0 + threadIdx.x; i < m; i += NTP)
        for (int k = m - 1; k >= 0; --k) {
            const int p = perm[k];
            if (p != k) {
                const double t = A[i + (int64_t)k * m];
                A[i + (int64_t)k * m] = A[i + (int64_t)p * m];
                A[i + (int64_t)p * m] = t;
            }
        }
}

__host__ __device__ inline size_t gj_blocked_lds(int m) {
    return ((size_t)GJB * m + GJB * GJB_CW + NWP) * sizeof(double) + (size_t)(NWP + GJB + m) * sizeof(int);
}

// Register-resident Gauss-Jordan inverse with partial pivoting for m <= MB.
// Thread t owns row i = t % MB and the CPT columns [h CPT, (h+1) CPT), h = t / MB;
// the matrix is padded with the identity beyond m.  Pivoting is implicit: step
// k takes the unused physical row p_k with the largest |A[p_k, k]| (lowest
// index on ties) as pivot row, without moving rows, so the storage ends as
// (P A)^{-1} by physical rows, and A^{-1}[k, p_l] = stored[p_k, l] on output.
// The pivot search of step k+1 runs inside the update of step k, so a step
// costs two barriers; every register index is a compile-time constant.
// `lds` needs 2 MB doubles + MB ints + 4 NWP (double, int) slots.
template <int MB>
__device__ bool gj_inverse_reg(double* __restrict__ A, int m, double* lds) {
    constexpr int TPR = NTP / MB;         // threads per row
    constexpr int CPT = MB / TPR;         // columns per thread
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    const int i = tid % MB, h = tid / MB, c0 = h * CPT;
    double* prow = lds;                   // MB: pivot row
    double* pcol = lds + MB;              // MB: pivot column (multipliers)
    int* pivrow = (int*)(lds + 2 * MB);   // MB: physical pivot row of each step
    double* rv = (double*)(pivrow + MB);  // 2 x NWP partial maxima (double-buffered)
    int* ri = (int*)(rv + 2 * NWP);       // 2 x NWP their rows
    double a[CPT];
#pragma unroll
    for (int jj = 0; jj < CPT; ++jj) {
        const int col = c0 + jj;
        a[jj] = (i < m && col < m) ? A[i + (int64_t)col * m] : (i == col ? 1.0 : 0.0);
    }
    bool used = i >= m;                   // padding rows never pivot
    int mystep = -1;
    // value of this thread's row in the next pivot column (owners only)
    double ck = (h == 0 && !used) ? a[0] : 0.0;
    // column k is held by the wavefronts [kh MB / WAVE, kh MB / WAVE + WPG)
    constexpr int WPG = MB >= WAVE ? MB / WAVE : 1;
    auto publish_max = [&](double cand, int buf) {
        double best = cand;
        int bi = cand >= 0.0 ? i : INT_MAX;
        wave_argmax(best, bi);
        if (lane == 0) { rv[buf * NWP + wv] = best; ri[buf * NWP + wv] = bi; }
    };
    // only the wavefronts that hold the next pivot column publish (for MB >= 64
    // a wavefront holds one column range; smaller MB mix ranges in a wavefront)
    if (MB < WAVE || h == 0) publish_max((h == 0 && !used) ? fabs(ck) : -1.0, 0);
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        const int buf = k & 1;
        const int kh = k / CPT;
        const int w0 = (kh * MB) / WAVE;
        double best = rv[buf * NWP + w0];
        int p = ri[buf * NWP + w0];
#pragma unroll
        for (int w = 1; w < WPG; ++w) {
            const double v = rv[buf * NWP + w0 + w];
            const int q = ri[buf * NWP + w0 + w];
            if (v > best || (v == best && q < p)) { best = v; p = q; }
        }
        if (!(best > 0.0)) return false;          // uniform: exactly singular
        if (i == p) {
#pragma unroll
            for (int jj = 0; jj < CPT; ++jj) prow[c0 + jj] = a[jj];
            used = true;
            mystep = k;
        }
        if (h == kh) pcol[i] = ck;
        if (tid == 0) pivrow[k] = p;
        __syncthreads();
        const double d = 1.0 / prow[k];
        const int kn = k + 1, knh = kn / CPT;
        double cnext = 0.0;
        if (i == p) {
#pragma unroll
            for (int jj = 0; jj < CPT; ++jj) {
                const int col = c0 + jj;
                a[jj] = (col == k) ? d : a[jj] * d;
                cnext = (col == kn) ? a[jj] : cnext;
            }
        } else {
            const double f = pcol[i] * d;
            if (h == kh || h == knh) {            // holds column k or k + 1
#pragma unroll
                for (int jj = 0; jj < CPT; ++jj) {
                    const int col = c0 + jj;
                    const double v = a[jj] - f * prow[col];
                    a[jj] = (col == k) ? -f : v;
                    cnext = (col == kn) ? a[jj] : cnext;
                }
            } else {
#pragma unroll
                for (int jj = 0; jj < CPT; ++jj) a[jj] -= f * prow[c0 + jj];
            }
        }
        ck = cnext;
        if (kn < m && (MB < WAVE || h == knh)) publish_max((h == knh && !used) ? fabs(ck) : -1.0, buf ^ 1);
        __syncthreads();
    }
    // A^{-1}[k, p_l] = stored[p_k, l]: this thread holds stored[i, c0..] with i = p_mystep
    if (mystep >= 0) {
#pragma unroll
        for (int jj = 0; jj < CPT; ++jj) {
            const int col = c0 + jj;
            if (col < m) A[mystep + (int64_t)pivrow[col] * m] = a[jj];
        }
    }
    __syncthreads();
    return true;
}

// Per super-node preparation (Sec. 4.3, Sec. 4.4): [R; Q] = B V into the
// blocks Mat(P -> p_k) and Mat(p_k -> P), the rewiring blocks V, V^T, -I, and
// the inverse of the pivot block.  With do_proj == 0 only the pivot is
// inverted (black nodes, after the Schur updates of their super-node).
__global__ __launch_bounds__(NTP) void k_node_prep(const DPrep* __restrict__ tasks,
                                                   const DProj* __restrict__ projs,
                                                   const int32_t* __restrict__ imap,
                                                   int32_t* __restrict__ info) {
    const DPrep T = tasks[blockIdx.x];
    const int tid = threadIdx.x;
    extern __shared__ double sm[];
    const int r = T.r, c = T.c;
    if (T.do_proj && r > 0) {
        // all pieces as one element range, so every thread has work
        int total = 0;
        for (int q = 0; q < T.nproj; ++q) total += projs[T.proj0 + q].nrows * r;
        int q = 0, qstart = 0;
        for (int e = tid; e < total; e += NTP) {
            while (e >= qstart + projs[T.proj0 + q].nrows * r) {
                qstart += projs[T.proj0 + q].nrows * r;
                ++q;
            }
            const DProj Pj = projs[T.proj0 + q];
            const int nrow = Pj.nrows, le = e - qstart;
            int a, t;
            if (!Pj.trans) { a = le % nrow; t = le / nrow; }
            else           { t = le % r;    a = le / r; }
            double v;
            if (T.svd) {                      // (B V)[row0 + a, t]
                const double* brow = T.B + (Pj.row0 + a);
                const double* vcol = T.V + (int64_t)t * c;
                double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
                int j = 0;
                for (; j + 4 <= c; j += 4) {
                    v0 += brow[(int64_t)j * T.M] * vcol[j];
                    v1 += brow[(int64_t)(j + 1) * T.M] * vcol[j + 1];
                    v2 += brow[(int64_t)(j + 2) * T.M] * vcol[j + 2];
                    v3 += brow[(int64_t)(j + 3) * T.M] * vcol[j + 3];
                }
                for (; j < c; ++j) v0 += brow[(int64_t)j * T.M] * vcol[j];
                v = (v0 + v1) + (v2 + v3);
            } else {                          // transformed row-pivoted block
                v = T.B[(int64_t)(Pj.row0 + a) * c + t];
            }
            if (!Pj.trans) Pj.dst.p[imap_at(imap, Pj.map, a) + (int64_t)t * Pj.dst.nr] = v;   // R_k
            else           Pj.dst.p[t + (int64_t)imap_at(imap, Pj.map, a) * r] = v;           // Q_k^T
        }
        for (int e = tid; e < c * r; e += NTP) {
            T.bs.p[e] = T.V[e];                          // V      (c x r)
            const int t = e % r, a = e / r;
            T.sb.p[e] = T.V[a + (int64_t)t * c];         // V^T    (r x c)
        }
        for (int e = tid; e < r * r; e += NTP) {
            const double v = (e % r == e / r) ? -1.0 : 0.0;
            T.bP.p[e] = v;
            T.Pb.p[e] = v;
        }
    }
    const int m = T.piv.nr;
    if (m == 0) return;
    __syncthreads();
    bool ok;
    if (m <= 32) ok = gj_inverse_reg<32>(T.piv.p, m, sm);
    else if (m <= 64) ok = gj_inverse_reg<64>(T.piv.p, m, sm);
    else if (m <= 128) ok = gj_inverse_reg<128>(T.piv.p, m, sm);
    else if (m <= GJB_MAX && gj_blocked_lds(m) <= (size_t)kLdsBudget)
        ok = true;                                   // inverted by the k_gj_* launches that follow
    else ok = gj_inverse_global(T.piv.p, m, sm, (int*)(sm + m), sm + 2 * m);
    if (!ok && tid == 0) info[T.info_slot] = 1;
}

// The blocked inverse of the pivots with 128 < m <= GJB_MAX over many
// work-groups (k_node_prep leaves them; inlining a one-work-group form there
// made the whole kernel spill): per panel, one work-group
// per task runs gj_panel, then one work-group per GJB_CW-column chunk and task
// applies the panel's transformation; finally the row order is undone.  perm:
// GJB_MAX ints per task.  A task whose pivot turns out singular gets its info
// slot set and is skipped from then on.
__device__ inline bool gj_deferred(const DPrep& T) {
    const int m = T.piv.nr;
    return m > 128 && m <= GJB_MAX && gj_blocked_lds(m) <= (size_t)kLdsBudget;
}

__global__ __launch_bounds__(NTP) void k_gj_panel(const DPrep* __restrict__ tasks, int j0, int* __restrict__ perm,
                                                  int32_t* __restrict__ info) {
    const DPrep T = tasks[blockIdx.x];
    const int m = T.piv.nr;
    if (!gj_deferred(T) || j0 >= m || info[T.info_slot]) return;   // uniform
    extern __shared__ double sm[];
    const bool ok = gj_panel(T.piv.p, m, j0, sm, perm + (size_t)blockIdx.x * GJB_MAX);
    if (!ok && threadIdx.x == 0) info[T.info_slot] = 1;
}

__global__ __launch_bounds__(NTP) void k_gj_update(const DPrep* __restrict__ tasks, int j0,
                                                   const int32_t* __restrict__ info) {
    const DPrep T = tasks[blockIdx.y];
    const int m = T.piv.nr;
    const int c0 = blockIdx.x * GJB_CW;
    if (!gj_deferred(T) || j0 >= m || c0 >= m || info[T.info_slot]) return;
    __shared__ double Tc[GJB * GJB_CW];
    gj_update_chunk(T.piv.p, m, j0, c0, Tc);
}

__global__ __launch_bounds__(NTP) void k_gj_unperm(const DPrep* __restrict__ tasks, const int* __restrict__ perm,
                                                   const int32_t* __restrict__ info) {
    const DPrep T = tasks[blockIdx.x];
    if (!gj_deferred(T) || info[T.info_slot]) return;
    gj_unperm(T.piv.p, T.piv.nr, perm + (size_t)blockIdx.x * GJB_MAX, 0);
}

// Tiled product with gathers and scatters (DGemm): one work-group per 32 x 32
// tile of C; the A panel (32 x K), the B panel (K x 32) and, for sub, the C tile
// are copied to LDS in one pass (every load in flight), then each thread
// accumulates a 2 x 2 block.  K is taken in chunks of gk <= GK.
constexpr int GT = 256;                      // threads per tile
constexpr int GK = 256;                      // K chunk held in LDS
constexpr int GLA = 33;                      // LDS leading dimension of A and C tiles

__global__ __launch_bounds__(GT) void k_gemm_tiles(const DGemm* __restrict__ gs,
                                                   const DTile* __restrict__ tiles,
                                                   const int32_t* __restrict__ imap, int gk) {
    extern __shared__ double sm[];
    const DTile tl = tiles[blockIdx.x];
    const DGemm G = gs[tl.g];
    const int tid = threadIdx.x;
    const int mt = min(32, G.M - tl.i0), nt = min(32, G.N - tl.j0);
    double* As = sm;                         // 32 x gk, ld GLA
    double* Cs = As + GLA * gk;              // 32 x 32, ld GLA
    double* Bs = Cs + GLA * 32;              // gk x 32, ld kb1 (odd)
    const int tx = tid % 16, ty = tid / 16;
    double acc00 = 0.0, acc01 = 0.0, acc10 = 0.0, acc11 = 0.0;
    for (int k0 = 0; k0 < G.K; k0 += gk) {
        const int kc = min(gk, G.K - k0);
        const int kb1 = kc | 1;
        // A panel: lane a = tid % 32 over rows, 8 column slots
        {
            const int a = tid % 32;
            if (a < mt)
                for (int t = tid / 32; t < kc; t += GT / 32) {
                    const int col = imap_at(imap, G.amap, k0 + t);
                    As[a + t * GLA] = G.A[(int64_t)(tl.i0 + a) + (int64_t)col * G.lda];
                }
        }
        // B panel: lane over K, 4 column slots
        {
            const int tt = tid % 64;
            for (int b = tid / 64; b < nt; b += GT / 64)
                for (int t = tt; t < kc; t += 64) {
                    const int row = imap_at(imap, G.bmap, k0 + t);
                    Bs[t + b * kb1] = G.B[(int64_t)row + (int64_t)(tl.j0 + b) * G.ldb];
                }
        }
        if (k0 == 0 && G.sub) {
            const int a = tid % 32;
            if (a < mt) {
                const int row = imap_at(imap, G.crmap, tl.i0 + a);
                for (int b = tid / 32; b < nt; b += GT / 32) {
                    const int col = imap_at(imap, G.ccmap, tl.j0 + b);
                    Cs[a + b * GLA] = G.C[G.tr ? (int64_t)col + (int64_t)row * G.ldc : (int64_t)row + (int64_t)col * G.ldc];
                }
            }
        }
        __syncthreads();
        const bool r0 = ty < mt, r1 = ty + 16 < mt, c0 = tx < nt, c1 = tx + 16 < nt;
        if ((r0 || r1) && (c0 || c1)) {
            const double* ap = As + ty;
            const double* bp0 = Bs + tx * kb1;
            const double* bp1 = Bs + (tx + 16) * kb1;
#pragma unroll 4
            for (int t = 0; t < kc; ++t) {
                const double x0 = ap[t * GLA], x1 = ap[t * GLA + 16];
                const double y0 = bp0[t], y1 = bp1[t];
                acc00 = fma(x0, y0, acc00);
                acc01 = fma(x0, y1, acc01);
                acc10 = fma(x1, y0, acc10);
                acc11 = fma(x1, y1, acc11);
            }
        }
        __syncthreads();
    }
    auto put = [&](int a, int b, double v) {
        if (a >= mt || b >= nt) return;
        const int row = imap_at(imap, G.crmap, tl.i0 + a);
        const int col = imap_at(imap, G.ccmap, tl.j0 + b);
        G.C[G.tr ? (int64_t)col + (int64_t)row * G.ldc : (int64_t)row + (int64_t)col * G.ldc] =
            G.sub ? Cs[a + b * GLA] - v : v;
    };
    put(ty, tx, acc00);
    put(ty, tx + 16, acc01);
    put(ty + 16, tx, acc10);
    put(ty + 16, tx + 16, acc11);
}

// ------------------------------------------------------------------ solve sweeps
// Interpreter of the staged node programs (formats in dev.hpp).  NK right-hand
// sides per launch; vector buffers in LDS keep a row stride of kSwKS.
// Copies the runs of one stage into LDS: every thread first issues the loads
// of U elements, then stores them, so a stage costs about one memory latency.
// A thread's elements are kSwThreads apart, so the position inside the current
// run advances by a fixed quotient and remainder; the fields of the current
// run stay in registers.
// Vector rows in LDS (kSwKS doubles each, right-hand side k of the row that
// starts at LDS double ra) keep element k at ra + (k ^ ((ra >> 5) & 3)): 8
// consecutive rows fill the 64 banks once, and the next 8 are shifted by the
// key, so lanes that read one element of 16 consecutive rows do not conflict.
static_assert(kSwKS == 4, "vector row swizzle assumes rows of 4 doubles");
__device__ __forceinline__ int sw_key(int ra) { return (ra >> 5) & 3; }
__device__ __forceinline__ int sw_slot(int ra, int k) { return ra + (k ^ sw_key(ra)); }

template <int NK>
__device__ __forceinline__ void sw_copy(const SwRun* runs, int nrun, const int32_t* D, int elems,
                                        const double* x, int ldx, double* dat) {
    constexpr int U = 16;
    if (nrun == 0 || threadIdx.x >= elems) return;
    int ri = 0, rstart = 0;
    // current run
    const void* src = nullptr;
    bool f32 = false;
    int len = 0, ld = 0, dld = 0, lds = 0, map = -1, cnt = 0, q = 0, r = 0;
    int t = 0, a = 0;                         // position of element g inside the run
    auto load_run = [&](int g) {
        const SwRun& R = runs[ri];
        src = R.src;
        f32 = R.es == 4;
        map = R.map;
        lds = R.lds;
        if (src) { len = R.len; ld = R.ld; dld = R.dld; }
        else { len = NK; ld = R.ld; dld = kSwKS; }
        cnt = len * R.nrun;
        q = kSwThreads / len;
        r = kSwThreads - q * len;
        const int li = g - rstart;
        t = li / len;
        a = li - t * len;
    };
    int g = threadIdx.x;
    while (g >= rstart + runs[ri].nrun * (runs[ri].src ? runs[ri].len : NK)) {
        rstart += runs[ri].nrun * (runs[ri].src ? runs[ri].len : NK);
        ++ri;
    }
    load_run(g);
    for (; g < elems;) {
        double v[U];
        int dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dst[u] = -1;
            v[u] = 0.0;
            if (g < elems) {
                if (g >= rstart + cnt) {
                    rstart += cnt;
                    ++ri;
                    while (g >= rstart + runs[ri].nrun * (runs[ri].src ? runs[ri].len : NK)) {
                        rstart += runs[ri].nrun * (runs[ri].src ? runs[ri].len : NK);
                        ++ri;
                    }
                    load_run(g);
                }
                if (src) {
                    const int64_t o = (int64_t)t * ld + a;
                    v[u] = f32 ? (double)static_cast<const float*>(src)[o] : static_cast<const double*>(src)[o];
                } else {
                    const int row = map < 0 ? ld + t : D[map + t];
                    v[u] = x[(int64_t)row * ldx + a];
                }
                dst[u] = src ? lds + t * dld + a : sw_slot(lds + t * kSwKS, a);
                g += kSwThreads;
                a += r;
                t += q;
                if (a >= len) { a -= len; ++t; }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (dst[u] >= 0) dat[dst[u]] = v[u];
    }
}

// One group: rows of its comps in parallel, 2^lglanes lanes per row (adjacent
// lanes of one wavefront, combined by shuffles).
template <int NK>
__device__ __forceinline__ void sw_group(const SwGroup& G, const SwComp* C, const int32_t* D,
                                         double* dat, double* x, int ldx) {
    const int lg = G.lglanes, L = 1 << lg;
    const int total = G.rows << lg;
    int ci = G.comp0, cstart = 0;
    for (int j = threadIdx.x; j < total; j += kSwThreads) {
        const int item = j >> lg, sub = j & (L - 1);
        while (item >= cstart + C[ci].nr) {
            cstart += C[ci].nr;
            ++ci;
        }
        const SwComp& c = C[ci];
        const int a = item - cstart;
        double acc[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) acc[k] = 0.0;
        const double* mp = dat + c.mat + a;
#pragma unroll 2
        for (int t = sub; t < c.nc; t += L) {
            const double mv = mp[t * c.ld];
            const int row = c.in_map < 0 ? t : D[c.in_map + t];
            const int ra = c.in + row * kSwKS, key = sw_key(ra);
            const double* iv = dat + ra;
#pragma unroll
            for (int k = 0; k < NK; ++k) acc[k] = fma(mv, iv[k ^ key], acc[k]);
        }
        // sum over the L adjacent lanes of the row (inside one 16-lane DPP row):
        // quad swaps, then the half-row and row mirrors; every lane gets the sum
        if (lg >= 1) {
#pragma unroll
            for (int k = 0; k < NK; ++k) acc[k] += dpp_mov<0xB1>(acc[k]);
        }
        if (lg >= 2) {
#pragma unroll
            for (int k = 0; k < NK; ++k) acc[k] += dpp_mov<0x4E>(acc[k]);
        }
        if (lg >= 3) {
#pragma unroll
            for (int k = 0; k < NK; ++k) acc[k] += dpp_mov<0x141>(acc[k]);
        }
        if (lg >= 4) {
#pragma unroll
            for (int k = 0; k < NK; ++k) acc[k] += dpp_mov<0x140>(acc[k]);
        }
        if (sub == 0) {
            double y[NK];
            if (c.init >= 0) {
                const int ra = c.init + (c.init_map < 0 ? a : D[c.init_map + a]) * kSwKS, key = sw_key(ra);
                const double* ip = dat + ra;
#pragma unroll
                for (int k = 0; k < NK; ++k) y[k] = ip[k ^ key] - acc[k];
            } else {
#pragma unroll
                for (int k = 0; k < NK; ++k) y[k] = acc[k];
            }
            if (c.out >= 0) {
                const int ra = c.out + (c.out_map < 0 ? a : D[c.out_map + a]) * kSwKS, key = sw_key(ra);
                double* op = dat + ra;
#pragma unroll
                for (int k = 0; k < NK; ++k) op[k ^ key] = y[k];
            }
            if (c.gmap >= 0 || c.gbase >= 0) {
                const int row = c.gmap >= 0 ? D[c.gmap + a] : c.gbase + a;
                double* xp = x + (int64_t)row * ldx;
#pragma unroll
                for (int k = 0; k < NK; ++k) xp[k] = y[k];
            }
        }
    }
}

// One work-group per super-node of a colour step and slice of NK right-hand
// sides; x is the extended vector (row-interleaved, ldx right-hand sides), this
// launch treats [k0, k0 + gridDim.y NK).
// Each run states the storage type of its block (FP64, or FP32 for off-diagonal
// blocks in mixed precision); LDS, vectors and accumulation stay FP64.
template <int NK>
__global__ __launch_bounds__(kSwThreads) void k_sweep(const SwNode* __restrict__ nodes,
                                                      double* __restrict__ x, int ldx, int k0) {
    extern __shared__ double smem[];
    int32_t* Dbuf = reinterpret_cast<int32_t*>(smem);
    double* dat = smem + kSwDescWords;           // after two descriptor buffers
    const int tid = threadIdx.x;
    const SwNode nd = nodes[blockIdx.x];
    if (nd.nstage == 0 || (nd.live && *nd.live == 0)) return;
    const int32_t* src = nd.desc;
    for (int w = tid; w < nd.words0; w += kSwThreads) Dbuf[w] = src[w];
    src += nd.words0;
    if (nd.x) x = nd.x;
    x += k0 + (int)blockIdx.y * NK;             // slice y of the launch: right-hand sides k0 + y NK ..
    __syncthreads();
    for (int s = 0; s < nd.nstage; ++s) {
        const int32_t* D = Dbuf + (s & 1) * kSwDescWords;
        int32_t* Dn = Dbuf + ((s + 1) & 1) * kSwDescWords;
        const SwHeader H = *reinterpret_cast<const SwHeader*>(D);
        constexpr int PW = kSwDescWords / kSwThreads;
        int32_t nw[PW];
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            const int w = tid + i * kSwThreads;
            nw[i] = w < H.words_next ? src[w] : 0;
        }
        sw_copy<NK>(reinterpret_cast<const SwRun*>(D + H.runs), H.nrun, D, H.elems_mat + H.xrows * NK,
                    x, ldx, dat);
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            const int w = tid + i * kSwThreads;
            if (w < H.words_next) Dn[w] = nw[i];
        }
        src += H.words_next;
        __syncthreads();
        const SwGroup* G = reinterpret_cast<const SwGroup*>(D + H.groups);
        const SwComp* C = reinterpret_cast<const SwComp*>(D + H.comps);
        for (int g = 0; g < H.ngroup; ++g) {
            sw_group<NK>(G[g], C, D, dat, x, ldx);
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ vectors
__global__ void k_gather_perm(const double* __restrict__ b, int64_t ldb, const int32_t* __restrict__ perm,
                              int n, int nrhs, double* __restrict__ xt, int64_t ntot) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntot * nrhs) return;
    const int64_t t = e / nrhs;
    const int k = (int)(e % nrhs);
    xt[e] = t < n ? b[perm[t] + (int64_t)k * ldb] : 0.0;
}

__global__ void k_scatter_perm(const double* __restrict__ xt, const int32_t* __restrict__ perm, int n,
                               int nrhs, double* __restrict__ x, int64_t ldx) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * nrhs) return;
    const int64_t t = e / nrhs;
    const int k = (int)(e % nrhs);
    x[perm[t] + (int64_t)k * ldx] = xt[e];
}

// ------------------------------------------------------------------ batched FGMRES vectors
// One work-group per chunk (DKryChunk) of rc rows of one system; chunks of
// systems whose act flag is 0 return at once.  Per system the arithmetic is
// fixed by its own chunks, so a system's iteration does not depend on the
// others in the batch.
struct KryRows {
    int64_t r0, r1;
};
__device__ inline KryRows kry_rows_of(const DKryChunk& C, int n, int rc) {
    KryRows r;
    r.r0 = C.row0;
    r.r1 = min((int64_t)n, (int64_t)C.row0 + rc);
    return r;
}

// mode 0: b = bin[perm] (tree order), x = 0; mode 1: xout[perm] = x
__global__ __launch_bounds__(256) void k_kry_perm(const DKry* __restrict__ sys, const DKryChunk* __restrict__ ch,
                                                  const int32_t* __restrict__ act, int nrhs, int rc, int mode,
                                                  int off) {
    const DKryChunk C = ch[blockIdx.x];
    if (!act[C.sys]) return;
    const DKry& S = sys[C.sys];
    const KryRows R = kry_rows_of(C, S.n, rc);
    const int64_t cnt = (R.r1 - R.r0) * nrhs;
    for (int64_t e = threadIdx.x; e < cnt; e += 256) {
        const int64_t i = R.r0 + e / nrhs;
        const int k = (int)(e % nrhs);
        const int64_t o = (int64_t)S.perm[i] + (int64_t)k * S.n;
        if (mode == 0) {
            S.b[i * nrhs + k] = S.bin[o];
            S.x[i * nrhs + k] = 0.0;
        } else if (mode == 2) {                         // initial guess, 0 where ||b|| = 0
            S.x[i * nrhs + k] = S.sm[off + k] > 0.0 ? S.xout[o] : 0.0;
        } else {
            S.xout[o] = S.x[i * nrhs + k];
        }
    }
}

// RES: r = b - A x;  otherwise w = A Z_j
template <bool RES>
__global__ __launch_bounds__(256) void k_kry_spmv(const DKry* __restrict__ sys, const DKryChunk* __restrict__ ch,
                                                  const int32_t* __restrict__ act, int nrhs, int rc, int j) {
    const DKryChunk C = ch[blockIdx.x];
    if (!act[C.sys]) return;
    const DKry& S = sys[C.sys];
    const KryRows R = kry_rows_of(C, S.n, rc);
    const double* __restrict__ x = RES ? S.x : S.Z + (int64_t)j * S.nv;
    double* __restrict__ y = RES ? S.r : S.w;
    const int64_t* __restrict__ rp = S.rp;
    const int32_t* __restrict__ ci = S.ci;
    const double* __restrict__ av = S.av;
    const int64_t cnt = (R.r1 - R.r0) * nrhs;
    for (int64_t e = threadIdx.x; e < cnt; e += 256) {
        const int64_t i = R.r0 + e / nrhs;
        const int k = (int)(e % nrhs);
        double s = 0.0;
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) s += av[q] * x[(int64_t)ci[q] * nrhs + k];
        y[i * nrhs + k] = RES ? S.b[i * nrhs + k] - s : s;
    }
}

// Partial sums of one chunk: part[(chunk * J + j) * nrhs + k] = sum_i a_j[i,k] c[i,k]
// with (mode 0) a_j = V_j, c = w, j < J; (mode 1) a = c = w; (mode 2) a = c = r.
// nrhs <= 256.
__global__ __launch_bounds__(256) void k_kry_dot(const DKry* __restrict__ sys, const DKryChunk* __restrict__ ch,
                                                 const int32_t* __restrict__ act, int nrhs, int rc, int J, int mode,
                                                 double* __restrict__ part) {
    __shared__ double red[256];
    const DKryChunk C = ch[blockIdx.x];
    if (!act[C.sys]) return;                  // uniform over the work-group
    const DKry& S = sys[C.sys];
    const KryRows R = kry_rows_of(C, S.n, rc);
    const int tid = threadIdx.x;
    const int rpb = 256 / nrhs, T = rpb * nrhs;
    const int k = tid % nrhs, r0 = tid / nrhs;
    const double* __restrict__ c = mode == 2 ? S.r : S.w;
    for (int j = 0; j < J; ++j) {
        const double* __restrict__ a = mode == 0 ? S.V + (int64_t)j * S.nv : c;
        double s = 0.0;
        if (tid < T)
            for (int64_t i = R.r0 + r0; i < R.r1; i += rpb) s += a[i * nrhs + k] * c[i * nrhs + k];
        red[tid] = s;
        __syncthreads();
        if (tid < nrhs) {
            double t = 0.0;
            for (int q = 0; q < rpb; ++q) t += red[q * nrhs + tid];
            part[((int64_t)blockIdx.x * J + j) * nrhs + tid] = t;
        }
        __syncthreads();
    }
}

// sm[out_off + q] = sum over the system's chunks of part[(chunk * J) * nrhs + q], q < J nrhs
// One wavefront per value q of one system: lanes take the chunks in turn, then
// a wavefront sum; the order depends on the system's own chunks only.
__global__ __launch_bounds__(WAVE) void k_kry_reduce(const DKry* __restrict__ sys, const int32_t* __restrict__ act,
                                                     int cnt, const double* __restrict__ part, int out_off) {
    const int s = blockIdx.y, q = blockIdx.x;
    if (!act[s] || q >= cnt) return;                  // uniform over the wavefront
    const DKry& S = sys[s];
    double t = 0.0;
    for (int c = S.chunk0 + (int)threadIdx.x; c < S.chunk0 + S.nchunk; c += WAVE) t += part[(int64_t)c * cnt + q];
    t = wave_sum(t);
    if (threadIdx.x == 0) S.sm[out_off + q] = t;
}

// op 0: w -= sum_{j<J} V_j h_j (h at sm[off]);  op 1: x += sum_{j<Js} Z_j y_j (y at
// sm[off], Js = sm[off2]);  op 2: V_j = src / sqrt(n2) (src: r if J == 0 else w,
// n2 at sm[off]);  op 3: xe = [V_j; 0];  op 4: Z_j = xe[0:n]
__global__ __launch_bounds__(256) void k_kry_axpy(const DKry* __restrict__ sys, const DKryChunk* __restrict__ ch,
                                                  const int32_t* __restrict__ act, int nrhs, int rc, int op, int J,
                                                  int j, int off, int off2) {
    const DKryChunk C = ch[blockIdx.x];
    if (!act[C.sys]) return;
    const DKry& S = sys[C.sys];
    const KryRows R = kry_rows_of(C, S.n, rc);
    const int64_t e0 = R.r0 * nrhs, e1 = R.r1 * nrhs;
    const double* __restrict__ sm = S.sm;
    if (op == 0) {
        for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
            const int k = (int)(e % nrhs);
            double s = S.w[e];
            for (int q = 0; q < J; ++q) s -= S.V[(int64_t)q * S.nv + e] * sm[off + q * nrhs + k];
            S.w[e] = s;
        }
    } else if (op == 1) {
        const int Js = (int)sm[off2];
        for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
            const int k = (int)(e % nrhs);
            double s = S.x[e];
            for (int q = 0; q < Js; ++q) s += S.Z[(int64_t)q * S.nv + e] * sm[off + q * nrhs + k];
            S.x[e] = s;
        }
    } else if (op == 2) {
        const double* __restrict__ src = J == 0 ? S.r : S.w;
        double* __restrict__ dst = S.V + (int64_t)j * S.nv;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
            const double q = sm[off + (int)(e % nrhs)];
            dst[e] = q > 0.0 ? src[e] / sqrt(q) : 0.0;
        }
    } else if (op == 3) {
        const double* __restrict__ src = S.V + (int64_t)j * S.nv;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) S.xe[e] = src[e];
        // the extension rows n..n_ext are shared out over the system's chunks
        const int64_t q = blockIdx.x - S.chunk0;
        for (int64_t e = S.nv + q * 256 + threadIdx.x; e < S.n_ext * nrhs; e += (int64_t)S.nchunk * 256)
            S.xe[e] = 0.0;
    } else {
        double* __restrict__ dst = S.Z + (int64_t)j * S.nv;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) dst[e] = S.xe[e];
    }
}

__global__ void k_gather_idx(double* __restrict__ dst, const double* __restrict__ src,
                             const int64_t* __restrict__ idx, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = src[idx[e]];
}

// Sums per block, then one atomic add per block on a global counter.
__global__ void k_count_nonfinite(const double* __restrict__ v, int64_t n, unsigned long long* cnt) {
    __shared__ int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    int c = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        c += isfinite(v[e]) ? 0 : 1;
    if (c) atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0 && s) atomicAdd(cnt, (unsigned long long)s);
}

// Sum of squares for the Frobenius rule: one 256-thread work-group per merge
// piece (its source block) or per chunk of a value array; partial[g] per group.
__global__ __launch_bounds__(256) void k_sumsq(const DMerge* __restrict__ pieces, const double* __restrict__ v,
                                               int64_t n, int64_t chunk, double* __restrict__ partial) {
    __shared__ double s_w[256 / WAVE];
    const double* p;
    int64_t len;
    if (!v) {
        const DMerge d = pieces[blockIdx.x];
        p = d.src.p;
        len = (int64_t)d.src.nr * d.src.nc;
    } else {
        const int64_t e0 = (int64_t)blockIdx.x * chunk;
        p = v + e0;
        len = n - e0 < chunk ? n - e0 : chunk;
    }
    double a = 0.0;
    for (int64_t e = threadIdx.x; e < len; e += 256) a += p[e] * p[e];
    a = wave_sum(a);
    if (threadIdx.x % WAVE == 0) s_w[threadIdx.x / WAVE] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 256 / WAVE; ++w) t += s_w[w];
        partial[blockIdx.x] = t;
    }
}

// state[0] += sum of partial[0..n) (fixed order), state[1] = eps sqrt(state[0]),
// state[2 + level] = sqrt(state[0]).  One work-group.
__global__ __launch_bounds__(256) void k_norm_accum(const double* __restrict__ partial, int n, double* state,
                                                    double eps, int level) {
    __shared__ double s_t[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += partial[i];
    s_t[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s_t[threadIdx.x] += s_t[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n2 = state[0] + s_t[0];
        state[0] = n2;
        state[1] = eps * sqrt(n2);
        state[2 + level] = sqrt(n2);
    }
}

inline unsigned nblocks(int64_t work, int bs) { return (unsigned)((work + bs - 1) / bs); }

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_scatter(double* dst_base, const int64_t* idx, const double* val, int64_t nnz,
                          hipStream_t st) {
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(nblocks(nnz, 256)), dim3(256), 0, st, dst_base, idx, val, nnz);
    return hipGetLastError();
}

hipError_t launch_gather_idx(double* dst, const double* src, const int64_t* idx, int64_t n,
                             hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_idx, dim3(nblocks(n, 256)), dim3(256), 0, st, dst, src, idx, n);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const double* v, int64_t n, int64_t* cnt, hipStream_t st) {
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int64_t), st);
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(k_count_nonfinite, dim3(256), dim3(256), 0, st, v, n, (unsigned long long*)cnt);
    return hipGetLastError();
}

hipError_t launch_level_norm(const DMerge* pieces, int npieces, const double* v, int64_t nv, double* state,
                             double* partial, double eps, int level, hipStream_t st) {
    constexpr int64_t chunk = 65536;
    const int ng = v ? (int)((nv + chunk - 1) / chunk) : npieces;
    if (ng > 0) {
        hipLaunchKernelGGL(k_sumsq, dim3(ng), dim3(256), 0, st, pieces, v, nv, chunk, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_norm_accum, dim3(1), dim3(256), 0, st, partial, ng, state, eps, level);
    return hipGetLastError();
}

int level_norm_groups(int npieces, int64_t nv) {
    return nv > 0 ? (int)((nv + 65535) / 65536) : npieces;
}

hipError_t launch_merge(const DMerge* t, int n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge, dim3(n), dim3(256), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_compress(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap,
                           int max_c, hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t lds = (size_t)2 * (max_c > 0 ? max_c : 1) * sizeof(double);
    hipLaunchKernelGGL(k_compress, dim3(n), dim3(NT), lds, st, t, pieces, imap);
    return hipGetLastError();
}

hipError_t launch_compress_svd(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap,
                               int max_c, int max_M, bool fp32, int nt, hipStream_t st, bool gram) {
    if (n == 0) return hipSuccess;
    if (max_c <= 64) {
        static std::atomic<bool> attr64{false};
        if (!attr64) {
            const void* fs[12] = {
                (const void*)k_compress_svd64<double, 256, false>, (const void*)k_compress_svd64<double, 512, false>,
                (const void*)k_compress_svd64<double, 1024, false>, (const void*)k_compress_svd64<float, 256, false>,
                (const void*)k_compress_svd64<float, 512, false>, (const void*)k_compress_svd64<float, 1024, false>,
                (const void*)k_compress_svd64<double, 256, true>, (const void*)k_compress_svd64<double, 512, true>,
                (const void*)k_compress_svd64<double, 1024, true>, (const void*)k_compress_svd64<float, 256, true>,
                (const void*)k_compress_svd64<float, 512, true>, (const void*)k_compress_svd64<float, 1024, true>};
            for (const void* f : fs) {
                hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
                if (e != hipSuccess) return e;
            }
            attr64 = true;
        }
        const int cap = (kLdsBudget - 4096) / (int)sizeof(double);   // static LDS of the kernel aside
        const size_t lds = (size_t)cap * sizeof(double);
#define LRX_SVD64(FT, NTV, GR) hipLaunchKernelGGL((k_compress_svd64<FT, NTV, GR>), dim3(n), dim3(NTV), lds, st, t, pieces, imap, cap)
        if (gram) {
            if (fp32) {
                if (nt == 256) LRX_SVD64(float, 256, true);
                else if (nt == 512) LRX_SVD64(float, 512, true);
                else LRX_SVD64(float, 1024, true);
            } else {
                if (nt == 256) LRX_SVD64(double, 256, true);
                else if (nt == 512) LRX_SVD64(double, 512, true);
                else LRX_SVD64(double, 1024, true);
            }
        } else if (fp32) {
            if (nt == 256) LRX_SVD64(float, 256, false);
            else if (nt == 512) LRX_SVD64(float, 512, false);
            else LRX_SVD64(float, 1024, false);
        } else {
            if (nt == 256) LRX_SVD64(double, 256, false);
            else if (nt == 512) LRX_SVD64(double, 512, false);
            else LRX_SVD64(double, 1024, false);
        }
#undef LRX_SVD64
        return hipGetLastError();
    }
    // LDS plan: R and V (2 c^2) plus a chunk of ch rows of B (ch c), within the
    // dynamic LDS budget; below 16 rows per chunk the workspace path is used.
    static std::atomic<bool> attr_set{false};
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void*)k_compress_svd<8>, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
        (void)hipFuncSetAttribute((const void*)k_compress_svd<16>, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
        attr_set = true;
    }
    const int cap = kLdsBudget / (int)sizeof(double);
    const size_t lds = (size_t)cap * sizeof(double);
    if (max_c <= 64)
        hipLaunchKernelGGL(k_compress_svd<8>, dim3(n), dim3(NT), lds, st, t, pieces, imap, cap);
    else
        hipLaunchKernelGGL(k_compress_svd<16>, dim3(n), dim3(NT), lds, st, t, pieces, imap, cap);
    return hipGetLastError();
}

hipError_t launch_rand_sketch(const DCompress* t, const DRand* rt, DCompress* ctasks, int n, const DPiece* pieces,
                              const int32_t* imap, int first, int bf16, hipStream_t st) {
    if (n == 0) return hipSuccess;
    static std::atomic<bool> attr{false};
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_rand_sketch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)kRandLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_rand_sketch, dim3(n), dim3(NTR), kRandLds, st, t, rt, ctasks, pieces, imap, first, bf16);
    return hipGetLastError();
}

hipError_t launch_v_sign(const DCompress* t, int n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_v_sign, dim3(n), dim3(WAVE), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_rand_finish(const DCompress* t, const DRand* rt, const DCompress* ctasks, int n, int32_t* flags,
                              hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rand_finish, dim3(n), dim3(256), 0, st, t, rt, ctasks, flags);
    return hipGetLastError();
}

template <int mode>
static void launch_large_mode(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap,
                              double trunc_rel, double jac_u, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_compress_large<mode>, dim3(n), dim3(NTL), lds, st, t, pieces, imap, trunc_rel, jac_u);
}

hipError_t launch_compress_large(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap, int max_c,
                                 int max_M, double trunc_rel, int mode, hipStream_t st, bool jac_f32) {
    const double jac_u = jac_f32 ? 5.9604644775390625e-8 : 1.1102230246251565e-16;
    if (n == 0) return hipSuccess;
    const size_t lds = compress_large_lds(max_M, max_c);
    if (lds > (size_t)kLdsBudget) return hipErrorInvalidValue;
    static std::atomic<bool> attr{false};
    if (!attr) {
        hipError_t e = hipSuccess;
        for (const void* f : {(const void*)k_compress_large<0>, (const void*)k_compress_large<2>,
                              (const void*)k_compress_large<5>,
                              (const void*)k_compress_large<6>, (const void*)k_compress_large<7>,
                              (const void*)k_compress_large<8>, (const void*)k_compress_large<9>,
                              (const void*)k_large_round})
            if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
        if (e != hipSuccess) return e;
        attr = true;
    }
    switch (mode) {
    case 0: launch_large_mode<0>(t, n, pieces, imap, trunc_rel, jac_u, lds, st); break;
    case 2: launch_large_mode<2>(t, n, pieces, imap, trunc_rel, jac_u, lds, st); break;
    case 5: launch_large_mode<5>(t, n, pieces, imap, trunc_rel, jac_u, lds, st); break;
    case 6: launch_large_mode<6>(t, n, pieces, imap, trunc_rel, jac_u, lds, st); break;
    case 7: launch_large_mode<7>(t, n, pieces, imap, trunc_rel, jac_u, lds, st); break;
    case 8: launch_large_mode<8>(t, n, pieces, imap, trunc_rel, jac_u, lds, st); break;
    case 9: launch_large_mode<9>(t, n, pieces, imap, trunc_rel, jac_u, lds, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_assemble_large(const DCompress* t, int n, const DPiece* pieces, const int32_t* imap,
                                 int64_t max_mc, int max_pieces, bool copy, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t per = (int64_t)ASM_T * 16;                      // elements per work-group and pass
    const int gx = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (max_mc + per - 1) / per));
    hipLaunchKernelGGL(k_asm_zero, dim3(gx, n), dim3(ASM_T), 0, st, t);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && max_pieces > 0) {
        hipLaunchKernelGGL(k_asm_scatter, dim3(max_pieces, n), dim3(ASM_T), 0, st, t, pieces, imap);
        e = hipGetLastError();
    }
    if (e == hipSuccess && copy) {
        hipLaunchKernelGGL(k_asm_scale, dim3(gx, n), dim3(ASM_T), 0, st, t);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_gram_chol(const DCompress* t, int n, int max_c, double trunc_rel, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t lds = (size_t)max_c * (sizeof(double) + sizeof(int));
    if (lds > (size_t)kLdsBudget) return hipErrorInvalidValue;
    static std::atomic<bool> attr{false};
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_chol_panel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kLdsBudget);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int ntile = (max_c + 31) / 32, npair = ntile * (ntile + 1) / 2;
    hipLaunchKernelGGL(k_gram_tile<false>, dim3(npair, n), dim3(GT_T), 0, st, t, 0);
    hipError_t e = hipGetLastError();
    for (int J0 = 0; J0 < max_c && e == hipSuccess; J0 += CHB) {
        hipLaunchKernelGGL(k_chol_panel, dim3(n), dim3(NTL), lds, st, t, J0, trunc_rel);
        e = hipGetLastError();
        if (e == hipSuccess && J0 + CHB < max_c) {
            hipLaunchKernelGGL(k_gram_tile<true>, dim3(npair, n), dim3(GT_T), 0, st, t, J0);
            e = hipGetLastError();
        }
    }
    return e;
}

template <int which>
static hipError_t qr_blocked(const DCompress* t, int n, int max_c, int max_M, hipStream_t st) {
    const int nrmax = which == 0 ? max_M : max_c;             // rows of the matrix factored
    const size_t lds = (size_t)(nrmax + 1) * sizeof(double);
    if (lds > (size_t)kLdsBudget) return hipErrorInvalidValue;
    static std::atomic<bool> attr{false};
    if (which != 2 && !attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_qr_panel<which == 2 ? 0 : which>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int kqmax = which == 0 ? (max_c < max_M ? max_c : max_M) : max_c;
    const int npanel = (kqmax + QB - 1) / QB;
    for (int p = 0; p < npanel; ++p) {
        const int j0 = (which == 2 ? npanel - 1 - p : p) * QB;   // Q2: last panel first
        if constexpr (which != 2) {
            hipLaunchKernelGGL(k_qr_panel<which>, dim3(n), dim3(NTL), lds, st, t, j0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        // columns the panel changes (a task's panel may be narrower than QB)
        const int nchunk = (max_c - j0 + QB - 1) / QB;
        if (nchunk > 0) {
            hipLaunchKernelGGL(k_qr_update<which>, dim3(nchunk, n), dim3(NTL), 0, st, t, j0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_qr_blocked(const DCompress* t, int n, int max_c, int max_M, int which, hipStream_t st) {
    if (n == 0) return hipSuccess;
    switch (which) {
    case 0: return qr_blocked<0>(t, n, max_c, max_M, st);
    case 1: return qr_blocked<1>(t, n, max_c, max_M, st);
    case 2: return qr_blocked<2>(t, n, max_c, max_M, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_large_round(const DCompress* t, int n, int max_c, int round, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int kkmax = max_c < KK_LDS_MAX ? max_c : KK_LDS_MAX;
    const int nbk = (kkmax + KK_BLK - 1) / KK_BLK, nb2 = nbk + (nbk & 1);
    const size_t lds = (size_t)2 * KK_BLK * kkmax * sizeof(double);
    hipLaunchKernelGGL(k_large_round, dim3(nb2 / 2, n), dim3(NTL), lds, st, t, round);
    return hipGetLastError();
}

int large_rounds(int max_c) {
    const int kkmax = max_c < KK_LDS_MAX ? max_c : KK_LDS_MAX;
    const int nbk = (kkmax + KK_BLK - 1) / KK_BLK, nb2 = nbk + (nbk & 1);
    return nb2 - 1;
}

hipError_t launch_large_flags(const DCompress* t, int n, int32_t* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_large_flags, dim3(nblocks(n, 64)), dim3(64), 0, st, t, n, out);
    return hipGetLastError();
}

hipError_t launch_node_prep(const DPrep* t, int n, int max_m, const DProj* proj, const int32_t* imap,
                            int32_t* info, hipStream_t st, int* gj_perm) {
    if (n == 0) return hipSuccess;
    const bool blocked = max_m > 128;                // some pivot may take the multi-work-group form
    if (blocked && !gj_perm) return hipErrorInvalidValue;
    // LDS: the Gauss-Jordan exchange buffers (4 KiB), or the global variant's
    // scratch (2 m + 1 doubles)
    const size_t need = std::max<size_t>(4096, (size_t)(2 * (size_t)max_m + 8) * sizeof(double));
    if (need > (size_t)kLdsBudget) return hipErrorInvalidValue;
    static std::atomic<bool> attr{false};
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_node_prep, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kLdsBudget);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_gj_panel, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_node_prep, dim3(n), dim3(NTP), need, st, t, proj, imap, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !blocked) return e;
    const int mm = max_m < GJB_MAX ? max_m : GJB_MAX;
    const size_t lds_p = gj_blocked_lds(mm);
    for (int j0 = 0; j0 < mm && e == hipSuccess; j0 += GJB) {
        hipLaunchKernelGGL(k_gj_panel, dim3(n), dim3(NTP), lds_p, st, t, j0, gj_perm, info);
        e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_gj_update, dim3((mm + GJB_CW - 1) / GJB_CW, n), dim3(NTP), 0, st, t, j0,
                               (const int32_t*)info);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gj_unperm, dim3(n), dim3(NTP), 0, st, t, (const int*)gj_perm, (const int32_t*)info);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_gemm_tiles(const DGemm* g, const DTile* tiles, int ntile, int kmax, const int32_t* imap,
                             hipStream_t st) {
    if (ntile == 0) return hipSuccess;
    static std::atomic<bool> attr{false};
    if (!attr) {
        constexpr size_t most = (size_t)(GLA * GK + GLA * 32 + (GK + 1) * 32) * sizeof(double);
        hipError_t e = hipFuncSetAttribute((const void*)k_gemm_tiles, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)most);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int gk = kmax < 1 ? 1 : (kmax > GK ? GK : kmax);
    const size_t lds = (size_t)(GLA * gk + GLA * 32 + (gk + 1) * 32) * sizeof(double);
    hipLaunchKernelGGL(k_gemm_tiles, dim3(ntile), dim3(GT), lds, st, g, tiles, imap, gk);
    return hipGetLastError();
}

template <int NK>
hipError_t launch_sweep_nk(const SwNode* nodes, int n, double* x, int ldx, int k0, int ns,
                           hipStream_t st) {
    constexpr size_t lds = (size_t)kSwDescWords * 2 * sizeof(int32_t) + (size_t)kSwData * sizeof(double);
    static std::atomic<bool> attr{false};
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_sweep<NK>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_sweep<NK>, dim3(n, ns), dim3(kSwThreads), lds, st, nodes, x, ldx, k0);
    return hipGetLastError();
}

hipError_t launch_sweep(const SwNode* nodes, int n, double* x, int ldx, int k0, int nk, int ns, hipStream_t st) {
    if (n == 0 || ns == 0) return hipSuccess;
    switch (nk) {                                // nk <= kSwKS
        case 4: return launch_sweep_nk<4>(nodes, n, x, ldx, k0, ns, st);
        case 2: return launch_sweep_nk<2>(nodes, n, x, ldx, k0, ns, st);
        case 1: return launch_sweep_nk<1>(nodes, n, x, ldx, k0, ns, st);
        default: return hipErrorInvalidValue;
    }
}

// dst[e] = src[e] (as FP32 or FP64) for every segment (one work-group per segment)
__global__ void k_to_f32(const DConv* __restrict__ segs) {
    const DConv S = segs[blockIdx.x];
    if (S.f64)
        for (int64_t e = threadIdx.x; e < S.n; e += blockDim.x) static_cast<double*>(S.dst)[e] = S.src[e];
    else
        for (int64_t e = threadIdx.x; e < S.n; e += blockDim.x) static_cast<float*>(S.dst)[e] = (float)S.src[e];
}

hipError_t launch_to_f32(const DConv* segs, int n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, dim3(n), dim3(256), 0, st, segs);
    return hipGetLastError();
}

hipError_t launch_gather_perm(const double* b, int64_t ldb, const int32_t* perm, int n, int nrhs,
                              double* xt, int64_t ntot, hipStream_t st) {
    int64_t work = ntot * nrhs;
    if (work == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_perm, dim3(nblocks(work, 256)), dim3(256), 0, st, b, ldb, perm, n, nrhs, xt, ntot);
    return hipGetLastError();
}

hipError_t launch_scatter_perm(const double* xt, const int32_t* perm, int n, int nrhs, double* x,
                               int64_t ldx, hipStream_t st) {
    int64_t work = (int64_t)n * nrhs;
    hipLaunchKernelGGL(k_scatter_perm, dim3(nblocks(work, 256)), dim3(256), 0, st, xt, perm, n, nrhs, x, ldx);
    return hipGetLastError();
}

hipError_t kry_perm(const KryLaunch& L, int mode, int off) {
    if (L.nchunk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kry_perm, dim3(L.nchunk), dim3(256), 0, L.st, L.sys, L.ch, L.act, L.nrhs, L.rc, mode, off);
    return hipGetLastError();
}

hipError_t kry_spmv(const KryLaunch& L, bool residual, int j) {
    if (L.nchunk == 0) return hipSuccess;
    if (residual)
        hipLaunchKernelGGL(k_kry_spmv<true>, dim3(L.nchunk), dim3(256), 0, L.st, L.sys, L.ch, L.act, L.nrhs, L.rc, j);
    else
        hipLaunchKernelGGL(k_kry_spmv<false>, dim3(L.nchunk), dim3(256), 0, L.st, L.sys, L.ch, L.act, L.nrhs, L.rc, j);
    return hipGetLastError();
}

hipError_t kry_dots(const KryLaunch& L, int mode, int J, double* part, int out_off) {
    if (L.nchunk == 0 || J == 0) return hipSuccess;
    if (L.nrhs < 1 || L.nrhs > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_kry_dot, dim3(L.nchunk), dim3(256), 0, L.st, L.sys, L.ch, L.act, L.nrhs, L.rc, J, mode,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cnt = J * L.nrhs;
    hipLaunchKernelGGL(k_kry_reduce, dim3(cnt, L.nsys), dim3(WAVE), 0, L.st, L.sys, L.act, cnt,
                       (const double*)part, out_off);
    return hipGetLastError();
}

hipError_t kry_axpy(const KryLaunch& L, int op, int J, int j, int off, int off2) {
    if (L.nchunk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kry_axpy, dim3(L.nchunk), dim3(256), 0, L.st, L.sys, L.ch, L.act, L.nrhs, L.rc, op, J, j,
                       off, off2);
    return hipGetLastError();
}

}  // namespace lrx
