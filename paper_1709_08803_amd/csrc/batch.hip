// Batched FP64 vector and preconditioner kernels: one launch per operation for
// all problems of a lockstep round (blockIdx.y = problem).  Reductions are
// two-pass with fixed order, so every problem's result is deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch.h"
#include "bim_common.h"

namespace bim {

namespace {

constexpr int kT = 256;

__device__ double bsum256(double v) {
    __shared__ double sh[kT / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kT / 64; ++q) r += sh[q];
    __syncthreads();
    return r;
}

// part[row * kBRedBlocks + bx]; row = blockIdx.z (multidot) or 0 (dot)
__global__ __launch_bounds__(kT) void k_bdot_part(const BOp *__restrict__ ops, int multi) {
    const BOp o = ops[blockIdx.y];
    if (o.n == 0) return;  // empty slot of a padded op list
    const int row = multi ? (int)blockIdx.z : 0;
    if (row >= (multi ? o.nv : 1)) return;
    const double *a = multi ? o.a + (size_t)row * o.ld : o.a;
    double v = 0.0;
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < o.n; e += (long)kBRedBlocks * kT) v = fma(a[e], o.b[e], v);
    v = bsum256(v);
    if (threadIdx.x == 0) o.part[(size_t)row * kBRedBlocks + blockIdx.x] = v;
}

__global__ __launch_bounds__(kT) void k_bdot_sum(const BOp *__restrict__ ops, int multi, int take_sqrt) {
    const BOp o = ops[blockIdx.y];
    if (o.n == 0) return;
    const int row = blockIdx.x;
    if (row >= (multi ? o.nv : 1)) return;
    double v = (threadIdx.x < kBRedBlocks) ? o.part[(size_t)row * kBRedBlocks + threadIdx.x] : 0.0;
    v = bsum256(v);
    if (threadIdx.x == 0) o.sc[row] = take_sqrt ? sqrt(v) : v;
}

__global__ __launch_bounds__(kT) void k_borth(const BOp *__restrict__ ops, double sign) {
    const BOp o = ops[blockIdx.y];
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < o.n; e += (long)gridDim.x * kT) {
        double acc = o.c[e];
        for (int r = 0; r < o.nv; ++r) acc = fma(sign * o.a[(size_t)r * o.ld + e], o.sa[r], acc);
        o.c[e] = acc;
    }
}

__global__ __launch_bounds__(kT) void k_belem(const BOp *__restrict__ ops, int kind) {
    const BOp o = ops[blockIdx.y];
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < o.n; e += (long)gridDim.x * kT) {
        switch (kind) {
            case 0: o.c[e] = o.a[e] / o.sa[0]; break;                     // scale_inv
            case 1: o.c[e] = fma(o.sa[0], o.b[e], o.a[e]); break;         // axpy_dev
            case 2: {                                                     // quotient
                const double h = o.sa[0];
                o.c[e] = (h != 0.0) ? (o.a[e] - o.b[e]) / h : 0.0;
                break;
            }
            default:                                                      // axpby
                o.c[e] = (o.beta == 0.0) ? o.alpha * o.a[e] : fma(o.alpha, o.a[e], o.beta * o.b[e]);
        }
    }
}

__global__ __launch_bounds__(kT) void k_bmax_part(const BOp *__restrict__ ops) {
    __shared__ double sh[kT];
    const BOp o = ops[blockIdx.y];
    if (o.n == 0) return;  // uniform across the workgroup: no barrier is skipped by part of it
    double v = 0.0;
    for (long e = (long)blockIdx.x * kT + threadIdx.x; e < o.n; e += (long)kBRedBlocks * kT) {
        const double x = fabs(o.a[e]);
        v = (x > v || x != x) ? x : v;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int q = kT / 2; q > 0; q >>= 1) {
        if (threadIdx.x < q) {
            const double y = sh[threadIdx.x + q];
            if (y > sh[threadIdx.x] || y != y) sh[threadIdx.x] = y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) o.part[blockIdx.x] = sh[0];
}

__global__ void k_bmax_sum(const BOp *__restrict__ ops, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const BOp o = ops[i];
    if (o.n == 0) return;
    double v = 0.0;
    for (int b = 0; b < kBRedBlocks; ++b) {
        const double y = o.part[b];
        if (y > v || y != y) v = y;
    }
    o.sc[0] = v;
}

__global__ void k_bshift(const BOp *__restrict__ ops, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const BOp o = ops[i];
    if (!o.sc) return;  // empty slot (shift ops carry no vector length)
    if (o.alpha > 0.0) {
        o.sc[2] = o.alpha;
    } else {
        const double nu = o.sc[0], nv = o.sc[1];
        o.sc[2] = (nv > 0.0) ? sqrt(o.beta) * (1.0 + nu) / nv : 0.0;
    }
}

// Banded and dense products of many problems in one launch (blockIdx.y picks
// the problem).  Each wave owns kBGR consecutive rows (of one slice for the
// banded product) and reads two elements per lane per row (16 bytes in FP64,
// 8 in FP32) when the rows are aligned to two elements (even s or lda),
// loading each x segment once for its rows; otherwise one element per lane.
constexpr int kBGR = 4;
typedef double bdouble2 __attribute__((ext_vector_type(2)));

template <typename TA>
__device__ __forceinline__ void brows_dot(const TA *const (&row)[kBGR], const double *__restrict__ x, int len,
                                          bool vec, int lane, double (&acc)[kBGR]) {
    typedef TA ta2 __attribute__((ext_vector_type(2)));
    if (vec) {
        for (int q = lane; q < (len >> 1); q += 64) {
            const bdouble2 xv = *reinterpret_cast<const bdouble2 *>(x + 2 * q);
#pragma unroll
            for (int r = 0; r < kBGR; ++r) {
                const ta2 av = *reinterpret_cast<const ta2 *>(row[r] + 2 * q);
                acc[r] = fma((double)av[0], xv[0], acc[r]);
                acc[r] = fma((double)av[1], xv[1], acc[r]);
            }
        }
        if ((len & 1) && lane == 0)
#pragma unroll
            for (int r = 0; r < kBGR; ++r) acc[r] = fma((double)row[r][len - 1], x[len - 1], acc[r]);
    } else {
        for (int j = lane; j < len; j += 64) {
            const double xv = x[j];
#pragma unroll
            for (int r = 0; r < kBGR; ++r) acc[r] = fma((double)row[r][j], xv, acc[r]);
        }
    }
}

__device__ __forceinline__ void brows_store(double (&acc)[kBGR], int lane, int nvalid, double *y, const double *c,
                                            int row0, double alpha, double beta) {
#pragma unroll
    for (int r = 0; r < kBGR; ++r)
        for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o, 64);
    if (lane < nvalid) {
        double v = acc[0];
#pragma unroll
        for (int r = 1; r < kBGR; ++r) v = (lane == r) ? acc[r] : v;
        const int row = row0 + lane;
        y[row] = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * c[row]);
    }
}

template <typename TA>
__device__ __forceinline__ void bband_rows(const BBand &o, int l, int r0, int lane, double (&acc)[kBGR]) {
    const TA *band = (const TA *)o.band;
    const int m0 = max(0, l - o.w), m1 = min(o.M - 1, l + o.w);
    const bool vec = (o.s % 2 == 0) && ((uintptr_t)band % (2 * sizeof(TA)) == 0) && ((uintptr_t)o.x % 16 == 0);
    if (vec) {
        // as k_bandmv_rows: the element pairs of all band blocks as one range,
        // 64 per step, in the same order (the same sums as one problem alone)
        typedef TA ta2 __attribute__((ext_vector_type(2)));
        const int s = o.s, pairs = s >> 1, total = (m1 - m0 + 1) * pairs;
        int mb = lane / pairs, q = lane - mb * pairs;
        const TA *rows = band + ((size_t)l * (2 * o.w + 1) + (m0 - l + o.w)) * s * s;
        for (int g = lane; g < total; g += 64) {
            const TA *blk = rows + (size_t)mb * s * s;
            const bdouble2 xv = *reinterpret_cast<const bdouble2 *>(o.x + (size_t)(m0 + mb) * s + 2 * q);
            ta2 a[kBGR];
#pragma unroll
            for (int r = 0; r < kBGR; ++r)
                a[r] = *reinterpret_cast<const ta2 *>(blk + (size_t)min(r0 + r, s - 1) * s + 2 * q);
#pragma unroll
            for (int r = 0; r < kBGR; ++r) {
                acc[r] = fma((double)a[r][0], xv[0], acc[r]);
                acc[r] = fma((double)a[r][1], xv[1], acc[r]);
            }
            q += 64;
            while (q >= pairs) {
                q -= pairs;
                ++mb;
            }
        }
        return;
    }
    for (int m = m0; m <= m1; ++m) {
        const TA *blk = band + ((size_t)l * (2 * o.w + 1) + (m - l + o.w)) * o.s * o.s;
        const TA *row[kBGR];
#pragma unroll
        for (int r = 0; r < kBGR; ++r) row[r] = blk + (size_t)min(r0 + r, o.s - 1) * o.s;
        brows_dot<TA>(row, o.x + (size_t)m * o.s, o.s, false, lane, acc);
    }
}

__global__ __launch_bounds__(256) void k_bbandmv(const BBand *__restrict__ ops) {
    const BBand o = ops[blockIdx.y];
    const int gps = (o.s + kBGR - 1) / kBGR;  // row groups per slice
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= o.M * gps) return;
    const int l = wave / gps, r0 = (wave - l * gps) * kBGR;
    double acc[kBGR] = {};
    if (o.f32) bband_rows<float>(o, l, r0, lane, acc);
    else bband_rows<double>(o, l, r0, lane, acc);
    brows_store(acc, lane, min(kBGR, o.s - r0), o.y, o.c, l * o.s + r0, o.alpha, o.beta);
}

// Strictly lower / upper triangular products: as k_gemv_tri of the single-
// problem path, one 256-thread workgroup per GR rows of one slice, the four
// waves on the four quarters of the row range, partial sums added in LDS.
template <typename TA>
__device__ __forceinline__ void bgemv_tri_rows(const BGemv &o, int l, int r0, int wv, int lane,
                                               double (&acc)[kBGR]) {
    const TA *A = (const TA *)o.A;
    const long c0 = (o.part == 1) ? 0 : (long)(l + 1) * o.s, c1 = (o.part == 1) ? (long)l * o.s : o.n;
    const long len = c1 - c0;
    const bool vec = (o.s % 2 == 0) && (o.n % 2 == 0) && ((uintptr_t)A % (2 * sizeof(TA)) == 0) &&
                     ((uintptr_t)o.x % 16 == 0);
    const long ql = vec ? 2 * ((len / 2 + 3) / 4) : (len + 3) / 4;
    const long q0 = min(len, (long)wv * ql), q1 = min(len, q0 + ql);
    const TA *row[kBGR];
#pragma unroll
    for (int r = 0; r < kBGR; ++r) row[r] = A + ((size_t)l * o.s + min(r0 + r, o.s - 1)) * o.n + c0 + q0;
    brows_dot<TA>(row, o.x + c0 + q0, (int)(q1 - q0), vec, lane, acc);
}

__global__ __launch_bounds__(256) void k_bgemv_tri(const BGemv *__restrict__ ops) {
    __shared__ double partial[4][kBGR];
    const BGemv o = ops[blockIdx.y];
    const int gps = (o.s + kBGR - 1) / kBGR;  // row groups per slice
    const int g = blockIdx.x;
    if (g >= o.M * gps) return;  // uniform in the workgroup (also the empty slots, M = 0)
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lw = g / gps, r0 = (g - lw * gps) * kBGR;
    const int l = (o.part == 1) ? o.M - 1 - lw : lw;  // the longest rows first
    double acc[kBGR] = {};
    if (o.f32) bgemv_tri_rows<float>(o, l, r0, wv, lane, acc);
    else bgemv_tri_rows<double>(o, l, r0, wv, lane, acc);
#pragma unroll
    for (int r = 0; r < kBGR; ++r)
        for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off, 64);
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < kBGR; ++r) partial[wv][r] = acc[r];
    __syncthreads();
    if (wv == 0 && lane < kBGR && r0 + lane < o.s) {
        const double v = ((partial[0][lane] + partial[1][lane]) + partial[2][lane]) + partial[3][lane];
        const long row = (long)l * o.s + r0 + lane;
        o.y[row] = (o.beta == 0.0) ? o.alpha * v : fma(o.alpha, v, o.beta * o.c[row]);
    }
}

__global__ void k_bgather(const BOp *__restrict__ ops) {
    const BOp o = ops[blockIdx.x];
    if (!o.c) return;  // empty slot
    for (int t = threadIdx.x; t < 8 + o.nv; t += blockDim.x) o.c[t] = (t < 8) ? o.a[t] : o.b[t - 8];
}

constexpr int kElemBlocks = 128;  // grid-stride blocks per problem for elementwise ops

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

int b_dot(const BOp *ops, int count, bool take_sqrt, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_bdot_part, dim3(kBRedBlocks, count), dim3(kT), 0, s, ops, 0);
    hipLaunchKernelGGL(k_bdot_sum, dim3(1, count), dim3(kT), 0, s, ops, 0, take_sqrt ? 1 : 0);
    return hip_check(hipGetLastError(), "batched dot launch");
}

int b_multidot(const BOp *ops, int count, int max_nv, hipStream_t s) {
    if (count <= 0 || max_nv <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_bdot_part, dim3(kBRedBlocks, count, max_nv), dim3(kT), 0, s, ops, 1);
    hipLaunchKernelGGL(k_bdot_sum, dim3(max_nv, count), dim3(kT), 0, s, ops, 1, 0);
    return hip_check(hipGetLastError(), "batched multidot launch");
}

int b_orth(const BOp *ops, int count, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_borth, dim3(kElemBlocks, count), dim3(kT), 0, s, ops, -1.0);
    return hip_check(hipGetLastError(), "batched orth launch");
}

int b_combine(const BOp *ops, int count, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_borth, dim3(kElemBlocks, count), dim3(kT), 0, s, ops, 1.0);
    return hip_check(hipGetLastError(), "batched combine launch");
}

static int elem(const BOp *ops, int count, int kind, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_belem, dim3(kElemBlocks, count), dim3(kT), 0, s, ops, kind);
    return hip_check(hipGetLastError(), "batched elementwise launch");
}
int b_scale_inv(const BOp *ops, int count, hipStream_t s) { return elem(ops, count, 0, s); }
int b_axpy_dev(const BOp *ops, int count, hipStream_t s) { return elem(ops, count, 1, s); }
int b_quotient(const BOp *ops, int count, hipStream_t s) { return elem(ops, count, 2, s); }
int b_axpby(const BOp *ops, int count, hipStream_t s) { return elem(ops, count, 3, s); }

int b_maxabs(const BOp *ops, int count, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_bmax_part, dim3(kBRedBlocks, count), dim3(kT), 0, s, ops);
    hipLaunchKernelGGL(k_bmax_sum, dim3(cdiv(count, 64)), dim3(64), 0, s, ops, count);
    return hip_check(hipGetLastError(), "batched max launch");
}

int b_shift(const BOp *ops, int count, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_bshift, dim3(cdiv(count, 64)), dim3(64), 0, s, ops, count);
    return hip_check(hipGetLastError(), "batched shift launch");
}

int b_gather(const BOp *ops, int count, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_bgather, dim3(count), dim3(128), 0, s, ops);
    return hip_check(hipGetLastError(), "batched gather launch");
}

int b_bandmv(const BBand *ops, int count, int max_groups, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_bbandmv, dim3(cdiv(max_groups, 4), count), dim3(256), 0, s, ops);
    return hip_check(hipGetLastError(), "batched bandmv launch");
}

int b_gemv_tri(const BGemv *ops, int count, int max_groups, hipStream_t s) {
    if (count <= 0) return BIM_OK;
    if (max_groups <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_bgemv_tri, dim3(max_groups, count), dim3(256), 0, s, ops);
    return hip_check(hipGetLastError(), "batched gemv launch");
}

}  // namespace bim
