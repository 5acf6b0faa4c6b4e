// FP64 dense building blocks for the preconditioner: batched GEMM, batched
// Gauss-Jordan inversion with partial pivoting, matrix-vector products.
#include <hip/hip_runtime.h>

#include <vector>

#include "bim_common.h"
#include "dense.h"

namespace bim {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// C = alpha A B + beta C (row-major).  64 x 64 output tile per 256-thread
// workgroup, 4 x 4 outputs per thread, K staged through LDS in steps of 16.
constexpr int TM = 64, TN = 64, TK = 16;

__global__ __launch_bounds__(256) void k_gemm(const GemmItem *__restrict__ items, int m, int n, int k,
                                              int lda, int ldb, int ldc, double alpha, double beta) {
    const GemmItem it = items[blockIdx.z];
    const double *__restrict__ A = it.A;
    const double *__restrict__ B = it.B;
    double *__restrict__ C = it.C;
    __shared__ double As[TK][TM + 1];
    __shared__ double Bs[TK][TN + 1];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < k; k0 += TK) {
        // A tile: 64 rows x 16 cols; B tile: 16 rows x 64 cols (4 loads each per thread)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            const int ar = e >> 4, ac = e & 15;
            const int gr = row0 + ar, gc = k0 + ac;
            As[ac][ar] = (gr < m && gc < k) ? A[(size_t)gr * lda + gc] : 0.0;
            const int br = e >> 6, bc = e & 63;
            const int hr = k0 + br, hc = col0 + bc;
            Bs[br][bc] = (hr < k && hc < n) ? B[(size_t)hr * ldb + hc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gr = row0 + ty * 4 + r;
        if (gr >= m) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int gc = col0 + tx * 4 + c;
            if (gc >= n) continue;
            double *p = C + (size_t)gr * ldc + gc;
            *p = (beta == 0.0) ? alpha * acc[r][c] : fma(alpha, acc[r][c], beta * (*p));
        }
    }
}

// Gauss-Jordan inversion with partial pivoting of an s x s matrix per
// workgroup, on the augmented [A | I] held in `work` (s x 2s per matrix).
constexpr int kInvThreads = 1024;
constexpr int kMaxS = 1024;

__global__ __launch_bounds__(kInvThreads) void k_invert(const InvItem *__restrict__ items, int s,
                                                        double *__restrict__ work, int *__restrict__ info) {
    const InvItem it = items[blockIdx.x];
    double *W = work + (size_t)blockIdx.x * s * 2 * s;
    const int ld = 2 * s;
    const int tid = threadIdx.x;
    __shared__ double fac[kMaxS];
    __shared__ double red_v[kInvThreads];
    __shared__ int red_i[kInvThreads];
    __shared__ int bad;
    if (tid == 0) bad = 0;
    for (size_t e = tid; e < (size_t)s * 2 * s; e += kInvThreads) {
        const int r = (int)(e / ld), c = (int)(e % ld);
        W[e] = (c < s) ? it.A[(size_t)r * it.lda + c] : (c - s == r ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int col = 0; col < s; ++col) {
        // pivot: largest |W[r][col]|, r >= col
        double bv = -1.0;
        int bi = col;
        for (int r = col + tid; r < s; r += kInvThreads) {
            const double v = fabs(W[(size_t)r * ld + col]);
            if (v > bv) { bv = v; bi = r; }
        }
        red_v[tid] = bv;
        red_i[tid] = bi;
        __syncthreads();
        for (int o = kInvThreads / 2; o > 0; o >>= 1) {
            if (tid < o) {
                const double v2 = red_v[tid + o];
                const int i2 = red_i[tid + o];
                if (v2 > red_v[tid] || (v2 == red_v[tid] && i2 < red_i[tid])) {
                    red_v[tid] = v2;
                    red_i[tid] = i2;
                }
            }
            __syncthreads();
        }
        const int p = red_i[0];
        const double pv = red_v[0];
        if (!(pv > 0.0) || !isfinite(pv)) {
            if (tid == 0) bad = col + 1;
            __syncthreads();
            break;
        }
        if (p != col)
            for (int c = tid; c < ld; c += kInvThreads) {
                const double a = W[(size_t)col * ld + c];
                W[(size_t)col * ld + c] = W[(size_t)p * ld + c];
                W[(size_t)p * ld + c] = a;
            }
        __syncthreads();
        const double inv = 1.0 / W[(size_t)col * ld + col];
        for (int r = tid; r < s; r += kInvThreads) fac[r] = W[(size_t)r * ld + col];
        __syncthreads();
        for (int c = tid; c < ld; c += kInvThreads) W[(size_t)col * ld + c] *= inv;
        __syncthreads();
        for (size_t e = tid; e < (size_t)s * ld; e += kInvThreads) {
            const int r = (int)(e / ld), c = (int)(e % ld);
            if (r != col) W[e] = fma(-fac[r], W[(size_t)col * ld + c], W[e]);
        }
        __syncthreads();
    }
    if (tid == 0 && info) info[blockIdx.x] = bad;
    if (bad) return;
    for (size_t e = tid; e < (size_t)s * s; e += kInvThreads) {
        const int r = (int)(e / s), c = (int)(e % s);
        it.Ainv[(size_t)r * it.ldinv + c] = W[(size_t)r * ld + s + c];
    }
}

// y[r] = alpha A[r, :] x + beta c[r] for a dense row-major n_rows x n_cols A:
// one wave per row.
__global__ __launch_bounds__(256) void k_gemv(const double *__restrict__ A, long lda, const double *__restrict__ x,
                                              const double *c, double *y, int n_rows, int n_cols,
                                              double alpha, double beta) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n_rows) return;
    const double *a = A + (size_t)row * lda;
    double v = 0.0;
    for (int j = lane; j < n_cols; j += 64) v = fma(a[j], x[j], v);
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) y[row] = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * c[row]);
}

// y_l = alpha sum_{m in band} B[l][m] x_m + beta c_l for slice-block-banded B
// (blocks s x s, half-width w): one wave per row of y.
__global__ __launch_bounds__(256) void k_bandmv(const double *__restrict__ band, int M, int w, int s,
                                                const double *__restrict__ x, const double *c, double *y,
                                                double alpha, double beta) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= M * s) return;
    const int l = row / s, r = row - l * s;
    double v = 0.0;
    const int m0 = max(0, l - w), m1 = min(M - 1, l + w);
    for (int m = m0; m <= m1; ++m) {
        const double *b = band + (((size_t)l * (2 * w + 1) + (m - l + w)) * s + r) * s;
        const double *xm = x + (size_t)m * s;
        for (int j = lane; j < s; j += 64) v = fma(b[j], xm[j], v);
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) y[row] = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * c[row]);
}

__global__ void k_copy2d(const double *__restrict__ src, long lds, double *__restrict__ dst, long ldd, int rows,
                         int cols) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    dst[(size_t)r * ldd + c] = src[(size_t)r * lds + c];
}

__global__ void k_identity(double *A, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    A[e] = (e / n == e % n) ? 1.0 : 0.0;
}

}  // namespace

int gemm_enqueue(const GemmItem *items_dev, int batch, int m, int n, int k, int lda, int ldb, int ldc,
                 double alpha, double beta, hipStream_t s) {
    if (batch <= 0 || m <= 0 || n <= 0) return BIM_OK;
    if (batch > 65535) return fail(BIM_EINVAL, "gemm batch too large");
    dim3 grid(cdiv(n, TN), cdiv(m, TM), batch);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, items_dev, m, n, k, lda, ldb, ldc, alpha, beta);
    return hip_check(hipGetLastError(), "gemm launch");
}

int invert_enqueue(const InvItem *items_dev, int batch, int s_dim, double *work, int *info, hipStream_t s) {
    if (s_dim > kMaxS) return fail(BIM_EINVAL, "block too large to invert");
    if (batch <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_invert, dim3(batch), dim3(kInvThreads), 0, s, items_dev, s_dim, work, info);
    return hip_check(hipGetLastError(), "invert launch");
}

int gemv_enqueue(const double *A, long lda, const double *x, const double *c, double *y, int rows, int cols,
                 double alpha, double beta, hipStream_t s) {
    hipLaunchKernelGGL(k_gemv, dim3(cdiv(rows, 4)), dim3(256), 0, s, A, lda, x, c, y, rows, cols, alpha, beta);
    return hip_check(hipGetLastError(), "gemv launch");
}

int bandmv_enqueue(const double *band, int M, int w, int s_dim, const double *x, const double *c, double *y,
                   double alpha, double beta, hipStream_t s) {
    hipLaunchKernelGGL(k_bandmv, dim3(cdiv((long)M * s_dim, 4)), dim3(256), 0, s, band, M, w, s_dim, x, c, y,
                       alpha, beta);
    return hip_check(hipGetLastError(), "bandmv launch");
}

int copy2d_enqueue(const double *src, long lds, double *dst, long ldd, int rows, int cols, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_copy2d, dim3(cdiv((long)rows * cols, 256)), dim3(256), 0, s, src, lds, dst, ldd, rows,
                       cols);
    return hip_check(hipGetLastError(), "copy launch");
}

int identity_enqueue(double *A, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_identity, dim3(cdiv(n * n, 256)), dim3(256), 0, s, A, n);
    return hip_check(hipGetLastError(), "identity launch");
}

}  // namespace bim
