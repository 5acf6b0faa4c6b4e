// Small FP64 vector kernels: deterministic reductions, axpy, difference quotient.
#include <hip/hip_runtime.h>

#include "bim_common.h"
#include "vec.h"

namespace bim {

namespace {

constexpr int kRedBlocks = 256;
constexpr int kRedThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-level sum of `v` over 256 threads; result valid in thread 0.
__device__ double block_sum(double v) {
    __shared__ double sh[kRedThreads / 64];
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kRedThreads / 64; ++q) r += sh[q];
    __syncthreads();
    return r;
}

// part[b] = sum over the block's grid-stride slice of a[i] * b[i]
__global__ __launch_bounds__(kRedThreads) void k_dot_partial(const double *__restrict__ a,
                                                             const double *__restrict__ b, long n,
                                                             double *__restrict__ part) {
    double v = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        v = fma(a[i], b[i], v);
    v = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// out[0] = sum of nparts partials (fixed order); optional sqrt
__global__ __launch_bounds__(kRedThreads) void k_sum_partials(const double *__restrict__ part, int nparts,
                                                              double *__restrict__ out, int take_sqrt) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += part[i];
    v = block_sum(v);
    if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(v) : v;
}

// h = sqrt(eps) (1 + |u|) / |v|  (0 when |v| = 0); scal = [|u|, |v|, h]
__global__ void k_fd_shift(double *scal, double sqrt_eps) {
    const double nu = scal[0], nv = scal[1];
    scal[2] = (nv > 0.0) ? sqrt_eps * (1.0 + nu) / nv : 0.0;
}

__global__ void k_axpy_dev(const double *__restrict__ x, const double *__restrict__ y, const double *hp,
                           double *__restrict__ out, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fma(hp[0], y[i], x[i]);
}

__global__ void k_quotient(const double *__restrict__ Fw, const double *__restrict__ Fu, const double *hp,
                           double *__restrict__ out, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double h = hp[0];
        out[i] = (h != 0.0) ? (Fw[i] - Fu[i]) / h : 0.0;
    }
}

__global__ void k_set(double *p, double v) { p[0] = v; }

// part[i * nb + b] = partial of V[i] . w over block b's grid-stride slice
__global__ __launch_bounds__(kRedThreads) void k_multidot_partial(const double *__restrict__ V, long ldv, int nv,
                                                                  const double *__restrict__ w, long n,
                                                                  double *__restrict__ part) {
    const int i = blockIdx.y;
    const double *vi = V + (size_t)i * ldv;
    double v = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        v = fma(vi[e], w[e], v);
    v = block_sum(v);
    if (threadIdx.x == 0) part[(size_t)i * gridDim.x + blockIdx.x] = v;
}

__global__ __launch_bounds__(kRedThreads) void k_sum_rows(const double *__restrict__ part, int nparts,
                                                          double *__restrict__ out, int accumulate) {
    const int i = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) v += part[(size_t)i * nparts + b];
    v = block_sum(v);
    if (threadIdx.x == 0) out[i] = accumulate ? out[i] + v : v;
}

// w -= sum_i V[i] h[i]
__global__ void k_orth_update(const double *__restrict__ V, long ldv, int nv, const double *__restrict__ h,
                              double *__restrict__ w, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double acc = w[e];
    for (int i = 0; i < nv; ++i) acc = fma(-V[(size_t)i * ldv + e], h[i], acc);
    w[e] = acc;
}

// x += sum_i Z[i] y[i]
__global__ void k_combine(const double *__restrict__ Z, long ldz, int nz, const double *__restrict__ y,
                          double *__restrict__ x, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double acc = x[e];
    for (int i = 0; i < nz; ++i) acc = fma(Z[(size_t)i * ldz + e], y[i], acc);
    x[e] = acc;
}

// out = x / (*den)
__global__ void k_scale_inv(const double *__restrict__ x, const double *den, double *__restrict__ out, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = x[e] / den[0];
}

// out = a x + b y
__global__ void k_axpby(double a, const double *__restrict__ x, double b, const double *y, double *out, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = (b == 0.0) ? a * x[e] : fma(a, x[e], b * y[e]);
}

__global__ __launch_bounds__(kRedThreads) void k_maxabs_partial(const double *__restrict__ a, long n,
                                                                double *__restrict__ part) {
    __shared__ double sh[kRedThreads];
    double v = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double x = fabs(a[i]);
        v = (x > v || x != x) ? x : v;  // NaN propagates
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double y = sh[threadIdx.x + o];
            if (y > sh[threadIdx.x] || y != y) sh[threadIdx.x] = y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_max_partials(const double *__restrict__ part, int nparts, double *out) {
    double v = 0.0;
    for (int i = 0; i < nparts; ++i) {
        const double y = part[i];
        if (y > v || y != y) v = y;
    }
    out[0] = v;
}

// u for zeta = 0, phi = psi = x (the undisturbed stream)
__global__ void k_uniform_stream(double *u, int N, int M, double x1) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nb = (long)(N + 1) * M;
    if (e >= 3 * nb) return;
    const int f = (int)(e / nb);
    const int c = (int)((e % nb) % (N + 1));
    u[e] = (f == 0) ? 0.0 : (c == 0 ? x1 : 1.0);
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

int reduce_parts() { return kRedBlocks; }

int multidot_enqueue(const double *V, long ldv, int nv, const double *w, long n, double *part, double *out,
                     bool accumulate, hipStream_t s) {
    if (nv <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_multidot_partial, dim3(kRedBlocks, nv), dim3(kRedThreads), 0, s, V, ldv, nv, w, n, part);
    hipLaunchKernelGGL(k_sum_rows, dim3(nv), dim3(kRedThreads), 0, s, part, kRedBlocks, out, accumulate ? 1 : 0);
    return hip_check(hipGetLastError(), "multidot launch");
}

int orth_update_enqueue(const double *V, long ldv, int nv, const double *h, double *w, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_orth_update, dim3(cdiv(n, 256)), dim3(256), 0, s, V, ldv, nv, h, w, n);
    return hip_check(hipGetLastError(), "orth launch");
}

int combine_enqueue(const double *Z, long ldz, int nz, const double *y, double *x, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3(cdiv(n, 256)), dim3(256), 0, s, Z, ldz, nz, y, x, n);
    return hip_check(hipGetLastError(), "combine launch");
}

int scale_inv_enqueue(const double *x, const double *den, double *out, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_inv, dim3(cdiv(n, 256)), dim3(256), 0, s, x, den, out, n);
    return hip_check(hipGetLastError(), "scale launch");
}

int axpby_enqueue(double a, const double *x, double b, const double *y, double *out, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(cdiv(n, 256)), dim3(256), 0, s, a, x, b, y, out, n);
    return hip_check(hipGetLastError(), "axpby launch");
}

int maxabs_enqueue(const double *a, long n, double *part, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_maxabs_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, n, part);
    hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(1), 0, s, part, kRedBlocks, out);
    return hip_check(hipGetLastError(), "maxabs launch");
}

int uniform_stream_enqueue(double *u, int N, int M, double x1, hipStream_t s) {
    hipLaunchKernelGGL(k_uniform_stream, dim3(cdiv(3L * (N + 1) * M, 256)), dim3(256), 0, s, u, N, M, x1);
    return hip_check(hipGetLastError(), "uniform stream launch");
}

int dot_enqueue(const double *a, const double *b, long n, double *part, double *out, bool take_sqrt,
                hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, n, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRedThreads), 0, s, part, kRedBlocks, out,
                       take_sqrt ? 1 : 0);
    return hip_check(hipGetLastError(), "dot kernel launch");
}

int fd_shift_enqueue(const double *u, const double *v, long n, double h, double eps, double *part,
                     double *scal, hipStream_t s) {
    if (h > 0.0) {
        hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, s, scal + 2, h);
        return hip_check(hipGetLastError(), "shift kernel launch");
    }
    int rc = dot_enqueue(u, u, n, part, scal + 0, true, s);
    if (rc) return rc;
    rc = dot_enqueue(v, v, n, part, scal + 1, true, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_fd_shift, dim3(1), dim3(1), 0, s, scal, sqrt(eps));
    return hip_check(hipGetLastError(), "shift kernel launch");
}

int axpy_dev_enqueue(const double *x, const double *y, const double *hp, double *out, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_dev, dim3(cdiv(n, 256)), dim3(256), 0, s, x, y, hp, out, n);
    return hip_check(hipGetLastError(), "axpy kernel launch");
}

int quotient_enqueue(const double *Fw, const double *Fu, const double *hp, double *out, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_quotient, dim3(cdiv(n, 256)), dim3(256), 0, s, Fw, Fu, hp, out, n);
    return hip_check(hipGetLastError(), "quotient kernel launch");
}

}  // namespace bim
