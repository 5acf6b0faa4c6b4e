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

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

int reduce_parts() { return kRedBlocks; }

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
