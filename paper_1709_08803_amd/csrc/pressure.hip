// Bottom pressure and the force on the topography (Section 2.1, eq.
// (bottompressure)): Bernoulli's equation on z = beta(x, y) evaluated from the
// bottom potential psi of a (converged) unknown vector.
//   k_psi_slices   psi at the nodes: psi_{1,j} plus the trapezoidal x-integral of
//                  (psi_x)_{.,j}, one wave per slice (64-wide scans)
//   k_pressure     psi_y by the y-differences used for zeta_y and phi_y, the
//                  pressure at every node, and per-workgroup partial sums of the
//                  force components
//   k_force        fixed-order sum of the partials (deterministic)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bim_common.h"

namespace bim {
namespace {

constexpr int kPresThreads = 256;
constexpr int kForceParts = 3;

__global__ __launch_bounds__(64) void k_psi_slices(const double *__restrict__ u, int N, int M, double dx,
                                                   double *__restrict__ psi) {
    const int j = blockIdx.x, lane = threadIdx.x;
    const double *s = u + (size_t)2 * (N + 1) * M + (size_t)j * (N + 1);  // [psi_1, psi_x(1..N)]
    double *o = psi + (size_t)j * N;
    const double hdx = 0.5 * dx;
    double run = s[0];
    for (int base = 0; base < N; base += 64) {
        const int i = base + lane;
        double inc = (i > 0 && i < N) ? hdx * (s[i] + s[i + 1]) : 0.0;
        for (int d = 1; d < 64; d <<= 1) {
            const double t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        if (i < N) o[i] = run + inc;
        run += __shfl(inc, 63, 64);
    }
}

// Second-order y-difference of a node field at (j, i): central inside, the
// one-sided three-point stencil on y_M, zero on the symmetry line of a half
// domain and the mirrored one-sided stencil on y_1 of a full domain.
__device__ __forceinline__ double y_diff(const double *g, int j, int i, int N, int M, double dy, int half) {
    const double c = 0.5 / dy;
    if (j > 0 && j < M - 1) return c * (g[(size_t)(j + 1) * N + i] - g[(size_t)(j - 1) * N + i]);
    if (j == M - 1)
        return c * (3.0 * g[(size_t)j * N + i] - 4.0 * g[(size_t)(j - 1) * N + i] + g[(size_t)(j - 2) * N + i]);
    return half ? 0.0 : c * (-3.0 * g[i] + 4.0 * g[(size_t)N + i] - g[(size_t)2 * N + i]);
}

__device__ __forceinline__ double wave_reduce(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(kPresThreads) void k_pressure(
    const double *__restrict__ u, const double *__restrict__ psi, const double *__restrict__ beta,
    const double *__restrict__ bx, const double *__restrict__ by, int N, int M, double dx, double dy, int half,
    double froude, double *__restrict__ pres, double *__restrict__ part) {
    __shared__ double red[kForceParts][kPresThreads / 64];
    const long n = (long)N * M;
    const long q = (long)blockIdx.x * kPresThreads + threadIdx.x;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (q < n) {
        const int j = (int)(q / N), i = (int)(q - (long)j * N);
        const double px = u[(size_t)2 * (N + 1) * M + (size_t)j * (N + 1) + 1 + i];
        const double py = y_diff(psi, j, i, N, M, dy, half);
        const double a = bx[q], b = by[q];
        const double kin = 0.5 * ((1.0 + a * a) * py * py + (1.0 + b * b) * px * px - 2.0 * a * b * px * py) /
                           (1.0 + a * a + b * b);
        const double inv_f2 = 1.0 / (froude * froude);
        const double p = 0.5 - kin - beta[q] * inv_f2;
        pres[q] = p;
        // trapezoidal weight of the node and the pressure beyond the undisturbed 1/F^2
        const double w = dx * dy * ((i == 0 || i == N - 1) ? 0.5 : 1.0) * ((j == 0 || j == M - 1) ? 0.5 : 1.0);
        const double dp = w * (p - inv_f2);
        fx = dp * a;
        fy = dp * b;
        fz = -dp;
    }
    fx = wave_reduce(fx);
    fy = wave_reduce(fy);
    fz = wave_reduce(fz);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = fx;
        red[1][wv] = fy;
        red[2][wv] = fz;
    }
    __syncthreads();
    if (threadIdx.x < kForceParts) {
        double s = 0.0;
        for (int k = 0; k < kPresThreads / 64; ++k) s += red[threadIdx.x][k];
        part[(size_t)blockIdx.x * kForceParts + threadIdx.x] = s;
    }
}

// force[c] = sum over workgroups of part[b][c] in a fixed order; on a half
// domain the mirror half doubles the x- and z-components and cancels y.
__global__ __launch_bounds__(64) void k_force(const double *__restrict__ part, int nparts, int half,
                                              double *__restrict__ force) {
    const int lane = threadIdx.x;
    for (int c = 0; c < kForceParts; ++c) {
        double s = 0.0;
        for (int b = lane; b < nparts; b += 64) s += part[(size_t)b * kForceParts + c];
        s = wave_reduce(s);
        if (lane == 0) force[c] = half ? (c == 1 ? 0.0 : 2.0 * s) : s;
    }
}

}  // namespace
}  // namespace bim

using namespace bim;

extern "C" int bim_bottom_pressure(const bim_problem *prob, const double *u, double *pres, double *force,
                                   void *stream) {
    int rc = validate(prob);
    if (rc) return rc;
    if (!u || !pres || !force) return fail(BIM_EINVAL, "u, pres and force must be device pointers");
    const Dims d(prob);
    hipStream_t s = (hipStream_t)stream;
    const int blocks = (int)((d.nnode + kPresThreads - 1) / kPresThreads);
    const size_t psi_bytes = ((sizeof(double) * d.nnode) + 255) & ~(size_t)255;
    void *ws = nullptr;
    if ((rc = hip_check(hipMallocAsync(&ws, psi_bytes + sizeof(double) * kForceParts * blocks, s),
                        "hipMallocAsync")))
        return rc;
    double *psi = (double *)ws;
    double *part = (double *)((char *)ws + psi_bytes);
    const int half = prob->half_domain ? 1 : 0;
    hipLaunchKernelGGL(k_psi_slices, dim3(d.M), dim3(64), 0, s, u, d.N, d.M, prob->dx, psi);
    hipLaunchKernelGGL(k_pressure, dim3(blocks), dim3(kPresThreads), 0, s, u, psi, prob->beta, prob->beta_x,
                       prob->beta_y, d.N, d.M, prob->dx, prob->dy, half, prob->froude, pres, part);
    hipLaunchKernelGGL(k_force, dim3(1), dim3(64), 0, s, part, blocks, half, force);
    rc = hip_check(hipGetLastError(), "bottom pressure launch");
    const int rf = hip_check(hipFreeAsync(ws, s), "hipFreeAsync");
    return rc ? rc : rf;
}
