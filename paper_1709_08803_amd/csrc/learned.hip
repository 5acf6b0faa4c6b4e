// Learned initial guess: a small convolutional encoder + MLP that maps
// (F, bottom topography on the mesh), and optionally the linear start itself,
// to a correction of the linear start's (zeta_x, phi_x) on the same mesh.  Hand-written bf16 kernels with FP32
// accumulation: matrix-core (MFMA 16x16x16 bf16) GEMMs for the dense
// contractions (convolutions through im2col, fully connected layers), and
// elementwise kernels for bias, ReLU, loss and Adam.  FP32 master weights.
//
// Layout (NHWC, row-major):
//   X0  [B][H][W][C0]     channels: (beta + 1) / 0.3, (F - 1.25) / 0.75 and, with
//                         in_linear, the linear start's zeta_x / 0.2, (phi_x - 1) / 0.2
//   Y1  [B][H1][W1][C1]   conv 3x3 stride 2 pad 1, ReLU      H1 = ceil(H/2), W1 = ceil(W/2)
//   Y2  [B][H2][W2][C2]   conv 3x3 stride 2 pad 1, ReLU      H2 = ceil(H1/2), W2 = ceil(W1/2)
//   Y3  [B][D3]           fully connected on [Y2, F], ReLU
//   Y4  [B][2 H W]        fully connected, linear: (dzeta_x, dphi_x) / out_scale, [2][H][W]
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <vector>

#include "bim_common.h"
#include "learned.h"

namespace bim {

namespace {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf/nan
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

// C[m][n] = alpha sum_k A(m,k) B(k,n) + beta C[m][n]  (FP32 C, bf16 A/B with
// arbitrary strides so transposed operands need no copies).  64 x 64 tile per
// workgroup; each of the 4 waves owns 32 x 32 = 2 x 2 MFMA 16x16x16 tiles.
__global__ __launch_bounds__(256) void k_gemm_bf16(const uint16_t *__restrict__ A, long sam, long sak,
                                                   const uint16_t *__restrict__ B, long sbk, long sbn,
                                                   float *__restrict__ C, long ldc, int M, int N, int K, float alpha,
                                                   float beta) {
    __shared__ uint16_t As[64][16 + 2];
    __shared__ uint16_t Bs[16][64 + 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    float4_t acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            {
                const int r = e >> 4, c = e & 15;
                const int gm = m0 + r, gk = k0 + c;
                As[r][c] = (gm < M && gk < K) ? A[(size_t)gm * sam + (size_t)gk * sak] : (uint16_t)0;
            }
            {
                const int r = e >> 6, c = e & 63;
                const int gk = k0 + r, gn = n0 + c;
                Bs[r][c] = (gk < K && gn < N) ? B[(size_t)gk * sbk + (size_t)gn * sbn] : (uint16_t)0;
            }
        }
        __syncthreads();
        const int li = lane & 15, kq = (lane >> 4) * 4;
        for (int a = 0; a < 2; ++a) {
            short4_t af;
            const int row = wm + a * 16 + li;
            af[0] = (short)As[row][kq + 0];
            af[1] = (short)As[row][kq + 1];
            af[2] = (short)As[row][kq + 2];
            af[3] = (short)As[row][kq + 3];
            for (int b = 0; b < 2; ++b) {
                short4_t bfr;
                const int col = wn + b * 16 + li;
                bfr[0] = (short)Bs[kq + 0][col];
                bfr[1] = (short)Bs[kq + 1][col];
                bfr[2] = (short)Bs[kq + 2][col];
                bfr[3] = (short)Bs[kq + 3][col];
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bfr, acc[a][b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const int li = lane & 15, rq = (lane >> 4) * 4;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + a * 16 + rq + r, gn = n0 + wn + b * 16 + li;
                if (gm < M && gn < N) {
                    float *p = C + (size_t)gm * ldc + gn;
                    *p = (beta == 0.f) ? alpha * acc[a][b][r] : alpha * acc[a][b][r] + beta * (*p);
                }
            }
}

// im2col for a 3x3, stride 2, pad 1 convolution on NHWC input.
// cols[(b, oy, ox)][(ky, kx, c)]  (K = 9 Cin), zero outside the image.
__global__ void k_im2col(const uint16_t *__restrict__ X, uint16_t *__restrict__ cols, int B, int H, int W, int Cin,
                         int Ho, int Wo) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long K = 9L * Cin;
    if (e >= (long)B * Ho * Wo * K) return;
    const long row = e / K;
    const int kk = (int)(e % K);
    const int c = kk % Cin, kx = (kk / Cin) % 3, ky = kk / (3 * Cin);
    const int ox = (int)(row % Wo), oy = (int)((row / Wo) % Ho), b = (int)(row / ((long)Wo * Ho));
    const int iy = 2 * oy - 1 + ky, ix = 2 * ox - 1 + kx;
    cols[e] = (iy >= 0 && iy < H && ix >= 0 && ix < W) ? X[(((size_t)b * H + iy) * W + ix) * Cin + c] : (uint16_t)0;
}

// col2im (adjoint of k_im2col), FP32: dX[b][iy][ix][c] = sum over the (oy, ox, ky, kx) that read it.
__global__ void k_col2im(const float *__restrict__ dcols, float *__restrict__ dX, int B, int H, int W, int Cin,
                         int Ho, int Wo) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)B * H * W * Cin) return;
    const int c = (int)(e % Cin);
    const int ix = (int)((e / Cin) % W), iy = (int)((e / ((long)Cin * W)) % H), b = (int)(e / ((long)Cin * W * H));
    float v = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
        const int ty = iy + 1 - ky;
        if (ty < 0 || (ty & 1)) continue;
        const int oy = ty >> 1;
        if (oy >= Ho) continue;
        for (int kx = 0; kx < 3; ++kx) {
            const int tx = ix + 1 - kx;
            if (tx < 0 || (tx & 1)) continue;
            const int ox = tx >> 1;
            if (ox >= Wo) continue;
            const long row = ((long)b * Ho + oy) * Wo + ox;
            v += dcols[row * 9L * Cin + (ky * 3 + kx) * Cin + c];
        }
    }
    dX[e] = v;
}

// Y (FP32, [rows][n]) += bias; optional ReLU; writes the bf16 activation (row stride lda_out).
__global__ void k_bias_act(float *__restrict__ Y, const float *__restrict__ bias, uint16_t *__restrict__ out,
                           long lda_out, long rows, int n, int relu) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * n) return;
    const long r = e / n;
    const int c = (int)(e % n);
    float v = Y[e] + bias[c];
    if (relu && v < 0.f) v = 0.f;
    Y[e] = v;
    if (out) out[r * lda_out + c] = f2bf(v);
}

// dY (FP32) *= (Y > 0) and its bf16 copy (for use as a GEMM operand)
__global__ void k_relu_back(float *__restrict__ dY, const float *__restrict__ Y, uint16_t *__restrict__ dYb, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float g = (Y[e] > 0.f) ? dY[e] : 0.f;
    dY[e] = g;
    dYb[e] = f2bf(g);
}

// column sums of a [rows][n] FP32 matrix (bias gradients), deterministic
__global__ void k_colsum(const float *__restrict__ G, float *__restrict__ out, long rows, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    float v = 0.f;
    for (long r = 0; r < rows; ++r) v += G[r * n + c];
    out[c] = v;
}

// loss: sum (Y - T)^2 / (2 B n) per sample row partials, dY = (Y - T) / (B n), bf16 copy
__global__ void k_mse(const float *__restrict__ Y, const float *__restrict__ T, float *__restrict__ dY,
                      uint16_t *__restrict__ dYb, float *__restrict__ lossp, int B, int n) {
    const int b = blockIdx.x;
    __shared__ float sh[256];
    float acc = 0.f;
    const float inv = 1.f / ((float)B * (float)n);
    for (int c = threadIdx.x; c < n; c += 256) {
        const size_t e = (size_t)b * n + c;
        const float d = Y[e] - T[e];
        acc += d * d;
        const float g = d * inv;
        dY[e] = g;
        dYb[e] = f2bf(g);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int q = 128; q > 0; q >>= 1) {
        if (threadIdx.x < q) sh[threadIdx.x] += sh[threadIdx.x + q];
        __syncthreads();
    }
    if (threadIdx.x == 0) lossp[b] = 0.5f * sh[0] * inv;
}

// Adam on FP32 master weights; refresh the bf16 copy
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       uint16_t *__restrict__ wb, long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float wi = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[e] = wi;
    if (wb) wb[e] = f2bf(wi);
}

__global__ void k_to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = f2bf(x[e]);
}

// network input from a problem: NHWC [H = M][W = N][C0]; C0 = 4 adds the
// linear start's x-derivative planes (u_lin in the unknown vector's order)
__global__ void k_make_input(const double *__restrict__ beta, double froude, const double *__restrict__ ulin,
                             uint16_t *__restrict__ X, int N, int M, int C0) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * M) return;
    X[C0 * e] = f2bf((float)((beta[e] + 1.0) / 0.3));
    X[C0 * e + 1] = f2bf((float)((froude - 1.25) / 0.75));
    if (C0 == 4) {
        const int j = e / N, i = e - j * N;
        const size_t nb = (size_t)(N + 1) * M, at = (size_t)j * (N + 1) + 1 + i;
        X[C0 * e + 2] = f2bf((float)(ulin[at] / 0.2));
        X[C0 * e + 3] = f2bf((float)((ulin[nb + at] - 1.0) / 0.2));
    }
}

// A2' = [A2 | F-feature | 0 pad]: copies rows of A2 into a wider buffer and sets the F column
__global__ void k_append_feature(const uint16_t *__restrict__ A2, uint16_t *__restrict__ A2p, const float *__restrict__ f,
                                 int B, int d2, int ld) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)B * ld) return;
    const int b = (int)(e / ld), c = (int)(e % ld);
    A2p[e] = (c < d2) ? A2[(size_t)b * d2 + c] : (c == d2 ? f2bf(f[b]) : (uint16_t)0);
}

// u = u_lin + correction: the zeta_x, phi_x entries get out_scale * Y; the upstream
// values f_1 and the psi block stay those of the linear start (an error in the
// predicted f_x at the first node would enter f_1 amplified by |x1| / n through
// the radiation rows).
__global__ void k_apply_correction(const double *__restrict__ ulin, const float *__restrict__ Y, double *__restrict__ u,
                                   int N, int M, double scale) {
    const long nb = (long)(N + 1) * M;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * nb) return;
    const int f = (int)(e / nb);
    const int j = (int)((e % nb) / (N + 1)), c = (int)((e % nb) % (N + 1));
    double v = ulin[e];
    if (f < 2 && c >= 1) v += scale * (double)Y[(size_t)f * N * M + (size_t)j * N + (c - 1)];
    u[e] = v;
}

}  // namespace

// ------------------------------------------------------------------ network object
struct LgNet {
    lg_arch a;
    int C0;  // input channels
    int H1, W1, H2, W2, D2, D2p, Dout;
    long nparam[4], nbias[4];
    // FP32 master parameters, gradients, Adam moments; bf16 weight copies
    float *w[4], *b[4], *gw[4], *gb[4], *mw[4], *vw[4], *mb[4], *vb[4];
    uint16_t *wb[4];
    // activations (max batch)
    int maxB = 0;
    uint16_t *X0, *cols1, *A1, *cols2, *A2, *A2p, *A3, *dY4b, *dY3b, *dY2b, *dY1b;
    float *Y1, *Y2, *Y3, *Y4, *dY4, *dA3, *dA2, *dcols2, *dA1, *lossp, *ffeat;
    void *mem = nullptr;
    int step = 0;
};

static int lg_alloc(LgNet *net, int maxB) {
    const lg_arch &a = net->a;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t bytes = 0;
    std::vector<std::pair<void **, size_t>> plan;
    auto want = [&](void **p, size_t b) { plan.push_back({p, b}); bytes += al(b); };
    for (int l = 0; l < 4; ++l) {
        const size_t nw = (size_t)net->nparam[l], nb = (size_t)net->nbias[l];
        want((void **)&net->w[l], 4 * nw);
        want((void **)&net->b[l], 4 * nb);
        want((void **)&net->gw[l], 4 * nw);
        want((void **)&net->gb[l], 4 * nb);
        want((void **)&net->mw[l], 4 * nw);
        want((void **)&net->vw[l], 4 * nw);
        want((void **)&net->mb[l], 4 * nb);
        want((void **)&net->vb[l], 4 * nb);
        want((void **)&net->wb[l], 2 * nw);
    }
    const size_t B = maxB;
    const size_t r1 = B * net->H1 * net->W1, r2 = B * net->H2 * net->W2;
    want((void **)&net->X0, 2 * B * a.H * a.W * net->C0);
    want((void **)&net->cols1, 2 * r1 * 9 * net->C0);
    want((void **)&net->A1, 2 * r1 * a.C1);
    want((void **)&net->cols2, 2 * r2 * 9 * a.C1);
    want((void **)&net->A2, 2 * B * net->D2);
    want((void **)&net->A2p, 2 * B * net->D2p);
    want((void **)&net->A3, 2 * B * a.D3);
    want((void **)&net->dY4b, 2 * B * net->Dout);
    want((void **)&net->dY3b, 2 * B * a.D3);
    want((void **)&net->dY2b, 2 * r2 * a.C2);
    want((void **)&net->dY1b, 2 * r1 * a.C1);
    want((void **)&net->Y1, 4 * r1 * a.C1);
    want((void **)&net->Y2, 4 * r2 * a.C2);
    want((void **)&net->Y3, 4 * B * a.D3);
    want((void **)&net->Y4, 4 * B * net->Dout);
    want((void **)&net->dY4, 4 * B * net->Dout);
    want((void **)&net->dA3, 4 * B * a.D3);
    want((void **)&net->dA2, 4 * B * net->D2p);
    want((void **)&net->dcols2, 4 * r2 * 9 * a.C1);
    want((void **)&net->dA1, 4 * r1 * a.C1);
    want((void **)&net->lossp, 4 * B);
    want((void **)&net->ffeat, 4 * B);
    int rc = hip_check(hipMalloc(&net->mem, bytes), "hipMalloc(learned net)");
    if (rc) return rc;
    char *p = (char *)net->mem;
    for (auto &q : plan) {
        *q.first = p;
        p += al(q.second);
    }
    net->maxB = maxB;
    return hip_check(hipMemset(net->mem, 0, bytes), "hipMemset");
}

static int gemm(const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk, long sbn, float *C, long ldc,
                int M, int N, int K, float alpha, float beta, hipStream_t s) {
    if (M <= 0 || N <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_gemm_bf16, dim3(cdiv(N, 64), cdiv(M, 64)), dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C,
                       ldc, M, N, K, alpha, beta);
    return hip_check(hipGetLastError(), "bf16 gemm launch");
}

static int forward_impl(LgNet *net, const uint16_t *X0, const float *ffeat, int B, hipStream_t s) {
    const lg_arch &a = net->a;
    int rc;
    const long r1 = (long)B * net->H1 * net->W1, r2 = (long)B * net->H2 * net->W2;
    // conv1
    const int K1 = 9 * net->C0;
    hipLaunchKernelGGL(k_im2col, dim3(cdiv(r1 * K1, 256)), dim3(256), 0, s, X0, net->cols1, B, a.H, a.W, net->C0,
                       net->H1, net->W1);
    if ((rc = gemm(net->cols1, K1, 1, net->wb[0], a.C1, 1, net->Y1, a.C1, (int)r1, a.C1, K1, 1.f, 0.f, s))) return rc;
    hipLaunchKernelGGL(k_bias_act, dim3(cdiv(r1 * a.C1, 256)), dim3(256), 0, s, net->Y1, net->b[0], net->A1,
                       (long)a.C1, r1, a.C1, 1);
    // conv2
    hipLaunchKernelGGL(k_im2col, dim3(cdiv(r2 * 9 * a.C1, 256)), dim3(256), 0, s, net->A1, net->cols2, B, net->H1,
                       net->W1, a.C1, net->H2, net->W2);
    if ((rc = gemm(net->cols2, 9L * a.C1, 1, net->wb[1], a.C2, 1, net->Y2, a.C2, (int)r2, a.C2, 9 * a.C1, 1.f, 0.f, s)))
        return rc;
    hipLaunchKernelGGL(k_bias_act, dim3(cdiv(r2 * a.C2, 256)), dim3(256), 0, s, net->Y2, net->b[1], net->A2,
                       (long)a.C2, r2, a.C2, 1);
    // fc1 on [A2, F]
    hipLaunchKernelGGL(k_append_feature, dim3(cdiv((long)B * net->D2p, 256)), dim3(256), 0, s, net->A2, net->A2p, ffeat,
                       B, net->D2, net->D2p);
    if ((rc = gemm(net->A2p, net->D2p, 1, net->wb[2], a.D3, 1, net->Y3, a.D3, B, a.D3, net->D2 + 1, 1.f, 0.f, s)))
        return rc;
    hipLaunchKernelGGL(k_bias_act, dim3(cdiv((long)B * a.D3, 256)), dim3(256), 0, s, net->Y3, net->b[2], net->A3,
                       (long)a.D3, (long)B, a.D3, 1);
    // fc2 (linear)
    if ((rc = gemm(net->A3, a.D3, 1, net->wb[3], net->Dout, 1, net->Y4, net->Dout, B, net->Dout, a.D3, 1.f, 0.f, s)))
        return rc;
    hipLaunchKernelGGL(k_bias_act, dim3(cdiv((long)B * net->Dout, 256)), dim3(256), 0, s, net->Y4, net->b[3],
                       (uint16_t *)nullptr, 0L, (long)B, net->Dout, 0);
    return hip_check(hipGetLastError(), "learned forward launch");
}

static int backward_impl(LgNet *net, int B, hipStream_t s) {
    // expects dY4 and dY4b filled
    const lg_arch &a = net->a;
    int rc;
    const long r1 = (long)B * net->H1 * net->W1, r2 = (long)B * net->H2 * net->W2;
    // fc2: dW4 = A3^T dY4, db4, dA3 = dY4 W4^T
    if ((rc = gemm(net->A3, 1, a.D3, net->dY4b, net->Dout, 1, net->gw[3], net->Dout, a.D3, net->Dout, B, 1.f, 0.f, s)))
        return rc;
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(net->Dout, 256)), dim3(256), 0, s, net->dY4, net->gb[3], (long)B, net->Dout);
    if ((rc = gemm(net->dY4b, net->Dout, 1, net->wb[3], 1, net->Dout, net->dA3, a.D3, B, a.D3, net->Dout, 1.f, 0.f, s)))
        return rc;
    hipLaunchKernelGGL(k_relu_back, dim3(cdiv((long)B * a.D3, 256)), dim3(256), 0, s, net->dA3, net->Y3, net->dY3b,
                       (long)B * a.D3);
    // fc1: dW3 = A2p^T dY3 (K rows = D2 + 1), db3, dA2 = dY3 W3^T
    if ((rc = gemm(net->A2p, 1, net->D2p, net->dY3b, a.D3, 1, net->gw[2], a.D3, net->D2 + 1, a.D3, B, 1.f, 0.f, s)))
        return rc;
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(a.D3, 256)), dim3(256), 0, s, net->dA3, net->gb[2], (long)B, a.D3);
    if ((rc = gemm(net->dY3b, a.D3, 1, net->wb[2], 1, a.D3, net->dA2, net->D2p, B, net->D2, a.D3, 1.f, 0.f, s)))
        return rc;
    // dA2 rows have stride D2p; the ReLU mask is Y2 [r2][C2] = [B][D2] contiguous: compact first
    {
        // in-place compaction is unsafe; copy rows of dA2 (stride D2p) into dcols2 scratch as [B][D2]
        const size_t pitch = sizeof(float) * net->D2p, w = sizeof(float) * net->D2;
        if ((rc = hip_check(hipMemcpy2DAsync(net->dcols2, w, net->dA2, pitch, w, B, hipMemcpyDeviceToDevice, s),
                            "copy")))
            return rc;
        if ((rc = hip_check(hipMemcpyAsync(net->dA2, net->dcols2, w * B, hipMemcpyDeviceToDevice, s), "copy")))
            return rc;
    }
    hipLaunchKernelGGL(k_relu_back, dim3(cdiv(r2 * a.C2, 256)), dim3(256), 0, s, net->dA2, net->Y2, net->dY2b,
                       r2 * a.C2);
    // conv2: dW2 = cols2^T dY2, db2, dcols2 = dY2 W2^T, col2im -> dA1
    if ((rc = gemm(net->cols2, 1, 9L * a.C1, net->dY2b, a.C2, 1, net->gw[1], a.C2, 9 * a.C1, a.C2, (int)r2, 1.f, 0.f,
                   s)))
        return rc;
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(a.C2, 256)), dim3(256), 0, s, net->dA2, net->gb[1], r2, a.C2);
    if ((rc = gemm(net->dY2b, a.C2, 1, net->wb[1], 1, a.C2, net->dcols2, 9L * a.C1, (int)r2, 9 * a.C1, a.C2, 1.f, 0.f,
                   s)))
        return rc;
    hipLaunchKernelGGL(k_col2im, dim3(cdiv(r1 * a.C1, 256)), dim3(256), 0, s, net->dcols2, net->dA1, B, net->H1,
                       net->W1, a.C1, net->H2, net->W2);
    hipLaunchKernelGGL(k_relu_back, dim3(cdiv(r1 * a.C1, 256)), dim3(256), 0, s, net->dA1, net->Y1, net->dY1b,
                       r1 * a.C1);
    // conv1: dW1 = cols1^T dY1, db1
    const int K1 = 9 * net->C0;
    if ((rc = gemm(net->cols1, 1, K1, net->dY1b, a.C1, 1, net->gw[0], a.C1, K1, a.C1, (int)r1, 1.f, 0.f, s))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(a.C1, 256)), dim3(256), 0, s, net->dA1, net->gb[0], r1, a.C1);
    return hip_check(hipGetLastError(), "learned backward launch");
}

}  // namespace bim

using namespace bim;

extern "C" {

void lg_default_arch(lg_arch *a, int N, int M) {
    a->W = N;
    a->H = M;
    a->C1 = 16;
    a->C2 = 32;
    a->D3 = 256;
    a->in_linear = 1;
    a->out_scale = 0.05;
}

int lg_create(const lg_arch *arch, uint64_t seed, int max_batch, lg_net **out) {
    if (!arch || !out || max_batch < 1) return fail(BIM_EINVAL, "bad learned-net arguments");
    if (arch->H < 3 || arch->W < 3 || arch->C1 < 1 || arch->C2 < 1 || arch->D3 < 1 ||
        (arch->in_linear != 0 && arch->in_linear != 1))
        return fail(BIM_EINVAL, "bad learned-net architecture");
    LgNet *net = new LgNet();
    net->a = *arch;
    net->C0 = arch->in_linear ? 4 : 2;
    net->H1 = (arch->H + 1) / 2;
    net->W1 = (arch->W + 1) / 2;
    net->H2 = (net->H1 + 1) / 2;
    net->W2 = (net->W1 + 1) / 2;
    net->D2 = net->H2 * net->W2 * arch->C2;
    net->D2p = ((net->D2 + 1 + 15) / 16) * 16;
    net->Dout = 2 * arch->H * arch->W;
    const long fan[4] = {9L * net->C0, 9L * arch->C1, (long)net->D2 + 1, arch->D3};
    const long outs[4] = {arch->C1, arch->C2, arch->D3, net->Dout};
    for (int l = 0; l < 4; ++l) {
        net->nparam[l] = fan[l] * outs[l];
        net->nbias[l] = outs[l];
    }
    int rc = lg_alloc(net, max_batch);
    if (rc) {
        if (net->mem) (void)hipFree(net->mem);
        delete net;
        return rc;
    }
    // He-normal initialisation from a seeded host generator (weights [fan_in][fan_out])
    std::mt19937_64 gen(seed);
    for (int l = 0; l < 4; ++l) {
        std::normal_distribution<float> nd(0.f, (float)std::sqrt((l == 3 ? 1.0 : 2.0) / (double)fan[l]));
        std::vector<float> h((size_t)net->nparam[l]);
        for (auto &x : h) x = nd(gen);
        if ((rc = hip_check(hipMemcpy(net->w[l], h.data(), 4 * h.size(), hipMemcpyHostToDevice), "copy"))) break;
        hipLaunchKernelGGL(k_to_bf16, dim3(cdiv((long)h.size(), 256)), dim3(256), 0, 0, net->w[l], net->wb[l],
                           (long)h.size());
    }
    if (!rc) rc = hip_check(hipDeviceSynchronize(), "sync");
    if (rc) {
        (void)hipFree(net->mem);
        delete net;
        return rc;
    }
    *out = (lg_net *)net;
    return BIM_OK;
}

void lg_destroy(lg_net *n) {
    LgNet *net = (LgNet *)n;
    if (!net) return;
    if (net->mem) (void)hipFree(net->mem);
    delete net;
}

int lg_num_params(const lg_net *n, int layer, int64_t *weights, int64_t *biases) {
    const LgNet *net = (const LgNet *)n;
    if (!net || layer < 0 || layer > 3) return fail(BIM_EINVAL, "bad layer");
    if (weights) *weights = net->nparam[layer];
    if (biases) *biases = net->nbias[layer];
    return BIM_OK;
}

int lg_set_params(lg_net *n, int layer, const float *w_host, const float *b_host) {
    LgNet *net = (LgNet *)n;
    if (!net || layer < 0 || layer > 3) return fail(BIM_EINVAL, "bad layer");
    int rc;
    if (w_host) {
        if ((rc = hip_check(hipMemcpy(net->w[layer], w_host, 4 * net->nparam[layer], hipMemcpyHostToDevice), "copy")))
            return rc;
        hipLaunchKernelGGL(k_to_bf16, dim3(cdiv(net->nparam[layer], 256)), dim3(256), 0, 0, net->w[layer],
                           net->wb[layer], net->nparam[layer]);
    }
    if (b_host &&
        (rc = hip_check(hipMemcpy(net->b[layer], b_host, 4 * net->nbias[layer], hipMemcpyHostToDevice), "copy")))
        return rc;
    return hip_check(hipDeviceSynchronize(), "sync");
}

int lg_get_params(const lg_net *n, int layer, float *w_host, float *b_host, float *gw_host, float *gb_host) {
    const LgNet *net = (const LgNet *)n;
    if (!net || layer < 0 || layer > 3) return fail(BIM_EINVAL, "bad layer");
    int rc = hip_check(hipDeviceSynchronize(), "sync");
    if (rc) return rc;
    const size_t nw = 4 * net->nparam[layer], nb = 4 * net->nbias[layer];
    if (w_host && (rc = hip_check(hipMemcpy(w_host, net->w[layer], nw, hipMemcpyDeviceToHost), "copy"))) return rc;
    if (b_host && (rc = hip_check(hipMemcpy(b_host, net->b[layer], nb, hipMemcpyDeviceToHost), "copy"))) return rc;
    if (gw_host && (rc = hip_check(hipMemcpy(gw_host, net->gw[layer], nw, hipMemcpyDeviceToHost), "copy"))) return rc;
    if (gb_host && (rc = hip_check(hipMemcpy(gb_host, net->gb[layer], nb, hipMemcpyDeviceToHost), "copy"))) return rc;
    return BIM_OK;
}

int lg_forward(lg_net *n, const uint16_t *X0, const float *ffeat, int B, float *Y_out, void *stream) {
    LgNet *net = (LgNet *)n;
    if (!net || !X0 || !ffeat || B < 1 || B > net->maxB) return fail(BIM_EINVAL, "bad forward arguments");
    hipStream_t s = (hipStream_t)stream;
    int rc = forward_impl(net, X0, ffeat, B, s);
    if (rc) return rc;
    if (Y_out)
        rc = hip_check(hipMemcpyAsync(Y_out, net->Y4, sizeof(float) * B * net->Dout, hipMemcpyDeviceToDevice, s),
                       "copy");
    return rc;
}

int lg_train_step(lg_net *n, const uint16_t *X0, const float *ffeat, const float *T, int B, float lr, int update,
                  float *loss_out, void *stream) {
    LgNet *net = (LgNet *)n;
    if (!net || !X0 || !ffeat || !T || B < 1 || B > net->maxB) return fail(BIM_EINVAL, "bad training arguments");
    hipStream_t s = (hipStream_t)stream;
    int rc = forward_impl(net, X0, ffeat, B, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mse, dim3(B), dim3(256), 0, s, net->Y4, T, net->dY4, net->dY4b, net->lossp, B, net->Dout);
    if ((rc = backward_impl(net, B, s))) return rc;
    if (update) {
        ++net->step;
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
        for (int l = 0; l < 4; ++l) {
            hipLaunchKernelGGL(k_adam, dim3(cdiv(net->nparam[l], 256)), dim3(256), 0, s, net->w[l], net->gw[l],
                               net->mw[l], net->vw[l], net->wb[l], net->nparam[l], lr, b1, b2, eps, c1, c2);
            hipLaunchKernelGGL(k_adam, dim3(cdiv(net->nbias[l], 256)), dim3(256), 0, s, net->b[l], net->gb[l],
                               net->mb[l], net->vb[l], (uint16_t *)nullptr, net->nbias[l], lr, b1, b2, eps, c1, c2);
        }
    }
    if (loss_out) {
        std::vector<float> lp(B);
        if ((rc = hip_check(hipMemcpyAsync(lp.data(), net->lossp, sizeof(float) * B, hipMemcpyDeviceToHost, s), "copy")))
            return rc;
        if ((rc = hip_check(hipStreamSynchronize(s), "sync"))) return rc;
        double L = 0.0;
        for (float v : lp) L += v;
        *loss_out = (float)L;
    }
    return hip_check(hipGetLastError(), "train step launch");
}

int lg_make_input(const bim_problem *prob, const double *u_lin, int in_linear, uint16_t *X0, float *ffeat,
                  void *stream) {
    int rc = validate(prob);
    if (rc) return rc;
    if (!X0 || !ffeat) return fail(BIM_EINVAL, "X0 and ffeat must be device pointers");
    if (in_linear != 0 && in_linear != 1) return fail(BIM_EINVAL, "in_linear must be 0 or 1");
    if (in_linear && !u_lin) return fail(BIM_EINVAL, "the linear start is needed for in_linear inputs");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_make_input, dim3(cdiv((long)prob->N * prob->M, 256)), dim3(256), 0, s, prob->beta,
                       prob->froude, u_lin, X0, prob->N, prob->M, in_linear ? 4 : 2);
    const float f = (float)((prob->froude - 1.25) / 0.75);
    if ((rc = hip_check(hipMemcpyAsync(ffeat, &f, sizeof(float), hipMemcpyHostToDevice, s), "copy"))) return rc;
    return hip_check(hipStreamSynchronize(s), "sync");
}

int lg_infer_start(lg_net *n, const bim_problem *prob, const bim_precond *P, double *u_out, void *stream) {
    LgNet *net = (LgNet *)n;
    int rc = validate(prob);
    if (rc) return rc;
    if (!net || !u_out) return fail(BIM_EINVAL, "bad inference arguments");
    if (prob->N != net->a.W || prob->M != net->a.H) return fail(BIM_EINVAL, "mesh does not match the network");
    hipStream_t s = (hipStream_t)stream;
    // the linear start (fallback and base of the correction)
    if ((rc = bim_linear_start(prob, P, u_out, 0.0, stream))) return rc;
    const long nvec = 3L * (prob->N + 1) * prob->M;
    double *ulin = nullptr;
    if ((rc = hip_check(hipMallocAsync((void **)&ulin, sizeof(double) * nvec, s), "hipMallocAsync"))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(ulin, u_out, sizeof(double) * nvec, hipMemcpyDeviceToDevice, s), "copy"))) {
        (void)hipFreeAsync(ulin, s);
        return rc;
    }
    hipLaunchKernelGGL(k_make_input, dim3(cdiv((long)prob->N * prob->M, 256)), dim3(256), 0, s, prob->beta,
                       prob->froude, ulin, net->X0, prob->N, prob->M, net->C0);
    const float f = (float)((prob->froude - 1.25) / 0.75);
    if ((rc = hip_check(hipMemcpyAsync(net->ffeat, &f, sizeof(float), hipMemcpyHostToDevice, s), "copy"))) {
        (void)hipFreeAsync(ulin, s);
        return rc;
    }
    if ((rc = forward_impl(net, net->X0, net->ffeat, 1, s))) {
        (void)hipFreeAsync(ulin, s);
        return rc;
    }
    hipLaunchKernelGGL(k_apply_correction, dim3(cdiv(nvec, 256)), dim3(256), 0, s, ulin, net->Y4, u_out, prob->N,
                       prob->M, net->a.out_scale);
    (void)hipFreeAsync(ulin, s);
    return hip_check(hipStreamSynchronize(s), "sync");
}

}  // extern "C"
