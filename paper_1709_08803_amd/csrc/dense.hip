// FP64 dense building blocks for the preconditioner: batched GEMM, batched
// Gauss-Jordan inversion with partial pivoting, matrix-vector products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "bim_common.h"
#include "dense.h"

namespace bim {

namespace {

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// Operand pointers in the global address space: generic (flat) loads count on
// the LDS counter as well, so an LDS read of the current K step would wait for
// the next step's operand loads.
template <typename T>
using GlobalPtr = __attribute__((address_space(1))) T *;

// C = alpha A B + beta C (row-major, FP64) on the matrix cores.  64 x 64 output
// tile per 256-thread workgroup; each wave owns 32 x 32 = 2 x 2 tiles of
// v_mfma_f64_16x16x4f64.  K advances through LDS in steps of 32, and the next
// step's operands are loaded into registers while the current step's MFMAs run.
// Operand layout of the 16x16x4 FP64 MFMA: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; the accumulator's element v of lane l is
// D[l / 16 + 4 v][l % 16] (lane layout checked on gfx950).  Registers are
// capped for three waves per SIMD (three workgroups per compute unit): a
// single wave per SIMD leaves the matrix unit idle between its MFMAs (measured:
// the preconditioner setup's batched block products 3 ms faster than at the
// compiler's choice of two).
constexpr int TM = 64, TN = 64, TK = 32;
typedef double double4_t __attribute__((ext_vector_type(4)));

// The tile (x, y) and item z of a workgroup, in an XCD-aware order.  The
// hardware hands workgroup i (linear over x, y, z) to XCD i mod 8, and each XCD
// has its own L2; workgroup i takes the logical tile base(i mod 8) + i / 8, so
// that each XCD works through one contiguous range of tiles in x, y, z order:
// the tiles of one product, and neighbouring products that share an operand
// block, then meet in one L2 (a bijection for any tile count).
struct Tile3 {
    int x, y, z;
};
__device__ __forceinline__ Tile3 xcd_tile() {
    constexpr unsigned kXcds = 8;
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned n = gx * gy * gridDim.z;
    const unsigned id = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned per = n / kXcds, rem = n % kXcds, x = id % kXcds;
    const unsigned t = x * per + min(x, rem) + id / kXcds;
    return {(int)(t % gx), (int)((t / gx) % gy), (int)(t / (gx * gy))};
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm(
    const GemmItem *__restrict__ items, int m, int n, int k, int lda, int ldb, int ldc, double alpha, double beta) {
    const Tile3 tl = xcd_tile();
    const GemmItem it = items[tl.z];
    const GlobalPtr<const double> A = (GlobalPtr<const double>)it.A;
    const GlobalPtr<const double> B = (GlobalPtr<const double>)it.B;
    const GlobalPtr<double> C = (GlobalPtr<double>)it.C;
    __shared__ double As[TM][TK + 1];
    __shared__ double Bs[TK][TN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int row0 = tl.y * TM, col0 = tl.x * TN;
    const int li = lane & 15, lk = lane >> 4;
    // each thread stages 8 elements of A (rows e >> 5, cols e & 31) and 8 of B
    // (rows e >> 6, cols e & 63).  Loads are unconditional, at indices clamped
    // into the matrices: a row of A or a column of B outside the product only
    // feeds outputs that are not stored, and B rows past k are zeroed when
    // staged (the select sits there so that no load waits for its value).
    double ra[8], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + q * 256;
            const int ar = e >> 5, ac = e & 31;
            ra[q] = A[(size_t)min(row0 + ar, m - 1) * lda + min(k0 + ac, k - 1)];
            const int br = e >> 6, bc = e & 63;
            rb[q] = B[(size_t)min(k0 + br, k - 1) * ldb + min(col0 + bc, n - 1)];
        }
    };
    auto store = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + q * 256;
            As[e >> 5][e & 31] = ra[q];
            Bs[e >> 6][e & 63] = (k0 + (e >> 6) < k) ? rb[q] : 0.0;
        }
    };
    double4_t acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[t][u] = double4_t{0.0, 0.0, 0.0, 0.0};
    if (k > 0) {
        load(0);
        store(0);
    }
    // C (for beta != 0) is read at the start, at clamped indices, so that its
    // loads are in flight during the products instead of after them
    const bool rmw = beta != 0.0;
    double cv[2][2][4];
    if (rmw) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int gr = row0 + wm + 16 * t + lk + 4 * v, gc = col0 + wn + 16 * u + li;
                    cv[t][u][v] = C[(size_t)min(gr, m - 1) * ldc + min(gc, n - 1)];
                }
    }
    __syncthreads();
    for (int k0 = 0; k0 < k; k0 += TK) {
        const bool more = k0 + TK < k;
        if (more) load(k0 + TK);
#pragma unroll
        for (int kk = 0; kk < TK; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = As[wm + 16 * t + li][kk + lk];
                b[t] = Bs[kk + lk][wn + 16 * t + li];
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
            store(k0 + TK);
            __syncthreads();
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = row0 + wm + 16 * t + lk + 4 * v, gc = col0 + wn + 16 * u + li;
                if (gr < m && gc < n)
                    C[(size_t)gr * ldc + gc] = rmw ? fma(alpha, acc[t][u][v], beta * cv[t][u][v]) : alpha * acc[t][u][v];
            }
}

// C = alpha sum_{b < it.nkb} A_b B_b + beta C, with A_b = A + b sA and
// B_b = B + b sB (each m x k, k x n, row-major): one product of K = nkb k whose
// K-blocks lie at fixed strides, as a block row of a slice-banded matrix times
// a block column of another.  The same 64 x 64 tiles and MFMA layout as k_gemm;
// the accumulator stays in registers over all nkb blocks, so C is read and
// written once instead of once per block.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm_kblocks(
    const GemmKItem *__restrict__ items, int m, int n, int k, int lda, int ldb, int ldc, long sA, long sB,
    double alpha, double beta) {
    const Tile3 tl = xcd_tile();
    const GemmKItem it = items[tl.z];
    const GlobalPtr<const double> A = (GlobalPtr<const double>)it.A;
    const GlobalPtr<const double> B = (GlobalPtr<const double>)it.B;
    const GlobalPtr<double> C = (GlobalPtr<double>)it.C;
    const int K = it.nkb * k;
    __shared__ double As[TM][TK + 1];
    __shared__ double Bs[TK][TN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int row0 = tl.y * TM, col0 = tl.x * TN;
    const int li = lane & 15, lk = lane >> 4;
    double ra[8], rb[8];
    // global K index g -> block g / k, column g % k; loads at clamped indices as in
    // k_gemm, the rows of B past K zeroed when staged
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + q * 256;
            const int ar = e >> 5, ac = e & 31;
            const int ga = min(k0 + ac, K - 1), ba = ga / k;
            ra[q] = A[(size_t)ba * sA + (size_t)min(row0 + ar, m - 1) * lda + (ga - ba * k)];
            const int br = e >> 6, bc = e & 63;
            const int gb = min(k0 + br, K - 1), bb = gb / k;
            rb[q] = B[(size_t)bb * sB + (size_t)(gb - bb * k) * ldb + min(col0 + bc, n - 1)];
        }
    };
    auto store = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + q * 256;
            As[e >> 5][e & 31] = ra[q];
            Bs[e >> 6][e & 63] = (k0 + (e >> 6) < K) ? rb[q] : 0.0;
        }
    };
    double4_t acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[t][u] = double4_t{0.0, 0.0, 0.0, 0.0};
    if (K > 0) {
        load(0);
        store(0);
    }
    const bool rmw = beta != 0.0;
    double cv[2][2][4];
    if (rmw) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int gr = row0 + wm + 16 * t + lk + 4 * v, gc = col0 + wn + 16 * u + li;
                    cv[t][u][v] = C[(size_t)min(gr, m - 1) * ldc + min(gc, n - 1)];
                }
    }
    __syncthreads();
    for (int k0 = 0; k0 < K; k0 += TK) {
        const bool more = k0 + TK < K;
        if (more) load(k0 + TK);
#pragma unroll
        for (int kk = 0; kk < TK; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = As[wm + 16 * t + li][kk + lk];
                b[t] = Bs[kk + lk][wn + 16 * t + li];
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
            store(k0 + TK);
            __syncthreads();
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = row0 + wm + 16 * t + lk + 4 * v, gc = col0 + wn + 16 * u + li;
                if (gr < m && gc < n)
                    C[(size_t)gr * ldc + gc] = rmw ? fma(alpha, acc[t][u][v], beta * cv[t][u][v]) : alpha * acc[t][u][v];
            }
}

// The same product for 128 < m <= 192 (the preconditioner's block rows, m = s):
// one workgroup holds all m rows of a TN-column panel, so that the workgroup
// count cdiv(n, TN) can be matched to the 256 compute units (a 64 x 64 tiling
// of 182 x 11102 gives 522 workgroups: three rounds, the last nearly empty).
// NW waves; wave w owns the 12 / NW row blocks of 16 rows from 16 (12 / NW) w
// (all TN / 16 column blocks).  K steps of 32 through two LDS buffers: the
// next step's operands are loaded into registers while the current step's
// MFMAs run and stored into the other buffer, one barrier per step.  The LDS
// buffers (118-135 KB) allow one workgroup per compute unit, so NW = 12 gives
// three waves per SIMD, which keep the matrix unit busy (with NW = 4, one wave
// per SIMD, the setup's S^-1 products took 10 ms more at 181 x 61).
constexpr int kTallM = 192, kTallK = 32, kTallWaves = 12;

// The 16x16x4 MFMA of each precision: operands as in k_gemm; the FP64
// accumulator holds D[l/16 + 4v][l%16], the FP32 one D[4(l/16) + v][l%16]
// (both lane layouts checked on gfx950 by in-bounds probes).
typedef float float4_t __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma16;
template <>
struct Mfma16<double> {
    typedef double4_t acc;
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma16<float> {
    typedef float4_t acc;
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

template <int TN, int NW, typename T = double>
__global__ __launch_bounds__(64 * NW) void k_gemm_tall(const GemmItemT<T> *__restrict__ items, int m, int n, int k,
                                                       int lda, int ldb, int ldc, double alpha, double beta) {
    constexpr int NT = 64 * NW, NB = TN / 16, RB = 12 / NW;
    constexpr int QA = kTallM * kTallK / NT, QB = (kTallK * TN + NT - 1) / NT;
    static_assert(QA * NT == kTallM * kTallK && RB * NW == 12, "tall tile shape");
    typedef Mfma16<T> MF;
    const GemmItemT<T> it = items[blockIdx.z];
    const GlobalPtr<const T> A = (GlobalPtr<const T>)it.A;
    const GlobalPtr<const T> B = (GlobalPtr<const T>)it.B;
    const GlobalPtr<T> C = (GlobalPtr<T>)it.C;
    __shared__ T As[2][kTallM][kTallK + 1];
    __shared__ T Bs[2][kTallK][TN + 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave * 16 * RB;
    const int col0 = blockIdx.x * TN;
    const int li = lane & 15, lk = lane >> 4;
    // unconditional loads at clamped indices, B rows past k zeroed when staged
    // (as in k_gemm)
    T ra[QA], rb[QB];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + q * NT;
            const int ar = e >> 5, ac = e & 31;
            ra[q] = A[(size_t)min(ar, m - 1) * lda + min(k0 + ac, k - 1)];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = min(tid + q * NT, kTallK * TN - 1);
            const int br = e / TN, bc = e - br * TN;
            rb[q] = B[(size_t)min(k0 + br, k - 1) * ldb + min(col0 + bc, n - 1)];
        }
    };
    auto store = [&](int buf, int k0) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + q * NT;
            As[buf][e >> 5][e & 31] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + q * NT;
            if (e < kTallK * TN) {
                const int br = e / TN;
                Bs[buf][br][e - br * TN] = (k0 + br < k) ? rb[q] : (T)0;
            }
        }
    };
    typename MF::acc acc[RB][NB];
#pragma unroll
    for (int t = 0; t < RB; ++t)
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[t][u] = typename MF::acc{0, 0, 0, 0};
    if (k > 0) {
        load(0);
        store(0, 0);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < k; k0 += kTallK) {
        const bool more = k0 + kTallK < k;
        if (more) load(k0 + kTallK);
        // the LDS operands of step kk + 4 are read before the MFMAs of step kk
        // (the scheduling barriers keep that order; left alone, the compiler read
        // them after the MFMAs and waited for them)
        T a[RB], b[NB];
#pragma unroll
        for (int t = 0; t < RB; ++t) a[t] = As[buf][wm + 16 * t + li][lk];
#pragma unroll
        for (int u = 0; u < NB; ++u) b[u] = Bs[buf][lk][16 * u + li];
#pragma unroll
        for (int kk = 0; kk < kTallK; kk += 4) {
            T an[RB], bn[NB];
            if (kk + 4 < kTallK) {
#pragma unroll
                for (int t = 0; t < RB; ++t) an[t] = As[buf][wm + 16 * t + li][kk + 4 + lk];
#pragma unroll
                for (int u = 0; u < NB; ++u) bn[u] = Bs[buf][kk + 4 + lk][16 * u + li];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < RB; ++t)
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    acc[t][u] = MF::step(a[t], b[u], acc[t][u]);
            __builtin_amdgcn_sched_barrier(0);
            if (kk + 4 < kTallK) {
#pragma unroll
                for (int t = 0; t < RB; ++t) a[t] = an[t];
#pragma unroll
                for (int u = 0; u < NB; ++u) b[u] = bn[u];
            }
        }
        // the other buffer was last read in the previous step, before its barrier
        if (more) store(buf ^ 1, k0 + kTallK);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int t = 0; t < RB; ++t)
#pragma unroll
        for (int u = 0; u < NB; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = wm + 16 * t + MF::row(lk, v), gc = col0 + 16 * u + li;
                if (gr < m && gc < n) {
                    const GlobalPtr<T> p = C + (size_t)gr * ldc + gc;
                    *p = (beta == 0.0) ? (T)alpha * acc[t][u][v] : fma((T)alpha, acc[t][u][v], (T)beta * (*p));
                }
            }
}

// Block-triangular product of the substitutions that invert unit block-
// triangular factors (blocks s x s): per item, for each output column block
// cb = cb0 .. cb0 + ncb - 1,
//   C[:, cb] = alpha sum_{j = klo .. khi-1} A[:, j] B[j, cb],
//   klo = max(0, cb - lo_off), khi = min(nk, cb - hi_off),
// with A an s x (nk s) row of blocks (leading dim lda), B nk block rows of
// leading dim ldb, C s rows of leading dim ldc (C = 0 where klo >= khi).  The
// K range of a column block leaves out the operand blocks that are zero by
// the triangular structure, which lets two factors' inverses share one array:
// the blocks of B outside the range may hold the other factor.  Workgroups as
// in k_gemm_tall: 192-row panels (blockIdx.y) of TN columns, ppb panels per
// column block (a panel never straddles two column blocks).  blockIdx.x walks
// the items' column blocks together (item = blockIdx.x % batch), each item
// from its deepest column block to its shallowest (`rev` reverses the column
// order for items whose K range grows with cb): the long workgroups start first
// and the short ones fill in after them (one workgroup per compute unit).
template <int TN, int NW, typename T = double>
__global__ __launch_bounds__(64 * NW) void k_gemm_tri(const GemmTriItemT<T> *__restrict__ items, int batch, int s,
                                                      int ppb, int lda, int ldb, int ldc, double alpha, int ntiles) {
    constexpr int NT = 64 * NW, NB = TN / 16, RB = 12 / NW;
    constexpr int QA = kTallM * kTallK / NT, QB = (kTallK * TN + NT - 1) / NT;
    static_assert(QA * NT == kTallM * kTallK && RB * NW == 12, "tall tile shape");
    typedef Mfma16<T> MF;
    // a grid narrower than the ntiles column tiles walks them with a stride
    // (every early exit below is uniform over the workgroup, and each tile's
    // last LDS reads are behind its K loop's final barrier)
    for (int bxl = blockIdx.x; bxl < ntiles; bxl += gridDim.x) {
    const int bx = bxl / batch;
    const GemmTriItemT<T> it = items[bxl - bx * batch];
    const int cbi = bx / ppb, pan = bx - cbi * ppb;
    if (cbi >= it.ncb) continue;
    const int cb = it.cb0 + (it.rev ? it.ncb - 1 - cbi : cbi);
    const int klo = max(0, cb - it.lo_off), khi = min(it.nk, cb - it.hi_off);
    const int row0 = blockIdx.y * kTallM, m = min(kTallM, s - row0);
    const int col0 = cb * s + pan * TN, cend = (cb + 1) * s;
    if (col0 >= cend) continue;
    const int k = max(0, khi - klo) * s;
    const GlobalPtr<const T> A = (GlobalPtr<const T>)(it.A + (size_t)row0 * lda + (size_t)klo * s);
    const GlobalPtr<const T> B = (GlobalPtr<const T>)(it.B + (size_t)klo * s * ldb);
    const GlobalPtr<T> C = (GlobalPtr<T>)(it.C + (size_t)row0 * ldc);
    // row pads: one element in FP64; in FP32, strides of 4 and 16 mod 32 words,
    // which spread a wave's 16 x 4 operand reads over distinct banks (a one-
    // float pad put 14% of the cycles in LDS bank conflicts)
    constexpr int PA = sizeof(T) == 4 ? 4 : 1, PB = sizeof(T) == 4 ? 16 : 1;
    __shared__ T As[2][kTallM][kTallK + PA];
    __shared__ T Bs[2][kTallK][TN + PB];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave * 16 * RB;
    const int li = lane & 15, lk = lane >> 4;
    // loads at clamped indices (rows past m, columns past the block's end), B
    // rows past k zeroed when staged
    T ra[QA], rb[QB];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + q * NT;
            const int ar = e >> 5, ac = e & 31;
            ra[q] = A[(size_t)min(ar, m - 1) * lda + min(k0 + ac, k - 1)];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = min(tid + q * NT, kTallK * TN - 1);
            const int br = e / TN, bc = e - br * TN;
            rb[q] = B[(size_t)min(k0 + br, k - 1) * ldb + min(col0 + bc, cend - 1)];
        }
    };
    auto store = [&](int buf, int k0) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + q * NT;
            As[buf][e >> 5][e & 31] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + q * NT;
            if (e < kTallK * TN) {
                const int br = e / TN;
                Bs[buf][br][e - br * TN] = (k0 + br < k) ? rb[q] : (T)0;
            }
        }
    };
    typename MF::acc acc[RB][NB];
#pragma unroll
    for (int t = 0; t < RB; ++t)
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[t][u] = typename MF::acc{0, 0, 0, 0};
    if (k > 0) {
        load(0);
        store(0, 0);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < k; k0 += kTallK) {
        const bool more = k0 + kTallK < k;
        if (more) load(k0 + kTallK);
        // the LDS operands of step kk + 4 are read before the MFMAs of step kk
        // (the scheduling barriers keep that order; left alone, the compiler read
        // them after the MFMAs and waited for them)
        T a[RB], b[NB];
#pragma unroll
        for (int t = 0; t < RB; ++t) a[t] = As[buf][wm + 16 * t + li][lk];
#pragma unroll
        for (int u = 0; u < NB; ++u) b[u] = Bs[buf][lk][16 * u + li];
#pragma unroll
        for (int kk = 0; kk < kTallK; kk += 4) {
            T an[RB], bn[NB];
            if (kk + 4 < kTallK) {
#pragma unroll
                for (int t = 0; t < RB; ++t) an[t] = As[buf][wm + 16 * t + li][kk + 4 + lk];
#pragma unroll
                for (int u = 0; u < NB; ++u) bn[u] = Bs[buf][kk + 4 + lk][16 * u + li];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < RB; ++t)
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    acc[t][u] = MF::step(a[t], b[u], acc[t][u]);
            __builtin_amdgcn_sched_barrier(0);
            if (kk + 4 < kTallK) {
#pragma unroll
                for (int t = 0; t < RB; ++t) a[t] = an[t];
#pragma unroll
                for (int u = 0; u < NB; ++u) b[u] = bn[u];
            }
        }
        if (more) store(buf ^ 1, k0 + kTallK);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int t = 0; t < RB; ++t)
#pragma unroll
        for (int u = 0; u < NB; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = wm + 16 * t + MF::row(lk, v), gc = col0 + 16 * u + li;
                if (gr < m && gc < cend) C[(size_t)gr * ldc + gc] = (T)alpha * acc[t][u][v];
            }
    }
}

// In-place Gauss-Jordan inversion of one s x s block (s <= 192) per 1024-thread
// workgroup, with the matrix held in registers: wave ty (= tid / 64, uniform in
// the wave) owns rows ty + 16 i (i < 12) and lane tx columns tx + 64 j (j < 3).
// Rows are eliminated in their natural order k = 0 .. s-1 with partial
// pivoting over the columns (the pivot of row k is its largest entry among the
// columns not yet used: partial pivoting of the transpose), so that the row
// being eliminated is known to every wave, and the pivot column q is read out
// of lane q % 64 with wave-uniform lane reads.  A column that has served as a
// pivot column is kept in its own scale: its true values are the stored ones
// times sc[q] = -1/p (row operations commute with column scaling), so that
// no step has to rescale it.  Step k:
//   wave k % 16 (row k is its register row k / 16) finds q (a DPP maximum of
//   packed pivot keys) and stages row k, scaled by 1/p and with 0 at column q,
//   in one of two LDS buffers (one barrier per step);
//   every row r: a[r][c] -= a[r][q] * rowk[c] (column q keeps a[r][q], which
//   is its new value -a[r][q]/p in the scale sc[q]);
//   row k becomes the staged row with -1 (= 1/p in that scale) at column q.
// After s steps the registers hold the inverse with rows and columns permuted
// by the pivot columns, storage[r][q_c] sc[q_c] = inverse[q_r][c]; the
// write-out applies the scales and undoes the permutation.  Only the owner
// wave indexes its registers by k / 16 (a switch); the update of all rows uses
// constant register indices.
constexpr int kRegTy = 16, kRegRows = 12, kRegCols = 3;
constexpr int kRegThreads = 64 * kRegTy;
constexpr int kRegMaxS = kRegTy * kRegRows;  // = 64 kRegCols = 192

// Largest value over the wave (unsigned): DPP shifts within rows of 16 lanes,
// then the row broadcasts of lanes 15 and 31; lane 63 ends with the maximum.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Pivot key of column c with value v: the upper 24 bits of the upper word of
// |v| (a non-negative double orders like its bit pattern; 12 mantissa bits
// are ample to choose a pivot), then 255 - c, so that ties go to the lowest
// column.  Columns already used (or beyond s) have key 0.
__device__ __forceinline__ unsigned pivot_key(double v, int c, bool usable) {
    const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(fabs(v)) >> 32);
    return usable ? ((hi & 0xffffff00u) | (unsigned)(255 - c)) : 0u;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

#define BIM_ROW_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11)

__global__ __launch_bounds__(kRegThreads) void k_invert_reg(const InvItem *__restrict__ items, int s,
                                                            int *__restrict__ info) {
    static_assert(kRegRows == 12, "BIM_ROW_CASES lists 12 register rows");
    const InvItem it = items[blockIdx.x];
    const int tx = threadIdx.x & 63;
    const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ double rowk[2][kRegMaxS], sc[kRegMaxS];
    __shared__ int qcol[kRegMaxS], qinv[kRegMaxS];
    __shared__ int s_bad;
    double a[kRegRows][kRegCols];
#pragma unroll
    for (int i = 0; i < kRegRows; ++i)
#pragma unroll
        for (int j = 0; j < kRegCols; ++j) {
            const int r = ty + kRegTy * i, c = tx + 64 * j;
            a[i][j] = (r < s && c < s) ? it.A[(size_t)r * it.lda + c] : 0.0;
        }
    unsigned used = 0;  // bit j: column tx + 64 j is a pivot column already (or lies beyond s)
#pragma unroll
    for (int j = 0; j < kRegCols; ++j)
        if (tx + 64 * j >= s) used |= 1u << j;
    if (threadIdx.x == 0) s_bad = 0;
    for (int c = threadIdx.x; c < kRegMaxS; c += kRegThreads) sc[c] = 1.0;
    __syncthreads();
    for (int k = 0; k < s; ++k) {
        const int w = k & (kRegTy - 1), ik = k / kRegTy;
        if (ty == w) {  // owner of row k: pivot column and the staged row
            double r0 = 0.0, r1 = 0.0, r2 = 0.0;
            switch (ik) {
#define BIM_GET(I)      \
    case I:             \
        r0 = a[I][0];   \
        r1 = a[I][1];   \
        r2 = a[I][2];   \
        break;
                BIM_ROW_CASES(BIM_GET)
#undef BIM_GET
            }
            unsigned key = pivot_key(r0, tx, !(used & 1u));
            key = max(key, pivot_key(r1, tx + 64, !(used & 2u)));
            key = max(key, pivot_key(r2, tx + 128, !(used & 4u)));
            const int q = 255 - (int)(wave_max_u32(key) & 0xffu);
            const bool inrange = q >= 0 && q < s;
            const int jq = inrange ? (q >> 6) : 0, lq = inrange ? (q & 63) : 0;
            const double piv = readlane_f64(jq == 0 ? r0 : (jq == 1 ? r1 : r2), lq);
            const bool ok = inrange && fabs(piv) > 0.0 && fabs(piv) <= 1.79e308;
            const double pinv = 1.0 / piv;
            double *rk = rowk[k & 1];
            rk[tx] = (tx == q) ? 0.0 : r0 * pinv;
            rk[tx + 64] = (tx + 64 == q) ? 0.0 : r1 * pinv;
            rk[tx + 128] = (tx + 128 == q) ? 0.0 : r2 * pinv;
            if (tx == 0) {
                qcol[k] = ok ? q : 0;
                sc[ok ? q : 0] = -pinv;
                if (!ok) s_bad = k + 1;
            }
        }
        __syncthreads();
        if (s_bad) break;
        const int q = __builtin_amdgcn_readfirstlane(qcol[k]);
        const int jq = q >> 6, lq = q & 63;
        const double *rk = rowk[k & 1];
        const double p0 = rk[tx], p1 = rk[tx + 64], p2 = rk[tx + 128];
        if (tx == lq) used |= 1u << jq;
        // factors a[r][q] of this wave's rows, from lane lq (wave-uniform)
        double f[kRegRows];
        if (jq == 0) {
#pragma unroll
            for (int r = 0; r < kRegRows; ++r) f[r] = readlane_f64(a[r][0], lq);
        } else if (jq == 1) {
#pragma unroll
            for (int r = 0; r < kRegRows; ++r) f[r] = readlane_f64(a[r][1], lq);
        } else {
#pragma unroll
            for (int r = 0; r < kRegRows; ++r) f[r] = readlane_f64(a[r][2], lq);
        }
#pragma unroll
        for (int r = 0; r < kRegRows; ++r) {
            a[r][0] = fma(-f[r], p0, a[r][0]);
            a[r][1] = fma(-f[r], p1, a[r][1]);
            a[r][2] = fma(-f[r], p2, a[r][2]);
        }
        if (ty == w) {  // row k: the staged row, -1 (1/p in the column's scale) at column q
            const double n0 = (tx == q) ? -1.0 : p0, n1 = (tx + 64 == q) ? -1.0 : p1,
                         n2 = (tx + 128 == q) ? -1.0 : p2;
            switch (ik) {
#define BIM_SET(I)      \
    case I:             \
        a[I][0] = n0;   \
        a[I][1] = n1;   \
        a[I][2] = n2;   \
        break;
                BIM_ROW_CASES(BIM_SET)
#undef BIM_SET
            }
        }
        // no barrier here: the next step stages its row in the other buffer, and
        // this buffer is rewritten only after every wave has passed the next
        // step's barrier, i.e. has finished this step
    }
    __syncthreads();
#undef BIM_ROW_CASES
    if (threadIdx.x == 0 && info) info[blockIdx.x] = s_bad;
    if (s_bad) return;
    for (int c = threadIdx.x; c < s; c += kRegThreads) qinv[qcol[c]] = c;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegRows; ++i)
#pragma unroll
        for (int j = 0; j < kRegCols; ++j) {
            const int r = ty + kRegTy * i, c = tx + 64 * j;
            if (r < s && c < s) it.Ainv[(size_t)qcol[r] * it.ldinv + qinv[c]] = a[i][j] * sc[c];
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

constexpr int GR = 4;  // rows per wave of the matrix-vector products

// y = alpha A' x + beta c for the strictly lower (part 1) or strictly upper
// (part 2) slice-block part A' of a dense n x n A (M slices of s): row block l
// reads columns [0, l s) or [(l+1) s, n).  Each 256-thread workgroup owns GR
// rows of one slice and its four waves split the row range in quarters (the
// rows' lengths run from 0 to n - s, and a single wave over a whole row would
// be the kernel's critical path); the four partial sums are added in LDS.
// Workgroups are numbered from the longest rows (the last slices of the lower
// part, the first of the upper).  With even s and aligned operands each lane
// reads two elements per row.
template <typename TA>
__global__ __launch_bounds__(256) void k_gemv_tri(const TA *__restrict__ A, long n, int M, int s, int part,
                                                  bool vec, const double *__restrict__ x, const double *c,
                                                  double *y, double alpha, double beta) {
    typedef double double2_t __attribute__((ext_vector_type(2)));
    typedef TA ta2_t __attribute__((ext_vector_type(2)));
    __shared__ double partial[4][GR];
    const int gps = (s + GR - 1) / GR;
    const int g = blockIdx.x;
    if (g >= M * gps) return;
    const int lw = g / gps, r0 = (g - lw * gps) * GR;
    const int l = (part == 1) ? M - 1 - lw : lw;
    const long c0 = (part == 1) ? 0 : (long)(l + 1) * s, c1 = (part == 1) ? (long)l * s : n;
    const long len = c1 - c0;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // this wave's quarter [q0, q1) of the row range (an even length when vec)
    const long ql = vec ? 2 * ((len / 2 + 3) / 4) : (len + 3) / 4;
    const long q0 = min(len, (long)wv * ql), q1 = min(len, q0 + ql);
    const TA *arow[GR];
#pragma unroll
    for (int r = 0; r < GR; ++r) arow[r] = A + ((size_t)l * s + min(r0 + r, s - 1)) * n + c0;
    const double *xs = x + c0;
    double acc[GR] = {};
    if (vec) {
        for (long q = q0 / 2 + lane; q < q1 / 2; q += 64) {
            const double2_t xv = *reinterpret_cast<const double2_t *>(xs + 2 * q);
#pragma unroll
            for (int r = 0; r < GR; ++r) {
                const ta2_t a = *reinterpret_cast<const ta2_t *>(arow[r] + 2 * q);
                acc[r] = fma((double)a[0], xv[0], acc[r]);
                acc[r] = fma((double)a[1], xv[1], acc[r]);
            }
        }
    } else {
        for (long j = q0 + lane; j < q1; j += 64) {
            const double xv = xs[j];
#pragma unroll
            for (int r = 0; r < GR; ++r) acc[r] = fma((double)arow[r][j], xv, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < GR; ++r)
        for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o, 64);
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < GR; ++r) partial[wv][r] = acc[r];
    __syncthreads();
    if (wv == 0 && lane < GR && r0 + lane < s) {
        const double v = ((partial[0][lane] + partial[1][lane]) + partial[2][lane]) + partial[3][lane];
        const long row = (long)l * s + r0 + lane;
        y[row] = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * c[row]);
    }
}

// y_l = alpha sum_{m in band} B[l][m] x_m + beta c_l for slice-block-banded B
// (blocks s x s, half-width w, elements of type TA): one wave per row of y.
template <typename TA>
__global__ __launch_bounds__(256) void k_bandmv(const TA *__restrict__ band, int M, int w, int s,
                                                const double *__restrict__ x, const double *c, double *y,
                                                double alpha, double beta) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= M * s) return;
    const int l = row / s, r = row - l * s;
    double v = 0.0;
    const int m0 = max(0, l - w), m1 = min(M - 1, l + w);
    for (int m = m0; m <= m1; ++m) {
        const TA *b = band + (((size_t)l * (2 * w + 1) + (m - l + w)) * s + r) * s;
        const double *xm = x + (size_t)m * s;
        for (int j = lane; j < s; j += 64) v = fma((double)b[j], xm[j], v);
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) y[row] = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * c[row]);
}

// Same banded product for even s and rows aligned to two elements: each wave
// owns GR consecutive rows of one slice and reads two elements per lane per
// row, loading every x segment once for its rows.
template <typename TA>
__global__ __launch_bounds__(256) void k_bandmv_rows(const TA *__restrict__ band, int M, int w, int s,
                                                     const double *__restrict__ x, const double *c, double *y,
                                                     double alpha, double beta) {
    typedef double double2_t __attribute__((ext_vector_type(2)));
    typedef TA ta2_t __attribute__((ext_vector_type(2)));
    const int gps = (s + GR - 1) / GR;  // row groups per slice
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= M * gps) return;
    const int l = wave / gps, r0 = (wave - l * gps) * GR;
    const int m0 = max(0, l - w), m1 = min(M - 1, l + w);
    const int pairs = s >> 1;
    // the element pairs of all band blocks of the rows as one range, 64 per step
    // (a block row of s = 182 is 91 pairs: walked block by block, the second
    // step of each left 37 of 64 lanes idle)
    const int total = (m1 - m0 + 1) * pairs;
    int mb = lane / pairs, q = lane - mb * pairs;  // this lane's block and pair
    const TA *rows = band + ((size_t)l * (2 * w + 1) + (m0 - l + w)) * s * s;
    double acc[GR] = {};
    for (int g = lane; g < total; g += 64) {
        const TA *blk = rows + (size_t)mb * s * s;
        const double2_t xv = *reinterpret_cast<const double2_t *>(x + (size_t)(m0 + mb) * s + 2 * q);
        ta2_t a[GR];
#pragma unroll
        for (int r = 0; r < GR; ++r)
            a[r] = *reinterpret_cast<const ta2_t *>(blk + (size_t)min(r0 + r, s - 1) * s + 2 * q);
#pragma unroll
        for (int r = 0; r < GR; ++r) {
            acc[r] = fma((double)a[r][0], xv[0], acc[r]);
            acc[r] = fma((double)a[r][1], xv[1], acc[r]);
        }
        q += 64;
        while (q >= pairs) {
            q -= pairs;
            ++mb;
        }
    }
#pragma unroll
    for (int r = 0; r < GR; ++r)
        for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o, 64);
    if (lane < GR && r0 + lane < s) {
        double v = acc[0];
#pragma unroll
        for (int r = 1; r < GR; ++r) v = (lane == r) ? acc[r] : v;
        const int row = l * s + r0 + lane;
        y[row] = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * c[row]);
    }
}

// FP64 -> FP32 element copy (grid-stride)
__global__ void k_to_float(const double *__restrict__ src, float *__restrict__ dst, size_t count) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
        dst[e] = (float)src[e];
}

__global__ void k_copy2d(const double *__restrict__ src, long lds, double *__restrict__ dst, long ldd, int rows,
                         int cols) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    dst[(size_t)r * ldd + c] = src[(size_t)r * lds + c];
}

// Block (l, j) of a strided family of rows x cols blocks, copied when
// l + j < lim: source src + l sl + j sj (leading dim lds), destination
// dst + l dl + j dj (leading dim ldd).  Grid (elements, l, j).
__global__ void k_copy_blocks(const double *__restrict__ src, long sl, long sj, long lds, double *__restrict__ dst,
                              long dl, long dj, long ldd, int rows, int cols, int lim) {
    const int l = blockIdx.y, j = blockIdx.z;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l + j >= lim || e >= (long)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    dst[(size_t)l * dl + (size_t)j * dj + (size_t)r * ldd + c] = src[(size_t)l * sl + (size_t)j * sj + (size_t)r * lds + c];
}

__global__ void k_identity(double *A, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    A[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// Panel width of the tall product for a single m x n product with
// 128 < m <= 192 (0: the 64 x 64 tiling).  Per compute unit the time goes as
// the rounds of 256 workgroups times the outputs of one workgroup: 64 x 64
// tiles against 192-row panels of width 32, 48 or 64; ties keep the tiles.
int tall_panel_width(int batch, int m, int n) {
    if (batch != 1 || m <= 128 || m > kTallM) return 0;
    int best = 0;
    long best_cost = (long)cdiv((long)cdiv(n, TN) * cdiv(m, TM), 256) * TM * TN;
    for (int tn : {64, 48, 32}) {
        const long cost = (long)cdiv(cdiv(n, tn), 256) * kTallM * tn;
        if (cost < best_cost) {
            best = tn;
            best_cost = cost;
        }
    }
    return best;
}

}  // namespace

int gemm_enqueue(const GemmItem *items_dev, int batch, int m, int n, int k, int lda, int ldb, int ldc,
                 double alpha, double beta, hipStream_t s) {
    if (batch <= 0 || m <= 0 || n <= 0) return BIM_OK;
    if (batch > 65535) return fail(BIM_EINVAL, "gemm batch too large");
    const int tn = tall_panel_width(batch, m, n);
    if (tn == 0) {
        dim3 grid(cdiv(n, TN), cdiv(m, TM), batch);
        hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, items_dev, m, n, k, lda, ldb, ldc, alpha, beta);
    } else {
        dim3 grid(cdiv(n, tn), 1, batch);
        constexpr int NW = kTallWaves;
        if (tn == 32)
            hipLaunchKernelGGL((k_gemm_tall<32, NW>), grid, dim3(64 * NW), 0, s, items_dev, m, n, k, lda, ldb, ldc,
                               alpha, beta);
        else if (tn == 48)
            hipLaunchKernelGGL((k_gemm_tall<48, NW>), grid, dim3(64 * NW), 0, s, items_dev, m, n, k, lda, ldb, ldc,
                               alpha, beta);
        else
            hipLaunchKernelGGL((k_gemm_tall<64, NW>), grid, dim3(64 * NW), 0, s, items_dev, m, n, k, lda, ldb, ldc,
                               alpha, beta);
    }
    return hip_check(hipGetLastError(), "gemm launch");
}

int gemm_kblocks_enqueue(const GemmKItem *items_dev, int batch, int m, int n, int k, int lda, int ldb, int ldc,
                         long sA, long sB, double alpha, double beta, hipStream_t s) {
    if (batch <= 0 || m <= 0 || n <= 0) return BIM_OK;
    if (batch > 65535) return fail(BIM_EINVAL, "gemm batch too large");
    dim3 grid(cdiv(n, TN), cdiv(m, TM), batch);
    hipLaunchKernelGGL(k_gemm_kblocks, grid, dim3(256), 0, s, items_dev, m, n, k, lda, ldb, ldc, sA, sB, alpha, beta);
    return hip_check(hipGetLastError(), "gemm launch");
}

int invert_enqueue(const InvItem *items_dev, int batch, int s_dim, double *work, int *info, hipStream_t s) {
    if (s_dim > kMaxS) return fail(BIM_EINVAL, "block too large to invert");
    if (batch <= 0) return BIM_OK;
    if (s_dim <= kRegMaxS)
        hipLaunchKernelGGL(k_invert_reg, dim3(batch), dim3(kRegThreads), 0, s, items_dev, s_dim, info);
    else
        hipLaunchKernelGGL(k_invert, dim3(batch), dim3(kInvThreads), 0, s, items_dev, s_dim, work, info);
    return hip_check(hipGetLastError(), "invert launch");
}

constexpr int kSplitS1 = kRegMaxS;

bool split_invert_applies(int s_dim) { return s_dim > kRegMaxS && s_dim <= 2 * kRegMaxS; }

size_t split_invert_scratch(int s_dim) {
    const size_t r = (size_t)std::max(0, s_dim - kSplitS1);
    return 2 * (size_t)kSplitS1 * r + r * r;
}

void split_invert_plan(const InvItem &it, int s_dim, double *scratch, SplitInv *P) {
    const int s1 = kSplitS1, r = s_dim - s1;
    const double *A = it.A;
    const long lda = it.lda, ldx = it.ldinv;
    double *X = it.Ainv;
    double *T = scratch, *W = scratch + (size_t)s1 * r, *Sc = W + (size_t)r * s1;
    double *X22 = X + (size_t)s1 * ldx + s1, *X21 = X + (size_t)s1 * ldx, *X12 = X + s1;
    P->inv11 = {A, lda, X, ldx};                  // A11^-1 into the leading block of X
    P->T = {X, A + s1, T};                        // T = A11^-1 A12           (s1 x r)
    P->Sc = {A + (size_t)s1 * lda, T, Sc};        // Sc = A22 - A21 T         (r x r; Sc holds A22)
    P->invS = {Sc, r, X22, ldx};                  // B22 = Sc^-1
    P->W = {A + (size_t)s1 * lda, X, W};          // W = A21 A11^-1           (r x s1)
    P->B21 = {X22, W, X21};                       // B21 = -B22 W
    P->B12 = {T, X22, X12};                       // B12 = -T B22
    P->B11 = {T, X21, X};                         // B11 = A11^-1 - T B21
}

int split_invert_enqueue(const SplitInv &P, const SplitInv *D, int s_dim, int *info, hipStream_t st) {
    if (!split_invert_applies(s_dim)) return fail(BIM_EINVAL, "split inversion needs 192 < s <= 384");
    const int s1 = kSplitS1, r = s_dim - s1;
    const int lda = (int)P.inv11.lda, ldx = (int)P.inv11.ldinv;
    int rc;
    hipLaunchKernelGGL(k_invert_reg, dim3(1), dim3(kRegThreads), 0, st, &D->inv11, s1, info);
    if ((rc = gemm_enqueue(&D->T, 1, s1, r, s1, ldx, lda, r, 1.0, 0.0, st))) return rc;
    if ((rc = copy2d_enqueue(P.inv11.A + (size_t)s1 * lda + s1, lda, const_cast<double *>(P.invS.A), r, r, r, st)))
        return rc;
    if ((rc = gemm_enqueue(&D->Sc, 1, r, r, s1, lda, r, r, -1.0, 1.0, st))) return rc;
    hipLaunchKernelGGL(k_invert_reg, dim3(1), dim3(kRegThreads), 0, st, &D->invS, r, info + 1);
    if ((rc = gemm_enqueue(&D->W, 1, r, s1, s1, lda, ldx, s1, 1.0, 0.0, st))) return rc;
    if ((rc = gemm_enqueue(&D->B21, 1, r, s1, r, ldx, s1, ldx, -1.0, 0.0, st))) return rc;
    if ((rc = gemm_enqueue(&D->B12, 1, s1, r, r, r, ldx, ldx, -1.0, 0.0, st))) return rc;
    if ((rc = gemm_enqueue(&D->B11, 1, s1, s1, r, r, ldx, ldx, -1.0, 1.0, st))) return rc;
    return hip_check(hipGetLastError(), "split inversion launch");
}

namespace {
template <typename TA>
int bandmv_launch(const TA *band, int M, int w, int s_dim, const double *x, const double *c, double *y,
                  double alpha, double beta, hipStream_t s) {
    const bool aligned = (s_dim % 2 == 0) && ((uintptr_t)band % (2 * sizeof(TA)) == 0) && ((uintptr_t)x % 16 == 0);
    if (aligned)
        hipLaunchKernelGGL(k_bandmv_rows<TA>, dim3(cdiv((long)M * ((s_dim + GR - 1) / GR), 4)), dim3(256), 0, s,
                           band, M, w, s_dim, x, c, y, alpha, beta);
    else
        hipLaunchKernelGGL(k_bandmv<TA>, dim3(cdiv((long)M * s_dim, 4)), dim3(256), 0, s, band, M, w, s_dim, x, c,
                           y, alpha, beta);
    return hip_check(hipGetLastError(), "bandmv launch");
}
}  // namespace

int bandmv_enqueue(const double *band, int M, int w, int s_dim, const double *x, const double *c, double *y,
                   double alpha, double beta, hipStream_t s) {
    return bandmv_launch(band, M, w, s_dim, x, c, y, alpha, beta, s);
}
int bandmv_enqueue(const float *band, int M, int w, int s_dim, const double *x, const double *c, double *y,
                   double alpha, double beta, hipStream_t s) {
    return bandmv_launch(band, M, w, s_dim, x, c, y, alpha, beta, s);
}

int to_float_enqueue(const double *src, float *dst, size_t count, hipStream_t s) {
    if (count == 0) return BIM_OK;
    const int blocks = (int)std::min<size_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(k_to_float, dim3(blocks), dim3(256), 0, s, src, dst, count);
    return hip_check(hipGetLastError(), "conversion launch");
}

namespace {
// Panel width of the block-triangular products: 32 (at 181 x 61 the setup took
// 50.3 ms with 32-wide panels throughout, 51.7 with 48, 54.2 with 64, and 51.0
// with a per-launch choice between them that weighed the deepest workgroup
// against the total work: more, narrower panels balance the compute units
// better than wider panels reuse their A operand).
constexpr int kTriPanel = 32;

template <typename T>
int gemm_tri_launch(const GemmTriItemT<T> *items_dev, int batch, int s, int max_ncb, int lda, int ldb, int ldc,
                    double alpha, int max_groups, hipStream_t st) {
    if (batch <= 0 || max_ncb <= 0 || s <= 0) return BIM_OK;
    if (batch > 65535) return fail(BIM_EINVAL, "gemm batch too large");
    if (max_groups < 0) return fail(BIM_EINVAL, "block-triangular product: negative workgroup cap");
    const int ppb = cdiv(s, kTriPanel);
    if ((long)max_ncb * ppb * batch > 0x7fffffffL) return fail(BIM_EINVAL, "block-triangular product too wide");
    const int ntiles = max_ncb * ppb * batch, panels = cdiv(s, kTallM);
    dim3 grid(max_groups > 0 ? std::min(ntiles, std::max(1, max_groups / panels)) : ntiles, panels, 1);
    hipLaunchKernelGGL((k_gemm_tri<kTriPanel, kTallWaves, T>), grid, dim3(64 * kTallWaves), 0, st, items_dev, batch, s,
                       ppb, lda, ldb, ldc, alpha, ntiles);
    return hip_check(hipGetLastError(), "block-triangular gemm launch");
}

template <typename TA>
int gemv_tri_launch(const TA *A, long n, int M, int s, int part, const double *x, const double *c, double *y,
                    double alpha, double beta, hipStream_t st) {
    if (M <= 0 || s <= 0) return BIM_OK;
    if (part != 1 && part != 2) return fail(BIM_EINVAL, "gemv_tri: part must be 1 (lower) or 2 (upper)");
    const bool vec = (s % 2 == 0) && (n % 2 == 0) && ((uintptr_t)A % (2 * sizeof(TA)) == 0) && ((uintptr_t)x % 16 == 0);
    const long groups = (long)M * ((s + GR - 1) / GR);
    if (groups > 0x7fffffffL) return fail(BIM_EINVAL, "gemv_tri: too many rows");
    hipLaunchKernelGGL(k_gemv_tri<TA>, dim3((unsigned)groups), dim3(256), 0, st, A, n, M, s, part, vec, x, c, y,
                       alpha, beta);
    return hip_check(hipGetLastError(), "gemv_tri launch");
}
}  // namespace

int gemm_tri_enqueue(const GemmTriItem *items_dev, int batch, int s, int max_ncb, int lda, int ldb, int ldc,
                     double alpha, hipStream_t st, int max_groups) {
    return gemm_tri_launch(items_dev, batch, s, max_ncb, lda, ldb, ldc, alpha, max_groups, st);
}
int gemm_tri_enqueue(const GemmTriItemF *items_dev, int batch, int s, int max_ncb, int lda, int ldb, int ldc,
                     double alpha, hipStream_t st, int max_groups) {
    return gemm_tri_launch(items_dev, batch, s, max_ncb, lda, ldb, ldc, alpha, max_groups, st);
}
int gemv_tri_enqueue(const double *A, long n, int M, int s, int part, const double *x, const double *c, double *y,
                     double alpha, double beta, hipStream_t st) {
    return gemv_tri_launch(A, n, M, s, part, x, c, y, alpha, beta, st);
}
int gemv_tri_enqueue(const float *A, long n, int M, int s, int part, const double *x, const double *c, double *y,
                     double alpha, double beta, hipStream_t st) {
    return gemv_tri_launch(A, n, M, s, part, x, c, y, alpha, beta, st);
}

int copy2d_enqueue(const double *src, long lds, double *dst, long ldd, int rows, int cols, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_copy2d, dim3(cdiv((long)rows * cols, 256)), dim3(256), 0, s, src, lds, dst, ldd, rows,
                       cols);
    return hip_check(hipGetLastError(), "copy launch");
}

int copy_blocks_enqueue(const double *src, long sl, long sj, long lds, double *dst, long dl, long dj, long ldd,
                        int rows, int cols, int nl, int nj, int lim, hipStream_t s) {
    if (rows <= 0 || cols <= 0 || nl <= 0 || nj <= 0) return BIM_OK;
    if (nl > 65535 || nj > 65535) return fail(BIM_EINVAL, "too many blocks to copy");
    hipLaunchKernelGGL(k_copy_blocks, dim3(cdiv((long)rows * cols, 256), nl, nj), dim3(256), 0, s, src, sl, sj, lds,
                       dst, dl, dj, ldd, rows, cols, lim);
    return hip_check(hipGetLastError(), "copy launch");
}

int identity_enqueue(double *A, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_identity, dim3(cdiv(n * n, 256)), dim3(256), 0, s, A, n);
    return hip_check(hipGetLastError(), "identity launch");
}

}  // namespace bim
