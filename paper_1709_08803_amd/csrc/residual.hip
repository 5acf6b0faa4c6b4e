// Residual F(u) of the discretised boundary-integral system (Section 3.1) on gfx950.
//
// Four kernels, stream-ordered:
//   k_integrate   unpack u and integrate f_x along each slice (trapezoidal rule)
//   k_records     y-derivatives at the nodes; source-node records for S and B;
//                 collocation-point records at (x_{k+1/2}, y_l)
//   k_allpairs    the dense sums of eq. (new_finite_boundary_integral): every
//                 collocation point against every node of both boundaries and
//                 both y-images (hot loop)
//   k_finalize    reduction of the all-pairs partial sums, closed-form S2
//                 integral, 2 pi term, dynamic condition, radiation rows, and
//                 the row order of Appendix B
// The three node-level kernels take a PairDesc by value; their _batched forms
// serve many problems in one launch, each workgroup finding its problem from
// the first-workgroup offsets in the descriptors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "bim_common.h"

namespace bim {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// ------------------------------------------------------------------ rsqrt
// FP32: the hardware reciprocal square root (about 1 ulp).
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64: an estimate y refined by one Newton-Raphson step y (1 + e/2),
// e = 1 - x y^2, whose truncation error is (3/8) e^2 relative.  The estimate is
// the FP32 reciprocal square root of x rounded to FP32 (relative error ~1e-7,
// so the refined value is good to ~2e-14, far below the parity bound of the
// sums, 1e-12 of the sum of |terms|): on gfx950 the two conversions and
// v_rsq_f32 issue in ~10 cycles per wave against ~17 for v_rsq_f64, and one
// first-order step costs one FMA less than the second-order one the FP64
// estimate would otherwise get (the sums are bound by VALU issue).  x is a
// squared distance or a positive quadratic form well inside the FP32 range.
__device__ __forceinline__ double rsq(double x) {
    const double y = (double)__builtin_amdgcn_rsqf((float)x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// ------------------------------------------------------------------ batched lookup
// Problem of workgroup b in a batched node-level launch: the number of
// problems whose first workgroup is <= b, minus one (a wave-wide count over
// the descriptors; uniform across the workgroup).  PART selects the launch.
template <int PART>
__device__ __forceinline__ int first_block(const PairDesc &D) {
    return PART == 0 ? D.blk_int : PART == 1 ? D.blk_rec : D.blk_fin;
}
template <int PART>
__device__ __forceinline__ int find_problem(const PairDesc *__restrict__ descs, int count, int b) {
    const int lane = threadIdx.x & 63;
    int n = 0;
    for (int base = 0; base < count; base += 64) {
        const int i = base + lane;
        const bool le = i < count && first_block<PART>(descs[i]) <= b;
        n += __popcll(__ballot(le));
    }
    return n - 1;
}

// ------------------------------------------------------------------ A1: unpack + x-integration
// f_{1,j} + trapezoidal integral of f_x along slice j (Section 3.1).  One wave
// per (field, slice): 64-wide inclusive scans of the trapezoid increments with
// the running total carried from one 64-node segment to the next.
__device__ __forceinline__ void integrate_body(const PairDesc &D, int idx) {
    const int N = D.N, M = D.M;
    const int f = idx / M, j = idx - f * M;  // idx = field * M + slice
    const int lane = threadIdx.x;
    const double *s = D.u + (size_t)f * (N + 1) * M + (size_t)j * (N + 1);
    double *o = D.nodes + ((size_t)f * M + j) * N;
    const double hdx = 0.5 * D.dx;
    double carry = s[0];
    for (int base = 0; base < N; base += 64) {
        const int i = base + lane;
        // increment into node i: (dx/2)(f_x,i-1 + f_x,i), zero for the first node
        double v = (i > 0 && i < N) ? hdx * (s[i] + s[i + 1]) : 0.0;
        for (int o2 = 1; o2 < 64; o2 <<= 1) {
            const double y = __shfl_up(v, o2, 64);
            if (lane >= o2) v += y;
        }
        if (i < N) o[i] = carry + v;
        carry += __shfl(v, 63, 64);
    }
}
__global__ __launch_bounds__(64) void k_integrate(PairDesc D) { integrate_body(D, blockIdx.x); }
__global__ __launch_bounds__(64) void k_integrate_batched(const PairDesc *__restrict__ descs, int count) {
    const PairDesc &D = descs[find_problem<0>(descs, count, blockIdx.x)];
    if (!D.active) return;
    integrate_body(D, blockIdx.x - D.blk_int);
}

// y-derivative of node field g at (j, i): central differences inside, the
// three-point one-sided stencil on the outer edge, zero on the symmetry line of
// a half domain (mirror of the outer stencil on a full domain).
__device__ __forceinline__ double ddy(const double *g, int j, int i, int N, int M, double dy, int half) {
    const double inv2 = 0.5 / dy;
    if (j > 0 && j < M - 1) return (g[(size_t)(j + 1) * N + i] - g[(size_t)(j - 1) * N + i]) * inv2;
    if (j == M - 1)
        return (3.0 * g[(size_t)j * N + i] - 4.0 * g[(size_t)(j - 1) * N + i] + g[(size_t)(j - 2) * N + i]) * inv2;
    if (half) return 0.0;
    return (-3.0 * g[i] + 4.0 * g[(size_t)N + i] - g[(size_t)2 * N + i]) * inv2;
}

// ------------------------------------------------------------------ records
// Node part (one thread per node of the mesh): y-derivatives of zeta and phi,
// and the source-node records of both boundaries.
template <typename T>
__device__ __forceinline__ void node_records(const PairDesc &D, int n) {
    const int N = D.N, M = D.M;
    const int j = n / N, i = n - j * N;
    const double dx = D.dx, dy = D.dy;
    const double *nodes = D.nodes;
    const double *zeta = nodes, *phi = nodes + (size_t)N * M, *psi = nodes + (size_t)2 * N * M;
    const double zy = ddy(zeta, j, i, N, M, dy, D.half);
    const double py = ddy(phi, j, i, N, M, dy, D.half);
    D.ydiv[n] = zy;
    D.ydiv[(size_t)N * M + n] = py;
    const double zx = D.u[(size_t)j * (N + 1) + 1 + i];
    const double x = D.x1 + i * dx;
    const double ci = (i == 0 || i == N - 1) ? 0.5 : 1.0;
    const double cj = (j == 0 || j == M - 1) ? 0.5 : 1.0;
    const double w = dx * dy * ci * cj;
    const bool linear = D.linear;
    // linear mode: the boundaries are the planes z = 0 and z = -1 (Section 4.2);
    // the layer densities are unchanged.
    // FP32 records are in grid units (lengths / dx, node x = its column index):
    // the double-layer and single-layer products are unchanged by the scaling
    // (w / dx^2 times K1 dx^2; w sigma / dx times K2 dx), the S2 sum carries a
    // factor 1 / dx that the all-pairs kernel removes, and s = x - x* is exact.
    const bool grid = sizeof(T) == 4;
    const double g = grid ? 1.0 / dx : 1.0;
    const double xr = grid ? (double)i : x;
    SrcRec<T> a;
    a.x = (T)xr;
    a.z = linear ? (T)0 : (T)(zeta[n] * g);
    a.zx = linear ? (T)0 : (T)zx;
    a.zy = linear ? (T)0 : (T)zy;
    a.wD = (T)(w * g * g * (phi[n] - x));
    a.ws = (T)(w * g * zx);
    a.w = (T)(w * g * g);
    a.pad = (T)0;
    ((SrcRec<T> *)D.srcS)[n] = a;
    // bottom: outward normal points down, so both layers enter with -w
    SrcRec<T> b;
    b.x = (T)xr;
    b.z = (T)((linear ? -1.0 : D.beta[n]) * g);
    b.zx = linear ? (T)0 : (T)D.beta_x[n];
    b.zy = linear ? (T)0 : (T)D.beta_y[n];
    b.wD = (T)(-w * g * g * (psi[n] - x));
    b.ws = (T)(-w * g * D.beta_x[n]);
    b.w = (T)(-w * g * g);
    b.pad = (T)0;
    ((SrcRec<T> *)D.srcB)[n] = b;
}

// Collocation part (one thread per collocation point).  tg layout: 8 arrays of
// 2 ntg entries: x*, y*, d, D*, A, B, C, sigma*; target t = st ntg + l (N-1) + k,
// st = 0 on the free surface, 1 on the bottom.  The FP32 copy tg32 holds the
// first 7 in grid units (x* = k + 1/2, y*, d / dx).  zeta_y at the two
// neighbouring nodes is formed here by the node part's own stencil.
__device__ __forceinline__ void target_records(const PairDesc &D, int t) {
    const int N = D.N, M = D.M;
    const int ntg = (N - 1) * M;
    const int st = t / ntg, r = t - st * ntg;
    const int l = r / (N - 1), k = r - l * (N - 1);
    const size_t n0 = (size_t)l * N + k, n1 = n0 + 1;
    const double dx = D.dx;
    const double xs = D.x1 + (k + 0.5) * dx, ys = D.y1 + l * D.dy;
    double d, Dst, ax, ay, sig;
    if (st == 0) {
        const double *zeta = D.nodes, *phi = D.nodes + (size_t)N * M;
        const double zx0 = D.u[(size_t)l * (N + 1) + 1 + k], zx1 = D.u[(size_t)l * (N + 1) + 2 + k];
        d = 0.5 * (zeta[n0] + zeta[n1]);
        Dst = 0.5 * (phi[n0] + phi[n1]) - xs;
        ax = 0.5 * (zx0 + zx1);
        ay = 0.5 * (ddy(zeta, l, k, N, M, D.dy, D.half) + ddy(zeta, l, k + 1, N, M, D.dy, D.half));
        sig = ax;
    } else {
        const double *psi = D.nodes + (size_t)2 * N * M;
        d = 0.5 * (D.beta[n0] + D.beta[n1]);
        Dst = 0.5 * (psi[n0] + psi[n1]) - xs;
        ax = 0.5 * (D.beta_x[n0] + D.beta_x[n1]);
        ay = 0.5 * (D.beta_y[n0] + D.beta_y[n1]);
        sig = -ax;
    }
    if (D.linear) {  // flat boundaries: elevation 0 or -1, S2 = 1/r
        d = st ? -1.0 : 0.0;
        ax = ay = 0.0;
    }
    const size_t T2 = (size_t)2 * ntg;
    const double v[8] = {xs, ys, d, Dst, 1.0 + ax * ax, 2.0 * ax * ay, 1.0 + ay * ay, sig};
    for (int q = 0; q < 8; ++q) D.tg64[q * T2 + t] = v[q];
    // FP32 copies in the grid units of the FP32 node records (x* = k + 1/2)
    const double g[7] = {0.0, 1.0 / dx, 1.0 / dx, 1.0, 1.0, 1.0, 1.0};
    for (int q = 0; q < 7; ++q) D.tg32[q * T2 + t] = (float)(q == 0 ? k + 0.5 : v[q] * g[q]);
}

// Workgroups [0, node_blocks) cover the nodes, the rest the collocation points.
__host__ __device__ __forceinline__ int node_blocks(int N, int M) { return (N * M + 255) / 256; }
__host__ __device__ __forceinline__ int record_blocks(int N, int M) {
    return node_blocks(N, M) + (2 * (N - 1) * M + 255) / 256;
}
template <typename T>
__device__ __forceinline__ void records_body(const PairDesc &D, int b) {
    const int nbn = node_blocks(D.N, D.M);
    if (b < nbn) {
        const int n = b * 256 + threadIdx.x;
        if (n < D.N * D.M) node_records<T>(D, n);
    } else {
        const int t = (b - nbn) * 256 + threadIdx.x;
        if (t < 2 * (D.N - 1) * D.M) target_records(D, t);
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_records(PairDesc D) { records_body<T>(D, blockIdx.x); }
template <typename T>
__global__ __launch_bounds__(256) void k_records_batched(const PairDesc *__restrict__ descs, int count) {
    const PairDesc &D = descs[find_problem<1>(descs, count, blockIdx.x)];
    if (!D.active) return;  // uniform over the workgroup
    records_body<T>(D, blockIdx.x - D.blk_rec);
}

// ------------------------------------------------------------------ A2: all-pairs sums (hot loop)
// The sums read through address-space qualified pointers.  Per-lane arrays are
// global memory.  Node records are read-only for a whole launch; the batched
// kernel, whose pointers come from a descriptor in memory and so carry no
// address space (flat loads, which count on the same counter as the scalar
// loads and break the record prefetch), reads them through the constant
// address space, where a wave-uniform address gives a scalar load.  The
// single-problem kernel keeps the kernel-argument pointers: the compiler infers
// them as global and keeps several FP64 record loads in flight, which it does
// not do for constant-space loads (measured: 3% on the FP64 sums).
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T *;
template <typename T>
using GlobalPtr = __attribute__((address_space(1))) T *;

// One source record as a single 8-wide vector load (one scalar load per node).
template <typename T>
struct RecVec;
template <>
struct RecVec<float> {
    typedef float type __attribute__((ext_vector_type(8)));
};
template <>
struct RecVec<double> {
    typedef double type __attribute__((ext_vector_type(8)));
};
template <typename T, bool CREC>
struct RecPtrs {  // generic pointers
    typedef const SrcRec<T> *rec;
    typedef const typename RecVec<T>::type *vec;
};
template <typename T>
struct RecPtrs<T, true> {  // constant address space
    typedef ConstPtr<SrcRec<T>> rec;
    typedef ConstPtr<typename RecVec<T>::type> vec;
};
template <typename T, bool CREC>
using RecPtr = typename RecPtrs<T, CREC>::rec;

template <typename T, bool CREC>
__device__ __forceinline__ SrcRec<T> load_rec(RecPtr<T, CREC> p) {
    const typename RecVec<T>::type v = *reinterpret_cast<typename RecPtrs<T, CREC>::vec>(p);
    SrcRec<T> r;
    r.x = v[0];
    r.z = v[1];
    r.zx = v[2];
    r.zy = v[3];
    r.wD = v[4];
    r.ws = v[5];
    r.w = v[6];
    r.pad = v[7];
    return r;
}

// Walk the N source records of one row in groups of UNROLL with the next
// group's scalar loads in flight while the current group is computed.  Scalar
// loads may return out of order, so a wait covers every load issued before
// it: the next group is loaded into separate registers and handed over only
// after the current group's arithmetic, which is where the single wait falls.
// The prefetch reads up to UNROLL records past the end of a row; the record
// arrays carry kRecPad spare records so that this stays inside them (the
// values read there are never used).
// FP64 records (two scalar loads of 16 dwords per pair of records) gain
// nothing from it (measured), so they keep the plain loop.
// body(p, slot) does the first part of record p's work (distances and every
// reciprocal square root) and returns the rest (the accumulations) as a
// closure; a group runs every record's first part before any second part, so
// the independent rsq of the group are issued ahead of their uses (second
// parts in reverse record order).  slot (a compile-time constant: the record's
// position in the group, mod 2) picks one of two FP32 running sums, so that
// each sums half of the row's terms.
// The FP32 walk is one loop: any fold of the running sums inside a row piece
// (a branch per segment, or a loop nest per segment) measured 6 - 12% slower.
template <int U, int K = 0, typename Body, typename Rec>
__device__ __forceinline__ void run_group(Body &body, const Rec *cur) {
    if constexpr (K < U) {
        auto rest = body(cur[K], std::integral_constant<int, K % 2>{});
        run_group<U, K + 1>(body, cur);
        rest();
    }
}
template <typename T, int UNROLL, bool CREC, typename Body>
__device__ __forceinline__ void walk_row(RecPtr<T, CREC> src, int N, Body &&body) {
    static_assert(UNROLL <= kRecPad, "prefetch beyond the record padding");
    if constexpr (sizeof(T) == 8) {
#pragma unroll UNROLL
        for (int i = 0; i < N; ++i) body(load_rec<T, CREC>(src + i), std::integral_constant<int, 0>{})();
        return;
    }
    const int full = N - N % UNROLL;
    SrcRec<T> cur[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) cur[u] = load_rec<T, CREC>(src + u);
    for (int i0 = 0; i0 < full; i0 += UNROLL) {
        SrcRec<T> nxt[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) nxt[u] = load_rec<T, CREC>(src + i0 + UNROLL + u);
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the arithmetic
        run_group<UNROLL>(body, cur);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) cur[u] = nxt[u];
    }
    // the tail indexes cur[] with constants only (a runtime index would put the
    // array in private memory)
#pragma unroll
    for (int u = 0; u < UNROLL - 1; ++u)
        if (u < N - full) body(cur[u], std::integral_constant<int, 0>{})();
}

// One wave = 64 collocation points of one boundary: consecutive entries of
// the list of (row group, x*_k) points of that boundary, where a row group is
// TPL mesh rows handled by the same lane (so rows need not fill whole waves).
// The wave walks a chunk of source rows (boundary, y-row) and, for each, all N
// nodes of that row.  Source records are read with wave-uniform addresses
// (scalar loads) and shared by the TPL targets of a lane; every y-dependent
// term is hoisted per source row.  On a half domain each record serves both
// images (x, y_j) and (x, -y_j), which share s, dz, s^2 + dz^2 and the
// x-part of the double-layer numerator.
// Per pair:
//   own boundary:   w (D - D*) K1 + w sigma K2  and  w S2   (two rsqrt)
//   other boundary: w D K1 + w sigma K2                      (one rsqrt)
// written as  ri (coef num ri^2 + w sigma)  with ri = 1/R.
// FP32C: two FP32 running sums per row piece (alternate nodes), combined across
// pieces with Neumaier's compensated summation; the chunk result is written in
// FP64.
template <typename T, int NI>
struct TargetState {
    double ys;                                   // y* (FP64, physical units)
    T d, Dst, A, B, C;                           // collocation data
    T t[NI], ti[NI], t2[NI], Bt[NI], Ct2[NI];    // per source row and image
    T acc[2], acc2[2];                           // per source row piece (two running sums each)
    T sum, comp, s2sum, s2comp;                  // across rows
};

// Folds the running sums of a row piece into the across-row sums (Neumaier's
// compensated summation in FP32C).  S2: the piece also carries the S2 sum (only
// rows of the target's own boundary).
template <typename T>
__device__ __forceinline__ void neumaier_add(T &sum, T &comp, T x) {
    const T t = sum + x;
    comp += (fabs(sum) >= fabs(x)) ? ((sum - t) + x) : ((x - t) + sum);
    sum = t;
}
template <typename T, bool COMP, int NI, bool S2 = true>
__device__ __forceinline__ void row_end(TargetState<T, NI> &g) {
    if (COMP) {
        neumaier_add(g.sum, g.comp, g.acc[0]);
        neumaier_add(g.sum, g.comp, g.acc[1]);
        if (S2) {
            neumaier_add(g.s2sum, g.s2comp, g.acc2[0]);
            neumaier_add(g.s2sum, g.s2comp, g.acc2[1]);
        }
    } else {  // FP64: one running sum (slot 0)
        g.sum += g.acc[0];
        if (S2) g.s2sum += g.acc2[0];
    }
}

// NI = 2: half domain (both images per source row); NI = 1: full domain.
// FP32 (grid units): t = (y_j - y*) / dx is formed in FP64 for every source row
// and the S2 sum is multiplied by dx on output; FP64 works in physical units.
// LIN: the linearised residual (Section 4.2), whose boundaries are the planes
// z = 0 and z = -1 with zero slopes.  On a record of the target's own plane the
// double-layer numerator is exactly zero, so the general body adds exactly
// w sigma / R, and the S2 radicand is exactly s^2 + t^2; on the other plane the
// numerator is exactly the plane separation.  The LIN bodies drop those zero
// terms and give bit-identical sums.
template <typename T, bool COMP, int TPL, int UNROLL, int NI, bool CREC, bool LIN = false>
__device__ __forceinline__ void pair_item(const SrcRec<T> *__restrict__ srcS, const SrcRec<T> *__restrict__ srcB,
                                          const T *__restrict__ tg, const double *__restrict__ tg64, int N, int M,
                                          double y1, double dx, double dy, int tiles_per_bnd, int row_groups,
                                          int chunks, double *__restrict__ part, int tt, int c, int lane) {
    const RecPtr<T, CREC> recS = (RecPtr<T, CREC>)srcS, recB = (RecPtr<T, CREC>)srcB;
    const GlobalPtr<const T> gtg = (GlobalPtr<const T>)tg;
    const GlobalPtr<const double> gtg64 = (GlobalPtr<const double>)tg64;
    const double gi = (sizeof(T) == 4) ? 1.0 / dx : 1.0;
    const int ntg = (N - 1) * M;
    const size_t T2 = (size_t)2 * ntg;
    const int st = tt / tiles_per_bnd;
    const int npts = row_groups * (N - 1);
    const int idx = (tt - st * tiles_per_bnd) * 64 + lane;
    const bool valid = idx < npts;
    const int ic = valid ? idx : npts - 1;
    const int lg = ic / (N - 1);
    const int k = ic - lg * (N - 1);
    TargetState<T, NI> ts[TPL];
    T xs = 0;
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
        const int l = min(lg * TPL + q, M - 1);
        const int tid = st * ntg + l * (N - 1) + k;
        xs = gtg[0 * T2 + tid];
        ts[q].ys = gtg64[1 * T2 + tid];
        ts[q].d = gtg[2 * T2 + tid];
        ts[q].Dst = gtg[3 * T2 + tid];
        ts[q].A = gtg[4 * T2 + tid];
        ts[q].B = gtg[5 * T2 + tid];
        ts[q].C = gtg[6 * T2 + tid];
        ts[q].sum = ts[q].comp = ts[q].s2sum = ts[q].s2comp = 0;
    }
    // chunk c: nodes [e0, e1) of the 2 M N source nodes in visit order (row r =
    // 2 j + boundary, so that every chunk mixes both boundaries); a chunk may
    // start and end inside a row.
    // (balanced split: the first nsrc % chunks chunks take one node more; 32-bit
    // arithmetic, as 2 M N is far below 2^31 for any mesh that fits the GPU)
    const int nsrc = 2 * M * N;
    const int q = nsrc / chunks, rem = nsrc - q * chunks;
    const int e0 = c * q + min(c, rem), e1 = e0 + q + (c < rem ? 1 : 0);
    for (int r = e0 / N; r * N < e1; ++r) {
        const int i0 = max(e0 - r * N, 0);
        const int i1 = min(e1 - r * N, N);
        const int ss = r & 1;
        const int j = r >> 1;
        const double yj = y1 + j * dy;
#pragma unroll
        for (int q = 0; q < TPL; ++q) {
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                // image i = 1 is (x, -y_j): a_y changes sign, which ti carries
                const T t = (T)((((i == 0) ? yj : -yj) - ts[q].ys) * gi);
                ts[q].t[i] = t;
                ts[q].ti[i] = (i == 0) ? t : -t;
                ts[q].t2[i] = t * t;
                ts[q].Bt[i] = ts[q].B * t;
                ts[q].Ct2[i] = ts[q].C * (t * t);
            }
            ts[q].acc[0] = ts[q].acc[1] = 0;
            ts[q].acc2[0] = ts[q].acc2[1] = 0;
        }
        const RecPtr<T, CREC> src = (ss ? recB : recS) + (size_t)j * N + i0;
        if (LIN && ss == st) {
            walk_row<T, UNROLL, CREC>(src, i1 - i0, [&](const SrcRec<T> &p, auto slot) {
                constexpr int a = decltype(slot)::value;
                const T s = p.x - xs;
                T ri[TPL][NI], rq[TPL][NI];
#pragma unroll
                for (int q = 0; q < TPL; ++q) {
                    const TargetState<T, NI> &e = ts[q];
                    const T dz = p.z - e.d;  // exactly zero: both points lie on one plane
                    const T base = (NI == 2) ? fma(s, s, dz * dz) : fma(s, s, e.t2[0]);
#pragma unroll
                    for (int i = 0; i < NI; ++i) {
                        ri[q][i] = rsq((NI == 2) ? base + e.t2[i] : fma(dz, dz, base));
                        // A = C = 1, B = 0: the S2 radicand is s^2 + t^2, in one rounding
                        rq[q][i] = (NI == 2) ? rsq(fma(s, s, e.t2[i])) : ri[q][i];
                    }
                }
                return [&, p, ri, rq]() {
#pragma unroll
                    for (int q = 0; q < TPL; ++q) {
                        TargetState<T, NI> &e = ts[q];
#pragma unroll
                        for (int i = 0; i < NI; ++i) {
                            e.acc[a] = fma(p.ws, ri[q][i], e.acc[a]);
                            e.acc2[a] = fma(p.w, rq[q][i], e.acc2[a]);
                        }
                    }
                };
            });
        } else if (ss == st) {
            walk_row<T, UNROLL, CREC>(src, i1 - i0, [&](const SrcRec<T> &p, auto slot) {
                constexpr int a = decltype(slot)::value;
                const T s = p.x - xs;
                T nb0[TPL], coef[TPL], ri[TPL][NI], rq[TPL][NI];
#pragma unroll
                for (int q = 0; q < TPL; ++q) {
                    const TargetState<T, NI> &e = ts[q];
                    const T dz = p.z - e.d;
                    const T base = (NI == 2) ? fma(s, s, dz * dz) : fma(s, s, e.t2[0]);
                    nb0[q] = fma(-s, p.zx, dz);
                    coef[q] = fma(-e.Dst, p.w, p.wD);
#pragma unroll
                    for (int i = 0; i < NI; ++i) {
                        ri[q][i] = rsq((NI == 2) ? base + e.t2[i] : fma(dz, dz, base));
                        rq[q][i] = rsq(fma(s, fma(e.A, s, e.Bt[i]), e.Ct2[i]));
                    }
                }
                return [&, p, nb0, coef, ri, rq]() {
#pragma unroll
                    for (int q = 0; q < TPL; ++q) {
                        TargetState<T, NI> &e = ts[q];
#pragma unroll
                        for (int i = 0; i < NI; ++i) {
                            const T num = fma(-e.ti[i], p.zy, nb0[q]);
                            const T bsum = fma(coef[q] * num, ri[q][i] * ri[q][i], p.ws);
                            e.acc[a] = fma(bsum, ri[q][i], e.acc[a]);
                            e.acc2[a] = fma(p.w, rq[q][i], e.acc2[a]);
                        }
                    }
                };
            });
        } else {
            walk_row<T, UNROLL, CREC>(src, i1 - i0, [&](const SrcRec<T> &p, auto slot) {
                constexpr int a = decltype(slot)::value;
                const T s = p.x - xs;
                T nb0[TPL], ri[TPL][NI];
#pragma unroll
                for (int q = 0; q < TPL; ++q) {
                    const TargetState<T, NI> &e = ts[q];
                    const T dz = p.z - e.d;
                    const T base = (NI == 2) ? fma(s, s, dz * dz) : fma(s, s, e.t2[0]);
                    nb0[q] = LIN ? dz : fma(-s, p.zx, dz);
#pragma unroll
                    for (int i = 0; i < NI; ++i) ri[q][i] = rsq((NI == 2) ? base + e.t2[i] : fma(dz, dz, base));
                }
                return [&, p, nb0, ri]() {
#pragma unroll
                    for (int q = 0; q < TPL; ++q) {
                        TargetState<T, NI> &e = ts[q];
#pragma unroll
                        for (int i = 0; i < NI; ++i) {
                            const T num = LIN ? nb0[q] : fma(-e.ti[i], p.zy, nb0[q]);
                            const T bsum = fma(p.wD * num, ri[q][i] * ri[q][i], p.ws);
                            e.acc[a] = fma(bsum, ri[q][i], e.acc[a]);
                        }
                    }
                };
            });
        }
#pragma unroll
        for (int q = 0; q < TPL; ++q) row_end<T, COMP, NI>(ts[q]);
    }
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
        const int l = lg * TPL + q;
        if (valid && l < M) {
            const int tid = st * ntg + l * (N - 1) + k;
            const GlobalPtr<double> o = (GlobalPtr<double>)part + ((size_t)c * T2 + tid) * 2;
            o[0] = (double)ts[q].sum + (double)ts[q].comp;
            o[1] = ((double)ts[q].s2sum + (double)ts[q].s2comp) * ((sizeof(T) == 4) ? dx : 1.0);
        }
    }
}

template <typename T, bool COMP, int TPL, int UNROLL, bool CREC, bool LIN = false>
__device__ __forceinline__ void pair_item_any(const SrcRec<T> *__restrict__ srcS, const SrcRec<T> *__restrict__ srcB,
                                              const T *__restrict__ tg, const double *__restrict__ tg64, int N,
                                              int M, int nimg, double y1, double dx, double dy, int tiles_per_bnd,
                                              int row_groups, int chunks, double *__restrict__ part, int tt,
                                              int c, int lane) {
    if (nimg == 2)
        pair_item<T, COMP, TPL, UNROLL, 2, CREC, LIN>(srcS, srcB, tg, tg64, N, M, y1, dx, dy, tiles_per_bnd,
                                                      row_groups, chunks, part, tt, c, lane);
    else
        pair_item<T, COMP, TPL, UNROLL, 1, CREC, LIN>(srcS, srcB, tg, tg64, N, M, y1, dx, dy, tiles_per_bnd,
                                                      row_groups, chunks, part, tt, c, lane);
}

// Resident waves per SIMD asked of the compiler: 8 for the FP32 variants whose
// registers allow it (the scalar registers of the record prefetch otherwise
// push the count to 7; what the limit moves out of scalar registers is spilled
// to vector lanes outside the inner loops), none (1) for the others.  Not used
// for the batched kernel, whose descriptor values would then be spilled inside
// its inner loops.
template <typename T, int TPL, int UNROLL>
constexpr int kMinWaves = (sizeof(T) == 4 && TPL == 1 && UNROLL <= 4) ? 8 : 1;

// Single problem: one wave per (target tile, source chunk).  LIN: the
// linearised residual (one launch shape per precision).
template <typename T, bool COMP, int TPL, int UNROLL, bool LIN = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMinWaves<T, TPL, UNROLL>))) void k_allpairs(
    const SrcRec<T> *__restrict__ srcS, const SrcRec<T> *__restrict__ srcB, const T *__restrict__ tg,
    const double *__restrict__ tg64, int N, int M, int nimg, double y1, double dx, double dy, int tiles_per_bnd,
    int row_groups, int target_tiles, int chunks, double *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    // the wave index is uniform: keep it (and everything derived) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = blockIdx.x * 4 + wave;
    const int tt = g % target_tiles, c = g / target_tiles;
    if (c >= chunks) return;
    pair_item_any<T, COMP, TPL, UNROLL, false, LIN>(srcS, srcB, tg, tg64, N, M, nimg, y1, dx, dy, tiles_per_bnd,
                                                    row_groups, chunks, part, tt, c, lane);
}

// Many problems in one persistent launch: the work items (target tile, source
// chunk) of all active problems form one list; every wave walks it with a fixed
// stride, so the schedule (and each problem's fixed-order reduction) is
// deterministic.  An inactive problem owns no items (its item0 equals the next
// problem's), so the walk never selects it.
template <typename T, bool COMP, int TPL, int UNROLL>
__global__ __launch_bounds__(256) void k_allpairs_batched(const PairDesc *__restrict__ descs, int count) {
    const long total_items = descs[0].batch_items;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long nwaves = (long)gridDim.x * 4;
    int inst = 0;
    for (long item = (long)blockIdx.x * 4 + wave; item < total_items; item += nwaves) {
        while (inst + 1 < count && descs[inst + 1].item0 <= item) ++inst;  // items grow monotonically
        const PairDesc &D = descs[inst];
        const int local = (int)(item - D.item0);
        const int tt = local % D.target_tiles, c = local / D.target_tiles;
        pair_item_any<T, COMP, TPL, UNROLL, true>((const SrcRec<T> *)D.srcS, (const SrcRec<T> *)D.srcB,
                                            (const T *)D.tg, D.tg64, D.N, D.M, D.nimg, D.y1, D.dx, D.dy,
                                            D.tiles_per_bnd, D.row_groups, D.chunks, D.part, tt, c, lane);
    }
}

// ------------------------------------------------------------------ A3 + A4: finalize
// Closed form of the integral of (A s^2 + B s t + C t^2)^(-1/2) over a rectangle
// from the antiderivative of Section 3.1; a term with a zero prefactor is its
// limit, zero.
__device__ double s2_antideriv(double A, double B, double C, double s, double t) {
    const double Q = A * s * s + B * s * t + C * t * t;
    double g = 0.0;
    if (t != 0.0) g += t / sqrt(A) * log(2.0 * A * s + B * t + 2.0 * sqrt(A * Q));
    if (s != 0.0) g += s / sqrt(C) * log(2.0 * C * t + B * s + 2.0 * sqrt(C * Q));
    return g;
}

// Workgroups [0, bie_blocks) hold 64 boundary-integral rows each (4 waves: wave
// w sums a quarter of the source chunks' partial sums and the w-th corner term
// of the closed-form S2 integral; wave 0 combines them in a fixed order), the
// rest one dynamic or radiation row per thread.
__host__ __device__ __forceinline__ int bie_blocks(int N, int M) { return (2 * (N - 1) * M + 63) / 64; }
__host__ __device__ __forceinline__ int finalize_blocks(int N, int M) {
    return bie_blocks(N, M) + ((N + 1) * M + 4 * M + 255) / 256;
}

__device__ __forceinline__ void finalize_bie(const PairDesc &D, int b, double (*red)[3][64]) {
    const int N = D.N, M = D.M;
    const int ntg = (N - 1) * M;
    const size_t T2 = (size_t)2 * ntg;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tid = b * 64 + lane;
    const bool valid = tid < 2 * ntg;
    const int t = valid ? tid : 2 * ntg - 1;
    // partial sums of chunks [c0, c1), in chunk order, eight loads in flight
    const int chunks = D.chunks;
    const int c0 = (w * chunks) >> 2, c1 = ((w + 1) * chunks) >> 2;
    const double2 *pp = (const double2 *)D.part + t;
    double acc = 0.0, acc2 = 0.0;
    int c = c0;
    for (; c + 8 <= c1; c += 8) {
        double2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = pp[(size_t)(c + q) * T2];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            acc += v[q].x;
            acc2 += v[q].y;
        }
    }
    for (; c < c1; ++c) {
        const double2 v = pp[(size_t)c * T2];
        acc += v.x;
        acc2 += v.y;
    }
    // corner w of the rectangle [x_1, x_N] x [y_lo, y_M] relative to the target,
    // from mesh indices: the offset to an edge through the target is exactly zero
    // (y_lo = -y_M on a half domain, where y_1 = 0; y_1 on a full one)
    const double *tg = D.tg64;
    const double A = tg[4 * T2 + t], B = tg[5 * T2 + t], C = tg[6 * T2 + t];
    const int tl = (t % ntg) / (N - 1), tk = (t % ntg) - tl * (N - 1);
    const double sc = (w & 1) ? -(tk + 0.5) * D.dx : (N - 1.5 - tk) * D.dx;
    const double tc = (w & 2) ? (D.half ? -(double)(M - 1 + tl) * D.dy : -(double)tl * D.dy)
                              : (double)(M - 1 - tl) * D.dy;
    const double corner = s2_antideriv(A, B, C, sc, tc);
    if (w > 0) {
        red[w - 1][0][lane] = acc;
        red[w - 1][1][lane] = acc2;
        red[w - 1][2][lane] = corner;
    }
    __syncthreads();
    if (w > 0 || !valid) return;
    acc = ((acc + red[0][0][lane]) + red[1][0][lane]) + red[2][0][lane];
    acc2 = ((acc2 + red[0][1][lane]) + red[1][1][lane]) + red[2][1][lane];
    // corners in the order (xhi, yhi) - (xlo, yhi) - (xhi, ylo) + (xlo, ylo)
    const double I2 = ((corner - red[0][2][lane]) - red[1][2][lane]) + red[2][2][lane];
    const int st = t / ntg, r = t - st * ntg;
    const int l = r / (N - 1), k = r - l * (N - 1);
    const int row = (st + 1) * (N + 1) * M + l * (N + 1) + k + 2;
    const double s2 = st ? -acc2 : acc2;  // bottom records carry -w
    const double Dst = tg[3 * T2 + t], sig = tg[7 * T2 + t];
    D.F[row] = acc - sig * s2 + sig * I2 - kTwoPi * Dst;
}

// Dynamic rows (block 0, columns >= 2) and radiation rows (columns 0, 1 of the
// three blocks); r enumerates block 0 and then the radiation pairs of blocks 1, 2.
// Second y-difference of the node field g (zeta: block 0 of the node array) at
// (l, i): central inside; on the symmetry line of a half domain the mirror node
// stands for row -1; one-sided four-point stencils on an outer edge (M >= 4).
__device__ __forceinline__ double y_second_diff(const double *g, int l, int i, int N, int M, double dy, int half) {
    const double c = 1.0 / (dy * dy);
    auto at = [&](int j) { return g[(size_t)j * N + i]; };
    if (l > 0 && l < M - 1) return c * (at(l + 1) - 2.0 * at(l) + at(l - 1));
    if (l == M - 1) return c * (2.0 * at(M - 1) - 5.0 * at(M - 2) + 4.0 * at(M - 3) - at(M - 4));
    return half ? c * 2.0 * (at(1) - at(0)) : c * (2.0 * at(0) - 5.0 * at(1) + 4.0 * at(2) - at(3));
}

__device__ __forceinline__ void finalize_rows(const PairDesc &D, int r) {
    const int N = D.N, M = D.M;
    const int nblk = (N + 1) * M;
    if (r >= nblk + 4 * M) return;
    int blk, l, col;
    if (r < nblk) {
        blk = 0;
        l = r / (N + 1);
        col = r - l * (N + 1);
    } else {
        const int q = r - nblk;
        blk = 1 + q / (2 * M);
        const int e = q - (blk - 1) * 2 * M;
        l = e >> 1;
        col = e & 1;
    }
    const int row = blk * nblk + l * (N + 1) + col;
    const double dx = D.dx, x1 = D.x1;
    const double *u = D.u, *nodes = D.nodes, *ydiv = D.ydiv;
    const double *fx = u + (size_t)blk * nblk + (size_t)l * (N + 1) + 1;  // (f_x)_{., l}
    const double *fv = nodes + ((size_t)blk * M + l) * N;                  // f_{., l}
    if (col < 2) {
        // radiation rows (eqs. scullen1-6 as discretised in Appendix B)
        const double fxx = (fx[1] - fx[0]) / dx;
        const double n_decay = D.n_decay;
        double v;
        if (blk == 0) {
            v = (col == 0) ? x1 * fx[0] + n_decay * fv[0] : x1 * fxx + n_decay * fx[0];
        } else {
            v = (col == 0) ? x1 * (fx[0] - 1.0) + n_decay * (fv[0] - x1) : x1 * fxx + n_decay * (fx[0] - 1.0);
        }
        D.F[row] = v;
        return;
    }
    // dynamic condition, eq. (new_finite_dynamic), at (x_{k+1/2}, y_l)
    const int k = col - 2;
    const size_t n0 = (size_t)l * N + k, n1 = n0 + 1;
    const double *zx = u + (size_t)l * (N + 1) + 1;
    const double *px = u + (size_t)nblk + (size_t)l * (N + 1) + 1;
    const double z = 0.5 * (nodes[n0] + nodes[n1]);
    const double a = 0.5 * (zx[k] + zx[k + 1]);
    const double b = 0.5 * (ydiv[n0] + ydiv[n1]);
    const double p = 0.5 * (px[k] + px[k + 1]);
    const double q = 0.5 * (ydiv[(size_t)N * M + n0] + ydiv[(size_t)N * M + n1]);
    const double kin = 0.5 * ((1.0 + a * a) * q * q + (1.0 + b * b) * p * p - 2.0 * a * b * p * q) /
                       (1.0 + a * a + b * b);
    const double fr2 = D.froude * D.froude;
    // linear mode: eq. (linear_dynamic2), phi*_x + zeta*/F^2 - 1
    double f1 = D.linear ? p + z / fr2 - 1.0 : kin + z / fr2 - 0.5;
    if (D.tau != 0.0) {
        // surface tension (Section 6): -tau K, K = div(grad zeta / |(1, grad zeta)|) from the
        // half-mesh slopes, the cell differences of zeta_x and zeta_y and the mean of the
        // node second y-differences; linear mode: -tau (zeta_xx + zeta_yy)
        const double zxx = (zx[k + 1] - zx[k]) / dx;
        const double zyy = 0.5 * (y_second_diff(nodes, l, k, N, M, D.dy, D.half) +
                                  y_second_diff(nodes, l, k + 1, N, M, D.dy, D.half));
        if (D.linear) {
            f1 -= D.tau * (zxx + zyy);
        } else {
            const double zxy = (ydiv[n1] - ydiv[n0]) / dx;
            const double qq = 1.0 + a * a + b * b;
            f1 -= D.tau * ((1.0 + b * b) * zxx - 2.0 * a * b * zxy + (1.0 + a * a) * zyy) / (qq * sqrt(qq));
        }
    }
    D.F[row] = f1;
}

__device__ __forceinline__ void finalize_body(const PairDesc &D, int b) {
    __shared__ double red[3][3][64];
    const int nb = bie_blocks(D.N, D.M);
    if (b < nb) finalize_bie(D, b, red);
    else finalize_rows(D, (b - nb) * 256 + threadIdx.x);
}
__global__ __launch_bounds__(256) void k_finalize(PairDesc D) { finalize_body(D, blockIdx.x); }
__global__ __launch_bounds__(256) void k_finalize_batched(const PairDesc *__restrict__ descs, int count) {
    const PairDesc &D = descs[find_problem<2>(descs, count, blockIdx.x)];
    if (!D.active) return;  // uniform over the workgroup
    finalize_body(D, blockIdx.x - D.blk_fin);
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace


size_t residual_work_bytes(const Dims &d, const PairLaunch &pl) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t b = 0;
    b += al(sizeof(double) * 3 * d.nnode);
    b += al(sizeof(double) * 2 * d.nnode);
    b += al(sizeof(double) * 8 * 2 * d.ntg);
    b += al(sizeof(float) * 7 * 2 * d.ntg);
    b += 2 * al(sizeof(SrcRec<double>) * (d.nnode + kRecPad));
    b += al(sizeof(double) * 2 * 2 * (size_t)d.ntg * pl.chunks);
    b += al(sizeof(double) * 4);
    return b;
}

void residual_work_carve(void *base, const Dims &d, const PairLaunch &pl, ResidualWork *w) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = (char *)base;
    w->nodes = (double *)p; p += al(sizeof(double) * 3 * d.nnode);
    w->ydiv = (double *)p; p += al(sizeof(double) * 2 * d.nnode);
    w->tg = (double *)p; p += al(sizeof(double) * 8 * 2 * d.ntg);
    w->tg32 = (float *)p; p += al(sizeof(float) * 7 * 2 * d.ntg);
    w->srcS = p; p += al(sizeof(SrcRec<double>) * (d.nnode + kRecPad));
    w->srcB = p; p += al(sizeof(SrcRec<double>) * (d.nnode + kRecPad));
    w->part = (double *)p; p += al(sizeof(double) * 2 * 2 * (size_t)d.ntg * pl.chunks);
    w->scal = (double *)p; p += al(sizeof(double) * 4);
    w->bytes = (size_t)(p - (char *)base);
}

namespace {

PairDesc make_desc(const bim_problem *p, const Dims &d, const PairLaunch &pl, const ResidualWork &w,
                   const double *u, double *F, int prec, int linear) {
    PairDesc D{};
    D.srcS = w.srcS;
    D.srcB = w.srcB;
    D.tg = (prec == BIM_FP64) ? (const void *)w.tg : (const void *)w.tg32;
    D.tg64 = w.tg;
    D.part = w.part;
    D.N = d.N;
    D.M = d.M;
    D.nimg = d.nimg;
    D.y1 = p->y1;
    D.dx = p->dx;
    D.dy = p->dy;
    D.tiles_per_bnd = pl.tiles_per_bnd;
    D.row_groups = pl.row_groups;
    D.target_tiles = pl.target_tiles;
    D.chunks = pl.chunks;
    D.item0 = 0;
    D.batch_items = 0;
    D.active = 1;
    D.u = u;
    D.F = F;
    D.nodes = w.nodes;
    D.ydiv = w.ydiv;
    D.tg32 = w.tg32;
    D.beta = p->beta;
    D.beta_x = p->beta_x;
    D.beta_y = p->beta_y;
    D.x1 = p->x1;
    D.n_decay = p->n_decay;
    D.froude = p->froude;
    D.tau = p->tau;
    D.half = p->half_domain ? 1 : 0;
    D.linear = linear;
    return D;
}

}  // namespace

int residual_enqueue(const bim_problem *p, const double *u, double *F, int prec, const PairLaunch &pl,
                     const ResidualWork &w, hipStream_t s, hipEvent_t *ev_pair, int linear) {
    const Dims d(p);
    const int N = d.N, M = d.M;
    const PairDesc D = make_desc(p, d, pl, w, u, F, prec, linear);
    hipLaunchKernelGGL(k_integrate, dim3(3 * M), dim3(64), 0, s, D);
    if (prec == BIM_FP64)
        hipLaunchKernelGGL(k_records<double>, dim3(record_blocks(N, M)), dim3(256), 0, s, D);
    else
        hipLaunchKernelGGL(k_records<float>, dim3(record_blocks(N, M)), dim3(256), 0, s, D);
    if (ev_pair) BIM_HIP(hipEventRecord(ev_pair[0], s));
#define BIM_LAUNCH_PAIRS(T, COMP, TPL, UNR, TG)                                                         \
    hipLaunchKernelGGL((k_allpairs<T, COMP, TPL, UNR>), dim3(pl.blocks), dim3(256), 0, s,               \
                       (const SrcRec<T> *)w.srcS, (const SrcRec<T> *)w.srcB, TG, w.tg, N, M, d.nimg,    \
                       p->y1, p->dx, p->dy, pl.tiles_per_bnd, pl.row_groups, pl.target_tiles, pl.chunks, \
                       w.part)
    const int vsel = (pl.tpl == 2 ? 3 : 0) + (pl.unroll == 2 ? 0 : pl.unroll == 4 ? 1 : 2);
    if (linear) {
        // the same source chunks (the partial-sum buffer and the finalize use
        // pl.chunks), one target row per lane and the default unroll
        const PairLaunch ll = pair_launch(d, 1, prec == BIM_FP64 ? 4 : 2, pl.chunks);
        if (prec == BIM_FP64)
            hipLaunchKernelGGL((k_allpairs<double, false, 1, 4, true>), dim3(ll.blocks), dim3(256), 0, s,
                               (const SrcRec<double> *)w.srcS, (const SrcRec<double> *)w.srcB, w.tg, w.tg, N, M,
                               d.nimg, p->y1, p->dx, p->dy, ll.tiles_per_bnd, ll.row_groups, ll.target_tiles,
                               ll.chunks, w.part);
        else
            hipLaunchKernelGGL((k_allpairs<float, true, 1, 2, true>), dim3(ll.blocks), dim3(256), 0, s,
                               (const SrcRec<float> *)w.srcS, (const SrcRec<float> *)w.srcB, w.tg32, w.tg, N, M,
                               d.nimg, p->y1, p->dx, p->dy, ll.tiles_per_bnd, ll.row_groups, ll.target_tiles,
                               ll.chunks, w.part);
    } else if (prec == BIM_FP64) {
        switch (vsel) {
            case 0: BIM_LAUNCH_PAIRS(double, false, 1, 2, w.tg); break;
            case 1: BIM_LAUNCH_PAIRS(double, false, 1, 4, w.tg); break;
            case 2: BIM_LAUNCH_PAIRS(double, false, 1, 8, w.tg); break;
            case 3: BIM_LAUNCH_PAIRS(double, false, 2, 2, w.tg); break;
            case 4: BIM_LAUNCH_PAIRS(double, false, 2, 4, w.tg); break;
            default: BIM_LAUNCH_PAIRS(double, false, 2, 8, w.tg); break;
        }
    } else {
        switch (vsel) {
            case 0: BIM_LAUNCH_PAIRS(float, true, 1, 2, w.tg32); break;
            case 1: BIM_LAUNCH_PAIRS(float, true, 1, 4, w.tg32); break;
            case 2: BIM_LAUNCH_PAIRS(float, true, 1, 8, w.tg32); break;
            case 3: BIM_LAUNCH_PAIRS(float, true, 2, 2, w.tg32); break;
            case 4: BIM_LAUNCH_PAIRS(float, true, 2, 4, w.tg32); break;
            default: BIM_LAUNCH_PAIRS(float, true, 2, 8, w.tg32); break;
        }
    }
#undef BIM_LAUNCH_PAIRS
    if (ev_pair) BIM_HIP(hipEventRecord(ev_pair[1], s));
    hipLaunchKernelGGL(k_finalize, dim3(finalize_blocks(N, M)), dim3(256), 0, s, D);
    return hip_check(hipGetLastError(), "residual kernel launch");
}


BatchShape residual_batched_shape(const bim_problem *probs, int count, const PairLaunch *pls, int max_blocks) {
    BatchShape sh{pls[0].tpl, pls[0].unroll, 0, 0, 0, 1};
    long total = 0;
    for (int i = 0; i < count; ++i) {
        const Dims d(&probs[i]);
        sh.b_int += 3 * d.M;
        sh.b_rec += record_blocks(d.N, d.M);
        sh.b_fin += finalize_blocks(d.N, d.M);
        total += (long)pls[i].target_tiles * pls[i].chunks;
    }
    const long want = (total + 3) / 4;
    sh.blocks = (int)std::max(1L, std::min(want, (long)(max_blocks > 0 ? max_blocks : 2048)));
    return sh;
}

int residual_batched_fill(const bim_problem *probs, int count, const int *active, const double *const *u,
                          double *const *F, int prec, const PairLaunch *pls, const ResidualWork *ws,
                          PairDesc *descs, long *total_items) {
    const int tpl = pls[0].tpl, unroll = pls[0].unroll;
    long total = 0;
    int b_int = 0, b_rec = 0, b_fin = 0;
    for (int i = 0; i < count; ++i) {
        const bim_problem *p = &probs[i];
        const Dims d(p);
        const PairLaunch &pl = pls[i];
        if (pl.tpl != tpl || pl.unroll != unroll) return fail(BIM_EINVAL, "batched launch needs one kernel variant");
        const int on = active ? active[i] : 1;
        if (on && (!u[i] || !F[i])) return fail(BIM_EINVAL, "an active problem needs u and F");
        PairDesc &D = descs[i];
        D = make_desc(p, d, pl, ws[i], on ? u[i] : nullptr, on ? F[i] : nullptr, prec, 0);
        D.active = on;
        D.item0 = total;
        if (on) total += (long)pl.target_tiles * pl.chunks;
        D.blk_int = b_int;
        D.blk_rec = b_rec;
        D.blk_fin = b_fin;
        b_int += 3 * d.M;
        b_rec += record_blocks(d.N, d.M);
        b_fin += finalize_blocks(d.N, d.M);
    }
    for (int i = 0; i < count; ++i) descs[i].batch_items = total;
    *total_items = total;
    return BIM_OK;
}

int residual_batched_launch(const PairDesc *descs_dev, int count, int prec, const BatchShape &sh, hipStream_t s,
                            hipEvent_t *ev_pair) {
    if (count <= 0) return BIM_OK;
    hipLaunchKernelGGL(k_integrate_batched, dim3(sh.b_int), dim3(64), 0, s, descs_dev, count);
    if (prec == BIM_FP64)
        hipLaunchKernelGGL(k_records_batched<double>, dim3(sh.b_rec), dim3(256), 0, s, descs_dev, count);
    else
        hipLaunchKernelGGL(k_records_batched<float>, dim3(sh.b_rec), dim3(256), 0, s, descs_dev, count);
    if (ev_pair) BIM_HIP(hipEventRecord(ev_pair[0], s));
#define BIM_LAUNCH_BATCH(T, COMP, TPL, UNR) \
    hipLaunchKernelGGL((k_allpairs_batched<T, COMP, TPL, UNR>), dim3(sh.blocks), dim3(256), 0, s, descs_dev, count)
    const int vsel = (sh.tpl == 2 ? 3 : 0) + (sh.unroll == 2 ? 0 : sh.unroll == 4 ? 1 : 2);
    if (prec == BIM_FP64) {
        switch (vsel) {
            case 0: BIM_LAUNCH_BATCH(double, false, 1, 2); break;
            case 1: BIM_LAUNCH_BATCH(double, false, 1, 4); break;
            case 2: BIM_LAUNCH_BATCH(double, false, 1, 8); break;
            case 3: BIM_LAUNCH_BATCH(double, false, 2, 2); break;
            case 4: BIM_LAUNCH_BATCH(double, false, 2, 4); break;
            default: BIM_LAUNCH_BATCH(double, false, 2, 8); break;
        }
    } else {
        switch (vsel) {
            case 0: BIM_LAUNCH_BATCH(float, true, 1, 2); break;
            case 1: BIM_LAUNCH_BATCH(float, true, 1, 4); break;
            case 2: BIM_LAUNCH_BATCH(float, true, 1, 8); break;
            case 3: BIM_LAUNCH_BATCH(float, true, 2, 2); break;
            case 4: BIM_LAUNCH_BATCH(float, true, 2, 4); break;
            default: BIM_LAUNCH_BATCH(float, true, 2, 8); break;
        }
    }
#undef BIM_LAUNCH_BATCH
    if (ev_pair) BIM_HIP(hipEventRecord(ev_pair[1], s));
    hipLaunchKernelGGL(k_finalize_batched, dim3(sh.b_fin), dim3(256), 0, s, descs_dev, count);
    return hip_check(hipGetLastError(), "batched residual launch");
}

int residual_batched_enqueue(const bim_problem *probs, int count, const double *const *u, double *const *F,
                             int prec, const PairLaunch *pls, const ResidualWork *ws, PairDesc *descs_dev,
                             int max_blocks, hipStream_t s, hipEvent_t *ev_pair) {
    if (count <= 0) return BIM_OK;
    std::vector<PairDesc> descs(count);
    long total = 0;
    int rc = residual_batched_fill(probs, count, nullptr, u, F, prec, pls, ws, descs.data(), &total);
    if (rc) return rc;
    BIM_HIP(hipMemcpyAsync(descs_dev, descs.data(), sizeof(PairDesc) * count, hipMemcpyHostToDevice, s));
    return residual_batched_launch(descs_dev, count, prec, residual_batched_shape(probs, count, pls, max_blocks), s,
                                   ev_pair);
}

}  // namespace bim
