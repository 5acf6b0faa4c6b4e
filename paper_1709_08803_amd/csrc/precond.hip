// Block-banded preconditioner P (Section 4.2 and Appendix A) on gfx950.
//
// P is the Jacobian J~ of the linearised discrete system (Appendix B) with its
// four dense blocks (2,1), (2,3), (3,1), (3,2) kept only for slice pairs
// |m - l| <= h (slice-block band).  With the unknowns and rows grouped in three
// blocks of n = (N+1) M (zeta | phi | psi; F1 | F2 | F7) and each block in M
// slices of s = N+1:
//      [ P11 P12  0  ]   P11, P12, P22 = P33: the same s x s block on every slice
//  P = [ P21 P22 P23 ]   P21, P23 = P32, P31: slice-block-banded, half-width h
//      [ P31 P32 P33 ]
// The paper factors P as a 3 x 3 block LU in the order 1, 2, 3, which leaves
// two dense n x n factor blocks (L32, U33).  Here the block-diagonal blocks
// 1 and 3 are eliminated first:
//      E = P11^-1 P12,  G = P33^-1 (P32 - P31 E)                 (band h)
//      S = P22 - P21 E - P23 G                                    (band 2h)
// so that P z = r is solved exactly by
//      a1 = P11^-1 r1,  a3 = P33^-1 (r3 - P31 a1)
//      z2 = S^-1 (r2 - P21 a1 - P23 a3),  z3 = a3 - G z2,  z1 = a1 - E z2.
// S is factored by a block LU without inter-block pivoting (its diagonal
// blocks are inverted with partial pivoting), S = L D V with L, V unit block-
// triangular and D the pivot blocks, and its inverse is kept explicitly as
// V^-1 D^-1 L^-1: the two triangular inverses in one dense n x n array, D^-1 in
// a block-diagonal one.  The apply is then two triangular GEMVs (together one
// pass over the array), a block-diagonal product and banded products, all
// bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "bim_common.h"
#include "dense.h"
#include "precond.h"

namespace bim {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// Coefficient of dx (f_x)_i in the trapezoidal node value f_k (0-based).
__device__ __forceinline__ double trap(int k, int i) {
    if (k == 0 || i > k) return 0.0;
    if (i == 0 || i == k) return 0.5;
    return 1.0;
}
// Coefficient of dx (f_x)_i in the half-mesh value f*_k = (f_k + f_{k+1}) / 2.
__device__ __forceinline__ double tau(int k, int i) { return 0.5 * (trap(k, i) + trap(k + 1, i)); }

// The three slice-diagonal blocks (identical on every slice):
//   D11: F5, F6, F1 on zeta;  D12: F1 on phi;  D22 (= D33): F3, F4, F2 on phi.
__global__ void k_diag_blocks(double *D11, double *D12, double *D22, int N, double x1, double dx, double n_decay,
                              double froude) {
    const int s = N + 1;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)s * s) return;
    const int r = (int)(e / s), c = (int)(e % s);
    double d11 = 0.0, d12 = 0.0, d22 = 0.0;
    if (r == 0) {  // F5 / F3: x1 f_x,1 + n f_1
        if (c == 0) d11 = d22 = n_decay;
        if (c == 1) d11 = d22 = x1;
    } else if (r == 1) {  // F6 / F4: (x1/dx) f_x,2 + (n - x1/dx) f_x,1
        if (c == 1) d11 = d22 = n_decay - x1 / dx;
        if (c == 2) d11 = d22 = x1 / dx;
    } else {
        const int k = r - 2;
        const double pt = (c == 0) ? 1.0 : dx * tau(k, c - 1);  // d f*_k / d u-slice
        // With surface tension the block stays that of the problem without it: the
        // in-slice -tau zeta*_xx would turn this lower-triangular block into a
        // recurrence with a growing (upstream capillary) mode, whose inverse -- which
        // the elimination below starts from -- overflows.  The Krylov solver takes
        // the whole tension term.
        d11 = pt / (froude * froude);
        d22 = -kTwoPi * pt;
        if (c == 1 + k || c == 2 + k) d12 = 0.5;
    }
    D11[e] = d11;
    D12[e] = d12;
    D22[e] = d22;
}

// Per collocation point (k, l): sum over every node and image of w K5, and the
// exact integral of K5 over the truncated (mirrored) rectangle.  The corners'
// offsets from the point are formed from mesh indices, so the offset to an edge
// through the point is exactly zero (its antiderivative term is then dropped);
// a difference of separately rounded coordinates can leave a few ulp there, and
// the logarithm of the near-zero argument that goes with it is not finite.
__global__ __launch_bounds__(64) void k_k5_rowsum(double *rowsum, double *I5, int N, int M, double x1, double dx,
                                                  double y1, double dy, int nimg) {
    const int t = blockIdx.x;  // l (N-1) + k
    const int l = t / (N - 1), k = t - l * (N - 1);
    const int lane = threadIdx.x;
    const double xs = x1 + (k + 0.5) * dx, ys = y1 + l * dy;
    double v = 0.0;
    for (int img = 0; img < nimg; ++img) {
        const double iota = img ? -1.0 : 1.0;
        for (int n = lane; n < N * M; n += 64) {
            const int m = n / N, i = n - m * N;
            const double ci = (i == 0 || i == N - 1) ? 0.5 : 1.0, cm = (m == 0 || m == M - 1) ? 0.5 : 1.0;
            const double s = x1 + i * dx - xs, tt = iota * (y1 + m * dy) - ys;
            v += dx * dy * ci * cm / sqrt(s * s + tt * tt);
        }
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) {
        rowsum[t] = v;
        auto G = [](double s, double tt) {
            double g = 0.0;
            const double q = sqrt(s * s + tt * tt);
            if (tt != 0.0) g += tt * log(2.0 * s + 2.0 * q);
            if (s != 0.0) g += s * log(2.0 * tt + 2.0 * q);
            return g;
        };
        // rectangle [x_1, x_N] x [y_lo, y_M], y_lo = -y_M on a half domain (y_1 = 0), else y_1
        const double s1 = -(k + 0.5) * dx, s2 = (N - 1.5 - k) * dx;
        const double t1 = (nimg == 2) ? -(double)(M - 1 + l) * dy : -(double)l * dy;
        const double t2 = (double)(M - 1 - l) * dy;
        I5[t] = G(s2, t2) - G(s1, t2) - G(s2, t1) + G(s1, t1);
    }
}

// Band blocks of P21 (K5 on zeta_x, with the singular subtraction on slice l),
// P31 (K7 on zeta_x) and P23 = P32 (K6 on the node values of a potential).
// One wave per (l, band offset, k) row; zero rows 0, 1 (radiation) are left
// from the initial clear.
__global__ __launch_bounds__(64) void k_band_rows(double *B21, double *B23, double *B31, const double *rowsum,
                                                  const double *I5, int N, int M, int h, double x1, double dx,
                                                  double y1, double dy, int nimg) {
    const int s = N + 1;
    const int idx = blockIdx.x;  // (l (2h+1) + off) (N-1) + k
    const int k = idx % (N - 1);
    const int lo = idx / (N - 1);
    const int off = lo % (2 * h + 1), l = lo / (2 * h + 1);
    const int m = l + off - h;
    if (m < 0 || m >= M) return;
    const int lane = threadIdx.x;
    const size_t blk = ((size_t)l * (2 * h + 1) + off) * s * s;
    double *r21 = B21 + blk + (size_t)(2 + k) * s;
    double *r23 = B23 + blk + (size_t)(2 + k) * s;
    double *r31 = B31 + blk + (size_t)(2 + k) * s;
    const double xs = x1 + (k + 0.5) * dx, ys = y1 + l * dy;
    const double cm = (m == 0 || m == M - 1) ? 0.5 : 1.0;
    // singular subtraction of the K5 row sum on the target's own slice (d/d zeta*_x)
    const double corr = (m == l) ? 0.5 * (rowsum[l * (N - 1) + k] - I5[l * (N - 1) + k]) : 0.0;
    // suffix sums of w K6 from the right end of the slice
    double carry = 0.0;
    const int nseg = (N + 63) / 64;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int i = seg * 64 + lane;
        double k5 = 0.0, k6 = 0.0, k7 = 0.0;
        if (i < N) {
            const double ci = (i == 0 || i == N - 1) ? 0.5 : 1.0;
            const double w = dx * dy * ci * cm;
            const double sx = x1 + i * dx - xs;
            for (int img = 0; img < nimg; ++img) {
                const double tt = (img ? -1.0 : 1.0) * (y1 + m * dy) - ys;
                const double r2 = sx * sx + tt * tt;
                k5 += w / sqrt(r2);
                const double q = 1.0 / sqrt(r2 + 1.0);
                k7 += w * q;
                k6 += w * q * q * q;
            }
            r21[1 + i] = k5 - ((i == k || i == k + 1) ? corr : 0.0);
            r31[1 + i] = k7;
        }
        // inclusive suffix scan of k6 within the segment (lane i gets sum over lanes >= i)
        double v = k6;
        for (int o = 1; o < 64; o <<= 1) {
            const double y = __shfl_down(v, o, 64);
            if (lane + o < 64) v += y;
        }
        const double strict_after = v - k6 + carry;  // sum over nodes > i
        if (i < N && i >= 1) r23[1 + i] = dx * (0.5 * k6 + strict_after);
        if (i == 0) {
            // column of f_1: sum of all; column of (f_x)_1: dx/2 sum over i >= 1
            const double total = v + carry;
            r23[0] = total;
            r23[1] = 0.5 * dx * (total - k6);
        }
        carry += __shfl(v, 0, 64);
    }
}

// Replicate one s x s block into every diagonal slot of a band-0 array.
__global__ void k_replicate(const double *src, double *dst, int M, long ss) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)M * ss) return;
    dst[e] = src[e % ss];
}

}  // namespace

// ------------------------------------------------------------------ host orchestration
struct DevArena {
    char *base = nullptr;
    size_t used = 0, cap = 0;
    template <typename T>
    T *take(size_t count) {
        size_t bytes = (sizeof(T) * count + 255) & ~(size_t)255;
        T *p = (T *)(base + used);
        used += bytes;
        return p;
    }
};

static size_t band_elems(int M, int w, int s) { return (size_t)M * (2 * w + 1) * s * s; }

static double *band_blk(double *band, int w, int s, int l, int m) {
    return band + ((size_t)l * (2 * w + 1) + (m - l + w)) * s * s;
}

// FP32 storage: the nine arrays the apply reads are rounded into a new, half-
// sized allocation (with the apply scratch), and the FP64 allocation is freed.
// In two parts: the allocation (pc->f32 then points into it; FP64 untouched),
// and the rounding of the FP64 arrays (all nine, or all but S^-1 when that was
// formed in FP32 already), after which the FP32 allocation is adopted.
struct Fp32Mem {
    void *mem = nullptr;
    size_t bytes = 0;
    double *scratch = nullptr;
};

static const int kNumArrays = 9;

static void precond_counts(const Precond *pc, size_t cnt[kNumArrays]) {
    const int M = pc->M, s = pc->s, h = pc->h;
    const size_t b0 = band_elems(M, 0, s), bh = band_elems(M, h, s);
    const size_t c[kNumArrays] = {b0, b0, b0, bh, bh, bh, bh, (size_t)pc->n * pc->n, b0};
    for (int q = 0; q < kNumArrays; ++q) cnt[q] = c[q];
}

static int precond_fp32_alloc(Precond *pc, Fp32Mem *f) {
    size_t cnt[kNumArrays];
    precond_counts(pc, cnt);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t bytes = 0;
    for (size_t c : cnt) bytes += al(sizeof(float) * c);
    bytes += al(sizeof(double) * 4 * pc->n);
    void *mem = nullptr;
    const int rc = hip_check(hipMalloc(&mem, bytes), "hipMalloc(preconditioner, FP32)");
    if (rc) return rc;
    DevArena ar{(char *)mem, 0, bytes};
    float **dst[kNumArrays] = {&pc->f32.Dinv11, &pc->f32.Dinv22, &pc->f32.E,    &pc->f32.B21, &pc->f32.B23,
                               &pc->f32.B31,    &pc->f32.G,      &pc->f32.Sinv, &pc->f32.Uinv};
    for (int q = 0; q < kNumArrays; ++q) *dst[q] = ar.take<float>(cnt[q]);
    f->scratch = ar.take<double>((size_t)4 * pc->n);
    f->mem = mem;
    f->bytes = bytes;
    return BIM_OK;
}

// Releases an FP32 allocation that was not adopted.
static void precond_fp32_drop(Precond *pc, Fp32Mem *f) {
    if (f->mem) (void)hipFree(f->mem);
    *f = Fp32Mem{};
    pc->f32 = PrecondArrays<float>{};
}

static int precond_fp32_finish(Precond *pc, Fp32Mem *f, bool with_sinv, hipStream_t st) {
    size_t cnt[kNumArrays];
    precond_counts(pc, cnt);
    const double *src[kNumArrays] = {pc->Dinv11, pc->Dinv22, pc->E, pc->B21, pc->B23, pc->B31, pc->G, pc->Sinv, pc->Uinv};
    float *dst[kNumArrays] = {pc->f32.Dinv11, pc->f32.Dinv22, pc->f32.E,    pc->f32.B21, pc->f32.B23,
                              pc->f32.B31,    pc->f32.G,      pc->f32.Sinv, pc->f32.Uinv};
    int rc = BIM_OK;
    for (int q = 0; q < kNumArrays && !rc; ++q)
        if (q != 7 || with_sinv) rc = to_float_enqueue(src[q], dst[q], cnt[q], st);
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (rc) return rc;  // (the caller releases f once no stream uses it)
    (void)hipFree(pc->mem);
    pc->mem = f->mem;
    pc->bytes = f->bytes;
    pc->scratch = f->scratch;
    *f = Fp32Mem{};
    pc->Dinv11 = pc->Dinv22 = pc->E = pc->B21 = pc->B23 = pc->B31 = pc->G = pc->Sinv = pc->Uinv = nullptr;
    pc->storage = BIM_STORE_FP32;
    return BIM_OK;
}

static int precond_round_to_fp32(Precond *pc, hipStream_t st) {
    Fp32Mem f;
    int rc = precond_fp32_alloc(pc, &f);
    if (!rc) rc = precond_fp32_finish(pc, &f, true, st);
    if (rc) {
        (void)hipStreamSynchronize(st);
        precond_fp32_drop(pc, &f);
    }
    return rc;
}

int precond_build(const bim_problem *p, int hb, int storage, Precond **out, hipStream_t st) {
    const Dims d(p);
    const int N = d.N, M = d.M, s = N + 1;
    const int h = hb;
    const long n = (long)s * M;
    const int w2 = 2 * h;
    Precond *pc = new Precond();
    pc->N = N;
    pc->M = M;
    pc->s = s;
    pc->h = h;
    pc->n = n;
    // layout of the persistent part
    size_t pers = 0;
    auto add = [&](size_t elems) { pers += (sizeof(double) * elems + 255) & ~(size_t)255; };
    add(band_elems(M, 0, s));  // Dinv11 replicated
    add(band_elems(M, 0, s));  // Dinv22 replicated
    add(band_elems(M, 0, s));  // E replicated
    add(band_elems(M, h, s));  // B21
    add(band_elems(M, h, s));  // B23
    add(band_elems(M, h, s));  // B31
    add(band_elems(M, h, s));  // G
    add((size_t)n * n);        // L^-1 | I | V^-1
    add(band_elems(M, 0, s));  // D^-1 (inverse pivot blocks)
    add((size_t)4 * n);        // apply scratch
    pc->bytes = pers;
    int rc = hip_check(hipMalloc(&pc->mem, pers), "hipMalloc(preconditioner)");
    if (rc) {
        delete pc;
        return rc;
    }
    DevArena ar{(char *)pc->mem, 0, pers};
    pc->Dinv11 = ar.take<double>(band_elems(M, 0, s));
    pc->Dinv22 = ar.take<double>(band_elems(M, 0, s));
    pc->E = ar.take<double>(band_elems(M, 0, s));
    pc->B21 = ar.take<double>(band_elems(M, h, s));
    pc->B23 = ar.take<double>(band_elems(M, h, s));
    pc->B31 = ar.take<double>(band_elems(M, h, s));
    pc->G = ar.take<double>(band_elems(M, h, s));
    pc->Sinv = ar.take<double>((size_t)n * n);
    pc->Uinv = ar.take<double>(band_elems(M, 0, s));
    pc->scratch = ar.take<double>((size_t)4 * n);

    // setup-only scratch
    size_t tmp = 0;
    auto addt = [&](size_t bytes) { tmp += (bytes + 255) & ~(size_t)255; };
    addt(sizeof(double) * 3 * s * s);               // D11, D12, D22
    addt(sizeof(double) * 2 * s * s);               // single inverses
    addt(sizeof(double) * 2 * d.ntg);               // rowsum5, I5
    addt(sizeof(double) * band_elems(M, h, s));     // T (band h)
    addt(sizeof(double) * band_elems(M, w2, s));    // S band 2h
    addt(sizeof(double) * (size_t)M * s * w2 * s);  // L rows
    addt(sizeof(double) * (size_t)M * s * w2 * s);  // U rows
    if (storage == BIM_STORE_FP32) addt(sizeof(float) * (size_t)M * s * w2 * s);  // L rows in FP32
    addt(sizeof(double) * (size_t)s * s);           // E (one block)
    addt(sizeof(double) * (size_t)4 * s * 2 * s);   // inversion work
    addt(sizeof(int) * 3 * (M + 2));                // info (2 more per block for split inversions)
    addt(sizeof(SplitInv) * (M + 2));               // split-inversion plans (192 < s <= 384)
    const size_t nitems = 64 + (size_t)M * (2 * h + 1) * 4 + (size_t)M * (2 * w2 + 1) * (2 * h + 3) +
                          (size_t)M * (w2 * w2 + w2 + 2) + 16;
    addt(sizeof(GemmItem) * nitems);
    addt(sizeof(GemmItem) * M);              // V rows
    addt(sizeof(GemmTriItem) * (2 * (size_t)M + 2));  // triangular substitutions (rows of L^-1 at 0, of V^-1 at M)
    addt(sizeof(GemmTriItemF) * 2 * M);      // the same in FP32
    addt(sizeof(InvItem) * (M + 4));
    addt(sizeof(GemmKItem) * (size_t)M * (2 * w2 + 1));
    void *tbase = nullptr;
    rc = hip_check(hipMallocAsync(&tbase, tmp, st), "hipMallocAsync(preconditioner setup)");
    if (rc) {
        (void)hipFree(pc->mem);
        delete pc;
        return rc;
    }
    DevArena ta{(char *)tbase, 0, tmp};
    double *D11 = ta.take<double>((size_t)3 * s * s);
    double *D12 = D11 + (size_t)s * s;
    double *D22 = D12 + (size_t)s * s;
    double *Dinv11 = ta.take<double>((size_t)2 * s * s);
    double *Dinv22 = Dinv11 + (size_t)s * s;
    double *rowsum = ta.take<double>((size_t)2 * d.ntg);
    double *I5 = rowsum + d.ntg;
    double *T = ta.take<double>(band_elems(M, h, s));
    double *S = ta.take<double>(band_elems(M, w2, s));
    double *const Uinv = pc->Uinv;
    double *Lrow = ta.take<double>((size_t)M * s * w2 * s);
    double *Urow = ta.take<double>((size_t)M * s * w2 * s);
    float *L32 = (storage == BIM_STORE_FP32) ? ta.take<float>((size_t)M * s * w2 * s) : nullptr;
    double *rowtmp = ta.take<double>((size_t)s * s);
    double *invwork = ta.take<double>((size_t)4 * s * 2 * s);
    int *info = ta.take<int>(3 * (M + 2));
    SplitInv *plans_dev = ta.take<SplitInv>(M + 2);

    GemmItem *items_dev = ta.take<GemmItem>(nitems);
    InvItem *inv_dev = ta.take<InvItem>(M + 4);
    GemmKItem *kitems_dev = ta.take<GemmKItem>((size_t)M * (2 * w2 + 1));
    GemmItem *vitems_dev = ta.take<GemmItem>(M);
    GemmTriItem *tri_dev = ta.take<GemmTriItem>(2 * (size_t)M + 2);
    GemmTriItemF *tri32_dev = ta.take<GemmTriItemF>((size_t)2 * M);

    std::vector<GemmItem> items;
    items.reserve(nitems);
    std::vector<InvItem> invs;
    const bool split = split_invert_applies(s);
    std::vector<SplitInv> plans;
    // inversions first .. first + count - 1 of `invs` (their items already on the device)
    auto invert_range = [&](int first, int count) -> int {
        if (!split) return invert_enqueue(inv_dev + first, count, s, invwork, info + first, st);
        for (int i = first; i < first + count; ++i)
            if (int q = split_invert_enqueue(plans[i], plans_dev + i, s, info + (M + 2) + 2 * i, st)) return q;
        return BIM_OK;
    };
    // plans of invs[first ..] (sharing the inversion scratch), copied to the device
    auto plan_range = [&](int first) -> int {
        if (!split) return BIM_OK;
        if (split_invert_scratch(s) > (size_t)4 * s * 2 * s) return fail(BIM_EINVAL, "split inversion scratch");
        plans.resize(invs.size());
        for (size_t i = first; i < invs.size(); ++i) split_invert_plan(invs[i], s, invwork, &plans[i]);
        return hip_check(hipMemcpyAsync(plans_dev + first, plans.data() + first, sizeof(SplitInv) * (invs.size() - first),
                                        hipMemcpyHostToDevice, st),
                         "copy");
    };
    struct Op {
        int kind;  // 0 gemm, 1 invert, 2 copy rows
        size_t first;
        int count, m, nn, k, lda, ldb, ldc;
        double alpha, beta;
    };
    std::vector<Op> ops;
    auto gemm = [&](std::vector<GemmItem> batch, int m_, int n_, int k_, int lda, int ldb, int ldc, double al,
                    double be) {
        if (batch.empty()) return;
        ops.push_back({0, items.size(), (int)batch.size(), m_, n_, k_, lda, ldb, ldc, al, be});
        items.insert(items.end(), batch.begin(), batch.end());
    };

#define RUN(x)                   \
    do {                         \
        const int rc_ = (x);     \
        if (rc_) return rc_;     \
    } while (0)

    hipStream_t aux = nullptr;  // the second stream (default priority) and its events
    hipEvent_t ev_l = nullptr, ev_f = nullptr;
    Fp32Mem f32mem;             // the FP32 operator's memory until it is adopted
    rc = [&]() -> int {
    // 1. diagonal blocks and their inverses, E = D11^-1 D12
    hipLaunchKernelGGL(k_diag_blocks, dim3(cdiv((long)s * s, 256)), dim3(256), 0, st, D11, D12, D22, N, p->x1,
                       p->dx, p->n_decay, p->froude);
    invs.push_back({D11, s, Dinv11, s});
    invs.push_back({D22, s, Dinv22, s});
    RUN(hip_check(hipMemcpyAsync(inv_dev, invs.data(), sizeof(InvItem) * 2, hipMemcpyHostToDevice, st), "copy"));
    RUN(plan_range(0));
    RUN(invert_range(0, 2));
    hipLaunchKernelGGL(k_replicate, dim3(cdiv((long)M * s * s, 256)), dim3(256), 0, st, Dinv11, pc->Dinv11, M,
                       (long)s * s);
    hipLaunchKernelGGL(k_replicate, dim3(cdiv((long)M * s * s, 256)), dim3(256), 0, st, Dinv22, pc->Dinv22, M,
                       (long)s * s);

    // 2. band blocks of P21, P23 (= P32), P31
    for (double *b : {pc->B21, pc->B23, pc->B31})
        RUN(hip_check(hipMemsetAsync(b, 0, sizeof(double) * band_elems(M, h, s), st), "memset"));
    hipLaunchKernelGGL(k_k5_rowsum, dim3(d.ntg), dim3(64), 0, st, rowsum, I5, N, M, p->x1, p->dx, p->y1, p->dy,
                       d.nimg);
    hipLaunchKernelGGL(k_band_rows, dim3(M * (2 * h + 1) * (N - 1)), dim3(64), 0, st, pc->B21, pc->B23, pc->B31,
                       rowsum, I5, N, M, h, p->x1, p->dx, p->y1, p->dy, d.nimg);
    RUN(hip_check(hipGetLastError(), "band assembly launch"));

    {
        // E (one block) then replicated
        gemm({{Dinv11, D12, rowtmp}}, s, s, s, s, s, s, 1.0, 0.0);
        // T[l][m] = B23[l][m] - B31[l][m] E ; G[l][m] = Dinv22 T[l][m]
        std::vector<GemmItem> b1, b2, b3;
        for (int l = 0; l < M; ++l)
            for (int m = std::max(0, l - h); m <= std::min(M - 1, l + h); ++m) {
                b1.push_back({band_blk(pc->B31, h, s, l, m), rowtmp, band_blk(T, h, s, l, m)});
                b2.push_back({Dinv22, band_blk(T, h, s, l, m), band_blk(pc->G, h, s, l, m)});
            }
        // S = D22 on the diagonal, - B21 E within band h, - sum_q B23[l][q] G[q][m]
        std::vector<GemmItem> bS1;
        for (int l = 0; l < M; ++l)
            for (int m = std::max(0, l - h); m <= std::min(M - 1, l + h); ++m)
                bS1.push_back({band_blk(pc->B21, h, s, l, m), rowtmp, band_blk(S, w2, s, l, m)});
        // enqueue in dependency order
        size_t op0 = ops.size();
        (void)op0;
        // E first (needs Dinv11)
        // T = B23 copy is done before the -B31 E accumulation (copy via GEMM with beta)
        gemm(b1, s, s, s, s, s, s, -1.0, 1.0);  // T := T - B31 E   (T pre-filled with B23)
        gemm(b2, s, s, s, s, s, s, 1.0, 0.0);   // G := Dinv22 T
        gemm(bS1, s, s, s, s, s, s, -1.0, 1.0); // S := S - B21 E   (S pre-filled with D22 on the diagonal)
    }
    // S[l][m] -= sum_q B23[l][q] G[q][m] over q in [max(0, l-h, m-h), min(M-1, l+h, m+h)]: one
    // product per output block with the q-blocks as K (consecutive q: the next block of row l of
    // B23, s^2 further; the same column m of G one band row down, 2h s^2 further)
    // (rows l in the order 0, 8, 16, .., 1, 9, ..: the product's workgroups are
    // split over the 8 XCDs in contiguous ranges, which then each hold a mix of
    // edge rows, with fewer q-blocks, and interior rows)
    std::vector<GemmKItem> kitems;
    std::vector<int> lorder;
    for (int r = 0; r < 8; ++r)
        for (int l = r; l < M; l += 8) lorder.push_back(l);
    for (int l : lorder)
        for (int m = std::max(0, l - w2); m <= std::min(M - 1, l + w2); ++m) {
            const int q0 = std::max(0, std::max(l - h, m - h)), q1 = std::min(M - 1, std::min(l + h, m + h));
            if (q0 <= q1)
                kitems.push_back({band_blk(pc->B23, h, s, l, q0), band_blk(pc->G, h, s, q0, m), band_blk(S, w2, s, l, m),
                                  (long)(q1 - q0 + 1)});
        }
    // block LU of S (band 2h): per step l, L[q][l] = S[q][l] Uinv[l] (into Lrow, leading
    // dim 2h s), then S[q][m] -= L[q][l] S[l][m] for q, m in l+1..l+2h
    const size_t elim_end = ops.size();
    std::vector<long> op_bl(M, -1), op_upd(M, -1);
    for (int l = 0; l < M; ++l) {
        const int hi = std::min(M - 1, l + w2);
        auto Lblk = [&](int q) { return Lrow + ((size_t)q * s) * (w2 * s) + (size_t)(l - (q - w2)) * s; };
        std::vector<GemmItem> bl, bu;
        for (int q = l + 1; q <= hi; ++q) bl.push_back({band_blk(S, w2, s, q, l), Uinv + (size_t)l * s * s, Lblk(q)});
        for (int q = l + 1; q <= hi; ++q)
            for (int m = l + 1; m <= hi; ++m) bu.push_back({Lblk(q), band_blk(S, w2, s, l, m), band_blk(S, w2, s, q, m)});
        if (!bl.empty()) op_bl[l] = (long)ops.size();
        gemm(bl, s, s, s, s, s, w2 * s, 1.0, 0.0);
        if (!bu.empty()) op_upd[l] = (long)ops.size();
        gemm(bu, s, s, s, w2 * s, s, s, -1.0, 1.0);
    }
    for (int l = 0; l < M; ++l) invs.push_back({band_blk(S, w2, s, l, l), s, Uinv + (size_t)l * s * s, s});

    // upload all item arrays once
    RUN(hip_check(hipMemcpyAsync(items_dev, items.data(), sizeof(GemmItem) * items.size(), hipMemcpyHostToDevice,
                                 st),
                  "copy"));
    RUN(hip_check(hipMemcpyAsync(inv_dev, invs.data(), sizeof(InvItem) * invs.size(), hipMemcpyHostToDevice, st),
                  "copy"));
    RUN(plan_range(2));
    RUN(hip_check(hipMemcpyAsync(kitems_dev, kitems.data(), sizeof(GemmKItem) * kitems.size(), hipMemcpyHostToDevice,
                                 st),
                  "copy"));
    {
        auto run_op = [&](const Op &o, hipStream_t on) {
            return gemm_enqueue(items_dev + o.first, o.count, o.m, o.nn, o.k, o.lda, o.ldb, o.ldc, o.alpha, o.beta,
                                on);
        };
        // E, replicated
        RUN(run_op(ops[0], st));
        hipLaunchKernelGGL(k_replicate, dim3(cdiv((long)M * s * s, 256)), dim3(256), 0, st, rowtmp, pc->E, M,
                           (long)s * s);
        // T := B23 ; S := 0 with D22 on the diagonal
        RUN(copy2d_enqueue(pc->B23, 1, T, 1, 1, (int)band_elems(M, h, s), st));
        RUN(hip_check(hipMemsetAsync(S, 0, sizeof(double) * band_elems(M, w2, s), st), "memset"));
        const long bs = (long)s * s, brow = (long)(2 * w2 + 1) * bs;  // one block; one block row of S
        RUN(copy_blocks_enqueue(D22, 0, 0, s, band_blk(S, w2, s, 0, 0), brow, 0, s, s, s, M, 1, M, st));
        for (size_t q = 1; q < elim_end; ++q) RUN(run_op(ops[q], st));
        RUN(gemm_kblocks_enqueue(kitems_dev, (int)kitems.size(), s, s, s, s, s, s, (long)s * s, (long)2 * h * s * s,
                                 -1.0, 1.0, st));
        // zero L/U row buffers (short rows at the ends stay zero)
        RUN(hip_check(hipMemsetAsync(Lrow, 0, sizeof(double) * (size_t)M * s * w2 * s, st), "memset"));
        RUN(hip_check(hipMemsetAsync(Urow, 0, sizeof(double) * (size_t)M * s * w2 * s, st), "memset"));
        // The rows of L^-1 (see below) run on a second stream during the block LU:
        // row j needs the L blocks of row j, all formed by step j - 1, and the
        // rows of L^-1 above it, and it touches nothing the LU reads or writes.
        // The pivot inversions leave all but one compute unit idle, and the
        // forward rows fill them.  In FP32 (FP32-stored operator and
        // 128 < s <= 384) the second stream first rounds row j of L to FP32 and
        // the rows of L^-1 are formed in FP32, directly in the FP32 operator.
        // The forward rows' workgroups (one per compute unit, by their LDS) are
        // capped so that compute units stay free: a pivot inversion needs a whole
        // compute unit's registers and would otherwise wait for one to drain.
        constexpr int kAuxTriGroups = 192;
        const bool bw32 = storage == BIM_STORE_FP32 && s > 128 && s <= 384;
        const int far = 1 << 29;  // an offset that leaves klo at 0 / khi at nk
        const size_t lrow = (size_t)s * w2 * s;  // elements of one block row of L (or V)
        float *S32 = nullptr;
        std::vector<GemmTriItem> fwd;
        std::vector<GemmTriItemF> fwd32;
        RUN(identity_enqueue(pc->Sinv, n, st));
        if (bw32) {
            // the FP32 operator's memory now, with S^-1 = I rounded into it
            RUN(precond_fp32_alloc(pc, &f32mem));
            S32 = pc->f32.Sinv;
            RUN(to_float_enqueue(pc->Sinv, S32, (size_t)n * n, st));
        }
        for (int j = 1; j < M; ++j) {
            const int lf = j, q0 = std::max(0, lf - w2), nkf = lf - q0;
            const size_t a_off = lf * lrow + (size_t)(q0 - (lf - w2)) * s;
            if (bw32)
                fwd32.push_back({L32 + a_off, S32 + (size_t)q0 * s * n, S32 + (size_t)lf * s * n, nkf, 0, lf, q0, -far,
                                 0});
            else
                fwd.push_back({Lrow + a_off, pc->Sinv + (size_t)q0 * s * n, pc->Sinv + (size_t)lf * s * n, nkf, 0, lf,
                               q0, -far, 0});
        }
        if (!fwd.empty())
            RUN(hip_check(hipMemcpyAsync(tri_dev, fwd.data(), sizeof(GemmTriItem) * fwd.size(), hipMemcpyHostToDevice,
                                         st),
                          "copy"));
        if (!fwd32.empty())
            RUN(hip_check(hipMemcpyAsync(tri32_dev, fwd32.data(), sizeof(GemmTriItemF) * fwd32.size(),
                                         hipMemcpyHostToDevice, st),
                          "copy"));
        RUN(hip_check(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking), "hipStreamCreate"));
        RUN(hip_check(hipEventCreateWithFlags(&ev_l, hipEventDisableTiming), "hipEventCreate"));
        RUN(hip_check(hipEventCreateWithFlags(&ev_f, hipEventDisableTiming), "hipEventCreate"));
        for (int l = 0; l < M; ++l) {
            RUN(invert_range(2 + l, 1));
            if (op_bl[l] >= 0) RUN(run_op(ops[op_bl[l]], st));
            if (l + 1 < M) {  // row l + 1 of L^-1
                RUN(hip_check(hipEventRecord(ev_l, st), "hipEventRecord"));
                RUN(hip_check(hipStreamWaitEvent(aux, ev_l, 0), "hipStreamWaitEvent"));
                if (bw32) {
                    RUN(to_float_enqueue(Lrow + (l + 1) * lrow, L32 + (l + 1) * lrow, lrow, aux));
                    RUN(gemm_tri_enqueue(tri32_dev + l, 1, s, l + 1, w2 * s, (int)n, (int)n, -1.0, aux,
                                         kAuxTriGroups));
                } else {
                    RUN(gemm_tri_enqueue(tri_dev + l, 1, s, l + 1, w2 * s, (int)n, (int)n, -1.0, aux, kAuxTriGroups));
                }
            }
            if (op_upd[l] >= 0) RUN(run_op(ops[op_upd[l]], st));
        }
        RUN(hip_check(hipEventRecord(ev_f, aux), "hipEventRecord"));
        // U rows: U[l][m] for m = l+1..l+2h packed as [l][s][2h s] (block j = m - l - 1,
        // copied while l + j + 1 < M)
        RUN(copy_blocks_enqueue(S + (size_t)(w2 + 1) * bs, brow, bs, s, Urow, (long)s * w2 * s, s, (long)w2 * s, s, s,
                                M, w2, M - 1, st));
        // S = L D V with D the pivot blocks and V = D^-1 U unit upper: the rows of V,
        // V[l][m] = Uinv[l] U[l][m], into the memory of S (no longer read)
        // (the host item arrays stay alive until the closing synchronisation)
        double *Vrow = S;
        std::vector<GemmItem> vi;
        {
            for (int l = 0; l < M; ++l)
                vi.push_back({pc->Uinv + (size_t)l * s * s, Urow + (size_t)l * s * w2 * s, Vrow + (size_t)l * s * w2 * s});
            RUN(hip_check(hipMemcpyAsync(vitems_dev, vi.data(), sizeof(GemmItem) * vi.size(), hipMemcpyHostToDevice, st),
                          "copy"));
            RUN(gemm_enqueue(vitems_dev, M, s, w2 * s, s, s, w2 * s, w2 * s, 1.0, 0.0, st));
        }
        // S^-1 = V^-1 D^-1 L^-1: L^-1 (unit lower) below the block diagonal of Sinv and
        // V^-1 (unit upper) above it, identity blocks on it, both read by the
        // substitutions and never written:
        //   row block l of L^-1:  X[l][c] = -sum_{q = max(q0, c)}^{l-1} L[l][q] X[q][c],  c < l
        //   row block l of V^-1:  Y[l][c] = -sum_{m = l+1}^{min(c, l+2h)} V[l][m] Y[m][c],  c > l
        // (q0 = max(0, l - 2h)).  The two touch disjoint triangles, so the rows of
        // V^-1 (step j: row M-1-j, j column blocks wide, at most 2h K blocks deep)
        // run while the second stream finishes the rows of L^-1.
        std::vector<GemmTriItem> bwd;
        std::vector<GemmTriItemF> bwd32;
        const float *V32 = nullptr;
        if (bw32) {
            // V into its FP32 copy (in the memory of the FP64 U rows), then the
            // other arrays of the operator rounded; the FP64 allocation is freed
            float *v32 = (float *)Urow;
            RUN(to_float_enqueue(Vrow, v32, (size_t)M * lrow, st));
            V32 = v32;
            RUN(precond_fp32_finish(pc, &f32mem, false, st));
        }
        for (int j = 1; j < M; ++j) {
            const int lb = M - 1 - j, nkb = std::min(M - 1, lb + w2) - lb;
            if (bw32)
                bwd32.push_back({V32 + lb * lrow, S32 + (size_t)(lb + 1) * s * n, S32 + (size_t)lb * s * n, nkb, lb + 1,
                                 M - 1 - lb, far, lb, 1});
            else
                bwd.push_back({Vrow + lb * lrow, pc->Sinv + (size_t)(lb + 1) * s * n, pc->Sinv + (size_t)lb * s * n,
                               nkb, lb + 1, M - 1 - lb, far, lb, 1});
        }
        if (!bwd.empty())
            RUN(hip_check(hipMemcpyAsync(tri_dev + M, bwd.data(), sizeof(GemmTriItem) * bwd.size(),
                                         hipMemcpyHostToDevice, st),
                          "copy"));
        if (!bwd32.empty())
            RUN(hip_check(hipMemcpyAsync(tri32_dev + M, bwd32.data(), sizeof(GemmTriItemF) * bwd32.size(),
                                         hipMemcpyHostToDevice, st),
                          "copy"));
        for (int j = 1; j < M; ++j) {
            if (bw32)
                RUN(gemm_tri_enqueue(tri32_dev + M + (j - 1), 1, s, j, w2 * s, (int)n, (int)n, -1.0, st));
            else
                RUN(gemm_tri_enqueue(tri_dev + M + (j - 1), 1, s, j, w2 * s, (int)n, (int)n, -1.0, st));
        }
        RUN(hip_check(hipStreamWaitEvent(st, ev_f, 0), "hipStreamWaitEvent"));
        // a zero pivot in any inverted block makes P singular in this factorisation
        std::vector<int> hinfo(3 * (2 + M), 0);
        RUN(hip_check(hipMemcpyAsync(hinfo.data(), info, sizeof(int) * 3 * (2 + M), hipMemcpyDeviceToHost, st),
                      "copy"));
        RUN(hip_check(hipStreamSynchronize(st), "hipStreamSynchronize"));
        for (int q = 0; q < 2 + M; ++q) {
            const bool bad = split ? (hinfo[(M + 2) + 2 * q] || hinfo[(M + 2) + 2 * q + 1]) : hinfo[q] != 0;
            if (bad) return fail(BIM_EDOMAIN, "preconditioner: singular diagonal block " + std::to_string(q));
        }
    }
    return BIM_OK;
    }();
#undef RUN
    if (aux) {
        (void)hipStreamSynchronize(aux);  // (on success `st` has already waited for it)
        (void)hipStreamDestroy(aux);
    }
    if (ev_l) (void)hipEventDestroy(ev_l);
    if (ev_f) (void)hipEventDestroy(ev_f);
    if (f32mem.mem) {  // allocated but not adopted: an error came first
        (void)hipStreamSynchronize(st);
        precond_fp32_drop(pc, &f32mem);
    }
    (void)hipFreeAsync(tbase, st);
    if (!rc && storage == BIM_STORE_FP32 && pc->storage != BIM_STORE_FP32) rc = precond_round_to_fp32(pc, st);
    if (rc) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(pc->mem);
        delete pc;
        return rc;
    }
    *out = pc;
    return BIM_OK;
}

template <typename T>
static int precond_apply_impl(const Precond *pc, const PrecondArrays<const T> &a, const double *r, double *z,
                              hipStream_t st) {
    const int M = pc->M, s = pc->s, h = pc->h;
    const long n = pc->n;
    const double *r1 = r, *r2 = r + n, *r3 = r + 2 * n;
    double *z1 = z, *z2 = z + n, *z3 = z + 2 * n;
    double *a1 = pc->scratch, *a3 = a1 + n, *t2 = a3 + n, *t3 = t2 + n;
    int rc;
    if ((rc = bandmv_enqueue(a.Dinv11, M, 0, s, r1, nullptr, a1, 1.0, 0.0, st))) return rc;       // a1
    if ((rc = bandmv_enqueue(a.B31, M, h, s, a1, r3, t3, -1.0, 1.0, st))) return rc;              // r3 - P31 a1
    if ((rc = bandmv_enqueue(a.Dinv22, M, 0, s, t3, nullptr, a3, 1.0, 0.0, st))) return rc;       // a3
    if ((rc = bandmv_enqueue(a.B21, M, h, s, a1, r2, t2, -1.0, 1.0, st))) return rc;              // r2 - P21 a1
    if ((rc = bandmv_enqueue(a.B23, M, h, s, a3, t2, t2, -1.0, 1.0, st))) return rc;              // - P23 a3
    // z2 = V^-1 D^-1 L^-1 t2 (t3 is free once a3 is formed)
    if ((rc = gemv_tri_enqueue(a.Sinv, n, M, s, 1, t2, t2, t3, 1.0, 1.0, st))) return rc;         // L^-1 t2
    if ((rc = bandmv_enqueue(a.Uinv, M, 0, s, t3, nullptr, t2, 1.0, 0.0, st))) return rc;         // D^-1
    if ((rc = gemv_tri_enqueue(a.Sinv, n, M, s, 2, t2, t2, z2, 1.0, 1.0, st))) return rc;         // V^-1
    if ((rc = bandmv_enqueue(a.G, M, h, s, z2, a3, z3, -1.0, 1.0, st))) return rc;                // z3
    return bandmv_enqueue(a.E, M, 0, s, z2, a1, z1, -1.0, 1.0, st);                               // z1
}

int precond_apply_enqueue(const Precond *pc, const double *r, double *z, hipStream_t st) {
    if (pc->storage == BIM_STORE_FP32) {
        const PrecondArrays<const float> a{pc->f32.Dinv11, pc->f32.Dinv22, pc->f32.E,    pc->f32.B21, pc->f32.B23,
                                           pc->f32.B31,    pc->f32.G,      pc->f32.Sinv, pc->f32.Uinv};
        return precond_apply_impl(pc, a, r, z, st);
    }
    const PrecondArrays<const double> a{pc->Dinv11, pc->Dinv22, pc->E,    pc->B21, pc->B23,
                                        pc->B31,    pc->G,      pc->Sinv, pc->Uinv};
    return precond_apply_impl(pc, a, r, z, st);
}

const void *precond_array(const Precond *pc, int which) {
    const bool f = pc->storage == BIM_STORE_FP32;
    switch (which) {
        case 0: return f ? (const void *)pc->f32.Dinv11 : (const void *)pc->Dinv11;
        case 1: return f ? (const void *)pc->f32.Dinv22 : (const void *)pc->Dinv22;
        case 2: return f ? (const void *)pc->f32.E : (const void *)pc->E;
        case 3: return f ? (const void *)pc->f32.B21 : (const void *)pc->B21;
        case 4: return f ? (const void *)pc->f32.B23 : (const void *)pc->B23;
        case 5: return f ? (const void *)pc->f32.B31 : (const void *)pc->B31;
        case 6: return f ? (const void *)pc->f32.G : (const void *)pc->G;
        case 7: return f ? (const void *)pc->f32.Sinv : (const void *)pc->Sinv;
        case 8: return f ? (const void *)pc->f32.Uinv : (const void *)pc->Uinv;
        default: return nullptr;
    }
}

void precond_free(Precond *pc) {
    if (!pc) return;
    if (pc->mem) (void)hipFree(pc->mem);
    delete pc;
}

}  // namespace bim

// ------------------------------------------------------------------ C ABI
struct bim_precond {
    bim::Precond *pc;
};

using namespace bim;

extern "C" {

int precond_setup(const bim_problem *prob, int band_halfwidth, bim_precond **out, void *stream) {
    return precond_setup_ex(prob, band_halfwidth, BIM_STORE_FP64, out, stream);
}

int precond_setup_ex(const bim_problem *prob, int band_halfwidth, int storage, bim_precond **out, void *stream) {
    int rc = validate(prob);
    if (rc) return rc;
    if (!out) return fail(BIM_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (storage != BIM_STORE_FP64 && storage != BIM_STORE_FP32) return fail(BIM_EINVAL, "unknown storage");
    // default: round(M / 6) slices, at most 10 (a wider band costs more setup than it
    // saves GMRES iterations: 151 x 151 full domain, F = 0.6, total FP64 time to
    // solution 545-560 ms at h = 8-10 against 830 ms at round(M / 6) = 25)
    const int hb = band_halfwidth < 0 ? std::max(1, std::min(10, (int)std::lround(prob->M / 6.0))) : band_halfwidth;
    if (hb < 1 || hb >= prob->M) return fail(BIM_EINVAL, "band half-width must be in [1, M-1]");
    if (prob->N + 1 > 1024) return fail(BIM_EINVAL, "N + 1 must not exceed 1024");
    Precond *pc = nullptr;
    rc = precond_build(prob, hb, storage, &pc, (hipStream_t)stream);
    if (rc) return rc;
    *out = new bim_precond{pc};
    return BIM_OK;
}

int precond_apply(const bim_precond *P, const double *r, double *z, void *stream) {
    if (!P || !P->pc) return fail(BIM_EINVAL, "preconditioner handle is NULL");
    if (!r || !z) return fail(BIM_EINVAL, "r and z must be device pointers");
    if (r == z) return fail(BIM_EINVAL, "z must not alias r");
    return precond_apply_enqueue(P->pc, r, z, (hipStream_t)stream);
}

void precond_destroy(bim_precond *P) {
    if (!P) return;
    precond_free(P->pc);
    delete P;
}

int64_t precond_bytes(const bim_precond *P) { return (P && P->pc) ? (int64_t)P->pc->bytes : 0; }

int precond_band(const bim_precond *P) { return (P && P->pc) ? P->pc->h : 0; }

int precond_storage(const bim_precond *P) { return (P && P->pc) ? P->pc->storage : -1; }

}  // extern "C"

namespace bim {
Precond *precond_impl(const bim_precond *P) { return P ? P->pc : nullptr; }
}  // namespace bim
