// FP64 dense kernels used by the preconditioner (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace bim {

// One product of a batched GEMM: C = alpha A B + beta C (row-major).
template <typename T>
struct GemmItemT {
    const T *A;
    const T *B;
    T *C;
};
using GemmItem = GemmItemT<double>;
// One product over nkb K-blocks at fixed strides: C = alpha sum_b A_b B_b + beta C.
struct GemmKItem {
    const double *A;
    const double *B;
    double *C;
    long nkb;
};
// One product of a block-triangular launch (blocks s x s): for each output
// column block cb = cb0 .. cb0 + ncb - 1,
//   C[:, cb] = alpha sum_{j = klo .. khi-1} A[:, j] B[j, cb],
//   klo = max(0, cb - lo_off), khi = min(nk, cb - hi_off)
// (A: s x (nk s); B: nk block rows; C: s rows; zero where klo >= khi).
// rev != 0: the column blocks are scheduled from the last to the first (for
// items whose K range grows with cb, so that the deepest start first).
template <typename T>
struct GemmTriItemT {
    const T *A;
    const T *B;
    T *C;
    int nk, cb0, ncb, lo_off, hi_off, rev;
};
using GemmTriItem = GemmTriItemT<double>;
using GemmTriItemF = GemmTriItemT<float>;
// One matrix of a batched inversion: Ainv = A^-1 (s x s, row-major).
struct InvItem {
    const double *A;
    long lda;
    double *Ainv;
    long ldinv;
};

// items_dev: device array of `batch` items; all share m, n, k and leading dims.
int gemm_enqueue(const GemmItem *items_dev, int batch, int m, int n, int k, int lda, int ldb, int ldc,
                 double alpha, double beta, hipStream_t s);
// C = alpha sum_{b < nkb} (A + b sA)(B + b sB) + beta C per item (every A_b
// m x k with leading dim lda, B_b k x n with ldb); nkb may differ per item.
int gemm_kblocks_enqueue(const GemmKItem *items_dev, int batch, int m, int n, int k, int lda, int ldb, int ldc,
                         long sA, long sB, double alpha, double beta, hipStream_t s);
// Block-triangular products of `batch` items (FP64 or FP32 matrix cores, any
// block size s); max_ncb: the largest ncb.  max_groups > 0 caps the workgroups
// of the launch (over all row panels; they then walk the column tiles with a
// stride), which leaves compute units free for other streams; 0: one
// workgroup per tile.
int gemm_tri_enqueue(const GemmTriItem *items_dev, int batch, int s, int max_ncb, int lda, int ldb, int ldc,
                     double alpha, hipStream_t st, int max_groups = 0);
int gemm_tri_enqueue(const GemmTriItemF *items_dev, int batch, int s, int max_ncb, int lda, int ldb, int ldc,
                     double alpha, hipStream_t st, int max_groups = 0);
// y = alpha A' x + beta c, A' the strictly lower (part 1) or strictly upper
// (part 2) block part of the dense n x n A with M x M blocks of s; c may equal x
// (read per row), y must not alias x.
int gemv_tri_enqueue(const double *A, long n, int M, int s, int part, const double *x, const double *c, double *y,
                     double alpha, double beta, hipStream_t st);
int gemv_tri_enqueue(const float *A, long n, int M, int s, int part, const double *x, const double *c, double *y,
                     double alpha, double beta, hipStream_t st);
// work: device scratch of batch * s * 2s doubles; info[b] = 0 or (1 + column of a zero pivot).
int invert_enqueue(const InvItem *items_dev, int batch, int s_dim, double *work, int *info, hipStream_t s);

// Inversion of one s x s block with 192 < s <= 384 as a 2 x 2 block matrix:
// the leading 192 x 192 block A11 and the Schur complement A22 - A21 A11^-1 A12
// by the register Gauss-Jordan kernel (partial pivoting within each), the rest
// by MFMA products:  B22 = (A22 - A21 T)^-1 with T = A11^-1 A12,
// B21 = -B22 A21 A11^-1, B12 = -T B22, B11 = A11^-1 - T B21.  (No pivoting
// across the split: A11 must be invertible on its own, as the blocks of the
// preconditioner's elimination are.)  The plan is built on the host, copied to
// device memory, then enqueued; inversions of one stream run in order and may
// share `scratch`.
struct SplitInv {
    InvItem inv11, invS;
    GemmItem T, Sc, W, B21, B12, B11;
};
bool split_invert_applies(int s_dim);
// scratch: device, at least split_invert_scratch(s) doubles (T, W and the Schur complement)
size_t split_invert_scratch(int s_dim);
void split_invert_plan(const InvItem &item, int s_dim, double *scratch, SplitInv *plan);
// plan_dev: a device copy of plan; info: two ints (zero-pivot flags of the two inversions)
int split_invert_enqueue(const SplitInv &plan, const SplitInv *plan_dev, int s_dim, int *info, hipStream_t s);
// y = alpha B x + beta c for a slice-block-banded B stored [M][2w+1][s][s]; c may equal y.
int bandmv_enqueue(const double *band, int M, int w, int s_dim, const double *x, const double *c, double *y,
                   double alpha, double beta, hipStream_t s);
int bandmv_enqueue(const float *band, int M, int w, int s_dim, const double *x, const double *c, double *y,
                   double alpha, double beta, hipStream_t s);
// dst[e] = (float) src[e], e < count
int to_float_enqueue(const double *src, float *dst, size_t count, hipStream_t s);
int copy2d_enqueue(const double *src, long lds, double *dst, long ldd, int rows, int cols, hipStream_t s);
// Copies the rows x cols blocks (l, j), l < nl, j < nj, l + j < lim, from
// src + l sl + j sj (leading dim lds) to dst + l dl + j dj (leading dim ldd).
int copy_blocks_enqueue(const double *src, long sl, long sj, long lds, double *dst, long dl, long dj, long ldd,
                        int rows, int cols, int nl, int nj, int lim, hipStream_t s);
int identity_enqueue(double *A, long n, hipStream_t s);

}  // namespace bim
