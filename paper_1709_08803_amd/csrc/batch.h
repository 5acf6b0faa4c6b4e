// Batched FP64 vector and preconditioner kernels for lockstep solves of many
// problems of different sizes (internal).  Every launch covers all problems of
// a round: blockIdx.y selects the problem's descriptor.
#pragma once

#include <hip/hip_runtime.h>

namespace bim {

// Operands of one problem in a batched vector operation.  Slot meaning is
// documented per operation below.
struct BOp {
    const double *a;
    const double *b;
    double *c;
    const double *sa;  // device scalar(s) read
    double *sc;        // device scalar(s) written
    double *part;      // reduction partials (>= nv * kBRedBlocks doubles)
    long n;            // vector length
    long ld;           // row stride of a multi-vector (V, Z)
    int nv;            // number of rows of a multi-vector
    double alpha, beta;
};

constexpr int kBRedBlocks = 64;

// sc[0] = a . b (sqrt if take_sqrt)
int b_dot(const BOp *ops, int count, bool take_sqrt, hipStream_t s);
// sc[r] = a[r] . b for r < nv (a: nv rows of stride ld)
int b_multidot(const BOp *ops, int count, int max_nv, hipStream_t s);
// c -= sum_r a[r] sa[r]   (a: nv rows of stride ld)
int b_orth(const BOp *ops, int count, hipStream_t s);
// c += sum_r a[r] sa[r]
int b_combine(const BOp *ops, int count, hipStream_t s);
// c = a / sa[0]
int b_scale_inv(const BOp *ops, int count, hipStream_t s);
// c = a + sa[0] b
int b_axpy_dev(const BOp *ops, int count, hipStream_t s);
// c = (a - b) / sa[0], or 0 when sa[0] == 0
int b_quotient(const BOp *ops, int count, hipStream_t s);
// c = alpha a + beta b (b unused when beta == 0)
int b_axpby(const BOp *ops, int count, hipStream_t s);
// sc[0] = max |a|
int b_maxabs(const BOp *ops, int count, hipStream_t s);
// sc[2] = alpha (> 0) or sqrt(beta) (1 + sc[0]) / sc[1] (0 when sc[1] == 0); sc[0], sc[1] computed before
int b_shift(const BOp *ops, int count, hipStream_t s);

// c[0..7] = a[0..7]; c[8..8+nv) = b[0..nv)   (gather of small per-problem results)
int b_gather(const BOp *ops, int count, hipStream_t s);

// One slice-block-banded product y = alpha B x + beta c of one problem.
// band holds FP64 elements, or FP32 ones when f32 != 0 (products and sums in FP64).
struct BBand {
    const void *band;
    const double *x;
    const double *c;
    double *y;
    int M, w, s;
    double alpha, beta;
    int f32;
};
// max_groups: the largest M ceil(s / 4) over the ops (waves needed by the largest problem)
int b_bandmv(const BBand *ops, int count, int max_groups, hipStream_t s);
// One product y = alpha A' x + beta c of one problem, A' the strictly lower
// (part 1) or strictly upper (part 2) slice-block part of a dense n x n A
// (M slices of s, row stride n).  A holds FP64 elements, or FP32 ones when
// f32 != 0.  c may equal x; y must not alias x.
struct BGemv {
    const void *A;
    const double *x;
    const double *c;
    double *y;
    long n;
    int M, s, part;
    double alpha, beta;
    int f32;
};
// max_groups: the largest M ceil(s / 4) over the ops
int b_gemv_tri(const BGemv *ops, int count, int max_groups, hipStream_t s);

}  // namespace bim
