// FP64 vector helpers (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace bim {

// Number of partial sums a reduction writes (size of `part`).
int reduce_parts();
// out[0] = a . b (or its square root), deterministic two-pass reduction.
int dot_enqueue(const double *a, const double *b, long n, double *part, double *out, bool take_sqrt,
                hipStream_t s);
// scal[2] = h: the given h if > 0, else sqrt(eps) (1 + |u|) / |v| (scal[0] = |u|, scal[1] = |v|).
int fd_shift_enqueue(const double *u, const double *v, long n, double h, double eps, double *part,
                     double *scal, hipStream_t s);
// out = x + (*hp) y
int axpy_dev_enqueue(const double *x, const double *y, const double *hp, double *out, long n, hipStream_t s);
// out = (Fw - Fu) / (*hp), or 0 when *hp == 0
int quotient_enqueue(const double *Fw, const double *Fu, const double *hp, double *out, long n, hipStream_t s);

// out[i] (+)= V[i] . w for i < nv (rows of V with leading dim ldv); part: nv * reduce_parts() doubles.
int multidot_enqueue(const double *V, long ldv, int nv, const double *w, long n, double *part, double *out,
                     bool accumulate, hipStream_t s);
// w -= sum_i V[i] h[i]   (h on the device)
int orth_update_enqueue(const double *V, long ldv, int nv, const double *h, double *w, long n, hipStream_t s);
// x += sum_i Z[i] y[i]   (y on the device)
int combine_enqueue(const double *Z, long ldz, int nz, const double *y, double *x, long n, hipStream_t s);
// out = x / den[0]   (den on the device)
int scale_inv_enqueue(const double *x, const double *den, double *out, long n, hipStream_t s);
// out = a x + b y (y unused when b == 0)
int axpby_enqueue(double a, const double *x, double b, const double *y, double *out, long n, hipStream_t s);
// out[0] = max |a_i| (NaN if any entry is NaN)
int maxabs_enqueue(const double *a, long n, double *part, double *out, hipStream_t s);
int uniform_stream_enqueue(double *u, int N, int M, double x1, hipStream_t s);

}  // namespace bim
