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

}  // namespace bim
