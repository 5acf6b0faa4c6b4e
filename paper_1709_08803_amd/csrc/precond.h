// Block-banded preconditioner (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "bim_common.h"

namespace bim {

struct Precond {
    int N, M, s, h;
    long n;
    void *mem = nullptr;     // one device allocation holding everything below
    size_t bytes = 0;
    double *Dinv11, *Dinv22, *E;  // band-0 arrays [M][s][s] (same block on every slice)
    double *B21, *B23, *B31, *G;  // band-h arrays [M][2h+1][s][s]
    double *Sinv;                 // dense [n][n]
    double *scratch;              // [4 n] apply temporaries
};

int precond_build(const bim_problem *p, int hb, Precond **out, hipStream_t st);
int precond_apply_enqueue(const Precond *pc, const double *r, double *z, hipStream_t st);
void precond_free(Precond *pc);

}  // namespace bim

struct bim_precond;
namespace bim {
Precond *precond_impl(const bim_precond *P);
}  // namespace bim
