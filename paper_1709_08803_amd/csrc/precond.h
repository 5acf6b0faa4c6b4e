// Block-banded preconditioner (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "bim_common.h"

namespace bim {

// The nine arrays the apply reads, in one element type.  S^-1 is kept as
// V^-1 D^-1 L^-1 (S = L D V: L, V unit block-triangular, D the pivot blocks):
// Sinv holds L^-1 below the block diagonal and V^-1 above it (identity blocks
// on it), Uinv the inverse pivot blocks D^-1.
template <typename T>
struct PrecondArrays {
    T *Dinv11, *Dinv22, *E;  // band-0 arrays [M][s][s] (same block on every slice)
    T *B21, *B23, *B31, *G;  // band-h arrays [M][2h+1][s][s]
    T *Sinv;                 // dense [n][n]: L^-1 | I | V^-1 by slice blocks
    T *Uinv;                 // band-0 array [M][s][s]: D^-1
};

struct Precond {
    int N, M, s, h;
    long n;
    int storage = BIM_STORE_FP64;  // element type of the stored operator
    void *mem = nullptr;           // one device allocation holding the arrays and the scratch
    size_t bytes = 0;
    // FP64 arrays (built first; kept when storage is FP64, else released)
    double *Dinv11, *Dinv22, *E;
    double *B21, *B23, *B31, *G;
    double *Sinv, *Uinv;
    PrecondArrays<float> f32{};   // FP32 copies when storage is FP32
    double *scratch;              // [4 n] apply temporaries
};

int precond_build(const bim_problem *p, int hb, int storage, Precond **out, hipStream_t st);
int precond_apply_enqueue(const Precond *pc, const double *r, double *z, hipStream_t st);
void precond_free(Precond *pc);
// The array `which` (0..8: Dinv11, Dinv22, E, B21, B23, B31, G, Sinv, Uinv) as stored
// (FP64 or FP32 per pc->storage).
const void *precond_array(const Precond *pc, int which);

}  // namespace bim

struct bim_precond;
namespace bim {
Precond *precond_impl(const bim_precond *P);
}  // namespace bim
