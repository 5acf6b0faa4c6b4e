/*
 * bim.h -- C ABI of the MI355X boundary-integral JFNK library (libbim.so).
 *
 * The library evaluates and solves the discrete system of Buttle, Pethiyagoda,
 * Moroney & McCue, "Three dimensional free-surface flow over arbitrary bottom
 * topography" (J. Fluid Mech.): for a bottom z = beta(x, y) and a depth-based
 * Froude number F, find the free surface zeta and the surface and bottom
 * potentials phi, psi (Section 2.1; boundary-integral form, Section 2.2).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers (HIP global memory on the current
 *     device) owned by the caller unless stated otherwise; the library never
 *     frees caller memory.  Structs (bim_problem, bim_jfnk_opts, reports) live
 *     in HOST memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it in order; entry points return once the work is queued
 *     unless stated otherwise.
 *   - Vectors u, F, v, Jv, z have 3 (N+1) M FP64 entries in the order of the
 *     unknown vector (Section 3.1, eq. (unknowns)): for each field f in
 *     (zeta, phi, psi) a block of M slices, slice j = [f_{1,j}, (f_x)_{1..N,j}].
 *     The residual rows follow the order printed in Appendix B: per slice
 *     [F5, F6, F1(1..N-1)], then [F3, F4, F2(1..N-1)], then [F8, F9, F7(1..N-1)].
 *   - Node arrays are [M][N] FP64 with x fastest.
 *   - Return codes: 0 success; < 0 error (nothing useful was written);
 *     > 0 soft failure (results written, see the report).  bim_last_error()
 *     returns a message for the calling thread's last failure.
 *   - Calls are not thread-safe on a shared handle; distinct handles may be
 *     used concurrently.
 */
#ifndef BIM_H
#define BIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BIM_OK = 0,
    BIM_EINVAL = -1,   /* bad sizes, null pointers, inconsistent mesh */
    BIM_EHIP = -2,     /* a HIP runtime call failed */
    BIM_ENOMEM = -3,   /* device allocation failed */
    BIM_EDOMAIN = -4,  /* non-finite input, or a value outside the method's domain */
    BIM_NOT_CONVERGED = 1,
    BIM_LINESEARCH_FAIL = 2
};

/* Precision of the all-pairs boundary-integral sums (the rest is always FP64). */
enum { BIM_FP64 = 0, BIM_FP32C = 1 };

/*
 * One discrete problem (Section 3.1): the truncated mesh x_i = x1 + i dx
 * (i = 0..N-1), y_j = y1 + j dy (j = 0..M-1), the Froude number and the bottom.
 *   half_domain = 1: data even in y, only y >= 0 stored (y1 must be 0); the
 *                    mirror half enters every integral as an image y -> -y.
 *   half_domain = 0: the full truncated mesh (the paper's y1 = -yM, or any y1).
 *   n_decay: the upstream decay rate n of the radiation condition (0.05 in the paper).
 *   beta, beta_x, beta_y: device node arrays of the bottom and its slopes.
 * Requirements: N >= 3, M >= 3, dx > 0, dy > 0, froude > 0.
 */
typedef struct bim_problem {
    int32_t N, M;
    double x1, dx, y1, dy;
    int32_t half_domain;
    double n_decay;
    double froude;
    const double *beta, *beta_x, *beta_y;
} bim_problem;

/*
 * F = F(u): the discrete residual of Section 3.1 -- boundary-integral rows on
 * the free surface (F2) and on the bottom (F7) from eq. (new_finite_boundary_
 * integral) with the trapezoidal rule, the S2 subtraction and its closed-form
 * integral; the dynamic condition eq. (new_finite_dynamic) (F1); and the
 * radiation conditions eqs. (scullen1)-(scullen6) (F3..F6, F8, F9).
 *   u: device [3(N+1)M] input; F: device [3(N+1)M] output (must not alias u).
 *   prec: BIM_FP64, or BIM_FP32C (all-pairs sums in FP32 with compensated
 *         accumulation; reconstruction, analytic terms and assembly in FP64).
 * Scratch memory is taken from the stream-ordered allocator on `stream`.
 */
int bim_residual(const bim_problem *prob, const double *u, double *F, int prec, void *stream);

/*
 * Jv = (F(u + h v) - Fu) / h: the first-order difference quotient that
 * replaces the Jacobian action in the Krylov solver (Section 3.2).
 *   Fu: F(u) evaluated with the same `prec` (device [3(N+1)M]).
 *   h > 0: the shift; h <= 0 selects h = sqrt(eps_prec) (1 + ||u||_2) / ||v||_2
 *   with eps_prec = 2^-52 (FP64) or 2^-23 (FP32C).  If ||v|| = 0, Jv = 0.
 *   Jv must not alias u, Fu or v.
 */
int bim_jv(const bim_problem *prob, const double *u, const double *Fu, const double *v,
           double h, double *Jv, int prec, void *stream);

/* Message describing the calling thread's most recent failure ("" if none). */
const char *bim_last_error(void);

/* Library version string. */
const char *bim_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BIM_H */
