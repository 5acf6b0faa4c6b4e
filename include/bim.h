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

#include <stddef.h>
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
    BIM_LINESEARCH_FAIL = 2,
    BIM_UNPHYSICAL = 3  /* solver: the last iterate rises above the limiting height F^2/2
                           (Bernoulli's equation with a stagnant crest; not checked with surface
                           tension) or the surface reaches the bottom (zeta - beta <= 0) */
};

/* Precision of the all-pairs boundary-integral sums (the rest is always FP64). */
enum { BIM_FP64 = 0, BIM_FP32C = 1 };
/* Storage of the preconditioner's operator (precond_setup_ex): FP64, or FP32
 * elements applied with FP64 products and sums. */
enum { BIM_STORE_FP64 = 0, BIM_STORE_FP32 = 1 };

/*
 * One discrete problem (Section 3.1): the truncated mesh x_i = x1 + i dx
 * (i = 0..N-1), y_j = y1 + j dy (j = 0..M-1), the Froude number and the bottom.
 *   half_domain = 1: data even in y, only y >= 0 stored (y1 must be 0); the
 *                    mirror half enters every integral as an image y -> -y.
 *   half_domain = 0: the full truncated mesh (the paper's y1 = -yM, or any y1).
 *   n_decay: the upstream decay rate n of the radiation condition (0.05 in the paper).
 *   beta, beta_x, beta_y: device node arrays of the bottom and its slopes.
 *   tau: surface-tension parameter T / (rho U^2 H) (Section 6); 0 for the
 *        gravity-wave problem of the paper.  With tau != 0 the dynamic condition
 *        gains -tau K, K twice the mean curvature of the free surface
 *        (div(grad zeta / sqrt(1 + |grad zeta|^2))), and the linearised one
 *        -tau (zeta_xx + zeta_yy); second y-differences are central inside,
 *        mirrored on the symmetry line of a half domain and one-sided
 *        (four points) on an outer edge, so M >= 4 is required.
 * Requirements: N >= 3, M >= 3, dx > 0, dy > 0, froude > 0, tau finite.
 */
typedef struct bim_problem {
    int32_t N, M;
    double x1, dx, y1, dy;
    int32_t half_domain;
    double n_decay;
    double froude;
    const double *beta, *beta_x, *beta_y;
    double tau;
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
 * Scratch memory: a workspace kept by the library per (device, stream) and
 * reused in stream order by later calls on that stream (see
 * bim_release_workspaces); it grows, with a synchronisation of `stream`, when a
 * call needs more.  Calls from several host threads are serialised while they
 * enqueue.  A call captured into a graph needs a workspace of sufficient size
 * from an earlier call on the same stream.
 */
int bim_residual(const bim_problem *prob, const double *u, double *F, int prec, void *stream);

/*
 * F_lin(u): the residual of the linearised problem (Section 4.2, Appendix B),
 * the operator whose root is the linear start.  The same discretisation and
 * unknowns as bim_residual, with both boundaries the planes z = 0 and z = -1
 * (zero slopes and elevations in the kernels; the layer densities phi - x,
 * zeta_x on the free surface and psi - x, -beta_x on the bottom are unchanged)
 * and the dynamic condition phi*_x + zeta* / F^2 - 1 = 0.  F_lin is affine in u.
 * Arguments, layout, precision, scratch memory and errors as bim_residual.
 */
int bim_residual_linear(const bim_problem *prob, const double *u, double *F, int prec, void *stream);

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

/*
 * Frees the workspaces bim_residual and bim_jv keep per (device, stream), after
 * waiting for the work of every stream that used one.  Later calls allocate
 * again.  Must not run concurrently with other calls of the library.
 */
int bim_release_workspaces(void);

/*
 * F = F(u) without any allocation: for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Computes exactly what bim_residual computes (FP64 or
 * FP32C sums, same kernels), with its workspace carved out of a fixed device
 * array of bim_residual_noalloc_max_bytes() bytes (64 MiB) that the library
 * holds on every GPU it runs on until the process ends; the array's device
 * address is looked up once per device, on the first call made with that
 * device current.  The call allocates nothing, frees nothing and never
 * synchronises.
 *   u, F, prec: as bim_residual.
 * Size limit: the default launch is used while its workspace fits (27.5 MiB
 * FP64 and 35.5 MiB FP32C at 181 x 61); a larger mesh runs with fewer source
 * chunks, so that its partial sums fit, giving the same sums rounded in a
 * different order; a mesh whose workspace does not fit even with one chunk
 * (about 178,000 nodes per boundary, e.g. 730 x 244) is rejected with
 * BIM_EINVAL before anything is enqueued.
 * Every call on one GPU uses the same array, and each call overwrites every
 * byte of it that it later reads: calls that may overlap on one GPU (two
 * streams, two host threads) race and must be ordered by the caller.
 */
int bim_residual_noalloc(const bim_problem *prob, const double *u, double *F, int prec, void *stream);
/* Size in bytes of the fixed device array used by bim_residual_noalloc. */
size_t bim_residual_noalloc_max_bytes(void);

/*
 * Launch shape of the all-pairs kernel (the sums of the boundary-integral rows).
 * The source side (2 M source-row visits of N nodes each, both boundaries) is
 * split into `chunks` contiguous, equal ranges of nodes (a range may start and
 * end inside a row); every (target tile, chunk) pair is one wave.
 *   targets_per_lane: collocation rows handled by one lane (1 or 2);
 *   unroll:           unroll depth of the loop over source nodes (2, 4 or 8);
 *   rows_per_chunk:   if chunks <= 0: chunks = ceil(2 M / rows_per_chunk);
 *   chunks:           number of source chunks (> 0 overrides rows_per_chunk).
 * With both <= 0 the library picks the chunk count that gives the launch about
 * 24 (FP64) or 32 (FP32C) waves per SIMD of the GPU (24576 or 32768 waves).
 */
typedef struct bim_pair_config {
    int32_t targets_per_lane;
    int32_t unroll;
    int32_t rows_per_chunk;
    int32_t chunks;
} bim_pair_config;

/*
 * Measurement aid for benchmarks: enqueues `iters` evaluations of F(u) (as
 * bim_residual) on `stream` with HIP events recorded on that stream around
 * every launch of the all-pairs kernel and around every whole evaluation,
 * waits for them, and returns the average durations in *kernel_ms and
 * *total_ms (host pointers).  cfg (host, may be NULL) forces a launch shape;
 * NULL uses the one bim_residual would use.
 */
int bim_residual_timed(const bim_problem *prob, const double *u, double *F, int prec, int iters,
                       const bim_pair_config *cfg, void *stream, double *kernel_ms, double *total_ms);

/*
 * Autotuner: times the all-pairs kernel for every supported launch shape on
 * this mesh and precision (with u as the evaluation point), remembers the
 * fastest for all later calls in this process with the same (N, M,
 * half_domain, prec), and returns it in *best (host, may be NULL) with its
 * kernel time in *best_ms (host, may be NULL).  Synchronises the stream.
 */
int bim_tune_residual(const bim_problem *prob, const double *u, int prec, void *stream,
                      bim_pair_config *best, double *best_ms);

/*
 * Preconditioner P (Section 4.2; Appendix A): the Jacobian J~ of the
 * linearised discrete problem (Appendix B, with the bottom single layer
 * entering with density -beta_x as in the residual), with its four dense
 * blocks kept only within a band of slices |m - l| <= band_halfwidth
 * ("b blocks of size (N+1) x (N+1) in each row", b = 2 band_halfwidth + 1).
 * P depends only on the mesh and F (not on u or the bottom).
 *   band_halfwidth < 0 selects max(1, min(10, round(M / 6))) (b ~ M/3 blocks up
 *   to 21: wider than the b ~ M/10 of Table 1, because GMRES iterations per
 *   Newton step fall several-fold for a modest rise in setup and apply cost;
 *   beyond 10 slices the setup grows faster than the solve shrinks).
 * precond_setup factors P on the device and returns a library-owned handle
 * (free with precond_destroy).  It synchronises `stream`; part of the work runs
 * on a second stream of its own (default priority), joined before it returns,
 * so it must not be called under stream capture.  Device memory used:
 * precond_bytes().  Requires N + 1 <= 1024.  Returns BIM_EDOMAIN if a block
 * that must be inverted is singular.
 * precond_apply enqueues z = P^-1 r (device vectors of 3(N+1)M, z must not
 * alias r).  Applies on one handle share its scratch: do not overlap them.
 */
typedef struct bim_precond bim_precond;
int precond_setup(const bim_problem *prob, int band_halfwidth, bim_precond **out, void *stream);
/*
 * precond_setup with the storage of the factored operator: BIM_STORE_FP64 (as
 * precond_setup), or BIM_STORE_FP32: the arrays the apply reads (the banded
 * blocks, the replicated diagonal inverses, the triangular inverses of the
 * Schur complement's block LU and its inverse pivot blocks) are held in FP32,
 * halving the apply's memory traffic and precond_bytes().  The block
 * elimination and the block LU run in FP64; for 128 < N + 1 <= 384 the
 * substitutions that form the triangular inverses run in FP32 on FP32 copies
 * of the factors, otherwise the FP64 inverses are rounded.  The apply still
 * forms its products and sums in FP64.  The rounding of the elements is
 * amplified by the conditioning of the Schur complement: the apply differs
 * from the FP64 one by ~1e-3 relative at 181 x 61.  GMRES sees a different but
 * about equally good preconditioner; the Newton residual, and so the
 * solution, is unchanged.  Returns BIM_EINVAL for any other storage value.
 */
int precond_setup_ex(const bim_problem *prob, int band_halfwidth, int storage, bim_precond **out, void *stream);
int precond_storage(const bim_precond *P);
int precond_apply(const bim_precond *P, const double *r, double *z, void *stream);
void precond_destroy(bim_precond *P);
int64_t precond_bytes(const bim_precond *P);
int precond_band(const bim_precond *P);

/*
 * Options of the Jacobian-free Newton-Krylov solver (Section 3.2).
 *   ftol:           stop when ||F(u)||_inf <= ftol (FP64 residual);
 *   gmres_rtol:     relative residual tolerance of each linear solve;
 *   restart:        GMRES restart length m (Krylov basis of m + 1 vectors);
 *   max_restarts:   restarts per linear solve;
 *   max_newton:     Newton steps;
 *   max_backtracks: halvings of the step length mu in the line search
 *                   (accept when ||F(u + mu du)||_2 <= (1 - 1e-4 mu) ||F(u)||_2);
 *   inner_prec:     precision of the all-pairs sums inside the Jacobian-vector
 *                   products (BIM_FP64 or BIM_FP32C); the Newton residual,
 *                   the line search and the update are always FP64;
 *   band_halfwidth: band of the preconditioner built when none is passed;
 *   use_precond:    0 runs GMRES without preconditioning;
 *   use_graphs, fd_eps, stall_steps, fp64_below, fp32c_gmres_rtol: see the fields.
 * jfnk_default_opts fills 1e-10, 1e-8, 30, 10, 30, 20, BIM_FP64, -1, 1, 1, 0.0, 0,
 * 0.0, 1e-2, BIM_STORE_FP64.
 * Invalid values (non-positive tolerances, restart outside [1, 200], negative
 * counts, fd_eps >= 1 or NaN, negative or NaN fp64_below, unknown precision
 * or storage)
 * give BIM_EINVAL.
 */
typedef struct bim_jfnk_opts {
    double ftol;
    double gmres_rtol;
    int32_t restart;
    int32_t max_restarts;
    int32_t max_newton;
    int32_t max_backtracks;
    int32_t inner_prec;
    int32_t band_halfwidth;
    int32_t use_precond;
    int32_t use_graphs;  /* 1: replay each Arnoldi step's device work from a HIP graph */
    double fd_eps;       /* epsilon of the shift rule h = sqrt(eps)(1 + |u|)/|v|; <= 0: the
                            unit roundoff of the inner precision (2^-52 or 2^-23) */
    int32_t stall_steps; /* s > 0: stop (BIM_NOT_CONVERGED) once ||F||_inf has not halved over
                            the last s Newton steps; 0: no such stop */
    double fp64_below;   /* with inner_prec BIM_FP32C: a Newton step taken at ||F||_inf <=
                            fp64_below uses FP64 inner sums (the FP32 sums' rounding limits the
                            Jacobian action once F is small); 0: never.  Ignored for FP64. */
    double fp32c_gmres_rtol; /* relative tolerance of the GMRES solves of Newton steps that use
                            FP32C inner sums (their Jacobian action carries rounding noise of
                            order 1e-6 relative, below which GMRES stalls): the effective
                            tolerance is max(this, gmres_rtol); default 1e-2, the contraction
                            Newton reaches per FP32C step anyway; <= 0: gmres_rtol */
    int32_t precond_storage; /* storage of a preconditioner the solver builds itself (P == NULL):
                            BIM_STORE_FP64 or BIM_STORE_FP32 (see precond_setup_ex) */
} bim_jfnk_opts;

/* Outcome of a solve (host struct).  history[k] = ||F||_inf after k Newton steps. */
typedef struct bim_jfnk_report {
    int32_t status;               /* return code of the solve */
    int32_t newton_iters;
    int32_t gmres_iters;          /* total Krylov iterations */
    int32_t residual_evals;       /* FP64 residual evaluations (Newton + line search) */
    int32_t inner_residual_evals; /* base evaluations F(u) in the inner precision */
    int32_t jv_evals;             /* Jacobian-vector products (one residual each) */
    int32_t backtracks;
    double fnorm_inf;             /* final ||F||_inf */
    double fnorm0_inf;            /* initial ||F||_inf */
    double gmres_relres_last;     /* relative residual estimate of the last linear solve */
    double time_ms;               /* wall time of the call, preconditioner setup included */
    double precond_ms;            /* preconditioner setup time (0 if one was passed) */
    double history[64];
    double max_zeta;              /* largest node elevation of the last iterate */
    double min_depth;             /* smallest zeta - beta over the nodes of the last iterate */
} bim_jfnk_report;

void jfnk_default_opts(bim_jfnk_opts *opts);

/*
 * Solves F(u) = 0 by damped inexact Newton (Section 3.2): each step solves
 * J(u) du = -F(u) by restarted GMRES with right preconditioning by P, where
 * J(u) v is the difference quotient of bim_jv (shift sqrt(eps)(1+||u||)/||v||,
 * eps of the inner precision), then backtracks on the step length.
 *   P: a preconditioner from precond_setup for this problem, or NULL to build
 *      one internally (timed in rep->precond_ms).
 *   u: device [3(N+1)M], the start on entry, the last iterate on exit.
 *   opts: NULL for the defaults.  rep: host, may be NULL.
 * Synchronises `stream` repeatedly (the host takes the Newton and Krylov
 * decisions).  Returns BIM_OK when ||F||_inf <= ftol, BIM_NOT_CONVERGED after
 * max_newton steps (or on the stall stop), BIM_LINESEARCH_FAIL when no step
 * length decreases ||F||, BIM_EDOMAIN on a non-finite residual, and
 * BIM_UNPHYSICAL (in place of any of the first three) when the last iterate
 * rises above F^2/2 or reaches the bottom (rep->max_zeta, rep->min_depth).
 */
int jfnk_solve(const bim_problem *prob, const bim_precond *P, double *u, const bim_jfnk_opts *opts,
               bim_jfnk_report *rep, void *stream);

/*
 * The discrete linear solution used as the Newton start: u_lin = u0 -
 * J~^-1 F_lin(u0), where u0 is the uniform stream (zeta = 0, phi = psi = x) and
 * F_lin the linearised residual (Section 4.2, Appendix B): the same
 * discretisation on the planes z = 0 and z = -1, forced by beta_x.  Solved by
 * GMRES preconditioned with P (NULL: built internally) to relative tolerance
 * rtol (<= 0: 1e-12).  u_out: device [3(N+1)M].
 */
int bim_linear_start(const bim_problem *prob, const bim_precond *P, double *u_out, double rtol, void *stream);
/*
 * bim_linear_start with the precision of the linear operator's products: prec =
 * BIM_FP64 (as bim_linear_start) or BIM_FP32C (the products of J~ use FP32C
 * sums; the right-hand side F_lin(u0) stays FP64).  The FP32C operator resolves
 * about 1e-6 relative, so rtol should not be set below ~1e-5.  The start only
 * seeds Newton, which then converges on the FP64 residual.
 */
int bim_linear_start_ex(const bim_problem *prob, const bim_precond *P, double *u_out, double rtol, int prec,
                        void *stream);

/*
 * Bottom pressure and the force on the topography (Section 2.1, eq.
 * (bottompressure)): once u is solved, Bernoulli's equation on z = beta gives
 *   p = 1/2 - [(1 + b_x^2) psi_y^2 + (1 + b_y^2) psi_x^2 - 2 b_x b_y psi_x psi_y]
 *             / (2 (1 + b_x^2 + b_y^2)) - beta / F^2
 * at every bottom node.  psi is reconstructed from u as phi is for the residual
 * (trapezoidal x-integral of psi_x from psi_1; psi_y by the same y-differences
 * as zeta_y and phi_y).  The force on the topography is the plan-area integral
 * of (p - 1/F^2) (beta_x, beta_y, -1) -- the pressure beyond that of the
 * undisturbed stream, along the fluid's outward normal times the area element
 * -- by the trapezoidal rule over the truncated mesh (over the mirrored mesh on
 * a half domain, where the y-component is zero by symmetry).
 *   u: device [3(N+1)M]; pres: device [M][N] output; force: device [3] output
 *   (Fx, Fy, Fz), summed in a fixed order (deterministic).
 * Uses stream-ordered scratch of about 8 N M bytes.
 */
int bim_bottom_pressure(const bim_problem *prob, const double *u, double *pres, double *force, void *stream);

/*
 * Exact solution of the linear problem (Section 4.1, eq. (exactsoln)) for a
 * topography that is a sum of Gaussian bumps of eq. (bottom),
 *   beta + 1 = sum_b eps_b exp(-((x - b1_b)^2 + (y - b2_b)^2) / (2 delta_b^2)),
 * evaluated on the mesh x_i = x1 + i dx (i < N), y_j = y1 + j dy (j < M).
 * Each bump's solution is eq. (exactsoln) with its transform
 * eps 2 pi delta^2 exp(-k^2 delta^2 / 2), shifted to its centre; the linear
 * problem being linear in beta + 1, they add.  The k-path below the pole k_1 is
 * the principal value plus the half-residue pi R sin(k_1 X) (the sign for which
 * zeta vanishes upstream); the downstream wave H(x) is as printed.
 * Quadrature: 16-point Gauss-Legendre panels in psi over (0, pi/2) (each node
 * standing for +-psi) and in k over [0, K], K the root of
 * k + k^2 delta^2 / 2 = decay for the widest transform; the pole at the centre
 * of a symmetric panel; panels hold at most periods_per_panel periods of the
 * oscillation at the mesh's largest |x - b1| + |y - b2|; geometric grading
 * next to small poles and toward psi_0 = arccos(1/F) (F > 1).  Accuracy about
 * 1e-15 (F < 1) to 1e-11 (F > 1) of eps with the defaults.  All node values and
 * sums on the GPU (FP64; the contraction over nodes on the matrix cores); the
 * host lays out the panel edges.
 *   bumps: host array of nbumps (1..16); zeta: device [M][N] output (x
 *   fastest); zeta_x: device [M][N] output of d zeta / dx, or NULL.
 *   config: host, may be NULL (defaults); info: host, may be NULL.
 * Errors: BIM_EDOMAIN for F not finite and positive, |F - 1| < 1e-3 (the linear
 * solution is singular at F = 1), or a bump with delta <= 0 or non-finite
 * values; BIM_EINVAL for bad sizes or pointers.  Uses stream-ordered scratch
 * (node table, 8 (6 + nbumps) bytes per node, and per-chunk partial tiles of
 * 2 x 64 x tile_cols doubles) and synchronises `stream` before it returns.
 */
typedef struct bim_bump {
    double eps;    /* height (negative: a crater) */
    double delta;  /* width, > 0 */
    double b1, b2; /* centre */
} bim_bump;

typedef struct bim_exact_config {
    double periods_per_panel; /* <= 0: 4 */
    double decay;             /* <= 0: 36 (k-cutoff where the transform is exp(-decay) of its scale) */
    double psi_width_max;     /* <= 0: 0.1 */
    double grade_start;       /* <= 0: 1e-10 (first graded psi panel next to psi_0) */
    int32_t workgroups;       /* <= 0: about 2048 for the contraction */
    int32_t timing;           /* 1: time the contraction kernel and the whole call with HIP events */
    int32_t tile_cols;        /* targets along y per workgroup tile: 64, 96 or 128; <= 0: chosen for M */
} bim_exact_config;

typedef struct bim_exact_info {
    int64_t nodes;      /* quadrature nodes (padded to 16 per kind) */
    int32_t psi_nodes;  /* psi nodes over (0, pi/2) */
    int32_t chunks;     /* node chunks of the contraction */
    int32_t tiles;      /* 64 x tile_cols target tiles */
    double kcut, hk;    /* k cutoff and k-panel width bound */
    double contract_ms; /* with timing: the contraction kernel */
    double total_ms;    /* with timing: the whole evaluation */
    int32_t tile_cols;  /* the tile width used */
} bim_exact_info;

int bim_exact_linear(double froude, const bim_bump *bumps, int nbumps, int N, int M, double x1, double dx,
                     double y1, double dy, double *zeta, double *zeta_x, const bim_exact_config *config,
                     bim_exact_info *info, void *stream);

/*
 * A start for Newton from the exact linear solution on the problem's mesh (the
 * mesh of bim_exact_linear's zeta, zeta_x): zeta_1 and zeta_x from it; phi_x =
 * 1 - zeta / F^2 (the linear dynamic condition, eq. (linear_dynamic)) and phi_1
 * from the radiation row F3; the bottom potential that of the uniform stream
 * (psi_1 = x1, psi_x = 1).
 *   zeta, zeta_x: device [M][N]; u_out: device [3(N+1)M].
 */
int bim_exact_start(const bim_problem *prob, const double *zeta, const double *zeta_x, double *u_out,
                    void *stream);

/*
 * F_i = F(u_i) for `count` problems (possibly of different mesh sizes) whose
 * all-pairs sums run in one persistent launch: the work items of all problems
 * form one list that every wave walks with a fixed stride, so each F_i is
 * deterministic and independent of the other problems in the batch.
 *   probs: host array of `count` problems; u, F: host arrays of device pointers.
 */
int bim_residual_batched(const bim_problem *probs, int count, const double *const *u, double *const *F,
                         int prec, void *stream);

/*
 * Solves `count` problems of possibly different mesh sizes together (a
 * parameter sweep).  Each problem follows the algorithm of jfnk_solve; the
 * problems advance in lockstep rounds in which every unfinished problem needs
 * one residual evaluation, and the all-pairs sums of all of them run in one
 * persistent launch (bim_residual_batched).  A problem that fails does not stop
 * the others.  A round is a fixed sequence of launches whose shapes do not
 * depend on the round (op lists with one slot per problem, residual launches
 * sized for every problem, inactive slots doing nothing); the host writes the
 * round's descriptors into pinned memory and, with opts->use_graphs (the
 * default), replays one HIP graph captured at the first round -- the copy of
 * the descriptors, every GMRES, preconditioner and residual kernel, and the copy
 * of the small results back -- so each round is one graph launch.  Graph replay
 * and eager launches (use_graphs = 0) give identical results.
 *   probs: host array; Ps: host array of preconditioners (or NULL entries /
 *   a NULL array to build them internally); no preconditioner may appear twice
 *   (each problem writes its preconditioner's apply scratch); us: host array of
 *   distinct device vectors (start in, last iterate out); opts: NULL for
 *   defaults (restart <= 30); reps: host array of `count` reports (may be NULL).
 *   Duplicate preconditioners or vectors: BIM_EINVAL.
 * Returns the most negative status among the problems, else the largest soft
 * status, else BIM_OK.
 */
int jfnk_solve_batched(const bim_problem *probs, int count, bim_precond *const *Ps, double *const *us,
                       const bim_jfnk_opts *opts, bim_jfnk_report *reps, void *stream);

/*
 * Learned initial guess (the network of the learned-start extension; not in
 * the paper).  A small network -- two 3x3 stride-2 convolutions with ReLU, a
 * fully connected ReLU layer that also sees F, and a linear fully connected
 * output -- maps (F, the bottom beta on the N x M mesh) and, with in_linear,
 * the discrete linear start's (zeta_x, phi_x) to a correction (dzeta_x,
 * dphi_x) of the linear start.  The upstream values f_1 and the psi block are
 * the linear start's.  Weights are FP32 masters with bf16 copies; every
 * contraction runs on bf16 matrix cores with FP32 accumulation.
 *   Input X0: device bf16 [B][M][N][C0], C0 = 2 + 2 in_linear (channels
 *   (beta+1)/0.3, (F-1.25)/0.75 and, with in_linear, zeta_x/0.2,
 *   (phi_x-1)/0.2 of the linear start); ffeat: device FP32 [B] ((F-1.25)/0.75);
 *   targets T / outputs Y: device FP32 [B][2][M][N] (correction / out_scale).
 *   Layer l's weights are [fan_in][fan_out] FP32 (conv fan_in ordered
 *   (ky, kx, c_in)).  Errors: BIM_EINVAL for sizes that do not match the
 *   network or batches above max_batch.
 */
typedef struct lg_arch {
    int32_t W, H;      /* mesh N (x) and M (y) */
    int32_t C1, C2;    /* convolution channels */
    int32_t D3;        /* hidden width */
    int32_t in_linear; /* 1: the linear start's (zeta_x, phi_x) are input channels */
    double out_scale;  /* output units */
} lg_arch;
typedef struct lg_net lg_net;
void lg_default_arch(lg_arch *arch, int N, int M);
int lg_create(const lg_arch *arch, uint64_t seed, int max_batch, lg_net **out);
void lg_destroy(lg_net *net);
int lg_num_params(const lg_net *net, int layer, int64_t *weights, int64_t *biases);
int lg_set_params(lg_net *net, int layer, const float *w_host, const float *b_host);
/* host copies of layer parameters and of the last backward pass's gradients (any may be NULL) */
int lg_get_params(const lg_net *net, int layer, float *w_host, float *b_host, float *gw_host, float *gb_host);
int lg_forward(lg_net *net, const uint16_t *X0, const float *ffeat, int B, float *Y_out, void *stream);
/* forward, mean-squared-error loss against T, backward, and (update != 0) one Adam step (lr);
   *loss_out (host, may be NULL) receives the loss (synchronises). */
int lg_train_step(lg_net *net, const uint16_t *X0, const float *ffeat, const float *T, int B, float lr, int update,
                  float *loss_out, void *stream);
/* network input of one problem (X0 [M][N][2 + 2 in_linear] bf16, ffeat [1]); u_lin
   (device, the linear start in the unknown vector's order) is read when in_linear = 1 */
int lg_make_input(const bim_problem *prob, const double *u_lin, int in_linear, uint16_t *X0, float *ffeat,
                  void *stream);
/* Newton start: the linear start (bim_linear_start with P) plus the network's correction. */
int lg_infer_start(lg_net *net, const bim_problem *prob, const bim_precond *P, double *u_out, void *stream);

/* Message describing the calling thread's most recent failure ("" if none). */
const char *bim_last_error(void);

/* Library version string. */
const char *bim_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BIM_H */
