// Internal declarations shared by the libbim translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "bim.h"

namespace bim {

// Records the message for bim_last_error() and returns `code`.
int fail(int code, const std::string &msg);
// Wraps a HIP call: on failure records "<what>: <hip error string>" and returns BIM_EHIP.
int hip_check(hipError_t e, const char *what);

#define BIM_HIP(call)                                        \
    do {                                                     \
        int _rc = ::bim::hip_check((call), #call);           \
        if (_rc != BIM_OK) return _rc;                       \
    } while (0)

// Validates a problem description; returns BIM_OK or BIM_EINVAL with a message.
int validate(const bim_problem *p);

// Largest node elevation max zeta and smallest depth min (zeta - beta) of the
// iterate u into out[0..1] (device); rows: device scratch of 2 M doubles.
int surface_extent_enqueue(const bim_problem *p, const double *u, double *rows, double *out, hipStream_t s);
// BIM_UNPHYSICAL when max_zeta exceeds the limiting height F^2 / 2 (checked
// without surface tension only) or min_depth <= 0, else BIM_OK.
int physical_status(const bim_problem *p, double max_zeta, double min_depth);

// Sizes derived from (N, M).
struct Dims {
    int N, M, nimg;
    int nblk;      // (N+1) M: one block of u or F
    int nvec;      // 3 (N+1) M
    int ntg;       // (N-1) M collocation points per boundary
    int nnode;     // N M nodes per boundary
    explicit Dims(const bim_problem *p)
        : N(p->N), M(p->M), nimg(p->half_domain ? 2 : 1), nblk((p->N + 1) * p->M),
          nvec(3 * (p->N + 1) * p->M), ntg((p->N - 1) * p->M), nnode(p->N * p->M) {}
};

// Source-node record streamed by the all-pairs kernel: position x, elevation z,
// slopes zx, zy, and the trapezoid weight w folded into the layer densities.
// Bottom records carry the outward-normal sign of Green's identity (w < 0).
template <typename T>
struct alignas(8 * sizeof(T)) SrcRec {
    T x, z, zx, zy, wD, ws, w, pad;
};

// Launch shape of the all-pairs kernel: target tiles of 64 collocation points
// on one mesh row; the source side (2 M source-row visits of N nodes, rows of
// the two boundaries interleaved) split into `chunks` equal contiguous node
// ranges (split-K over sources).  One wave per (target tile, chunk).
struct PairLaunch {
    int tpl;             // collocation rows per lane (1 or 2)
    int unroll;          // inner-loop unroll over source nodes (2, 4 or 8)
    int row_groups;      // ceil(M / tpl)
    int tiles_per_bnd;   // ceil(row_groups (N-1) / 64): 64-lane tiles per boundary
    int target_tiles;    // 2 tiles_per_bnd
    int src_rows;        // 2 M source-row visits (both images of a row in one visit)
    int chunks;          // source chunks, 1 .. 2 M N
    int blocks;          // workgroups of 4 waves
};
// tpl/unroll outside the supported set fall back to 1/4; chunks is clamped to
// [1, 2 M N].
PairLaunch pair_launch(const Dims &d, int tpl, int unroll, int chunks);
// Launch for the config fields: chunks > 0 wins, else rows_per_chunk > 0,
// else the default wave count (chunks_for_waves).
PairLaunch pair_launch_cfg(const Dims &d, int prec, const bim_pair_config &cfg);
// Chunks that give the launch about want_waves waves.
int chunks_for_waves(const Dims &d, int tpl, int unroll, long want_waves);
// The launch used by the public entry points: the autotuned choice for this
// (mesh, precision) if bim_tune_residual has run, else the default.
PairLaunch pair_launch_for(const bim_problem *p, int prec);
// Chunks giving every work item about pairs_target pairs per collocation
// point (node ranges of pairs_target / nimg nodes), to even out work items
// across the meshes of a batch.
int balanced_chunks(const Dims &d, int pairs_target);

// Spare source records after each record array (read, never used, by the
// all-pairs prefetch at the end of a row).
constexpr int kRecPad = 8;

// One problem of a residual evaluation: the arguments of its node-level
// kernels (unpack, records, finalize) and of its all-pairs work.  Passed by
// value to the single-problem kernels; a batched evaluation keeps an array of
// them in device memory.  tg points at the T-precision collocation records of
// the all-pairs sums (tg64 or tg32).
struct PairDesc {
    void *srcS;
    void *srcB;
    const void *tg;
    double *tg64;  // FP64 collocation records (y* for the per-row t)
    double *part;
    int N, M, nimg;
    double y1, dx, dy;
    int tiles_per_bnd, row_groups, target_tiles, chunks;
    long item0;  // index of this problem's first work item in the batch
    long batch_items;  // work items of the whole batch (the same in every descriptor of a batch)
    int active;        // 0: the problem takes no part in this evaluation (no work items, no rows)
    // node-level kernels
    const double *u;
    double *F;
    double *nodes, *ydiv;
    float *tg32;
    const double *beta, *beta_x, *beta_y;
    double x1, n_decay, froude, tau;
    int half, linear;
    int blk_int, blk_rec, blk_fin;  // first workgroup of this problem in each batched node-level launch
};

// Device workspace of one residual evaluation.
struct ResidualWork {
    double *nodes;   // [3][M][N]  zeta, phi, psi at the nodes
    double *ydiv;    // [2][M][N]  zeta_y, phi_y at the nodes
    double *tg;      // [8][2 ntg] x*, y*, d, D*, A, B, C, sigma* (FP64)
    float *tg32;     // [7][2 ntg] FP32 copies for the FP32C kernel
    void *srcS;      // SrcRec<T>[nnode]
    void *srcB;      // SrcRec<T>[nnode]
    double *part;    // [chunks][2 ntg][2]
    double *scal;    // [4] device scalars (h, norms)
    size_t bytes;
};
size_t residual_work_bytes(const Dims &d, const PairLaunch &pl);
void residual_work_carve(void *base, const Dims &d, const PairLaunch &pl, ResidualWork *w);

// Enqueues F = F(u) using a caller-provided workspace (no allocation).
// ev_pair (optional): two events recorded right before and after the all-pairs launch.
// linear = 1 evaluates the linearised residual F_lin of Section 4.2 instead.
int residual_enqueue(const bim_problem *p, const double *u, double *F, int prec,
                     const PairLaunch &pl, const ResidualWork &w, hipStream_t s,
                     hipEvent_t *ev_pair = nullptr, int linear = 0);

// Enqueues F_i = F(u_i) for `count` problems whose all-pairs sums share one
// persistent launch.  pls[i] must have the same tpl/unroll for every i; ws[i]
// is problem i's workspace; descs_dev: device array of `count` PairDesc.
// max_blocks caps the persistent grid (<= 0: 2048 workgroups).
int residual_batched_enqueue(const bim_problem *probs, int count, const double *const *u, double *const *F,
                             int prec, const PairLaunch *pls, const ResidualWork *ws, PairDesc *descs_dev,
                             int max_blocks, hipStream_t s, hipEvent_t *ev_pair = nullptr);

// The batched residual split into a host part and a launch of fixed shape, so
// that one captured graph serves every evaluation of a batch whatever subset of
// its problems takes part (the descriptors are rewritten before each replay):
//   residual_batched_fill writes the descriptors of all `count` problems into
//   host memory (u[i], F[i] of an inactive problem may be NULL) and returns
//   the total number of work items of the active ones;
//   residual_batched_launch enqueues the four kernels over the descriptors
//   already in device memory, with grids sized for all problems active.
struct BatchShape {
    int tpl, unroll;
    int b_int, b_rec, b_fin;  // node-level workgroups of all problems
    int blocks;               // persistent all-pairs grid
};
BatchShape residual_batched_shape(const bim_problem *probs, int count, const PairLaunch *pls, int max_blocks);
int residual_batched_fill(const bim_problem *probs, int count, const int *active, const double *const *u,
                          double *const *F, int prec, const PairLaunch *pls, const ResidualWork *ws,
                          PairDesc *descs_host, long *total_items);
int residual_batched_launch(const PairDesc *descs_dev, int count, int prec, const BatchShape &shape, hipStream_t s,
                            hipEvent_t *ev_pair = nullptr);

}  // namespace bim
