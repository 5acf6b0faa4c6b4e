// Exact linear solution of Section 4.1 (eq. (exactsoln)) on a rectangular mesh,
// by one fixed quadrature whose nodes serve every target point.
//
// For one bump of eq. (bottom) centred at (b1, b2) -- transform
// beta~(k) = eps 2 pi delta^2 exp(-k^2 delta^2 / 2), real and isotropic -- and
// xi = x - b1, eta = y - b2, the parts of eq. (exactsoln) are sums over
// quadrature nodes q of W_q f_q(xi) cos(b_q eta):
//   kind 0  the (psi, k) nodes of the first term, psi in (0, pi/2), each node
//           standing for the pair +-psi (cos(A + B) + cos(A - B) = 2 cos A cos B):
//           f = cos(a |xi|), a = k cos psi, b = k sin psi,
//           W = 2 w_psi w_k F^2 / (2 pi^2) k^2 sech(k) beta~(k) / g(k),
//           g = k F^2 - sec^2(psi) tanh k;
//   kind 1  the half-residue of the k-path below the pole k_1(psi) (the root of
//           g), folded the same way: f = sin(a |xi|), a = k_1 cos psi,
//           b = k_1 sin psi, W = 2 w_psi F^2 / (2 pi^2) pi R beta~(k_1),
//           R = k_1^2 sech k_1 / (F^2 - sec^2 psi sech^2 k_1);
//   kind 2  the downstream wave H(x): f = -H(xi) sin(a xi),
//           W = w_psi (2 F^2 / pi) R beta~(k_1).
// zeta_x uses d f / d xi (with sign(0) = 0 and H(0) = 1/2, the mean of the
// one-sided derivatives, which agree since zeta is smooth).  Several bumps add
// (the linear problem is linear in beta + 1).
//
// The principal value needs no subtraction: the pole is the centre of a
// 16-point Gauss-Legendre panel symmetric about it, on which the rule
// integrates c / (k - k_1) to zero exactly, and g is evaluated there as
// (k - k_1) [F^2 - sec^2 psi (1 - tanh k tanh k_1) tanh(k - k_1) / (k - k_1)],
// free of cancellation near the pole.  Panels hold at most `periods_per_panel`
// periods of cos(k X) for the largest |X| = |xi| + |eta| on the mesh; next to a
// small pole (F > 1 just above psi_0 = arccos(1/F)), or to the near-zero of g / k
// just below psi_0, they grow geometrically from the scale of that point; in
// psi they are as wide as the phase rates allow and graded geometrically toward
// psi_0.  The panel edges are laid out on the host (a few hundred panels); every
// node value is computed on the GPU.
//
// Kernels:
//   k_exact_nodes     one workgroup per psi node: k_1 by Newton, its k-panels
//                     and nodes (a, b, and W for every bump), kinds in three
//                     sections padded to 16 nodes
//   k_exact_contract  zeta[j][i] = sum_q L[i][q] R[j][q], L = W f(xi_i) (and
//                     W f'(xi_i) for zeta_x), R = cos(b eta_j): a dense
//                     contraction over 10^5..10^6 nodes of two operands
//                     generated 16 nodes at a time in LDS and multiplied on the
//                     FP64 matrix cores (v_mfma_f64_16x16x4), the nodes split
//                     over workgroups
//   k_exact_reduce    fixed-order sum over the node chunks (deterministic)
//   k_exact_start     an unknown vector from zeta and zeta_x
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

#include "bim_common.h"

namespace bim {
namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kGL = 16;          // Gauss-Legendre nodes per panel
constexpr int kStep = 16;        // nodes per LDS stage
constexpr int kMaxBumps = 16;

struct GL16 {
    double x[kGL], w[kGL];
};

struct Bumps {
    int n;
    double eps[kMaxBumps], delta[kMaxBumps], b1[kMaxBumps], b2[kMaxBumps];
};

// One psi node: its weight, the first of its kind-0 nodes, and the k-panel
// counts (type 0: pole panel present, nL uniform panels left of it, nG
// geometric and nR uniform right of it; type 1: no pole panel, nG geometric
// panels from 0 then nR uniform).
struct PsiNode {
    double psi, w;
    long off;
    int type, nL, nG, nR, pole;  // pole: index among the type-0 nodes
    int pad;
};

// Newton for the root of h(k) = k F^2 - sec^2 tanh k (F^2 < sec^2) from
// k = sec^2 / F^2, where h >= 0: h is convex for k > 0, so the iterates decrease
// monotonically to the root; stop once they no longer do.
__host__ __device__ inline double pole_k1(double F2, double sec2) {
    double k = sec2 / F2;
    for (int it = 0; it < 300; ++it) {
        const double t = tanh(k);
        const double h = k * F2 - sec2 * t;
        if (!(h > 0.0)) break;
        const double dh = F2 - sec2 * (1.0 - t * t);
        if (!(dh > 0.0)) break;
        const double kn = k - h / dh;
        if (!(kn < k)) break;
        k = kn;
    }
    return k;
}

__device__ inline double sech_(double k) {
    const double e = exp(-k);
    return 2.0 * e / (1.0 + e * e);
}

// k - tanh k; below 0.1 by the Taylor series of tanh (no cancellation)
__device__ inline double k_minus_tanh(double k) {
    if (k >= 0.1) return k - tanh(k);
    const double k2 = k * k;
    return k * k2 *
           (1.0 / 3 - k2 * (2.0 / 15 - k2 * (17.0 / 315 - k2 * (62.0 / 2835 - k2 * (1382.0 / 155925 -
                                                                                   k2 * 21844.0 / 6081075)))));
}

__device__ inline double bump_tr(const Bumps &bs, int b, double k) {
    const double d2 = bs.delta[b] * bs.delta[b];
    return bs.eps[b] * 2.0 * kPi * d2 * exp(-0.5 * k * k * d2);
}

// The rotation factors of one node: cos and sin of a dx and of b dy (stepping the
// operands' phases from one mesh row or column to the next).
__device__ __forceinline__ void rot_factors(double a, double b, double dx, double dy, long q, double *__restrict__ rot,
                                            long qpad) {
    double s1, c1, s2, c2;
    sincos(a * dx, &s1, &c1);
    sincos(b * dy, &s2, &c2);
    rot[q] = c1;
    rot[qpad + q] = s1;
    rot[2 * qpad + q] = c2;
    rot[3 * qpad + q] = s2;
}

__global__ __launch_bounds__(64) void k_exact_nodes(const PsiNode *__restrict__ pn, GL16 gl, Bumps bs, double F,
                                                    double K, double hk, long q1off, long q2off, long qpad,
                                                    double dx, double dy, double *__restrict__ na,
                                                    double *__restrict__ nb, double *__restrict__ nw,
                                                    double *__restrict__ rot) {
    const PsiNode P = pn[blockIdx.x];
    const double c = cos(P.psi), s = sin(P.psi), sec2 = 1.0 / (c * c), F2 = F * F;
    const bool pole = P.type == 0;
    double k1 = 0.0, d = 0.0, t1 = 0.0, w0;
    if (pole) {
        k1 = pole_k1(F2, sec2);
        d = fmin(k1, 0.5 * hk);
        t1 = tanh(k1);
        w0 = 2.0 * d;
    } else {
        w0 = (F2 > sec2) ? sqrt(3.0 * (F2 - sec2) / sec2) : 0.0;
    }
    const double g0 = pole ? k1 + d : 0.0;                   // start of the geometric panels
    const double gend = g0 + w0 * (ldexp(1.0, P.nG) - 1.0);  // and their end
    const double kend = fmax(K, gend);
    const double wL = P.nL > 0 ? (k1 - d) / P.nL : 0.0;
    const double wR = P.nR > 0 ? (kend - gend) / P.nR : 0.0;
    const int npan = P.nL + (pole ? 1 : 0) + P.nG + P.nR;
    const double scale = 2.0 * P.w * F2 / (2.0 * kPi * kPi);
    for (int t = threadIdx.x; t < kGL * npan; t += 64) {
        int r = t / kGL;
        const int g = t % kGL;
        double lo, wid;
        if (pole && r < P.nL) {
            lo = r * wL;
            wid = wL;
        } else {
            if (pole) r -= P.nL;
            if (pole && r == 0) {
                lo = k1 - d;
                wid = 2.0 * d;
            } else {
                if (pole) r -= 1;
                if (r < P.nG) {
                    lo = g0 + w0 * (ldexp(1.0, r) - 1.0);
                    wid = ldexp(w0, r);
                } else {
                    lo = gend + (r - P.nG) * wR;
                    wid = wR;
                }
            }
        }
        const double k = lo + 0.5 * (gl.x[g] + 1.0) * wid;
        const double wk = 0.5 * gl.w[g] * wid;
        double gk;
        if (pole) {
            const double dd = k - k1;
            gk = dd * (F2 - sec2 * (1.0 - tanh(k) * t1) * (tanh(dd) / dd));
        } else {
            gk = k * (F2 - sec2) + sec2 * k_minus_tanh(k);
        }
        const double base = scale * wk * k * k * sech_(k) / gk;
        const long q = P.off + t;
        na[q] = k * c;
        nb[q] = k * s;
        rot_factors(k * c, k * s, dx, dy, q, rot, qpad);
        for (int b = 0; b < bs.n; ++b) nw[b * qpad + q] = base * bump_tr(bs, b, k);
    }
    if (pole && threadIdx.x == 0) {
        const double sh = sech_(k1);
        const double R = k1 * k1 * sh / (F2 - sec2 * sh * sh);
        const long q1 = q1off + P.pole, q2 = q2off + P.pole;
        na[q1] = na[q2] = k1 * c;
        nb[q1] = nb[q2] = k1 * s;
        rot_factors(k1 * c, k1 * s, dx, dy, q1, rot, qpad);
        rot_factors(k1 * c, k1 * s, dx, dy, q2, rot, qpad);
        for (int b = 0; b < bs.n; ++b) {
            const double bt = bump_tr(bs, b, k1);
            nw[b * qpad + q1] = scale * kPi * R * bt;
            nw[b * qpad + q2] = P.w * (2.0 * F2 / kPi) * R * bt;
        }
    }
}

typedef double d4 __attribute__((ext_vector_type(4)));

// One workgroup: a 64 x 64 tile of targets (i along x, j along y) and a range of
// node steps (16 nodes of one bump each).  Wave w owns the 32 x 32 quarter
// (i half w & 1, j half w >> 1) as 2 x 2 blocks of 16 x 16 for each output.
// MFMA operand layout (v_mfma_f64_16x16x4): lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; the result block holds D[l / 16 + 4 r][l % 16] in
// element r of lane l (rows interleaved, unlike the FP32 16x16x4 form).
// Software pipeline, one barrier per step: while the matrix cores multiply
// step st out of one LDS buffer, the waves generate step st + 1 into the other
// from node data loaded during step st - 1.
// Operand generation: thread t takes node gq = t / 16 of the step and the four
// consecutive rows (and columns) 4 (t % 16) .. + 3 of the tile: one sincos at the
// first row, then three rotations by exp(+-i a dx) (the sign of the step of |xi|),
// the same for the columns with exp(i b dy); rows on both sides of the bump
// centre (|xi| not monotone) take a sincos each.
struct NodeData {
    double a, b, w, ca, sa, cb, sb;
};

__device__ __forceinline__ void load_node(const double *__restrict__ na, const double *__restrict__ nb,
                                          const double *__restrict__ nw, const double *__restrict__ rot, long qpad,
                                          long sq, long st, int gq, NodeData &nd) {
    const int bump = (int)(st / sq);
    const long q = (st - (long)bump * sq) * kStep + gq;
    nd.a = na[q];
    nd.b = nb[q];
    nd.w = nw[(long)bump * qpad + q];
    nd.ca = rot[q];
    nd.sa = rot[qpad + q];
    nd.cb = rot[2 * qpad + q];
    nd.sb = rot[3 * qpad + q];
}

// LDS row strides (doubles) of the operand buffers: 64 + 16 and JT + 16 (JT = 96:
// 112), so that the four node rows an MFMA operand read touches fall on
// alternate halves of the 64 banks (row strides of 32 mod 64 dwords).
template <int W>
struct LdsStride {
    static constexpr int value = W + 16;
};

// Generation of one step's operands: thread t takes node gq = t / 16 and the
// four rows 4 g .. 4 g + 3 (g = t % 16) of L and the JT / 16 columns
// (JT / 16) g .. of R: one sincos at the first row (column), then rotations by
// exp(+-i a dx) (the sign of the step of |xi|) and exp(i b dy); rows on both
// sides of the bump centre (|xi| not monotone) take a sincos each.
template <int JT>
__device__ __forceinline__ void gen_step(const NodeData &nd, const Bumps &bs, long sq, long st, long q1off,
                                         long q2off, double x0, double y0, double dx, double dy, int gq, int g,
                                         double (*sL)[LdsStride<64>::value], double (*sLx)[LdsStride<64>::value],
                                         double (*sR)[LdsStride<JT>::value]) {
    constexpr int RJ = JT / 16;
    const int r0 = 4 * g, c0 = RJ * g;
    const int b = (int)(st / sq);
    const long q0 = (st - (long)b * sq) * kStep;
    const int kind = q0 < q1off ? 0 : (q0 < q2off ? 1 : 2);
    const double xi0 = x0 - bs.b1[b], eta0 = y0 - bs.b2[b];
    const double a = nd.a, w = nd.w;
    double sn[4], cs[4];
    if (xi0 >= 0.0 || xi0 + 3.0 * dx <= 0.0) {
        // |xi| = |xi0| +- r dx on all four rows
        const double dir = xi0 >= 0.0 ? 1.0 : -1.0;
        const double sa = dir * nd.sa;
        sincos(a * fabs(xi0), &sn[0], &cs[0]);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            cs[r] = cs[r - 1] * nd.ca - sn[r - 1] * sa;
            sn[r] = sn[r - 1] * nd.ca + cs[r - 1] * sa;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) sincos(a * fabs(xi0 + r * dx), &sn[r], &cs[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double xi = xi0 + r * dx;
        const double sg = (xi > 0.0) ? 1.0 : (xi < 0.0 ? -1.0 : 0.0);
        double f, fx;
        if (kind == 0) {
            f = cs[r];
            fx = -a * sg * sn[r];
        } else if (kind == 1) {
            f = sn[r];
            fx = a * sg * cs[r];
        } else {  // a |xi| = a xi wherever H(xi) != 0
            const double H = (xi > 0.0) ? 1.0 : (xi == 0.0 ? 0.5 : 0.0);
            f = -H * sn[r];
            fx = -H * a * cs[r];
        }
        sL[gq][r0 + r] = w * f;
        sLx[gq][r0 + r] = w * fx;
    }
    double sy, cy;
    sincos(nd.b * eta0, &sy, &cy);
    sR[gq][c0] = cy;
#pragma unroll
    for (int r = 1; r < RJ; ++r) {
        const double c2 = cy * nd.cb - sy * nd.sb;
        sy = sy * nd.cb + cy * nd.sb;
        cy = c2;
        sR[gq][c0 + r] = cy;
    }
}

// One workgroup: a 64 x JT tile of targets (i along x, j along y) and a range of
// node steps (16 nodes of one bump each).  Wave w owns the 32 x JT/2 part
// (i half w & 1, j half w >> 1) as 2 x JT/32 blocks of 16 x 16 for each output.
// MFMA operand layout (v_mfma_f64_16x16x4): lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; the result block holds D[l / 16 + 4 r][l % 16] in
// element r of lane l (rows interleaved, unlike the FP32 16x16x4 form).
// Software pipeline, one barrier per step: while the matrix cores multiply
// step st out of one LDS buffer, the waves generate step st + 1 into the other
// from node data loaded during step st - 1.  A wider tile (JT = 96, 128) spends
// more matrix work per generated operand (the rows' L is shared by more
// columns), at the price of more padding on meshes that are not a multiple of JT.
// Two waves per SIMD are requested (registers capped at 256, the accumulators in
// ordinary VGPRs): with one, the operand generation of a wave cannot overlap the
// matrix work of another.
template <int JT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_exact_contract(
    const double *__restrict__ na, const double *__restrict__ nb, const double *__restrict__ nw,
    const double *__restrict__ rot, long qpad, long q1off, long q2off, Bumps bs, double x1, double dx, double y1,
    double dy, int tiles_i, long steps_total, long steps_per_chunk, double *__restrict__ part) {
    constexpr int SI = LdsStride<64>::value, SJ = LdsStride<JT>::value, BJ = JT / 32;
    __shared__ double sL[2][kStep][SI], sLx[2][kStep][SI], sR[2][kStep][SJ];
    const int tile = blockIdx.x, chunk = blockIdx.y;
    const int ti = tile % tiles_i, tj = tile / tiles_i;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int ih = wave & 1, jh = wave >> 1;
    d4 acc[2][2][BJ];
    for (int o = 0; o < 2; ++o)
        for (int bi = 0; bi < 2; ++bi)
            for (int bj = 0; bj < BJ; ++bj) acc[o][bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
    const long sq = qpad / kStep;  // steps per bump
    const long s0 = (long)chunk * steps_per_chunk;
    const long s1 = s0 + steps_per_chunk < steps_total ? s0 + steps_per_chunk : steps_total;
    const int gq = t >> 4, g = t & 15;  // generation: node gq, row group g
    const double x0 = x1 + (double)(ti * 64 + 4 * g) * dx;
    const double y0 = y1 + (double)(tj * JT + (JT / 16) * g) * dy;
    if (s0 < s1) {
        NodeData nd;
        load_node(na, nb, nw, rot, qpad, sq, s0, gq, nd);
        gen_step<JT>(nd, bs, sq, s0, q1off, q2off, x0, y0, dx, dy, gq, g, sL[0], sLx[0], sR[0]);
        if (s0 + 1 < s1) load_node(na, nb, nw, rot, qpad, sq, s0 + 1, gq, nd);
        __syncthreads();
        int cur = 0;
        for (long st = s0; st < s1; ++st) {
            if (st + 1 < s1) {
                gen_step<JT>(nd, bs, sq, st + 1, q1off, q2off, x0, y0, dx, dy, gq, g, sL[cur ^ 1], sLx[cur ^ 1],
                             sR[cur ^ 1]);
                if (st + 2 < s1) load_node(na, nb, nw, rot, qpad, sq, st + 2, gq, nd);
            }
#pragma unroll
            for (int ks = 0; ks < kStep / 4; ++ks) {
                const int kk = 4 * ks + (lane >> 4), r16 = lane & 15;
                double A0[2], A1[2], B[BJ];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    A0[h] = sL[cur][kk][32 * ih + 16 * h + r16];
                    A1[h] = sLx[cur][kk][32 * ih + 16 * h + r16];
                }
#pragma unroll
                for (int h = 0; h < BJ; ++h) B[h] = sR[cur][kk][(JT / 2) * jh + 16 * h + r16];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < BJ; ++bj) {
                        acc[0][bi][bj] =
                            __builtin_amdgcn_mfma_f64_16x16x4f64(A0[bi], B[bj], acc[0][bi][bj], 0, 0, 0);
                        acc[1][bi][bj] =
                            __builtin_amdgcn_mfma_f64_16x16x4f64(A1[bi], B[bj], acc[1][bi][bj], 0, 0, 0);
                    }
            }
            // one barrier: buffer cur ^ 1 is complete for the next step, and every
            // wave is done reading buffer cur before it is overwritten at st + 2
            __syncthreads();
            cur ^= 1;
        }
    }
    // partial tile, [out][j local][i local]
    double *pt = part + ((long)chunk * gridDim.x + tile) * 2 * 64 * JT;
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int il = 32 * ih + 16 * bi + (lane >> 4) + 4 * r;
                    const int jl = (JT / 2) * jh + 16 * bj + (lane & 15);
                    pt[(long)o * 64 * JT + jl * 64 + il] = acc[o][bi][bj][r];
                }
}

__global__ __launch_bounds__(256) void k_exact_reduce(const double *__restrict__ part, int chunks, int tiles,
                                                      int tiles_i, int jt, int N, int M, double *__restrict__ zeta,
                                                      double *__restrict__ zeta_x) {
    const long nm = (long)N * M;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * nm) return;
    const int o = (int)(e / nm);
    if (o == 1 && !zeta_x) return;
    const long r = e - o * nm;
    const int j = (int)(r / N), i = (int)(r % N);
    const int tile = i / 64 + (j / jt) * tiles_i;
    const long tsz = 2L * 64 * jt;
    const long loc = (long)o * 64 * jt + (j % jt) * 64 + (i % 64);
    double sum = 0.0;
    for (int c = 0; c < chunks; ++c) sum += part[((long)c * tiles + tile) * tsz + loc];
    (o ? zeta_x : zeta)[r] = sum;
}

// u from the linear solution: zeta_1 and zeta_x from the exact solution; phi_x =
// 1 - zeta / F^2 (the linear dynamic condition) and phi_1 from the radiation row
// F3; the bottom potential the uniform stream (psi_1 = x_1, psi_x = 1).
__global__ __launch_bounds__(256) void k_exact_start(const double *__restrict__ zeta,
                                                     const double *__restrict__ zeta_x, int N, int M, double x1,
                                                     double froude, double n_decay, double *__restrict__ u) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long s = N + 1;
    if (e >= s * M) return;
    const int j = (int)(e / s), c = (int)(e % s);
    const long nb = s * M;
    const double iF2 = 1.0 / (froude * froude);
    if (c == 0) {
        const double phx1 = 1.0 - zeta[(long)j * N] * iF2;
        u[e] = zeta[(long)j * N];
        u[nb + e] = x1 - x1 * (phx1 - 1.0) / n_decay;
        u[2 * nb + e] = x1;
    } else {
        const long k = (long)j * N + (c - 1);
        u[e] = zeta_x[k];
        u[nb + e] = 1.0 - zeta[k] * iF2;
        u[2 * nb + e] = 1.0;
    }
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton on P_16 from the
// Chebyshev-like guesses cos(pi (i + 3/4) / (n + 1/2)).
const GL16 &gauss_legendre16() {
    static const GL16 gl = [] {
        GL16 g{};
        const int n = kGL;
        for (int i = 0; i < n; ++i) {
            double x = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = x;
                for (int m = 2; m <= n; ++m) {
                    const double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (x * p1 - p0) / (x * x - 1.0);
                const double dx_ = p1 / dp;
                x -= dx_;
                if (std::fabs(dx_) < 1e-17) break;
            }
            g.x[i] = x;
            g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
        }
        return g;
    }();
    return gl;
}

struct Layout {
    std::vector<PsiNode> psi;
    double K, hk;
    long q0, q1off, q2off, qpad;  // kind-0 nodes; starts of the kind-1 and kind-2 sections; padded total
    int npole;
};

inline long pad16(long n) { return (n + kStep - 1) / kStep * kStep; }

// The k-panel counts of one psi node (see PsiNode).
void k_panels(double F, double psi, double K, double hk, PsiNode &P) {
    const double c = std::cos(psi), sec2 = 1.0 / (c * c), F2 = F * F;
    const bool has_pole = sec2 - F2 > 1e-14 * sec2;
    const double k1 = has_pole ? pole_k1(F2, sec2) : 0.0;
    P.nL = 0;
    double pos, w;
    if (has_pole && k1 < K + hk) {
        P.type = 0;
        const double d = std::min(k1, 0.5 * hk);
        P.nL = k1 - d > 0.0 ? (int)std::ceil((k1 - d) / hk - 1e-12) : 0;
        pos = k1 + d;
        w = 2.0 * d;
    } else {
        P.type = 1;
        pos = 0.0;
        w = F2 > sec2 ? std::sqrt(3.0 * (F2 - sec2) / sec2) : HUGE_VAL;
    }
    P.nG = 0;
    while (w < hk && pos + w < K && P.nG < 60) {
        pos += w;
        w *= 2.0;
        ++P.nG;
    }
    P.nR = (int)std::ceil(std::max(K - pos, 0.0) / hk - 1e-12);
}

int make_layout(double F, const bim_bump *bumps, int nb, double x1, double xN, double y1, double yM,
                const bim_exact_config &cfg, Layout &L) {
    const double P = cfg.periods_per_panel, decay = cfg.decay, wcap = cfg.psi_width_max, e0 = cfg.grade_start;
    const double F2 = F * F;
    double K = 0.0, Xmax = 0.0, Rmax = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double a = 0.5 * bumps[b].delta * bumps[b].delta;
        K = std::max(K, (-1.0 + std::sqrt(1.0 + 4.0 * a * decay)) / (2.0 * a));  // k + a k^2 = decay
        const double ex = std::max(std::fabs(x1 - bumps[b].b1), std::fabs(xN - bumps[b].b1));
        const double ey = std::max(std::fabs(y1 - bumps[b].b2), std::fabs(yM - bumps[b].b2));
        Xmax = std::max(Xmax, ex + ey);
        Rmax = std::max(Rmax, std::hypot(ex, ey));
    }
    Xmax = std::max(Xmax, 1e-3);
    Rmax = std::max(Rmax, 1e-3);
    const double hk = std::min(1.0, 2.0 * kPi * P / Xmax);
    // phase rate of the psi-integrands: k X over k <= K, and k_1(psi) X for the
    // pole terms while k_1 <= K + hk (their weight beyond is below exp(-decay))
    auto rate = [&](double psi) {
        const double c = std::cos(psi), sec2 = 1.0 / (c * c);
        double r = K * Rmax;
        if (sec2 - F2 > 1e-14 * sec2) {
            const double k1 = pole_k1(F2, sec2);
            if (k1 <= K + hk) {
                const double th = std::tanh(k1), sech2 = 1.0 - th * th;
                const double den = F2 - sec2 * sech2;
                if (den > 0.0) r += std::fabs(2.0 * sec2 * std::tan(psi) * th / den) * Xmax;
            }
        }
        return r;
    };
    auto width = [&](double psi) { return std::min(wcap, 2.0 * kPi * P / rate(psi)); };
    // edges from a toward b; graded: geometric widths e0, 4 e0, ... from a until the rate's width
    auto walk = [&](double a, double b, bool graded, std::vector<double> &out) {
        out.push_back(a);
        double cur = a, e = e0;
        const double sgn = b > a ? 1.0 : -1.0, lo = std::min(a, b), hi = std::max(a, b);
        for (int guard = 0; (b - cur) * sgn > 0.0; ++guard) {
            if (guard > 1000000) return fail(BIM_EDOMAIN, "exact linear solution: psi layout did not terminate");
            double w = width(cur);
            w = std::min(w, width(std::min(std::max(cur + sgn * w, lo), hi)));
            if (graded && e < w) {
                w = e;
                e *= 4.0;
            }
            double nxt = cur + sgn * w;
            if ((b - nxt) * sgn <= 0.5 * w) nxt = b;
            out.push_back(nxt);
            cur = nxt;
        }
        return (int)BIM_OK;
    };
    std::vector<double> edges;
    int rc;
    if (F < 1.0) {
        if ((rc = walk(0.0, 0.5 * kPi, false, edges))) return rc;
    } else {
        const double psi0 = std::acos(1.0 / F);
        std::vector<double> lo, hi;
        if ((rc = walk(psi0, 0.0, true, lo))) return rc;
        if ((rc = walk(psi0, 0.5 * kPi, true, hi))) return rc;
        edges.assign(lo.rbegin(), lo.rend());
        edges.insert(edges.end(), hi.begin() + 1, hi.end());
    }
    const GL16 &gl = gauss_legendre16();
    L.psi.clear();
    L.K = K;
    L.hk = hk;
    long off = 0;
    int npole = 0;
    for (size_t e = 0; e + 1 < edges.size(); ++e) {
        const double a = edges[e], b = edges[e + 1];
        for (int g = 0; g < kGL; ++g) {
            PsiNode P{};
            P.psi = a + 0.5 * (gl.x[g] + 1.0) * (b - a);
            P.w = 0.5 * gl.w[g] * (b - a);
            k_panels(F, P.psi, K, hk, P);
            P.off = off;
            P.pole = P.type == 0 ? npole++ : -1;
            off += (long)kGL * (P.nL + (P.type == 0 ? 1 : 0) + P.nG + P.nR);
            L.psi.push_back(P);
        }
    }
    L.q0 = off;
    L.npole = npole;
    L.q1off = pad16(off);
    L.q2off = L.q1off + pad16(npole);
    L.qpad = L.q2off + pad16(npole);
    return BIM_OK;
}

bim_exact_config resolve(const bim_exact_config *c) {
    bim_exact_config r{};
    r.periods_per_panel = (c && c->periods_per_panel > 0) ? c->periods_per_panel : 4.0;
    r.decay = (c && c->decay > 0) ? c->decay : 36.0;
    r.psi_width_max = (c && c->psi_width_max > 0) ? c->psi_width_max : 0.1;
    r.grade_start = (c && c->grade_start > 0) ? c->grade_start : 1e-10;
    r.workgroups = (c && c->workgroups > 0) ? c->workgroups : 2048;
    r.timing = (c && c->timing) ? 1 : 0;
    r.tile_cols = c ? c->tile_cols : 0;
    return r;
}

}  // namespace
}  // namespace bim

using namespace bim;

extern "C" int bim_exact_linear(double froude, const bim_bump *bumps, int nbumps, int N, int M, double x1,
                                double dx, double y1, double dy, double *zeta, double *zeta_x,
                                const bim_exact_config *config, bim_exact_info *info, void *stream) {
    if (!(std::isfinite(froude) && froude > 0.0))
        return fail(BIM_EDOMAIN, "exact linear solution: F must be finite and positive");
    if (std::fabs(froude - 1.0) < 1e-3)
        return fail(BIM_EDOMAIN, "exact linear solution: F within 1e-3 of 1 (the linear solution is singular at F = 1)");
    if (!bumps || nbumps < 1 || nbumps > kMaxBumps)
        return fail(BIM_EINVAL, "exact linear solution: 1 to 16 bumps (host array) required");
    for (int b = 0; b < nbumps; ++b)
        if (!(std::isfinite(bumps[b].eps) && std::isfinite(bumps[b].b1) && std::isfinite(bumps[b].b2) &&
              std::isfinite(bumps[b].delta) && bumps[b].delta > 0.0))
            return fail(BIM_EDOMAIN, "exact linear solution: bump with non-finite values or delta <= 0");
    if (N < 1 || M < 1 || (long)N * M > (1L << 28))
        return fail(BIM_EINVAL, "exact linear solution: mesh sizes must be in 1 .. 2^28 points");
    if (!(std::isfinite(x1) && std::isfinite(y1) && std::isfinite(dx) && std::isfinite(dy) && dx > 0.0 && dy > 0.0))
        return fail(BIM_EINVAL, "exact linear solution: x1, y1 finite and dx, dy > 0 required");
    if (!zeta) return fail(BIM_EINVAL, "exact linear solution: zeta must be a device pointer");
    const bim_exact_config cfg = resolve(config);
    if (!(cfg.tile_cols <= 0 || cfg.tile_cols == 64 || cfg.tile_cols == 96 || cfg.tile_cols == 128))
        return fail(BIM_EINVAL, "exact linear solution: tile_cols must be 64, 96 or 128 (or <= 0)");
    if (!(cfg.periods_per_panel <= 64.0 && cfg.decay <= 700.0 && cfg.psi_width_max <= 1.0 && cfg.grade_start < 1e-2))
        return fail(BIM_EINVAL, "exact linear solution: config outside periods_per_panel <= 64, decay <= 700, "
                                "psi_width_max <= 1, grade_start < 1e-2");
    Layout L;
    int rc = make_layout(froude, bumps, nbumps, x1, x1 + (N - 1) * dx, y1, y1 + (M - 1) * dy, cfg, L);
    if (rc) return rc;
    Bumps bs{};
    bs.n = nbumps;
    for (int b = 0; b < nbumps; ++b) {
        bs.eps[b] = bumps[b].eps;
        bs.delta[b] = bumps[b].delta;
        bs.b1[b] = bumps[b].b1;
        bs.b2[b] = bumps[b].b2;
    }
    // tile width along y: the one of 64, 96, 128 with the least padded work per
    // generated operand (padded columns x (1 + 64 / JT): the rows' operands are
    // shared by JT columns), unless the config fixes it
    int jt = cfg.tile_cols;
    if (jt <= 0) {
        double best = 1e300;
        for (int c : {64, 96, 128}) {
            const double cost = (double)((M + c - 1) / c) * c * (1.0 + 64.0 / c);
            if (cost < best - 1e-9) {
                best = cost;
                jt = c;
            }
        }
    }
    const int tiles_i = (N + 63) / 64, tiles_j = (M + jt - 1) / jt, tiles = tiles_i * tiles_j;
    const long steps_total = (long)nbumps * (L.qpad / kStep);
    long chunks = std::max(1L, std::min(steps_total, (long)(cfg.workgroups + tiles - 1) / tiles));
    const long spc = (steps_total + chunks - 1) / chunks;
    chunks = (steps_total + spc - 1) / spc;
    if (chunks > 65535) return fail(BIM_EINVAL, "exact linear solution: too many node chunks");
    const size_t npsi = L.psi.size();
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_psi = al(sizeof(PsiNode) * npsi), b_n = al(sizeof(double) * L.qpad),
                 b_w = al(sizeof(double) * L.qpad * nbumps), b_rot = al(sizeof(double) * 4 * L.qpad),
                 b_part = al(sizeof(double) * (size_t)chunks * tiles * 2 * 64 * jt);
    hipStream_t s = (hipStream_t)stream;
    char *ws = nullptr;
    if ((rc = hip_check(hipMallocAsync((void **)&ws, b_psi + 2 * b_n + b_w + b_rot + b_part, s), "hipMallocAsync")))
        return rc;
    PsiNode *d_psi = (PsiNode *)ws;
    double *na = (double *)(ws + b_psi), *nb_ = (double *)(ws + b_psi + b_n), *nw = (double *)(ws + b_psi + 2 * b_n);
    double *rot = (double *)(ws + b_psi + 2 * b_n + b_w);
    double *part = (double *)(ws + b_psi + 2 * b_n + b_w + b_rot);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    rc = [&]() -> int {
        if (cfg.timing)
            for (auto &e : ev) BIM_HIP(hipEventCreate(&e));
        if (cfg.timing) BIM_HIP(hipEventRecord(ev[0], s));
        BIM_HIP(hipMemcpyAsync(d_psi, L.psi.data(), sizeof(PsiNode) * npsi, hipMemcpyHostToDevice, s));
        BIM_HIP(hipMemsetAsync(na, 0, 2 * b_n + b_w + b_rot, s));  // padding nodes: a = b = W = 0
        hipLaunchKernelGGL(k_exact_nodes, dim3((unsigned)npsi), dim3(64), 0, s, d_psi, gauss_legendre16(), bs,
                           froude, L.K, L.hk, L.q1off, L.q2off, L.qpad, dx, dy, na, nb_, nw, rot);
        if (cfg.timing) BIM_HIP(hipEventRecord(ev[1], s));
        const dim3 cgrid(tiles, (unsigned)chunks);
        if (jt == 128)
            hipLaunchKernelGGL(k_exact_contract<128>, cgrid, dim3(256), 0, s, na, nb_, nw, rot, L.qpad, L.q1off,
                               L.q2off, bs, x1, dx, y1, dy, tiles_i, steps_total, spc, part);
        else if (jt == 96)
            hipLaunchKernelGGL(k_exact_contract<96>, cgrid, dim3(256), 0, s, na, nb_, nw, rot, L.qpad, L.q1off,
                               L.q2off, bs, x1, dx, y1, dy, tiles_i, steps_total, spc, part);
        else
            hipLaunchKernelGGL(k_exact_contract<64>, cgrid, dim3(256), 0, s, na, nb_, nw, rot, L.qpad, L.q1off,
                               L.q2off, bs, x1, dx, y1, dy, tiles_i, steps_total, spc, part);
        if (cfg.timing) BIM_HIP(hipEventRecord(ev[2], s));
        const long outs = 2L * N * M;
        hipLaunchKernelGGL(k_exact_reduce, dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, s, part, (int)chunks,
                           tiles, tiles_i, jt, N, M, zeta, zeta_x);
        BIM_HIP(hipGetLastError());
        if (cfg.timing) BIM_HIP(hipEventRecord(ev[3], s));
        // the host node table must outlive its copy
        BIM_HIP(hipStreamSynchronize(s));
        if (cfg.timing && info) {
            float c_ms = 0.f, t_ms = 0.f;
            BIM_HIP(hipEventElapsedTime(&c_ms, ev[1], ev[2]));
            BIM_HIP(hipEventElapsedTime(&t_ms, ev[0], ev[3]));
            info->contract_ms = c_ms;
            info->total_ms = t_ms;
        }
        return BIM_OK;
    }();
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    const int rf = hip_check(hipFreeAsync(ws, s), "hipFreeAsync");
    if (info) {
        if (!cfg.timing) info->contract_ms = info->total_ms = 0.0;
        info->tile_cols = jt;
        info->nodes = L.qpad;
        info->psi_nodes = (int)npsi;
        info->kcut = L.K;
        info->hk = L.hk;
        info->chunks = (int)chunks;
        info->tiles = tiles;
    }
    return rc ? rc : rf;
}

extern "C" int bim_exact_start(const bim_problem *prob, const double *zeta, const double *zeta_x, double *u_out,
                               void *stream) {
    int rc = validate(prob);
    if (rc) return rc;
    if (!zeta || !zeta_x || !u_out) return fail(BIM_EINVAL, "exact start: zeta, zeta_x and u_out must be device pointers");
    const long n = (long)(prob->N + 1) * prob->M;
    hipLaunchKernelGGL(k_exact_start, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, zeta,
                       zeta_x, prob->N, prob->M, prob->x1, prob->froude, prob->n_decay, u_out);
    return hip_check(hipGetLastError(), "exact start launch");
}
