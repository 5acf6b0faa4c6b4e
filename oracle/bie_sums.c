/*
 * Plain FP64 CPU oracle for the boundary-integral sums of the discretised
 * integral equation (Section 2.2, eq. (new_finite_boundary_integral) with the
 * kernels K1, K2; Section 3.1 trapezoidal rule and the subtraction of the
 * singular part S2 of I2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; it exists to check the GPU path.  It is deliberately slow and
 * plain: one target at a time, every source node and image, libm sqrt, no
 * blocking or reordering beyond the textbook double loop.
 *
 * For every target r (a collocation point on the free surface or on the
 * bottom) it returns five raw trapezoidal sums over the truncated mesh
 * (weights w_ij = dx dy c_i c_j, c = 1/2 on the edges, 1 inside):
 *
 *   out[5r+0] = sum_S  w (D_S - [self==0] D*) K1(zeta; d)     double layer over S
 *   out[5r+1] = sum_S  w sigma_S K2(zeta; d)                  single layer over S
 *   out[5r+2] = sum_B  w (D_B - [self==1] D*) K1(beta; d)     double layer over B
 *   out[5r+3] = sum_B  w sigma_B K2(beta; d)                  single layer over B
 *   out[5r+4] = sum_self w (A s^2 + B s t + C t^2)^(-1/2)     singular kernel S2
 *
 * with s = x - x*, t = y - y*, K1(a; d) = (a - d - s a_x - t a_y) / R^3,
 * K2(a; d) = 1 / R, R^2 = s^2 + t^2 + (a - d)^2  (the kernels of Section 2.2).
 * The signs with which these sums enter the residual are applied by the
 * caller.  When `half` is nonzero the mesh holds y >= 0 of data that are even
 * in y; the mirror half is added as an image with y -> -y and a_y -> -a_y
 * (so the sum runs over the full mirrored mesh).
 * With absmode nonzero every term is replaced by its absolute value, which
 * gives the magnitude sum_|term| used to scale comparison tolerances.
 */
#include <math.h>
#include <stddef.h>

void oracle_bie_sums(int N, int M, double x1, double dx, double y1, double dy, int half,
                     const double *zs, const double *zsx, const double *zsy,
                     const double *Ds, const double *sigs,
                     const double *zb, const double *zbx, const double *zby,
                     const double *Db, const double *sigb,
                     int T, const double *tx, const double *ty, const double *td,
                     const double *tD, const double *tA, const double *tB, const double *tC,
                     const int *tself, int absmode, double *out)
{
    const int nimg = half ? 2 : 1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int r = 0; r < T; ++r) {
        const double xs = tx[r], ys = ty[r], d = td[r], Dst = tD[r];
        const double A = tA[r], B = tB[r], C = tC[r];
        const int self = tself[r];
        double dlS = 0.0, slS = 0.0, dlB = 0.0, slB = 0.0, s2 = 0.0;
        for (int img = 0; img < nimg; ++img) {
            const double iota = (img == 0) ? 1.0 : -1.0;
            for (int j = 0; j < M; ++j) {
                const double cj = (j == 0 || j == M - 1) ? 0.5 : 1.0;
                const double t = iota * (y1 + j * dy) - ys;
                for (int i = 0; i < N; ++i) {
                    const double ci = (i == 0 || i == N - 1) ? 0.5 : 1.0;
                    const double w = dx * dy * ci * cj;
                    const double s = (x1 + i * dx) - xs;
                    const size_t n = (size_t)j * N + i;
                    /* free-surface node */
                    {
                        const double a = zs[n], ax = zsx[n], ay = iota * zsy[n];
                        const double R = sqrt(s * s + t * t + (a - d) * (a - d));
                        const double K1 = (a - d - s * ax - t * ay) / (R * R * R);
                        const double K2 = 1.0 / R;
                        const double dens = Ds[n] - (self == 0 ? Dst : 0.0);
                        dlS += absmode ? fabs(w * dens * K1) : w * dens * K1;
                        slS += absmode ? fabs(w * sigs[n] * K2) : w * sigs[n] * K2;
                    }
                    /* bottom node */
                    {
                        const double a = zb[n], ax = zbx[n], ay = iota * zby[n];
                        const double R = sqrt(s * s + t * t + (a - d) * (a - d));
                        const double K1 = (a - d - s * ax - t * ay) / (R * R * R);
                        const double K2 = 1.0 / R;
                        const double dens = Db[n] - (self == 1 ? Dst : 0.0);
                        dlB += absmode ? fabs(w * dens * K1) : w * dens * K1;
                        slB += absmode ? fabs(w * sigb[n] * K2) : w * sigb[n] * K2;
                    }
                    /* singular kernel of the target's own surface */
                    s2 += w / sqrt(A * s * s + B * s * t + C * t * t);
                }
            }
        }
        out[5 * (size_t)r + 0] = dlS;
        out[5 * (size_t)r + 1] = slS;
        out[5 * (size_t)r + 2] = dlB;
        out[5 * (size_t)r + 3] = slB;
        out[5 * (size_t)r + 4] = s2;
    }
}
