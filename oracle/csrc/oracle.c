/*
 * Plain FP64 CPU reference for the 1D/2D/3D nonuniform FFT (test infrastructure).
 *
 * This file is part of the oracle: it is used only by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  It shares no
 * code with the GPU library and must never be linked into it.
 *
 * Contents
 *   orc_direct_type1   exact exponential sum of type 1 (Sec. I, eq. (1) and its
 *                      3D analogue) on a tensor-product subset of modes
 *   orc_direct_type2   exact exponential sum of type 2 (Sec. I, eq. (3)) at a
 *                      subset of target points, over all modes
 *   orc_spread         type 1 step 1 of Sec. II-A: spreading with the
 *                      periodised ES kernel of eq. (es)
 *   orc_interp         type 2 step 3 of Sec. II-B: interpolation with the same
 *                      kernel (the exact transpose of orc_spread)
 *   orc_direct_type3   exact exponential sum of type 3 (nonuniform points to
 *                      nonuniform frequencies), named in Sec. I-B and Sec. VI
 *                      as beyond the paper's scope
 *
 * Dimension 1 (dim = 1, y = z = NULL) is accepted everywhere: the paper's
 * formulas restricted to one coordinate.
 *
 * All arithmetic is IEEE double.  Complex arrays are interleaved (re, im).
 * Fine grids are stored with the first coordinate fastest: index
 * l1 + n1*(l2 + n2*l3).
 *
 * Lattice convention: fine-grid point l in dimension i sits at l*h_i - pi with
 * h_i = 2*pi/n_i, so the grid coordinate of a point x is g = (x + pi)/h_i,
 * the same rounding used for binning in Sec. III-A.  The resulting phase
 * (-1)^k is applied in the correction step by the Python side.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_PI 3.141592653589793238462643383279502884

/* Points are summed in blocks of this many terms before being added to the
 * running total, which keeps the summation error at O((B + M/B) u). */
#define ORC_SUMBLOCK 1024

/* ---------------------------------------------------------------------- */
/* Exact sums (ground truth)                                              */
/* ---------------------------------------------------------------------- */

/* f[(i3*K2 + i2)*K1 + i1] = sum_j c_j exp(iflag * i * (k1[i1] x_j + k2[i2] y_j
 * + k3[i3] z_j)).  In 2D pass K3 = 1, k3 = {0}, z = NULL; in 1D also K2 = 1,
 * k2 = {0}, y = NULL.  The product of the
 * per-dimension exponentials equals the exponential of the sum exactly; each
 * per-dimension factor is one call of sin and cos of k*x in double. */
void orc_direct_type1(int dim, int64_t M, const double *x, const double *y,
                      const double *z, const double *c, int iflag,
                      int64_t K1, const int64_t *k1, int64_t K2,
                      const int64_t *k2, int64_t K3, const int64_t *k3,
                      double *out)
{
    const int64_t K = K1 * K2 * K3;
    const double s = (iflag >= 0) ? 1.0 : -1.0;
    memset(out, 0, sizeof(double) * 2 * K);
#pragma omp parallel
    {
        double *tot = (double *)calloc(2 * K, sizeof(double));
        double *blk = (double *)calloc(2 * K, sizeof(double));
        double *e1 = (double *)malloc(sizeof(double) * 2 * K1);
        double *e2 = (double *)malloc(sizeof(double) * 2 * K2);
        double *e3 = (double *)malloc(sizeof(double) * 2 * K3);
        int64_t inblk = 0;
#pragma omp for schedule(static)
        for (int64_t j = 0; j < M; ++j) {
            for (int64_t a = 0; a < K1; ++a) {
                double ph = s * (double)k1[a] * x[j];
                e1[2 * a] = cos(ph);
                e1[2 * a + 1] = sin(ph);
            }
            for (int64_t a = 0; a < K2; ++a) {
                double ph = (dim >= 2) ? s * (double)k2[a] * y[j] : 0.0;
                e2[2 * a] = cos(ph);
                e2[2 * a + 1] = sin(ph);
            }
            for (int64_t a = 0; a < K3; ++a) {
                double ph = (dim == 3) ? s * (double)k3[a] * z[j] : 0.0;
                e3[2 * a] = cos(ph);
                e3[2 * a + 1] = sin(ph);
            }
            const double cr = c[2 * j], ci = c[2 * j + 1];
            for (int64_t i3 = 0; i3 < K3; ++i3) {
                double ar = cr * e3[2 * i3] - ci * e3[2 * i3 + 1];
                double ai = cr * e3[2 * i3 + 1] + ci * e3[2 * i3];
                for (int64_t i2 = 0; i2 < K2; ++i2) {
                    double br = ar * e2[2 * i2] - ai * e2[2 * i2 + 1];
                    double bi = ar * e2[2 * i2 + 1] + ai * e2[2 * i2];
                    double *o = blk + 2 * ((i3 * K2 + i2) * K1);
                    for (int64_t i1 = 0; i1 < K1; ++i1) {
                        o[2 * i1] += br * e1[2 * i1] - bi * e1[2 * i1 + 1];
                        o[2 * i1 + 1] += br * e1[2 * i1 + 1] + bi * e1[2 * i1];
                    }
                }
            }
            if (++inblk == ORC_SUMBLOCK) {
                for (int64_t q = 0; q < 2 * K; ++q) { tot[q] += blk[q]; blk[q] = 0.0; }
                inblk = 0;
            }
        }
        for (int64_t q = 0; q < 2 * K; ++q) tot[q] += blk[q];
#pragma omp critical
        for (int64_t q = 0; q < 2 * K; ++q) out[q] += tot[q];
        free(tot); free(blk); free(e1); free(e2); free(e3);
    }
}

/* c_out[q] = sum_k f_k exp(iflag * i * k . x_{idx[q]}) over all modes
 * k in I_N1 x I_N2 (x I_N3), I_N = {-floor(N/2), ..., ceil(N/2) - 1}, with f
 * stored k1 fastest.  nq target points are given by their indices idx. */
void orc_direct_type2(int dim, const int64_t N[3], const double *x,
                      const double *y, const double *z, const double *f,
                      int iflag, int64_t nq, const int64_t *idx, double *out)
{
    const double s = (iflag >= 0) ? 1.0 : -1.0;
    const int64_t N1 = N[0], N2 = (dim >= 2) ? N[1] : 1, N3 = (dim == 3) ? N[2] : 1;
#pragma omp parallel
    {
        double *e1 = (double *)malloc(sizeof(double) * 2 * N1);
        double *e2 = (double *)malloc(sizeof(double) * 2 * N2);
        double *e3 = (double *)malloc(sizeof(double) * 2 * N3);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < nq; ++q) {
            const int64_t j = idx[q];
            for (int64_t a = 0; a < N1; ++a) {
                double ph = s * (double)(a - N1 / 2) * x[j];
                e1[2 * a] = cos(ph); e1[2 * a + 1] = sin(ph);
            }
            for (int64_t a = 0; a < N2; ++a) {
                double ph = (dim >= 2) ? s * (double)(a - N2 / 2) * y[j] : 0.0;
                e2[2 * a] = cos(ph); e2[2 * a + 1] = sin(ph);
            }
            for (int64_t a = 0; a < N3; ++a) {
                double ph = (dim == 3) ? s * (double)(a - N3 / 2) * z[j] : 0.0;
                e3[2 * a] = cos(ph); e3[2 * a + 1] = sin(ph);
            }
            double sr = 0.0, si = 0.0;
            for (int64_t i3 = 0; i3 < N3; ++i3) {
                double r3 = 0.0, m3 = 0.0;
                for (int64_t i2 = 0; i2 < N2; ++i2) {
                    const double *fr = f + 2 * ((i3 * N2 + i2) * N1);
                    double r1 = 0.0, m1 = 0.0;
                    for (int64_t i1 = 0; i1 < N1; ++i1) {
                        r1 += fr[2 * i1] * e1[2 * i1] - fr[2 * i1 + 1] * e1[2 * i1 + 1];
                        m1 += fr[2 * i1] * e1[2 * i1 + 1] + fr[2 * i1 + 1] * e1[2 * i1];
                    }
                    r3 += r1 * e2[2 * i2] - m1 * e2[2 * i2 + 1];
                    m3 += r1 * e2[2 * i2 + 1] + m1 * e2[2 * i2];
                }
                sr += r3 * e3[2 * i3] - m3 * e3[2 * i3 + 1];
                si += r3 * e3[2 * i3 + 1] + m3 * e3[2 * i3];
            }
            out[2 * q] = sr;
            out[2 * q + 1] = si;
        }
        free(e1); free(e2); free(e3);
    }
}

/* ---------------------------------------------------------------------- */
/* The three-step algorithm: spreading and interpolation (Sec. II)        */
/* ---------------------------------------------------------------------- */

/* ES kernel, eq. (es): exp(beta*(sqrt(1-z^2)-1)) on |z| <= 1, else 0. */
static double orc_es(double zz, double beta)
{
    if (fabs(zz) > 1.0) return 0.0;
    return exp(beta * (sqrt(1.0 - zz * zz) - 1.0));
}

/* Grid coordinate of x on a periodic grid of n points: (x + pi) * n/(2 pi),
 * brought into [0, n) by whole periods. */
static double orc_gridcoord(double x, int64_t n)
{
    const double S = (double)n / (2.0 * ORC_PI);
    double g = (x + ORC_PI) * S;
    g = g - floor(g / (double)n) * (double)n;
    if (g >= (double)n) g -= (double)n;
    if (g < 0.0) g = 0.0;
    return g;
}

/* The w kernel values and wrapped grid indices that a point touches in one
 * dimension: taps l = l0 + a, a = 0..w-1, l0 = ceil(g - w/2), weight
 * phi(2 (l - g)/w).  This is the rescaled kernel phi(x/alpha) with
 * alpha = w*pi/n evaluated at the grid spacing h = 2 pi/n. */
static void orc_taps(double g, int64_t n, int w, double beta, double *ker,
                     int64_t *ind)
{
    const double l0 = ceil(g - 0.5 * (double)w);
    for (int a = 0; a < w; ++a) {
        double l = l0 + (double)a;
        ker[a] = orc_es(2.0 * (l - g) / (double)w, beta);
        int64_t li = (int64_t)l % n;
        if (li < 0) li += n;
        ind[a] = li;
    }
}

/* grid += sum_j c_j psi_per(l h - pi - x_j) (Sec. II-A step 1).  The grid must
 * be zeroed by the caller.  Accumulation uses atomic adds, so the order of
 * additions (and hence the last bits) may differ from run to run. */
void orc_spread(int dim, const int64_t n[3], int w, double beta, int64_t M,
                const double *x, const double *y, const double *z,
                const double *c, double *grid)
{
    const int64_t n1 = n[0], n2 = (dim >= 2) ? n[1] : 1, n3 = (dim == 3) ? n[2] : 1;
#pragma omp parallel
    {
        double k1[32], k2[32], k3[32];
        int64_t i1[32], i2[32], i3[32];
#pragma omp for schedule(static)
        for (int64_t j = 0; j < M; ++j) {
            orc_taps(orc_gridcoord(x[j], n1), n1, w, beta, k1, i1);
            int w2 = 1;
            k2[0] = 1.0; i2[0] = 0;
            if (dim >= 2) { orc_taps(orc_gridcoord(y[j], n2), n2, w, beta, k2, i2); w2 = w; }
            int w3 = 1;
            k3[0] = 1.0; i3[0] = 0;
            if (dim == 3) { orc_taps(orc_gridcoord(z[j], n3), n3, w, beta, k3, i3); w3 = w; }
            for (int a3 = 0; a3 < w3; ++a3)
                for (int a2 = 0; a2 < w2; ++a2) {
                    const double k23 = k3[a3] * k2[a2];
                    const int64_t row = (i3[a3] * n2 + i2[a2]) * n1;
                    for (int a1 = 0; a1 < w; ++a1) {
                        const double kk = k23 * k1[a1];
                        double *b = grid + 2 * (row + i1[a1]);
#pragma omp atomic
                        b[0] += kk * c[2 * j];
#pragma omp atomic
                        b[1] += kk * c[2 * j + 1];
                    }
                }
        }
    }
}

/* c_j = sum_l grid_l psi_per(l h - pi - x_j) (Sec. II-B step 3). */
void orc_interp(int dim, const int64_t n[3], int w, double beta, int64_t M,
                const double *x, const double *y, const double *z,
                const double *grid, double *c)
{
    const int64_t n1 = n[0], n2 = (dim >= 2) ? n[1] : 1, n3 = (dim == 3) ? n[2] : 1;
#pragma omp parallel
    {
        double k1[32], k2[32], k3[32];
        int64_t i1[32], i2[32], i3[32];
#pragma omp for schedule(static)
        for (int64_t j = 0; j < M; ++j) {
            orc_taps(orc_gridcoord(x[j], n1), n1, w, beta, k1, i1);
            int w2 = 1;
            k2[0] = 1.0; i2[0] = 0;
            if (dim >= 2) { orc_taps(orc_gridcoord(y[j], n2), n2, w, beta, k2, i2); w2 = w; }
            int w3 = 1;
            k3[0] = 1.0; i3[0] = 0;
            if (dim == 3) { orc_taps(orc_gridcoord(z[j], n3), n3, w, beta, k3, i3); w3 = w; }
            double sr = 0.0, si = 0.0;
            for (int a3 = 0; a3 < w3; ++a3)
                for (int a2 = 0; a2 < w2; ++a2) {
                    const double k23 = k3[a3] * k2[a2];
                    const int64_t row = (i3[a3] * n2 + i2[a2]) * n1;
                    for (int a1 = 0; a1 < w; ++a1) {
                        const double kk = k23 * k1[a1];
                        const double *b = grid + 2 * (row + i1[a1]);
                        sr += kk * b[0];
                        si += kk * b[1];
                    }
                }
            c[2 * j] = sr;
            c[2 * j + 1] = si;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Type 3: nonuniform points to nonuniform frequencies                    */
/* ---------------------------------------------------------------------- */

/* out[q] = sum_j c_j exp(iflag * i * (s_k x_j + t_k y_j + u_k z_j)) for the nq
 * frequencies k = idx[q] (real, arbitrary); t, y are unused in 1D and u, z in
 * 1D and 2D.  Every phase is formed in double and passed to cos and sin once. */
void orc_direct_type3(int dim, int64_t M, const double *x, const double *y,
                      const double *z, const double *c, int iflag,
                      const double *s, const double *t, const double *u,
                      int64_t nq, const int64_t *idx, double *out)
{
    const double sg = (iflag >= 0) ? 1.0 : -1.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
        const int64_t k = idx[q];
        double tr = 0.0, ti = 0.0, br = 0.0, bi = 0.0;
        int64_t inblk = 0;
        for (int64_t j = 0; j < M; ++j) {
            double ph = s[k] * x[j];
            if (dim >= 2) ph += t[k] * y[j];
            if (dim == 3) ph += u[k] * z[j];
            ph *= sg;
            const double er = cos(ph), ei = sin(ph);
            br += c[2 * j] * er - c[2 * j + 1] * ei;
            bi += c[2 * j] * ei + c[2 * j + 1] * er;
            if (++inblk == ORC_SUMBLOCK) {
                tr += br; ti += bi; br = 0.0; bi = 0.0;
                inblk = 0;
            }
        }
        out[2 * q] = tr + br;
        out[2 * q + 1] = ti + bi;
    }
}

/* Number of OpenMP threads the reference will use. */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* Thread count of the OpenMP loops above (timing control only; the results
 * do not depend on it beyond summation order). */
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
