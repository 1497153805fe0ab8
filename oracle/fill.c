/*
 * Oracle (test infrastructure only): dense Galerkin EFIE impedance matrix of a
 * regular lattice of z-directed thin-wire dipoles, written as the plain
 * definition with no use of translation invariance, Toeplitz structure or
 * symmetry.  Only tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library; the GPU product path never does.
 *
 * Method-of-Moments matrix Z of the linear system Z I = V (paper, Sec. II-D,
 * eq. (eqProb)).  The paper meshes its elements with RWG functions and gives
 * no fill formulas, so the element here is the thin-wire dipole of the
 * benchmark workloads, filled as follows (one reading, fixed once):
 *
 *   wire along z over [-L/2, L/2], Ns = M+1 equal segments of length D = L/Ns;
 *   basis p = 0..M-1 is the rooftop peaking at node z_{p+1} = -L/2 + (p+1) D,
 *   rising on segment p and falling on segment p+1;
 *   unknown n = e*M + p, element e = iy*nx + ix at (ix*dx, iy*dy);
 *
 *   Z_mn = j*eta*( k*A_mn - Phi_mn / k ),
 *   A_mn   = sum over supports, 4x4 Gauss-Legendre points of f_m(z) f_n(z') G(R)
 *   Phi_mn = same with the derivatives f'_m f'_n = (+-1/D)(+-1/D),
 *   G(R)   = exp(-j k R) / (4 pi R),  R = sqrt(rho^2 + (z - z')^2 + a^2)
 *
 * (the reduced thin-wire kernel with the a^2 term added for every pair).
 * kernel_mode 1 replaces G by the real polynomial R^2; four-point Gauss-Legendre
 * is then exact, which lets tests compare against closed-form integrals.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* Four-point Gauss-Legendre rule on [-1,1]: nodes +-sqrt(3/7 -+ (2/7) sqrt(6/5)),
 * weights (18 +- sqrt(30))/36. */
static void gl4(double x[4], double w[4]) {
    double a = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
    double b = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
    double wa = (18.0 + sqrt(30.0)) / 36.0;
    double wb = (18.0 - sqrt(30.0)) / 36.0;
    x[0] = -b; w[0] = wb;
    x[1] = -a; w[1] = wa;
    x[2] = a;  w[2] = wa;
    x[3] = b;  w[3] = wb;
}

void oracle_gl4(double* x, double* w) { gl4(x, w); }

typedef struct {
    int nx, ny, M;
    double dx, dy, L, a, k, eta;
    int kernel_mode;
    double u[4], wu[4]; /* points and weights mapped to [0,1] */
} fillctx;

static void init_ctx(fillctx* c, int nx, int ny, double dx, double dy, double L, double a,
                     int M, double k, double eta, int kernel_mode) {
    double x[4], w[4];
    gl4(x, w);
    c->nx = nx; c->ny = ny; c->M = M;
    c->dx = dx; c->dy = dy; c->L = L; c->a = a; c->k = k; c->eta = eta;
    c->kernel_mode = kernel_mode;
    for (int i = 0; i < 4; ++i) {
        c->u[i] = 0.5 * (1.0 + x[i]);
        c->wu[i] = 0.5 * w[i];
    }
}

/* One matrix entry Z_mn, computed from absolute positions. */
static void entry(const fillctx* c, int64_t m, int64_t n, double* re, double* im) {
    const int M = c->M;
    const double D = c->L / (double)(M + 1);
    int64_t em = m / M, en = n / M;
    int pm = (int)(m % M), pn = (int)(n % M);
    double xm = (double)(em % c->nx) * c->dx, ym = (double)(em / c->nx) * c->dy;
    double xn = (double)(en % c->nx) * c->dx, yn = (double)(en / c->nx) * c->dy;
    double rho2 = (xm - xn) * (xm - xn) + (ym - yn) * (ym - yn);
    double Are = 0, Aim = 0, Pre = 0, Pim = 0;
    for (int sm = 0; sm < 2; ++sm) {          /* 0: rising segment pm, 1: falling segment pm+1 */
        int segm = pm + sm;
        double dm = (sm == 0) ? 1.0 / D : -1.0 / D;
        for (int sn = 0; sn < 2; ++sn) {
            int segn = pn + sn;
            double dn = (sn == 0) ? 1.0 / D : -1.0 / D;
            for (int i = 0; i < 4; ++i) {
                double z = -0.5 * c->L + ((double)segm + c->u[i]) * D;
                double fm = (sm == 0) ? c->u[i] : 1.0 - c->u[i];
                for (int j = 0; j < 4; ++j) {
                    double zp = -0.5 * c->L + ((double)segn + c->u[j]) * D;
                    double fn = (sn == 0) ? c->u[j] : 1.0 - c->u[j];
                    double R2 = rho2 + (z - zp) * (z - zp) + c->a * c->a;
                    double gre, gim;
                    if (c->kernel_mode == 0) {
                        double R = sqrt(R2);
                        double s = 1.0 / (4.0 * M_PI * R);
                        gre = cos(c->k * R) * s;
                        gim = -sin(c->k * R) * s;
                    } else {
                        gre = R2;
                        gim = 0.0;
                    }
                    double wgt = c->wu[i] * c->wu[j] * D * D;
                    Are += wgt * fm * fn * gre;
                    Aim += wgt * fm * fn * gim;
                    Pre += wgt * dm * dn * gre;
                    Pim += wgt * dm * dn * gim;
                }
            }
        }
    }
    /* Z = j*eta*(k*A - Phi/k) */
    double tre = c->k * Are - Pre / c->k;
    double tim = c->k * Aim - Pim / c->k;
    *re = -c->eta * tim;
    *im = c->eta * tre;
}

/* Dense N x N matrix, row-major, interleaved complex (Z[2*(m*N+n)] = Re Z_mn). */
int oracle_fill_dense(int nx, int ny, double dx, double dy, double L, double a, int M,
                      double k, double eta, int kernel_mode, double* Z) {
    if (nx < 1 || ny < 1 || M < 1 || L <= 0 || a <= 0 || k <= 0) return -1;
    fillctx c;
    init_ctx(&c, nx, ny, dx, dy, L, a, M, k, eta, kernel_mode);
    int64_t N = (int64_t)nx * ny * M;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t m = 0; m < N; ++m)
        for (int64_t n = 0; n < N; ++n)
            entry(&c, m, n, &Z[2 * (m * N + n)], &Z[2 * (m * N + n) + 1]);
    return 0;
}

/* Selected entries (rows[i], cols[i]) of the same matrix. */
int oracle_fill_entries(int nx, int ny, double dx, double dy, double L, double a, int M,
                        double k, double eta, int kernel_mode, const int64_t* rows,
                        const int64_t* cols, int64_t count, double* out) {
    if (nx < 1 || ny < 1 || M < 1 || L <= 0 || a <= 0 || k <= 0) return -1;
    fillctx c;
    init_ctx(&c, nx, ny, dx, dy, L, a, M, k, eta, kernel_mode);
    int64_t N = (int64_t)nx * ny * M;
    for (int64_t i = 0; i < count; ++i)
        if (rows[i] < 0 || rows[i] >= N || cols[i] < 0 || cols[i] >= N) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) entry(&c, rows[i], cols[i], &out[2 * i], &out[2 * i + 1]);
    return 0;
}
