/*
 * ns_oracle.c -- plain FP64 CPU oracle for the compressible Navier-Stokes
 * residual, the three-stage low-storage Runge-Kutta update and the
 * Taylor-Green vortex diagnostics of Jammy, Jacobs, Lusher & Sandham,
 * "Energy efficiency of finite difference algorithms on multicore CPUs,
 * GPUs, and Intel Xeon Phi processors" (arXiv:1709.09713).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the HIP path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table or constant with the GPU library.
 *
 * Written for obviousness, not speed: every derivative is evaluated at the
 * point where it is needed by gathering its stencil taps with periodic
 * (modular) indexing; there is no blocking, no fusion and no reordering
 * beyond what the equations state.  Compile with -O2 -ffp-contract=off (no
 * fast-math): IEEE double, round-to-nearest-even, no FMA contraction.
 *
 * Field layout: five conserved fields Q = (rho, rho*u0, rho*u1, rho*u2, rho*E)
 * each nx*ny*nz doubles, field-major, x (i) fastest, then y (j), then z (k).
 * Grid point (i,j,k) sits at (i*hx, j*hy, k*hz), h = length / n (periodic,
 * no duplicated end point).
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *  - Energy equation, convective part: the printed signs inside the
 *    skew-symmetric bracket of the energy equation are read as all "+",
 *    as in the mass and momentum equations (the printed form is not a
 *    conservation law).
 *  - The Runge-Kutta recurrence of the temporal-discretisation section is
 *    read as the two-register low-storage scheme of the generic algorithm
 *    figure (save-state, then per stage: evaluate R, evaluate Q^{k+1},
 *    advance the n+1 level) with a = (2/3, 5/12, 3/5), b = (1/4, 3/20, 3/5).
 *  - Mixed derivatives d2 u_j / dx_i dx_j (i != j) are nested fourth-order
 *    first derivatives D_i(D_j u_j); for i == j the second-derivative stencil
 *    is used.
 *  - Initial density rho = gamma M^2 p (T = 1 everywhere at t = 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n[3];
    double h[3];
    double gamma, prandtl, reynolds, mach;
} orc_grid;

static orc_grid make_grid(int nx, int ny, int nz, double lx, double ly,
                          double lz, double gamma, double pr, double re,
                          double mach)
{
    orc_grid g;
    g.n[0] = nx; g.n[1] = ny; g.n[2] = nz;
    g.h[0] = lx / nx; g.h[1] = ly / ny; g.h[2] = lz / nz;
    g.gamma = gamma; g.prandtl = pr; g.reynolds = re; g.mach = mach;
    return g;
}

static size_t npts(const orc_grid *g)
{
    return (size_t)g->n[0] * (size_t)g->n[1] * (size_t)g->n[2];
}

static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* Linear index of point (i,j,k) shifted by s points along direction d,
 * wrapped periodically. */
static size_t at(const orc_grid *g, int i, int j, int k, int d, int s)
{
    int c[3] = {i, j, k};
    c[d] = wrap(c[d] + s, g->n[d]);
    return ((size_t)c[2] * g->n[1] + c[1]) * g->n[0] + c[0];
}

/* ---------------------------------------------------------------------
 * Fourth-order central stencils, equations (fd) and (sd) of the
 * spatial-discretisation section.  The tap values are passed in, so the
 * same arithmetic serves plain (non-periodic) arrays and the periodic grid.
 * ------------------------------------------------------------------- */

/* First derivative: (f[-2]/12 - 2 f[-1]/3 + 2 f[+1]/3 - f[+2]/12) / h,
 * grouped as differences so a constant field gives exactly zero. */
double orc_d1(double fm2, double fm1, double fp1, double fp2, double h)
{
    return ((2.0 / 3.0) * (fp1 - fm1) - (1.0 / 12.0) * (fp2 - fm2)) / h;
}

/* Second derivative: (-f[-2]/12 + 4 f[-1]/3 - 5 f[0]/2 + 4 f[+1]/3
 * - f[+2]/12) / h^2. */
double orc_d2(double fm2, double fm1, double f0, double fp1, double fp2,
              double h)
{
    return ((4.0 / 3.0) * (fm1 + fp1) - (1.0 / 12.0) * (fm2 + fp2)
            - (5.0 / 2.0) * f0) / (h * h);
}

/* Apply the first (order 1) or second (order 2) derivative stencil to a
 * plain 1-D array f[0..n) at the interior points 2..n-3; other entries of
 * out are left untouched.  Used to check the stencils on polynomials. */
void orc_stencil_line(const double *f, int n, double h, int order,
                      double *out)
{
    for (int i = 2; i < n - 2; ++i) {
        if (order == 1)
            out[i] = orc_d1(f[i - 2], f[i - 1], f[i + 1], f[i + 2], h);
        else
            out[i] = orc_d2(f[i - 2], f[i - 1], f[i], f[i + 1], f[i + 2], h);
    }
}

/* Nested mixed derivative D_x(D_y f) on a plain 2-D array f[j*nx + i]
 * at the interior points 2 <= i < nx-2, 2 <= j < ny-2. */
void orc_mixed_plane(const double *f, int nx, int ny, double hx, double hy,
                     double *out)
{
    for (int j = 2; j < ny - 2; ++j)
        for (int i = 2; i < nx - 2; ++i) {
            double dy[5];
            for (int s = -2; s <= 2; ++s) {
                int ii = i + s;
                dy[s + 2] = orc_d1(f[(j - 2) * nx + ii], f[(j - 1) * nx + ii],
                                   f[(j + 1) * nx + ii], f[(j + 2) * nx + ii],
                                   hy);
            }
            out[j * nx + i] = orc_d1(dy[0], dy[1], dy[3], dy[4], hx);
        }
}

/* ---------------------------------------------------------------------
 * Periodic derivatives of grid functions at one point.
 * ------------------------------------------------------------------- */

static double d1_at(const orc_grid *g, const double *f, int i, int j, int k,
                    int d)
{
    return orc_d1(f[at(g, i, j, k, d, -2)], f[at(g, i, j, k, d, -1)],
                  f[at(g, i, j, k, d, 1)], f[at(g, i, j, k, d, 2)], g->h[d]);
}

static double d2_at(const orc_grid *g, const double *f, int i, int j, int k,
                    int d)
{
    return orc_d2(f[at(g, i, j, k, d, -2)], f[at(g, i, j, k, d, -1)],
                  f[at(g, i, j, k, d, 0)], f[at(g, i, j, k, d, 1)],
                  f[at(g, i, j, k, d, 2)], g->h[d]);
}

/* First derivative along d of the pointwise product a*b (the product is
 * formed at every tap, as a temporary would hold it). */
static double d1_prod_at(const orc_grid *g, const double *a, const double *b,
                         int i, int j, int k, int d)
{
    size_t m2 = at(g, i, j, k, d, -2), m1 = at(g, i, j, k, d, -1);
    size_t p1 = at(g, i, j, k, d, 1), p2 = at(g, i, j, k, d, 2);
    return orc_d1(a[m2] * b[m2], a[m1] * b[m1], a[p1] * b[p1],
                  a[p2] * b[p2], g->h[d]);
}

/* Nested mixed derivative D_di(D_dk f) at (i,j,k), di != dk. */
static double dmix_at(const orc_grid *g, const double *f, int i, int j, int k,
                      int di, int dk)
{
    double t[5];
    for (int s = -2; s <= 2; ++s) {
        int c[3] = {i, j, k};
        c[di] = wrap(c[di] + s, g->n[di]);
        t[s + 2] = d1_at(g, f, c[0], c[1], c[2], dk);
    }
    return orc_d1(t[0], t[1], t[3], t[4], g->h[di]);
}

/* d^2 u_j / dx_i dx_j: second-derivative stencil when i == j, nested first
 * derivatives otherwise. */
static double dd_at(const orc_grid *g, const double *uj, int i, int j, int k,
                    int di, int dj)
{
    if (di == dj)
        return d2_at(g, uj, i, j, k, di);
    return dmix_at(g, uj, i, j, k, di, dj);
}

/* Periodic derivative of a whole grid function: order 1 (eq. fd) or
 * order 2 (eq. sd) along direction d. */
void orc_deriv_field(int nx, int ny, int nz, double lx, double ly, double lz,
                     const double *f, int d, int order, double *out)
{
    orc_grid g = make_grid(nx, ny, nz, lx, ly, lz, 1.4, 1.0, 1.0, 1.0);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                out[at(&g, i, j, k, 0, 0)] =
                    order == 1 ? d1_at(&g, f, i, j, k, d)
                               : d2_at(&g, f, i, j, k, d);
}

/* Nested periodic mixed derivative D_di(D_dk f) of a whole grid function. */
void orc_mixed_field(int nx, int ny, int nz, double lx, double ly, double lz,
                     const double *f, int di, int dk, double *out)
{
    orc_grid g = make_grid(nx, ny, nz, lx, ly, lz, 1.4, 1.0, 1.0, 1.0);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                out[at(&g, i, j, k, 0, 0)] = dmix_at(&g, f, i, j, k, di, dk);
}

/* ---------------------------------------------------------------------
 * Primitive variables, equations (pinprimitive) and (Tinprimitive):
 *   u_i = rho u_i / rho,  p = (gamma-1)(rho E - rho u_j u_j / 2),
 *   T = gamma M^2 p / rho.
 * prim holds u0, u1, u2, p, T (five fields of N points).
 * ------------------------------------------------------------------- */
static void primitives(const orc_grid *g, const double *Q, double *prim)
{
    size_t N = npts(g);
    const double *rho = Q, *m0 = Q + N, *m1 = Q + 2 * N, *m2 = Q + 3 * N;
    const double *rE = Q + 4 * N;
    double *u0 = prim, *u1 = prim + N, *u2 = prim + 2 * N;
    double *p = prim + 3 * N, *T = prim + 4 * N;
    double gm = g->gamma, M = g->mach;
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < (long long)N; ++q) {
        u0[q] = m0[q] / rho[q];
        u1[q] = m1[q] / rho[q];
        u2[q] = m2[q] / rho[q];
        double ke = 0.5 * rho[q] * (u0[q] * u0[q] + u1[q] * u1[q]
                                    + u2[q] * u2[q]);
        p[q] = (gm - 1.0) * (rE[q] - ke);
        T[q] = gm * M * M * p[q] / rho[q];
    }
}

/* ---------------------------------------------------------------------
 * Residual R(Q) at one point: the mass, momentum and energy equations of
 * the methodology section, skew-symmetric (Blaisdell) convection,
 * Laplacian-form viscous terms with constant viscosity, heat conduction
 * proportional to the Laplacian of T.
 * ------------------------------------------------------------------- */
static void residual_at(const orc_grid *g, const double *Q, const double *prim,
                        int i, int j, int k, double R[5])
{
    size_t N = npts(g);
    size_t c = at(g, i, j, k, 0, 0);
    const double *rho = Q, *rE = Q + 4 * N;
    const double *m[3] = {Q + N, Q + 2 * N, Q + 3 * N};
    const double *u[3] = {prim, prim + N, prim + 2 * N};
    const double *p = prim + 3 * N, *T = prim + 4 * N;
    double inv_re = 1.0 / g->reynolds;
    double kappa = 1.0 / ((g->gamma - 1.0) * g->mach * g->mach * g->prandtl
                          * g->reynolds);

    /* Velocity gradient du[i][j] = d u_i / d x_j and the divergence. */
    double du[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            du[a][b] = d1_at(g, u[a], i, j, k, b);
    double div = du[0][0] + du[1][1] + du[2][2];

    /* Mass: -1/2 ( d(rho u_j)/dx_j + rho du_j/dx_j + u_j drho/dx_j ). */
    double s = 0.0;
    for (int b = 0; b < 3; ++b)
        s += d1_at(g, m[b], i, j, k, b) + rho[c] * du[b][b]
             + u[b][c] * d1_at(g, rho, i, j, k, b);
    R[0] = -0.5 * s;

    /* Viscous bracket of the momentum equation for component a:
     * d2u_a/dx_j^2 + d2u_j/dx_a dx_j - (2/3) d2u_k/dx_a dx_k. */
    double visc[3];
    for (int a = 0; a < 3; ++a) {
        double lap = 0.0, cross = 0.0, dil = 0.0;
        for (int b = 0; b < 3; ++b)
            lap += d2_at(g, u[a], i, j, k, b);
        for (int b = 0; b < 3; ++b)
            cross += dd_at(g, u[b], i, j, k, a, b);
        for (int kk = 0; kk < 3; ++kk)
            dil += dd_at(g, u[kk], i, j, k, a, kk);
        visc[a] = lap + cross - (2.0 / 3.0) * dil;
    }

    /* Momentum: -1/2 ( d(rho u_a u_j)/dx_j + rho u_a du_j/dx_j
     *                  + u_j d(rho u_a)/dx_j ) - dp/dx_a + visc_a / Re. */
    for (int a = 0; a < 3; ++a) {
        double conv = 0.0;
        for (int b = 0; b < 3; ++b)
            conv += d1_prod_at(g, m[a], u[b], i, j, k, b) + m[a][c] * du[b][b]
                    + u[b][c] * d1_at(g, m[a], i, j, k, b);
        R[1 + a] = -0.5 * conv - d1_at(g, p, i, j, k, a) + inv_re * visc[a];
    }

    /* Energy: -1/2 ( rho E du_j/dx_j + u_j d(rho E)/dx_j + d(rho E u_j)/dx_j )
     *         - d(p u_j)/dx_j + (u_a / Re) visc_a
     *         + (1/Re) du_a/dx_j (du_a/dx_j + du_j/dx_a - (2/3) div delta_aj)
     *         + kappa d2T/dx_j^2. */
    double conv = 0.0, pw = 0.0, work = 0.0, diss = 0.0, heat = 0.0;
    for (int b = 0; b < 3; ++b) {
        conv += rE[c] * du[b][b] + u[b][c] * d1_at(g, rE, i, j, k, b)
                + d1_prod_at(g, rE, u[b], i, j, k, b);
        pw += d1_prod_at(g, p, u[b], i, j, k, b);
        heat += d2_at(g, T, i, j, k, b);
    }
    for (int a = 0; a < 3; ++a) {
        work += u[a][c] * visc[a];
        for (int b = 0; b < 3; ++b)
            diss += du[a][b] * (du[a][b] + du[b][a]
                                - (a == b ? (2.0 / 3.0) * div : 0.0));
    }
    R[4] = -0.5 * conv - pw + inv_re * work + inv_re * diss + kappa * heat;
}

/* R(Q) on the whole periodic grid.  Q and R hold 5*N doubles. */
void orc_residual(int nx, int ny, int nz, double lx, double ly, double lz,
                  double gamma, double pr, double re, double mach,
                  const double *Q, double *R)
{
    orc_grid g = make_grid(nx, ny, nz, lx, ly, lz, gamma, pr, re, mach);
    size_t N = npts(&g);
    double *prim = (double *)malloc(5 * N * sizeof(double));
    primitives(&g, Q, prim);
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double r[5];
                residual_at(&g, Q, prim, i, j, k, r);
                size_t c = at(&g, i, j, k, 0, 0);
                for (int v = 0; v < 5; ++v)
                    R[v * N + c] = r[v];
            }
    free(prim);
}

/* R(Q) at a list of points only (linear indices into the grid); out holds
 * 5 doubles per point, in point order.  For sampled checks of large grids:
 * the primitives are only evaluated where a stencil reaches. */
void orc_residual_points(int nx, int ny, int nz, double lx, double ly,
                         double lz, double gamma, double pr, double re,
                         double mach, const double *Q, int64_t npoint,
                         const int64_t *points, double *out)
{
    orc_grid g = make_grid(nx, ny, nz, lx, ly, lz, gamma, pr, re, mach);
    size_t N = npts(&g);
    /* Primitives on the whole grid are cheap compared with a residual and
     * keep this routine identical in arithmetic to orc_residual. */
    double *prim = (double *)malloc(5 * N * sizeof(double));
    primitives(&g, Q, prim);
#pragma omp parallel for schedule(dynamic)
    for (int64_t q = 0; q < npoint; ++q) {
        int64_t lin = points[q];
        int i = (int)(lin % nx);
        int j = (int)((lin / nx) % ny);
        int k = (int)(lin / ((int64_t)nx * ny));
        residual_at(&g, Q, prim, i, j, k, out + 5 * q);
    }
    free(prim);
}

/* ---------------------------------------------------------------------
 * Time advancement: the generic algorithm figure with the three-stage
 * low-storage Runge-Kutta scheme.  Per step: save-state Q_acc = Q^n; for
 * each stage k: R = R(Q); Q <- Q_acc + a_k dt R; Q_acc <- Q_acc + b_k dt R.
 * After the third stage Q holds Q^{n+1} (a_3 = b_3).
 * ------------------------------------------------------------------- */
static const double RK_A[3] = {2.0 / 3.0, 5.0 / 12.0, 3.0 / 5.0};
static const double RK_B[3] = {1.0 / 4.0, 3.0 / 20.0, 3.0 / 5.0};

void orc_rk3(int nx, int ny, int nz, double lx, double ly, double lz,
             double gamma, double pr, double re, double mach, double dt,
             int nsteps, double *Q)
{
    size_t n5 = 5 * (size_t)nx * ny * nz;
    double *R = (double *)malloc(n5 * sizeof(double));
    double *acc = (double *)malloc(n5 * sizeof(double));
    for (int step = 0; step < nsteps; ++step) {
        memcpy(acc, Q, n5 * sizeof(double));
        for (int st = 0; st < 3; ++st) {
            orc_residual(nx, ny, nz, lx, ly, lz, gamma, pr, re, mach, Q, R);
#pragma omp parallel for schedule(static)
            for (long long q = 0; q < (long long)n5; ++q) {
                Q[q] = acc[q] + RK_A[st] * dt * R[q];
                acc[q] = acc[q] + RK_B[st] * dt * R[q];
            }
        }
    }
    free(R);
    free(acc);
}

/* ---------------------------------------------------------------------
 * Taylor-Green vortex initial state (results section): on [0, 2 pi L]^3,
 *   u0 = sin(x/L) cos(y/L) cos(z/L),  u1 = -cos(x/L) sin(y/L) cos(z/L),
 *   u2 = 0,
 *   p  = 1/(gamma M^2) + (cos(2x/L) + cos(2y/L)) (2 + cos(2z/L)) / 16,
 * with rho = gamma M^2 p (so T = 1) and rho E = p/(gamma-1) + rho |u|^2 / 2.
 * L is taken per direction as length / (2 pi).
 * ------------------------------------------------------------------- */
void orc_tgv_init(int nx, int ny, int nz, double lx, double ly, double lz,
                  double gamma, double mach, double *Q)
{
    orc_grid g = make_grid(nx, ny, nz, lx, ly, lz, gamma, 1.0, 1.0, mach);
    size_t N = npts(&g);
    double two_pi = 2.0 * 3.14159265358979323846;
    double Lx = lx / two_pi, Ly = ly / two_pi, Lz = lz / two_pi;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double x = i * g.h[0] / Lx, y = j * g.h[1] / Ly;
                double z = k * g.h[2] / Lz;
                double u = sin(x) * cos(y) * cos(z);
                double v = -cos(x) * sin(y) * cos(z);
                double w = 0.0;
                double p = 1.0 / (gamma * mach * mach)
                           + (cos(2.0 * x) + cos(2.0 * y))
                                 * (2.0 + cos(2.0 * z)) / 16.0;
                double rho = gamma * mach * mach * p;
                size_t c = at(&g, i, j, k, 0, 0);
                Q[c] = rho;
                Q[N + c] = rho * u;
                Q[2 * N + c] = rho * v;
                Q[3 * N + c] = rho * w;
                Q[4 * N + c] = p / (gamma - 1.0)
                               + 0.5 * rho * (u * u + v * v + w * w);
            }
}

/* ---------------------------------------------------------------------
 * Diagnostics of a state (the quantities of the kinetic-energy /
 * enstrophy validation data set of the results section):
 *   out[0]   mass           = hx hy hz sum rho
 *   out[1-3] momentum_i     = hx hy hz sum rho u_i
 *   out[4]   energy         = hx hy hz sum rho E
 *   out[5]   kinetic energy = mean of rho |u|^2 / 2
 *   out[6]   enstrophy      = mean of rho |omega|^2 / 2, omega = curl u
 *            (fourth-order first derivatives)
 *   out[7]   dissipation    = 2 enstrophy / Re
 * Sums are plain sequential loops in grid order.
 * ------------------------------------------------------------------- */
void orc_diagnostics(int nx, int ny, int nz, double lx, double ly, double lz,
                     double gamma, double pr, double re, double mach,
                     const double *Q, double out[8])
{
    orc_grid g = make_grid(nx, ny, nz, lx, ly, lz, gamma, pr, re, mach);
    size_t N = npts(&g);
    double *prim = (double *)malloc(5 * N * sizeof(double));
    primitives(&g, Q, prim);
    const double *u[3] = {prim, prim + N, prim + 2 * N};
    double mass = 0, mom[3] = {0, 0, 0}, energy = 0, ke = 0, ens = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = at(&g, i, j, k, 0, 0);
                double rho = Q[c];
                mass += rho;
                for (int a = 0; a < 3; ++a)
                    mom[a] += Q[(1 + a) * N + c];
                energy += Q[4 * N + c];
                ke += 0.5 * rho * (u[0][c] * u[0][c] + u[1][c] * u[1][c]
                                   + u[2][c] * u[2][c]);
                double wx = d1_at(&g, u[2], i, j, k, 1)
                            - d1_at(&g, u[1], i, j, k, 2);
                double wy = d1_at(&g, u[0], i, j, k, 2)
                            - d1_at(&g, u[2], i, j, k, 0);
                double wz = d1_at(&g, u[1], i, j, k, 0)
                            - d1_at(&g, u[0], i, j, k, 1);
                ens += 0.5 * rho * (wx * wx + wy * wy + wz * wz);
            }
    double vol = g.h[0] * g.h[1] * g.h[2];
    out[0] = vol * mass;
    out[1] = vol * mom[0];
    out[2] = vol * mom[1];
    out[3] = vol * mom[2];
    out[4] = vol * energy;
    out[5] = ke / (double)N;
    out[6] = ens / (double)N;
    out[7] = 2.0 * out[6] / re;
    free(prim);
}
