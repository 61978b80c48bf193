/*
 * FP64 CPU oracle for the direct-sum boundary-integral linearized
 * Poisson-Boltzmann solver of Geng & Jacob, "A GPU-accelerated Direct-sum
 * Boundary Integral Poisson-Boltzmann Solver" (arXiv:1301.5885).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the HIP library is checked against.  It shares no code with
 * the library; only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.
 *
 * Every quantity is written out from its definition in the paper, in double
 * precision, with sums over j taken in index order:
 *   - fundamental solutions G0, Gk: Section 2.1, eq. (eq_potential);
 *   - kernels K1..K4 and source terms S1, S2: Section 2.1, eqs. (Eq_Ls),
 *     (Eq_Ss), used in (eqbim_3)/(eqbim_4);
 *   - flat-triangle centroid collocation, self term dropped: Section 2.2;
 *   - discrete product Au: Section 2.2, eqs. (eqdbef1)/(eqdbef2);
 *   - restarted GMRES with x0 = 0 and warm restarts: Section 2.2 and
 *     Section 2.4 (Saad & Schultz);
 *   - solvation energy: Section 2.3, eq. (solvation_energy).
 *
 * Readings where the paper is silent or inconsistent:
 *   - eps = eps2/eps1.  The paper prints eps1/eps2 after (Eq_Ls), but its
 *     own kernels and the (1+eps)/2, (1+1/eps)/2 diagonals follow from the
 *     interface conditions only with eps = eps2/eps1.
 *   - S1 and S2 carry a factor 1/eps1 (from eq. (eq1)); moot at eps1 = 1.
 *   - Charges are in units of e, the 1/(4 pi) stays inside G, and energies
 *     are converted to kcal/mol with 4 pi * 332.0716 kcal A/(mol e^2).
 *   - Element data: centroid = vertex mean, normal = normalised
 *     (v1-v0)x(v2-v0), area = |(v1-v0)x(v2-v0)|/2.
 *   - GMRES stops when the explicit relative residual ||b-Ax||/||b|| <= tol;
 *     inside a cycle the Givens estimate |g_{j+1}|/||b|| ends the cycle early.
 *
 * Parallelism: OpenMP over independent output rows only; each row's sum is
 * sequential in j, so results do not depend on the thread count.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846
#define ORACLE_COULOMB 332.0716 /* kcal A / (mol e^2) */

/* Threads an OpenMP region of the oracle uses (1 without OpenMP).          */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of later OpenMP regions (t >= 1; for timing runs).       */
void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t >= 1) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* Element data from a triangle mesh (Section 2.2).                          */
/* ------------------------------------------------------------------------ */
void oracle_mesh_elements(int64_t nv, const double *xyz, int64_t nf,
                          const int32_t *tri, double *cx, double *cy,
                          double *cz, double *nx, double *ny, double *nz,
                          double *area)
{
    (void)nv;
    for (int64_t f = 0; f < nf; ++f) {
        const double *a = xyz + 3 * (int64_t)tri[3 * f + 0];
        const double *b = xyz + 3 * (int64_t)tri[3 * f + 1];
        const double *c = xyz + 3 * (int64_t)tri[3 * f + 2];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1],
                        e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
        double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        cx[f] = (a[0] + b[0] + c[0]) / 3.0;
        cy[f] = (a[1] + b[1] + c[1]) / 3.0;
        cz[f] = (a[2] + b[2] + c[2]) / 3.0;
        nx[f] = cr[0] / len;
        ny[f] = cr[1] / len;
        nz[f] = cr[2] / len;
        area[f] = 0.5 * len;
    }
}

/* ------------------------------------------------------------------------ */
/* Fundamental solutions and their normal derivatives (eq_potential).       */
/* x is the target with unit normal nux, y the source with unit normal nuy. */
/* ------------------------------------------------------------------------ */
typedef struct {
    double G0, Gk;          /* G0(x,y), Gk(x,y)                        */
    double dG0_dny, dGk_dny; /* d/d nu_y                                 */
    double dG0_dnx, dGk_dnx; /* d/d nu_x                                 */
    double d2G0, d2Gk;       /* d^2 / (d nu_x d nu_y)                    */
} green_t;

static green_t greens(const double x[3], const double nux[3],
                      const double y[3], const double nuy[3], double kappa)
{
    /* G(r) with r = |x - y|.  grad_y r = -(x-y)/r, grad_x r = (x-y)/r.     */
    double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double ux = d[0] * nux[0] + d[1] * nux[1] + d[2] * nux[2];  /* (x-y).nu_x */
    double uy = d[0] * nuy[0] + d[1] * nuy[1] + d[2] * nuy[2];  /* (x-y).nu_y */
    double nn = nux[0] * nuy[0] + nux[1] * nuy[1] + nux[2] * nuy[2];
    double e = exp(-kappa * r);
    double fourpi = 4.0 * ORACLE_PI;
    green_t g;
    /* G0 = 1/(4 pi r); dG0/dr = -1/(4 pi r^2); d2G0/dr2 = 2/(4 pi r^3)     */
    /* Gk = e^{-k r}/(4 pi r); dGk/dr = -e (1 + k r)/(4 pi r^2);            */
    /* d2Gk/dr2 = e (2 + 2 k r + k^2 r^2)/(4 pi r^3)                        */
    double dG0dr = -1.0 / (fourpi * r * r);
    double dGkdr = -e * (1.0 + kappa * r) / (fourpi * r * r);
    double d2G0dr2 = 2.0 / (fourpi * r * r * r);
    double d2Gkdr2 = e * (2.0 + 2.0 * kappa * r + kappa * kappa * r * r)
                     / (fourpi * r * r * r);
    /* directional derivatives of r:                                        */
    /*   dr/dnu_y = -uy/r, dr/dnu_x = ux/r,                                 */
    /*   d2r/(dnu_x dnu_y) = (-nn + ux uy / r^2)/r                          */
    double drdny = -uy / r;
    double drdnx = ux / r;
    double d2r = (-nn + ux * uy / (r * r)) / r;
    g.G0 = 1.0 / (fourpi * r);
    g.Gk = e / (fourpi * r);
    g.dG0_dny = dG0dr * drdny;
    g.dGk_dny = dGkdr * drdny;
    g.dG0_dnx = dG0dr * drdnx;
    g.dGk_dnx = dGkdr * drdnx;
    /* chain rule: d2G = G''(r) r_x r_y + G'(r) r_xy                        */
    g.d2G0 = d2G0dr2 * drdnx * drdny + dG0dr * d2r;
    g.d2Gk = d2Gkdr2 * drdnx * drdny + dGkdr * d2r;
    return g;
}

/* K1..K4 of (Eq_Ls) with eps = eps2/eps1.                                  */
void oracle_pair_kernels(const double x[3], const double nux[3],
                         const double y[3], const double nuy[3],
                         double kappa, double eps, double K[4])
{
    green_t g = greens(x, nux, y, nuy, kappa);
    K[0] = g.G0 - g.Gk;                       /* K1 */
    K[1] = eps * g.dGk_dny - g.dG0_dny;       /* K2 */
    K[2] = g.dG0_dnx - g.dGk_dnx / eps;       /* K3 */
    K[3] = g.d2Gk - g.d2G0;                   /* K4 */
}

/* Fundamental-solution values exposed for the finite-difference pins.      */
void oracle_greens(const double x[3], const double nux[3], const double y[3],
                   const double nuy[3], double kappa, double out[8])
{
    green_t g = greens(x, nux, y, nuy, kappa);
    out[0] = g.G0; out[1] = g.Gk;
    out[2] = g.dG0_dny; out[3] = g.dGk_dny;
    out[4] = g.dG0_dnx; out[5] = g.dGk_dnx;
    out[6] = g.d2G0; out[7] = g.d2Gk;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side b = [S1(x_i); S2(x_i)] / eps1 (Eq_Ss).                    */
/* ------------------------------------------------------------------------ */
void oracle_rhs(int64_t n, const double *cx, const double *cy,
                const double *cz, const double *nx, const double *ny,
                const double *nz, int64_t nc, const double *px,
                const double *py, const double *pz, const double *q,
                double eps1, double *b)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x[3] = {cx[i], cy[i], cz[i]};
        double nu[3] = {nx[i], ny[i], nz[i]};
        double zero[3] = {0.0, 0.0, 0.0};
        double s1 = 0.0, s2 = 0.0;
        for (int64_t k = 0; k < nc; ++k) {
            double y[3] = {px[k], py[k], pz[k]};
            green_t g = greens(x, nu, y, zero, 0.0);
            s1 += q[k] * g.G0;
            s2 += q[k] * g.dG0_dnx;
        }
        b[i] = s1 / eps1;
        b[n + i] = s2 / eps1;
    }
}

/* ------------------------------------------------------------------------ */
/* y = A u, (eqdbef1)/(eqdbef2); u = [phi; psi], psi = d phi_1 / d nu.       */
/* ------------------------------------------------------------------------ */
void oracle_matvec(int64_t n, const double *cx, const double *cy,
                   const double *cz, const double *nx, const double *ny,
                   const double *nz, const double *area, double eps1,
                   double eps2, double kappa, const double *u, double *y)
{
    double eps = eps2 / eps1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double xi[3] = {cx[i], cy[i], cz[i]};
        double ni[3] = {nx[i], ny[i], nz[i]};
        double s_top = 0.0, s_bot = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue; /* singular self term removed (Section 2.2) */
            double xj[3] = {cx[j], cy[j], cz[j]};
            double nj[3] = {nx[j], ny[j], nz[j]};
            double K[4];
            oracle_pair_kernels(xi, ni, xj, nj, kappa, eps, K);
            s_top += area[j] * (K[0] * u[n + j] + K[1] * u[j]);
            s_bot += area[j] * (K[2] * u[n + j] + K[3] * u[j]);
        }
        y[i] = 0.5 * (1.0 + eps) * u[i] - s_top;
        y[n + i] = 0.5 * (1.0 + 1.0 / eps) * u[n + i] - s_bot;
    }
}

/* Selected rows of A u: rows[r] in [0, 2n).  For sampled parity at sizes   */
/* where a full product is too slow.                                        */
void oracle_matvec_rows(int64_t n, const double *cx, const double *cy,
                        const double *cz, const double *nx, const double *ny,
                        const double *nz, const double *area, double eps1,
                        double eps2, double kappa, const double *u,
                        int64_t nrows, const int64_t *rows, double *out)
{
    double eps = eps2 / eps1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t row = rows[r];
        int64_t i = row < n ? row : row - n;
        int bottom = row >= n;
        double xi[3] = {cx[i], cy[i], cz[i]};
        double ni[3] = {nx[i], ny[i], nz[i]};
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double xj[3] = {cx[j], cy[j], cz[j]};
            double nj[3] = {nx[j], ny[j], nz[j]};
            double K[4];
            oracle_pair_kernels(xi, ni, xj, nj, kappa, eps, K);
            if (!bottom)
                s += area[j] * (K[0] * u[n + j] + K[1] * u[j]);
            else
                s += area[j] * (K[2] * u[n + j] + K[3] * u[j]);
        }
        out[r] = bottom ? 0.5 * (1.0 + 1.0 / eps) * u[n + i] - s
                        : 0.5 * (1.0 + eps) * u[i] - s;
    }
}

/* Dense 2n x 2n matrix of the same operator, row-major (small n only).     */
void oracle_assemble(int64_t n, const double *cx, const double *cy,
                     const double *cz, const double *nx, const double *ny,
                     const double *nz, const double *area, double eps1,
                     double eps2, double kappa, double *A)
{
    double eps = eps2 / eps1;
    int64_t m = 2 * n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[3] = {cx[i], cy[i], cz[i]};
        double ni[3] = {nx[i], ny[i], nz[i]};
        double *top = A + i * m, *bot = A + (n + i) * m;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) {
                top[j] = 0.5 * (1.0 + eps);
                top[n + j] = 0.0;
                bot[j] = 0.0;
                bot[n + j] = 0.5 * (1.0 + 1.0 / eps);
                continue;
            }
            double xj[3] = {cx[j], cy[j], cz[j]};
            double nj[3] = {nx[j], ny[j], nz[j]};
            double K[4];
            oracle_pair_kernels(xi, ni, xj, nj, kappa, eps, K);
            top[j] = -area[j] * K[1];
            top[n + j] = -area[j] * K[0];
            bot[j] = -area[j] * K[3];
            bot[n + j] = -area[j] * K[2];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Restarted GMRES(m) (Saad & Schultz), x0 given (zero in the paper).       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t iterations;  /* Arnoldi steps                                  */
    int64_t matvecs;     /* products with A, explicit residuals included   */
    int64_t restarts;    /* completed cycles                               */
    double rel_residual; /* explicit ||b - A x|| / ||b|| at exit           */
    int64_t converged;
} oracle_gmres_info;

static double dot(int64_t m, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
}

int oracle_gmres(int64_t n, const double *cx, const double *cy,
                 const double *cz, const double *nx, const double *ny,
                 const double *nz, const double *area, double eps1,
                 double eps2, double kappa, const double *b, int64_t restart,
                 double tol, int64_t maxit, double *x, oracle_gmres_info *info)
{
    int64_t len = 2 * n, m = restart;
    double *V = malloc(sizeof(double) * len * (m + 1));
    double *H = calloc((m + 1) * m, sizeof(double)); /* H[i*m + j] */
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *g = malloc(sizeof(double) * (m + 1)), *yk = malloc(sizeof(double) * m);
    double *r = malloc(sizeof(double) * len), *w = malloc(sizeof(double) * len);
    if (!V || !H || !cs || !sn || !g || !yk || !r || !w) return -4;

    memset(info, 0, sizeof(*info));
    double beta = sqrt(dot(len, b, b));
    if (beta == 0.0) {
        memset(x, 0, sizeof(double) * len);
        info->converged = 1;
        goto done;
    }
    /* initial residual */
    int x_zero = 1;
    for (int64_t i = 0; i < len; ++i) if (x[i] != 0.0) { x_zero = 0; break; }
    if (x_zero) {
        memcpy(r, b, sizeof(double) * len);
    } else {
        oracle_matvec(n, cx, cy, cz, nx, ny, nz, area, eps1, eps2, kappa, x, w);
        info->matvecs++;
        for (int64_t i = 0; i < len; ++i) r[i] = b[i] - w[i];
    }
    double rnorm = sqrt(dot(len, r, r));
    info->rel_residual = rnorm / beta;
    if (rnorm / beta <= tol) { info->converged = 1; goto done; }

    while (info->iterations < maxit) {
        memset(H, 0, sizeof(double) * (m + 1) * m);
        for (int64_t i = 0; i < len; ++i) V[i] = r[i] / rnorm;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = rnorm;
        int64_t k = 0; /* steps taken in this cycle */
        for (int64_t j = 0; j < m; ++j) {
            double *vj = V + j * len;
            oracle_matvec(n, cx, cy, cz, nx, ny, nz, area, eps1, eps2, kappa,
                          vj, w);
            info->matvecs++;
            /* modified Gram-Schmidt */
            for (int64_t i = 0; i <= j; ++i) {
                double *vi = V + i * len;
                double h = dot(len, w, vi);
                H[i * m + j] = h;
                for (int64_t t = 0; t < len; ++t) w[t] -= h * vi[t];
            }
            double hn = sqrt(dot(len, w, w));
            H[(j + 1) * m + j] = hn;
            /* previous rotations on column j */
            for (int64_t i = 0; i < j; ++i) {
                double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * m + j], c = H[(j + 1) * m + j];
            double den = hypot(a, c);
            cs[j] = a / den;
            sn[j] = c / den;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            info->iterations++;
            k = j + 1;
            if (fabs(g[j + 1]) / beta <= tol || info->iterations >= maxit ||
                hn == 0.0)
                break;
            double *vn = V + (j + 1) * len;
            for (int64_t t = 0; t < len; ++t) vn[t] = w[t] / hn;
        }
        /* back substitution H(0:k,0:k) y = g(0:k) */
        for (int64_t i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int64_t t = i + 1; t < k; ++t) s -= H[i * m + t] * yk[t];
            yk[i] = s / H[i * m + i];
        }
        for (int64_t i = 0; i < k; ++i) {
            double *vi = V + i * len;
            for (int64_t t = 0; t < len; ++t) x[t] += yk[i] * vi[t];
        }
        info->restarts++;
        /* explicit residual: warm restart from the current iterate */
        oracle_matvec(n, cx, cy, cz, nx, ny, nz, area, eps1, eps2, kappa, x, w);
        info->matvecs++;
        for (int64_t i = 0; i < len; ++i) r[i] = b[i] - w[i];
        rnorm = sqrt(dot(len, r, r));
        info->rel_residual = rnorm / beta;
        if (rnorm / beta <= tol) { info->converged = 1; break; }
        if (rnorm == 0.0) { info->converged = 1; break; }
    }
done:
    free(V); free(H); free(cs); free(sn); free(g); free(yk); free(r); free(w);
    return info->converged ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* Reaction potential at the charges and solvation energy (solvation_energy)*/
/* ------------------------------------------------------------------------ */
void oracle_reaction_potential(int64_t n, const double *cx, const double *cy,
                               const double *cz, const double *nx,
                               const double *ny, const double *nz,
                               const double *area, double eps1, double eps2,
                               double kappa, const double *u, int64_t nc,
                               const double *px, const double *py,
                               const double *pz, double *phi_reac)
{
    double eps = eps2 / eps1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nc; ++k) {
        double xk[3] = {px[k], py[k], pz[k]};
        double zero[3] = {0.0, 0.0, 0.0}; /* K1, K2 do not use nu_x */
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double xj[3] = {cx[j], cy[j], cz[j]};
            double nj[3] = {nx[j], ny[j], nz[j]};
            double K[4];
            oracle_pair_kernels(xk, zero, xj, nj, kappa, eps, K);
            s += area[j] * (K[0] * u[n + j] + K[1] * u[j]);
        }
        phi_reac[k] = s;
    }
}

double oracle_energy(int64_t n, const double *cx, const double *cy,
                     const double *cz, const double *nx, const double *ny,
                     const double *nz, const double *area, double eps1,
                     double eps2, double kappa, const double *u, int64_t nc,
                     const double *px, const double *py, const double *pz,
                     const double *q)
{
    double *phi = malloc(sizeof(double) * (nc > 0 ? nc : 1));
    if (!phi) return NAN;
    oracle_reaction_potential(n, cx, cy, cz, nx, ny, nz, area, eps1, eps2,
                              kappa, u, nc, px, py, pz, phi);
    double e = 0.0;
    for (int64_t k = 0; k < nc; ++k) e += q[k] * phi[k];
    free(phi);
    return 0.5 * e * 4.0 * ORACLE_PI * ORACLE_COULOMB;
}
