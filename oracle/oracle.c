/*
 * oracle.c -- plain FP64 CPU oracle for the quasi-implicit alternating-direction
 * isogeometric (IGA-ADS) wildfire time stepper.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP library.
 *
 * It is written to be checked against the paper by eye: Cox-de Boor basis
 * functions, closed-form Gauss-Legendre rules, quadrature of the 1D matrices
 * (Section 3.1, "Matrix formulation"), direct element-by-element quadrature of
 * the right-hand side (variational forms of Sections 3.1 and 3.2 and the
 * compute_rhs listing of Section 7), a banded LU without pivoting, and the
 * Kronecker-product solves eq. (matrixPR) and eq. (matrixCN): x-lines first,
 * then y-lines.  No sum factorisation, no fusion, no reordering.
 *
 * Three schemes: Peaceman-Rachford (Section 3.1), Strang splitting with
 * Crank-Nicolson substeps (Section 3.2), and the explicit L2-projection step
 * the paper uses as its accuracy baseline for eq. (linear) in Section 6.1:
 * every term of the equation evaluated at T^n and weighted by tau, then the
 * (Mx (x) My) solve -- the compute_rhs listing of Section 7 read as one step.
 *
 * Readings of points the paper leaves open (all FP64):
 *  - F is evaluated from the state entering each substep (PR: T^n then
 *    T^{n+1/2}; Strang: S1 from T^n with weight tau/2, S3 from T** with weight
 *    tau/2, S2 has none).
 *  - The implicit wind is a constant bbar inside the 1D operators; the rest,
 *    (b - bbar).grad T, is explicit.
 *  - The ignition indicator is [T > T_ig and fuel > fuel_thr] with strict
 *    inequalities, evaluated per quadrature point on spline values; the
 *    Arrhenius factor is evaluated only where the indicator is 1.
 *  - The fuel is updated once per full step, explicitly from (T^n, fuel^n),
 *    and projected with Mx (x) My (the compute_rhs listing of Section 7).
 *  - p + 1 Gauss points per direction per element.
 *
 * Pins (tests/test_oracle_pins.py, tests/test_manufactured.py,
 * tests/test_ring_of_fire.py) check every function against closed forms,
 * library routines, dense brute force and invariants of the schemes.
 * Parity unpinned: the values of c_ign and fuel_rate (the reaction-rate scale
 * A_r and M/M1 are not given in the paper); with them the full model is
 * checked only for boundedness and consistency under dt halving.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Constants: Table (tab:parameters) of Section 2.2 divided by rho * c_p.    */
/* ------------------------------------------------------------------------ */
void oracle_default_coeffs(oracle_coeffs *c)
{
    const double cp = 1.0, rho = 1.293, kappa = 0.3, sigma = 5.67e-8;
    const double eps = 0.05, ch = 1.0, hc = -70.0, cw = 0.5, chi = 2e-2;
    const double t_amb = 300.0, t_ig = 800.0;
    const double delta_x = 3.5e-2 / eps, delta_z = 1.5 * eps;
    /* Reaction-rate scale of the listing (A_r, M/M1 are not given in the
     * paper): A_r = 1.5e-4, M/M1 = 1. */
    const double a_r = 1.5e-4, m_ratio = 1.0;
    const double rc = rho * cp;

    c->c_adv = cw;                                   /* Q_W / (rho c_p)   */
    c->c_diff = kappa / rc;                          /* q_C               */
    c->c_react = -chi / rc;                          /* linear Q_conv     */
    c->c_nld = 4.0 * sigma * eps * delta_x / rc;     /* q_r               */
    c->c_rad = sigma * eps / (delta_z * rc);         /* Q_rz, T^4 part    */
    c->c_forcing = (chi * t_amb + sigma * eps * pow(t_amb, 4) / delta_z) / rc;
    /* R_C / (rho c_p) with the listing's 1e4 factor: -1e4 c_h h_c (M/M1) A_r */
    c->c_ign = -1e4 * ch * hc * m_ratio * a_r / cp;
    c->t_ig = t_ig;
    c->fuel_thr = 0.2;
    c->t_act = 300.0;
    c->fuel_rate = 3e2 * a_r;                        /* fuel ODE of listing */
}

/* ------------------------------------------------------------------------ */
/* Knots, Gauss rule, Cox-de Boor basis (Section 3.1)                        */
/* ------------------------------------------------------------------------ */
int oracle_knots(int n, int p, double L, double *t)
{
    if (n < 1 || p < 0 || !t) return 1;
    for (int k = 0; k <= p; ++k) t[k] = 0.0;
    for (int k = 1; k < n; ++k) t[p + k] = L * (double)k / (double)n;
    for (int k = 0; k <= p; ++k) t[n + p + k] = L;
    return 0;
}

int oracle_gauss(int npts, double *x, double *w)
{
    switch (npts) {
    case 1:
        x[0] = 0.0; w[0] = 2.0;
        return 0;
    case 2:
        x[0] = -1.0 / sqrt(3.0); x[1] = -x[0];
        w[0] = w[1] = 1.0;
        return 0;
    case 3:
        x[0] = -sqrt(3.0 / 5.0); x[1] = 0.0; x[2] = -x[0];
        w[0] = w[2] = 5.0 / 9.0; w[1] = 8.0 / 9.0;
        return 0;
    case 4: {
        double a = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
        double b = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
        x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
        w[1] = w[2] = (18.0 + sqrt(30.0)) / 36.0;
        w[0] = w[3] = (18.0 - sqrt(30.0)) / 36.0;
        return 0;
    }
    default:
        return 1;
    }
}

/* N_{i,k}(x) by the Cox-de Boor recursion with 0/0 := 0; the last non-empty
 * knot span is closed on the right so that the basis is defined at x = L. */
static double cdb(const double *t, int i, int k, double x, int last_span)
{
    if (k == 0) {
        if (t[i] <= x && x < t[i + 1]) return 1.0;
        if (i == last_span && x == t[i + 1]) return 1.0;
        return 0.0;
    }
    double r = 0.0;
    double d1 = t[i + k] - t[i], d2 = t[i + k + 1] - t[i + 1];
    if (d1 > 0.0) r += (x - t[i]) / d1 * cdb(t, i, k - 1, x, last_span);
    if (d2 > 0.0) r += (t[i + k + 1] - x) / d2 * cdb(t, i + 1, k - 1, x, last_span);
    return r;
}

/* d/dx N_{i,k}(x) = k/(t_{i+k}-t_i) N_{i,k-1} - k/(t_{i+k+1}-t_{i+1}) N_{i+1,k-1} */
static double cdb_der(const double *t, int i, int k, double x, int last_span)
{
    double r = 0.0;
    double d1 = t[i + k] - t[i], d2 = t[i + k + 1] - t[i + 1];
    if (d1 > 0.0) r += k / d1 * cdb(t, i, k - 1, x, last_span);
    if (d2 > 0.0) r -= k / d2 * cdb(t, i + 1, k - 1, x, last_span);
    return r;
}

int oracle_basis_eval(int n, int p, double L, int deriv, const double *xs,
                      int nx, double *out)
{
    if (n < 1 || p < 1 || p > 3) return 1;
    int N = n + p;
    double *t = malloc(sizeof(double) * (size_t)(n + 2 * p + 1));
    if (!t) return 2;
    oracle_knots(n, p, L, t);
    for (int k = 0; k < nx; ++k)
        for (int i = 0; i < N; ++i)
            out[(size_t)k * N + i] = deriv ? cdb_der(t, i, p, xs[k], n + p - 1)
                                           : cdb(t, i, p, xs[k], n + p - 1);
    free(t);
    return 0;
}

/* Per-direction quadrature data: on element e (knot span [t_{p+e},
 * t_{p+e+1}]) the non-zero functions are N_e ... N_{e+p}. */
typedef struct {
    int n, p, N, nq;
    double L;
    double *xq;   /* [n * nq] physical quadrature points              */
    double *wq;   /* [n * nq] weights times the element Jacobian h/2  */
    double *bv;   /* [(e * nq + q) * (p+1) + a] values N_{e+a}(x_q)   */
    double *bd;   /* same, first derivatives                          */
} dir1d;

static void dir_free(dir1d *D)
{
    free(D->xq); free(D->wq); free(D->bv); free(D->bd);
    memset(D, 0, sizeof *D);
}

static int dir_init(dir1d *D, int n, int p, double L)
{
    memset(D, 0, sizeof *D);
    if (n < 1 || p < 1 || p > 3 || !(L > 0.0)) return 1;
    D->n = n; D->p = p; D->N = n + p; D->nq = p + 1; D->L = L;
    double *t = malloc(sizeof(double) * (size_t)(n + 2 * p + 1));
    size_t nqt = (size_t)n * D->nq;
    D->xq = malloc(sizeof(double) * nqt);
    D->wq = malloc(sizeof(double) * nqt);
    D->bv = malloc(sizeof(double) * nqt * (p + 1));
    D->bd = malloc(sizeof(double) * nqt * (p + 1));
    if (!t || !D->xq || !D->wq || !D->bv || !D->bd) { free(t); dir_free(D); return 2; }
    oracle_knots(n, p, L, t);
    double gx[4], gw[4];
    oracle_gauss(D->nq, gx, gw);
    for (int e = 0; e < n; ++e) {
        double a = t[p + e], b = t[p + e + 1], h = b - a;
        for (int q = 0; q < D->nq; ++q) {
            size_t eq = (size_t)e * D->nq + q;
            double x = a + 0.5 * (gx[q] + 1.0) * h;
            D->xq[eq] = x;
            D->wq[eq] = gw[q] * 0.5 * h;
            for (int k = 0; k <= p; ++k) {
                D->bv[eq * (p + 1) + k] = cdb(t, e + k, p, x, n + p - 1);
                D->bd[eq * (p + 1) + k] = cdb_der(t, e + k, p, x, n + p - 1);
            }
        }
    }
    free(t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 1D matrices (Section 3.1):  M_ik = int B_i B_k,  K_ik = int B_i' B_k',    */
/* G_ik = int B_i B_k'  (row i = test function).  Band storage.              */
/* ------------------------------------------------------------------------ */
static int mat1d_from_dir(const dir1d *D, int kind, double *band)
{
    int p = D->p, N = D->N, W = 2 * p + 1;
    memset(band, 0, sizeof(double) * (size_t)N * W);
    for (int e = 0; e < D->n; ++e)
        for (int q = 0; q < D->nq; ++q) {
            size_t eq = (size_t)e * D->nq + q;
            const double *v = D->bv + eq * (p + 1), *d = D->bd + eq * (p + 1);
            for (int a = 0; a <= p; ++a)
                for (int c = 0; c <= p; ++c) {
                    double val;
                    if (kind == 0) val = v[a] * v[c];
                    else if (kind == 1) val = d[a] * d[c];
                    else val = v[a] * d[c];
                    int i = e + a, k = e + c;
                    band[(size_t)i * W + (k - i + p)] += D->wq[eq] * val;
                }
        }
    return 0;
}

int oracle_mat1d(int n, int p, double L, int kind, double *band)
{
    if (kind < 0 || kind > 2 || !band) return 1;
    dir1d D;
    int rc = dir_init(&D, n, p, L);
    if (rc) return rc;
    mat1d_from_dir(&D, kind, band);
    dir_free(&D);
    return 0;
}

/* Implicit directional operators of eq. (varPR_wildfire) / eq. (varCN):
 *   x (with reaction): A = (1 - g C_react) M + g (C_diff K + C_adv bbar_x G)
 *   y:                 A = M + g (C_diff K + C_adv bbar_y G)
 * and the explicit counterpart B (signs of the g terms flipped), where
 * g = tau/2 (PR, both directions; Strang y) or tau/4 (Strang x).  The explicit
 * scheme inverts the mass matrices only: g = 0, A = B = M. */
static void operator_gamma(const oracle_desc *d, int dir, double *g, double *react)
{
    if (d->scheme == ORACLE_PR) *g = 0.5 * d->dt;
    else if (d->scheme == ORACLE_EXPLICIT) *g = 0.0;
    else *g = (dir == 0) ? 0.25 * d->dt : 0.5 * d->dt;
    *react = (dir == 0) ? d->c.c_react : 0.0;
}

int oracle_operator(const oracle_desc *d, int dir, int which, double *band)
{
    if (!d || !band || dir < 0 || dir > 1 || which < 0 || which > 2) return 1;
    int n = dir ? d->nel_y : d->nel_x;
    double L = dir ? d->len_y : d->len_x;
    double bbar = dir ? d->bbar_y : d->bbar_x;
    int p = d->p, W = 2 * p + 1;
    dir1d D;
    int rc = dir_init(&D, n, p, L);
    if (rc) return rc;
    int N = D.N;
    double *M = malloc(sizeof(double) * (size_t)N * W);
    double *K = malloc(sizeof(double) * (size_t)N * W);
    double *G = malloc(sizeof(double) * (size_t)N * W);
    if (!M || !K || !G) { free(M); free(K); free(G); dir_free(&D); return 2; }
    mat1d_from_dir(&D, 0, M);
    mat1d_from_dir(&D, 1, K);
    mat1d_from_dir(&D, 2, G);
    double g, react;
    operator_gamma(d, dir, &g, &react);
    for (size_t k = 0; k < (size_t)N * W; ++k) {
        double lin = d->c.c_diff * K[k] + d->c.c_adv * bbar * G[k];
        if (which == 1) band[k] = M[k];
        else if (which == 0) band[k] = (1.0 - g * react) * M[k] + g * lin;
        else band[k] = (1.0 + g * react) * M[k] - g * lin;
    }
    free(M); free(K); free(G);
    dir_free(&D);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Banded LU without pivoting (Doolittle) and the line solves                */
/* ------------------------------------------------------------------------ */
static void band_lu(int N, int p, double *a)
{
    int W = 2 * p + 1;
#define AB(i, k) a[(size_t)(i) * W + ((k) - (i) + p)]
    for (int k = 0; k < N; ++k) {
        int iend = k + p < N - 1 ? k + p : N - 1;
        for (int i = k + 1; i <= iend; ++i) {
            double l = AB(i, k) / AB(k, k);
            AB(i, k) = l;
            for (int j = k + 1; j <= iend; ++j) AB(i, j) -= l * AB(k, j);
        }
    }
#undef AB
}

static void lu_solve_one(int N, int p, const double *lu, double *x, long stride)
{
    int W = 2 * p + 1;
#define LU(i, k) lu[(size_t)(i) * W + ((k) - (i) + p)]
    for (int i = 0; i < N; ++i) {
        double s = x[i * stride];
        for (int k = (i - p > 0 ? i - p : 0); k < i; ++k) s -= LU(i, k) * x[k * stride];
        x[i * stride] = s;
    }
    for (int i = N - 1; i >= 0; --i) {
        double s = x[i * stride];
        int kend = i + p < N - 1 ? i + p : N - 1;
        for (int k = i + 1; k <= kend; ++k) s -= LU(i, k) * x[k * stride];
        x[i * stride] = s / LU(i, i);
    }
#undef LU
}

int oracle_band_solve(int N, int p, const double *band, double *x, int nrhs,
                      long stride, long dist)
{
    int W = 2 * p + 1;
    double *lu = malloc(sizeof(double) * (size_t)N * W);
    if (!lu) return 2;
    memcpy(lu, band, sizeof(double) * (size_t)N * W);
    band_lu(N, p, lu);
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrhs; ++r) lu_solve_one(N, p, lu, x + (size_t)r * dist, stride);
    free(lu);
    return 0;
}

/* y = band * x along every line of direction dir of the 2D field X. */
static void band_apply_lines(const oracle_desc *d, int dir, const double *band, double *X)
{
    int p = d->p, W = 2 * p + 1;
    int Nx = d->nel_x + p, Ny = d->nel_y + p;
    int N = dir ? Ny : Nx, nlines = dir ? Nx : Ny;
    long stride = dir ? 1 : Ny, dist = dir ? Ny : 1;
#pragma omp parallel
    {
        double *tmp = malloc(sizeof(double) * (size_t)N);
#pragma omp for schedule(static)
        for (int r = 0; r < nlines; ++r) {
            double *x = X + (size_t)r * dist;
            for (int i = 0; i < N; ++i) {
                double s = 0.0;
                for (int k = i - p; k <= i + p; ++k)
                    if (k >= 0 && k < N) s += band[(size_t)i * W + (k - i + p)] * x[k * stride];
                tmp[i] = s;
            }
            for (int i = 0; i < N; ++i) x[i * stride] = tmp[i];
        }
        free(tmp);
    }
}

int oracle_line_solve(const oracle_desc *d, int dir, int which, double *X)
{
    if (!d || !X || dir < 0 || dir > 1 || which < 0 || which > 2) return 1;
    int p = d->p, W = 2 * p + 1;
    int Nx = d->nel_x + p, Ny = d->nel_y + p;
    int N = dir ? Ny : Nx, nlines = dir ? Nx : Ny;
    long stride = dir ? 1 : Ny, dist = dir ? Ny : 1;
    double *band = malloc(sizeof(double) * (size_t)N * W);
    if (!band) return 2;
    int rc = 0;
    if (which == 2) {
        rc = oracle_operator(d, dir, 2, band);
        if (!rc) band_apply_lines(d, dir, band, X);
        if (!rc) rc = oracle_operator(d, dir, 0, band);
    } else {
        rc = oracle_operator(d, dir, which, band);
    }
    if (!rc) rc = oracle_band_solve(N, p, band, X, nlines, stride, dist);
    free(band);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side by direct quadrature                                       */
/* ------------------------------------------------------------------------ */
#define TWO_PI 6.283185307179586476925286766559

static void wind_at(const oracle_desc *d, double x, double y, double *bx, double *by)
{
    if (d->wind_kind == ORACLE_WIND_SINCOS) {
        *bx = d->bx + d->ax * sin(TWO_PI * y / d->len_y);
        *by = d->by + d->ay * cos(TWO_PI * x / d->len_x);
    } else {
        *bx = d->bx;
        *by = d->by;
    }
}

/* Weak form of one substep with explicit F, in the variables of eq.
 * (varPR_wildfire) and eq. (varCN):
 *   R_ij = sum_e sum_q w |J| [ S v - ax ( C_diff S_x v_x + C_adv bbar_x S_x v - C_react S v )
 *                                  - ay ( C_diff S_y v_y + C_adv bbar_y S_y v )
 *                              + beta ( f v - C_nld S^3 grad S . grad v ) ]
 * where ax, ay weigh the explicit linear part of L1 (x, with the reaction)
 * and L2 (y): one of them is zero in a PR or Strang substep, both are tau in
 * the explicit scheme,
 *   f = -C_adv (b - bbar).grad S + C_forcing - C_rad S^4
 *       + [S > T_ig and fuel > thr] C_ign S exp(-T_act / S)
 * plus, when src is given, a source s sampled at the quadrature points (the
 * forcing f of eq. (linear) / eq. (nonlinear) in the manufactured-solution
 * study of Section 6.1), src[(ex*nq + qx) * (nel_y*nq) + ey*nq + qy];
 * and, when rhs_fuel is given, the fuel right-hand side of the compute_rhs
 * listing,  fuel v - tau * rate * [ign] S exp(-T_act/S) fuel v. */
/* Elements whose ignition decision is within (dT, dF) of its thresholds at
 * some quadrature point (test support: there a lower-precision evaluation of
 * S or fuel may legitimately decide the other way). */
typedef struct {
    double dT, dF;
    unsigned char *flags;   /* [nel_x][nel_y], set to 1, never cleared */
} ambiguity;

static int assemble_quadrature(const oracle_desc *d, double ax, double ay,
                               double beta, const double *T, const double *fuel,
                               const double *src, double *rhs_T, double *rhs_fuel,
                               const ambiguity *amb)
{
    int p = d->p, nq = p + 1;
    int Ny = d->nel_y + p, Nx = d->nel_x + p;
    dir1d X, Y;
    if (dir_init(&X, d->nel_x, p, d->len_x)) return 1;
    if (dir_init(&Y, d->nel_y, p, d->len_y)) { dir_free(&X); return 1; }
    const oracle_coeffs *c = &d->c;
    memset(rhs_T, 0, sizeof(double) * (size_t)Nx * Ny);
    if (rhs_fuel) memset(rhs_fuel, 0, sizeof(double) * (size_t)Nx * Ny);

    /* Elements in x-rows ex = colour (mod p+1) touch disjoint dof rows, so
     * each colour can run its rows in parallel with a fixed summation order. */
    for (int colour = 0; colour <= p; ++colour) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int ex = colour; ex < d->nel_x; ex += p + 1) {
            for (int ey = 0; ey < d->nel_y; ++ey) {
                for (int qx = 0; qx < nq; ++qx) {
                    size_t eqx = (size_t)ex * nq + qx;
                    const double *vx = X.bv + eqx * (p + 1), *dx = X.bd + eqx * (p + 1);
                    for (int qy = 0; qy < nq; ++qy) {
                        size_t eqy = (size_t)ey * nq + qy;
                        const double *vy = Y.bv + eqy * (p + 1), *dy = Y.bd + eqy * (p + 1);
                        double w = X.wq[eqx] * Y.wq[eqy];
                        double S = 0, Sx = 0, Sy = 0, Fu = 0;
                        for (int a = 0; a <= p; ++a)
                            for (int b = 0; b <= p; ++b) {
                                size_t k = (size_t)(ex + a) * Ny + (ey + b);
                                S += T[k] * vx[a] * vy[b];
                                Sx += T[k] * dx[a] * vy[b];
                                Sy += T[k] * vx[a] * dy[b];
                                Fu += fuel[k] * vx[a] * vy[b];
                            }
                        double bxv, byv;
                        wind_at(d, X.xq[eqx], Y.xq[eqy], &bxv, &byv);
                        int ign = (S > c->t_ig) && (Fu > c->fuel_thr);
                        if (amb && ((fabs(S - c->t_ig) <= amb->dT && Fu > c->fuel_thr - amb->dF) ||
                                    (fabs(Fu - c->fuel_thr) <= amb->dF && S > c->t_ig - amb->dT)))
                            amb->flags[(size_t)ex * d->nel_y + ey] = 1;
                        double arr = ign ? S * exp(-c->t_act / S) : 0.0;
                        double S2 = S * S;
                        double f = -c->c_adv * ((bxv - d->bbar_x) * Sx + (byv - d->bbar_y) * Sy)
                                   + c->c_forcing - c->c_rad * S2 * S2 + c->c_ign * arr;
                        if (src) f += src[eqx * ((size_t)d->nel_y * nq) + eqy];
                        double g = c->c_nld * S2 * S;
                        for (int a = 0; a <= p; ++a)
                            for (int b = 0; b <= p; ++b) {
                                double v = vx[a] * vy[b];
                                double v_x = dx[a] * vy[b];
                                double v_y = vx[a] * dy[b];
                                double val = S * v
                                    - ax * (c->c_diff * Sx * v_x + c->c_adv * d->bbar_x * Sx * v
                                            - c->c_react * S * v)
                                    - ay * (c->c_diff * Sy * v_y + c->c_adv * d->bbar_y * Sy * v)
                                    + beta * (f * v - g * (Sx * v_x + Sy * v_y));
                                size_t k = (size_t)(ex + a) * Ny + (ey + b);
                                rhs_T[k] += w * val;
                                if (rhs_fuel)
                                    rhs_fuel[k] += w * (Fu * v - d->dt * c->fuel_rate * arr * Fu * v);
                            }
                    }
                }
            }
        }
    }
    dir_free(&X);
    dir_free(&Y);
    return 0;
}

/* Substep parameters: the weights ax, ay of the explicit linear parts of L1
 * and L2, and beta of F. */
static int substep_params(const oracle_desc *d, int substep, double *ax, double *ay,
                          double *beta)
{
    if (d->scheme == ORACLE_PR) {
        if (substep < 0 || substep > 1) return 1;
        /* substep 0: x implicit, L2 explicit; substep 1: y implicit, L1 explicit */
        *ax = substep == 0 ? 0.0 : 0.5 * d->dt;
        *ay = substep == 0 ? 0.5 * d->dt : 0.0;
        *beta = 0.5 * d->dt;
        return 0;
    }
    if (d->scheme == ORACLE_EXPLICIT) {
        /* eq. (linear), every term at T^n with weight tau */
        if (substep != 0) return 1;
        *ax = *ay = *beta = d->dt;
        return 0;
    }
    if (substep != 0 && substep != 2) return 1;
    /* Strang S1 / S3: Crank-Nicolson on P1 over tau/2 */
    *ax = 0.25 * d->dt;
    *ay = 0.0;
    *beta = 0.5 * d->dt;
    return 0;
}

static int valid_desc(const oracle_desc *d)
{
    return d && d->p >= 1 && d->p <= 3 && d->nel_x >= 1 && d->nel_y >= 1 &&
           d->len_x > 0 && d->len_y > 0 && d->dt > 0 &&
           (d->scheme == ORACLE_PR || d->scheme == ORACLE_STRANG ||
            d->scheme == ORACLE_EXPLICIT);
}

int oracle_assemble(const oracle_desc *d, int substep, const double *T,
                    const double *fuel, double *rhs_T, double *rhs_fuel)
{
    if (!valid_desc(d) || !T || !fuel || !rhs_T) return 1;
    if (d->scheme == ORACLE_STRANG && substep == 1) {
        /* eq. (matrixCN), middle line: R = (Mx (x) By) T* */
        int Nx = d->nel_x + d->p, Ny = d->nel_y + d->p, W = 2 * d->p + 1;
        double *band = malloc(sizeof(double) * (size_t)(Nx > Ny ? Nx : Ny) * W);
        if (!band) return 2;
        memcpy(rhs_T, T, sizeof(double) * (size_t)Nx * Ny);
        int rc = oracle_operator(d, 1, 2, band);
        if (!rc) band_apply_lines(d, 1, band, rhs_T);
        if (!rc) rc = oracle_operator(d, 0, 1, band);
        if (!rc) band_apply_lines(d, 0, band, rhs_T);
        free(band);
        return rc;
    }
    double ax, ay, beta;
    if (substep_params(d, substep, &ax, &ay, &beta)) return 1;
    return assemble_quadrature(d, ax, ay, beta, T, fuel, NULL, rhs_T, rhs_fuel, NULL);
}

static int assemble_checked(const oracle_desc *d, int substep, const double *T,
                            const double *fuel, const double *src, double *rhs_T,
                            double *rhs_fuel, const ambiguity *amb)
{
    if ((!amb && !src) || (d->scheme == ORACLE_STRANG && substep == 1))
        return oracle_assemble(d, substep, T, fuel, rhs_T, rhs_fuel);
    double ax, ay, beta;
    if (substep_params(d, substep, &ax, &ay, &beta)) return 1;
    return assemble_quadrature(d, ax, ay, beta, T, fuel, src, rhs_T, rhs_fuel, amb);
}

/* (A (x) B) X = R: solve A along the x-lines, then B along the y-lines. */
static int kron_solve(const oracle_desc *d, int which_x, int which_y, double *X)
{
    int rc = oracle_line_solve(d, 0, which_x, X);
    if (!rc) rc = oracle_line_solve(d, 1, which_y, X);
    return rc;
}

/* src0 / src1: sources of the first / second quadrature substep (or NULL) */
static int step_impl(const oracle_desc *d, double *T, double *fuel, const ambiguity *amb,
                     const double *src0, const double *src1)
{
    if (!valid_desc(d) || !T || !fuel) return 1;
    size_t n = (size_t)(d->nel_x + d->p) * (d->nel_y + d->p);
    double *R = malloc(sizeof(double) * n);
    double *RF = malloc(sizeof(double) * n);
    if (!R || !RF) { free(R); free(RF); return 2; }
    int rc;
    if (d->scheme == ORACLE_PR) {
        /* eq. (matrixPR): [A^x (x) M^y] T^{n+1/2} = ..., [M^x (x) A^y] T^{n+1} = ... */
        rc = assemble_checked(d, 0, T, fuel, src0, R, RF, amb);
        if (!rc) rc = kron_solve(d, 0, 1, R);
        if (!rc) memcpy(T, R, sizeof(double) * n);
        if (!rc) rc = assemble_checked(d, 1, T, fuel, src1, R, NULL, amb);
        if (!rc) rc = kron_solve(d, 1, 0, R);
        if (!rc) memcpy(T, R, sizeof(double) * n);
    } else if (d->scheme == ORACLE_EXPLICIT) {
        /* (Mx (x) My) T^{n+1} = R(T^n, fuel^n) */
        rc = assemble_checked(d, 0, T, fuel, src0, R, RF, amb);
        if (!rc) rc = kron_solve(d, 1, 1, R);
        if (!rc) memcpy(T, R, sizeof(double) * n);
    } else {
        /* eq. (matrixCN): T^n -> T* -> T** -> T^{n+1} */
        rc = assemble_checked(d, 0, T, fuel, src0, R, RF, amb);
        if (!rc) rc = kron_solve(d, 0, 1, R);
        if (!rc) rc = oracle_assemble(d, 1, R, fuel, T, NULL);
        if (!rc) rc = kron_solve(d, 1, 0, T);
        if (!rc) rc = assemble_checked(d, 2, T, fuel, src1, R, NULL, amb);
        if (!rc) rc = kron_solve(d, 0, 1, R);
        if (!rc) memcpy(T, R, sizeof(double) * n);
    }
    /* fuel^{n+1} = (Mx (x) My)^{-1} R_fuel(T^n, fuel^n) */
    if (!rc) rc = kron_solve(d, 1, 1, RF);
    if (!rc) memcpy(fuel, RF, sizeof(double) * n);
    free(R);
    free(RF);
    return rc;
}

int oracle_step(const oracle_desc *d, double *T, double *fuel)
{
    return step_impl(d, T, fuel, NULL, NULL, NULL);
}

int oracle_step_forced(const oracle_desc *d, double *T, double *fuel, const double *src0,
                       const double *src1)
{
    if (!src0 || (d && d->scheme == ORACLE_EXPLICIT && src1) ||
        (d && d->scheme != ORACLE_EXPLICIT && !src1))
        return 1;
    return step_impl(d, T, fuel, NULL, src0, src1);
}

int oracle_quad_points(int n, int p, double L, double *xq)
{
    if (!xq || n < 1 || p < 1 || p > 3 || !(L > 0)) return 1;
    dir1d D;
    int rc = dir_init(&D, n, p, L);
    if (rc) return rc;
    memcpy(xq, D.xq, sizeof(double) * (size_t)n * (p + 1));
    dir_free(&D);
    return 0;
}

int oracle_step_flagged(const oracle_desc *d, double *T, double *fuel, double dT, double dF,
                        unsigned char *flags)
{
    if (!flags || !(dT >= 0) || !(dF >= 0)) return 1;
    ambiguity amb = {dT, dF, flags};
    return step_impl(d, T, fuel, &amb, NULL, NULL);
}

int oracle_run(const oracle_desc *d, double *T, double *fuel, int nsteps)
{
    for (int s = 0; s < nsteps; ++s) {
        int rc = oracle_step(d, T, fuel);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Evaluation helpers                                                         */
/* ------------------------------------------------------------------------ */
/* Values of the p+1 functions that are non-zero on the element containing x
 * (elements are the knot spans [t_{p+e}, t_{p+e+1}); x = L belongs to the
 * last one); returns that element's first function index e. */
static int span_values(const double *t, int n, int p, double x, double *v)
{
    int e = n - 1;
    for (int k = 0; k < n; ++k)
        if (x < t[p + k + 1]) { e = k; break; }
    for (int a = 0; a <= p; ++a) v[a] = cdb(t, e + a, p, x, n + p - 1);
    return e;
}

int oracle_eval_grid(const oracle_desc *d, const double *C, const double *xs,
                     int nx, const double *ys, int ny, double *out)
{
    if (!valid_desc(d)) return 1;
    int p = d->p, Ny = d->nel_y + p;
    double *tx = malloc(sizeof(double) * (size_t)(d->nel_x + 2 * p + 1));
    double *ty = malloc(sizeof(double) * (size_t)(d->nel_y + 2 * p + 1));
    int *fx = malloc(sizeof(int) * (size_t)nx), *fy = malloc(sizeof(int) * (size_t)ny);
    double *vx = malloc(sizeof(double) * (size_t)nx * (p + 1));
    double *vy = malloc(sizeof(double) * (size_t)ny * (p + 1));
    if (!tx || !ty || !fx || !fy || !vx || !vy) {
        free(tx); free(ty); free(fx); free(fy); free(vx); free(vy);
        return 2;
    }
    oracle_knots(d->nel_x, p, d->len_x, tx);
    oracle_knots(d->nel_y, p, d->len_y, ty);
    for (int a = 0; a < nx; ++a) fx[a] = span_values(tx, d->nel_x, p, xs[a], vx + (size_t)a * (p + 1));
    for (int b = 0; b < ny; ++b) fy[b] = span_values(ty, d->nel_y, p, ys[b], vy + (size_t)b * (p + 1));
#pragma omp parallel for schedule(static)
    for (int a = 0; a < nx; ++a)
        for (int b = 0; b < ny; ++b) {
            double s = 0.0;
            for (int i = 0; i <= p; ++i)
                for (int j = 0; j <= p; ++j)
                    s += C[(size_t)(fx[a] + i) * Ny + fy[b] + j] * vx[(size_t)a * (p + 1) + i]
                         * vy[(size_t)b * (p + 1) + j];
            out[(size_t)a * ny + b] = s;
        }
    free(tx); free(ty); free(fx); free(fy); free(vx); free(vy);
    return 0;
}

double oracle_burned_fraction(const oracle_desc *d, const double *fuel, double thr)
{
    if (!valid_desc(d)) return -1.0;
    int nx = d->nel_x, ny = d->nel_y;
    double *xs = malloc(sizeof(double) * (size_t)nx), *ys = malloc(sizeof(double) * (size_t)ny);
    double *v = malloc(sizeof(double) * (size_t)nx * ny);
    if (!xs || !ys || !v) { free(xs); free(ys); free(v); return -1.0; }
    for (int e = 0; e < nx; ++e) xs[e] = (e + 0.5) * d->len_x / nx;
    for (int e = 0; e < ny; ++e) ys[e] = (e + 0.5) * d->len_y / ny;
    double frac = -1.0;
    if (!oracle_eval_grid(d, fuel, xs, nx, ys, ny, v)) {
        size_t burned = 0;
        for (size_t k = 0; k < (size_t)nx * ny; ++k) burned += v[k] < thr;
        frac = (double)burned / ((double)nx * ny);
    }
    free(xs); free(ys); free(v);
    return frac;
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
