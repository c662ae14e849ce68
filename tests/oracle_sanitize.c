/*
 * Driver for the sanitizer build of the oracle (test infrastructure): calls
 * every entry point of oracle.h on small, non-square meshes for p = 1, 2, 3
 * and each scheme, checks return codes and finiteness, and lets
 * AddressSanitizer and UndefinedBehaviorSanitizer catch out-of-bounds
 * accesses, leaks and undefined arithmetic.  Exit status 0 means clean.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static int fails = 0;

#define CHECK(cond, what)                                                        \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "FAIL p=%d scheme=%d: %s\n", p, scheme, what);       \
            ++fails;                                                             \
        }                                                                        \
    } while (0)

static int all_finite(const double *v, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static void fill_state(const oracle_desc *d, double *T, double *F)
{
    const int Nx = d->nel_x + d->p, Ny = d->nel_y + d->p;
    for (int i = 0; i < Nx; ++i)
        for (int j = 0; j < Ny; ++j) {
            const double x = (double)i / (Nx - 1) - 0.45, y = (double)j / (Ny - 1) - 0.55;
            T[i * Ny + j] = 300.0 + 900.0 * exp(-(x * x + y * y) / (2 * 0.04));
            F[i * Ny + j] = 0.5 + 0.5 * (double)((i * 7 + j * 3) % 11) / 10.0;
        }
}

static void run_case(int p, int scheme)
{
    oracle_desc d = {0};
    d.nel_x = 5 + p;
    d.nel_y = 4 + 2 * p;
    d.p = p;
    d.len_x = d.nel_x;
    d.len_y = d.nel_y;
    d.dt = 1e-3;
    d.scheme = scheme;
    oracle_default_coeffs(&d.c);
    d.wind_kind = ORACLE_WIND_SINCOS;
    d.bx = 1.0;
    d.by = 0.0;
    d.ax = 0.3;
    d.ay = 0.5;
    d.bbar_x = 1.0;
    d.bbar_y = 0.0;
    const int Nx = d.nel_x + p, Ny = d.nel_y + p, Q = p + 1, B = 2 * p + 1;
    const long nf = (long)Nx * Ny;

    double *T = malloc(sizeof(double) * nf), *F = malloc(sizeof(double) * nf);
    double *R = malloc(sizeof(double) * nf), *RF = malloc(sizeof(double) * nf);
    fill_state(&d, T, F);

    /* 1D building blocks */
    double *t = malloc(sizeof(double) * (d.nel_x + 2 * p + 1));
    CHECK(oracle_knots(d.nel_x, p, d.len_x, t) == 0, "knots");
    double gx[4], gw[4];
    CHECK(oracle_gauss(Q, gx, gw) == 0, "gauss");
    double xs[9];
    for (int k = 0; k < 9; ++k) xs[k] = d.len_x * k / 8.0;
    double *bv = malloc(sizeof(double) * 9 * Nx);
    for (int der = 0; der < 2; ++der) {
        CHECK(oracle_basis_eval(d.nel_x, p, d.len_x, der, xs, 9, bv) == 0, "basis_eval");
        CHECK(all_finite(bv, 9L * Nx), "basis_eval finite");
    }
    double *band = malloc(sizeof(double) * (long)(Nx > Ny ? Nx : Ny) * B);
    for (int kind = 0; kind < 3; ++kind) {
        CHECK(oracle_mat1d(d.nel_x, p, d.len_x, kind, band) == 0, "mat1d");
        CHECK(all_finite(band, (long)Nx * B), "mat1d finite");
    }
    for (int dir = 0; dir < 2; ++dir)
        for (int which = 0; which < 3; ++which) {
            const int N = dir ? Ny : Nx;
            CHECK(oracle_operator(&d, dir, which, band) == 0, "operator");
            CHECK(all_finite(band, (long)N * B), "operator finite");
        }
    CHECK(oracle_operator(&d, 0, 1, band) == 0, "mass operator");
    double *rhs = malloc(sizeof(double) * Nx * 3);
    for (int k = 0; k < Nx * 3; ++k) rhs[k] = 1.0 + 0.1 * k;
    CHECK(oracle_band_solve(Nx, p, band, rhs, 3, 1, Nx) == 0, "band_solve");
    CHECK(all_finite(rhs, Nx * 3L), "band_solve finite");
    double *xq = malloc(sizeof(double) * d.nel_x * Q);
    CHECK(oracle_quad_points(d.nel_x, p, d.len_x, xq) == 0, "quad_points");

    /* line solves and assembly of every substep */
    for (int dir = 0; dir < 2; ++dir)
        for (int which = 0; which < 3; ++which) {
            for (long k = 0; k < nf; ++k) R[k] = T[k];
            CHECK(oracle_line_solve(&d, dir, which, R) == 0, "line_solve");
            CHECK(all_finite(R, nf), "line_solve finite");
        }
    const int nsub = scheme == ORACLE_PR ? 2 : scheme == ORACLE_STRANG ? 3 : 1;
    for (int s = 0; s < nsub; ++s) {
        CHECK(oracle_assemble(&d, s, T, F, R, RF) == 0, "assemble");
        CHECK(all_finite(R, nf) && all_finite(RF, nf), "assemble finite");
        CHECK(oracle_assemble(&d, s, T, F, R, NULL) == 0, "assemble without fuel rhs");
    }

    /* steps: plain, run, flagged, forced */
    CHECK(oracle_step(&d, T, F) == 0, "step");
    CHECK(oracle_run(&d, T, F, 3) == 0, "run");
    unsigned char *flags = calloc((size_t)d.nel_x * d.nel_y, 1);
    CHECK(oracle_step_flagged(&d, T, F, 1e-6, 1e-9, flags) == 0, "step_flagged");
    const long nq = (long)d.nel_x * Q * d.nel_y * Q;
    double *src0 = malloc(sizeof(double) * nq), *src1 = malloc(sizeof(double) * nq);
    for (long k = 0; k < nq; ++k) {
        src0[k] = 0.01 * (double)(k % 13);
        src1[k] = 0.02 * (double)(k % 7);
    }
    CHECK(oracle_step_forced(&d, T, F, src0, scheme == ORACLE_EXPLICIT ? NULL : src1) == 0,
          "step_forced");
    CHECK(all_finite(T, nf) && all_finite(F, nf), "state finite");

    /* evaluation helpers */
    double ys[5], out[9 * 5];
    for (int k = 0; k < 5; ++k) ys[k] = d.len_y * k / 4.0;
    CHECK(oracle_eval_grid(&d, T, xs, 9, ys, 5, out) == 0, "eval_grid");
    CHECK(all_finite(out, 45), "eval_grid finite");
    const double bf = oracle_burned_fraction(&d, F, 0.1);
    CHECK(bf >= 0.0 && bf <= 1.0, "burned_fraction");

    free(T); free(F); free(R); free(RF); free(t); free(bv); free(band); free(rhs); free(xq);
    free(flags); free(src0); free(src1);
}

int main(void)
{
    oracle_set_threads(2);
    for (int p = 1; p <= 3; ++p)
        for (int scheme = 0; scheme < 3; ++scheme) run_case(p, scheme);
    if (fails) fprintf(stderr, "%d checks failed\n", fails);
    else printf("oracle sanitizer run: clean\n");
    return fails ? 1 : 0;
}
