/*
 * oracle.h -- plain FP64 CPU oracle for the quasi-implicit alternating-direction
 * isogeometric (IGA-ADS) wildfire time stepper.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library against
 * the paper's method.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * Layout of every 2D field: dof (i, j) -- i the x index, j the y index -- at
 * offset i * Ny + j, with Nx = nel_x + p and Ny = nel_y + p.
 */
#ifndef WILDFIRE_ORACLE_H
#define WILDFIRE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Coefficients of the generic equation of Section 3 (the one with C_advection,
 * C_diffusion, C_reaction, the non-linear diffusion, ignition, forcing and
 * radiation terms), plus the Arrhenius activation temperature, the ignition
 * thresholds and the fuel-consumption rate of the compute_rhs listing. */
typedef struct {
    double c_adv, c_diff, c_react, c_nld, c_ign;
    double t_ig, fuel_thr, t_act;
    double c_forcing, c_rad, fuel_rate;
} oracle_coeffs;

enum { ORACLE_PR = 0, ORACLE_STRANG = 1, ORACLE_EXPLICIT = 2 };
enum { ORACLE_WIND_CONST = 0, ORACLE_WIND_SINCOS = 1 };

typedef struct {
    int nel_x, nel_y, p;
    double len_x, len_y;      /* physical edge lengths (m) */
    double dt;                /* tau */
    int scheme;               /* ORACLE_PR, ORACLE_STRANG or ORACLE_EXPLICIT */
    oracle_coeffs c;
    /* wind b(x,y): CONST  -> (bx, by)
     *              SINCOS -> (bx + ax sin(2 pi y/len_y), by + ay cos(2 pi x/len_x))
     * bbar = constant part treated implicitly inside the 1D operators. */
    int wind_kind;
    double bx, by, ax, ay, bbar_x, bbar_y;
} oracle_desc;

/* Parameter table of Section 2.2 divided through by rho*c_p. */
void oracle_default_coeffs(oracle_coeffs *c);

/* Uniform open knot vector, n + 2p + 1 entries. */
int oracle_knots(int n, int p, double L, double *t);
/* Gauss-Legendre rule on [-1, 1]; npts in 1..4. */
int oracle_gauss(int npts, double *x, double *w);
/* All N = n + p basis functions (deriv 0) or their first derivatives
 * (deriv 1) at nx points; out[k * N + i]. */
int oracle_basis_eval(int n, int p, double L, int deriv, const double *xs,
                      int nx, double *out);
/* 1D matrix in band storage band[i * (2p+1) + (k - i + p)], kind 0 = M,
 * 1 = K (stiffness), 2 = G (row = test function, column = differentiated
 * trial function). */
int oracle_mat1d(int n, int p, double L, int kind, double *band);
/* The banded 1D operator the scheme inverts along direction dir (0 = x,
 * 1 = y): which 0 = implicit operator A, 1 = mass matrix M, 2 = explicit
 * Crank-Nicolson operator B of the Strang middle substep (the explicit scheme:
 * A = B = M). */
int oracle_operator(const oracle_desc *d, int dir, int which, double *band);
/* Solve band * x = b for `nrhs` right-hand sides stored with stride `stride`
 * between successive rows and `dist` between right-hand sides (no pivoting). */
int oracle_band_solve(int N, int p, const double *band, double *x, int nrhs,
                      long stride, long dist);
/* Line solve on a 2D field: op^{-1} along direction dir on every line
 * (which as in oracle_operator; which 2 applies A^{-1} B). */
int oracle_line_solve(const oracle_desc *d, int dir, int which, double *X);
/* Quadrature right-hand side of one substep (PR: 0, 1; Strang: 0, 1, 2;
 * explicit: 0).
 * rhs_fuel (may be NULL) receives the fuel right-hand side of the step. */
int oracle_assemble(const oracle_desc *d, int substep, const double *T,
                    const double *fuel, double *rhs_T, double *rhs_fuel);
/* One full time step, in place. */
int oracle_step(const oracle_desc *d, double *T, double *fuel);
/* One step with a source s added to F (the forcing f of the manufactured-
 * solution study, Section 6.1), sampled at the quadrature points:
 * src[(ex*(p+1) + qx) * (nel_y*(p+1)) + ey*(p+1) + qy] at the points that
 * oracle_quad_points lists.  src0 feeds the first quadrature substep (PR 0,
 * Strang S1, explicit), src1 the second (PR 1, Strang S3; NULL for the
 * explicit scheme, required otherwise). */
int oracle_step_forced(const oracle_desc *d, double *T, double *fuel, const double *src0,
                       const double *src1);
/* Gauss points of the n elements of [0, L], element by element:
 * xq[e*(p+1) + q], ascending. */
int oracle_quad_points(int n, int p, double L, double *xq);
/* oracle_step, and flags[ex * nel_y + ey] = 1 for every element with a
 * quadrature point, in any substep, where the ignition decision is within dT
 * of T_ig (with fuel above thr - dF) or within dF of the fuel threshold (with
 * S above T_ig - dT).  flags is not cleared first. */
int oracle_step_flagged(const oracle_desc *d, double *T, double *fuel, double dT, double dF,
                        unsigned char *flags);
int oracle_run(const oracle_desc *d, double *T, double *fuel, int nsteps);
/* Evaluate the spline with coefficients C at the tensor grid xs x ys
 * (out[a * ny + b]). */
int oracle_eval_grid(const oracle_desc *d, const double *C, const double *xs,
                     int nx, const double *ys, int ny, double *out);
/* Share of elements whose fuel spline value at the element centre is < thr. */
double oracle_burned_fraction(const oracle_desc *d, const double *fuel,
                              double thr);
/* Number of OpenMP threads the oracle uses (0 = library default). */
void oracle_set_threads(int n);
int oracle_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
