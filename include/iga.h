/*
 * iga.h -- C ABI of the MI355X (gfx950) quasi-implicit alternating-direction
 * isogeometric wildfire stepper.
 *
 * Method (arXiv 2604.19370): the temperature T and the fuel fraction are
 * spline coefficient arrays on a tensor-product B-spline space of degree p
 * with uniform open knots (Section 3.1).  Each time step is a
 * Peaceman-Rachford step (Section 3.1, eq. PR / eq. matrixPR) or a Strang
 * splitting step with Crank-Nicolson substeps (Section 3.2, eq. CN /
 * eq. matrixCN).  Every substep with explicit terms assembles a right-hand
 * side by Gauss quadrature on the elements -- the non-linear diffusion
 * C_nld T^3 grad T, the ignition source C_ign [T > T_ig and fuel > thr]
 * T exp(-T_act / T), forcing and T^4 radiation, the explicit part of the
 * linear operator and the non-constant part of the wind (generic equation at
 * the start of Section 3) -- and then solves a Kronecker-product system
 * (A (x) B) X = R as independent banded 1D systems along x, then along y
 * (Section 4).  The fuel is consumed explicitly once per step and L2-projected
 * (the compute_rhs listing of Section 7).
 *
 * Conventions shared by every entry point
 *  - Field layout: dof (i, j), i the x index in [0, Nx), j the y index in
 *    [0, Ny), Nx = nel_x + p, Ny = nel_y + p, is element i * Ny + j of a dense
 *    row-major array (the ordering on which A^x (x) A^y acts with the x factor
 *    on the slow index).  Element type: double for IGA_FP64 plans, float for
 *    IGA_FP32_REFINE plans.  Every field pointer is a device pointer, 16-byte
 *    aligned, owned by the caller; the library never frees it and never keeps
 *    it past the call, except that iga_run keeps a captured HIP graph bound to
 *    the (T, fuel) pair it was last called with (re-captured when they change).
 *  - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *    Every call only enqueues work on that stream and returns; nothing
 *    synchronises unless stated.  A plan must not be used from two streams at
 *    once (it owns scratch buffers).
 *  - Errors: every function returns an iga_status.  IGA_EINVAL is returned
 *    synchronously for bad arguments before any work is enqueued; HIP runtime
 *    failures return IGA_EDEVICE.  iga_last_error() returns a description of
 *    the most recent failure on the calling thread.
 */
#ifndef IGA_H
#define IGA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IGA_OK = 0,
    IGA_EINVAL = 1,       /* invalid argument or descriptor                 */
    IGA_ENOMEM = 2,       /* device or host allocation failed               */
    IGA_EDEVICE = 3,      /* a HIP runtime call or kernel launch failed     */
    IGA_ENONFINITE = 4,   /* iga_run found a NaN/Inf in the state            */
    IGA_EUNSUPPORTED = 5, /* valid request the library does not implement    */
    IGA_ESTATE = 6        /* call out of order (e.g. step before factor)    */
} iga_status;

/* IGA_PR: Peaceman-Rachford alternating directions (Section 3.1).
 * IGA_STRANG_CN: Strang splitting with Crank-Nicolson substeps (Section 3.2).
 * IGA_EXPLICIT: the explicit L2-projection step the paper compares against
 * for eq. (linear) in Section 6.1 (the compute_rhs listing of Section 7 taken
 * as one step): every term at T^n with weight tau, then (M^x (x) M^y)^{-1}.
 * Only conditionally stable. */
typedef enum { IGA_PR = 0, IGA_STRANG_CN = 1, IGA_EXPLICIT = 2 } iga_scheme;

/* IGA_FP64: every kernel in double.
 * IGA_FP32_REFINE: state, right-hand sides and line solves in float with float
 * accumulation; the 1D LU factorisations are computed in double, and each 1D
 * solve is followed by one step of iterative refinement whose residual
 * b - A x0 is formed in double with the double operator. */
typedef enum { IGA_FP64 = 0, IGA_FP32_REFINE = 1 } iga_precision;

typedef enum { IGA_WIND_CONST = 0, IGA_WIND_SINCOS = 1 } iga_wind_kind;

/* Coefficients of the generic equation at the start of Section 3:
 *   dT/dt + c_adv b.grad T - c_diff lap T - c_react T - div(c_nld T^3 grad T)
 *     = c_ign [T > t_ig and fuel > fuel_thr] T exp(-t_act/T) + c_forcing - c_rad T^4
 * and the fuel consumption of the compute_rhs listing (Section 7):
 *   d fuel/dt = -fuel_rate [T > t_ig and fuel > fuel_thr] T exp(-t_act/T) fuel. */
typedef struct {
    double c_adv, c_diff, c_react, c_nld, c_ign;
    double t_ig, fuel_thr, t_act;
    double c_forcing, c_rad, fuel_rate;
} iga_coeffs;

/* Wind b(x, y):  CONST:  (bx, by)
 *                SINCOS: (bx + ax sin(2 pi y / len_y), by + ay cos(2 pi x / len_x)).
 * (bbar_x, bbar_y) is the constant part kept inside the implicit 1D operators
 * (the G matrices of eq. matrixPR / matrixCN); b - bbar is treated explicitly. */
typedef struct {
    int32_t kind;
    double bx, by, ax, ay;
    double bbar_x, bbar_y;
} iga_wind;

typedef struct {
    int32_t nel_x, nel_y;   /* elements per direction, >= 2p+1 and <= 65536     */
    int32_t p;              /* B-spline degree, 1, 2 or 3                         */
    double len_x, len_y;    /* physical edge lengths (m), > 0                     */
    double dt;              /* time step tau (s), > 0                             */
    int32_t scheme;         /* iga_scheme                                         */
    int32_t precision;      /* iga_precision                                      */
    iga_coeffs c;
    iga_wind wind;
    int32_t check_every;    /* iga_run: test the state for NaN/Inf every k steps  */
                            /* (0 = never; > 0 makes iga_run synchronise)         */
} iga_plan_desc;

typedef struct iga_plan iga_plan;   /* opaque; owned by the library */

/* Section 2.2 parameter table divided by rho c_p (c_p = 1, rho = 1.293, ...),
 * with the reaction-rate scale A_r = 1.5e-4 and M/M1 = 1 that the paper
 * leaves unspecified.  Never fails. */
void iga_default_coeffs(iga_coeffs *out);

/* Build a plan: knots, Gauss rules, basis tables at the quadrature points, the
 * 1D matrices M, K, G (Section 3.1) and the directional operators of the
 * scheme, uploaded to the current HIP device.  Allocates device memory (tables
 * and scratch of about 2 fields).  *out is NULL on failure.
 * Errors: IGA_EINVAL (NULL pointers, p not in {1,2,3}, nel < 2p+1, lengths or dt
 * not > 0, unknown enum), IGA_ENOMEM, IGA_EDEVICE. */
iga_status iga_plan_create(const iga_plan_desc *desc, iga_plan **out);

/* Release a plan and everything it owns (synchronises the device first).
 * NULL is accepted. */
iga_status iga_plan_destroy(iga_plan *plan);

/* Sizes: Nx, Ny (dofs per direction) and the number of dofs. */
iga_status iga_plan_dims(const iga_plan *plan, int64_t *nx, int64_t *ny, int64_t *ndof);

/* Factor every banded 1D operator of the plan (eq. matrixPR / matrixCN, the
 * banded structure of Section 4) with a banded LU without pivoting, in double,
 * on the device; also precomputes the chunk-transfer tables the line solves
 * use, and the float copies for IGA_FP32_REFINE plans.  Must be called once
 * before any solve; enqueued on `stream`. */
iga_status iga_factor_1d(iga_plan *plan, void *stream);

/* Quadrature right-hand side of one substep (weak forms eq. varPR_wildfire
 * and eq. varCN).  substep: PR 0 (x implicit) or 1 (y implicit); Strang 0 (S1)
 * or 2 (S3); explicit 0 (all terms, weight tau).  Reads T and fuel, writes
 * rhs_T; when rhs_fuel is not NULL also
 * writes the fuel right-hand side fuel v - tau fuel_rate [ign] T exp(-t_act/T)
 * fuel v.  All four are fields (layout above); rhs buffers must not alias the
 * inputs.  The Strang middle substep has no quadrature right-hand side (it is
 * iga_line_solve(dir = 1, which = 2)): substep 1 of a Strang plan is
 * IGA_EINVAL.
 * IGA_FP32_REFINE plans return the increment form R - (A^x (x) M^y) T
 * (PR substep 1: R - (M^x (x) A^y) T; explicit: R - (M^x (x) M^y) T; fuel:
 * R_fuel - (M^x (x) M^y) fuel), whose solve is the change of the state over
 * the substep. */
iga_status iga_assemble_rhs(const iga_plan *plan, int32_t substep, const void *T,
                            const void *fuel, void *rhs_T, void *rhs_fuel, void *stream);

/* In-place line solve on the field x along direction dir (0 = x: Ny lines of
 * length Nx; 1 = y: Nx lines of length Ny) -- one factor of the Kronecker
 * solve (A (x) B)^{-1} = (A^{-1} (x) I)(I (x) B^{-1}) of Section 4:
 *   which 0: x <- A^{-1} x  with A the scheme's implicit operator in dir
 *            (PR: (1 - tau/2 c_react) M + tau/2 (c_diff K + c_adv bbar G) along
 *            x, M + tau/2 (...) along y; Strang: tau/4 and reaction along x,
 *            tau/2 along y; explicit: A = M);
 *   which 1: x <- M^{-1} x;
 *   which 2: x <- A^{-1} B x with B the explicit Crank-Nicolson counterpart of
 *            A (signs of the tau terms flipped) -- the Strang middle substep
 *            (explicit plans: B = M, so this is the identity up to rounding).
 * Requires iga_factor_1d. */
iga_status iga_line_solve(const iga_plan *plan, int32_t dir, int32_t which, void *x,
                          void *stream);

/* One full time step, in place on (T, fuel): PR = assemble, A^x (x) M^y solve,
 * assemble, M^x (x) A^y solve; Strang-CN = S1 (assemble, A^x (x) M^y), S2
 * (A^{-1} B along y), S3 (assemble, A^x (x) M^y); explicit = assemble,
 * M^x (x) M^y solve; then the fuel update (Mx (x) My)^{-1} R_fuel(T^n, fuel^n).
 * Requires iga_factor_1d. */
iga_status iga_step(iga_plan *plan, void *T, void *fuel, void *stream);

/* One step with a source term s(x, y) added to F (the forcing f of the
 * manufactured-solution study of Section 6.1), sampled at the Gauss points
 * that iga_plan_quadrature_points lists: src[(ex*Q + qx) * (nel_y*Q) + ey*Q
 * + qy], Q = p + 1, point (x_{ex*Q+qx}, y_{ey*Q+qy}), in the plan's precision,
 * device memory, 16-byte aligned, not aliasing the state.  src0 feeds the
 * first quadrature substep (PR substep 0, Strang S1, explicit), src1 the
 * second (PR substep 1, Strang S3; must be NULL for explicit plans, non-NULL
 * otherwise); the caller samples each at the time it stands for (for
 * instance the start of the substep).  Errors as iga_step. */
iga_status iga_step_forced(iga_plan *plan, void *T, void *fuel, const void *src0, const void *src1,
                           void *stream);

/* The Gauss points of direction dir (0 = x, 1 = y): nel*(p+1) coordinates,
 * element by element, ascending, written to the host array x. */
iga_status iga_plan_quadrature_points(const iga_plan *plan, int32_t dir, double *x);

/* Spline values of a field (a coefficient array of the plan, in its
 * precision) at the nx * ny points (xs[a], ys[b]) of a tensor grid:
 *   out[a * ny + b] = sum_ij field[i * Ny + j] B_i(xs[a]) B_j(ys[b])
 * with the plan's tensor-product B-spline basis (Section 3.1), evaluated in
 * double.  Physical coordinates; points outside [0, len] are clamped to the
 * domain.  xs, ys and out are device arrays of double owned by the caller
 * (out must not alias the field).  For comparing fields at sample points
 * (e.g. 256^2 cell centres) independently of the mesh.  Errors: IGA_EINVAL
 * for NULL pointers or negative counts. */
iga_status iga_sample_points(const iga_plan *plan, const void *field, const double *xs, int32_t nx,
                             const double *ys, int32_t ny, double *out, void *stream);

/* Number of quadrature points (p + 1 Gauss points per direction and
 * element, as in the assembly) whose ignition decision [T > t_ig and
 * fuel > fuel_thr] (generic equation at the start of Section 3) lies near a
 * threshold: |T - t_ig| <= dT with fuel > fuel_thr - dF, or
 * |fuel - fuel_thr| <= dF with T > t_ig - dT, T and fuel evaluated in double
 * from the coefficients.  These are the points where evaluations in float
 * and in double may decide differently.  *count is a device int64 (8-byte
 * aligned) that the call overwrites.  Errors: IGA_EINVAL for NULL or
 * misaligned pointers or negative distances. */
iga_status iga_count_ambiguous(const iga_plan *plan, const void *T, const void *fuel, double dT,
                               double dF, int64_t *count, void *stream);

/* nsteps steps, in place, replayed from a HIP graph captured on first use for
 * this (T, fuel) pair.  With desc.check_every > 0 the state is tested for
 * NaN/Inf every check_every steps (this synchronises `stream`) and
 * IGA_ENONFINITE is returned at the first failure (state left as computed). */
iga_status iga_run(iga_plan *plan, void *T, void *fuel, int64_t nsteps, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step of
 * iga_step, with the right-hand-side scratch taken from a fixed device array
 * of IGA_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of the plan's own buffers.  Calls no
 * allocating routine.  The plan needs 2 fields (4 under column-wave x
 * sweeps) of ndof * element size bytes, each rounded up to 256 bytes; a plan
 * that needs more returns IGA_EINVAL (so at most about 8.3M dofs for FP32
 * plans, 4.1M for FP64).  The first call on a device looks the array's
 * address up once.  Every call on one GPU shares its array, which keeps the
 * last call's contents (nothing in it has to start at zero): calls that
 * overlap on one GPU -- two streams, or two host threads -- race, and the
 * caller must serialise them.  Results equal iga_step's bit for bit.
 * Requires iga_factor_1d; other errors as iga_step. */
#define IGA_NOALLOC_SCRATCH_BYTES (64u << 20)
iga_status iga_step_noalloc(iga_plan *plan, void *T, void *fuel, void *stream);

/* Line-solve schedule of direction dir: lines per workgroup, wavefronts per
 * line, rows per lane (each line is split into 64 * waves_per_line chunks of
 * that many rows) and the largest compressed coefficient table (rows kept per
 * operator after merging the identical interior rows).  Any output pointer
 * may be NULL. */
iga_status iga_plan_schedule(const iga_plan *plan, int32_t dir, int32_t *lines,
                             int32_t *waves_per_line, int32_t *rows_per_lane,
                             int32_t *table_rows);

/* Choose an exact (chunk-scan) line-solve schedule of direction dir: lines
 * in {1, 2, 4, 8, 16} lines per workgroup, waves_per_line in {1, 2, 4, 8} (0:
 * the fewest that fit the register budget), lines * waves_per_line <= 16.
 * IGA_EUNSUPPORTED if the schedule does not fit the register or LDS budget
 * for this line length; the previous schedule is kept. */
iga_status iga_plan_set_schedule(iga_plan *plan, int32_t dir, int32_t lines,
                                 int32_t waves_per_line);

/* Windowed line solves of direction dir (the default after iga_factor_1d
 * wherever the operators allow them).  Each lane restarts forward and backward
 * substitution from a zero state `warmup` rows outside its chunk of
 * rows_per_lane rows; the plan chooses warmup from the factors so that the
 * restart changes the result by less than 2^-55 relative to the state (FP64
 * plans) or, for FP32 plans, 2^-20 in the first solve and 2^-12 in the
 * correction solve of the FP64-residual refinement (which also corrects the
 * first solve's truncation), and refuses (IGA_EUNSUPPORTED) operators that
 * would need more than 96 rows.
 * rows_per_lane in {9, 13, 17, 25, 33} (0: 17); lines in {1, 2, 4, 8, 16}.
 * Must follow iga_factor_1d; on failure the previous schedule is kept. */
iga_status iga_plan_set_window_schedule(iga_plan *plan, int32_t dir, int32_t lines,
                                        int32_t rows_per_lane);

/* LDS form of the windowed solves of direction dir: buffers = 2 keeps two
 * line buffers per line (lanes publish into one while others still read the
 * other); 1 keeps one (a barrier before every overwrite), and a job with two
 * operators (Strang S1 with S2) stages the second operator's tables over the
 * first's once its solve is done; 0 (the default) picks 1 where that lets
 * more workgroups share a compute unit, else 2.  Both forms compute the same
 * values in the same order (bitwise equal results).  Applies to the current
 * and later windowed schedules of the direction; IGA_EINVAL for other
 * values.  iga_plan_window_buffers returns the form in use (1 or 2), 0 if
 * direction dir is not solved by windowed solves, -1 for a NULL plan or a
 * bad dir. */
iga_status iga_plan_set_window_buffers(iga_plan *plan, int32_t dir, int32_t buffers);
int32_t iga_plan_window_buffers(const iga_plan *plan, int32_t dir);

/* Column waves for the x-lines of an FP32 plan: one line per lane, 64
 * adjacent lines per wavefront, each wavefront a chunk of rows_per_chunk rows
 * (16 or 32; 0: 32) with its own warm-up rows on both sides, so every access
 * is a coalesced row and lanes never exchange data.  The x sweeps of a step
 * then write into a second pair of scratch fields.  Under this schedule
 * iga_line_solve(0, which) goes through a scratch field (which 0, 1) and
 * refuses which 2 (IGA_EUNSUPPORTED).  IGA_EUNSUPPORTED for FP64 plans or x
 * operators that decay too slowly for the kernel's compiled warm-ups.  Must
 * follow iga_factor_1d; on failure the previous schedule is kept. */
iga_status iga_plan_set_column_schedule(iga_plan *plan, int32_t rows_per_chunk);

/* Solver of direction dir: *windowed = 2 for column waves, 1 for windowed
 * solves, 0 for the exact chunk scan of iga_plan_set_schedule; *warmup = the
 * windowed warm-up rows (0 if windowed solves are not possible or before
 * factorisation).  Either pointer may be NULL. */
iga_status iga_plan_solver(const iga_plan *plan, int32_t dir, int32_t *windowed, int32_t *warmup);

/* Assembly schedule: dof rows per wavefront tile, at least p + 1
 * (IGA_EINVAL below).  A workgroup takes four consecutive tiles of a strip.
 * Stacked (1): only its first tile, p rows shorter than the others,
 * re-evaluates the p elements above it; the rows where two of its tiles meet
 * are summed in two parts through LDS (deterministic).  Unstacked (0): every
 * tile re-evaluates its own p halo elements, and the wavefronts never wait
 * for each other.  Defaults: 16 rows (32 from 2048 dof rows), stacked for
 * FP32 plans of degree <= 2; iga_autotune times both kinds.  stacked must be
 * 0 or 1 (IGA_EINVAL). */
iga_status iga_plan_set_assembly_rows(iga_plan *plan, int32_t rows);
int32_t iga_plan_assembly_rows(const iga_plan *plan);
iga_status iga_plan_set_assembly_stacking(iga_plan *plan, int32_t stacked);
int32_t iga_plan_assembly_stacking(const iga_plan *plan);

/* Autotuner: times, with HIP events on `stream`, the assembly of the first
 * substep for every tile height (stacked and unstacked) and the line solves
 * of each direction for every windowed and exact schedule that fits, on the
 * plan's scratch buffers (T and fuel are only read), and keeps the fastest
 * of each (column waves included for the x-lines of FP32 plans).  The eight
 * fastest assembly tilings, then the eight fastest line-solve schedules of
 * each direction, then the tilings once more beside the chosen line solves,
 * are timed again as a captured graph of reps steps (as
 * iga_run replays them; the fastest of three replays counts), on device
 * copies of T and fuel that the call allocates and frees, and the fastest
 * step wins.  Synchronises `stream`; must follow iga_factor_1d.  reps >= 1
 * launches (or steps) per candidate. */
iga_status iga_autotune(iga_plan *plan, const void *T, const void *fuel, int32_t reps,
                        void *stream);

/* ------------------------------------------------------------------------
 * Ensembles: independent scenarios (for instance perturbed fuel maps, winds
 * and ignitions of one region) stepped together on one GPU, each member the
 * method of Sections 3-4 on its own mesh.  Members may differ in grid size,
 * lengths, dt, scheme, wind, coefficients and fields, but share the degree p
 * and the precision.  Every phase of a step (the two assemblies, the four
 * line sweeps) runs as one launch over all members per line-solve schedule
 * group (members with equal rows per lane, lines per workgroup and wavefronts
 * per line), so the per-step launch count does not grow with the member
 * count.  Explicit-scheme members take part in the first assembly and the
 * first two sweeps only.  Each member's result is, up to rounding, the one its own plan
 * would compute with the same line-solve schedule (the batched kernels are
 * separately compiled and may contract multiply-adds differently).
 * ------------------------------------------------------------------------ */
typedef struct iga_ensemble iga_ensemble;

/* Create n >= 1 member plans from members[0..n) (each checked as by
 * iga_plan_create), factor them (as iga_factor_1d on the legacy default
 * stream; synchronises the device), and give every member the same
 * line-solve schedule per direction.  IGA_EINVAL if members differ in p or
 * precision.  The ensemble owns its plans; free with iga_ensemble_destroy. */
iga_status iga_ensemble_create(const iga_plan_desc *members, int32_t n, iga_ensemble **out);
iga_status iga_ensemble_destroy(iga_ensemble *ens);
iga_status iga_ensemble_size(const iga_ensemble *ens, int32_t *n);

/* Kernel launches per step: 1 assembly + 1 sweep per schedule group and
 * direction, and the same again over the members that have a second phase
 * (every scheme but the explicit one). */
iga_status iga_ensemble_launches(const iga_ensemble *ens, int32_t *per_step);

/* One step of every member, in place: T[m], fuel[m] are member m's fields
 * (layout and type as for a plan of members[m]).  The pointer arrays are read
 * during the call; the launches prepared for them are kept and reused while
 * the same pointers are passed (rebuilt otherwise, which copies a few KB of
 * parameters to the device and synchronises). */
iga_status iga_ensemble_step(iga_ensemble *ens, void *const *T, void *const *fuel, void *stream);

/* nsteps steps of every member, replayed from captured HIP graphs (re-captured
 * when the pointers or the schedules change). */
iga_status iga_ensemble_run(iga_ensemble *ens, void *const *T, void *const *fuel, int64_t nsteps,
                            void *stream);

/* Exact (chunk-scan) line-solve schedule of direction dir for every member:
 * `lines` per workgroup, at least waves_per_line wavefronts per line (more
 * for members whose lines need them).  On IGA_EUNSUPPORTED the previous
 * schedules are restored. */
iga_status iga_ensemble_set_schedule(iga_ensemble *ens, int32_t dir, int32_t lines,
                                     int32_t waves_per_line);
/* Windowed line solves (as iga_plan_set_window_schedule) on every member
 * that allows them, the exact schedule with the same lines elsewhere.
 * `lines` applies to the members whose lines need the most wavefronts; a
 * member needing 1/f of them takes f times the lines per workgroup where
 * that fits, so that its workgroups have the same size and it shares their
 * launch (members of one launch share rows per lane and workgroup size).
 * The default after iga_ensemble_create is (4, 17) along x and (2, 17) along
 * y. */
iga_status iga_ensemble_set_window_schedule(iga_ensemble *ens, int32_t dir, int32_t lines,
                                            int32_t rows_per_lane);
/* As iga_plan_set_assembly_rows, on every member (rows >= p + 1). */
iga_status iga_ensemble_set_assembly_rows(iga_ensemble *ens, int32_t rows);
/* As iga_plan_set_assembly_stacking, on every member. */
iga_status iga_ensemble_set_assembly_stacking(iga_ensemble *ens, int32_t stacked);

/* Autotuner of the batched launches: tile height and stacking of the
 * assembly, and the line-solve schedule of each direction (windowed rows per
 * lane or exact waves per line, lines per workgroup) timed on both of the
 * step's launches of that direction with the step's own jobs; all timed with
 * HIP events on `stream` on the members' scratch buffers (the fields are
 * only read).  Synchronises. */
iga_status iga_ensemble_autotune(iga_ensemble *ens, void *const *T, void *const *fuel, int32_t reps,
                                 void *stream);

/* Thread-local description of the last error ("" if none). */
const char *iga_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGA_H */
