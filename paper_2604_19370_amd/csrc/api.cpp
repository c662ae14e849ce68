// api.cpp -- the C ABI (include/iga.h): argument checking, the step
// sequences of the schemes, and the graph-replayed run loop.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "iga_internal.h"

namespace iga {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

iga_status fail(iga_status st, const std::string &msg)
{
    g_error = msg;
    return st;
}

iga_status hip_fail(hipError_t e, const char *what)
{
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? IGA_ENOMEM : IGA_EDEVICE;
}

void GraphEntry::reset()
{
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    T = fuel = nullptr;
    steps = 0;
}

static bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

iga_status check_desc(const iga_plan_desc *d)
{
    if (!d) return fail(IGA_EINVAL, "desc is NULL");
    if (d->p < 1 || d->p > 3) return fail(IGA_EINVAL, "p must be 1, 2 or 3");
    if (d->nel_x < 2 * d->p + 1 || d->nel_y < 2 * d->p + 1)
        return fail(IGA_EINVAL, "nel_x and nel_y must be >= 2p+1");
    if (d->nel_x > 65536 || d->nel_y > 65536) return fail(IGA_EINVAL, "nel above 65536");
    if (!(d->len_x > 0) || !(d->len_y > 0) || !std::isfinite(d->len_x) || !std::isfinite(d->len_y))
        return fail(IGA_EINVAL, "lengths must be finite and > 0");
    if (!(d->dt > 0) || !std::isfinite(d->dt)) return fail(IGA_EINVAL, "dt must be finite and > 0");
    if (d->scheme != IGA_PR && d->scheme != IGA_STRANG_CN && d->scheme != IGA_EXPLICIT)
        return fail(IGA_EINVAL, "unknown scheme");
    if (d->precision != IGA_FP64 && d->precision != IGA_FP32_REFINE)
        return fail(IGA_EINVAL, "unknown precision");
    if (d->wind.kind != IGA_WIND_CONST && d->wind.kind != IGA_WIND_SINCOS)
        return fail(IGA_EINVAL, "unknown wind kind");
    if (d->check_every < 0) return fail(IGA_EINVAL, "check_every must be >= 0");
    const double *c = &d->c.c_adv;
    for (int i = 0; i < 11; ++i)
        if (!std::isfinite(c[i])) return fail(IGA_EINVAL, "non-finite coefficient");
    if (!(d->c.t_act > 0)) return fail(IGA_EINVAL, "t_act must be > 0");
    return IGA_OK;
}

iga_status check_field(const void *p, const char *name)
{
    if (!p) return fail(IGA_EINVAL, std::string(name) + " is NULL");
    if (!aligned(p)) return fail(IGA_EINVAL, std::string(name) + " is not 16-byte aligned");
    return IGA_OK;
}

// One step in place; the right-hand sides live in the plan's scratch buffers.
// FP32 plans advance in increment form: the assembled right-hand sides are
// R - (implicit operator) S, the solves give the increment, and the y sweep
// adds the state it was taken from.  A PR or Strang step is six launches:
// assembly, x sweep, y sweep, twice; an explicit step is the first three.
// The x sweeps solve in place, or into second scratch fields under a
// column-wave x schedule (whose waves read rows around their own chunk).
// work: NULL for the plan's scratch fields, else four fields (R, R_fuel and,
// under column waves, their x-solved copies) that replace them.
void step_phases(const iga_plan *pl, void *T, void *fuel, StepPhases &sp, void *const *work)
{
    void *R = work ? work[0] : pl->scratch_r.ptr, *RF = work ? work[1] : pl->scratch_rf.ptr;
    const bool col = pl->sched[0].col != 0;
    void *XR = col ? (work ? work[2] : pl->scratch_r2.ptr) : R;
    void *XRF = col ? (work ? work[3] : pl->scratch_rf2.ptr) : RF;
    const void *bT = pl->delta ? T : nullptr, *bF = pl->delta ? fuel : nullptr;
    const int add = pl->delta ? 1 : 0;
    const bool pr = pl->d.scheme == IGA_PR;
    // substep 1 (PR: x implicit; Strang: S1) + the fuel right-hand side
    // FP32 plans: the fuel increment vanishes exactly outside the burning
    // region, and so do the windowed solves of it; those line blocks are skipped
    const int zs = pl->delta ? 1 : 0;
    sp.a1 = AsmArgs{0, T, fuel, R, RF};
    sp.x1 = {{R, XR, OP_AX, -1, -1, nullptr, 0}, {RF, XRF, OP_MX, -1, -1, nullptr, 0, zs}};
    sp.two = true;
    if (pl->d.scheme == IGA_EXPLICIT) {
        // (M^x (x) M^y) solves of both right-hand sides, in the same launches
        sp.x1[0].op0 = OP_MX;
        sp.y1 = {{XR, T, OP_MY, -1, -1, bT, 0}, {XRF, fuel, OP_MY, -1, -1, bF, 0, zs}};
        sp.two = false;
        sp.x2.clear();
        sp.y2.clear();
    } else if (pr) {
        sp.y1 = {{XR, T, OP_MY, -1, -1, bT, 0}};
        // substep 2: y implicit
        sp.a2 = AsmArgs{1, T, fuel, R, nullptr};
        sp.x2 = {{R, XR, OP_MX, -1, -1, nullptr, 0}};
        sp.y2 = {{XR, T, OP_AY, -1, -1, bT, 0}, {XRF, fuel, OP_MY, -1, -1, bF, 0, zs}};
    } else {
        // S1's y solve fused with S2: T** = (A^y)^{-1} B^y T* along y, with
        // T* = (M^y)^{-1} R (+ T^n in increment form)
        sp.y1 = {{XR, T, OP_MY, BAND_BY, OP_AY, bT, add}};
        // S3
        sp.a2 = AsmArgs{2, T, fuel, R, nullptr};
        sp.x2 = {{R, XR, OP_AX, -1, -1, nullptr, 0}};
        sp.y2 = {{XR, T, OP_MY, -1, -1, bT, 0}, {XRF, fuel, OP_MY, -1, -1, bF, 0, zs}};
    }
}

// src0 / src1: sources of the first / second quadrature substep (forced steps);
// work: replacement scratch fields (see step_phases), or NULL
iga_status step_impl(const iga_plan *pl, void *T, void *fuel, hipStream_t s, const void *src0,
                     const void *src1, void *const *work)
{
    StepPhases sp;
    step_phases(pl, T, fuel, sp, work);
    iga_status st;
    auto sweep = [&](int dir, const std::vector<SweepJob> &j) {
        return launch_sweep(pl, dir, j.data(), (int)j.size(), s);
    };
    if ((st = launch_assemble(pl, sp.a1.substep, sp.a1.T, sp.a1.fuel, sp.a1.R, sp.a1.RF, s, src0)))
        return st;
    if ((st = sweep(0, sp.x1)) || (st = sweep(1, sp.y1))) return st;
    if (!sp.two) return IGA_OK;
    if ((st = launch_assemble(pl, sp.a2.substep, sp.a2.T, sp.a2.fuel, sp.a2.R, sp.a2.RF, s, src1)))
        return st;
    if ((st = sweep(0, sp.x2)) || (st = sweep(1, sp.y2))) return st;
    return IGA_OK;
}

// Capture `steps` steps on a private stream into g (kernels only; no memset
// or host callbacks are recorded).
static iga_status capture(iga_plan *pl, GraphEntry &g, void *T, void *fuel, int64_t steps)
{
    if (g.exec && g.T == T && g.fuel == fuel && g.steps == steps) return IGA_OK;
    iga_status st = capture_graph(g, steps, [&](hipStream_t cs) { return step_impl(pl, T, fuel, cs); });
    if (st) return st;
    g.T = T;
    g.fuel = fuel;
    return IGA_OK;
}

}  // namespace iga

using namespace iga;

extern "C" {

const char *iga_last_error(void) { return g_error.c_str(); }

void iga_default_coeffs(iga_coeffs *out)
{
    if (!out) return;
    // Table of Section 2.2, every term divided by rho c_p
    const double cp = 1.0, rho = 1.293, kappa = 0.3, sigma = 5.67e-8, emis = 0.05;
    const double ch = 1.0, hc = -70.0, cw = 0.5, chi = 2e-2, t_amb = 300.0;
    const double dx = 3.5e-2 / emis, dz = 1.5 * emis;
    const double a_r = 1.5e-4, m_over_m1 = 1.0;  // not given in the paper
    const double rc = rho * cp;
    out->c_adv = cw;
    out->c_diff = kappa / rc;
    out->c_react = -chi / rc;
    out->c_nld = 4.0 * sigma * emis * dx / rc;
    out->c_rad = sigma * emis / dz / rc;
    out->c_forcing = (chi * t_amb + sigma * emis / dz * t_amb * t_amb * t_amb * t_amb) / rc;
    out->c_ign = 1e4 * ch * (-hc) * m_over_m1 * a_r / cp;
    out->t_ig = 800.0;
    out->fuel_thr = 0.2;
    out->t_act = 300.0;
    out->fuel_rate = 300.0 * a_r;
}

iga_status iga_plan_create(const iga_plan_desc *desc, iga_plan **out)
{
    if (!out) return fail(IGA_EINVAL, "out is NULL");
    *out = nullptr;
    iga_status st = check_desc(desc);
    if (st) return st;
    iga_plan *pl = new (std::nothrow) iga_plan();
    if (!pl) return fail(IGA_ENOMEM, "host allocation failed");
    try {
        pl->d = *desc;
        if ((st = build_plan_host(pl)) || (st = upload_plan(pl)) ||
            (st = choose_schedule(pl, 0, 0, 0)) || (st = choose_schedule(pl, 1, 0, 0))) {
            delete pl;
            return st;
        }
        pl->asm_rows = pl->Nx >= 2048 ? 32 : 16;
        pl->asm_stack = pl->fp32 && pl->P <= 2;
    } catch (const std::bad_alloc &) {
        delete pl;
        return fail(IGA_ENOMEM, "host allocation failed");
    }
    *out = pl;
    return IGA_OK;
}

iga_status iga_plan_destroy(iga_plan *plan)
{
    if (!plan) return IGA_OK;
    (void)hipDeviceSynchronize();
    plan->graph.reset();
    delete plan;
    return IGA_OK;
}

iga_status iga_plan_dims(const iga_plan *plan, int64_t *nx, int64_t *ny, int64_t *ndof)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (nx) *nx = plan->Nx;
    if (ny) *ny = plan->Ny;
    if (ndof) *ndof = (int64_t)plan->ndof;
    return IGA_OK;
}

iga_status iga_factor_1d(iga_plan *plan, void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st = launch_factor(plan, static_cast<hipStream_t>(stream));
    if (st) return st;
    // the tables are known now: windowed solves where the operators decay
    // fast enough, else an exact schedule that fits LDS
    for (int dir = 0; dir < 2; ++dir) {
        if (choose_window_schedule(plan, dir, 0, 0) == IGA_OK) continue;
        (void)hipGetLastError();   // the fallback below is deliberate
        if ((st = choose_schedule(plan, dir, 0, 0))) return st;
    }
    set_error("");
    plan->factored = true;
    plan->graph.reset();
    return IGA_OK;
}

iga_status iga_assemble_rhs(const iga_plan *plan, int32_t substep, const void *T, const void *fuel,
                            void *rhs_T, void *rhs_fuel, void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st;
    if ((st = check_field(T, "T")) || (st = check_field(fuel, "fuel")) ||
        (st = check_field(rhs_T, "rhs_T")))
        return st;
    if (rhs_fuel && !aligned(rhs_fuel)) return fail(IGA_EINVAL, "rhs_fuel is not 16-byte aligned");
    if (rhs_T == T || rhs_T == fuel || (rhs_fuel && (rhs_fuel == T || rhs_fuel == fuel)))
        return fail(IGA_EINVAL, "right-hand sides must not alias the state");
    if (plan->d.scheme == IGA_PR) {
        if (substep != 0 && substep != 1) return fail(IGA_EINVAL, "PR substep must be 0 or 1");
    } else if (plan->d.scheme == IGA_EXPLICIT) {
        if (substep != 0) return fail(IGA_EINVAL, "explicit substep must be 0");
    } else if (substep != 0 && substep != 2) {
        return fail(IGA_EINVAL,
                    "Strang substep must be 0 or 2 (the middle substep is iga_line_solve(1, 2))");
    }
    return launch_assemble(plan, substep, T, fuel, rhs_T, rhs_fuel, static_cast<hipStream_t>(stream));
}

iga_status iga_line_solve(const iga_plan *plan, int32_t dir, int32_t which, void *x, void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    if (which < 0 || which > 2) return fail(IGA_EINVAL, "which must be 0, 1 or 2");
    iga_status st = check_field(x, "x");
    if (st) return st;
    if (!plan->factored) return fail(IGA_ESTATE, "iga_factor_1d has not been called");
    const int A = dir ? OP_AY : OP_AX, M = dir ? OP_MY : OP_MX;
    const int B = dir ? BAND_BY : BAND_BX;
    hipStream_t s = static_cast<hipStream_t>(stream);
    SweepJob j{x, x, A, -1, -1, nullptr, 0};
    if (which == 1) j.op0 = M;
    if (plan->sched[dir].col) {
        // column waves solve out of place: through the plan's scratch field
        if (which == 2)
            return fail(IGA_EUNSUPPORTED, "x <- A^{-1} B x needs a windowed or exact x schedule");
        j.dst = plan->scratch_r2.ptr;
        if ((st = launch_sweep(plan, dir, &j, 1, s))) return st;
        IGA_HIP(hipMemcpyAsync(x, plan->scratch_r2.ptr, plan->ndof * plan->wsize,
                               hipMemcpyDeviceToDevice, s));
        return IGA_OK;
    }
    if (which == 2) j = SweepJob{x, x, -1, B, A, nullptr, plan->delta ? 1 : 0};
    return launch_sweep(plan, dir, &j, 1, s);
}

iga_status iga_step(iga_plan *plan, void *T, void *fuel, void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st;
    if ((st = check_field(T, "T")) || (st = check_field(fuel, "fuel"))) return st;
    if (T == fuel) return fail(IGA_EINVAL, "T and fuel must be different buffers");
    if (!plan->factored) return fail(IGA_ESTATE, "iga_factor_1d has not been called");
    return step_impl(plan, T, fuel, static_cast<hipStream_t>(stream));
}

iga_status iga_step_forced(iga_plan *plan, void *T, void *fuel, const void *src0, const void *src1,
                           void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st;
    if ((st = check_field(T, "T")) || (st = check_field(fuel, "fuel")) ||
        (st = check_field(src0, "src0")))
        return st;
    if (plan->d.scheme == IGA_EXPLICIT) {
        if (src1) return fail(IGA_EINVAL, "explicit plans take one source (src1 must be NULL)");
    } else if ((st = check_field(src1, "src1"))) {
        return st;
    }
    if (T == fuel) return fail(IGA_EINVAL, "T and fuel must be different buffers");
    if (src0 == T || src0 == fuel || (src1 && (src1 == T || src1 == fuel)))
        return fail(IGA_EINVAL, "sources must not alias the state");
    if (!plan->factored) return fail(IGA_ESTATE, "iga_factor_1d has not been called");
    return step_impl(plan, T, fuel, static_cast<hipStream_t>(stream), src0, src1);
}

iga_status iga_plan_quadrature_points(const iga_plan *plan, int32_t dir, double *x)
{
    if (!plan || !x) return fail(IGA_EINVAL, "NULL argument");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    const std::vector<double> &q = dir ? plan->Y.xq : plan->X.xq;
    std::memcpy(x, q.data(), q.size() * sizeof(double));
    return IGA_OK;
}

iga_status iga_run(iga_plan *plan, void *T, void *fuel, int64_t nsteps, void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st;
    if ((st = check_field(T, "T")) || (st = check_field(fuel, "fuel"))) return st;
    if (T == fuel) return fail(IGA_EINVAL, "T and fuel must be different buffers");
    if (nsteps < 0) return fail(IGA_EINVAL, "nsteps must be >= 0");
    if (!plan->factored) return fail(IGA_ESTATE, "iga_factor_1d has not been called");
    if (nsteps == 0) return IGA_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // graph of `chunk` steps replayed; a tail graph for the remainder
    const int64_t chunk = plan->d.check_every > 0 ? std::min<int64_t>(plan->d.check_every, nsteps)
                                                  : std::min<int64_t>(nsteps, 256);
    const int64_t tail = nsteps % chunk;
    if ((st = capture(plan, plan->graph.main, T, fuel, chunk))) return st;
    if (tail && (st = capture(plan, plan->graph.tail, T, fuel, tail))) return st;
    int *flag = plan->flag.as<int>();
    int64_t done = 0;
    while (done < nsteps) {
        const int64_t k = std::min<int64_t>(chunk, nsteps - done);
        IGA_HIP(hipGraphLaunch(k == chunk ? plan->graph.main.exec : plan->graph.tail.exec, s));
        done += k;
        if (plan->d.check_every > 0) {
            IGA_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
            if ((st = launch_nonfinite(plan, T, fuel, flag, s))) return st;
            int h = 0;
            IGA_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
            IGA_HIP(hipStreamSynchronize(s));
            if (h) return fail(IGA_ENONFINITE, "non-finite value after step " + std::to_string(done));
        }
    }
    return IGA_OK;
}

iga_status iga_plan_schedule(const iga_plan *plan, int32_t dir, int32_t *lines,
                             int32_t *waves_per_line, int32_t *rows_per_lane, int32_t *table_rows)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    const Schedule &sc = plan->sched[dir];
    if (lines) *lines = sc.lines;
    if (waves_per_line) *waves_per_line = sc.wpl;
    if (rows_per_lane) *rows_per_lane = sc.mm;
    if (table_rows) {
        int r = 0;
        for (int op = 0; op < NOPS; ++op)
            if (op_dir(op) == dir) r = std::max(r, plan->op_host[op].nrows);
        *table_rows = r;
    }
    return IGA_OK;
}

iga_status iga_plan_set_schedule(iga_plan *plan, int32_t dir, int32_t lines, int32_t waves_per_line)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    auto pow2 = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8 || v == 16; };
    if (!pow2(lines)) return fail(IGA_EINVAL, "lines must be 1, 2, 4, 8 or 16");
    if (waves_per_line != 0 && (!pow2(waves_per_line) || waves_per_line > 8))
        return fail(IGA_EINVAL, "waves_per_line must be 0 (automatic), 1, 2, 4 or 8");
    Schedule old = plan->sched[dir];
    iga_status st = choose_schedule(plan, dir, lines, waves_per_line);
    if (st) {
        if (plan->sched[dir].wpl != old.wpl || plan->sched[dir].mm != old.mm) {
            plan->sched[dir] = old;
            (void)build_scan_tables(plan, dir);
        }
        plan->sched[dir] = old;
        return st;
    }
    plan->graph.reset();
    return IGA_OK;
}

iga_status iga_plan_set_window_schedule(iga_plan *plan, int32_t dir, int32_t lines,
                                       int32_t rows_per_lane)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    if (lines != 1 && lines != 2 && lines != 4 && lines != 8 && lines != 16)
        return fail(IGA_EINVAL, "lines must be 1, 2, 4, 8 or 16");
    if (!plan->factored) return fail(IGA_ESTATE, "iga_factor_1d has not been called");
    iga_status st = choose_window_schedule(plan, dir, lines, rows_per_lane);
    if (st) return st;
    plan->graph.reset();
    return IGA_OK;
}

iga_status iga_plan_set_window_buffers(iga_plan *plan, int32_t dir, int32_t buffers)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    if (buffers < 0 || buffers > 2) return fail(IGA_EINVAL, "buffers must be 0, 1 or 2");
    plan->win_buffers[dir] = buffers;
    if (plan->sched[dir].win && !plan->sched[dir].col) {
        iga_status st = wsweep_prepare(plan, dir);
        if (st) return st;
    }
    plan->graph.reset();
    return IGA_OK;
}

int32_t iga_plan_window_buffers(const iga_plan *plan, int32_t dir)
{
    if (!plan || (dir != 0 && dir != 1)) return -1;
    const Schedule &sc = plan->sched[dir];
    if (!sc.win || sc.col) return 0;
    return sc.compact ? 1 : 2;
}

iga_status iga_plan_set_column_schedule(iga_plan *plan, int32_t rows_per_chunk)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (!plan->factored) return fail(IGA_ESTATE, "iga_factor_1d has not been called");
    iga_status st = choose_column_schedule(plan, rows_per_chunk);
    if (st) return st;
    plan->graph.reset();
    return IGA_OK;
}

iga_status iga_plan_solver(const iga_plan *plan, int32_t dir, int32_t *windowed, int32_t *warmup)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    if (windowed) *windowed = plan->sched[dir].col ? 2 : plan->sched[dir].win;
    if (warmup) *warmup = plan->factored ? warmup_rows(plan, dir) : 0;
    return IGA_OK;
}

iga_status iga_plan_set_assembly_rows(iga_plan *plan, int32_t rows)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (rows < plan->P + 1) return fail(IGA_EINVAL, "rows must be at least p + 1");
    plan->asm_rows = rows;
    plan->graph.reset();
    return IGA_OK;
}

int32_t iga_plan_assembly_rows(const iga_plan *plan) { return plan ? plan->asm_rows : 0; }

iga_status iga_plan_set_assembly_stacking(iga_plan *plan, int32_t stacked)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    if (stacked != 0 && stacked != 1) return fail(IGA_EINVAL, "stacked must be 0 or 1");
    plan->asm_stack = stacked;
    plan->graph.reset();
    return IGA_OK;
}

int32_t iga_plan_assembly_stacking(const iga_plan *plan) { return plan ? plan->asm_stack : 0; }

iga_status iga_autotune(iga_plan *plan, const void *T, const void *fuel, int32_t reps, void *stream)
{
    if (!plan) return fail(IGA_EINVAL, "plan is NULL");
    iga_status st;
    if ((st = check_field(T, "T")) || (st = check_field(fuel, "fuel"))) return st;
    if (reps < 1) return fail(IGA_EINVAL, "reps must be >= 1");
    if (!plan->factored) return fail(IGA_ESTATE, "iga_factor_1d has not been called");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *R = plan->scratch_r.ptr, *RF = plan->scratch_rf.ptr;
    DevBuf out;   // two output fields, so the two jobs of a launch never share one
    IGA_HIP(out.alloc(2 * plan->ndof * plan->wsize));
    void *out2 = out.as<char>() + plan->ndof * plan->wsize;
    // assembly: dof rows per wavefront tile, stacked or not
    std::vector<std::pair<float, std::pair<int, int>>> asm_timed;   // (ms, (rows, stacked))
    {
        int best = plan->asm_rows, best_stack = plan->asm_stack;
        float best_ms = 1e30f;
        for (int stack : {0, 1})
            for (int rows : ASSEMBLY_ROW_CANDIDATES) {
                if ((rows > plan->Nx && rows != 4) || rows < plan->P + 1) continue;
                plan->asm_rows = rows;
                plan->asm_stack = stack;
                float ms =
                    time_launches(s, reps, [&] { return launch_assemble(plan, 0, T, fuel, R, RF, s); });
                if (ms >= 0) asm_timed.emplace_back(ms, std::make_pair(rows, stack));
                if (ms >= 0 && ms < best_ms) {
                    best_ms = ms;
                    best = rows;
                    best_stack = stack;
                }
            }
        plan->asm_rows = best;
        plan->asm_stack = best_stack;
        if ((st = launch_assemble(plan, 0, T, fuel, R, RF, s))) return st;
    }
    // line solves: lines per workgroup, timed on the step's own jobs
    const void *bT = plan->delta ? T : nullptr;
    const int add = plan->delta ? 1 : 0;
    auto apply = [&](int dir, const Schedule &sc) {
        if (sc.col) return choose_column_schedule(plan, sc.mm);
        if (sc.win) return choose_window_schedule(plan, dir, sc.lines, sc.mm);
        return choose_schedule(plan, dir, sc.lines, sc.wpl);
    };
    std::vector<std::pair<float, Schedule>> timed[2];   // every candidate, launched alone
    for (int dir = 0; dir < 2; ++dir) {
        SweepJob jobs[2];
        int nj;
        if (dir == 0) {
            jobs[0] = SweepJob{R, out.ptr, OP_AX, -1, -1, nullptr, 0};
            jobs[1] = SweepJob{RF, out2, OP_MX, -1, -1, nullptr, 0};
            nj = 2;
        } else if (plan->d.scheme == IGA_STRANG_CN) {
            jobs[0] = SweepJob{R, out.ptr, OP_MY, BAND_BY, OP_AY, bT, add};
            nj = 1;
        } else {
            jobs[0] = SweepJob{R, out.ptr, OP_MY, -1, -1, bT, 0};
            nj = 1;
        }
        const Schedule keep = plan->sched[dir];
        Schedule best = keep;
        float best_ms = 1e30f;
        auto consider = [&] {
            float ms = time_launches(s, reps, [&] { return launch_sweep(plan, dir, jobs, nj, s); });
            if (ms >= 0) timed[dir].emplace_back(ms, plan->sched[dir]);
            if (ms >= 0 && ms < best_ms) {
                best_ms = ms;
                best = plan->sched[dir];
            }
        };
        // column waves (x-lines, FP32), then windowed solves (where the
        // operators decay fast enough)
        if (dir == 0)
            for (int mm : {16, 32})
                if (choose_column_schedule(plan, mm) == IGA_OK) consider();
        for (int mm : {9, 13, 17, 25, 33})
            for (int w : {1, 2, 4, 8, 16})
                if (choose_window_schedule(plan, dir, w, mm) == IGA_OK) consider();
        // exact chunk-scan solves
        int wmin = 1;
        while (wmin < 8 && choose_schedule(plan, dir, 1, wmin) != IGA_OK) wmin *= 2;
        for (int wpl : {wmin, 2 * wmin, 4 * wmin}) {
            if (wpl > 8) continue;
            for (int w : {1, 2, 4, 8, 16}) {
                if (w * wpl > 16) continue;
                if (choose_schedule(plan, dir, w, wpl) != IGA_OK) continue;
                consider();
            }
        }
        if ((st = apply(dir, best))) return st;
    }
    // Refinement: the fastest few assembly tilings, then the fastest few
    // line-solve candidates of each direction, again, timed
    // as graph-replayed steps (as iga_run executes them) on copies of T and
    // fuel.  Inside a step a sweep reads what the kernel before it has just
    // written from every XCD, which the launches above, repeated on the same
    // input, do not show.
    {
        const size_t fb = plan->ndof * plan->wsize;
        DevBuf state;
        IGA_HIP(state.alloc(2 * fb));
        void *sT = state.ptr, *sF = state.as<char>() + fb;
        auto step_ms = [&]() -> float {
            if (hipMemcpyAsync(sT, T, fb, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipMemcpyAsync(sF, fuel, fb, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return -1.f;
            GraphEntry g;
            float ms = -1.f;
            if (capture(plan, g, sT, sF, reps) == IGA_OK) {
                // the fastest of three replays: candidates here often differ
                // by a few per cent, about what one replay varies by
                auto replay = [&] { return hipGraphLaunch(g.exec, s) == hipSuccess ? IGA_OK : IGA_EDEVICE; };
                for (int i = 0; i < 3; ++i) {
                    const float t = time_launches(s, 1, replay);
                    if (t < 0) {
                        ms = -1.f;
                        break;
                    }
                    if (ms < 0 || t < ms) ms = t;
                }
            }
            (void)hipStreamSynchronize(s);
            g.reset();
            return ms < 0 ? ms : ms / reps;
        };
        constexpr size_t NREFINE = 8;
        std::stable_sort(asm_timed.begin(), asm_timed.end(),
                         [](const auto &a, const auto &b) { return a.first < b.first; });
        auto refine_assembly = [&] {
            if (asm_timed.size() < 2) return;
            int best = plan->asm_rows, best_stack = plan->asm_stack;
            float best_ms = 1e30f;
            for (size_t i = 0; i < std::min(asm_timed.size(), NREFINE); ++i) {
                plan->asm_rows = asm_timed[i].second.first;
                plan->asm_stack = asm_timed[i].second.second;
                const float ms = step_ms();
                if (ms >= 0 && ms < best_ms) {
                    best_ms = ms;
                    best = plan->asm_rows;
                    best_stack = plan->asm_stack;
                }
            }
            plan->asm_rows = best;
            plan->asm_stack = best_stack;
        };
        refine_assembly();
        for (int dir = 0; dir < 2; ++dir) {
            auto &c = timed[dir];
            std::stable_sort(c.begin(), c.end(),
                             [](const auto &a, const auto &b) { return a.first < b.first; });
            if (c.size() < 2) continue;
            Schedule best = plan->sched[dir];
            float best_ms = 1e30f;
            for (size_t i = 0; i < std::min(c.size(), NREFINE); ++i) {
                if (apply(dir, c[i].second) != IGA_OK) continue;
                const float ms = step_ms();
                if (ms >= 0 && ms < best_ms) {
                    best_ms = ms;
                    best = c[i].second;
                }
            }
            if ((st = apply(dir, best))) return st;
        }
        // the assembly again, now beside the line solves the step will run
        refine_assembly();
        IGA_HIP(hipStreamSynchronize(s));
    }
    IGA_HIP(hipStreamSynchronize(s));
    plan->graph.reset();
    set_error("");
    return IGA_OK;
}

}  // extern "C"
