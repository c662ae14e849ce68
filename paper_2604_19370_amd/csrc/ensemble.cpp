// ensemble.cpp -- ensembles of independent scenarios (uneven grids, winds,
// fuel maps, ignitions, schemes) stepped together.  Every phase of a step (the
// two assemblies and four sweeps) is one batched launch over all members per
// line-solve schedule group, so small members share the GPU instead of each
// launching grids too small to fill it; run() replays the step loop from a
// HIP graph.  Members of the explicit scheme take part in the first three
// phases only.  Members are independent: no data moves between them.
#include <algorithm>

#include "iga_internal.h"

using namespace iga;

struct iga_ensemble {
    std::vector<iga_plan *> plans;
    int P = 2;
    bool fp32 = false;
    // launches prepared for the bound fields
    std::vector<void *> T, F;
    bool bound = false;
    BatchLaunch a1, a2;
    std::vector<BatchLaunch> x1, y1, x2, y2;
    bool two = false;   // some member has a second assembly and sweep pair
    GraphCache graph;

    ~iga_ensemble()
    {
        graph.reset();
        for (iga_plan *p : plans) iga_plan_destroy(p);
    }
    void unbind()
    {
        bound = false;
        graph.reset();
    }
};

namespace {

iga_status check_fields(const iga_ensemble *e, void *const *T, void *const *F)
{
    if (!T || !F) return fail(IGA_EINVAL, "field arrays are NULL");
    iga_status st;
    for (size_t m = 0; m < e->plans.size(); ++m) {
        if ((st = check_field(T[m], "T[m]")) || (st = check_field(F[m], "fuel[m]"))) return st;
        if (T[m] == F[m]) return fail(IGA_EINVAL, "T[m] and fuel[m] must be different buffers");
    }
    return IGA_OK;
}

// (Re)build the batched launches when the field pointers change.
iga_status bind(iga_ensemble *e, void *const *T, void *const *F)
{
    const size_t n = e->plans.size();
    if (e->bound && std::equal(T, T + n, e->T.begin()) && std::equal(F, F + n, e->F.begin()))
        return IGA_OK;
    e->unbind();
    std::vector<AsmArgs> a1(n), a2;
    std::vector<std::vector<SweepJob>> x1(n), y1(n), x2, y2;
    std::vector<iga_plan *> second;   // members with a second phase
    for (size_t m = 0; m < n; ++m) {
        StepPhases sp;
        step_phases(e->plans[m], T[m], F[m], sp);
        a1[m] = sp.a1;
        x1[m] = sp.x1;
        y1[m] = sp.y1;
        if (sp.two) {
            second.push_back(e->plans[m]);
            a2.push_back(sp.a2);
            x2.push_back(sp.x2);
            y2.push_back(sp.y2);
        }
    }
    iga_status st;
    if ((st = build_assemble_batch(e->plans, a1, e->a1)) ||
        (st = build_sweep_batch(e->plans, 0, x1, e->x1)) || (st = build_sweep_batch(e->plans, 1, y1, e->y1)))
        return st;
    e->two = !second.empty();
    if (e->two &&
        ((st = build_assemble_batch(second, a2, e->a2)) || (st = build_sweep_batch(second, 0, x2, e->x2)) ||
         (st = build_sweep_batch(second, 1, y2, e->y2))))
        return st;
    e->T.assign(T, T + n);
    e->F.assign(F, F + n);
    e->bound = true;
    return IGA_OK;
}

iga_status launch_all(const std::vector<BatchLaunch> &v, hipStream_t s)
{
    for (const BatchLaunch &b : v) {
        iga_status st = launch_batch(b, s);
        if (st) return st;
    }
    return IGA_OK;
}

iga_status step_bound(iga_ensemble *e, hipStream_t s)
{
    iga_status st;
    if ((st = launch_batch(e->a1, s)) || (st = launch_all(e->x1, s)) || (st = launch_all(e->y1, s)))
        return st;
    if (e->two &&
        ((st = launch_batch(e->a2, s)) || (st = launch_all(e->x2, s)) || (st = launch_all(e->y2, s))))
        return st;
    return IGA_OK;
}

iga_status capture(iga_ensemble *e, GraphEntry &g, int64_t steps)
{
    if (g.exec && g.steps == steps) return IGA_OK;
    return capture_graph(g, steps, [&](hipStream_t cs) { return step_bound(e, cs); });
}

// schedule of one direction on every member: `lines` lines per workgroup and
// at least `wpl` wavefronts per line (more where a member's lines need them)
iga_status set_schedule_all(iga_ensemble *e, int dir, int lines, int wpl)
{
    for (iga_plan *pl : e->plans) {
        iga_status st = IGA_EUNSUPPORTED;
        for (int w = std::max(wpl, 1); w <= 8 && st; w *= 2) st = choose_schedule(pl, dir, lines, w);
        if (st) return st;
    }
    e->unbind();
    return IGA_OK;
}

// windowed schedule of one direction on every member (`lines` lines per
// workgroup for the members with the longest lines, mm rows per lane);
// members whose operators do not allow it get the exact schedule with the
// same lines and the fewest waves per line.  A member whose lines need 1/f of
// the wavefronts takes f times the lines per workgroup where that fits, so
// that its workgroups have the same shape and it shares their launch.
iga_status set_window_all(iga_ensemble *e, int dir, int lines, int mm)
{
    auto waves = [&](const iga_plan *pl) {
        const int N = dir ? pl->Ny : pl->Nx;
        return (N + 64 * mm - 1) / (64 * mm);
    };
    int wmax = 1;
    for (const iga_plan *pl : e->plans) wmax = std::max(wmax, waves(pl));
    for (iga_plan *pl : e->plans) {
        const int w = waves(pl), f = wmax / w;
        if (wmax % w == 0 && f > 1 && (f & (f - 1)) == 0 && lines * f <= 16 &&
            choose_window_schedule(pl, dir, lines * f, mm) == IGA_OK)
            continue;
        (void)hipGetLastError();
        if (choose_window_schedule(pl, dir, lines, mm) == IGA_OK) continue;
        (void)hipGetLastError();   // the fallback below is deliberate
        iga_status st = IGA_EUNSUPPORTED;
        for (int ww = 1; ww <= 8 && st; ww *= 2) st = choose_schedule(pl, dir, lines, ww);
        if (st) return st;
    }
    set_error("");
    e->unbind();
    return IGA_OK;
}

// schedule groups of direction dir among all members (second = false) or
// among the members with a second assembly and sweep pair (second = true)
int groups(const iga_ensemble *e, int dir, bool second = false)
{
    std::vector<Schedule> seen;
    for (const iga_plan *pl : e->plans) {
        if (second && pl->d.scheme == IGA_EXPLICIT) continue;
        const Schedule &s = pl->sched[dir];
        bool found = false;
        for (const Schedule &t : seen)
            found = found || (t.mm == s.mm && t.lines * t.wpl == s.lines * s.wpl && t.win == s.win);
        if (!found) seen.push_back(s);
    }
    return (int)seen.size();
}

}  // namespace

extern "C" {

iga_status iga_ensemble_create(const iga_plan_desc *members, int32_t n, iga_ensemble **out)
{
    if (!out) return fail(IGA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!members) return fail(IGA_EINVAL, "members is NULL");
    if (n < 1 || n > 4096) return fail(IGA_EINVAL, "member count must be in [1, 4096]");
    iga_status st;
    for (int m = 0; m < n; ++m) {
        if ((st = check_desc(&members[m]))) return st;
        if (members[m].p != members[0].p || members[m].precision != members[0].precision)
            return fail(IGA_EINVAL, "members must share degree and precision");
    }
    iga_ensemble *e = new (std::nothrow) iga_ensemble;
    if (!e) return fail(IGA_ENOMEM, "ensemble allocation");
    e->P = members[0].p;
    e->fp32 = members[0].precision == IGA_FP32_REFINE;
    for (int m = 0; m < n; ++m) {
        iga_plan *pl = nullptr;
        if ((st = iga_plan_create(&members[m], &pl)) || (st = iga_factor_1d(pl, nullptr))) {
            if (pl) iga_plan_destroy(pl);
            delete e;
            return st;
        }
        e->plans.push_back(pl);
    }
    // one schedule per direction for all members, so that members of equal
    // line-solve shape share a launch
    if ((st = set_window_all(e, 0, 4, 17)) || (st = set_window_all(e, 1, 2, 17))) {
        delete e;
        return st;
    }
    *out = e;
    return IGA_OK;
}

iga_status iga_ensemble_destroy(iga_ensemble *ens)
{
    delete ens;
    return IGA_OK;
}

iga_status iga_ensemble_size(const iga_ensemble *ens, int32_t *n)
{
    if (!ens || !n) return fail(IGA_EINVAL, "NULL argument");
    *n = (int32_t)ens->plans.size();
    return IGA_OK;
}

iga_status iga_ensemble_launches(const iga_ensemble *ens, int32_t *per_step)
{
    if (!ens || !per_step) return fail(IGA_EINVAL, "NULL argument");
    const int g2 = groups(ens, 0, true) + groups(ens, 1, true);
    *per_step = 1 + groups(ens, 0) + groups(ens, 1) + (g2 ? 1 + g2 : 0);
    return IGA_OK;
}

iga_status iga_ensemble_step(iga_ensemble *ens, void *const *T, void *const *fuel, void *stream)
{
    if (!ens) return fail(IGA_EINVAL, "ensemble is NULL");
    iga_status st;
    if ((st = check_fields(ens, T, fuel)) || (st = bind(ens, T, fuel))) return st;
    return step_bound(ens, static_cast<hipStream_t>(stream));
}

iga_status iga_ensemble_run(iga_ensemble *ens, void *const *T, void *const *fuel, int64_t nsteps,
                            void *stream)
{
    if (!ens) return fail(IGA_EINVAL, "ensemble is NULL");
    if (nsteps < 0) return fail(IGA_EINVAL, "nsteps must be >= 0");
    iga_status st;
    if ((st = check_fields(ens, T, fuel)) || (st = bind(ens, T, fuel))) return st;
    if (nsteps == 0) return IGA_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t chunk = std::min<int64_t>(nsteps, 64);
    const int64_t tail = nsteps % chunk;
    if ((st = capture(ens, ens->graph.main, chunk))) return st;
    if (tail && (st = capture(ens, ens->graph.tail, tail))) return st;
    for (int64_t done = 0; done < nsteps;) {
        const int64_t k = std::min<int64_t>(chunk, nsteps - done);
        IGA_HIP(hipGraphLaunch(k == chunk ? ens->graph.main.exec : ens->graph.tail.exec, s));
        done += k;
    }
    return IGA_OK;
}

iga_status iga_ensemble_set_schedule(iga_ensemble *ens, int32_t dir, int32_t lines,
                                     int32_t waves_per_line)
{
    if (!ens) return fail(IGA_EINVAL, "ensemble is NULL");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    auto pow2 = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8 || v == 16; };
    if (!pow2(lines)) return fail(IGA_EINVAL, "lines must be 1, 2, 4, 8 or 16");
    if (!pow2(waves_per_line) || waves_per_line > 8)
        return fail(IGA_EINVAL, "waves_per_line must be 1, 2, 4 or 8");
    std::vector<Schedule> keep;
    for (iga_plan *pl : ens->plans) keep.push_back(pl->sched[dir]);
    iga_status st = set_schedule_all(ens, dir, lines, waves_per_line);
    if (st) {
        for (size_t m = 0; m < ens->plans.size(); ++m) {
            if (keep[m].win) (void)choose_window_schedule(ens->plans[m], dir, keep[m].lines, keep[m].mm);
            else (void)choose_schedule(ens->plans[m], dir, keep[m].lines, keep[m].wpl);
        }
        ens->unbind();
    }
    return st;
}

iga_status iga_ensemble_set_window_schedule(iga_ensemble *ens, int32_t dir, int32_t lines,
                                            int32_t rows_per_lane)
{
    if (!ens) return fail(IGA_EINVAL, "ensemble is NULL");
    if (dir != 0 && dir != 1) return fail(IGA_EINVAL, "dir must be 0 or 1");
    if (lines != 1 && lines != 2 && lines != 4 && lines != 8 && lines != 16)
        return fail(IGA_EINVAL, "lines must be 1, 2, 4, 8 or 16");
    std::vector<Schedule> keep;
    for (iga_plan *pl : ens->plans) keep.push_back(pl->sched[dir]);
    iga_status st = set_window_all(ens, dir, lines, rows_per_lane);
    if (st) {
        for (size_t m = 0; m < ens->plans.size(); ++m) {
            if (keep[m].win) (void)choose_window_schedule(ens->plans[m], dir, keep[m].lines, keep[m].mm);
            else (void)choose_schedule(ens->plans[m], dir, keep[m].lines, keep[m].wpl);
        }
        ens->unbind();
    }
    return st;
}

iga_status iga_ensemble_set_assembly_rows(iga_ensemble *ens, int32_t rows)
{
    if (!ens) return fail(IGA_EINVAL, "ensemble is NULL");
    if (rows < ens->P + 1) return fail(IGA_EINVAL, "rows must be at least p + 1");
    for (iga_plan *pl : ens->plans) pl->asm_rows = rows;
    ens->unbind();
    return IGA_OK;
}

iga_status iga_ensemble_set_assembly_stacking(iga_ensemble *ens, int32_t stacked)
{
    if (!ens) return fail(IGA_EINVAL, "ensemble is NULL");
    if (stacked != 0 && stacked != 1) return fail(IGA_EINVAL, "stacked must be 0 or 1");
    for (iga_plan *pl : ens->plans) pl->asm_stack = stacked;
    ens->unbind();
    return IGA_OK;
}

iga_status iga_ensemble_autotune(iga_ensemble *ens, void *const *T, void *const *fuel, int32_t reps,
                                 void *stream)
{
    if (!ens) return fail(IGA_EINVAL, "ensemble is NULL");
    if (reps < 1) return fail(IGA_EINVAL, "reps must be >= 1");
    iga_status st;
    if ((st = check_fields(ens, T, fuel))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = ens->plans.size();
    // assembly rows, timed on the first assembly (it writes scratch only)
    {
        int best = ens->plans[0]->asm_rows, best_stack = ens->plans[0]->asm_stack;
        float best_ms = 1e30f;
        for (int stack : {0, 1})
            for (int rows : ASSEMBLY_ROW_CANDIDATES) {
                if (rows < ens->P + 1) continue;
                if ((st = iga_ensemble_set_assembly_rows(ens, rows)) ||
                    (st = iga_ensemble_set_assembly_stacking(ens, stack)) || (st = bind(ens, T, fuel)))
                    return st;
                float ms = time_launches(s, reps, [&] { return launch_batch(ens->a1, s); });
                if (ms >= 0 && ms < best_ms) {
                    best_ms = ms;
                    best = rows;
                    best_stack = stack;
                }
            }
        if ((st = iga_ensemble_set_assembly_rows(ens, best)) ||
            (st = iga_ensemble_set_assembly_stacking(ens, best_stack)))
            return st;
    }
    // line solves: lines per workgroup x wavefronts per line (or rows per
    // lane), timed on both of the step's launches of the direction with the
    // step's own jobs (fused Crank-Nicolson solves, base states, zero skips),
    // every state field replaced by a scratch buffer of the member: the
    // caller's fields are not written
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<iga_plan *> second;
        std::vector<std::vector<SweepJob>> ja(n), jb;
        for (size_t m = 0; m < n; ++m) {
            iga_plan *pl = ens->plans[m];
            const bool r2 = pl->scratch_r2.ptr != nullptr;   // FP32 plans
            StepPhases sp;
            step_phases(pl, r2 ? pl->scratch_r2.ptr : pl->scratch_r.ptr,
                        r2 ? pl->scratch_rf2.ptr : pl->scratch_rf.ptr, sp);
            ja[m] = dir == 0 ? sp.x1 : sp.y1;
            if (sp.two) {
                second.push_back(pl);
                jb.push_back(dir == 0 ? sp.x2 : sp.y2);
            }
        }
        int best_l = 0, best_w = 0, best_win = 0;
        float best_ms = 1e30f;
        auto consider = [&](int lines, int w, int win) {
            std::vector<BatchLaunch> bla, blb;
            if (build_sweep_batch(ens->plans, dir, ja, bla) != IGA_OK) return;
            if (!second.empty() && build_sweep_batch(second, dir, jb, blb) != IGA_OK) return;
            float ms = time_launches(s, reps, [&] {
                iga_status e = launch_all(bla, s);
                return e ? e : launch_all(blb, s);
            });
            if (ms >= 0 && ms < best_ms) {
                best_ms = ms;
                best_l = lines;
                best_w = w;
                best_win = win;
            }
        };
        for (int mm : {9, 13, 17, 25, 33})
            for (int lines : {1, 2, 4, 8, 16})
                if (set_window_all(ens, dir, lines, mm) == IGA_OK) consider(lines, mm, 1);
        for (int wpl : {1, 2, 4}) {
            for (int lines : {1, 2, 4, 8, 16}) {
                if (lines * wpl > 16) continue;
                if (set_schedule_all(ens, dir, lines, wpl) != IGA_OK) continue;
                consider(lines, wpl, 0);
            }
        }
        if (!best_l) return fail(IGA_EUNSUPPORTED, "no line-solve schedule fits every member");
        if ((st = best_win ? set_window_all(ens, dir, best_l, best_w)
                           : set_schedule_all(ens, dir, best_l, best_w)))
            return st;
    }
    IGA_HIP(hipStreamSynchronize(s));
    ens->unbind();
    set_error("");
    return IGA_OK;
}

}  // extern "C"
