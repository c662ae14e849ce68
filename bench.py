#!/usr/bin/env python
"""Throughput of the quasi-implicit IGA-ADS wildfire stepper on one MI355X.

Workload: 1024 x 1024 quadratic B-spline elements (1026^2 = 1,052,676 dofs),
Strang splitting with Crank-Nicolson substeps, dt = 5e-4, seeded synthetic
regional inputs (filtered fuel map with 3 firebreaks, 3 Gaussian ignitions,
wind (1 + 0.3 sin 2 pi y^, 0.5 cos 2 pi x^)).  The headline value is the
FP32-with-FP64-refinement stepper in DOF-steps/s; the FP64 stepper on the same
inputs is reported beside it.

One JSON line on stdout.  `roofline` describes the dominant kernel of the FP32
step (measured here with HIP events on the stream it runs on);
`cpu_baseline` is the FP64 CPU oracle timed on the host cores on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_VALU_PEAK = 157.3          # TFLOP/s, MI355X vector FP32 (published)
FP64_VALU_PEAK = 78.6           # TFLOP/s, MI355X vector FP64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nel", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--kernels-only", action="store_true",
                    help="only launch each kernel of the FP32 step --kernel-reps times, plus a "
                         "copy kernel of known size (for profiler runs)")
    ap.add_argument("--tune", action="store_true",
                    help="with --kernels-only: autotune first (as the timed runs do)")
    ap.add_argument("--schedule", type=str, default=None,
                    help="fixed exact line-solve schedule 'xlines,xwpl,ylines,ywpl,asmrows[,stacked]' "
                         "instead of autotuning")
    ap.add_argument("--window-schedule", type=str, default=None,
                    help="fixed windowed line-solve schedule 'xlines,xrows,ylines,yrows,asmrows[,stacked]' "
                         "(rows per lane; stacked 0 or 1, else the plan's default tiling) "
                         "instead of autotuning")
    ap.add_argument("--column-schedule", type=int, default=0,
                    help="with --kernels-only: column-wave x-line solves with this many rows "
                         "per chunk (16 or 32), after --window-schedule")
    ap.add_argument("--no-other-schemes", action="store_true",
                    help="skip the PR and explicit-scheme lines at the same size")
    ap.add_argument("--no-ensembles", action="store_true",
                    help="skip the ensemble workloads (64 uneven members; 16 cubic 2048^2 members)")
    ap.add_argument("--no-paper-meshes", action="store_true",
                    help="skip the FP64 runs on the meshes of the paper's scalability study")
    ap.add_argument("--no-4096", action="store_true",
                    help="skip the 4096^2 precision-form workload")
    return ap.parse_args()


def time_steps(pl, sc, steps, warmup, torch):
    """Graph-replayed timed region of exactly `steps` steps after `warmup`
    eager steps; the graphs are captured beforehand on the same buffers."""
    dt = pl.dtype
    T0 = torch.tensor(sc.T0, dtype=dt, device="cuda")
    F0 = torch.tensor(sc.fuel0, dtype=dt, device="cuda")
    T, F = T0.clone(), F0.clone()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pl.run(T, F, steps, stream)            # captures the graphs (untimed)
        T.copy_(T0)
        F.copy_(F0)
        for _ in range(warmup):
            pl.step(T, F, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        e0.record(stream)
        pl.run(T, F, steps, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    wall = t1 - t0
    ev = e0.elapsed_time(e1) / 1e3
    assert torch.isfinite(T).all() and torch.isfinite(F).all()
    return wall, ev, T, F


AMB_DT, AMB_DF = 0.01, 1e-5    # near-threshold window of the ignition decision (K, fuel)


def sample_grid(sc, n=256):
    import numpy as np
    s = (np.arange(n) + 0.5) / n
    return s * sc.len_x, s * sc.len_y


FLIP_K = 0.5    # kelvin: dofs differing by more are counted as affected by a flipped decision


def burned_elements(pl, fuel, sc):
    """Elements whose centre fuel is below 0.1 (the burned area)."""
    import numpy as np
    cx = (np.arange(sc.nel_x) + 0.5) * sc.len_x / sc.nel_x
    cy = (np.arange(sc.nel_y) + 0.5) * sc.len_y / sc.nel_y
    return int(pl.sample_points(fuel, cx, cy).lt(0.1).sum())


def rel_l2(a, b, torch):
    return float(torch.linalg.vector_norm((a.double() - b.double()).flatten())
                 / torch.linalg.vector_norm(b.double().flatten()))


def precision_errors(pl32, T32, F32, pl64, T64, F64, sc, torch):
    """FP32+refine against FP64 on the same inputs after the same steps:
    relative L2 of the T and fuel coefficients and of T at 256^2 cell-centred
    points (evaluated by the library), the dofs whose T differs by more than
    0.5 K (ignition decisions taken the other way), the burned elements of
    each, and the quadrature points of the FP32 state whose ignition decision
    lies within (0.01 K, 1e-5) of a threshold."""
    xs, ys = sample_grid(sc)
    g32 = pl32.sample_points(T32, xs, ys)
    g64 = pl64.sample_points(T64, xs, ys)
    return {"rel_l2_T": rel_l2(T32, T64, torch), "rel_l2_fuel": rel_l2(F32, F64, torch),
            "rel_l2_T_256": rel_l2(g32, g64, torch),
            "dofs_off_by_0.5K": int((T32.double() - T64).abs().gt(FLIP_K).sum()),
            "burned_elements": [burned_elements(pl32, F32, sc), burned_elements(pl64, F64, sc)],
            "near_threshold_points": pl32.count_ambiguous(T32, F32, AMB_DT, AMB_DF)}


def kernel_times(pl, sc, reps, torch):
    """Average duration of each kernel of one step, launched through the C ABI
    on one stream between HIP events (same grids as inside the step)."""
    dt = pl.dtype
    T = torch.tensor(sc.T0, dtype=dt, device="cuda")
    F = torch.tensor(sc.fuel0, dtype=dt, device="cuda")
    R, RF = torch.empty_like(T), torch.empty_like(T)
    X = torch.randn_like(T)
    stream = torch.cuda.Stream()
    out = {}
    cases = {
        "assemble_s1_fuel": lambda: pl.assemble_rhs(0, T, F, R, RF, stream),
        "assemble_s3": lambda: pl.assemble_rhs(2, T, F, R, None, stream),
        "sweep_x_A": lambda: pl.line_solve(0, 0, X, stream),
        "sweep_y_M": lambda: pl.line_solve(1, 1, X, stream),
        "sweep_y_cn": lambda: pl.line_solve(1, 2, X, stream),
    }
    with torch.cuda.stream(stream):
        for name, fn in cases.items():
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out[name] = e0.elapsed_time(e1) / 1e3 / reps
            if name.startswith("sweep"):
                X.copy_(torch.randn_like(X))
    return out


# Algorithmic work per unit (p = 2, FP32 plan).  Assembly: flops per element of
# the sum-factorised quadrature (row reuse along the marching direction) plus the
# pointwise terms; sweeps and the assembly's memory side: bytes per dof.
def assembly_flops(p, fuel):
    n = q = p + 1
    fma = 2 * q * n + 3 * q * q * n          # T, dT/dx, dT/dy at the points
    fma += 3 * n * q * q + 2 * n * n * q     # test contraction (v, dv/dx, dv/dy)
    if fuel:
        fma += q * n + q * q * n             # fuel at the points (also read by S3's indicator)
        fma += n * q * q + n * n * q         # fuel right-hand side
    else:
        fma += q * n + q * q * n
    pointwise = 26 if fuel else 24           # flops per quadrature point
    return 2 * fma + pointwise * q * q


# counter-summary entries per kernel of the step (the first one present is
# used: x-lines run windowed or, where the autotuner picks them, by column waves)
KERNEL_FAMILY = {"assemble_s1_fuel": ("k_assemble<float,p=2,fuel=true>",),
                 "assemble_s3": ("k_assemble<float,p=2,fuel=false>",),
                 "sweep_x_A": ("k_wsweep<float,p=2,x-lines>", "k_csweep<2,32>", "k_csweep<2,16>"),
                 "sweep_y_M": ("k_wsweep<float,p=2,y-lines>",),
                 "sweep_y_cn": ("k_wsweep<float,p=2,y-lines>",)}
SOURCES = {"k_assemble": ("assemble.hip",),
           "k_wsweep": ("sweep_win.h", "sweep_kernels.h", "sweep.hip"),
           "k_csweep": ("sweep_col.h", "sweep_col.hip")}


def measured_traffic(kernel, nel):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none for this workload or the kernel's sources changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_regional_strang_{nel}_fp32.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    table = json.loads(m.group(1))["kernels"]
    fam = next((f for f in KERNEL_FAMILY[kernel] if f in table), None)
    if fam is None:
        return None
    ent = table[fam]
    h = hashlib.sha256()
    for f in SOURCES[fam.split("<")[0]]:
        h.update(open(os.path.join(ROOT, "paper_2604_19370_amd", "csrc", f), "rb").read())
    return ent["traffic_bytes"] if h.hexdigest()[:16] == ent["source_hash"] else None


def ambient_elements(sc):
    """Elements whose (p+1)^2 temperature coefficients, in float, all equal
    the ambient temperature (the fixed point of the source): the FP32
    assembly does no work for them (their contribution is exactly zero), so
    they are not counted as algorithmic work of the state the kernels are
    timed on (the initial state)."""
    import numpy as np
    from paper_2604_19370_amd import inputs
    T = np.asarray(sc.T0, dtype=np.float32)
    amb = T == np.float32(inputs.T_AMBIENT)
    e = np.ones((sc.nel_x, sc.nel_y), dtype=bool)
    for a in range(sc.p + 1):
        for b in range(sc.p + 1):
            e &= amb[a:a + sc.nel_x, b:b + sc.nel_y]
    return int(e.sum())


def roofline(kt, p, ndof, nel, nel_x, ambient=0):
    """Roofline entry of the dominant (longest) kernel of the FP32 step.
    ambient: elements the assembly skips (their flops are not counted)."""
    w = 4
    alg_bytes = {"assemble_s1_fuel": 4 * w * ndof, "assemble_s3": 3 * w * ndof,
                 "sweep_x_A": 2 * w * ndof, "sweep_y_M": 2 * w * ndof, "sweep_y_cn": 2 * w * ndof}
    dom = max(kt, key=kt.get)
    traffic = measured_traffic(dom, nel_x)
    roof = {"kernel": dom}
    if dom.startswith("assemble"):
        flops = assembly_flops(p, dom == "assemble_s1_fuel") * (nel - ambient)
        achieved = flops / kt[dom] / 1e12
        roof.update(bound="alu", achieved=round(achieved, 2), peak=FP32_VALU_PEAK, unit="TFLOP/s",
                    frac=round(achieved / FP32_VALU_PEAK, 4),
                    traffic=traffic,
                    elements=nel, elements_ambient=ambient,
                    hbm_gbs=round(alg_bytes[dom] / kt[dom] / 1e9, 1),
                    hbm_frac=round(alg_bytes[dom] / kt[dom] / 1e9 / HBM_PEAK_GBS, 4),
                    flops_per_element=assembly_flops(p, dom == "assemble_s1_fuel"),
                    peak_non_packed=FP32_VALU_PEAK / 2)
    else:
        achieved = alg_bytes[dom] / kt[dom] / 1e9
        roof.update(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic)
    roof["avg_us"] = round(kt[dom] * 1e6, 2)
    roof["kernel_us"] = {k: round(v * 1e6, 2) for k, v in kt.items()}
    return roof


def copy_kernel(n_bytes, reps, torch):
    """Plain device copy (one read and one write of n_bytes per launch): the
    calibration kernel for the profiler's FETCH_SIZE / WRITE_SIZE counters."""
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()


def apply_schedule(pl, spec, windowed=False):
    v = [int(x) for x in spec.split(",")]
    xl, xw, yl, yw, ar = v[:5]
    if windowed:
        pl.set_window_schedule(0, xl, xw)
        pl.set_window_schedule(1, yl, yw)
    else:
        pl.set_schedule(0, xl, xw)
        pl.set_schedule(1, yl, yw)
    pl.set_assembly_rows(ar)
    if len(v) > 5:
        pl.set_assembly_stacking(bool(v[5]))


def ensemble_throughput(scs, steps, torch, iga):
    """DOF-steps/s of an FP32+refine ensemble: autotuned, graph captured
    (untimed), then `steps` graph-replayed steps between HIP events."""
    ens = iga.Ensemble.from_scenarios(scs, precision="fp32")
    Ts = [torch.tensor(sc.T0, dtype=torch.float32, device="cuda") for sc in scs]
    Fs = [torch.tensor(sc.fuel0, dtype=torch.float32, device="cuda") for sc in scs]
    T0 = [t.clone() for t in Ts]
    F0 = [f.clone() for f in Fs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ens.autotune(Ts, Fs, reps=3, stream=stream)
        ens.run(Ts, Fs, steps, stream)             # captures the graphs
        for t, t0, f, f0 in zip(Ts, T0, Fs, F0):
            t.copy_(t0)
            f.copy_(f0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        e0.record(stream)
        ens.run(Ts, Fs, steps, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    launches = ens.launches_per_step
    ok = all(bool(torch.isfinite(t).all()) for t in Ts)
    ens.close()
    # the same steps in FP64 (default schedules, untimed) for the precision
    # error, and the near-threshold points of every FP32 member
    e64 = iga.Ensemble.from_scenarios(scs, precision="fp64")
    T64 = [torch.tensor(sc.T0, dtype=torch.float64, device="cuda") for sc in scs]
    F64 = [torch.tensor(sc.fuel0, dtype=torch.float64, device="cuda") for sc in scs]
    with torch.cuda.stream(stream):
        e64.run(T64, F64, steps, stream)   # the FP32 state is `steps` steps from T0
    torch.cuda.synchronize()
    e64.close()
    worst = {"rel_l2_T": 0.0, "rel_l2_fuel": 0.0, "rel_l2_T_256": 0.0}
    near = flipped = dburn = 0
    for m, sc in enumerate(scs):
        worst["rel_l2_T"] = max(worst["rel_l2_T"], rel_l2(Ts[m], T64[m], torch))
        worst["rel_l2_fuel"] = max(worst["rel_l2_fuel"], rel_l2(Fs[m], F64[m], torch))
        flipped += int((Ts[m].double() - T64[m]).abs().gt(FLIP_K).sum())
        pm = iga.Plan.from_scenario(sc, precision="fp32")
        p64 = iga.Plan.from_scenario(sc, precision="fp64")
        near += pm.count_ambiguous(Ts[m], Fs[m], AMB_DT, AMB_DF)
        xs, ys = sample_grid(sc)
        worst["rel_l2_T_256"] = max(worst["rel_l2_T_256"],
                                    rel_l2(pm.sample_points(Ts[m], xs, ys),
                                           p64.sample_points(T64[m], xs, ys), torch))
        dburn = max(dburn, abs(burned_elements(pm, Fs[m], sc) - burned_elements(p64, F64[m], sc)))
        pm.close()
        p64.close()
    del T64, F64
    dofs = sum(sc.ndof for sc in scs)
    bpd = 60 if scs[0].scheme == "strang" else 52
    out = {"members": len(scs), "dofs": dofs, "steps": steps, "p": scs[0].p,
           "scheme": scs[0].scheme, "value": round(dofs * steps / wall, 1),
           "unit": "DOF-steps/s", "ms_per_step": round(wall / steps * 1e3, 4),
           "event_ms_per_step": round(e0.elapsed_time(e1) / steps, 4),
           "launches_per_step": launches,
           "step_hbm_frac": round(dofs * steps / wall * bpd / (HBM_PEAK_GBS * 1e9), 4),
           "finite": ok,
           "fp32_vs_fp64_after_steps": steps,
           "worst_member_rel_l2_T": worst["rel_l2_T"],
           "worst_member_rel_l2_fuel": worst["rel_l2_fuel"],
           "worst_member_rel_l2_T_256": worst["rel_l2_T_256"],
           "dofs_off_by_0.5K": flipped,
           "worst_member_burned_element_difference": dburn,
           "near_threshold_points": near}
    return out


def ensembles(torch, iga, inputs):
    res = {}
    scs = inputs.mixed_ensemble(64)
    res["mixed64_256to1024_p2_strang"] = ensemble_throughput(scs, 300, torch, iga)
    del scs
    cubic = inputs.cubic_ensemble(16, scheme="strang")
    res["cubic16_2048_p3_strang"] = ensemble_throughput(cubic, 500, torch, iga)
    for sc in cubic:
        sc.scheme = "pr"
    res["cubic16_2048_p3_pr"] = ensemble_throughput(cubic, 500, torch, iga)
    return res


def other_schemes(nel, steps, torch, iga, inputs):
    """The other two schemes on the same regional inputs: Peaceman-Rachford
    (6 launches per step) and the explicit L2 projection of Section 6.1 (3
    launches per step), FP32+refine and FP64, autotuned, graph-replayed."""
    out = {}
    for scheme in ("pr", "explicit"):
        sc = inputs.regional_strang(seed=1, nel=nel, steps=steps)
        sc.scheme = scheme
        for prec in ("fp32", "fp64"):
            pl = iga.Plan.from_scenario(sc, precision=prec)
            pl.factor()
            Tt = torch.tensor(sc.T0, dtype=pl.dtype, device="cuda")
            Ft = torch.tensor(sc.fuel0, dtype=pl.dtype, device="cuda")
            pl.autotune(Tt, Ft, reps=5)
            del Tt, Ft
            wall, ev, T, F = time_steps(pl, sc, steps, 5, torch)
            out[f"{scheme}_{prec}"] = {"value": round(sc.ndof * steps / wall, 1),
                                       "unit": "DOF-steps/s",
                                       "ms_per_step": round(wall / steps * 1e3, 5)}
            pl.close()
    return out


# The meshes and step counts of the paper's CPU scalability study (Section 7):
# 100^2 / 600^2 / 1500^2 elements, 120 / 720 / 1080 steps, p = 1, 2, 3.  The
# paper does not state the scheme or the inputs of those runs; here they are
# the regional Strang-CN inputs at that size, FP64 (the paper's precision),
# graph-replayed.
PAPER_MESHES = ((100, 120), (600, 720), (1500, 1080))


def paper_meshes(torch, iga, inputs):
    out = {}
    for p in (1, 2, 3):
        for nel, steps in PAPER_MESHES:
            sc = inputs.regional_strang(seed=1, nel=nel, steps=steps, p=p)
            pl = iga.Plan.from_scenario(sc, precision="fp64")
            pl.factor()
            wall, ev, T, F = time_steps(pl, sc, steps, 2, torch)
            out[f"p{p}_{nel}x{nel}_{steps}steps"] = {
                "dofs": sc.ndof, "seconds": round(wall, 5),
                "value": round(sc.ndof * steps / wall, 1), "unit": "DOF-steps/s"}
            pl.close()
    return out


def cpu_baseline(sc, budget_s, plans, torch):
    """The FP64 oracle on the host cores over the first steps of the workload
    (as many as fit the time budget), and the GPU steppers' states after the
    same number of steps from the same inputs against the oracle's."""
    import oracle
    d = oracle.desc_from_scenario(sc)
    threads = oracle.get_threads()
    T, F = sc.T0, sc.fuel0
    t0 = time.perf_counter()
    T, F = oracle.step(d, T, F)
    one = time.perf_counter() - t0
    n = max(1, int(budget_s / max(one, 1e-6)) - 1)
    t0 = time.perf_counter()
    T, F = oracle.run(d, T, F, n)
    el = time.perf_counter() - t0
    n_total = n + 1
    el_total = el + one
    errors = {"steps": n_total}
    for prec, pl in plans.items():
        Tg = torch.tensor(sc.T0, dtype=pl.dtype, device="cuda")
        Fg = torch.tensor(sc.fuel0, dtype=pl.dtype, device="cuda")
        pl.run(Tg, Fg, n_total)
        torch.cuda.synchronize()
        To = torch.from_numpy(T).cuda()
        Fo = torch.from_numpy(F).cuda()
        errors[prec] = {"rel_l2_T": rel_l2(Tg, To, torch), "rel_l2_fuel": rel_l2(Fg, Fo, torch)}
    # the same oracle on one core, over the next steps of the run (bounded to
    # a few seconds)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        T1, F1 = oracle.step(d, T, F)
        k1, el1 = 1, time.perf_counter() - t0
        while el1 < min(4.0, budget_s / 3):
            t0 = time.perf_counter()
            T1, F1 = oracle.step(d, T1, F1)
            k1, el1 = k1 + 1, el1 + time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    return {"value": sc.ndof * n_total / el_total, "unit": "DOF-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sc.nel_x}x{sc.nel_y} p={sc.p} Strang-CN FP64: the first {n_total} steps "
                      f"from the initial state ({el_total:.1f} s on {threads} OpenMP threads)",
            "value_1core": sc.ndof * k1 / el1,
            "sample_1core": f"steps {n_total + 1}-{n_total + k1} on one OpenMP thread ({el1:.1f} s)",
            "gpu_vs_oracle": errors}


def stepper_leg(sc, steps, warmup, args, torch, iga):
    """FP32+refine and FP64 on one workload: autotuned (or the fixed
    schedule), graph-replayed timed run, per-kernel event times, and the
    precision errors between the two final states.  Returns the plans (open)
    and the measurements."""
    res, ktimes, plans, finals = {}, {}, {}, {}
    for prec in ("fp32", "fp64"):
        pl = iga.Plan.from_scenario(sc, precision=prec)
        pl.factor()
        Tt = torch.tensor(sc.T0, dtype=pl.dtype, device="cuda")
        Ft = torch.tensor(sc.fuel0, dtype=pl.dtype, device="cuda")
        if args.schedule:
            apply_schedule(pl, args.schedule)
        elif args.window_schedule and prec == "fp32":
            apply_schedule(pl, args.window_schedule, windowed=True)
        else:
            pl.autotune(Tt, Ft, reps=10)      # untimed: picks tiles / workgroup widths
        del Tt, Ft
        wall, ev, T, F = time_steps(pl, sc, steps, warmup, torch)
        res[prec] = dict(wall=wall, ev=ev, dofs=sc.ndof * steps / wall,
                         sched=[dict(pl.schedule(0), **pl.solver(0)),
                                dict(pl.schedule(1), **pl.solver(1)),
                                {"assembly_rows": pl.assembly_rows, "assembly_stacked": pl.assembly_stacked}])
        ktimes[prec] = kernel_times(pl, sc, args.kernel_reps, torch)
        plans[prec], finals[prec] = pl, (T, F)
    errs = precision_errors(plans["fp32"], *finals["fp32"], plans["fp64"], *finals["fp64"], sc, torch)
    errs["after_steps"] = warmup + steps
    return plans, res, ktimes, errs


def config_4096(args, torch, iga, inputs):
    """The precision form at scale: 4096^2 quadratic, Strang-CN, FP32+refine
    against FP64 on the same inputs, with the roofline of its dominant
    kernel and the whole step against HBM."""
    sc = inputs.regional_strang(seed=1, nel=4096, steps=args.steps)
    plans, res, ktimes, errs = stepper_leg(sc, args.steps, args.warmup, args, torch, iga)
    for pl in plans.values():
        pl.close()
    kt = ktimes["fp32"]
    out = {"workload": "regional Strang-CN 4096x4096 quadratic, dt 5e-4",
           "dofs": sc.ndof, "steps": args.steps,
           "value": round(res["fp32"]["dofs"], 1), "unit": "DOF-steps/s",
           "ms_per_step": round(res["fp32"]["wall"] / args.steps * 1e3, 5),
           "fp64": {"value": round(res["fp64"]["dofs"], 1),
                    "ms_per_step": round(res["fp64"]["wall"] / args.steps * 1e3, 5),
                    "kernel_us": {k: round(v * 1e6, 2) for k, v in ktimes["fp64"].items()}},
           "fp32_over_fp64": round(res["fp32"]["dofs"] / res["fp64"]["dofs"], 3),
           "step_hbm_frac": round(res["fp32"]["dofs"] * 60 / (HBM_PEAK_GBS * 1e9), 4),
           "roofline": roofline(kt, sc.p, sc.ndof, sc.nel_x * sc.nel_y, sc.nel_x,
                                ambient_elements(sc)),
           "fp32_vs_fp64": errs,
           "schedules": res["fp32"]["sched"]}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this stepper runs on one GPU only; use --gpus 1 (ensemble members "
              "would shard across GPUs with no exchange, one process per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2604_19370_amd import iga, inputs

    sc = inputs.regional_strang(seed=1, nel=args.nel, steps=args.steps)
    if args.kernels_only:
        pl = iga.Plan.from_scenario(sc, precision="fp32")
        pl.factor()
        if args.schedule:
            apply_schedule(pl, args.schedule)
        if args.window_schedule:
            apply_schedule(pl, args.window_schedule, windowed=True)
        if args.column_schedule:
            pl.set_column_schedule(args.column_schedule)
        if args.tune:
            Tt = torch.tensor(sc.T0, dtype=pl.dtype, device="cuda")
            Ft = torch.tensor(sc.fuel0, dtype=pl.dtype, device="cuda")
            pl.autotune(Tt, Ft, reps=10)
            del Tt, Ft
        kt = kernel_times(pl, sc, args.kernel_reps, torch)
        copy_kernel(4 * sc.ndof, args.kernel_reps, torch)
        print(json.dumps({"kernel_us": {k: round(v * 1e6, 2) for k, v in kt.items()},
                          "schedules": [dict(pl.schedule(0), **pl.solver(0)),
                                        dict(pl.schedule(1), **pl.solver(1)),
                                        {"assembly_rows": pl.assembly_rows, "assembly_stacked": pl.assembly_stacked}],
                          "copy_bytes": 4 * sc.ndof}), flush=True)
        pl.close()
        return
    plans, res, ktimes, errs = stepper_leg(sc, args.steps, args.warmup, args, torch, iga)

    kt = ktimes["fp32"]
    ndof = sc.ndof
    nel = sc.nel_x * sc.nel_y
    roof = roofline(kt, sc.p, ndof, nel, sc.nel_x, ambient_elements(sc))

    line = {
        "metric": "DOF-steps/s at 1024^2 quadratic IGA (Strang-CN), FP32+refine; FP64 beside",
        "value": round(res["fp32"]["dofs"], 1),
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["fp32"]["wall"] / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (1D LU and refinement residual f64)",
        "data": "synthetic",
        "config": {"workload": f"regional Strang-CN {sc.nel_x}x{sc.nel_y} quadratic, dt 5e-4",
                   "dofs": ndof, "elements": nel, "steps": args.steps},
        "fp64": {"value": round(res["fp64"]["dofs"], 1),
                 "ms_per_step": round(res["fp64"]["wall"] / args.steps * 1e3, 5),
                 "kernel_us": {k: round(v * 1e6, 2) for k, v in ktimes["fp64"].items()}},
        "fp32_over_fp64": round(res["fp32"]["dofs"] / res["fp64"]["dofs"], 3),
        "fp32_vs_fp64": errs,
        # whole step against HBM: 15 fields of 4 B move per DOF-step in the
        # fused minimum of a Strang step
        "step_hbm_frac": round(res["fp32"]["dofs"] * 60 / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roof,
        "schedules": res["fp32"]["sched"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds, plans, torch)
    for pl in plans.values():
        pl.close()
    del plans
    torch.cuda.empty_cache()
    if not args.no_4096:
        line["config_4096"] = config_4096(args, torch, iga, inputs)
        torch.cuda.empty_cache()
    if not args.no_other_schemes:
        line["other_schemes"] = other_schemes(args.nel, args.steps, torch, iga, inputs)
    if not args.no_ensembles:
        line["ensembles"] = ensembles(torch, iga, inputs)
    if not args.no_paper_meshes:
        line["paper_meshes_fp64"] = paper_meshes(torch, iga, inputs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
