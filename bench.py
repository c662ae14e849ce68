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
    ap.add_argument("--schedule", type=str, default=None,
                    help="fixed exact line-solve schedule 'xlines,xwpl,ylines,ywpl,asmrows' "
                         "instead of autotuning")
    ap.add_argument("--window-schedule", type=str, default=None,
                    help="fixed windowed line-solve schedule 'xlines,xrows,ylines,yrows,asmrows' "
                         "(rows per lane) instead of autotuning")
    ap.add_argument("--no-other-schemes", action="store_true",
                    help="skip the PR and explicit-scheme lines at the same size")
    ap.add_argument("--no-ensembles", action="store_true",
                    help="skip the ensemble workloads (64 uneven members; 16 cubic 2048^2 members)")
    ap.add_argument("--no-paper-meshes", action="store_true",
                    help="skip the FP64 runs on the meshes of the paper's scalability study")
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


KERNEL_FAMILY = {"assemble_s1_fuel": "k_assemble<float,p=2,fuel=true>",
                 "assemble_s3": "k_assemble<float,p=2,fuel=false>",
                 "sweep_x_A": "k_wsweep<float,p=2,x-lines>",
                 "sweep_y_M": "k_wsweep<float,p=2,y-lines>",
                 "sweep_y_cn": "k_wsweep<float,p=2,y-lines>"}
SOURCES = {"k_assemble": ("assemble.hip",),
           "k_wsweep": ("sweep_win.h", "sweep_kernels.h", "sweep.hip")}


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
    fam = KERNEL_FAMILY[kernel]
    ent = json.loads(m.group(1))["kernels"].get(fam)
    if ent is None:
        return None
    h = hashlib.sha256()
    for f in SOURCES[fam.split("<")[0]]:
        h.update(open(os.path.join(ROOT, "paper_2604_19370_amd", "csrc", f), "rb").read())
    return ent["traffic_bytes"] if h.hexdigest()[:16] == ent["source_hash"] else None


def roofline(kt, p, ndof, nel, nel_x):
    """Roofline entry of the dominant (longest) kernel of the FP32 step."""
    w = 4
    alg_bytes = {"assemble_s1_fuel": 4 * w * ndof, "assemble_s3": 3 * w * ndof,
                 "sweep_x_A": 2 * w * ndof, "sweep_y_M": 2 * w * ndof, "sweep_y_cn": 2 * w * ndof}
    dom = max(kt, key=kt.get)
    traffic = measured_traffic(dom, nel_x)
    roof = {"kernel": dom}
    if dom.startswith("assemble"):
        flops = assembly_flops(p, dom == "assemble_s1_fuel") * nel
        achieved = flops / kt[dom] / 1e12
        roof.update(bound="alu", achieved=round(achieved, 2), peak=FP32_VALU_PEAK, unit="TFLOP/s",
                    frac=round(achieved / FP32_VALU_PEAK, 4),
                    traffic=traffic,
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
    xl, xw, yl, yw, ar = (int(v) for v in spec.split(","))
    if windowed:
        pl.set_window_schedule(0, xl, xw)
        pl.set_window_schedule(1, yl, yw)
    else:
        pl.set_schedule(0, xl, xw)
        pl.set_schedule(1, yl, yw)
    pl.set_assembly_rows(ar)


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
    ok = all(bool(torch.isfinite(t).all()) for t in Ts)
    dofs = sum(sc.ndof for sc in scs)
    bpd = 60 if scs[0].scheme == "strang" else 52
    out = {"members": len(scs), "dofs": dofs, "steps": steps, "p": scs[0].p,
           "scheme": scs[0].scheme, "value": round(dofs * steps / wall, 1),
           "unit": "DOF-steps/s", "ms_per_step": round(wall / steps * 1e3, 4),
           "event_ms_per_step": round(e0.elapsed_time(e1) / steps, 4),
           "launches_per_step": ens.launches_per_step,
           "step_hbm_frac": round(dofs * steps / wall * bpd / (HBM_PEAK_GBS * 1e9), 4),
           "finite": ok}
    ens.close()
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


def cpu_baseline(sc, budget_s):
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
            "sample": f"{sc.nel_x}x{sc.nel_y} p={sc.p} Strang-CN FP64, first {n_total} of "
                      f"{sc.steps} steps ({el_total:.1f} s, {threads} OpenMP threads)",
            "value_1core": sc.ndof * k1 / el1,
            "sample_1core": f"steps {n_total + 1}-{n_total + k1} on one OpenMP thread ({el1:.1f} s)"}


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
        kt = kernel_times(pl, sc, args.kernel_reps, torch)
        copy_kernel(4 * sc.ndof, args.kernel_reps, torch)
        print(json.dumps({"kernel_us": {k: round(v * 1e6, 2) for k, v in kt.items()},
                          "schedules": [dict(pl.schedule(0), **pl.solver(0)),
                                        dict(pl.schedule(1), **pl.solver(1)),
                                        {"assembly_rows": pl.assembly_rows, "assembly_stacked": pl.assembly_stacked}],
                          "copy_bytes": 4 * sc.ndof}), flush=True)
        pl.close()
        return
    res = {}
    ktimes = {}
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
        wall, ev, T, F = time_steps(pl, sc, args.steps, args.warmup, torch)
        res[prec] = dict(wall=wall, ev=ev, dofs=sc.ndof * args.steps / wall,
                         sched=[dict(pl.schedule(0), **pl.solver(0)),
                                dict(pl.schedule(1), **pl.solver(1)),
                                {"assembly_rows": pl.assembly_rows, "assembly_stacked": pl.assembly_stacked}])
        ktimes[prec] = kernel_times(pl, sc, args.kernel_reps, torch)
        pl.close()

    kt = ktimes["fp32"]
    ndof = sc.ndof
    nel = sc.nel_x * sc.nel_y
    roof = roofline(kt, sc.p, ndof, nel, sc.nel_x)

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
        # whole step against HBM: 15 fields of 4 B move per DOF-step in the
        # fused minimum of a Strang step
        "step_hbm_frac": round(res["fp32"]["dofs"] * 60 / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roof,
        "schedules": res["fp32"]["sched"],
    }
    if not args.no_other_schemes:
        line["other_schemes"] = other_schemes(args.nel, args.steps, torch, iga, inputs)
    if not args.no_ensembles:
        line["ensembles"] = ensembles(torch, iga, inputs)
    if not args.no_paper_meshes:
        line["paper_meshes_fp64"] = paper_meshes(torch, iga, inputs)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
