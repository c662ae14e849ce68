"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times: autotuned schedules and graph-replayed runs (`iga_run`).

Regional Strang-CN workload (p = 2, dt 5e-4, filtered fuel map with
firebreaks, three ignitions, sin/cos wind):
- 1024^2: FP64 per step against the oracle stepping from the GPU's own
  previous state (1e-12); FP32+refine per step (1e-6, away from elements
  whose ignition decision is within float rounding of its threshold), and
  after 200 steps against the oracle run from the same initial state (1e-5
  without the ignition term; with it, 1e-4 and the same burned area).
- 4096^2: one step of each precision against the oracle; 200 FP32+refine
  steps against 200 FP64 steps on the GPU, compared on the coefficients and
  on temperatures at 256^2 cell-centred points.
"""
import numpy as np
import pytest

import oracle
from paper_2604_19370_amd import iga, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def tuned_plan(sc, precision):
    pl = iga.Plan.from_scenario(sc, precision=precision)
    pl.factor()
    T = dev(sc.T0, pl.dtype)
    F = dev(sc.fuel0, pl.dtype)
    pl.autotune(T, F, reps=3)
    return pl, T, F


# FP32: where a quadrature point's ignition decision lies within float
# rounding of T_ig (or of the fuel threshold) the FP32 kernel and the FP64
# oracle may both be right and decide differently.  The oracle flags those
# elements; dofs farther than MASK_RADIUS elements from them are compared at
# the full tolerance (a flipped source term decays by ~0.43 per row through
# the mass-dominated 1D inverses, below 1e-4 of its size at 12 rows), and
# inside the mask the difference is bounded by the flipped source term.
AMB_DT, AMB_DF, MASK_RADIUS = 0.01, 1e-5, 12


def masked_rel(gpu, ref, flags, p):
    from scipy.ndimage import maximum_filter
    near = np.zeros(ref.shape, dtype=bool)
    ex, ey = np.nonzero(flags)
    for a in range(p + 1):
        for b in range(p + 1):
            near[ex + a, ey + b] = True
    if near.any():
        near = maximum_filter(near, size=2 * MASK_RADIUS + 1)
    diff = gpu - ref
    outside = float(np.linalg.norm(diff[~near]) / np.linalg.norm(ref))
    inside = float(np.abs(diff[near]).max()) if near.any() else 0.0
    return outside, inside, float(near.mean())


def run_steps(pl, T, F, n):
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pl.run(T, F, n, stream)
    torch.cuda.synchronize()


def sample_points(n=256):
    return (np.arange(n) + 0.5) / n


@pytest.fixture(scope="module")
def regional_1024():
    return inputs.regional_strang(seed=1, nel=1024, steps=200)


@pytest.fixture(scope="module")
def regional_4096():
    return inputs.regional_strang(seed=1, nel=4096, steps=200)


def test_1024_fp64_per_step(regional_1024):
    sc = regional_1024
    print(f"1024^2 fp64 per step ({sc.name})", flush=True)
    od = oracle.desc_from_scenario(sc)
    pl, T, F = tuned_plan(sc, "fp64")
    Th, Fh = sc.T0, sc.fuel0
    worst = 0.0
    for k in range(20):
        run_steps(pl, T, F, 1)
        To, Fo = oracle.step(od, Th, Fh)
        Th, Fh = host(T), host(F)
        worst = max(worst, rel(Th, To), rel(Fh, Fo))
        # continue from the GPU state so each comparison is one step
    print(f"worst per-step rel L2 over 20 steps: {worst:.3e}", flush=True)
    assert worst < 1e-12
    pl.close()


def test_1024_fp32_per_step(regional_1024):
    sc = regional_1024
    print(f"1024^2 fp32 per step ({sc.name})", flush=True)
    od = oracle.desc_from_scenario(sc)
    pl, T, F = tuned_plan(sc, "fp32")
    Th, Fh = sc.T0, sc.fuel0
    worst, worst_in, masked = 0.0, 0.0, 0.0
    for k in range(5):
        run_steps(pl, T, F, 1)
        To, Fo, fl = oracle.step_flagged(od, Th, Fh, AMB_DT, AMB_DF)
        Th, Fh = host(T), host(F)
        for g, o in ((Th, To), (Fh, Fo)):
            out, inside, frac = masked_rel(g, o, fl, sc.p)
            worst, worst_in, masked = max(worst, out), max(worst_in, inside), max(masked, frac)
    print(f"per-step rel L2 over 5 steps: {worst:.3e} outside ambiguous elements "
          f"(masked fraction {masked:.2e}, max diff inside {worst_in:.3e})", flush=True)
    assert worst < 1e-6
    assert worst_in < 50.0
    pl.close()


@pytest.mark.parametrize("ignition", [True, False])
def test_1024_fp32_200_steps_vs_oracle(regional_1024, ignition):
    """200 FP32+refine steps against 200 oracle steps from the same state.
    Without the ignition term the trajectories stay within 1e-5.  With it,
    threshold re-decisions along the fire front (the FP32 state differs from
    the FP64 one by ~1e-4 K near T_ig) separate them locally, by ~1e-5; the
    burned area agrees."""
    sc = regional_1024
    coeffs = None if ignition else {"c_ign": 0.0}
    print(f"1024^2 fp32 200 steps vs oracle, ignition {ignition}", flush=True)
    od = oracle.desc_from_scenario(sc, coeffs=coeffs)
    pl = iga.Plan.from_scenario(sc, precision="fp32", coeffs=coeffs)
    pl.factor()
    T, F = dev(sc.T0, pl.dtype), dev(sc.fuel0, pl.dtype)
    pl.autotune(T, F, reps=3)
    run_steps(pl, T, F, 200)
    To, Fo = oracle.run(od, sc.T0, sc.fuel0, 200)
    eT, eF = rel(host(T), To), rel(host(F), Fo)
    bo, bg = oracle.burned_fraction(od, Fo), oracle.burned_fraction(od, host(F))
    print(f"after 200 steps: rel L2 T {eT:.3e}, fuel {eF:.3e}; burned fraction oracle {bo:.5f} "
          f"gpu {bg:.5f}", flush=True)
    if ignition:
        assert eT < 1e-4 and eF < 1e-4
        assert abs(bo - bg) < 1e-3 * max(bo, 1e-3)
    else:
        assert eT < 1e-5 and eF < 1e-5
    pl.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_4096_one_step(regional_4096, precision, tol):
    sc = regional_4096
    print(f"4096^2 {precision} one step", flush=True)
    od = oracle.desc_from_scenario(sc)
    pl, T, F = tuned_plan(sc, precision)
    run_steps(pl, T, F, 1)
    if precision == "fp64":
        To, Fo = oracle.step(od, sc.T0, sc.fuel0)
        eT, eF = rel(host(T), To), rel(host(F), Fo)
        print(f"rel L2 T {eT:.3e}, fuel {eF:.3e}", flush=True)
        assert eT < tol and eF < tol
    else:
        To, Fo, fl = oracle.step_flagged(od, sc.T0, sc.fuel0, AMB_DT, AMB_DF)
        eT, iT, frac = masked_rel(host(T), To, fl, sc.p)
        eF, iF, _ = masked_rel(host(F), Fo, fl, sc.p)
        print(f"rel L2 outside {fl.sum()} ambiguous elements (masked dofs {frac:.2e}): "
              f"T {eT:.3e}, fuel {eF:.3e}; max diff inside: T {iT:.3e}, fuel {iF:.3e}",
              flush=True)
        assert eT < tol and eF < tol
        assert iT < 50.0 and iF < 0.05
    pl.close()


@pytest.mark.parametrize("ignition", [True, False])
def test_4096_fp32_vs_fp64_200_steps(regional_4096, ignition):
    """200 steps of FP32+refine against FP64 on the GPU (FP64 matches the
    oracle to ~1e-14 per step above).  Without the ignition term the FP32
    trajectory stays within 1e-5.  With it, the threshold indicator turns
    the FP32 state's rounding (~1e-4 K near T_ig) into a different decision
    at a few hundred quadrature points per step along the fire front, each a
    local O(10 K) change of the source: the trajectories then separate along
    the front, by ~1e-4 relative L2 after 200 steps, while the burned area
    agrees."""
    sc = regional_4096
    coeffs = None if ignition else {"c_ign": 0.0}
    print(f"4096^2 fp32 vs fp64, 200 steps, ignition {ignition}", flush=True)
    od = oracle.desc_from_scenario(sc, coeffs=coeffs)
    out = {}
    for precision in ("fp64", "fp32"):
        pl = iga.Plan.from_scenario(sc, precision=precision, coeffs=coeffs)
        pl.factor()
        T = dev(sc.T0, pl.dtype)
        F = dev(sc.fuel0, pl.dtype)
        pl.autotune(T, F, reps=3)
        run_steps(pl, T, F, 200)
        out[precision] = (host(T), host(F))
        assert np.isfinite(out[precision][0]).all()
        pl.close()
        del T, F
        torch.cuda.empty_cache()
    eT = rel(out["fp32"][0], out["fp64"][0])
    eF = rel(out["fp32"][1], out["fp64"][1])
    xs = sample_points() * sc.len_x
    ys = sample_points() * sc.len_y
    g32 = oracle.eval_grid(od, out["fp32"][0], xs, ys)
    g64 = oracle.eval_grid(od, out["fp64"][0], xs, ys)
    eg = rel(g32, g64)
    b32 = oracle.burned_fraction(od, out["fp32"][1])
    b64 = oracle.burned_fraction(od, out["fp64"][1])
    print(f"200 steps fp32 vs fp64: rel L2 T {eT:.3e}, fuel {eF:.3e}, T at 256^2 points {eg:.3e}; "
          f"burned fraction {b32:.5f} / {b64:.5f}", flush=True)
    if ignition:
        assert eT < 5e-4 and eF < 1e-4 and eg < 2e-4
        assert abs(b32 - b64) < 1e-3 * max(b64, 1e-3)
    else:
        assert eT < 1e-5 and eF < 1e-5 and eg < 1e-5
