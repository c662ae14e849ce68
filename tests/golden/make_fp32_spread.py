"""Writes tests/golden/fp32_spread.json: how far the FP64 oracle's own
trajectory moves when its state is perturbed at float32 resolution.

TEST INFRASTRUCTURE ONLY: calls nothing but ``oracle/`` and the shared input
generators.  Every quantity here is an oracle-versus-oracle comparison.

Why.  The ignition indicator [T > T_ig and fuel > thr] of the generic equation
(start of Section 3) is discontinuous.  A state stored in float32 differs
from the FP64 one by about half an ulp (6e-5 K at 800 K), so quadrature points
within that distance of T_ig can be decided either way by two correct
implementations, and each such decision changes the local source by
O(10 K) * tau.  Over many steps the trajectories then separate along the fire
front.  This script measures that separation for the model itself, with FP64
arithmetic throughout:

  ref          the oracle from (T0, fuel0);
  round_each   the oracle with (T, fuel) rounded to float32 after every step
               (the least perturbation any implementation that keeps its
               state in float32 carries);
  round_init   the oracle from float32-rounded (T0, fuel0) only;
  perturb_k    the oracle with (T, fuel) multiplied by (1 + u 2^-24),
               u ~ U(-1, 1) seeded with k, after every step (a different
               perturbation of the same size).

For each variant against ref: relative L2 of the T and fuel coefficients,
relative L2 of T at 256^2 cell-centred points, the max |dT|, the dofs whose
T differs by more than 0.5 K (taken as affected by a flipped decision) and
the relative L2 away from them, and the burned fractions (element-centre
fuel < 0.1).  The 4096^2 case also stores the
oracle's own temperature at the 256^2 points after 200 steps
(oracle_regional4096_200steps_256.npz).

Usage:  python tests/golden/make_fp32_spread.py CASE [CASE ...]
Cases are merged into the existing JSON file.  Costs on 8 host threads:
regional256 ~10 s, regional1024 ~8 min (all variants), mixed_members ~14 min,
cubic20 ~10 min, regional4096 ~40 min.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

sys.path.insert(0, os.path.dirname(HERE))
import oracle  # noqa: E402
import parity_util as pu  # noqa: E402
from paper_2604_19370_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "fp32_spread.json")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def f32(a):
    return a.astype(np.float32).astype(np.float64)


def run_variant(od, T0, F0, steps, kind, seed=0, checkpoints=()):
    """The variant's state after `steps` steps, and at each checkpoint."""
    at = {}
    if kind in ("ref", "round_init"):
        T, F = (T0, F0) if kind == "ref" else (f32(T0), f32(F0))
        done = 0
        for k in sorted(set(checkpoints) | {steps}):
            T, F = oracle.run(od, T, F, k - done)
            done = k
            at[k] = (T, F)
        return at[steps], at
    rng = np.random.default_rng(seed)
    T, F = (f32(T0), f32(F0)) if kind == "round_each" else (T0.copy(), F0.copy())
    for k in range(1, steps + 1):
        T, F = oracle.step(od, T, F)
        if kind == "round_each":
            T, F = f32(T), f32(F)
        else:
            T = T * (1.0 + rng.uniform(-1, 1, T.shape) * 2.0 ** -24)
            F = F * (1.0 + rng.uniform(-1, 1, F.shape) * 2.0 ** -24)
        if k in checkpoints:
            at[k] = (T, F)
    at[steps] = (T, F)
    return (T, F), at


def compare(od, sc, ref, var):
    xs = (np.arange(256) + 0.5) / 256 * sc.len_x
    ys = (np.arange(256) + 0.5) / 256 * sc.len_y
    gr = oracle.eval_grid(od, ref[0], xs, ys)
    gv = oracle.eval_grid(od, var[0], xs, ys)
    fl = pu.flip_report(var[0], ref[0])
    return {
        "rel_T": rel(var[0], ref[0]),
        "rel_fuel": rel(var[1], ref[1]),
        "rel_T_256": rel(gv, gr),
        "max_abs_T": float(np.abs(var[0] - ref[0]).max()),
        "flipped_dofs": fl["flipped"],
        "flipped_frac": fl["flipped_frac"],
        "rel_T_away_from_flips": fl["out_rel"],
        "burned_ref": oracle.burned_fraction(od, ref[1]),
        "burned_var": oracle.burned_fraction(od, var[1]),
    }


def spread(sc, variants, coeffs=None, save_grid=None, checkpoints=()):
    od = oracle.desc_from_scenario(sc, coeffs=coeffs)
    t0 = time.time()
    ref, ref_at = run_variant(od, sc.T0, sc.fuel0, sc.steps, "ref", checkpoints=checkpoints)
    out = {"steps": sc.steps, "dofs": int(sc.T0.size)}
    if save_grid:
        # the oracle's temperature at 256^2 cell-centred points after the run,
        # and its burned fraction, for comparisons at the sampled points
        xs = (np.arange(256) + 0.5) / 256 * sc.len_x
        ys = (np.arange(256) + 0.5) / 256 * sc.len_y
        np.savez_compressed(os.path.join(HERE, save_grid), xs=xs, ys=ys,
                            T=oracle.eval_grid(od, ref[0], xs, ys),
                            burned=oracle.burned_fraction(od, ref[1]), steps=sc.steps)
    for v in variants:
        kind, seed = (v.split("_")[0], int(v.split("_")[1])) if v.startswith("perturb") else (v, 0)
        var, var_at = run_variant(od, sc.T0, sc.fuel0, sc.steps, kind, seed, checkpoints)
        out[v] = compare(od, sc, ref, var)
        if checkpoints:
            out[v]["at_step"] = {str(k): compare(od, sc, ref_at[k], var_at[k]) for k in checkpoints}
        print(f"  {v}: {out[v]}  ({time.time() - t0:.0f} s)", flush=True)
    return out


def cubic_members(scheme, members, steps):
    scs = inputs.cubic_ensemble(max(members) + 1, scheme=scheme)
    out = {}
    for m in members:
        sc = scs[m]
        sc.steps = steps
        out[f"member{m}"] = spread(sc, ["round_each"])
    return out


CASES = {
    # regional Strang-CN workload (p = 2, dt 5e-4, seed 1), 200 steps
    "regional256": lambda: {
        "ignition": spread(inputs.regional_strang(seed=1, nel=256, steps=200),
                           ["round_each", "round_init"])},
    "regional1024": lambda: {
        "ignition": spread(inputs.regional_strang(seed=1, nel=1024, steps=200),
                           ["round_each", "round_init", "perturb_1", "perturb_2"]),
        "no_ignition": spread(inputs.regional_strang(seed=1, nel=1024, steps=200),
                              ["round_each"], coeffs={"c_ign": 0.0})},
    "regional4096": lambda: {
        "ignition": spread(inputs.regional_strang(seed=1, nel=4096, steps=200), ["round_each"],
                           save_grid="oracle_regional4096_200steps_256.npz", checkpoints=(20,))},
    # members 0 and 15 of the 16-member cubic 2048^2 ensembles (seeds 2000,
    # 2015), 20 steps of each scheme
    "cubic20": lambda: {s: cubic_members(s, (0, 15), 20) for s in ("strang", "pr")},
    # members 0-3 of the 64-member uneven ensemble (seeds 1000-1003), 300 steps
    "mixed_members": lambda: {
        f"member{m}": spread(inputs.mixed_ensemble(4)[m], ["round_each"]) for m in range(4)},
}


def main(argv):
    for case in argv:
        print(f"{case} on {oracle.get_threads()} threads", flush=True)
        result = CASES[case]()
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}   # merge with other runs
        data[case] = result
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ["regional256"])
