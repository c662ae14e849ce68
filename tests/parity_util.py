"""Comparison helpers of the GPU parity tests (test infrastructure; uses the
oracle as the checker).

FP32 plans keep their state in float.  Where a quadrature point's ignition
decision [T > T_ig and fuel > thr] (generic equation at the start of Section 3)
lies within float rounding of a threshold, the float kernel and the FP64
oracle can both be right and decide differently.  The oracle flags the
elements whose decision lies within AMB_DT kelvin of T_ig or AMB_DF of the
fuel threshold.  Dofs farther than MASK_RADIUS elements from flagged elements
are compared element by element and in relative L2 at the FP32 tolerance.
A flipped source decays by about 0.43 per row through the mass-dominated 1D
inverses, to below 1e-4 of its size at 12 rows.

Inside the mask the difference must stay within what flipped decisions can
cause.  The bracket is two oracle steps with both thresholds moved by
(AMB_DT, AMB_DF), one in each direction: every ambiguous decision is taken the
same way in each.  An implementation that decides a subset differently moves
the state by the sum of the responses to its flips.  Flips of one sign have
responses whose sum is the bracket's, up to the partial cancellation of the
alternating rows of the 1D inverses, so twice the bracket's largest
difference bounds it.
"""
from __future__ import annotations


import numpy as np

import oracle

AMB_DT, AMB_DF, MASK_RADIUS = 0.01, 1e-5, 12
EPS32 = 2.0 ** -24


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def absmax(a):
    return float(np.abs(a).max()) if a.size else 0.0


def near_mask(flags, p, radius=MASK_RADIUS):
    """Dofs within `radius` elements of a flagged element's (p+1)^2 dofs."""
    from scipy.ndimage import maximum_filter
    Nx, Ny = flags.shape[0] + p, flags.shape[1] + p
    near = np.zeros((Nx, Ny), dtype=bool)
    ex, ey = np.nonzero(flags)
    for a in range(p + 1):
        for b in range(p + 1):
            near[ex + a, ey + b] = True
    if near.any():
        near = maximum_filter(near, size=2 * radius + 1)
    return near


def shifted_desc(od, dT, dF):
    """The descriptor with the ignition thresholds moved by (dT, dF)."""
    d = oracle.Desc.from_buffer_copy(od)
    d.c.t_ig = od.c.t_ig + dT
    d.c.fuel_thr = od.c.fuel_thr + dF
    return d


def bracket_step(od, T, F, dT=AMB_DT, dF=AMB_DF):
    """Oracle steps with every ambiguous decision taken one way, then the
    other: (T, fuel) with the thresholds lowered, and raised."""
    lo = oracle.step(shifted_desc(od, -dT, -dF), T, F)
    hi = oracle.step(shifted_desc(od, dT, dF), T, F)
    return lo, hi


def step_report_fp32(od, p, Tprev, Fprev, Tg, Fg):
    """One FP32 step on the GPU, (Tprev, Fprev) -> (Tg, Fg), against the
    oracle's step from the same state.  Returns the measured quantities."""
    To, Fo, fl = oracle.step_flagged(od, Tprev, Fprev, AMB_DT, AMB_DF)
    near = near_mask(fl, p)
    out = ~near
    r = {"flagged": int(fl.sum()), "masked": float(near.mean())}
    for name, g, o, prev in (("T", Tg, To, Tprev), ("fuel", Fg, Fo, Fprev)):
        d = g - o
        r[f"{name}_rel"] = float(np.linalg.norm(d[out]) / np.linalg.norm(o))
        r[f"{name}_max"] = absmax(d[out])
        r[f"{name}_scale"] = absmax(o)                 # largest value
        r[f"{name}_change"] = absmax((o - prev)[out])  # largest change over the step
        r[f"{name}_inside"] = absmax(d[near])
        r[f"{name}_bracket"] = 0.0
    if near.any():
        (Tl, Fl), (Th, Fh) = bracket_step(od, Tprev, Fprev)
        r["T_bracket"] = absmax((Tl - Th)[near])
        r["fuel_bracket"] = absmax((Fl - Fh)[near])
    return r


def fp32_elementwise_bound(r, name):
    """Element-wise bound outside the mask: a few float ulps of the largest
    value (the state is rounded to float every step) plus 1e-5 of the largest
    change over the step (the float increment)."""
    return 8 * EPS32 * r[f"{name}_scale"] + 1e-5 * r[f"{name}_change"]


def assert_step_fp32(r, tol=1e-6, what=""):
    for name in ("T", "fuel"):
        assert r[f"{name}_rel"] < tol, (what, name, r)
        assert r[f"{name}_max"] <= fp32_elementwise_bound(r, name), (what, name, r)
        inside_bound = 2.0 * r[f"{name}_bracket"] + fp32_elementwise_bound(r, name)
        assert r[f"{name}_inside"] <= inside_bound, (what, name, r)


def assert_close_fp64(g, o, tol=1e-12, what=""):
    """Relative L2 and element-wise against the largest value."""
    e = rel(g, o)
    m = absmax(g - o)
    assert e < tol, (what, e)
    assert m <= tol * absmax(o), (what, m, absmax(o))
    return e


def f32(a):
    """The float32 value of an FP64 array, as FP64 (what an FP32 plan holds)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def band_apply(band, X, axis):
    """A X along `axis` for a banded operator in the oracle's band layout
    (band[i, k - i + p] = A[i, k])."""
    p = (band.shape[1] - 1) // 2
    Xm = np.moveaxis(np.asarray(X, dtype=np.float64), axis, 0)
    N = Xm.shape[0]
    pad = np.zeros((N + 2 * p,) + Xm.shape[1:])
    pad[p:p + N] = Xm
    out = np.zeros_like(Xm)
    for j in range(2 * p + 1):
        shape = (N,) + (1,) * (Xm.ndim - 1)
        out += band[:, j].reshape(shape) * pad[j:j + N]
    return np.moveaxis(out, 0, axis)


def increment_rhs(od, substep, R, RF, T, F):
    """The increment form an FP32 plan assembles: R - A_impl T with the
    substep's implicit Kronecker operator, and R_fuel - (M^x (x) M^y) fuel."""
    ax, mx = oracle.operator(od, 0, 0), oracle.operator(od, 0, 1)
    ay, my = oracle.operator(od, 1, 0), oracle.operator(od, 1, 1)
    if od.scheme == oracle.PR and substep == 1:
        first, second = mx, ay
    elif od.scheme == oracle.EXPLICIT:
        first, second = mx, my
    else:
        first, second = ax, my
    dR = R - band_apply(second, band_apply(first, T, 0), 1)
    dRF = None if RF is None else RF - band_apply(my, band_apply(mx, F, 0), 1)
    return dR, dRF


FLIP_K = 0.5   # kelvin: a dof that differs by more is taken as affected by a flipped decision


def points_radius(nel, npts=256):
    """Sample-grid rows that cover MASK_RADIUS element rows on an nel mesh."""
    return max(1, -(-MASK_RADIUS * npts // nel))


def flip_report(g, r, radius=MASK_RADIUS, thresh=FLIP_K):
    """Compare two temperature coefficient arrays from runs that may have
    decided ambiguous ignition points differently.  A flipped decision ignites
    (or spares) an element a step earlier, a local difference of up to tens
    of kelvin that then moves with the front.  Returns the relative L2 over
    all dofs, the number and fraction of dofs differing by more than `thresh`
    kelvin, and the relative L2 over the dofs farther than `radius` rows from
    any of them (where the runs must agree to the FP32 tolerance)."""
    from scipy.ndimage import maximum_filter
    d = g - r
    hit = np.abs(d) > thresh
    near = maximum_filter(hit, size=2 * radius + 1) if hit.any() else hit
    return {"rel": rel(g, r), "max_abs": absmax(d), "flipped": int(hit.sum()),
            "flipped_frac": float(hit.mean()), "near_frac": float(near.mean()),
            "out_rel": float(np.linalg.norm(d[~near]) / np.linalg.norm(r))}
