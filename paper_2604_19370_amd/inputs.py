"""Seeded synthetic workloads for the wildfire stepper.

This module only *generates inputs*: fuel rasters, ignition points, wind
descriptions and the initial spline-coefficient arrays of temperature and fuel.
It holds none of the stepper's arithmetic (no quadrature, no matrices, no
solves), so both the HIP library and the CPU oracle can start from the same
arrays.

The paper's own workloads (satellite-derived fuel maps of the Valparaiso and
Gran Canaria fires, Section 6) are not available; these generators stand in for
them with fields shaped like regional domains: a fuel raster in [0, 1] with
burnable patches and straight zero-fuel firebreaks, Gaussian-smoothed
ignitions added to the ambient temperature (Section 2.1, "Ignition
initialization"), and a steady wind.

Initial coefficients.  The state is a pair of coefficient arrays on the
tensor-product B-spline space (uniform open knots, degree p).  A field given as
a function (the ignition Gaussians) or as a per-element raster (fuel) is turned
into coefficients by sampling it at the Greville abscissae -- the
variation-diminishing spline approximation -- so coefficients, and therefore
the spline values, stay within the range of the input.  Layout: dof (i, j) at
``[i, j]`` of an ``(nel_x + p, nel_y + p)`` float64 array.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

T_AMBIENT = 300.0


@dataclasses.dataclass
class Wind:
    """b(x, y).  'const': (bx, by).  'sincos': (bx + ax sin 2 pi y^, by + ay cos 2 pi x^)
    with x^, y^ the coordinates scaled to [0, 1].  (bbar_x, bbar_y) is the
    constant part that the scheme treats implicitly (the domain mean of b)."""
    kind: str = "const"
    bx: float = 0.0
    by: float = 0.0
    ax: float = 0.0
    ay: float = 0.0
    bbar_x: Optional[float] = None
    bbar_y: Optional[float] = None

    def as_dict(self) -> dict:
        d = dataclasses.asdict(self)
        if d["bbar_x"] is None:
            d["bbar_x"] = self.bx
        if d["bbar_y"] is None:
            d["bbar_y"] = self.by
        return d


@dataclasses.dataclass
class Scenario:
    name: str
    nel_x: int
    nel_y: int
    p: int
    len_x: float
    len_y: float
    dt: float
    scheme: str          # 'pr' or 'strang'
    steps: int
    wind: Wind
    seed: int
    ignitions: List[Tuple[float, float]]
    T0: Optional[np.ndarray] = None
    fuel0: Optional[np.ndarray] = None
    fuel_raster: Optional[np.ndarray] = None

    @property
    def Nx(self) -> int:
        return self.nel_x + self.p

    @property
    def Ny(self) -> int:
        return self.nel_y + self.p

    @property
    def ndof(self) -> int:
        return self.Nx * self.Ny

    def wind_dict(self) -> dict:
        return self.wind.as_dict()


# ---------------------------------------------------------------------------
# sampling points
# ---------------------------------------------------------------------------
def greville(nel: int, p: int) -> np.ndarray:
    """Greville abscissae in [0, 1] of the uniform open knot vector with nel
    elements: xi_i = (t_{i+1} + ... + t_{i+p}) / p, i = 0 .. nel+p-1."""
    k = np.arange(nel + 2 * p + 1)
    t = np.clip((k - p) / nel, 0.0, 1.0)
    return np.array([t[i + 1:i + p + 1].mean() for i in range(nel + p)])


def _element_of(xi: np.ndarray, nel: int) -> np.ndarray:
    return np.minimum((xi * nel).astype(np.int64), nel - 1)


def raster_to_coeffs(raster: np.ndarray, p: int) -> np.ndarray:
    """Per-element raster (nel_x, nel_y) -> coefficients: the raster value of
    the element holding each Greville point."""
    nx, ny = raster.shape
    ex = _element_of(greville(nx, p), nx)
    ey = _element_of(greville(ny, p), ny)
    return np.ascontiguousarray(raster[np.ix_(ex, ey)], dtype=np.float64)


def ignition_coeffs(nel_x: int, nel_y: int, p: int, centres, sigma: float = 0.05,
                    peak: float = 600.0, ambient: float = T_AMBIENT) -> np.ndarray:
    """ambient + peak * max_k exp(-|x^ - c_k|^2 / (2 sigma^2)) at the Greville points."""
    gx = greville(nel_x, p)[:, None]
    gy = greville(nel_y, p)[None, :]
    bump = np.zeros((gx.size, gy.size))
    for cx, cy in centres:
        bump = np.maximum(bump, np.exp(-((gx - cx) ** 2 + (gy - cy) ** 2) / (2.0 * sigma ** 2)))
    return np.ascontiguousarray(ambient + peak * bump, dtype=np.float64)


# ---------------------------------------------------------------------------
# fuel rasters
# ---------------------------------------------------------------------------
def fuel_iid(rng: np.random.Generator, nel_x: int, nel_y: int, lo=0.5, hi=1.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=(nel_x, nel_y))


def fuel_filtered(rng: np.random.Generator, nel_x: int, nel_y: int, sigma_cells=8.0,
                  mean=0.6, spread=0.25, n_breaks=3, break_width=4) -> np.ndarray:
    """White noise -> Gaussian filter (sigma in cells, reflecting borders,
    truncated at 4 sigma) -> standardised -> clip(mean + spread z, 0, 1), then
    `n_breaks` straight zero-fuel strips `break_width` cells wide, each
    horizontal or vertical with probability 1/2, offset uniform in
    [0.1, 0.9) of the extent, running the full length of the domain."""
    from scipy.ndimage import gaussian_filter

    z = rng.standard_normal((nel_x, nel_y))
    z = gaussian_filter(z, sigma=sigma_cells, mode="reflect", truncate=4.0)
    z = (z - z.mean()) / max(z.std(), 1e-300)
    fuel = np.clip(mean + spread * z, 0.0, 1.0)
    for _ in range(n_breaks):
        vertical = rng.uniform() < 0.5
        extent = nel_x if vertical else nel_y
        off = int(rng.uniform(0.1, 0.9) * extent)
        sl = slice(off, min(off + break_width, extent))
        if vertical:
            fuel[sl, :] = 0.0
        else:
            fuel[:, sl] = 0.0
    return fuel


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def _finish(sc: Scenario, raster: np.ndarray) -> Scenario:
    sc.fuel_raster = raster
    sc.fuel0 = raster_to_coeffs(raster, sc.p)
    sc.T0 = ignition_coeffs(sc.nel_x, sc.nel_y, sc.p, sc.ignitions)
    return sc


def plain_pr_64(seed: int = 0, nel: int = 64, steps: int = 20) -> Scenario:
    """64x64 quadratic, Peaceman-Rachford, dt 1e-3, 20 steps; one ignition with
    centre uniform in [0.3, 0.7]^2; fuel i.i.d. U[0.5, 1] per element; constant
    wind (1.0, 0.5)."""
    rng = np.random.default_rng(seed)
    centre = tuple(rng.uniform(0.3, 0.7, size=2))
    raster = fuel_iid(rng, nel, nel)
    sc = Scenario(name=f"plain_pr_{nel}", nel_x=nel, nel_y=nel, p=2, len_x=float(nel),
                  len_y=float(nel), dt=1e-3, scheme="pr", steps=steps,
                  wind=Wind("const", 1.0, 0.5), seed=seed, ignitions=[centre])
    return _finish(sc, raster)


def regional_strang(seed: int = 1, nel: int = 1024, steps: int = 200, p: int = 2,
                    dt: float = 5e-4) -> Scenario:
    """nel^2 quadratic, Strang with Crank-Nicolson substeps, dt 5e-4; filtered
    fuel map with 3 firebreaks; wind (1 + 0.3 sin 2 pi y^, 0.5 cos 2 pi x^)
    (mean (1, 0)); 3 ignitions with centres uniform in [0.1, 0.9]^2."""
    rng = np.random.default_rng(seed)
    raster = fuel_filtered(rng, nel, nel)
    centres = [tuple(rng.uniform(0.1, 0.9, size=2)) for _ in range(3)]
    sc = Scenario(name=f"regional_strang_{nel}", nel_x=nel, nel_y=nel, p=p,
                  len_x=float(nel), len_y=float(nel), dt=dt, scheme="strang", steps=steps,
                  wind=Wind("sincos", bx=1.0, by=0.0, ax=0.3, ay=0.5, bbar_x=1.0, bbar_y=0.0),
                  seed=seed, ignitions=centres)
    return _finish(sc, raster)


def ensemble_member(seed: int, sizes=(256, 384, 512, 768, 1024), p: int = 2,
                    scheme: str = "strang", steps: int = 300, dt: float = 5e-4) -> Scenario:
    """One ensemble scenario: grid drawn from `sizes`, its own filtered fuel
    map, constant wind of magnitude U[0, 3] and direction U[0, 2 pi), and 1-4
    ignitions."""
    rng = np.random.default_rng(seed)
    nel = int(rng.choice(np.asarray(sizes)))
    mag = rng.uniform(0.0, 3.0)
    ang = rng.uniform(0.0, 2.0 * np.pi)
    k = int(rng.integers(1, 5))
    raster = fuel_filtered(rng, nel, nel)
    centres = [tuple(rng.uniform(0.1, 0.9, size=2)) for _ in range(k)]
    sc = Scenario(name=f"member_{seed}_{nel}", nel_x=nel, nel_y=nel, p=p, len_x=float(nel),
                  len_y=float(nel), dt=dt, scheme=scheme, steps=steps,
                  wind=Wind("const", mag * np.cos(ang), mag * np.sin(ang)), seed=seed,
                  ignitions=centres)
    return _finish(sc, raster)


def mixed_ensemble(n_members: int = 64, base_seed: int = 1000, **kw) -> List[Scenario]:
    return [ensemble_member(base_seed + m, **kw) for m in range(n_members)]


def cubic_ensemble(n_members: int = 16, base_seed: int = 2000, nel: int = 2048,
                   scheme: str = "strang", steps: int = 500) -> List[Scenario]:
    return [ensemble_member(base_seed + m, sizes=(nel,), p=3, scheme=scheme, steps=steps)
            for m in range(n_members)]


def small_case(seed: int, nel_x: int, nel_y: int, p: int, scheme: str, dt: float = 1e-3,
               wind: Optional[Wind] = None, n_ign: int = 2, filtered: bool = False) -> Scenario:
    """Small random case for parity tests (several tiles and ragged tails)."""
    rng = np.random.default_rng(seed)
    raster = (fuel_filtered(rng, nel_x, nel_y, sigma_cells=2.0) if filtered
              else fuel_iid(rng, nel_x, nel_y))
    centres = [tuple(rng.uniform(0.2, 0.8, size=2)) for _ in range(n_ign)]
    if wind is None:
        wind = Wind("sincos", bx=0.7, by=-0.2, ax=0.3, ay=0.5, bbar_x=0.7, bbar_y=-0.2)
    sc = Scenario(name=f"small_{nel_x}x{nel_y}_p{p}_{scheme}", nel_x=nel_x, nel_y=nel_y, p=p,
                  len_x=float(nel_x), len_y=float(nel_y), dt=dt, scheme=scheme, steps=1,
                  wind=wind, seed=seed, ignitions=centres)
    return _finish(sc, raster)


def ring_of_fire(nel: int = 100, p: int = 2, scheme: str = "strang", dt: float = 5e-3,
                 steps: int = 200, length: float = 100.0, t_comb: float = 1200.0) -> Scenario:
    """The verification problem of Section 5: zero wind, fuel 1 everywhere, and
    a smooth ball of heat at the centre of the square [0, length]^2 (the paper
    uses length 100 and nel = 100).  With d the distance to the centre, the
    initial temperature is 300 + t_comb * g(d) where g is 1 within d <= 5,
    0 beyond d >= 15, and (1 - s^2)^2 with s = (d - 5) / 10 in between (the
    paper gives the two radii as fractions of the domain: 10/200 and 30/200
    of a distance normalised by 100).  Coefficients are Greville samples, as
    for the other workloads.  The paper does not state the time step of this
    run: 5e-3 keeps the explicitly treated nonlinear diffusion (C_nld T^3,
    about 20 at 1500 K) stable on 1 m elements, and 200 steps carry the front
    to a radius of about 30, inside the domain."""
    # distance of each Greville point to the centre, averaged with its mirror
    # point's so the initial state is exactly symmetric under both reflections
    # and under x <-> y (the Greville sums themselves round asymmetrically)
    off = np.abs(greville(nel, p) * length - 0.5 * length)
    off = 0.5 * (off + off[::-1])
    d = np.sqrt(off[:, None] ** 2 + off[None, :] ** 2)
    s = np.clip((d - 5.0) / 10.0, 0.0, 1.0)
    bump = (1.0 - s * s) ** 2
    sc = Scenario(name=f"ring_of_fire_{nel}_p{p}_{scheme}", nel_x=nel, nel_y=nel, p=p,
                  len_x=float(length), len_y=float(length), dt=dt, scheme=scheme,
                  steps=steps, wind=Wind("const", 0.0, 0.0), seed=0, ignitions=[(0.5, 0.5)])
    sc.fuel_raster = np.ones((nel, nel))
    sc.fuel0 = np.ones((sc.Nx, sc.Ny))
    sc.T0 = np.ascontiguousarray(T_AMBIENT + t_comb * bump, dtype=np.float64)
    return sc


# ---------------------------------------------------------------------------
# manufactured solution (Section 6.1, stability and order study)
# ---------------------------------------------------------------------------
MMS_AMPS = ((80.0, 3.0), (30.0, 5.0), (110.0, 1.5))   # (amplitude, lambda) of the three terms


@dataclasses.dataclass
class Manufactured:
    """u(x, y, t) = 300 + sum_k A_k (1 - cos 2 pi x/L)(1 - cos 2 pi y/L) e^{-lambda_k t}
    on [0, L]^2 with L = 100, the exact solution of the paper's order study
    (the mode indices the paper attaches to each term do not enter its
    formula, so all three terms share one spatial shape).  Its normal
    derivative vanishes on the boundary, matching the natural (zero-flux)
    condition of the weak form.  `source` is the forcing f that makes u solve

      u_t = -c_adv b.grad u + c_diff lap u + c_react u + div(c_nld u^3 grad u)
            + c_forcing - c_rad u^4 + f

    -- the generic equation with every smooth term; the fuel is zero, so the
    ignition term is off.  The coefficients and the constant wind b are the
    ones the stepper is given."""
    coeffs: dict
    bx: float = 0.0
    by: float = 0.0
    length: float = 100.0

    def _parts(self, x, y, t):
        a = 2.0 * np.pi / self.length
        x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
        cx, cy, sx, sy = np.cos(a * x), np.cos(a * y), np.sin(a * x), np.sin(a * y)
        g = sum(A * np.exp(-lam * t) for A, lam in MMS_AMPS)
        dg = sum(-lam * A * np.exp(-lam * t) for A, lam in MMS_AMPS)
        phi = (1.0 - cx) * (1.0 - cy)
        phx = a * sx * (1.0 - cy)
        phy = a * (1.0 - cx) * sy
        lap = a * a * (cx * (1.0 - cy) + (1.0 - cx) * cy)
        return g, dg, phi, phx, phy, lap

    def exact(self, x, y, t):
        g, _, phi, _, _, _ = self._parts(x, y, t)
        return T_AMBIENT + g * phi

    def source(self, x, y, t):
        c = self.coeffs
        g, dg, phi, phx, phy, lap = self._parts(x, y, t)
        u = T_AMBIENT + g * phi
        ux, uy, ulap = g * phx, g * phy, g * lap
        div_nld = c["c_nld"] * (3.0 * u * u * (ux * ux + uy * uy) + u ** 3 * ulap)
        return (dg * phi + c["c_adv"] * (self.bx * ux + self.by * uy) - c["c_diff"] * ulap
                - c["c_react"] * u - div_nld - c["c_forcing"] + c["c_rad"] * u ** 4)


def manufactured(coeffs: dict, nel: int = 50, p: int = 2, scheme: str = "pr", dt: float = 1.0 / 16,
                 t_end: float = 1.0, bx: float = 0.0, by: float = 0.0):
    """Scenario of the order study on [0, 100]^2 with nel^2 elements: the
    initial state is u(., ., 0) at the Greville points, the fuel zero, the
    wind the constant (bx, by) (the paper does not state one; zero by
    default).  Returns (scenario, Manufactured)."""
    mms = Manufactured(coeffs=dict(coeffs), bx=bx, by=by)
    L = mms.length
    g = greville(nel, p) * L
    steps = int(round(t_end / dt))
    sc = Scenario(name=f"manufactured_{nel}_p{p}_{scheme}_dt{dt:g}", nel_x=nel, nel_y=nel, p=p,
                  len_x=L, len_y=L, dt=dt, scheme=scheme, steps=steps,
                  wind=Wind("const", bx, by), seed=0, ignitions=[])
    sc.fuel_raster = np.zeros((nel, nel))
    sc.fuel0 = np.zeros((sc.Nx, sc.Ny))
    sc.T0 = np.ascontiguousarray(mms.exact(g[:, None], g[None, :], 0.0), dtype=np.float64)
    return sc, mms
