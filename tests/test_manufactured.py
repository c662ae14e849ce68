"""Forced steps and the manufactured-solution study (Section 6.1) on the oracle.

Pins of the forced step, against what the mathematics fixes:
- the Gauss points are the Gauss-Legendre nodes of numpy mapped to each element;
- with every other term off, a constant source c raises every coefficient by
  exactly tau c per step (the splines reproduce constants), in all schemes;
- a source s(x, y) = x (or y) raises the coefficients by tau times the
  Greville abscissae along x (or y) -- x lies in the spline space and its
  coefficients are those abscissae -- which fixes the sample layout;
- the generator's source matches finite differences of its exact solution
  put into the equation.

Properties the paper states for the study, on the oracle (50^2, p = 2):
- "linear" reading (nonlinear terms off): every scheme converges at first
  order in dt toward the exact solution;
- "full" reading (all smooth terms on): no scheme is unconditionally stable
  (dt = 1/4 diverges), and all are accurate for small steps (dt = 1/64).
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import oracle
from paper_2604_19370_amd import inputs

ALL_OFF = dict(c_adv=0.0, c_diff=0.0, c_react=0.0, c_nld=0.0, c_ign=0.0, c_forcing=0.0, c_rad=0.0)
NONLINEAR_OFF = dict(c_nld=0.0, c_rad=0.0, c_forcing=0.0, c_ign=0.0)
GRID = np.linspace(0.0, 100.0, 201)


def srcs(scheme, f0, f1):
    return (f0, None) if scheme == "explicit" else (f0, f1)


def test_quad_points_are_mapped_gauss_legendre():
    for n, p, L in ((7, 1, 3.5), (10, 2, 100.0), (5, 3, 12.0)):
        g, _ = leggauss(p + 1)
        h = L / n
        want = np.concatenate([e * h + (g + 1.0) * h / 2.0 for e in range(n)])
        np.testing.assert_allclose(oracle.quad_points(n, p, L), want, rtol=0, atol=1e-13 * L)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("scheme", ["pr", "strang", "explicit"])
def test_constant_source_adds_tau_c(p, scheme):
    tau, c = 0.3, 7.5
    d = oracle.make_desc(9, 6, p, 9.0, 6.0, tau, scheme, coeffs=ALL_OFF)
    q = p + 1
    T = 300 + np.random.default_rng(1).uniform(0, 100, (9 + p, 6 + p))
    S = np.full((9 * q, 6 * q), c)
    Tn, Fn = oracle.step_forced(d, T, np.zeros_like(T), *srcs(scheme, S, S))
    np.testing.assert_allclose(Tn, T + tau * c, rtol=0, atol=1e-12 * 400)
    assert np.all(Fn == 0.0)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("scheme", ["pr", "strang", "explicit"])
def test_linear_source_layout(p, scheme):
    tau, nx, ny, Lx, Ly = 0.5, 8, 5, 16.0, 10.0
    d = oracle.make_desc(nx, ny, p, Lx, Ly, tau, scheme, coeffs=ALL_OFF)
    xq, yq = oracle.quad_points(nx, p, Lx), oracle.quad_points(ny, p, Ly)
    T = np.zeros((nx + p, ny + p))
    Sx = np.repeat(xq[:, None], yq.size, axis=1)
    Sy = np.repeat(yq[None, :], xq.size, axis=0)
    Tn, _ = oracle.step_forced(d, T, np.zeros_like(T), *srcs(scheme, Sx, Sx))
    want = tau * Lx * inputs.greville(nx, p)[:, None] * np.ones((1, ny + p))
    np.testing.assert_allclose(Tn, want, rtol=0, atol=1e-12 * tau * Lx)
    Tn, _ = oracle.step_forced(d, T, np.zeros_like(T), *srcs(scheme, Sy, Sy))
    want = tau * Ly * np.ones((nx + p, 1)) * inputs.greville(ny, p)[None, :]
    np.testing.assert_allclose(Tn, want, rtol=0, atol=1e-12 * tau * Ly)


@pytest.mark.parametrize("wind", [(0.0, 0.0), (1.0, -0.5)])
def test_manufactured_source_matches_finite_differences(wind):
    c = oracle.default_coeffs()
    _, m = inputs.manufactured(c, 10, bx=wind[0], by=wind[1])
    rng = np.random.default_rng(5)
    h, k = 1e-3, 1e-5
    for x, y, t in rng.uniform([2, 2, 0.1], [98, 98, 0.9], size=(20, 3)):
        u = lambda a, b, s: float(m.exact(a, b, s))
        ut = (u(x, y, t + k) - u(x, y, t - k)) / (2 * k)
        ux = (u(x + h, y, t) - u(x - h, y, t)) / (2 * h)
        uy = (u(x, y + h, t) - u(x, y - h, t)) / (2 * h)
        # div(D(u) grad u) with D = c_diff + c_nld u^3, by differences of fluxes
        D = lambda a, b: c["c_diff"] + c["c_nld"] * u(a, b, t) ** 3
        fx = lambda a: D(a, y) * (u(a + h, y, t) - u(a - h, y, t)) / (2 * h)
        fy = lambda b: D(x, b) * (u(x, b + h, t) - u(x, b - h, t)) / (2 * h)
        div = (fx(x + h) - fx(x - h)) / (2 * h) + (fy(y + h) - fy(y - h)) / (2 * h)
        U = u(x, y, t)
        rhs = (-c["c_adv"] * (wind[0] * ux + wind[1] * uy) + div + c["c_react"] * U
               + c["c_forcing"] - c["c_rad"] * U ** 4)
        f = float(m.source(x, y, t))
        assert abs((ut - rhs) - f) < 1e-5 * max(abs(f), abs(ut), 1.0)


def oracle_error(nel, scheme, dt, coeffs, p=2):
    """Relative L2 error at t = 1 of the oracle's forced run (None: unstable)."""
    sc, m = inputs.manufactured(coeffs, nel, p, scheme, dt)
    d = oracle.make_desc(nel, nel, p, 100.0, 100.0, dt, scheme, coeffs=coeffs)
    xq = oracle.quad_points(nel, p, 100.0)
    X, Y = xq[:, None], xq[None, :]
    T, F = sc.T0.copy(), sc.fuel0.copy()
    for n in range(sc.steps):
        t = n * dt
        T, F = oracle.step_forced(d, T, F, *srcs(scheme, m.source(X, Y, t),
                                                  m.source(X, Y, t + 0.5 * dt)))
        if not np.isfinite(T).all() or np.abs(T).max() > 1e9:
            return None
    V = oracle.eval_grid(d, T, GRID, GRID)
    E = m.exact(GRID[:, None], GRID[None, :], sc.steps * dt)
    e = float(np.linalg.norm(V - E) / np.linalg.norm(E))
    return e if e <= 1.0 else None


@pytest.mark.parametrize("scheme", ["explicit", "pr", "strang"])
def test_first_order_convergence_linear_reading(scheme):
    co = oracle.default_coeffs()
    co.update(NONLINEAR_OFF)
    errs = [oracle_error(50, scheme, dt, co) for dt in (1 / 16, 1 / 32, 1 / 64)]
    assert all(e is not None for e in errs), errs
    orders = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(0.8 < o < 1.3 for o in orders), (errs, orders)


@pytest.mark.parametrize("scheme", ["explicit", "pr", "strang"])
def test_full_reading_is_conditionally_stable(scheme):
    co = oracle.default_coeffs()
    assert oracle_error(50, scheme, 1 / 4, co) is None       # diverges
    e = oracle_error(50, scheme, 1 / 64, co)
    assert e is not None and e < 2e-3, e
