"""Dense brute-force checks for the oracle on tiny grids (test helper).

Independent of ``oracle/``: B-spline bases come from ``scipy.interpolate.BSpline``,
Gauss rules from ``numpy.polynomial.legendre.leggauss``, and every operator is a
dense matrix built by quadrature and combined with ``np.kron`` /
``numpy.linalg.solve``.  Sizes are meant for grids of at most ~10 x 10 elements.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.interpolate import BSpline


def knots(nel, p, L):
    return np.concatenate([np.zeros(p), np.linspace(0.0, L, nel + 1), np.full(p, L)])


def basis(nel, p, L, x, deriv=0):
    """(len(x), nel+p) values (deriv 0) or derivatives of all basis functions."""
    N = nel + p
    spl = BSpline(knots(nel, p, L), np.eye(N), p, extrapolate=True)
    if deriv:
        spl = spl.derivative(deriv)
    return np.asarray(spl(np.asarray(x, dtype=np.float64)))


def quad_1d(nel, L, nq):
    g, w = leggauss(nq)
    h = L / nel
    xs = np.concatenate([e * h + (g + 1.0) * h / 2.0 for e in range(nel)])
    ws = np.concatenate([w * h / 2.0 for _ in range(nel)])
    return xs, ws


def mats_1d(nel, p, L, nq=None):
    nq = nq or p + 1
    x, w = quad_1d(nel, L, nq)
    Bv, Bd = basis(nel, p, L, x), basis(nel, p, L, x, 1)
    M = Bv.T @ (w[:, None] * Bv)
    K = Bd.T @ (w[:, None] * Bd)
    G = Bv.T @ (w[:, None] * Bd)   # row = test function, column = d/dx trial
    return M, K, G


def dense_2d_operator(nel_x, nel_y, p, Lx, Ly, cx, cy):
    """Dense 2D operator  sum over 2D quadrature points of
    w [cx[0] u v + cx[1] u_x v_x + cx[2] u_x v]  applied along x with mass in y,
    i.e. the weak form (u, v)-(u_x, v_x)-(u_x, v) terms of one direction,
    plus the same with the roles of x and y in cy.  Built from 2D basis
    values B_i(x)B_j(y) at the tensor quadrature points (not from 1D matrices)."""
    xq, wx = quad_1d(nel_x, Lx, p + 1)
    yq, wy = quad_1d(nel_y, Ly, p + 1)
    Vx, Dx = basis(nel_x, p, Lx, xq), basis(nel_x, p, Lx, xq, 1)
    Vy, Dy = basis(nel_y, p, Ly, yq), basis(nel_y, p, Ly, yq, 1)
    Phi = np.einsum("ai,bj->abij", Vx, Vy).reshape(xq.size * yq.size, -1)
    Phx = np.einsum("ai,bj->abij", Dx, Vy).reshape(xq.size * yq.size, -1)
    Phy = np.einsum("ai,bj->abij", Vx, Dy).reshape(xq.size * yq.size, -1)
    W = np.outer(wx, wy).ravel()[:, None]
    A = (cx[0] + cy[0]) * Phi.T @ (W * Phi)
    A += cx[1] * Phx.T @ (W * Phx) + cx[2] * Phi.T @ (W * Phx)
    A += cy[1] * Phy.T @ (W * Phy) + cy[2] * Phi.T @ (W * Phy)
    return A


def rhs(sc_desc, T, fuel, edir, alpha, beta, with_fuel=False):
    """Quadrature right-hand side of one substep with dense basis tables.
    sc_desc: dict with nel_x, nel_y, p, len_x, len_y, dt, coefficients and wind."""
    d = sc_desc
    p = d["p"]
    xq, wx = quad_1d(d["nel_x"], d["len_x"], p + 1)
    yq, wy = quad_1d(d["nel_y"], d["len_y"], p + 1)
    Vx, Dx = basis(d["nel_x"], p, d["len_x"], xq), basis(d["nel_x"], p, d["len_x"], xq, 1)
    Vy, Dy = basis(d["nel_y"], p, d["len_y"], yq), basis(d["nel_y"], p, d["len_y"], yq, 1)
    S = Vx @ T @ Vy.T
    Sx = Dx @ T @ Vy.T
    Sy = Vx @ T @ Dy.T
    Fu = Vx @ fuel @ Vy.T
    X, Y = np.meshgrid(xq, yq, indexing="ij")
    if d["wind_kind"] == "sincos":
        bx = d["bx"] + d["ax"] * np.sin(2 * np.pi * Y / d["len_y"])
        by = d["by"] + d["ay"] * np.cos(2 * np.pi * X / d["len_x"])
    else:
        bx = np.full_like(X, d["bx"])
        by = np.full_like(X, d["by"])
    ign = (S > d["t_ig"]) & (Fu > d["fuel_thr"])
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        arr = np.where(ign, S * np.exp(-d["t_act"] / np.where(ign, S, 1.0)), 0.0)
    f = (-d["c_adv"] * ((bx - d["bbar_x"]) * Sx + (by - d["bbar_y"]) * Sy)
         + d["c_forcing"] - d["c_rad"] * S ** 4 + d["c_ign"] * arr)
    g = d["c_nld"] * S ** 3
    W = np.outer(wx, wy)
    dSe = Sy if edir else Sx
    bbar_e = d["bbar_y"] if edir else d["bbar_x"]
    react = 0.0 if edir else d["c_react"]
    a0 = W * (S - alpha * (d["c_adv"] * bbar_e * dSe - react * S) + beta * f)
    ax = W * (-(0.0 if edir else alpha * d["c_diff"]) * Sx - beta * g * Sx)
    ay = W * (-(alpha * d["c_diff"] if edir else 0.0) * Sy - beta * g * Sy)
    R = Vx.T @ a0 @ Vy + Dx.T @ ax @ Vy + Vx.T @ ay @ Dy
    if not with_fuel:
        return R
    af = W * (Fu - d["dt"] * d["fuel_rate"] * arr * Fu)
    return R, Vx.T @ af @ Vy


def directional(d, dirn, which):
    """Dense 1D operator of the scheme (which 0 = A, 1 = M, 2 = B)."""
    n = d["nel_y"] if dirn else d["nel_x"]
    L = d["len_y"] if dirn else d["len_x"]
    M, K, G = mats_1d(n, d["p"], L)
    if d["scheme"] == "explicit":
        g = 0.0
    elif d["scheme"] == "pr":
        g = 0.5 * d["dt"]
    else:
        g = 0.25 * d["dt"] if dirn == 0 else 0.5 * d["dt"]
    react = 0.0 if dirn else d["c_react"]
    bbar = d["bbar_y"] if dirn else d["bbar_x"]
    lin = d["c_diff"] * K + d["c_adv"] * bbar * G
    if which == 1:
        return M
    if which == 0:
        return (1 - g * react) * M + g * lin
    return (1 + g * react) * M - g * lin


def kron_solve(A, B, R):
    n = R.size
    return np.linalg.solve(np.kron(A, B), R.reshape(n)).reshape(R.shape)


def explicit_rhs(d, T, fuel):
    """Right-hand side of the explicit L2-projection step written straight
    from the equation (no split of the operator, the full wind b): per
    quadrature point  S v + tau [ -C_diff grad S . grad v - C_adv (b . grad S) v
    + C_react S v + (C_forcing - C_rad S^4 + C_ign [ign] S e^{-T_act/S}) v
    - C_nld S^3 grad S . grad v ],  and the fuel  Fu v - tau rate [ign] S e^{-T_act/S} Fu v."""
    p, tau = d["p"], d["dt"]
    xq, wx = quad_1d(d["nel_x"], d["len_x"], p + 1)
    yq, wy = quad_1d(d["nel_y"], d["len_y"], p + 1)
    Vx, Dx = basis(d["nel_x"], p, d["len_x"], xq), basis(d["nel_x"], p, d["len_x"], xq, 1)
    Vy, Dy = basis(d["nel_y"], p, d["len_y"], yq), basis(d["nel_y"], p, d["len_y"], yq, 1)
    # 2D basis tables: rows = quadrature points, columns = dofs (i, j)
    Phi = np.einsum("ai,bj->abij", Vx, Vy).reshape(xq.size * yq.size, -1)
    Phx = np.einsum("ai,bj->abij", Dx, Vy).reshape(xq.size * yq.size, -1)
    Phy = np.einsum("ai,bj->abij", Vx, Dy).reshape(xq.size * yq.size, -1)
    W = np.outer(wx, wy).ravel()
    S, Sx, Sy, Fu = Phi @ T.ravel(), Phx @ T.ravel(), Phy @ T.ravel(), Phi @ fuel.ravel()
    X, Y = np.meshgrid(xq, yq, indexing="ij")
    X, Y = X.ravel(), Y.ravel()
    if d["wind_kind"] == "sincos":
        bx = d["bx"] + d["ax"] * np.sin(2 * np.pi * Y / d["len_y"])
        by = d["by"] + d["ay"] * np.cos(2 * np.pi * X / d["len_x"])
    else:
        bx, by = np.full_like(X, d["bx"]), np.full_like(X, d["by"])
    ign = (S > d["t_ig"]) & (Fu > d["fuel_thr"])
    arr = np.zeros_like(S)
    arr[ign] = S[ign] * np.exp(-d["t_act"] / S[ign])
    flux = -(d["c_diff"] + d["c_nld"] * S ** 3)          # coefficient of grad S . grad v
    src = (-d["c_adv"] * (bx * Sx + by * Sy) + d["c_react"] * S + d["c_forcing"]
           - d["c_rad"] * S ** 4 + d["c_ign"] * arr)     # coefficient of v
    R = Phi.T @ (W * (S + tau * src)) + Phx.T @ (W * tau * flux * Sx) + Phy.T @ (W * tau * flux * Sy)
    RF = Phi.T @ (W * (Fu - tau * d["fuel_rate"] * arr * Fu))
    return R.reshape(T.shape), RF.reshape(T.shape)


def step(d, T, fuel):
    """One full step with dense Kronecker matrices and numpy.linalg.solve."""
    Mx, My = directional(d, 0, 1), directional(d, 1, 1)
    if d["scheme"] == "explicit":
        R, RF = explicit_rhs(d, T, fuel)
        return kron_solve(Mx, My, R), kron_solve(Mx, My, RF)
    Ax, Ay = directional(d, 0, 0), directional(d, 1, 0)
    if d["scheme"] == "pr":
        R, RF = rhs(d, T, fuel, 1, 0.5 * d["dt"], 0.5 * d["dt"], with_fuel=True)
        Th = kron_solve(Ax, My, R)
        R2 = rhs(d, Th, fuel, 0, 0.5 * d["dt"], 0.5 * d["dt"])
        Tn = kron_solve(Mx, Ay, R2)
    else:
        R, RF = rhs(d, T, fuel, 0, 0.25 * d["dt"], 0.5 * d["dt"], with_fuel=True)
        Ts = kron_solve(Ax, My, R)
        By = directional(d, 1, 2)
        R2 = (np.kron(Mx, By) @ Ts.ravel()).reshape(Ts.shape)
        Tss = kron_solve(Mx, Ay, R2)
        R3 = rhs(d, Tss, fuel, 0, 0.25 * d["dt"], 0.5 * d["dt"])
        Tn = kron_solve(Ax, My, R3)
    return Tn, kron_solve(Mx, My, RF)
