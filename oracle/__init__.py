"""FP64 CPU oracle of the quasi-implicit IGA-ADS wildfire stepper (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library: the C source ``oracle.c`` is compiled by ``build()`` with
gcc into ``liboracle.so`` next to this file.

Every array is float64, C-contiguous, with dof (i, j) at ``[i, j]`` of an
``(Nx, Ny)`` array (Nx = nel_x + p, Ny = nel_y + p).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

PR, STRANG, EXPLICIT = 0, 1, 2
WIND_CONST, WIND_SINCOS = 0, 1

_COEFF_NAMES = ("c_adv", "c_diff", "c_react", "c_nld", "c_ign", "t_ig", "fuel_thr",
                "t_act", "c_forcing", "c_rad", "fuel_rate")


class Coeffs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in _COEFF_NAMES]


class Desc(ctypes.Structure):
    _fields_ = [("nel_x", ctypes.c_int), ("nel_y", ctypes.c_int), ("p", ctypes.c_int),
                ("len_x", ctypes.c_double), ("len_y", ctypes.c_double),
                ("dt", ctypes.c_double), ("scheme", ctypes.c_int), ("c", Coeffs),
                ("wind_kind", ctypes.c_int), ("bx", ctypes.c_double), ("by", ctypes.c_double),
                ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("bbar_x", ctypes.c_double), ("bbar_y", ctypes.c_double)]


def build(verbose: bool = False) -> str:
    """Compile oracle.c with gcc (FP64, IEEE semantics, OpenMP for timing)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-shared", "-fPIC",
           _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    global _lib
    _lib = None
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_default_coeffs.argtypes = [ctypes.POINTER(Coeffs)]
        L.oracle_knots.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        L.oracle_gauss.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_basis_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                        dp, ctypes.c_int, dp]
        L.oracle_mat1d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_operator.argtypes = [ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_int, dp]
        L.oracle_band_solve.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                        ctypes.c_long, ctypes.c_long]
        L.oracle_line_solve.argtypes = [ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_int, dp]
        L.oracle_assemble.argtypes = [ctypes.POINTER(Desc), ctypes.c_int, dp, dp, dp, dp]
        L.oracle_step.argtypes = [ctypes.POINTER(Desc), dp, dp]
        L.oracle_step_flagged.argtypes = [ctypes.POINTER(Desc), dp, dp, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_void_p]
        L.oracle_run.argtypes = [ctypes.POINTER(Desc), dp, dp, ctypes.c_int]
        L.oracle_step_forced.argtypes = [ctypes.POINTER(Desc), dp, dp, dp, dp]
        L.oracle_quad_points.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        L.oracle_eval_grid.argtypes = [ctypes.POINTER(Desc), dp, dp, ctypes.c_int, dp,
                                       ctypes.c_int, dp]
        L.oracle_burned_fraction.argtypes = [ctypes.POINTER(Desc), dp, ctypes.c_double]
        L.oracle_burned_fraction.restype = ctypes.c_double
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def default_coeffs() -> dict:
    c = Coeffs()
    lib().oracle_default_coeffs(ctypes.byref(c))
    return {n: getattr(c, n) for n in _COEFF_NAMES}


def make_desc(nel_x, nel_y, p, len_x, len_y, dt, scheme, coeffs=None, wind=None) -> Desc:
    """wind: mapping with kind ('const'|'sincos'), bx, by, ax, ay, bbar_x, bbar_y."""
    d = Desc()
    d.nel_x, d.nel_y, d.p = int(nel_x), int(nel_y), int(p)
    d.len_x, d.len_y, d.dt = float(len_x), float(len_y), float(dt)
    d.scheme = {"pr": PR, "strang": STRANG, "explicit": EXPLICIT}.get(scheme, scheme)
    co = default_coeffs()
    if coeffs:
        co.update(coeffs)
    for n in _COEFF_NAMES:
        setattr(d.c, n, float(co[n]))
    w = dict(kind="const", bx=0.0, by=0.0, ax=0.0, ay=0.0, bbar_x=None, bbar_y=None)
    if wind:
        w.update(wind)
    d.wind_kind = {"const": WIND_CONST, "sincos": WIND_SINCOS}[w["kind"]]
    d.bx, d.by, d.ax, d.ay = float(w["bx"]), float(w["by"]), float(w["ax"]), float(w["ay"])
    d.bbar_x = float(w["bx"] if w["bbar_x"] is None else w["bbar_x"])
    d.bbar_y = float(w["by"] if w["bbar_y"] is None else w["bbar_y"])
    return d


def desc_from_scenario(sc, coeffs=None) -> Desc:
    return make_desc(sc.nel_x, sc.nel_y, sc.p, sc.len_x, sc.len_y, sc.dt, sc.scheme,
                     coeffs=coeffs, wind=sc.wind_dict())


def knots(n, p, L):
    t = np.zeros(n + 2 * p + 1)
    _check(lib().oracle_knots(n, p, L, _p(t)), "knots")
    return t


def gauss(npts):
    x, w = np.zeros(npts), np.zeros(npts)
    _check(lib().oracle_gauss(npts, _p(x), _p(w)), "gauss")
    return x, w


def basis_eval(n, p, L, xs, deriv=0):
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    out = np.zeros((xs.size, n + p))
    _check(lib().oracle_basis_eval(n, p, L, deriv, _p(xs), xs.size, _p(out)), "basis_eval")
    return out


def band_to_dense(band: np.ndarray, p: int) -> np.ndarray:
    N = band.shape[0]
    A = np.zeros((N, N))
    for i in range(N):
        for k in range(max(0, i - p), min(N, i + p + 1)):
            A[i, k] = band[i, k - i + p]
    return A


def mat1d(n, p, L, kind):
    band = np.zeros((n + p, 2 * p + 1))
    _check(lib().oracle_mat1d(n, p, L, {"M": 0, "K": 1, "G": 2}.get(kind, kind), _p(band)),
           "mat1d")
    return band


def operator(desc: Desc, dir: int, which: int):
    n = desc.nel_y if dir else desc.nel_x
    band = np.zeros((n + desc.p, 2 * desc.p + 1))
    _check(lib().oracle_operator(ctypes.byref(desc), dir, which, _p(band)), "operator")
    return band


def line_solve(desc: Desc, dir: int, which: int, X: np.ndarray) -> np.ndarray:
    Y = np.array(X, dtype=np.float64, order="C", copy=True)
    _check(lib().oracle_line_solve(ctypes.byref(desc), dir, which, _p(Y)), "line_solve")
    return Y


def assemble(desc: Desc, substep: int, T: np.ndarray, fuel: np.ndarray, with_fuel=False):
    T = np.ascontiguousarray(T, dtype=np.float64)
    fuel = np.ascontiguousarray(fuel, dtype=np.float64)
    R = np.zeros_like(T)
    RF = np.zeros_like(T) if with_fuel else None
    rc = lib().oracle_assemble(ctypes.byref(desc), substep, _p(T), _p(fuel), _p(R),
                               _p(RF) if with_fuel else None)
    _check(rc, "assemble")
    return (R, RF) if with_fuel else R


def step(desc: Desc, T: np.ndarray, fuel: np.ndarray):
    T = np.array(T, dtype=np.float64, order="C", copy=True)
    fuel = np.array(fuel, dtype=np.float64, order="C", copy=True)
    _check(lib().oracle_step(ctypes.byref(desc), _p(T), _p(fuel)), "step")
    return T, fuel


def step_forced(desc: Desc, T: np.ndarray, fuel: np.ndarray, src0: np.ndarray, src1=None):
    """One step with a source added to F, sampled at the quadrature points
    (arrays of shape (nel_x*(p+1), nel_y*(p+1)); src1 None for the explicit
    scheme)."""
    T = np.array(T, dtype=np.float64, order="C", copy=True)
    fuel = np.array(fuel, dtype=np.float64, order="C", copy=True)
    s0 = np.ascontiguousarray(src0, dtype=np.float64)
    s1 = None if src1 is None else np.ascontiguousarray(src1, dtype=np.float64)
    q = desc.p + 1
    for a in (s0, s1):
        if a is not None and a.shape != (desc.nel_x * q, desc.nel_y * q):
            raise ValueError(f"source shape {a.shape}")
    _check(lib().oracle_step_forced(ctypes.byref(desc), _p(T), _p(fuel), _p(s0),
                                    None if s1 is None else _p(s1)), "step_forced")
    return T, fuel


def quad_points(n: int, p: int, L: float) -> np.ndarray:
    """Gauss points of the n elements of [0, L], element by element."""
    x = np.zeros(n * (p + 1))
    _check(lib().oracle_quad_points(n, p, L, _p(x)), "quad_points")
    return x


def step_flagged(desc: Desc, T: np.ndarray, fuel: np.ndarray, dT: float, dF: float):
    """One step, plus a boolean (nel_x, nel_y) map of the elements where the
    ignition decision of some substep lies within (dT, dF) of its thresholds."""
    T = np.array(T, dtype=np.float64, order="C", copy=True)
    fuel = np.array(fuel, dtype=np.float64, order="C", copy=True)
    flags = np.zeros((desc.nel_x, desc.nel_y), dtype=np.uint8)
    _check(lib().oracle_step_flagged(ctypes.byref(desc), _p(T), _p(fuel), float(dT), float(dF),
                                     flags.ctypes.data_as(ctypes.c_void_p)), "step_flagged")
    return T, fuel, flags.astype(bool)


def run(desc: Desc, T: np.ndarray, fuel: np.ndarray, nsteps: int):
    T = np.array(T, dtype=np.float64, order="C", copy=True)
    fuel = np.array(fuel, dtype=np.float64, order="C", copy=True)
    _check(lib().oracle_run(ctypes.byref(desc), _p(T), _p(fuel), int(nsteps)), "run")
    return T, fuel


def eval_grid(desc: Desc, C: np.ndarray, xs, ys):
    C = np.ascontiguousarray(C, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    ys = np.ascontiguousarray(ys, dtype=np.float64)
    out = np.zeros((xs.size, ys.size))
    _check(lib().oracle_eval_grid(ctypes.byref(desc), _p(C), _p(xs), xs.size, _p(ys),
                                  ys.size, _p(out)), "eval_grid")
    return out


def burned_fraction(desc: Desc, fuel: np.ndarray, thr: float = 0.1) -> float:
    fuel = np.ascontiguousarray(fuel, dtype=np.float64)
    return float(lib().oracle_burned_fraction(ctypes.byref(desc), _p(fuel), thr))


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())
