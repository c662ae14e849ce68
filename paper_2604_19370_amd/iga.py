"""ctypes binding of ``libiga.so`` (the C ABI declared in ``include/iga.h``).

Argument marshalling only: every step of the stepper runs in the HIP library.
The library is loaded on first use; if it is missing the call raises -- there
is no fallback.  PyTorch is used for device memory and streams: fields are
``torch.Tensor`` objects on a HIP device (float64 for FP64 plans, float32 for
FP32-with-refinement plans) of shape ``(Nx, Ny)``, C-contiguous.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiga.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EUNSUPPORTED, ESTATE = range(7)
PR, STRANG_CN, EXPLICIT = 0, 1, 2
FP64, FP32_REFINE = 0, 1
WIND_CONST, WIND_SINCOS = 0, 1

EXPORTED = ("iga_default_coeffs", "iga_plan_create", "iga_plan_destroy", "iga_plan_dims",
            "iga_factor_1d", "iga_assemble_rhs", "iga_line_solve", "iga_step", "iga_run",
            "iga_plan_schedule", "iga_plan_set_schedule", "iga_plan_set_assembly_rows",
            "iga_plan_assembly_rows", "iga_autotune", "iga_plan_set_window_schedule",
            "iga_plan_solver", "iga_ensemble_create", "iga_ensemble_destroy",
            "iga_ensemble_size", "iga_ensemble_launches", "iga_ensemble_step", "iga_ensemble_run",
            "iga_ensemble_set_schedule", "iga_ensemble_set_window_schedule",
            "iga_ensemble_set_assembly_rows", "iga_ensemble_autotune", "iga_step_forced",
            "iga_plan_quadrature_points", "iga_plan_set_column_schedule",
            "iga_plan_set_assembly_stacking", "iga_plan_assembly_stacking",
            "iga_ensemble_set_assembly_stacking", "iga_step_noalloc", "iga_sample_points",
            "iga_count_ambiguous", "iga_plan_set_window_buffers", "iga_plan_window_buffers",
            "iga_last_error")

_COEFF_NAMES = ("c_adv", "c_diff", "c_react", "c_nld", "c_ign", "t_ig", "fuel_thr", "t_act",
                "c_forcing", "c_rad", "fuel_rate")


class Coeffs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in _COEFF_NAMES]


class Wind(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("bx", ctypes.c_double), ("by", ctypes.c_double),
                ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("bbar_x", ctypes.c_double), ("bbar_y", ctypes.c_double)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("nel_x", ctypes.c_int32), ("nel_y", ctypes.c_int32), ("p", ctypes.c_int32),
                ("len_x", ctypes.c_double), ("len_y", ctypes.c_double), ("dt", ctypes.c_double),
                ("scheme", ctypes.c_int32), ("precision", ctypes.c_int32), ("c", Coeffs),
                ("wind", Wind), ("check_every", ctypes.c_int32)]


class IgaError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str):
        super().__init__(f"{what} failed (status {status}): {msg}")
        self.status = status


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load libiga.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2604_19370_amd.build`")
        # torch ships its own HIP runtime under the same soname as the system
        # one libiga.so is linked against.  Loaded after torch's, libiga.so
        # binds to it; loaded first, it would pull in the system copy and
        # torch would then load a second runtime that finds no GPU.  So torch
        # (which owns the device memory and streams passed in) loads first.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.iga_default_coeffs.argtypes = [ctypes.POINTER(Coeffs)]
        L.iga_default_coeffs.restype = None
        L.iga_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
        L.iga_plan_destroy.argtypes = [vp]
        L.iga_plan_dims.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
        L.iga_factor_1d.argtypes = [vp, vp]
        L.iga_assemble_rhs.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.iga_line_solve.argtypes = [vp, i32, i32, vp, vp]
        L.iga_step.argtypes = [vp, vp, vp, vp]
        L.iga_step_noalloc.argtypes = [vp, vp, vp, vp]
        L.iga_sample_points.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp]
        L.iga_count_ambiguous.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp]
        L.iga_run.argtypes = [vp, vp, vp, i64, vp]
        L.iga_plan_schedule.argtypes = [vp, i32] + [ctypes.POINTER(i32)] * 4
        L.iga_plan_set_schedule.argtypes = [vp, i32, i32, i32]
        L.iga_plan_set_assembly_rows.argtypes = [vp, i32]
        L.iga_plan_assembly_rows.argtypes = [vp]
        L.iga_plan_assembly_rows.restype = i32
        L.iga_autotune.argtypes = [vp, vp, vp, i32, vp]
        L.iga_plan_set_window_schedule.argtypes = [vp, i32, i32, i32]
        L.iga_plan_solver.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.iga_ensemble_set_window_schedule.argtypes = [vp, i32, i32, i32]
        pp = ctypes.POINTER(vp)
        L.iga_ensemble_create.argtypes = [ctypes.POINTER(PlanDesc), i32, ctypes.POINTER(vp)]
        L.iga_ensemble_destroy.argtypes = [vp]
        L.iga_ensemble_size.argtypes = [vp, ctypes.POINTER(i32)]
        L.iga_ensemble_launches.argtypes = [vp, ctypes.POINTER(i32)]
        L.iga_ensemble_step.argtypes = [vp, pp, pp, vp]
        L.iga_ensemble_run.argtypes = [vp, pp, pp, i64, vp]
        L.iga_ensemble_set_schedule.argtypes = [vp, i32, i32, i32]
        L.iga_ensemble_set_assembly_rows.argtypes = [vp, i32]
        L.iga_ensemble_autotune.argtypes = [vp, pp, pp, i32, vp]
        L.iga_step_forced.argtypes = [vp, vp, vp, vp, vp, vp]
        L.iga_plan_set_column_schedule.argtypes = [vp, i32]
        L.iga_plan_quadrature_points.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
        L.iga_plan_set_assembly_stacking.argtypes = [vp, i32]
        L.iga_plan_assembly_stacking.argtypes = [vp]
        L.iga_plan_assembly_stacking.restype = i32
        L.iga_ensemble_set_assembly_stacking.argtypes = [vp, i32]
        L.iga_plan_set_window_buffers.argtypes = [vp, i32, i32]
        L.iga_plan_window_buffers.argtypes = [vp, i32]
        L.iga_plan_window_buffers.restype = i32
        L.iga_last_error.argtypes = []
        L.iga_last_error.restype = ctypes.c_char_p
        for name in EXPORTED[1:-1]:
            if name not in ("iga_plan_assembly_rows", "iga_plan_assembly_stacking",
                            "iga_plan_window_buffers"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().iga_last_error().decode()


def _check(status: int, what: str):
    if status != OK:
        raise IgaError(status, what, last_error())


def default_coeffs() -> dict:
    c = Coeffs()
    lib().iga_default_coeffs(ctypes.byref(c))
    return {n: getattr(c, n) for n in _COEFF_NAMES}


def make_desc(nel_x, nel_y, p, len_x, len_y, dt, scheme, precision="fp64", wind=None,
              coeffs=None, check_every=0) -> PlanDesc:
    d = PlanDesc()
    d.nel_x, d.nel_y, d.p = int(nel_x), int(nel_y), int(p)
    d.len_x, d.len_y, d.dt = float(len_x), float(len_y), float(dt)
    d.scheme = {"pr": PR, "strang": STRANG_CN, "explicit": EXPLICIT}.get(scheme, scheme)
    d.precision = {"fp64": FP64, "fp32": FP32_REFINE, "fp32_refine": FP32_REFINE}.get(precision,
                                                                                      precision)
    co = default_coeffs()
    if coeffs:
        co.update(coeffs)
    for n in _COEFF_NAMES:
        setattr(d.c, n, float(co[n]))
    w = dict(kind="const", bx=0.0, by=0.0, ax=0.0, ay=0.0, bbar_x=None, bbar_y=None)
    if wind:
        w.update(wind)
    d.wind.kind = {"const": WIND_CONST, "sincos": WIND_SINCOS}.get(w["kind"], w["kind"])
    d.wind.bx, d.wind.by = float(w["bx"]), float(w["by"])
    d.wind.ax, d.wind.ay = float(w["ax"]), float(w["ay"])
    d.wind.bbar_x = float(w["bx"] if w["bbar_x"] is None else w["bbar_x"])
    d.wind.bbar_y = float(w["by"] if w["bbar_y"] is None else w["bbar_y"])
    d.check_every = int(check_every)
    return d


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Plan:
    """An iga_plan (knots, quadrature tables, factored 1D operators, scratch)."""

    def __init__(self, desc: PlanDesc):
        self.desc = desc
        h = ctypes.c_void_p()
        _check(lib().iga_plan_create(ctypes.byref(desc), ctypes.byref(h)), "iga_plan_create")
        self._h = h
        nx, ny, nd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().iga_plan_dims(h, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(nd)),
               "iga_plan_dims")
        self.Nx, self.Ny, self.ndof = nx.value, ny.value, nd.value
        self.fp32 = desc.precision == FP32_REFINE

    @classmethod
    def from_scenario(cls, sc, precision="fp64", coeffs=None, check_every=0) -> "Plan":
        return cls(make_desc(sc.nel_x, sc.nel_y, sc.p, sc.len_x, sc.len_y, sc.dt, sc.scheme,
                             precision=precision, wind=sc.wind_dict(), coeffs=coeffs,
                             check_every=check_every))

    @property
    def handle(self):
        return self._h

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.fp32 else torch.float64

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().iga_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _field(self, t, name):
        if t.dtype != self.dtype or not t.is_contiguous() or tuple(t.shape) != (self.Nx, self.Ny):
            raise ValueError(f"{name}: expected contiguous {self.dtype} tensor of shape "
                             f"({self.Nx}, {self.Ny}), got {t.dtype} {tuple(t.shape)}")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be on the GPU")
        return _ptr(t)

    def factor(self, stream=None):
        _check(lib().iga_factor_1d(self._h, _stream(stream)), "iga_factor_1d")

    def assemble_rhs(self, substep, T, fuel, rhs_T, rhs_fuel=None, stream=None):
        _check(lib().iga_assemble_rhs(self._h, int(substep), self._field(T, "T"),
                                      self._field(fuel, "fuel"), self._field(rhs_T, "rhs_T"),
                                      self._field(rhs_fuel, "rhs_fuel") if rhs_fuel is not None
                                      else None, _stream(stream)), "iga_assemble_rhs")

    def line_solve(self, dir, which, x, stream=None):
        _check(lib().iga_line_solve(self._h, int(dir), int(which), self._field(x, "x"),
                                    _stream(stream)), "iga_line_solve")

    def step(self, T, fuel, stream=None):
        _check(lib().iga_step(self._h, self._field(T, "T"), self._field(fuel, "fuel"),
                              _stream(stream)), "iga_step")

    def step_noalloc(self, T, fuel, stream=None):
        _check(lib().iga_step_noalloc(self._h, self._field(T, "T"), self._field(fuel, "fuel"),
                                      _stream(stream)), "iga_step_noalloc")

    def sample_points(self, field, xs, ys, stream=None):
        """Spline values of `field` at the grid (xs[a], ys[b]) (physical
        coordinates, host sequences); returns a (len(xs), len(ys)) float64
        device tensor."""
        import torch
        x = torch.as_tensor(np.asarray(xs, dtype=np.float64)).cuda()
        y = torch.as_tensor(np.asarray(ys, dtype=np.float64)).cuda()
        out = torch.empty((x.numel(), y.numel()), dtype=torch.float64, device="cuda")
        _check(lib().iga_sample_points(self._h, self._field(field, "field"), _ptr(x), x.numel(),
                                       _ptr(y), y.numel(), _ptr(out), _stream(stream)),
               "iga_sample_points")
        return out

    def count_ambiguous(self, T, fuel, dT, dF, stream=None) -> int:
        """Quadrature points whose ignition decision lies within (dT, dF) of
        its thresholds (synchronises)."""
        import torch
        c = torch.empty(1, dtype=torch.int64, device="cuda")
        _check(lib().iga_count_ambiguous(self._h, self._field(T, "T"), self._field(fuel, "fuel"),
                                         float(dT), float(dF), _ptr(c), _stream(stream)),
               "iga_count_ambiguous")
        return int(c.item())

    def run(self, T, fuel, nsteps, stream=None):
        _check(lib().iga_run(self._h, self._field(T, "T"), self._field(fuel, "fuel"),
                             int(nsteps), _stream(stream)), "iga_run")

    def quadrature_points(self, dir):
        """Gauss points of direction dir, element by element (numpy float64)."""
        import numpy as np
        n = (self.desc.nel_y if dir else self.desc.nel_x) * (self.desc.p + 1)
        x = np.zeros(n)
        _check(lib().iga_plan_quadrature_points(
            self._h, int(dir), x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
            "iga_plan_quadrature_points")
        return x

    def _source(self, t, name):
        q = self.desc.p + 1
        shape = (self.desc.nel_x * q, self.desc.nel_y * q)
        if t.dtype != self.dtype or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"{name}: expected contiguous {self.dtype} tensor of shape {shape}, "
                             f"got {t.dtype} {tuple(t.shape)}")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be on the GPU")
        return _ptr(t)

    def step_forced(self, T, fuel, src0, src1=None, stream=None):
        """One step with sources sampled at the quadrature points added to F
        (src1 None for the explicit scheme)."""
        _check(lib().iga_step_forced(self._h, self._field(T, "T"), self._field(fuel, "fuel"),
                                     self._source(src0, "src0"),
                                     None if src1 is None else self._source(src1, "src1"),
                                     _stream(stream)), "iga_step_forced")

    def schedule(self, dir):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().iga_plan_schedule(self._h, int(dir), *[ctypes.byref(x) for x in v]),
               "iga_plan_schedule")
        return dict(lines=v[0].value, waves_per_line=v[1].value, rows_per_lane=v[2].value,
                    table_rows=v[3].value)

    @property
    def assembly_rows(self) -> int:
        return int(lib().iga_plan_assembly_rows(self._h))

    def autotune(self, T, fuel, reps=20, stream=None):
        _check(lib().iga_autotune(self._h, self._field(T, "T"), self._field(fuel, "fuel"),
                                  int(reps), _stream(stream)), "iga_autotune")

    def set_schedule(self, dir, lines, waves_per_line=0):
        _check(lib().iga_plan_set_schedule(self._h, int(dir), int(lines), int(waves_per_line)),
               "iga_plan_set_schedule")

    def set_assembly_rows(self, rows):
        _check(lib().iga_plan_set_assembly_rows(self._h, int(rows)), "iga_plan_set_assembly_rows")

    @property
    def assembly_stacked(self) -> bool:
        return bool(lib().iga_plan_assembly_stacking(self._h))

    def set_assembly_stacking(self, stacked):
        _check(lib().iga_plan_set_assembly_stacking(self._h, int(stacked)),
               "iga_plan_set_assembly_stacking")

    def set_window_schedule(self, dir, lines, rows_per_lane=0):
        _check(lib().iga_plan_set_window_schedule(self._h, int(dir), int(lines), int(rows_per_lane)),
               "iga_plan_set_window_schedule")

    def set_window_buffers(self, dir, buffers):
        """LDS form of the windowed solves of `dir`: 0 automatic, 1 or 2 line buffers."""
        _check(lib().iga_plan_set_window_buffers(self._h, int(dir), int(buffers)),
               "iga_plan_set_window_buffers")

    def window_buffers(self, dir) -> int:
        """Line buffers of the windowed solves of `dir` in use (0: not windowed)."""
        return int(lib().iga_plan_window_buffers(self._h, int(dir)))

    def set_column_schedule(self, rows_per_chunk=0):
        _check(lib().iga_plan_set_column_schedule(self._h, int(rows_per_chunk)),
               "iga_plan_set_column_schedule")

    def solver(self, dir):
        w, h = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().iga_plan_solver(self._h, int(dir), ctypes.byref(w), ctypes.byref(h)),
               "iga_plan_solver")
        return dict(windowed=bool(w.value), warmup=h.value, column=w.value == 2)


class Ensemble:
    """An iga_ensemble: member plans stepped together by batched launches.

    ``descs`` is a list of PlanDesc (same degree and precision).  Fields are
    passed as lists of tensors, member m's of shape (Nx_m, Ny_m)."""

    def __init__(self, descs):
        n = len(descs)
        arr = (PlanDesc * n)(*descs)
        h = ctypes.c_void_p()
        _check(lib().iga_ensemble_create(arr, n, ctypes.byref(h)), "iga_ensemble_create")
        self._h = h
        self.descs = list(descs)
        self.shapes = [(d.nel_x + d.p, d.nel_y + d.p) for d in descs]
        self.fp32 = descs[0].precision == FP32_REFINE

    @classmethod
    def from_scenarios(cls, scs, precision="fp32", coeffs=None) -> "Ensemble":
        return cls([make_desc(sc.nel_x, sc.nel_y, sc.p, sc.len_x, sc.len_y, sc.dt, sc.scheme,
                              precision=precision, wind=sc.wind_dict(), coeffs=coeffs)
                    for sc in scs])

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.fp32 else torch.float64

    def __len__(self):
        return len(self.shapes)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().iga_ensemble_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fields(self, ts, name):
        if len(ts) != len(self.shapes):
            raise ValueError(f"{name}: expected {len(self.shapes)} tensors")
        for m, t in enumerate(ts):
            if t.dtype != self.dtype or not t.is_contiguous() or tuple(t.shape) != self.shapes[m]:
                raise ValueError(f"{name}[{m}]: expected contiguous {self.dtype} tensor of shape "
                                 f"{self.shapes[m]}, got {t.dtype} {tuple(t.shape)}")
            if t.device.type != "cuda":
                raise ValueError(f"{name}[{m}] must be on the GPU")
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    @property
    def launches_per_step(self) -> int:
        v = ctypes.c_int32()
        _check(lib().iga_ensemble_launches(self._h, ctypes.byref(v)), "iga_ensemble_launches")
        return v.value

    def step(self, Ts, Fs, stream=None):
        _check(lib().iga_ensemble_step(self._h, self._fields(Ts, "T"), self._fields(Fs, "fuel"),
                                       _stream(stream)), "iga_ensemble_step")

    def run(self, Ts, Fs, nsteps, stream=None):
        _check(lib().iga_ensemble_run(self._h, self._fields(Ts, "T"), self._fields(Fs, "fuel"),
                                      int(nsteps), _stream(stream)), "iga_ensemble_run")

    def set_schedule(self, dir, lines, waves_per_line=1):
        _check(lib().iga_ensemble_set_schedule(self._h, int(dir), int(lines), int(waves_per_line)),
               "iga_ensemble_set_schedule")

    def set_window_schedule(self, dir, lines, rows_per_lane=17):
        _check(lib().iga_ensemble_set_window_schedule(self._h, int(dir), int(lines),
                                                      int(rows_per_lane)),
               "iga_ensemble_set_window_schedule")

    def set_assembly_rows(self, rows):
        _check(lib().iga_ensemble_set_assembly_rows(self._h, int(rows)),
               "iga_ensemble_set_assembly_rows")

    def set_assembly_stacking(self, stacked):
        _check(lib().iga_ensemble_set_assembly_stacking(self._h, int(stacked)),
               "iga_ensemble_set_assembly_stacking")

    def autotune(self, Ts, Fs, reps=10, stream=None):
        _check(lib().iga_ensemble_autotune(self._h, self._fields(Ts, "T"), self._fields(Fs, "fuel"),
                                           int(reps), _stream(stream)), "iga_ensemble_autotune")
