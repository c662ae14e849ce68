"""Host-side checks of the HIP C-ABI library (no GPU work is launched)."""
import ctypes
import os
import re

import pytest

from paper_2604_19370_amd import iga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "iga.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(iga_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "iga_step" in names and "iga_run" in names and len(names) >= 12
    L = iga.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(iga.EXPORTED) == set(names)


def test_default_coeffs_match_the_parameter_table():
    import oracle
    a, b = iga.default_coeffs(), oracle.default_coeffs()
    for k in b:
        assert a[k] == pytest.approx(b[k], rel=1e-14), k
    # T_amb is a fixed point of the loss terms
    assert abs(a["c_react"] * 300 + a["c_forcing"] - a["c_rad"] * 300 ** 4) < 1e-10


@pytest.mark.parametrize("field,value", [("p", 0), ("p", 4), ("nel_x", 4), ("nel_y", 2),
                                         ("dt", 0.0), ("dt", -1.0), ("len_x", 0.0),
                                         ("scheme", 7), ("precision", 3), ("check_every", -1)])
def test_plan_create_rejects_bad_descriptors(field, value):
    d = iga.make_desc(16, 16, 2, 16.0, 16.0, 1e-3, "pr")
    setattr(d, field, value)
    h = ctypes.c_void_p()
    st = iga.lib().iga_plan_create(ctypes.byref(d), ctypes.byref(h))
    assert st == iga.EINVAL
    assert h.value is None
    assert iga.last_error()


def test_null_arguments_are_rejected():
    L = iga.lib()
    assert L.iga_plan_create(None, None) == iga.EINVAL
    assert L.iga_step(None, None, None, None) == iga.EINVAL
    assert L.iga_run(None, None, None, 1, None) == iga.EINVAL
    assert L.iga_line_solve(None, 0, 0, None, None) == iga.EINVAL
    assert L.iga_assemble_rhs(None, 0, None, None, None, None, None) == iga.EINVAL
    assert L.iga_plan_destroy(None) == iga.OK
    assert L.iga_plan_set_window_buffers(None, 0, 0) == iga.EINVAL
    assert L.iga_plan_window_buffers(None, 0) == -1
    bad_wind = iga.make_desc(16, 16, 2, 16.0, 16.0, 1e-3, "pr")
    bad_wind.wind.kind = 5
    h = ctypes.c_void_p()
    assert L.iga_plan_create(ctypes.byref(bad_wind), ctypes.byref(h)) == iga.EINVAL


def test_ensemble_arguments_are_checked_before_any_device_work():
    L = iga.lib()
    h = ctypes.c_void_p()
    good = iga.make_desc(16, 16, 2, 16.0, 16.0, 1e-3, "pr")
    cubic = iga.make_desc(16, 16, 3, 16.0, 16.0, 1e-3, "pr")
    f32 = iga.make_desc(16, 16, 2, 16.0, 16.0, 1e-3, "pr", precision="fp32")
    bad = iga.make_desc(16, 16, 2, 16.0, -1.0, 1e-3, "pr")
    assert L.iga_ensemble_create(None, 1, ctypes.byref(h)) == iga.EINVAL
    assert L.iga_ensemble_create((iga.PlanDesc * 1)(good), 0, ctypes.byref(h)) == iga.EINVAL
    assert L.iga_ensemble_create((iga.PlanDesc * 1)(good), 1, None) == iga.EINVAL
    for other in (cubic, f32, bad):
        arr = (iga.PlanDesc * 2)(good, other)
        assert L.iga_ensemble_create(arr, 2, ctypes.byref(h)) == iga.EINVAL
        assert not h.value
    assert L.iga_ensemble_destroy(None) == iga.OK
    assert L.iga_ensemble_step(None, None, None, None) == iga.EINVAL
    assert L.iga_ensemble_run(None, None, None, 1, None) == iga.EINVAL
    assert L.iga_ensemble_autotune(None, None, None, 1, None) == iga.EINVAL
    assert L.iga_ensemble_set_schedule(None, 0, 1, 1) == iga.EINVAL
    assert L.iga_ensemble_set_assembly_rows(None, 4) == iga.EINVAL
    n = ctypes.c_int32()
    assert L.iga_ensemble_size(None, ctypes.byref(n)) == iga.EINVAL
    assert L.iga_ensemble_launches(None, ctypes.byref(n)) == iga.EINVAL


def test_one_hip_runtime_whatever_loads_first():
    """Loading the library before anything imports torch must not leave two
    HIP runtimes in the process (the second would find no GPU)."""
    import subprocess
    import sys
    code = ("from paper_2604_19370_amd import iga; iga.default_coeffs(); import torch; "
            "m = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
