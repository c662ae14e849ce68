"""Forced steps (iga_step_forced) and the order study of Section 6.1 on the GPU.

- The plan's Gauss points equal the oracle's; forced steps match the oracle
  per step (FP64 1e-12, FP32 + refinement 1e-6) for random sources on ragged
  meshes and for the manufactured source, in all three schemes, p = 1, 2, 3.
- The order study's GPU runs (50^2, p = 2, full reading) reproduce the
  oracle's errors at t = 1 and its stability pattern (dt = 1/4 diverges for
  every scheme; dt = 1/16 is stable for PR and Strang; dt = 1/64 for all).
- Argument errors of the forced step.
"""
import numpy as np
import pytest

import oracle
import parity_util as pu
from paper_2604_19370_amd import iga, inputs, study

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_srcs(scheme, s0, s1):
    return (s0, None) if scheme == "explicit" else (s0, s1)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("scheme", ["pr", "strang", "explicit"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_forced_steps_random_source(p, scheme, precision):
    sc = inputs.small_case(60 + p, 37, 29 + p, p, scheme, dt=2e-3)
    print(f"forced {sc.name} {precision}", flush=True)
    pl = iga.Plan.from_scenario(sc, precision=precision)
    pl.factor()
    od = oracle.desc_from_scenario(sc)
    xq, yq = pl.quadrature_points(0), pl.quadrature_points(1)
    np.testing.assert_allclose(xq, oracle.quad_points(sc.nel_x, p, sc.len_x), rtol=0, atol=1e-13)
    np.testing.assert_allclose(yq, oracle.quad_points(sc.nel_y, p, sc.len_y), rtol=0, atol=1e-13)
    rng = np.random.default_rng(7 * p)
    tol = 1e-12 if precision == "fp64" else 1e-6
    Th, Fh = sc.T0, sc.fuel0    # the oracle's trajectory; each GPU step starts from it
    for k in range(3):
        s0 = rng.normal(0.0, 500.0, (xq.size, yq.size))
        s1 = rng.normal(0.0, 500.0, (xq.size, yq.size))
        if precision == "fp32":
            s0, s1 = s0.astype(np.float32).astype(np.float64), s1.astype(np.float32).astype(np.float64)
        Tp, Fp = (pu.f32(Th), pu.f32(Fh)) if precision == "fp32" else (Th, Fh)
        T, F = dev(Tp, pl.dtype), dev(Fp, pl.dtype)
        pl.step_forced(T, F, dev(s0, pl.dtype), None if scheme == "explicit" else dev(s1, pl.dtype))
        To, Fo = oracle.step_forced(od, Tp, Fp, *oracle_srcs(scheme, s0, s1))
        eT, eF = rel(host(T), To), rel(host(F), Fo)
        assert eT < tol and eF < tol, (k, eT, eF)
        Th, Fh = oracle.step_forced(od, Th, Fh, *oracle_srcs(scheme, s0, s1))
    pl.close()


@pytest.mark.parametrize("scheme", ["pr", "strang", "explicit"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_forced_steps_manufactured_source(scheme, precision):
    co = oracle.default_coeffs()
    sc, m = inputs.manufactured(co, 40, 2, scheme, 1 / 64, bx=1.0, by=-0.5)
    print(f"manufactured {sc.name} {precision}", flush=True)
    pl = iga.Plan.from_scenario(sc, precision=precision, coeffs=co)
    pl.factor()
    od = oracle.desc_from_scenario(sc, coeffs=co)
    X, Y = pl.quadrature_points(0)[:, None], pl.quadrature_points(1)[None, :]
    tol = 1e-12 if precision == "fp64" else 1e-6
    Th, Fh = sc.T0, sc.fuel0    # the oracle's trajectory; each GPU step starts from it
    for n in range(4):
        t = n * sc.dt
        s0, s1 = m.source(X, Y, t), m.source(X, Y, t + 0.5 * sc.dt)
        if precision == "fp32":
            s0, s1 = s0.astype(np.float32).astype(np.float64), s1.astype(np.float32).astype(np.float64)
        Tp, Fp = (pu.f32(Th), pu.f32(Fh)) if precision == "fp32" else (Th, Fh)
        T, F = dev(Tp, pl.dtype), dev(Fp, pl.dtype)
        pl.step_forced(T, F, dev(s0, pl.dtype), None if scheme == "explicit" else dev(s1, pl.dtype))
        To, _ = oracle.step_forced(od, Tp, Fp, *oracle_srcs(scheme, s0, s1))
        assert rel(host(T), To) < tol, n
        assert np.all(host(F) == 0.0)
        Th, Fh = oracle.step_forced(od, Th, Fh, *oracle_srcs(scheme, s0, s1))
    pl.close()


def oracle_error(nel, scheme, dt, coeffs, p=2):
    sc, m = inputs.manufactured(coeffs, nel, p, scheme, dt)
    d = oracle.make_desc(nel, nel, p, 100.0, 100.0, dt, scheme, coeffs=coeffs)
    xq = oracle.quad_points(nel, p, 100.0)
    X, Y = xq[:, None], xq[None, :]
    T, F = sc.T0.copy(), sc.fuel0.copy()
    for n in range(sc.steps):
        t = n * dt
        T, F = oracle.step_forced(d, T, F, *oracle_srcs(scheme, m.source(X, Y, t),
                                                         m.source(X, Y, t + 0.5 * dt)))
        if not np.isfinite(T).all():
            return None
    V = oracle.eval_grid(d, T, study.GRID, study.GRID)
    E = m.exact(study.GRID[:, None], study.GRID[None, :], sc.steps * dt)
    e = float(np.linalg.norm(V - E) / np.linalg.norm(E))
    return e if e <= 1.0 else None


@pytest.mark.parametrize("scheme", ["explicit", "pr", "strang"])
def test_order_study_matches_oracle(scheme):
    co = study.reading_coeffs("full")
    for dt in (1 / 4, 1 / 16, 1 / 64):
        e_gpu, _ = study.run_case(50, 2, scheme, dt, co)
        e_orc = oracle_error(50, scheme, dt, co)
        print(f"{scheme} dt={dt:g}: gpu {e_gpu} oracle {e_orc}", flush=True)
        assert (e_gpu is None) == (e_orc is None)
        if e_orc is not None:
            assert abs(e_gpu - e_orc) < 1e-9 * max(e_orc, 1e-3)
    assert study.run_case(50, 2, scheme, 1 / 4, co)[0] is None
    assert study.run_case(50, 2, scheme, 1 / 64, co)[0] < 2e-3
    if scheme != "explicit":
        assert study.run_case(50, 2, scheme, 1 / 16, co)[0] is not None
    e32, _ = study.run_case(50, 2, scheme, 1 / 64, co, precision="fp32")
    e64, _ = study.run_case(50, 2, scheme, 1 / 64, co)
    assert abs(e32 - e64) < 1e-5, (e32, e64)


def test_forced_step_argument_errors():
    sc = inputs.small_case(3, 20, 20, 2, "explicit")
    pl = iga.Plan.from_scenario(sc)
    pl.factor()
    q = 3
    T, F = dev(sc.T0, torch.float64), dev(sc.fuel0, torch.float64)
    s = torch.zeros(20 * q, 20 * q, dtype=torch.float64, device="cuda")
    with pytest.raises(iga.IgaError) as e:
        pl.step_forced(T, F, s, s.clone())     # explicit plans take one source
    assert e.value.status == iga.EINVAL
    with pytest.raises(ValueError):
        pl.step_forced(T, F, s[:, :-1].contiguous())
    pl.close()
    sc = inputs.small_case(3, 20, 20, 2, "pr")
    pl = iga.Plan.from_scenario(sc)
    pl.factor()
    with pytest.raises(iga.IgaError) as e:
        pl.step_forced(T, F, s)                # PR needs both sources
    assert e.value.status == iga.EINVAL
    pl.close()
