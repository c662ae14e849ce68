"""CPU checks of the comparison helpers the GPU parity tests rely on."""
import numpy as np
import pytest

import oracle
import parity_util as pu


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("axis", [0, 1])
def test_band_apply_equals_dense_product(p, axis):
    d = oracle.make_desc(9, 7, p, 9.0, 7.0, 1e-3, "strang")
    band = oracle.operator(d, axis, 0)
    A = oracle.band_to_dense(band, p)
    X = np.random.default_rng(p).normal(size=(9 + p, 7 + p))
    want = A @ X if axis == 0 else X @ A.T
    np.testing.assert_allclose(pu.band_apply(band, X, axis), want, atol=1e-13)


@pytest.mark.parametrize("scheme,substep", [("pr", 0), ("pr", 1), ("strang", 0), ("strang", 2),
                                            ("explicit", 0)])
def test_increment_rhs_matches_kronecker_form(scheme, substep):
    """R - A_impl T with A_impl = A^x (x) M^y (PR substep 1: M^x (x) A^y;
    explicit: M^x (x) M^y), and R_fuel - (M^x (x) M^y) fuel, against dense
    Kronecker products."""
    p, nx, ny = 2, 8, 6
    d = oracle.make_desc(nx, ny, p, 8.0, 6.0, 1e-3, scheme)
    rng = np.random.default_rng(1)
    T, F = rng.uniform(300, 900, (nx + p, ny + p)), rng.uniform(0, 1, (nx + p, ny + p))
    R, RF = rng.normal(size=T.shape), rng.normal(size=T.shape)
    ax, mx = (oracle.band_to_dense(oracle.operator(d, 0, w), p) for w in (0, 1))
    ay, my = (oracle.band_to_dense(oracle.operator(d, 1, w), p) for w in (0, 1))
    if scheme == "pr" and substep == 1:
        K = np.kron(mx, ay)
    elif scheme == "explicit":
        K = np.kron(mx, my)
    else:
        K = np.kron(ax, my)
    dR, dRF = pu.increment_rhs(d, substep, R, RF, T, F)
    np.testing.assert_allclose(dR, R - (K @ T.ravel()).reshape(T.shape), atol=1e-10)
    np.testing.assert_allclose(dRF, RF - (np.kron(mx, my) @ F.ravel()).reshape(F.shape), atol=1e-12)


def test_flip_report_localises_differences():
    rng = np.random.default_rng(2)
    ref = 300 + rng.uniform(0, 1, (200, 180))
    g = ref * (1 + 1e-7 * rng.standard_normal(ref.shape))
    r = pu.flip_report(g, ref)
    assert r["flipped"] == 0 and r["out_rel"] == pytest.approx(r["rel"])
    g2 = g.copy()
    g2[100, 90] += 40.0                      # one flipped dof
    r2 = pu.flip_report(g2, ref)
    assert r2["flipped"] == 1 and r2["max_abs"] == pytest.approx(40.0, rel=1e-6)
    assert r2["rel"] > 1e-4 and r2["out_rel"] < 2e-7
    assert r2["near_frac"] == pytest.approx((2 * pu.MASK_RADIUS + 1) ** 2 / ref.size)
    assert pu.points_radius(4096) == 1 and pu.points_radius(2048) == 2 and pu.points_radius(256) == 12


def test_near_mask_covers_the_elements_dofs_and_radius():
    flags = np.zeros((30, 20), dtype=bool)
    flags[10, 5] = True
    m = pu.near_mask(flags, 2, radius=1)
    # dofs 10..12 x 5..7, dilated by one
    assert m[9:14, 4:9].all() and m.sum() == 5 * 5


def test_shifted_desc_moves_only_the_thresholds():
    d = oracle.make_desc(8, 8, 2, 8.0, 8.0, 1e-3, "strang")
    s = pu.shifted_desc(d, 0.01, -1e-5)
    assert s.c.t_ig == d.c.t_ig + 0.01 and s.c.fuel_thr == d.c.fuel_thr - 1e-5
    assert s.c.c_ign == d.c.c_ign and s.dt == d.dt and d.c.t_ig == 800.0
