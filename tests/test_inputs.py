"""Seeded input generators: determinism, ranges and the structure the workloads ask for."""
import numpy as np
import pytest

from paper_2604_19370_amd import inputs


def test_greville_uniform_open():
    g = inputs.greville(4, 2)
    np.testing.assert_allclose(g, [0.0, 0.125, 0.375, 0.625, 0.875, 1.0])
    assert inputs.greville(64, 3).size == 67


def test_plain_pr_64_deterministic_and_ranges():
    a, b = inputs.plain_pr_64(0), inputs.plain_pr_64(0)
    np.testing.assert_array_equal(a.T0, b.T0)
    np.testing.assert_array_equal(a.fuel0, b.fuel0)
    assert a.T0.shape == (66, 66) and a.ndof == 4356
    assert 0.5 <= a.fuel0.min() and a.fuel0.max() <= 1.0
    assert a.T0.min() == pytest.approx(300.0, abs=1e-6)
    assert 850.0 < a.T0.max() <= 900.0
    cx, cy = a.ignitions[0]
    assert 0.3 <= cx <= 0.7 and 0.3 <= cy <= 0.7
    assert not np.array_equal(inputs.plain_pr_64(1).fuel0, a.fuel0)


def test_regional_fuel_map_structure():
    sc = inputs.regional_strang(seed=1, nel=256, steps=1)
    f = sc.fuel_raster
    assert f.shape == (256, 256)
    assert f.min() == 0.0 and f.max() <= 1.0
    zero_rows = np.where((f == 0).all(1))[0].size
    zero_cols = np.where((f == 0).all(0))[0].size
    assert zero_rows + zero_cols >= 4          # firebreak strips, 4 cells wide
    burnable = f[f > 0]
    assert 0.5 < burnable.mean() < 0.7
    assert len(sc.ignitions) == 3 and sc.wind.kind == "sincos"
    assert sc.wind.as_dict()["bbar_x"] == 1.0 and sc.wind.as_dict()["bbar_y"] == 0.0


def test_ensemble_members():
    ens = inputs.mixed_ensemble(8, sizes=(32, 48))
    assert len({m.nel_x for m in ens}) >= 1
    for m in ens:
        assert m.nel_x in (32, 48) and m.nel_x == m.nel_y
        assert 1 <= len(m.ignitions) <= 4
        assert np.hypot(m.wind.bx, m.wind.by) <= 3.0
        assert m.T0.shape == (m.nel_x + 2, m.nel_y + 2)
    c = inputs.cubic_ensemble(2, nel=32)
    assert c[0].p == 3 and c[0].T0.shape == (35, 35)
