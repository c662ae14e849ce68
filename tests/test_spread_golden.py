"""The stored float32-spread data (tests/golden/fp32_spread.json) is what the
committed script computes from the oracle: its small case is recomputed here
and must match; the larger cases are checked for internal consistency."""
import importlib.util
import json
import os

import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_script():
    spec = importlib.util.spec_from_file_location("make_fp32_spread",
                                                  os.path.join(GOLD, "make_fp32_spread.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_small_case_reproduces():
    stored = json.load(open(os.path.join(GOLD, "fp32_spread.json")))["regional256"]
    got = load_script().CASES["regional256"]()
    for variant in ("round_each", "round_init"):
        a, b = got["ignition"][variant], stored["ignition"][variant]
        for key in ("rel_T", "rel_fuel", "rel_T_256", "max_abs_T", "burned_ref", "burned_var"):
            assert a[key] == pytest.approx(b[key], rel=1e-6, abs=1e-15), (variant, key)


def test_stored_cases_are_consistent():
    d = json.load(open(os.path.join(GOLD, "fp32_spread.json")))
    assert {"regional256", "regional1024", "regional4096", "mixed_members", "cubic20"} <= set(d)
    for case in d.values():
        for runs in case.values():
            for r in ([runs] if "steps" in runs else runs.values()):
                for v in r.values():
                    if not isinstance(v, dict) or "rel_T" not in v:
                        continue
                    # away from flipped dofs the spread is at most the whole-field one,
                    # and a run without flipped dofs has the two equal
                    assert v["rel_T_away_from_flips"] <= v["rel_T"] * (1 + 1e-12)
                    if v["flipped_dofs"] == 0:
                        assert v["rel_T_away_from_flips"] == pytest.approx(v["rel_T"])
                    assert v["max_abs_T"] > 0.5 or v["flipped_dofs"] == 0
    # rounding only the initial state moves the 1024^2 run far less than rounding every step
    r = d["regional1024"]["ignition"]
    assert r["round_init"]["rel_T"] < 0.05 * r["round_each"]["rel_T"]
