"""Stored oracle values (tests/golden/oracle_values.json, written by
tests/golden/make_golden.py from the oracle alone) still come out of the
oracle, and each equals its closed form: a guard against silent drift of the
oracle's arithmetic."""
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def stored():
    with open(os.path.join(HERE, "golden", "oracle_values.json")) as fh:
        return json.load(fh)


def test_golden_values_reproduce(stored):
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    fresh = {"force_newtonian_two_body": mg.force_cases(), "lattice_most_bound": mg.lattice_case(),
             "plane_wave_power": mg.plane_wave_case()}
    for a, b in zip(fresh["force_newtonian_two_body"], stored["force_newtonian_two_body"]):
        np.testing.assert_allclose(a["oracle_a0"], b["oracle_a0"], rtol=1e-13)
        assert a["pairs"] == b["pairs"] == 2
    assert fresh["lattice_most_bound"]["most_bound_position"] == stored["lattice_most_bound"]["most_bound_position"]
    assert fresh["plane_wave_power"]["p_bin3"] == pytest.approx(stored["plane_wave_power"]["p_bin3"], rel=1e-12)


def test_golden_values_equal_their_closed_forms(stored):
    for c in stored["force_newtonian_two_body"]:
        np.testing.assert_allclose(c["oracle_a0"], c["closed_form_a0"], rtol=1e-12)
    lat = stored["lattice_most_bound"]
    assert lat["most_bound_position"] == lat["closed_form_position"]
    pw = stored["plane_wave_power"]
    assert pw["p_bin3"] == pytest.approx(pw["closed_form_p_bin3"], rel=1e-10)
