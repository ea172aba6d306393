"""Pins against the values the paper prints (text fixtures in tests/golden/).

Table 2 (Sec. 4.1) is copied in three places: the oracle's fit module, the
seeded workload generator and the closed-form tests.  A slip in any copy (a
swapped pair of mechanisms, a wrong exponent) changes every attenuation pin
and every parity case built on it, so each copy is checked against the printed
table here, and the printed table is put through the oracle's dispersion
relation and held to the accuracy the paper states for its fits.
"""
import inspect

import numpy as np
import pytest

import workloads as W
from oracle import fit, physics, relaxation


def test_table2_fixture_is_whole_and_inside_its_bounds(golden):
    t = golden.table2()
    assert len(t) == 10
    for name, (opt, lo, hi) in t.items():
        assert lo <= opt <= hi, name
    # kappa is searched linearly, d and alpha over eight and seven decades
    assert {t[n][1:] for n in t if n.startswith("kappa")} == {(0.8, 1.2)}
    assert {t[n][1:] for n in t if n.startswith("d_")} == {(1e2, 1e10)}
    assert {t[n][1:] for n in t if n.startswith("alpha_")} == {(1e5, 1e12)}


def test_every_copy_of_table2_is_the_printed_one(golden):
    row = golden.table2_row()
    assert list(fit.TABLE2) == row
    assert list(W.TABLE2_ROW) == row
    t = golden.table2()
    assert fit.KAPPA_BOUNDS == t["kappa_x1"][1:]
    assert fit.D_BOUNDS == t["d_x1_nu1"][1:]
    assert fit.ALPHA_BOUNDS == t["alpha_x1_nu1"][1:]


def test_fit_weight_is_the_stated_one(golden):
    assert fit.W_ALPHA == golden.stated()["w_alpha"]


def test_printed_table2_meets_stated_accuracy_from_2_to_20_mhz(golden):
    """The printed three-digit Table 2 through Eq. dispersion_relations:
    attenuation within the stated 5 % of alpha_ref f^y and phase velocity
    within the stated 0.5 % of the Kramers-Kronig curve (anchored at the
    model's own 10 MHz velocity), from 2 MHz to the top of the stated band.
    At 1 MHz the rounding of the printed values leaves about -9 % of
    attenuation (recorded in the closed-form tests)."""
    s = golden.stated()
    row = np.array(golden.table2_row())
    f = np.linspace(2e6, s["band_high_hz"], 37)
    att, vel = relaxation.model_attenuation_velocity(f, 1540.0, row, 2)
    target = s["alpha_ref_db_cm_mhz"] * (f / 1e6) ** s["y_ref"]
    assert np.max(np.abs(att / target - 1)) < s["attenuation_rel_error_max"]
    v10 = relaxation.model_attenuation_velocity(np.array([10e6]), 1540.0, row, 2)[1][0]
    ct = physics.kk_phase_velocity(f, s["alpha_ref_db_cm_mhz"], s["y_ref"], v10, 10e6)
    assert np.max(np.abs(vel / ct - 1)) < s["phase_velocity_rel_error_max"]


def test_swapped_mechanisms_fail_the_stated_accuracy(golden):
    """Planted mistake: exchanging the two x1 mechanisms' alpha values (a
    plausible transcription slip) must break the 5 % attenuation bound."""
    s = golden.stated()
    row = np.array(golden.table2_row())
    row[6], row[7] = row[7], row[6]
    f = np.linspace(2e6, s["band_high_hz"], 37)
    att, _ = relaxation.model_attenuation_velocity(f, 1540.0, row, 2)
    target = s["alpha_ref_db_cm_mhz"] * (f / 1e6) ** s["y_ref"]
    assert np.max(np.abs(att / target - 1)) > s["attenuation_rel_error_max"]


@pytest.mark.parametrize("gen", [W.homogeneous, W.plain_2d, W.abdominal_2d, W.skull_3d])
def test_workloads_default_to_stated_discretisation(golden, gen):
    """Sec. 3.4: every simulation of the paper runs at CFL 0.4 and 12 points
    per wavelength; the synthetic workloads default to the same."""
    s = golden.stated()
    p = inspect.signature(gen).parameters
    assert p["cfl"].default == s["cfl_simulations"]
    assert p["ppw"].default == s["ppw_simulations"]


def test_small_abdominal_workload_keeps_stated_cfl(golden):
    prob = W.abdominal_2d(nx=256, ny=128, n_steps=4)
    cfl = prob.dt * float(prob.c.max()) / prob.h
    assert cfl == pytest.approx(golden.stated()["cfl_simulations"], rel=1e-12)
