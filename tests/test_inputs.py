"""The case generators reproduce every parameter value the paper prints
(golden fixture tests/golden/paper_parameters.json, each entry cited), and
the generated initial fields have the stated shapes and symmetries."""
import json
import os

import numpy as np
import pytest

from paper_2101_06769_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def test_rti2d_parameter_mapping_matches_printed_values():
    d = GOLDEN["rti2d"]
    for c in d["cases"]:
        g, nu = inputs.rti_parameters(d["L"], c["Re"])
        assert abs(g - d["g"]) / d["g"] < 1e-12
        assert abs(nu - c["nu"]) < 5e-5  # printed to 4 decimals
    assert abs(inputs.atwood_to_rho_light(d["At"]) - 1 / 3) < 1e-15


def test_rti3d_parameter_mapping_matches_printed_values():
    d = GOLDEN["rti3d"]
    g, nu = inputs.rti_parameters(d["L"], d["Re"])
    assert abs(g - d["g"]) / d["g"] < 1e-12
    assert abs(nu - d["nu"]) < 5e-7


def test_impact_parameter_matches_printed_values():
    # the paper prints K to one decimal (55.78 appears as 55.7, 263.76 as 263.8)
    for c in GOLDEN["splash2d"]["cases"]:
        assert abs(inputs.impact_parameter(c["We"], c["Re"]) - c["K"]) < 0.1


def test_rti3d_headline_case_shape_and_parameters():
    case = inputs.rti3d(nx=16, ny=16, nz=64, amp=0.05 * 16)
    assert case.phi.shape == (64, 16, 16)
    p = case.params
    assert p["bc"] == (0, 0, 1) and p["g"][2] < 0 and p["rho_l"] == pytest.approx(1 / 3)
    # heavy fluid (phi -> 1) on top, light below
    assert case.phi[-1].min() > 0.999 and case.phi[0].max() < 1e-3
    # hydrostatic initial pressure: dp/dz = rho g_z in the bulk
    rho = p["rho_l"] + (p["rho_h"] - p["rho_l"]) * case.phi
    dp = np.diff(case.p, axis=0)
    assert np.allclose(dp[2:20], 0.5 * (rho[3:21] + rho[2:20]) * p["g"][2])


def test_splash3d_uses_liquid_density_weber_number():
    case = inputs.splash3d(nx=48, ny=48, nz=48, D=24.0)
    p = case.params
    assert p["rho_l"] == pytest.approx(1e-3)
    assert p["nu_l"] / p["nu_h"] == pytest.approx(15.0)
    assert p["sigma"] == pytest.approx(1.0 * 24.0 * 0.05 ** 2 / 8000.0)
    assert case.u[2].min() == pytest.approx(-0.05, rel=1e-4)


def test_batch_generator_is_seeded_and_uneven():
    a = inputs.batch_rti3d(count=6, seed=0, edges=(8, 12), steps=10)
    b = inputs.batch_rti3d(count=6, seed=0, edges=(8, 12), steps=10)
    assert [c.params["n"] for c in a] == [c.params["n"] for c in b]
    assert all(np.array_equal(x.phi, y.phi) for x, y in zip(a, b))
    for c in a:
        nx, ny, nz = c.params["n"]
        assert nz == 4 * nx and nx == ny
        assert 0.1 <= c.meta["At"] <= 0.9 and 100 <= c.meta["Re"] <= 3000


def test_serving_spec_is_seeded_and_within_ranges():
    a = inputs.serving_spec(seed=1, count=400)
    b = inputs.serving_spec(seed=1, count=400)
    assert a == b
    arr = np.array([s["arrival"] for s in a])
    assert np.all(np.diff(arr) > 0)
    # Poisson at 20/s: mean gap 0.05 s
    assert abs(np.diff(arr).mean() - 0.05) < 0.01
    for s in a:
        assert 64 <= s["edge"] <= 1024 and 500 <= s["steps"] <= 20000
        assert 3.0 <= s["rho_ratio"] <= 1000.0
        assert s["kind"] in ("rti", "static_drop", "impacting_drop")
    kinds = {k: sum(s["kind"] == k for s in a) for k in ("rti", "static_drop", "impacting_drop")}
    assert min(kinds.values()) > 100
    # each kind builds a 2-D case of the requested size and density ratio
    for kind in kinds:
        s = next(x for x in a if x["kind"] == kind and x["edge"] < 128)
        c = inputs.serving_case(s)
        assert c.params["dim"] == 2 and c.params["n"] == (s["edge"], s["edge"], 1)
        assert abs(c.params["rho_h"] / c.params["rho_l"] - s["rho_ratio"]) < 1e-9 * s["rho_ratio"]
        assert 0.0 <= c.phi.min() and c.phi.max() <= 1.0


def test_splash2d_is_mirror_symmetric_with_the_paper_parameters():
    c = inputs.splash2d(D=40.0, Re=1000.0, We=2200.0)
    assert c.params["bc"] == (inputs.BC_SYMMETRY, inputs.BC_WALL, inputs.BC_PERIODIC)
    assert c.params["n"] == (320, 160, 1)
    # density ratio 1000 and viscosity ratio 15 (Sec. 3.4)
    assert abs(c.params["rho_h"] / c.params["rho_l"] - 1000.0) < 1e-9
    assert abs(c.params["nu_l"] / c.params["nu_h"] - 15.0) < 1e-12
    # Re = rho_h U0 D / mu_h, We = rho_liquid D U0^2 / sigma, K = We^1/2 Re^1/4
    assert abs(0.05 * 40.0 / c.params["nu_h"] - 1000.0) < 1e-9
    assert abs(40.0 * 0.05 ** 2 / c.params["sigma"] - 2200.0) < 1e-9
    assert abs(c.meta["K"] - 2200.0 ** 0.5 * 1000.0 ** 0.25) < 1e-9
    # mirror symmetry about the box axis, for phi and u_y; u_x = 0
    assert np.array_equal(c.phi[0], c.phi[0][:, ::-1])
    assert np.array_equal(c.u[1, 0], c.u[1, 0][:, ::-1]) and not c.u[0].any()
