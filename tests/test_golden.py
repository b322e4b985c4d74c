"""The production workloads against the numbers the paper prints for its
axisymmetric runs (tests/golden/production_case.json, cited there): domain,
resolution, time step and length, temperature, bunch size and charge in
plasma units, the benchmark's reading of the paper's run time, and the
device memory of this implementation beside the paper's. No GPU needed."""
import ctypes
import json
import math
import os

import pytest

from paper_2309_04872_amd import workloads

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "production_case.json")))

# CODATA 2018 (exact or recommended values)
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
EPS0 = 8.8541878128e-12
C = 299792458.0
MC2_KEV = 510.99895


@pytest.mark.parametrize("name", ["wake_axi_lec", "wake_axi_warmc"])
def test_grid_and_time_step(name):
    w = workloads.workload(name)
    g = GOLDEN
    assert w["geom"] == "axi" and w["dvel"] == 3.0
    assert w["delta"] == g["delta_kp"]
    assert w["nz"] == round(g["L_z_over_kp"] / g["delta_kp"]) and w["nx"] == round(g["L_r_over_kp"] / g["delta_kp"])
    assert math.isclose(w["dt"], g["dt_omega_p"], rel_tol=1e-12)
    assert w["steps"] == g["steps"] == round(g["t_end_omega_p"] / g["dt_omega_p"])
    assert w.get("tau_tilde", 0.53) == g["tau_over_dt_3d"]
    assert w["mu"] == g["mu_i"]


def test_temperature_in_kev():
    """mu_i = k_B T_i / (m c^2): 0.04 m c^2 = 20.4 keV, printed as 20 keV."""
    assert abs(GOLDEN["mu_i"] * MC2_KEV - GOLDEN["kT_keV"]) / GOLDEN["kT_keV"] < 0.025


@pytest.mark.parametrize("name", ["wake_axi_lec", "wake_axi_warmc"])
def test_bunch_in_plasma_units(name):
    """k_p = omega_p / c with omega_p^2 = e^2 n_i / (m eps0): 25 um at
    1e16 cm^-3 is 0.4704 / k_p; alpha from eq. Qtilde with D = 3."""
    n = GOLDEN["n_i_cm3"] * 1e6
    kp = math.sqrt(E_CHARGE ** 2 * n / (M_E * EPS0)) / C
    w = workloads.workload(name)
    assert math.isclose(kp * GOLDEN["sigma_z_um"] * 1e-6, w["sigma_z"], rel_tol=2e-4)
    assert math.isclose(kp * GOLDEN["sigma_r_um"] * 1e-6, w["sigma_x"], rel_tol=2e-4)
    q = (2 * math.pi) ** 1.5 * w["sigma_z"] * w["sigma_x"] ** 2 * w["alpha"]
    assert math.isclose(q, GOLDEN["q_tilde"], rel_tol=1e-12)


def test_paper_rate():
    """The benchmark's `paper_baseline`: nodes x steps over the printed run time."""
    import bench

    g = GOLDEN
    nodes = round(g["L_z_over_kp"] / g["delta_kp"]) * round(g["L_r_over_kp"] / g["delta_kp"])
    for name, minutes in (("wake_axi_lec", g["minutes_lec"]), ("wake_axi_warmc", g["minutes_warmc"])):
        assert math.isclose(bench.PAPER_MLUPS[name], nodes * g["steps"] / (minutes * 60) / 1e6, rel_tol=1e-12)


def test_memory_beside_the_paper():
    """Device workspace of one simulation of the production grid (FP64
    populations, both buffers, fields, lagged values, staging) against the
    memory the paper reports for its code: 0.9 and 2.3 GB here."""
    from paper_2309_04872_amd import _lib

    L = _lib.load()
    out = {}
    for name, closure, paper in (("wake_axi_lec", 0, GOLDEN["memory_gb_lec"]),
                                 ("wake_axi_warmc", 1, GOLDEN["memory_gb_warmc"])):
        w = workloads.workload(name)
        g = _lib.GridDesc()
        g.dims, g.nz, g.nx, g.delta, g.dt, g.tau_tilde = 2, w["nz"], w["nx"], w["delta"], w["dt"], 0.53
        g.closure, g.dvel, g.storage, g.bc_z, g.bc_x, g.geom = closure, 3.0, 0, 0, 0, 1
        nbytes = L.lbw_workspace_bytes(ctypes.byref(g))
        assert nbytes > 0
        out[name] = nbytes / 1e9
        assert nbytes / 1e9 < paper
    print(out)
