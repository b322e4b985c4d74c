"""Pins of the oracle's diagnostics (sum of n dV, field energy, kinetic
energy, max |u| / Lambda) against closed forms, and planted mistakes that
each pin must catch.

- Energy. A uniform cold plasma oscillation obeys p' = -E, E' = p / gamma
  (Sec. 3 / Sec. 4 equations with mu -> 0, Maxwell-Ampere of Sec. 5): the
  energy per volume gamma - 1 + E^2 / 2 is conserved. At t = 0 (E = 0) the
  kinetic sum is (gamma_0 - 1) times the volume exactly; the sum of the two
  diagnostics stays at that value to first order in dt (the explicit
  scheme's error), and the field part reaches it when u = 0.
- Field energy of the bunch's initial field (Sec. 5), a closed form in z
  times a one-dimensional integral over the transverse profile: slab
  E_x = B_y = -g(zeta) sigma_x sqrt(pi/2) erf(x / (sqrt 2 sigma_x)),
  axisymmetric E_r = B_phi = -g(zeta) sigma_r^2 (1 - e^{-r^2 / 2 sigma_r^2}) / r,
  with int g^2 dzeta = alpha^2 sigma_z sqrt(pi). Only the real Yee slots
  count: with open boundaries the field spans the nodes' extent.
- Axisymmetric volume weights (2 pi r per unit cell area, nodes at
  r_j = (j + 1/2) delta): the midpoint sum of a uniform column over nr rows is
  pi (nr delta)^2 L_z exactly.
"""
import numpy as np
import pytest
from scipy import integrate, special

@pytest.fixture(autouse=True)
def one_thread(oracle_mod):
    """These grids have a few nodes: one oracle thread avoids OpenMP start-up
    and oversubscription costs."""
    n = oracle_mod.num_threads()
    oracle_mod.set_threads(1)
    yield
    oracle_mod.set_threads(n)


def _cold_oscillation(oracle_mod, closure, dt, u0=0.8, t_end=10.0, library=None):
    """1D uniform oscillation at u0 on 4 periodic nodes (delta = 10 dt):
    diagnostics at t = 0 and the largest relative deviation of the field
    plus kinetic energy from (gamma_0 - 1) L over t_end."""
    d = 10 * dt
    o = oracle_mod.Oracle(1, 4, delta=d, dt=dt, closure=closure, dvel=1.0, mu=1e-9,
                          bc_z=oracle_mod.PERIODIC, library=library)
    o.init(uz=u0)
    L = 4 * d
    g0 = 1 / np.sqrt(1 - u0 * u0)
    d0 = o.diagnostics()
    dev, fe_max = 0.0, 0.0
    for _ in range(int(t_end / dt) // 10):
        dg = o.diagnostics()
        dev = max(dev, abs((dg[1] + dg[2]) / L - (g0 - 1)) / (g0 - 1))
        fe_max = max(fe_max, dg[1] / L)
        o.step(10)
    return d0, L, g0, dev, fe_max


@pytest.mark.parametrize("closure", [0, 1])
def test_diag_energy_cold_relativistic_1d(oracle_mod, closure):
    """Measured deviation of the energy from its initial value over about
    1.3 periods: LEC 1.6e-3, 8.2e-4, 4.1e-4 and WARMC 8.6e-3, 4.3e-3, 2.1e-3
    at dt = 0.004, 0.002, 0.001 (first order)."""
    u0 = 0.8
    d0, L, g0, _, _ = _cold_oscillation(oracle_mod, closure, 0.002, t_end=0.0)
    assert abs(d0[0] - L) <= 1e-14 * L  # sum n dV, n = 1
    assert d0[1] == 0.0  # no field yet
    assert abs(d0[2] - (g0 - 1) * L) <= 1e-13 * L
    assert abs(d0[4] - u0 / 10.0) <= 1e-15  # Lambda = delta / dt = 10
    devs = []
    for dt in (0.004, 0.002):
        _, _, _, dev, fe_max = _cold_oscillation(oracle_mod, closure, dt, u0)
        devs.append(dev)
        # at u = 0 the whole energy sits in the field
        assert abs(fe_max / (g0 - 1) - 1) <= 2 * dev + 1e-4
    assert devs[1] <= (2e-3 if closure == 0 else 1e-2)
    assert abs(devs[0] / devs[1] - 2.0) <= 0.1


@pytest.mark.parametrize("closure", [0, 1])
def test_diag_energy_uniform_2d_with_by(oracle_mod, closure):
    """2D uniform oscillation along z in a uniform B_y: u_z and u_x couple
    through u x B, E_z and E_x both carry energy, B_y stays uniform
    (curl E = 0). Field plus kinetic energy minus the constant magnetic part
    is conserved at first order in dt; at t = 0 the field energy is the
    magnetic energy B0^2 / 2 times the area exactly. Measured deviation:
    LEC 1.09e-2, 5.4e-3, 2.7e-3 and WARMC 1.44e-2, 7.2e-3, 3.6e-3 at
    dt = 0.004, 0.002, 0.001."""
    u0, B0 = 0.5, 0.7
    g0 = 1 / np.sqrt(1 - u0 * u0)
    devs = []
    for dt in (0.004, 0.002):
        d = 10 * dt
        o = oracle_mod.Oracle(2, 4, 4, delta=d, dt=dt, closure=closure, dvel=3.0, mu=1e-9,
                              bc_z=oracle_mod.PERIODIC, bc_x=oracle_mod.PERIODIC)
        o.init(uz=u0)
        o.set_yee("by", B0)
        area = 16 * d * d
        d0 = o.diagnostics()
        assert abs(d0[1] - 0.5 * B0 * B0 * area) <= 1e-14 * area
        assert abs(d0[2] - (g0 - 1) * area) <= 1e-13 * area
        dev, ex_seen = 0.0, 0.0
        for _ in range(int(8.0 / dt) // 10):
            dg = o.diagnostics()
            w = dg[1] - 0.5 * B0 * B0 * area + dg[2]
            dev = max(dev, abs(w / area - (g0 - 1)) / (g0 - 1))
            ex_seen = max(ex_seen, abs(o.get("ex_yee")[0, 0]))
            o.step(10)
        assert ex_seen > 0.1  # the x motion and its field are active
        devs.append(dev)
    assert devs[1] <= (7e-3 if closure == 0 else 9e-3)
    assert abs(devs[0] / devs[1] - 2.0) <= 0.1


def _slab_field_energy_error(oracle_mod, ndiv, library=None):
    d = 2 * np.pi / ndiv
    nz, nx = int(16.0 / d), int(6.0 / d)
    sz, sx, al = 1.0, 0.5, 1.0
    o = oracle_mod.Oracle(2, nz, nx, delta=d, mu=1e-2, alpha=al, sigma_z=sz, sigma_x=sx, library=library)
    o.init()
    fe = o.diagnostics()[1]
    x0, x1 = -(nx - 1) / 2 * d, (nx - 1) / 2 * d
    fx = integrate.quad(lambda x: (sx * np.sqrt(np.pi / 2) * special.erf(x / (np.sqrt(2) * sx))) ** 2,
                        x0, x1, limit=200)[0]
    ref = 0.5 * (al * al * sz * np.sqrt(np.pi)) * fx * 2  # E_x and B_y
    return fe / ref - 1


def _axi_field_energy_error(oracle_mod, ndiv, library=None):
    d = 2 * np.pi / ndiv
    nz, nr = int(16.0 / d), int(6.0 / d)
    sz, sr, al = 1.0, 0.5, 1.0
    o = oracle_mod.Oracle(2, nz, nr, delta=d, mu=1e-2, alpha=al, sigma_z=sz, sigma_x=sr,
                          geom=oracle_mod.AXI, library=library)
    o.init()
    fe = o.diagnostics()[1]
    # E_r at r_{j+1/2} = (j + 1) delta for the real slots j <= nr - 2: the
    # midpoint rule over [delta / 2, (nr - 1/2) delta]
    fr = integrate.quad(lambda r: 2 * np.pi * r * (sr * sr * (-np.expm1(-r * r / (2 * sr * sr))) / r) ** 2,
                        0.5 * d, (nr - 0.5) * d, limit=200)[0]
    ref = 0.5 * (al * al * sz * np.sqrt(np.pi)) * fr * 2
    return fe / ref - 1


def test_diag_initial_field_energy_slab(oracle_mod):
    """Measured 1.8e-10 / 1.5e-11 at lambda_p / 32 and / 64 (Gaussian in z,
    erf^2 in x: the midpoint sums are nearly exact). Counting the ghost row
    too would add 4.3 % / 2.1 %."""
    for ndiv in (32, 64):
        assert abs(_slab_field_energy_error(oracle_mod, ndiv)) <= 1e-8


def test_diag_initial_field_energy_axi(oracle_mod):
    """Second order in delta: measured 9.3e-5, 9.8e-6, 1.6e-6 at
    lambda_p / 32, 64, 128."""
    e32 = _axi_field_energy_error(oracle_mod, 32)
    e64 = _axi_field_energy_error(oracle_mod, 64)
    assert abs(e64) <= 2e-5
    assert abs(e32 / e64) >= 4.0


def _axi_column(oracle_mod, uz=0.0, ur_slope=0.0, library=None):
    d = 2 * np.pi / 64
    nz, nr = 16, 40
    o = oracle_mod.Oracle(2, nz, nr, delta=d, mu=1e-2, geom=oracle_mod.AXI, bc_z=oracle_mod.PERIODIC,
                          library=library)
    r = (np.arange(nr) + 0.5) * d
    o.init(uz=uz, ux=np.repeat((ur_slope * r)[:, None], nz, 1), fields_from_driver=False)
    return o, np.pi * (nr * d) ** 2 * (nz * d), r[-1]


def test_diag_axi_column_sums(oracle_mod):
    """A uniform column: sum n dV = pi R^2 L_z and the kinetic energy
    (gamma - 1) pi R^2 L_z, both exact to rounding; max |u| / Lambda."""
    uz = 0.6
    o, V, _ = _axi_column(oracle_mod, uz=uz)
    dg = o.diagnostics()
    assert abs(dg[0] / V - 1) <= 1e-13
    assert abs(dg[2] / (V * (1 / np.sqrt(1 - uz * uz) - 1)) - 1) <= 1e-13
    assert abs(dg[4] - uz / 10.0) <= 1e-15


def test_diag_max_lattice_mach(oracle_mod):
    """u_r = eps r on a column: the largest |u| is eps r at the outermost
    node row; with u_z = 0.3 on top, |u| = sqrt(u_z^2 + u_r^2) there."""
    eps = 0.02
    o, _, rmax = _axi_column(oracle_mod, uz=0.3, ur_slope=eps)
    dg = o.diagnostics()
    assert abs(dg[4] - np.hypot(0.3, eps * rmax) / 10.0) <= 1e-15


# ---------------------------------------------------------------------------
# Planted mistakes: each pin above must fail when the diagnostic it covers is
# computed wrongly.

PLANTED = {
    "ghost_row_counted": [("int rx = s->p.bc_x == ORC_BC_PERIODIC || j < nx - 1;", "int rx = 1;")],
    "field_half_dropped": [("if (rx) fe += 0.5 * s->Ex[c] * s->Ex[c] * dVh;",
                            "if (rx) fe += s->Ex[c] * s->Ex[c] * dVh;")],
    "kinetic_gamma": [("ke += n * (g - 1.0) * dV;", "ke += n * g * dV;")],
    "half_slot_weight_at_node": [("const double dVh = axi ? 2.0 * M_PI * node_x(s, j + 0.5) * dV0 : dV0;",
                                  "const double dVh = axi ? 2.0 * M_PI * node_x(s, j) * dV0 : dV0;")],
    "mach_without_lambda": [("double um = sqrt(uz * uz + ux * ux) / Lam;", "double um = sqrt(uz * uz + ux * ux);")],
    "mach_z_only": [("double um = sqrt(uz * uz + ux * ux) / Lam;", "double um = fabs(uz) / Lam;")],
}


@pytest.fixture(scope="module")
def planted(oracle_mod):
    return {k: oracle_mod.variant(k, v) for k, v in PLANTED.items()}


def test_diag_planted_mistakes_fail(oracle_mod, planted):
    assert abs(_slab_field_energy_error(oracle_mod, 64, planted["ghost_row_counted"])) > 1e-2
    assert abs(_slab_field_energy_error(oracle_mod, 64, planted["field_half_dropped"])) > 0.3
    d0, L, g0, _, _ = _cold_oscillation(oracle_mod, 0, 0.002, t_end=0.0, library=planted["kinetic_gamma"])
    assert abs(d0[2] - (g0 - 1) * L) > 0.5 * L
    assert abs(_axi_field_energy_error(oracle_mod, 64, planted["half_slot_weight_at_node"])) > 1e-3
    for tag in ("mach_without_lambda", "mach_z_only"):
        o, _, rmax = _axi_column(oracle_mod, uz=0.3, ur_slope=0.02, library=planted[tag])
        assert abs(o.diagnostics()[4] - np.hypot(0.3, 0.02 * rmax) / 10.0) > 1e-4, tag
