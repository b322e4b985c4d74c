"""Pins of the oracle's axisymmetric (r, z) geometry (Sec. 2.2 and App. A:
cylindrical divergence moved into sources -u_r A / r, reflective axis) against
what the cylindrical equations fix (no GPU).

Layout: node row j sits at r_j = (j + 1/2) delta, E_r and B_phi at
r_{j+1/2} = (j + 1) delta, so the axis is the face below row 0 and E_r, B_phi
vanish there; the ghost row below the axis holds the mirror image of row 0.
"""
import numpy as np
import pytest
from scipy import integrate

LP = 2 * np.pi


def _axi(oracle_mod, nz, nr, ndiv, **kw):
    d = LP / ndiv
    kw.setdefault("dt", 0.1 * d)
    kw.setdefault("closure", oracle_mod.LEC)
    kw.setdefault("dvel", 3.0)
    return oracle_mod.Oracle(2, nz, nr, delta=d, geom=oracle_mod.AXI, **kw)


def test_axi_parameter_checks(oracle_mod):
    """The axisymmetric geometry is two-dimensional, local-equilibrium, with
    an open outer radius and the driver on the axis."""
    ok = dict(nz=16, nx=8, mu=1e-3)
    oracle_mod.Oracle(2, geom=oracle_mod.AXI, **ok)
    bad = [dict(closure=oracle_mod.WARMC), dict(bc_x=oracle_mod.PERIODIC), dict(x0=0.5)]
    for b in bad:
        with pytest.raises(Exception):
            oracle_mod.Oracle(2, geom=oracle_mod.AXI, **ok, **b)
    with pytest.raises(Exception):
        oracle_mod.Oracle(1, 16, 1, geom=oracle_mod.AXI, mu=1e-3)


def test_axi_rest_state(oracle_mod):
    """A uniform warm plasma at rest with no driver stays at rest: every
    cylindrical source carries a factor u_r, and the mirrored ghost of a
    uniform state at rest is that state."""
    o = _axi(oracle_mod, 24, 16, 64, mu=1e-2, tau_tilde=0.53, bc_z=oracle_mod.PERIODIC)
    o.init(fields_from_driver=False).step(200)
    assert np.abs(o.get("n") - 1).max() <= 1e-13
    for q in ("uz", "ux", "ez_yee", "ex_yee", "by_yee"):
        assert np.abs(o.get(q)).max() <= 1e-13, q


def _gauss_residual(o, alpha, sz, sr, z0, t):
    """max over interior nodes of |(1/r) d_r (r E_r) + d_z E_z - rho| / alpha
    with rho = 1 - n - n_b (the cylindrical Gauss law on the Yee grid)."""
    ez, er, n = o.get("ez_yee"), o.get("ex_yee"), o.get("n")
    nr, nz = n.shape
    d = o.params.delta
    j = np.arange(nr)[:, None]
    r = (j + 0.5) * d
    erm = np.vstack([np.zeros((1, nz)), er[:-1]])  # E_r at r_{j-1/2}; zero on the axis
    div = (ez - np.roll(ez, 1, axis=1)) / d + ((j + 1) * er - j * erm) / ((j + 0.5) * d)
    zeta = np.arange(nz) * d - z0 - t
    nb = alpha * np.exp(-zeta[None, :] ** 2 / (2 * sz * sz)) * np.exp(-r ** 2 / (2 * sr * sr))
    res = div - (1 - n - nb)
    return np.abs(res[: nr - 2, 2: nz - 2]).max() / alpha


def test_axi_gauss_law(oracle_mod):
    """Initial fields: the driver's transverse field E_r = B_phi solves the
    cylindrical Gauss law (1/r) d_r (r E_r) = -n_b; the discrete residual is
    second order in delta. In time the Yee update with the cylindrical curl
    (1/r) d_r (r B_phi) keeps Gauss's law up to the mismatch between the
    lattice Boltzmann continuity and the Yee current, first order in delta.
    A Cartesian curl in the E_z update leaves a residual of 0.6 alpha."""
    alpha, sz, sr, z0 = 1e-3, 0.5, 0.5, 3.0
    out = {}
    for ndiv in (64, 128):
        d = LP / ndiv
        steps = 200 * ndiv // 64
        nz = int((z0 + steps * 0.1 * d + 4 * sz) / d) + 8
        o = _axi(oracle_mod, nz, int(4.0 / d), ndiv, mu=1e-6, alpha=alpha, sigma_z=sz,
                 sigma_x=sr, z0=z0, tau_tilde=0.51).init()
        r0 = _gauss_residual(o, alpha, sz, sr, z0, 0.0)
        o.step(steps)
        r1 = _gauss_residual(o, alpha, sz, sr, z0, steps * 0.1 * d)
        out[ndiv] = (r0, r1)
    assert out[64][0] <= 6e-3 and out[128][0] <= 0.3 * out[64][0], out
    assert out[64][1] <= 2e-2 and out[128][1] <= 0.75 * out[64][1], out


def _cold_wake_n(zeta, alpha, sz):
    """Linear cold plasma density behind a Gaussian bunch moving at c:
    (d_zeta^2 + 1) n_1 = -n_b (App. B at mu = 0)."""
    nb = lambda zp: alpha * np.exp(-zp ** 2 / (2 * sz ** 2))
    return np.array([-integrate.quad(lambda zp: nb(zp) * np.sin(zp - ze), max(ze, -9 * sz), 9 * sz)[0]
                     for ze in zeta])


def _wake_ratio(oracle_mod, ndiv, js, tau=0.51, alpha=1e-3, sz=0.5, sr=0.5, T=20.0):
    d = LP / ndiv
    dt = 0.1 * d
    steps = int(round(T / dt))
    z0 = 6 * sz
    nz = int((z0 + steps * dt + 4 * sz) / d) + 8
    o = _axi(oracle_mod, nz, int(5.0 / d) + 4, ndiv, dt=dt, tau_tilde=tau, mu=1e-6, alpha=alpha,
             sigma_z=sz, sigma_x=sr, z0=z0)
    o.init().step(steps)
    zeta = np.arange(nz) * d - (z0 + steps * dt)
    m = (zeta < -3 * sz) & (zeta > -3 * sz - 2 * LP)
    age = np.abs(zeta[m])
    kappa = (100 / 3) * (tau - 0.5) * dt  # eq. diff-coeff, Delta / Delta t = 10
    se2 = sr * sr + kappa * age
    base = _cold_wake_n(zeta[m], alpha, sz) * np.exp(-0.5 * kappa * age) * np.sqrt(sr * sr / se2)
    n = o.get("n")
    out = []
    for j in js:
        r = (j + 0.5) * d
        th = base * np.exp(-r * r / (2 * se2))
        a = n[j][m] - 1
        out.append(float(np.dot(a, th) / np.dot(th, th)))
    return np.array(out)


@pytest.mark.slow
def test_axi_cold_density_wake(oracle_mod):
    """Linear cold wake of a Gaussian bunch (sigma_z = sigma_r = 0.5): the
    density obeys a local oscillator, (d_zeta^2 + 1) n_1(r, zeta) =
    -n_b(r, zeta) (App. B with mu = 0: c_s = 0, a_e = a_b = 1), so
    n_1 / g_perp(r) is the 1D wake at every radius. The lattice adds the
    numerical diffusion kappa of eq. diff-coeff, which damps the wave by
    exp(-kappa |zeta| / 2) (as in 1D) and widens the transverse Gaussian to
    sigma^2 + kappa |zeta|. The fitted amplitude ratio at r = 0, 0.5 and 1
    approaches 1 at first order in delta; its Richardson extrapolation from
    delta = lambda_p / 64 and / 128 is 1 within 1.5 %. A plain copy of the
    populations into the ghost row for the density (mass through the axis)
    gives 1.27 and 1.49 on the axis and fails this."""
    r64 = _wake_ratio(oracle_mod, 64, (0, 5, 10))
    r128 = _wake_ratio(oracle_mod, 128, (0, 10, 20))
    extrap = 2 * r128 - r64
    assert np.all(np.abs(1 - r128) < np.abs(1 - r64)), (r64, r128)
    assert np.all(np.abs(1 - r128) <= 0.03), r128
    assert np.all(np.abs(extrap - 1) <= 0.015), (r64, r128, extrap)


def _breathing_ode(eps, U, T):
    """Cold non-relativistic uniform breathing of a plasma column: n(t)
    uniform, u_r = a(t) r, E_r = b(t) r, plus a uniform axial oscillation
    u_z(t), E_z(t). The cylindrical continuity, radial and axial momentum,
    Gauss and Ampere laws reduce to
      n' = -2 a n,  a' = -a^2 - b,  b' = n a,  u_z' = -E_z,  E_z' = n u_z.
    The a^2 comes from the -u_r A_r / r source (without it a' = -b), and the
    axial equation is free of a u_z only with the -u_r A_z / r source."""
    from scipy.integrate import solve_ivp

    f = lambda t, y: [-2 * y[1] * y[0], -y[1] ** 2 - y[2], y[0] * y[1], -y[4], y[0] * y[3]]
    s = solve_ivp(f, (0, T), [1.0, eps, 0.0, U, 0.0], rtol=1e-12, atol=1e-14)
    return s.y[:, -1]


def test_axi_breathing_mode(oracle_mod):
    """Nonlinear check of the three cylindrical sources. The column is run
    with initial u_r = +-eps r (eps = 0.02) and u_z = U = 0.02, out to
    t = 1.5, on r < 8 with the outer boundary out of causal reach of r < 2.
    Relativistic corrections are odd in eps at the order kept, so the part
    of n and u_r / r that is even in eps is the second-order response of the
    non-relativistic equations, and the part of u_z that is odd in eps is
    the eps U coupling. Measured (delta = 0.05): 1 % and 0.05 %; a dropped or
    sign-flipped A_r source moves the even parts by a factor 2 or more, a
    dropped A_z source moves the odd u_z part by 60 %."""
    d, R, T, eps, U = 0.05, 8.0, 1.5, 0.02, 0.02
    nr, nz = int(R / d), 4
    steps = int(round(T / (0.1 * d)))
    r = (np.arange(nr) + 0.5) * d
    got, ref = {}, {}
    for e in (eps, -eps):
        o = oracle_mod.Oracle(2, nz, nr, delta=d, dt=0.1 * d, tau_tilde=0.53, closure=oracle_mod.LEC,
                              dvel=3.0, mu=1e-8, bc_z=oracle_mod.PERIODIC, geom=oracle_mod.AXI)
        o.init(uz=np.full((nr, nz), U), ux=np.repeat((e * r)[:, None], nz, 1), fields_from_driver=False)
        o.step(steps)
        m = r < 2.0
        got[e] = (o.get("n")[m, 0], o.get("ux")[m, 0] / r[m], o.get("uz")[m, 0])
        ref[e] = _breathing_ode(e, U, steps * 0.1 * d)
    (n_p, a_p, z_p), (n_m, a_m, z_m) = got[eps], got[-eps]
    yp, ym = ref[eps], ref[-eps]
    # first order: the breathing itself
    assert np.abs(n_p - yp[0]).max() <= 0.01 * abs(yp[0] - 1)
    assert np.abs(a_p - yp[1]).max() <= 0.01 * eps  # a(1.5) is near a zero of a(t)
    # second order, even in eps
    n2, n2_ref = 0.5 * (n_p + n_m) - 1, 0.5 * (yp[0] + ym[0]) - 1
    a2, a2_ref = 0.5 * (a_p + a_m), 0.5 * (yp[1] + ym[1])
    assert np.abs(n2 - n2_ref).max() <= 0.03 * abs(n2_ref), (n2[:3], n2_ref)
    assert np.abs(a2 - a2_ref).max() <= 0.05 * abs(a2_ref), (a2[:3], a2_ref)
    # eps U coupling, odd in eps
    zc, zc_ref = 0.5 * (z_p - z_m), 0.5 * (yp[3] - ym[3])
    assert np.abs(zc - zc_ref).max() <= 0.01 * abs(zc_ref), (zc[:3], zc_ref)
