"""Pins of the oracle's time stepping against what the paper and the
mathematics fix (no GPU). Each test names the passage it checks.

Conventions: plasma units (c = omega_p = k_p = n_i = 1), Delta t = Delta / 10
(the paper's ratio, Sec. 5), tau~ = 0.52 in 1D and 0.53 in 2D unless stated.
"""
import numpy as np
import pytest
from scipy import integrate, optimize

D128 = 2 * np.pi / 128


def h0_lec(mu, D):
    """Enthalpy factor 1 + (1 + D/2) mu (eq. lb-ade-lec-comps-A at n = 1, u = 0)."""
    return 1.0 + (1.0 + D / 2.0) * mu


# ---------------------------------------------------------------------------
# Moment-matching ADE (Sec. 2.2, eq. ade and eq. diff-coeff): a Gaussian pulse
# advected at constant u and spread by kappa = nu^2 (tau - dt/2). The
# tolerance on the variance leaves room for the O((u dt/delta)^2) lattice
# correction; tau in place of tau - dt/2 would miss by 67 %.

@pytest.mark.parametrize("dims", [1, 2])
def test_ade_gaussian_advection_diffusion(oracle_mod, dims):
    nz, nx = 512, (320 if dims == 2 else 1)
    d, lam, tau = 1.0, 10.0, 0.8
    dt = d / lam
    uz, ux = 0.3 * lam / 10, (0.15 * lam / 10 if dims == 2 else 0.0)
    z = np.arange(nz) * d
    x = np.arange(nx) * d
    s0 = 12.0
    Z, X = np.meshgrid(z, x)
    A0 = np.exp(-((Z - 100.0) ** 2) / (2 * s0 ** 2))
    if dims == 2:
        A0 = A0 * np.exp(-((X - 150.0) ** 2) / (2 * (s0 * 0.5) ** 2))
    steps = 1500
    A = oracle_mod.ade_run(dims, A0 if dims == 2 else A0[0], d, dt, tau, uz, ux, steps)
    A = np.atleast_2d(A)
    t = steps * dt
    kappa = lam * lam / 3.0 * (tau - 0.5) * dt
    m0 = A0.sum()
    assert abs(A.sum() - m0) <= 1e-13 * m0          # conservation
    pz = A.sum(axis=0) / m0
    cz = (pz * z).sum()
    vz = (pz * (z - cz) ** 2).sum()
    assert abs(cz - (100.0 + uz * t)) <= 1e-9 * 100
    assert abs(vz - (s0 ** 2 + 2 * kappa * t)) <= 1e-3 * (s0 ** 2 + 2 * kappa * t)
    if dims == 2:
        px = A.sum(axis=1) / m0
        cx = (px * x).sum()
        vx = (px * (x - cx) ** 2).sum()
        assert abs(cx - (150.0 + ux * t)) <= 1e-9 * 100
        assert abs(vx - ((s0 * 0.5) ** 2 + 2 * kappa * t)) <= 1e-3 * ((s0 * 0.5) ** 2 + 2 * kappa * t)


# ---------------------------------------------------------------------------
# Conservation: the density scalar has F = 0 (eq. lb-ade-lec-comps-F,
# eq. lb-ade-warmc-comps-F), BGK and streaming conserve sum_i f_i, so the
# total number of electrons is conserved to round-off on a periodic domain,
# whatever the fields and the driver do.

@pytest.mark.parametrize("closure", [0, 1])
@pytest.mark.parametrize("dims", [1, 2])
def test_number_conservation_periodic(oracle_mod, closure, dims):
    nz, nx = (256, 1) if dims == 1 else (96, 48)
    rng = np.random.default_rng(7)
    z = np.arange(nz) * D128
    x = np.arange(nx) * D128
    Z, X = np.meshgrid(z, x)
    n = 1 + 0.2 * np.sin(2 * np.pi * Z / (nz * D128)) + 0.01 * rng.uniform(-1, 1, Z.shape)
    uz = 0.05 * np.cos(2 * np.pi * Z / (nz * D128))
    ux = 0.03 * np.sin(2 * np.pi * X / (nx * D128)) if dims == 2 else None
    o = oracle_mod.Oracle(dims, nz, nx, closure=closure, mu=0.02, alpha=0.3, sigma_z=0.5,
                          sigma_x=0.5, z0=2.0, bc_z=oracle_mod.PERIODIC, bc_x=oracle_mod.PERIODIC)
    o.init(n=n if dims == 2 else n[0], uz=uz if dims == 2 else uz[0], ux=ux)
    n_start = o.diagnostics()[0]
    o.step(150)
    dg = o.diagnostics()
    assert dg[5] == 0
    assert abs(dg[0] - n_start) <= 1e-13 * n_start


# ---------------------------------------------------------------------------
# A uniform plasma at rest without driver: every gradient vanishes, u = 0,
# E = B = 0, so every force is exactly zero and the state stays uniform and at
# rest to the bit (the density moves at most by round-off of sum_i w_i).

@pytest.mark.parametrize("closure", [0, 1])
@pytest.mark.parametrize("dims", [1, 2])
def test_rest_state_invariant(oracle_mod, closure, dims):
    nz, nx = (64, 1) if dims == 1 else (32, 16)
    o = oracle_mod.Oracle(dims, nz, nx, closure=closure, mu=0.05, alpha=0.0)
    o.init()
    o.step(200)
    n = o.get("n")
    for q in ("uz", "ux", "ez", "ex", "by"):
        assert np.all(o.get(q) == 0.0), q
    assert np.all(n == n.flat[0])
    assert abs(n.flat[0] - 1.0) <= 1e-14
    if closure == 1:
        thzz = o.get("thzz")
        assert np.all(thzz == thzz.flat[0])


# ---------------------------------------------------------------------------
# k = 0 plasma oscillation. For a uniform state the streaming is the identity
# and BGK conserves every zeroth moment, so each scalar obeys
# A^{n+1} = A^n + dt F^n exactly (eq. lbe with S_i = w_i F), and the field
# obeys E^{n+1} = E^n + dt n u^{n+1}. At small amplitude that is a linear
# recurrence whose continuum limit has omega^2 = 1/(1 + (1 + D/2) mu) (LEC) and
# omega^2 = 1/(lambda_0 + mu) (WARMC); at O(mu) both are 1 - (5/2) mu for D = 3
# (Sec. 5.2 and App. B).

def _k0_model(closure, D, mu, lam0, dt, u0, steps, B=0.0):
    """Linearised uniform-state recurrence: returns u_z, u_x, E_z, E_x series."""
    inert = h0_lec(mu, D) if closure == 0 else lam0
    uz, ux, ez, ex = u0, 0.0, 0.0, 0.0
    uz_prev, ux_prev = uz, ux
    out = []
    for _ in range(steps):
        out.append((uz, ux, ez, ex))
        if closure == 0:
            # A = h0 n gamma u, F = -n (E + u x B)
            fz = -(ez + ux * B)
            fx = -(ex - uz * B)
            nuz = uz + dt * fz / inert
            nux = ux + dt * fx / inert
        else:
            # n lambda u_i: F = -d_t theta^{0i} - n (E + u x B)_i, theta^{0i} = mu u_i
            fz = -(ez + ux * B) - mu * (uz - uz_prev) / dt
            fx = -(ex - uz * B) - mu * (ux - ux_prev) / dt
            nuz = uz + dt * fz / inert
            nux = ux + dt * fx / inert
        uz_prev, ux_prev = uz, ux
        uz, ux = nuz, nux
        ez = ez + dt * uz
        ex = ex + dt * ux
    return np.array(out)


def _run_k0(oracle_mod, closure, D, dims, direction, steps, u0=1e-6, mu=0.04, B=0.0):
    nz, nx = (8, 1) if dims == 1 else (8, 8)
    o = oracle_mod.Oracle(dims, nz, nx, closure=closure, dvel=D, mu=mu,
                          bc_z=oracle_mod.PERIODIC, bc_x=oracle_mod.PERIODIC)
    if direction == "z":
        o.init(uz=u0)
    else:
        o.init(ux=u0)
    if B != 0.0:
        o.set_yee("by", B)
    rec = []
    for _ in range(steps):
        rec.append([float(np.ravel(o.get(q))[3]) for q in ("uz", "ux", "ez", "ex")])
        o.step(1)
    return np.array(rec)


@pytest.mark.parametrize("closure,D", [(0, 1.0), (0, 3.0), (1, 1.0), (1, 3.0)])
def test_k0_oscillation_1d(oracle_mod, closure, D):
    mu, u0 = 0.04, 1e-6
    dt = 0.1 * D128
    steps = 4200
    lam0 = oracle_mod.lambda0(mu, D)
    got = _run_k0(oracle_mod, closure, D, 1, "z", steps, u0, mu)
    ref = _k0_model(closure, D, mu, lam0, dt, u0, steps)
    assert np.abs(got[:, 0] - ref[:, 0]).max() <= 1e-8 * u0
    assert np.abs(got[:, 2] - ref[:, 2]).max() <= 1e-8 * u0
    # continuum frequency from the zero crossings of u
    t = np.arange(steps) * dt
    u = got[:, 0]
    zc = [t[i] - u[i] * (t[i + 1] - t[i]) / (u[i + 1] - u[i])
          for i in range(steps - 1) if u[i] > 0 >= u[i + 1]]
    omega = 2 * np.pi / np.mean(np.diff(zc))
    w2 = 1 / h0_lec(mu, D) if closure == 0 else 1 / (lam0 + mu)
    tol = 1e-4 if closure == 0 else 1e-3
    assert abs(omega ** 2 - w2) <= tol * w2
    if D == 3.0:  # O(mu) form printed for the 3V case; 1/(1+5/2 mu) differs at 6.25 mu^2
        assert abs(omega ** 2 - (1 - 2.5 * mu)) <= 8 * mu * mu


@pytest.mark.parametrize("closure", [0, 1])
@pytest.mark.parametrize("direction", ["z", "x"])
def test_k0_oscillation_2d(oracle_mod, closure, direction):
    mu, u0, D = 0.04, 1e-6, 3.0
    dt = 0.1 * D128
    steps = 500
    lam0 = oracle_mod.lambda0(mu, D)
    got = _run_k0(oracle_mod, closure, D, 2, direction, steps, u0, mu)
    ref = _k0_model(closure, D, mu, lam0, dt, u0, steps)
    if direction == "x":
        ref = ref[:, [1, 0, 3, 2]]
    assert np.abs(got - ref).max() <= 1e-8 * u0


@pytest.mark.parametrize("closure", [0, 1])
def test_k0_upper_hybrid_uniform_by(oracle_mod, closure):
    """Uniform B_y: the uniform oscillation couples u_z and u_x through
    u x B (App. A Lorentz terms); B stays uniform because curl E = 0."""
    mu, u0, D, B = 0.04, 1e-6, 3.0, 0.7
    dt = 0.1 * D128
    steps = 600
    lam0 = oracle_mod.lambda0(mu, D)
    got = _run_k0(oracle_mod, closure, D, 2, "z", steps, u0, mu, B=B)
    ref = _k0_model(closure, D, mu, lam0, dt, u0, steps, B=B)
    assert np.abs(got - ref).max() <= 1e-8 * u0
    assert np.abs(got[:, 1]).max() > 0.1 * u0  # the u_x coupling is active


def test_warmc_pressure_rotation_uniform_by(oracle_mod):
    """WARMC, fluid at rest in a uniform B_y with an anisotropic pressure
    tensor: only the Lorentz terms of the lambda theta equations act
    (App. A: -2(E theta^0 - B theta^{xz}), -2(E theta^0 + B theta^{xz}),
    -[... + B (theta^{xx} - theta^{zz})]); u and E stay zero."""
    mu, B = 0.03, 0.9
    dt = 0.1 * D128
    nz, nx = 8, 8
    o = oracle_mod.Oracle(2, nz, nx, closure=1, dvel=3.0, mu=mu,
                          bc_z=oracle_mod.PERIODIC, bc_x=oracle_mod.PERIODIC)
    lam = 1.02
    thzz, thxx, thyy, thxz = 0.03, 0.01, 0.02, 0.004
    A = np.zeros((8, nx, nz))
    A[0] = 1.0
    A[1] = lam
    A[4], A[5], A[6], A[7] = lam * thzz, lam * thxx, lam * thyy, lam * thxz
    o.init_moments(A)
    o.set_yee("by", B)
    steps = 400
    got, ref = [], []
    a_zz, a_xx, a_xz = thzz, thxx, thxz
    for _ in range(steps):
        got.append([o.get(q).flat[5] for q in ("thzz", "thxx", "thxz", "thyy", "uz", "ex")])
        ref.append([a_zz, a_xx, a_xz, thyy, 0.0, 0.0])
        f_xx = 2 * B * a_xz
        f_zz = -2 * B * a_xz
        f_xz = -B * (a_xx - a_zz)
        a_xx, a_zz, a_xz = a_xx + dt * f_xx / lam, a_zz + dt * f_zz / lam, a_xz + dt * f_xz / lam
        o.step(1)
    got, ref = np.array(got), np.array(ref)
    assert np.abs(got - ref).max() <= 1e-15 * steps
    # the tensor turns: theta^{xz} changes sign within a quarter cyclotron period
    assert got[:, 2].min() < 0 < got[:, 2].max()


# ---------------------------------------------------------------------------
# Finite-k Langmuir waves (Sec. 5.2, App. B): the linearised equations give
# LEC: omega^2 = (1 + (1 + 2/D) mu k^2) / (1 + (1 + D/2) mu)
# WARMC: omega^2 = (1 + (3 mu - mu^2/lambda_0) k^2) / (lambda_0 + mu)
# which at O(mu) and D = 3 are the printed 1 - 5/2 mu + 5/3 mu k^2 and
# 1 - 5/2 mu + 3 mu k^2.

def _measure_omega(series, dt):
    t = np.arange(len(series)) * dt
    f = lambda tt, A, w, ph, g: A * np.exp(-g * tt) * np.cos(w * tt + ph)
    p, _ = optimize.curve_fit(f, t, series, p0=[series[0], 1.0, 0.0, 0.0], maxfev=20000)
    return abs(p[1])


def _disp_model(closure, D, mu, lam0, k):
    if closure == 0:
        return (1 + (1 + 2 / D) * mu * k * k) / h0_lec(mu, D)
    return (1 + (3 * mu - mu * mu / lam0) * k * k) / (lam0 + mu)


@pytest.mark.parametrize("closure,D", [(0, 1.0), (0, 3.0), (1, 1.0), (1, 3.0)])
def test_langmuir_dispersion_1d(oracle_mod, closure, D):
    mu, k, nz = 0.04, 2.0, 256
    L = 2 * np.pi / k
    d = L / nz
    dt = 0.1 * d
    lam0 = oracle_mod.lambda0(mu, D)
    z = np.arange(nz) * d
    o = oracle_mod.Oracle(1, nz, delta=d, dt=dt, closure=closure, dvel=D, mu=mu,
                          bc_z=oracle_mod.PERIODIC)
    o.init(uz=1e-5 * np.sin(k * z))
    steps, stride = 12000, 20
    amp = []
    for _ in range(steps // stride):
        amp.append(2 / nz * (o.get("uz") * np.sin(k * z)).sum())
        o.step(stride)
    w = _measure_omega(np.array(amp), stride * dt)
    w2 = _disp_model(closure, D, mu, lam0, k)
    # second-order scheme: 3.5e-4 at 128 cells per wavelength, 1.2e-4 at 256
    assert abs(w * w - w2) <= 2e-4 * w2
    if D == 3.0:
        printed = 1 - 2.5 * mu + (5 / 3 if closure == 0 else 3.0) * mu * k * k
        assert abs(w * w - printed) <= 8 * mu * mu * (1 + k * k)


@pytest.mark.parametrize("closure", [0, 1])
def test_langmuir_dispersion_2d_along_x(oracle_mod, closure):
    """A longitudinal wave along x in 2D checks the x gradients (pressure,
    theta^{xx}) and the E_x part of the Yee update."""
    mu, k, D = 0.04, 2.0, 3.0
    nx = 128
    L = 2 * np.pi / k
    d = L / nx
    dt = 0.1 * d
    lam0 = oracle_mod.lambda0(mu, D)
    x = (np.arange(nx) - 0.5 * (nx - 1)) * d
    o = oracle_mod.Oracle(2, 4, nx, delta=d, dt=dt, closure=closure, dvel=D, mu=mu,
                          bc_z=oracle_mod.PERIODIC, bc_x=oracle_mod.PERIODIC)
    ux0 = 1e-5 * np.sin(k * x)[:, None] * np.ones((1, 4))
    o.init(ux=ux0)
    steps, stride = 8000, 16
    amp = []
    for _ in range(steps // stride):
        amp.append(2 / nx * (o.get("ux")[:, 1] * np.sin(k * x)).sum())
        o.step(stride)
    w = _measure_omega(np.array(amp), stride * dt)
    w2 = _disp_model(closure, D, mu, lam0, k)
    # second order: the edge average of J_x and the node average of E_x add
    # (k delta)^2/4 to the plasma term (3.2e-3 at 64 cells, 8e-4 at 128)
    assert abs(w * w - w2) <= 1.5e-3 * w2


def _transverse_model(closure, mu, lam0, D, k):
    """Transverse wave (E_x, B_y, u_x along z): omega^2 = k^2 + 1/h0 (LEC);
    WARMC adds the shear stress theta^{xz}: (k^2 - w^2)(mu k^2 - (lambda_0 + mu) w^2) = w^2."""
    if closure == 0:
        return k * k + 1 / h0_lec(mu, D)
    a = lam0 + mu
    # a w^4 - (a k^2 + mu k^2 + 1) w^2 + mu k^4 = 0 : the electromagnetic root
    b = a * k * k + mu * k * k + 1
    return (b + np.sqrt(b * b - 4 * a * mu * k ** 4)) / (2 * a)


@pytest.mark.parametrize("closure", [0, 1])
@pytest.mark.parametrize("direction", ["z", "x"])
def test_transverse_em_wave_2d(oracle_mod, closure, direction):
    """Yee curl terms (Faraday, Ampere) and the transverse current: along z the
    wave is (E_x, B_y, u_x), along x it is (E_z, B_y, u_z); WARMC adds the
    shear stress theta^{xz}."""
    mu, k, D = 0.04, 1.0, 3.0
    nn = 128
    L = 2 * np.pi / k
    d = L / nn
    dt = 0.1 * d
    lam0 = oracle_mod.lambda0(mu, D)
    if direction == "z":
        nz, nx = nn, 4
    else:
        nz, nx = 4, nn
    o = oracle_mod.Oracle(2, nz, nx, delta=d, dt=dt, closure=closure, dvel=D, mu=mu,
                          bc_z=oracle_mod.PERIODIC, bc_x=oracle_mod.PERIODIC)
    o.init()
    if direction == "z":
        coord = np.arange(nz) * d
        o.set_yee("ex", 1e-5 * np.sin(k * coord)[None, :] * np.ones((nx, 1)))
        probe = lambda: o.get("ex_yee")[1]
    else:
        coord = (np.arange(nx) - 0.5 * (nx - 1)) * d
        o.set_yee("ez", 1e-5 * np.sin(k * coord)[:, None] * np.ones((1, nz)))
        probe = lambda: o.get("ez_yee")[:, 1]
    steps, stride = 5000, 10
    amp = []
    for _ in range(steps // stride):
        amp.append(2 / nn * (probe() * np.sin(k * coord)).sum())
        o.step(stride)
    w = _measure_omega(np.array(amp), stride * dt)
    w2 = _transverse_model(closure, mu, lam0, D, k)
    assert abs(w * w - w2) <= 6e-4 * w2


# ---------------------------------------------------------------------------
# Driven wakes in 1D (Sec. 5.1, App. B). The bunch moves at c along +z; ahead
# of it the plasma is at rest, so every cell it has passed carries the
# steady co-moving response. Cold limit (c_s = 0, a_e = a_b = 1, mirrored to
# +z propagation): n_1 = -int_zeta^inf n_b sin(zeta' - zeta), E_z = int n_b cos.
# The LB numerical diffusion (eq. diff-coeff) damps the velocity at kappa k^2
# while the field is not diffused, so the oscillation decays at kappa/2 per
# unit distance behind the bunch (k_w = 1).

def _cold_wake(zeta, alpha, sz):
    nb = lambda zp: alpha * np.exp(-zp ** 2 / (2 * sz ** 2))
    n = np.array([-integrate.quad(lambda zp: nb(zp) * np.sin(zp - ze), max(ze, -9 * sz), 9 * sz)[0]
                  for ze in zeta])
    e = np.array([integrate.quad(lambda zp: nb(zp) * np.cos(zp - ze), max(ze, -9 * sz), 9 * sz)[0]
                  for ze in zeta])
    return n, e


@pytest.mark.parametrize("closure", [0, 1])
def test_cold_linear_wake_1d(oracle_mod, closure):
    alpha, sz, mu, nz = 1e-3, 0.5, 1e-6, 2048
    dt = 0.1 * D128
    o = oracle_mod.Oracle(1, nz, closure=closure, dvel=1.0, mu=mu, alpha=alpha, sigma_z=sz)
    o.init()
    steps = 4200
    o.step(steps)
    t = steps * dt
    z = np.arange(nz) * D128
    zeta = z - (6 * sz + t)
    m = (zeta < -3 * sz) & (zeta > -3 * sz - 2 * 2 * np.pi)
    n_th, e_th = _cold_wake(zeta[m], alpha, sz)
    kappa = (100 / 3) * (0.52 - 0.5) * dt
    damp = np.exp(-0.5 * kappa * np.abs(zeta[m]))
    amp = alpha * np.sqrt(2 * np.pi) * sz * np.exp(-sz * sz / 2)
    assert abs(np.abs(e_th).max() - amp) <= 1e-3 * amp
    assert np.abs(o.get("ez")[m] - e_th * damp).max() <= 2e-3 * amp
    assert np.abs(o.get("n")[m] - 1 - n_th * damp).max() <= 4e-3 * amp
    # Gauss's law in the wake: dE_z/dz = 1 - n - n_b
    ez, n = o.get("ez"), o.get("n")
    dez = (ez[2:] - ez[:-2]) / (2 * D128)
    mm = m[1:-1]
    nb = alpha * np.exp(-zeta[1:-1] ** 2 / (2 * sz * sz))
    assert np.abs(dez[mm] - (1 - n[1:-1][mm] - nb[mm])).max() <= 5e-3 * amp


def _wake_k(oracle_mod, closure, D, mu, alpha=1e-3, sz=0.5, nz=4096, steps=10000):
    dt = 0.1 * D128
    o = oracle_mod.Oracle(1, nz, closure=closure, dvel=D, mu=mu, alpha=alpha, sigma_z=sz)
    o.init()
    o.step(steps)
    t = steps * dt
    z = np.arange(nz) * D128
    zeta = z - (6 * sz + t)
    # steady region: behind the bunch, ahead of what the initial transient
    # (sound at c_s from the start position) can reach
    cs = np.sqrt(3 * mu)
    m = (zeta < -4 * sz) & (zeta > -(1 - 1.5 * cs) * t + 4 * sz) & (zeta > -4 * sz - 4 * 2 * np.pi)
    ez = o.get("ez")
    f = lambda ze, A, k, ph, g: A * np.exp(g * ze) * np.cos(k * ze + ph)
    p, _ = optimize.curve_fit(f, zeta[m], ez[m], p0=[np.abs(ez[m]).max(), 1.0, 0.0, 0.0],
                              maxfev=20000)
    return abs(p[1]), m.sum() * D128, abs(p[0])


@pytest.mark.parametrize("closure,D", [(0, 1.0), (0, 3.0), (1, 1.0), (1, 3.0)])
def test_warm_wake_wavelength(oracle_mod, closure, D):
    """Wake behind a bunch at c: k_w^2 = a_e^2 / (1 - c_s^2) from the comoving
    forced Klein-Gordon equation (App. B, eq. fhow-comoving), i.e.
    1/(h0 - (1 + 2/D) mu) (LEC) and 1/(lambda_0 - 2 mu + mu^2/lambda_0) (WARMC);
    O(mu) and D = 3: 1 - 5/6 mu (LEC), 1 + mu/2 (WARMC) (eq. disp-rel1/2);
    D = 1: both 1 + 3/2 mu, the closures coincide (Sec. 5.1)."""
    mu = 0.04
    lam0 = oracle_mod.lambda0(mu, D)
    k, span, _ = _wake_k(oracle_mod, closure, D, mu)
    assert span >= 2 * 2 * np.pi
    if closure == 0:
        kw2 = 1 / (h0_lec(mu, D) - (1 + 2 / D) * mu)
    else:
        kw2 = 1 / (lam0 - 2 * mu + mu * mu / lam0)
    assert abs(k - np.sqrt(kw2)) <= 1e-3 * np.sqrt(kw2)
    printed = {3.0: (1 - 5 / 6 * mu) if closure == 0 else (1 + 0.5 * mu), 1.0: 1 + 1.5 * mu}[D]
    assert abs(k * k - printed) <= 3 * mu * mu


@pytest.mark.parametrize("closure,D", [(0, 1.0), (0, 3.0), (1, 1.0), (1, 3.0)])
def test_warm_wake_amplitude(oracle_mod, closure, D):
    """Amplitude of the warm linear wake (App. B, eq. fhow-comoving):
    (1 - c_s^2) n_1'' = -a_e^2 n_1 - a_b^2 n_b behind a Gaussian bunch gives,
    with Gauss's law E_z' = -(n_1 + n_b), an E_z amplitude
    (a_b^2 / a_e^2) alpha sqrt(2 pi) sigma_z exp(-k_w^2 sigma_z^2 / 2),
    k_w^2 = a_e^2 / (1 - c_s^2). The bunch enters the equations of both
    closures only through Gauss's law, exactly as the plasma charge does, so
    linearising them gives a_b = a_e (LEC 1/h0, WARMC 1/(lambda_0 + mu)).
    App. B prints a_b^2 = 1 - mu/2 for the warm closure against
    a_e^2 = 1 - 5/2 mu, which would make the amplitude 8.9 % larger at
    mu = 0.04 and D = 3; the scheme follows its equations (measured ratio
    0.9999 for every case; the fit's damping factor carries the LB
    diffusion)."""
    mu, sz, alpha = 0.04, 0.5, 1e-3
    lam0 = oracle_mod.lambda0(mu, D)
    if closure == 0:
        ae2 = 1 / h0_lec(mu, D)
        cs2 = (1 + 2 / D) * mu * ae2
    else:
        ae2 = 1 / (lam0 + mu)
        cs2 = (3 * mu - mu * mu / lam0) * ae2
    kw2 = ae2 / (1 - cs2)
    _, _, amp = _wake_k(oracle_mod, closure, D, mu, alpha=alpha, sz=sz)
    theory = alpha * np.sqrt(2 * np.pi) * sz * np.exp(-kw2 * sz * sz / 2)
    assert abs(amp / theory - 1) <= 2e-3, amp / theory


# ---------------------------------------------------------------------------
# Initial fields (Sec. 5: fields of the bunch alone, Gauss-consistent).

def test_initial_field_gauss_1d(oracle_mod):
    sz, alpha, nz = 0.5, 0.1, 512
    o = oracle_mod.Oracle(1, nz, mu=1e-3, alpha=alpha, sigma_z=sz)
    o.init()
    ez = o.get("ez")
    z = np.arange(nz) * D128
    nb = alpha * np.exp(-(z - 6 * sz) ** 2 / (2 * sz * sz))
    dez = (ez[2:] - ez[:-2]) / (2 * D128)
    assert np.abs(dez + nb[1:-1]).max() <= 2e-3 * alpha
    assert abs(ez[0] - alpha * sz * np.sqrt(2 * np.pi)) <= 1e-9  # the tail beyond -6 sigma_z
    assert np.abs(ez[z > 6 * sz + 8 * sz]).max() <= 1e-12


def test_initial_field_2d_vacuum_solution(oracle_mod):
    """E_z = 0, E_x odd in x with dE_x/dx = -n_b, B_y = E_x (travelling at c)."""
    nz, nx, sz, sx, alpha = 128, 64, 1.0, 0.5, 1.0
    d = 2 * np.pi / 64
    o = oracle_mod.Oracle(2, nz, nx, delta=d, mu=1e-2, alpha=alpha, sigma_z=sz, sigma_x=sx)
    o.init()
    ex = o.get("ex_yee")
    assert np.all(o.get("ez_yee") == 0)
    # odd about the axis: E_x at x_{j+1/2} and x_{nx-2-j+1/2} are mirror images
    assert np.allclose(ex[:-1], -ex[:-1][::-1], atol=1e-14)
    diag = o.diagnostics()
    assert diag[3] <= 2e-3 * alpha


# ---------------------------------------------------------------------------
# Symmetry of the 2D driven problem under x -> -x: n, u_z, E_z even; u_x,
# E_x, B_y odd (the bunch sits on the axis).

@pytest.mark.parametrize("closure", [0, 1])
def test_mirror_symmetry_2d(oracle_mod, closure):
    nz, nx = 96, 48
    d = 2 * np.pi / 32
    o = oracle_mod.Oracle(2, nz, nx, delta=d, closure=closure, mu=0.02, alpha=0.5,
                          sigma_z=1.0, sigma_x=0.5)
    o.init()
    o.step(120)
    for q, sgn in (("n", 1), ("uz", 1), ("ez", 1), ("ux", -1), ("ex", -1), ("by", -1)):
        v = o.get(q)
        scale = max(np.abs(v).max(), 1e-30)
        assert np.abs(v - sgn * v[::-1]).max() <= 1e-11 * scale, q
    assert np.abs(o.get("ux")).max() > 1e-4


# ---------------------------------------------------------------------------
# Rotation covariance in the (x, z) plane. Both closures are written with
# vectors and tensors (Secs. 3 and 4, App. A with the 1/r terms dropped), so a
# plane Langmuir wave travelling along s = (3 x + 4 z)/5 must be, in the frame
# (s, t) with t = (4 x - 3 z)/5, the same wave as one travelling along z, up to
# the lattice's anisotropy, which vanishes as delta -> 0. On an N x N periodic
# grid with N = 5 M the oblique wave is a function of p = (3 i_x + 4 i_z) mod N
# alone (the shift (4, -3) keeps p and generates every such translation), and
# the nodes with p = 5 m carry the phase of node m of the wave along z on M
# nodes. The oblique wave drives every cross term of the warm closure that the
# wave along z leaves at zero (u_x u_z, theta^{xz}, theta^{0x}); at u = 0.2
# those are a few per cent of the motion, so a dropped or wrongly signed one
# leaves a difference that does not shrink with delta.

def _oblique_vs_axis(oracle_mod, closure, npw, u0=0.2, mu=0.1, k=1.5, periods=0.5):
    """Maximum differences, oblique wave minus wave along z, at the nodes
    with p = 5 m, relative to each quantity's amplitude: density, lambda,
    velocity along s and across it, E along s, B_y, and theta^{ss},
    theta^{tt}, theta^{st} (theta^{zz}, theta^{xx}, 0 for the wave along z)."""
    M, N = npw, 5 * npw
    d = 2 * np.pi / (npw * k)
    steps = int(round(periods * 2 * np.pi / (0.1 * d)))
    warm = closure == 1
    qs = ["n", "uz", "ux", "ez", "ex", "by"] + (["lambda", "thzz", "thxx", "thxz"] if warm else [])
    a = oracle_mod.Oracle(2, M, 4, delta=d, closure=closure, mu=mu,
                          bc_z=oracle_mod.PERIODIC, bc_x=oracle_mod.PERIODIC)
    a.init(uz=np.broadcast_to(u0 * np.sin(2 * np.pi * np.arange(M) / M), (4, M)), ux=0.0,
           fields_from_driver=False)
    a.step(steps)
    A = {q: a.get(q)[0] for q in qs}
    b = oracle_mod.Oracle(2, N, N, delta=d, closure=closure, mu=mu,
                          bc_z=oracle_mod.PERIODIC, bc_x=oracle_mod.PERIODIC)
    ix, iz = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")  # [nx][nz]
    p = (3 * ix + 4 * iz) % N
    us = u0 * np.sin(2 * np.pi * p / N)
    b.init(uz=0.8 * us, ux=0.6 * us, fields_from_driver=False)
    b.step(steps)
    sel = p % 5 == 0
    m = p[sel] // 5
    B = {q: b.get(q)[sel] for q in qs}
    cx, cz = 0.6, 0.8  # s = (cx, cz) in (x, z); t = (cz, -cx)
    obl = {"n": B["n"], "us": cx * B["ux"] + cz * B["uz"], "ut": cz * B["ux"] - cx * B["uz"],
           "es": cx * B["ex"] + cz * B["ez"], "by": B["by"]}
    ref = {"n": A["n"][m], "us": A["uz"][m], "ut": A["ux"][m], "es": A["ez"][m], "by": A["by"][m]}
    amp = {"n": np.ptp(A["n"]) / 2, "us": np.abs(A["uz"]).max(), "ut": np.abs(A["uz"]).max(),
           "es": np.abs(A["ez"]).max(), "by": np.abs(A["ez"]).max()}
    if warm:
        obl.update(lam=B["lambda"],
                   thss=cx * cx * B["thxx"] + 2 * cx * cz * B["thxz"] + cz * cz * B["thzz"],
                   thtt=cz * cz * B["thxx"] - 2 * cx * cz * B["thxz"] + cx * cx * B["thzz"],
                   thst=cx * cz * (B["thxx"] - B["thzz"]) + (cz * cz - cx * cx) * B["thxz"])
        ref.update(lam=A["lambda"][m], thss=A["thzz"][m], thtt=A["thxx"][m], thst=A["thxz"][m])
        amp.update(lam=np.ptp(A["lambda"]) / 2, thss=np.ptp(A["thzz"]) / 2, thtt=np.ptp(A["thxx"]) / 2,
                   thst=np.ptp(A["thzz"]) / 2)
    assert np.ptp(b.get("n")[p == 5]) == 0.0  # a function of p alone
    return {q: np.abs(obl[q] - ref[q]).max() / amp[q] for q in obl}


# twice the differences measured at 48 nodes per wavelength
BOUND_OBLIQUE = {
    0: dict(n=3.1e-2, us=3.3e-3, ut=1.0e-3, es=4.5e-2, by=1.1e-2),
    1: dict(n=3.5e-2, us=5.8e-3, ut=6.5e-4, es=2.0e-2, by=5.6e-3, lam=2.5e-2, thss=4.4e-2, thtt=3.5e-2,
            thst=1.8e-3),
}


@pytest.mark.parametrize("closure", [0, 1])
def test_rotation_covariance_oblique_wave(oracle_mod, closure):
    """Half a plasma period of a u = 0.2 wave (k = 1.5, mu = 0.1) at 24 and
    48 nodes per wavelength: every difference shrinks at least 2.2x when the
    resolution doubles (measured 2.4x ... 5.7x) and stays below twice its
    measured value at 48 nodes. Each of these mistakes planted in the warm
    closure fails both checks (largest factor over the bound at 48 nodes):
    -2 theta^{xz} d_x(lambda u_z) dropped from F(lambda theta^{zz}) (15x, on
    theta^{st}), -2 theta^{xz} d_z(lambda u_x) dropped from F(lambda
    theta^{xx}) (15x); the sign of -theta^{xz} d_x(lambda u_x) (6.4x) or of
    -theta^{xz} d_z(lambda u_z) (12x) in F(lambda theta^{xz}) flipped;
    -theta^{0z} d_t(lambda u_x) dropped from F(lambda theta^{xz}) (2.3x),
    -2 theta^{0x} d_t(lambda u_x) from F(lambda theta^{xx}) (5.4x); u_z
    theta^{xz} dropped from theta^{0x} (6.8x, on u_t); -d_x theta^{0x} dropped
    from F(n lambda) (12x, on lambda)."""
    d24 = _oblique_vs_axis(oracle_mod, closure, 24)
    d48 = _oblique_vs_axis(oracle_mod, closure, 48)
    print({q: (float(f"{d24[q]:.3g}"), float(f"{d48[q]:.3g}")) for q in d24})
    bound = BOUND_OBLIQUE[closure]
    for q in d48:
        assert d48[q] <= d24[q] / 2.2, q
        assert d48[q] <= bound[q], q


# ---------------------------------------------------------------------------
# Large-amplitude uniform oscillations (nonlinear terms). For a uniform state
# every scalar obeys dA/dt = F exactly as above, so the continuum dynamics is
# an ODE with closed-form integrals:
# - cold relativistic limit (mu -> 0, both closures): p' = -E, E' = p/gamma,
#   energy gamma + E^2/2 is conserved and the period is
#   T = 4 int_0^{p_max} dp / E(p);
# - LEC (Sec. 3): d(h n p)/dt = -n E, dE/dt = n u with h = h(n/gamma); the
#   conserved energy is T^00 + E^2/2 = n h gamma - P0 + E^2/2, so
#   T = 4 int dA / (n E(A));
# - WARMC (Sec. 4): T^00 = theta^00 + n lambda, so n lambda + theta^00 + E^2/2
#   is conserved, and the trace condition (eq. traces3)
#   theta^mu_mu = h (1 - (n0/h)^2) holds along the motion.

def _uniform_series(oracle_mod, closure, D, mu, u0, steps, dt, quantities):
    o = oracle_mod.Oracle(1, 4, delta=10 * dt, dt=dt, closure=closure, dvel=D, mu=mu,
                          bc_z=oracle_mod.PERIODIC)
    o.init(uz=u0)
    rec = []
    for _ in range(steps):
        rec.append([float(o.get(q)[1]) for q in quantities])
        o.step(1)
    return np.array(rec)


def _period_from_crossings(t, u):
    zc = [t[i] - u[i] * (t[i + 1] - t[i]) / (u[i + 1] - u[i])
          for i in range(len(u) - 1) if u[i] > 0 >= u[i + 1]]
    return np.mean(np.diff(zc))


@pytest.mark.parametrize("closure", [0, 1])
def test_cold_relativistic_k0_period(oracle_mod, closure):
    """LEC advects p itself, so its period error is second order in dt; WARMC
    advects n lambda (the energy) and n lambda u separately with an explicit
    force, so the mass shell lambda^2 - (lambda u)^2 = 1 drifts at first order:
    its error must halve with dt."""
    u0 = 0.8
    g0 = 1 / np.sqrt(1 - u0 * u0)
    pmax = g0 * u0
    # E(p)^2 = 2 (gamma_max - gamma(p))
    T = 4 * integrate.quad(lambda p: 1 / np.sqrt(2 * (g0 - np.sqrt(1 + p * p))), 0, pmax,
                           limit=200)[0]
    assert T > 2 * np.pi * 1.1  # relativistic lengthening is visible
    errs = []
    for dt in (0.004, 0.002):
        steps = int(3.2 * T / dt)
        s = _uniform_series(oracle_mod, closure, 1.0, 1e-9, u0, steps, dt, ["uz"])
        errs.append((_period_from_crossings(np.arange(steps) * dt, s[:, 0]) - T) / T)
    if closure == 0:
        assert abs(errs[1]) <= 2e-4
    else:
        assert abs(errs[1]) <= 2e-3
        assert abs(errs[0] / errs[1] - 2.0) <= 0.05


@pytest.mark.parametrize("D", [1.0, 3.0])
def test_lec_warm_nonlinear_k0_period(oracle_mod, D):
    mu, u0, dt = 0.05, 0.6, 0.002
    a = (1 + D / 2) * mu
    h = lambda n0: 1 + a * n0 ** (2 / D)
    g0 = 1 / np.sqrt(1 - u0 * u0)
    p0 = g0 * u0
    # uniform n = 1: A(p) = h(1/gamma) p; energy W(p) = h gamma - mu (1/gamma)^{1+2/D}
    W = lambda p: h(1 / np.sqrt(1 + p * p)) * np.sqrt(1 + p * p) - mu * (1 + p * p) ** (-(1 + 2 / D) / 2)
    A = lambda p: h(1 / np.sqrt(1 + p * p)) * p
    dA = lambda p: (A(p + 1e-7) - A(p - 1e-7)) / 2e-7
    T = 4 * integrate.quad(lambda p: dA(p) / np.sqrt(2 * (W(p0) - W(p))), 0, p0, limit=200)[0]
    steps = int(3.2 * T / dt)
    s = _uniform_series(oracle_mod, 0, D, mu, u0, steps, dt, ["uz"])
    Tm = _period_from_crossings(np.arange(steps) * dt, s[:, 0])
    assert abs(Tm - T) <= 2e-4 * T


@pytest.mark.parametrize("D", [1.0, 3.0])
def test_warmc_nonlinear_k0_invariants(oracle_mod, D):
    """Energy n lambda + theta^00 + E^2/2 and the trace condition converge to
    exact invariants at first order in dt (explicit force on n lambda). In 1D
    the transverse lambda theta^{xx}, lambda theta^{yy} (D = 3) are passive
    (conserved in a uniform state), so theta^{xx} = lambda(0) P0 / lambda(t)."""
    mu, u0 = 0.05, 0.5
    res = []
    for dt in (0.002, 0.001):
        steps = int(12 / dt)
        s = _uniform_series(oracle_mod, 1, D, mu, u0, steps, dt, ["n", "lambda", "uz", "thzz", "ez"])
        n, lam, uz, thzz, ez = s.T
        assert np.abs(uz).max() > 0.45
        th00 = uz * uz * thzz
        energy = n * lam + th00 + 0.5 * ez * ez
        gam = 1 / np.sqrt(1 - uz * uz)
        g0 = 1 / np.sqrt(1 - u0 * u0)
        p0 = (n[0] / g0) * mu
        thxx = lam[0] * p0 / lam if D == 3.0 else 0.0 * lam
        hh = n / lam
        # eq. traces3: theta^00 - sum theta^{ii} = h (1 - (n0/h)^2), n0 = n / gamma
        resid = th00 - thzz - 2 * thxx - hh * (1 - (n / gam / hh) ** 2)
        res.append((np.abs(energy - energy[0]).max() / energy[0], np.abs(resid).max() / (D * mu)))
    (e1, r1), (e2, r2) = res
    assert e2 <= 1e-3 and abs(e1 / e2 - 2) <= 0.1
    assert r2 <= 0.03 and abs(r1 / r2 - 2) <= 0.1
