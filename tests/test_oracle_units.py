"""Pins of the oracle's per-node functions against what the paper fixes.

- Equilibrium (Sec. 2.2, eq. ade-feq): its zeroth, first and second discrete
  moments must equal A, A u and A (nu^2 I + u u) exactly (moment matching).
- LEC recovery (Sec. 3.1): building the advected momentum from a chosen p and
  recovering must return p (round trip), for D = 1 and D = 3.
- WARMC recovery (Sec. 4.1, App. A): round trip of (n, lambda, u, theta) and
  the mass-shell identities U_nu theta^{mu nu} = 0 (eq. traces4).
- Rest-state lambda (eq. traces3): lambda - 1/lambda = D mu.
- Longitudinal pressure read-out (App. A item 3) against a double boost
  (eq. double-boost) of a rest-frame tensor diag(0, Pperp, Pperp, Ppar).
"""
import numpy as np
import pytest

# Stencil velocities in the oracle's documented order (z, x components).
E1 = np.array([[0], [1], [-1]])
E2 = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [1, 1], [-1, -1], [1, -1], [-1, 1]])


@pytest.mark.parametrize("dims", [1, 2])
def test_feq_moment_matching(oracle_mod, dims):
    rng = np.random.default_rng(1)
    lam = 10.0
    nu2 = lam * lam / 3.0
    E = E1 if dims == 1 else E2
    for _ in range(200):
        A = rng.uniform(-2, 3)
        uz = rng.uniform(-0.9, 0.9)
        ux = rng.uniform(-0.9, 0.9) if dims == 2 else 0.0
        f = oracle_mod.feq(dims, A, uz, ux, lam)
        u = np.array([uz, ux][:dims])
        xi = lam * E[:, :dims]
        tol = 1e-12 * max(1.0, abs(A)) * lam * lam
        assert abs(f.sum() - A) <= 1e-12 * max(1.0, abs(A))
        assert np.allclose(xi.T @ f, A * u, rtol=0, atol=1e-12 * lam * max(1, abs(A)))
        second = (xi.T * f) @ xi
        assert np.allclose(second, A * (nu2 * np.eye(dims) + np.outer(u, u)), rtol=0, atol=tol)


def test_feq_rest_weights(oracle_mod):
    """At u = 0 the equilibrium is w_i A: D1Q3 and D2Q9 weights are the exact
    projections of the 19-velocity stencil of Fig. 1 (1/3, 1/18, 1/36)."""
    w19 = {}
    vel = [(0, 0, 0)]
    for a in range(3):
        for s in (1, -1):
            v = [0, 0, 0]; v[a] = s; vel.append(tuple(v))
    for a in range(3):
        for b in range(a + 1, 3):
            for s in (1, -1):
                for t in (1, -1):
                    v = [0, 0, 0]; v[a] = s; v[b] = t; vel.append(tuple(v))
    assert len(vel) == 19
    for v in vel:
        w19[v] = 1 / 3 if v == (0, 0, 0) else (1 / 18 if sum(map(abs, v)) == 1 else 1 / 36)
    w1 = {}
    w2 = {}
    for v, w in w19.items():
        w1[v[2]] = w1.get(v[2], 0) + w
        w2[(v[2], v[0])] = w2.get((v[2], v[0]), 0) + w
    f1 = oracle_mod.feq(1, 1.0, 0.0, 0.0, 10.0)
    assert np.allclose(f1, [w1[e[0]] for e in E1], rtol=0, atol=1e-15)
    f2 = oracle_mod.feq(2, 1.0, 0.0, 0.0, 10.0)
    assert np.allclose(f2, [w2[(e[0], e[1])] for e in E2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("D", [1.0, 3.0])
def test_lec_recovery_round_trip(oracle_mod, D):
    rng = np.random.default_rng(2)
    for _ in range(300):
        mu = 10 ** rng.uniform(-4, -1)
        n = rng.uniform(0.2, 3.0) if D == 3.0 else rng.uniform(0.2, 2.0)
        p = rng.uniform(-3, 3, size=2)
        g = np.sqrt(1 + p @ p)
        n0 = n / g
        h = 1 + (1 + D / 2) * mu * n0 ** (2 / D)
        A1 = h * n * p
        uz, ux, gam, it = oracle_mod.lec_recover(n, A1[0], A1[1], D, mu)
        u = p / g
        assert it > 0
        assert abs(uz - u[0]) <= 1e-14 and abs(ux - u[1]) <= 1e-14
        assert abs(gam - g) <= 1e-13 * g


def test_lec_recovery_fallback(oracle_mod):
    """D = 1 dense relativistic cell where the plain fixed point does not
    contract: the bracketed fallback must still return a root."""
    D, mu, n = 1.0, 0.1, 7.0
    P = 3.0
    uz, ux, gam, it = oracle_mod.lec_recover(n, P * n, 0.0, D, mu)
    p = uz * gam
    h = 1 + (1 + D / 2) * mu * (n / np.sqrt(1 + p * p)) ** (2 / D)
    assert abs(p * h - P) <= 1e-12 * P


def _warm_state(rng, dims):
    n = rng.uniform(0.5, 2.0)
    lam = rng.uniform(0.9, 1.2)
    uz, ux = rng.uniform(-0.5, 0.5), (rng.uniform(-0.5, 0.5) if dims == 2 else 0.0)
    th = rng.uniform(0.001, 0.1, size=4)
    th[3] = rng.uniform(-0.01, 0.01) if dims == 2 else 0.0
    if dims == 1:
        th[1] = th[2] = 0.0
    return n, lam, uz, ux, th


@pytest.mark.parametrize("dims", [1, 2])
def test_warmc_recovery_round_trip(oracle_mod, dims):
    rng = np.random.default_rng(3)
    for _ in range(200):
        n, lam, uz, ux, (thzz, thxx, thyy, thxz) = _warm_state(rng, dims)
        if dims == 1:
            A = [n, n * lam, n * lam * uz, lam * thzz]
        else:
            A = [n, n * lam, n * lam * uz, n * lam * ux, lam * thzz, lam * thxx, lam * thyy,
                 lam * thxz]
        o = oracle_mod.warmc_recover(dims, A)
        assert np.allclose(o[:7], [lam, uz, ux, thzz, thxx, thyy, thxz], rtol=1e-14, atol=1e-16)
        # eq. traces4: U_nu theta^{mu nu} = 0 with U = gamma (1, u), metric (+,-,-,-)
        th = np.zeros((4, 4))
        th[0, 0] = o[9]
        th[0, 3] = th[3, 0] = o[7]
        th[0, 1] = th[1, 0] = o[8]
        th[3, 3], th[1, 1], th[2, 2] = o[3], o[4], o[5]
        th[1, 3] = th[3, 1] = o[6]
        Ulow = np.array([1.0, -ux, 0.0, -uz])
        assert np.allclose(th @ Ulow, 0.0, atol=1e-15)
        assert abs(o[10] - lam * uz) <= 1e-14 and abs(o[11] - lam * ux) <= 1e-14


@pytest.mark.parametrize("D", [1.0, 3.0])
def test_lambda0_trace_condition(oracle_mod, D):
    for mu in [1e-6, 1e-3, 0.04, 0.1, 0.5]:
        lam = oracle_mod.lambda0(mu, D)
        n = 1.3
        h = n / lam
        # eq. traces3 at rest: theta^mu_mu = -D n mu = h (1 - (n0/h)^2), n0 = n
        assert abs(-D * n * mu - h * (1 - lam * lam)) <= 1e-14 * max(1, n)
        assert lam > 1


def _boost(ux, uz):
    """Lorentz boost from the rest frame to the lab, fluid velocity (ux, 0, uz)."""
    v = np.array([ux, 0.0, uz])
    v2 = v @ v
    g = 1 / np.sqrt(1 - v2)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = g * v
    L[1:, 0] = g * v
    if v2 > 0:
        L[1:, 1:] += (g - 1) * np.outer(v, v) / v2
    return L


def test_ppar_double_boost_round_trip(oracle_mod):
    rng = np.random.default_rng(4)
    for _ in range(200):
        pperp, ppar = rng.uniform(0.001, 0.1, size=2)
        ux, uz = rng.uniform(-0.6, 0.6, size=2)
        if ux * ux + uz * uz >= 0.95:
            continue
        # order (t, x, y, z); rest-frame theta_0 = diag(0, Pperp, Pperp, Ppar)
        th0 = np.diag([0.0, pperp, pperp, ppar])
        L = _boost(ux, uz)
        th = L @ th0 @ L.T
        got = oracle_mod.ppar(th[1, 1], th[2, 2], th[3, 3], th[0, 0], ux, uz)
        assert abs(got - ppar) <= 1e-13
        assert abs(th[2, 2] - pperp) <= 1e-15  # P_perp = theta^{yy}
