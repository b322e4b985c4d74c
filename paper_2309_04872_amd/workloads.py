"""Seeded synthetic inputs and the named workloads (configuration data only,
none of the method's arithmetic). Shared by the tests, the benchmark and the
oracle-side checks; it imports neither the HIP binding nor the oracle.

The paper simulates no dataset: every input is a uniform plasma (optionally
with seeded density noise) and an analytic driver bunch (Sec. 5). Grid
spacings are fractions of the plasma wavelength lambda_p = 2 pi / k_p; the
time step is delta / 10 and tau~ is 0.52 (1D) / 0.53 (2D), the paper's ratios.
"""
from __future__ import annotations

import math

import numpy as np

LAMBDA_P = 2.0 * math.pi


def density_noise(shape, amp, seed):
    """n = 1 + amp * U(-1, 1), numpy PCG64 stream of ``seed``."""
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.uniform(-1.0, 1.0, size=shape)


def slice_weights(nslices, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=nslices)


def batch_scan(n_inst=256, seed=0):
    """Parameter scan of independent 1D instances: Nz ~ U{1024..16384},
    n_b/n0 log-uniform [0.01, 3], sigma_z ~ U[0.3, 2], T log-uniform
    [1e-4, 1e-1] m c^2, closures alternating."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        out.append(dict(
            nz=int(rng.integers(1024, 16385)),
            alpha=float(10 ** rng.uniform(math.log10(0.01), math.log10(3.0))),
            sigma_z=float(rng.uniform(0.3, 2.0)),
            mu=float(10 ** rng.uniform(-4.0, -1.0)),
            closure="lec" if i % 2 == 0 else "warmc",
        ))
    return out


# Named workloads: grid, closure, storage, plasma, driver, length.
WORKLOADS = {
    "wake1d_lec_fp64": dict(
        dims=1, nz=4096, nx=1, delta=LAMBDA_P / 128, closure="lec", dvel=1.0, storage="fp64",
        mu=1e-3, noise=1e-8, seed=0, alpha=0.1, sigma_z=0.5, sigma_x=1.0, steps=4096),
    "wake2d_lec_fp32": dict(
        dims=2, nz=2048, nx=512, delta=LAMBDA_P / 64, closure="lec", dvel=3.0, storage="fp32",
        mu=1e-2, noise=0.0, seed=0, alpha=1.0, sigma_z=1.0, sigma_x=0.5, steps=8000),
    "wake2d_warmc": dict(
        dims=2, nz=4096, nx=1024, delta=LAMBDA_P / 64, closure="warmc", dvel=3.0, storage="fp64",
        mu=5e-2, noise=0.0, seed=0, alpha=2.0, sigma_z=1.0, sigma_x=0.5, steps=8000),
    # The paper's 3D3V production case (Sec. 5, Fig. 4 and 5): axisymmetric
    # (z, r), L_z = 30, L_r = 6 at delta = 0.01 (3000 x 600 nodes), 30 000
    # steps, mu = 0.04 (20 keV), Q~ = 0.5 with sigma_z = sigma_r = 25 um at
    # n_i = 1e16 cm^-3 (0.4704 / k_p, rms convention).
    "wake_axi_lec": dict(
        dims=2, geom="axi", nz=3000, nx=600, delta=0.01, closure="lec", dvel=3.0, storage="fp64",
        mu=0.04, noise=0.0, seed=0, alpha=None, q_tilde=0.5, sigma_z=0.4704, sigma_x=0.4704,
        steps=30000),
    "wake_axi_warmc": dict(
        dims=2, geom="axi", nz=3000, nx=600, delta=0.01, closure="warmc", dvel=3.0, storage="fp64",
        mu=0.04, noise=0.0, seed=0, alpha=None, q_tilde=0.5, sigma_z=0.4704, sigma_x=0.4704,
        steps=30000),
    "wake2d_lec_adjoint": dict(
        dims=2, nz=1024, nx=256, delta=LAMBDA_P / 64, closure="lec", dvel=3.0, storage="fp32",
        mu=1e-2, noise=0.0, seed=0, alpha=0.5, sigma_z=1.0, sigma_x=0.5, steps=2000,
        nslices=64, slice_lo=0.5, slice_hi=1.5),
}


def alpha_of_q_tilde(q_tilde, sigma_z, sigma_r, D=3):
    """Peak bunch density n_b / n_i for the normalised charge
    Q~ = (2 pi)^{D/2} sigma_z sigma_r^{D-1} alpha (eq. Qtilde, plasma units)."""
    return q_tilde / ((2.0 * math.pi) ** (D / 2.0) * sigma_z * sigma_r ** (D - 1))


def workload(name, **overrides):
    w = dict(WORKLOADS[name])
    w.update(overrides)
    w.setdefault("geom", "slab")
    if w.get("alpha") is None:
        w["alpha"] = alpha_of_q_tilde(w["q_tilde"], w["sigma_z"], w["sigma_x"])
    w["dt"] = 0.1 * w["delta"]
    w["tau_tilde"] = 0.52 if w["dims"] == 1 else 0.53
    w["z0"] = 6.0 * w["sigma_z"]
    return w


def initial_density(w):
    shape = (w["nx"], w["nz"])
    if w.get("noise", 0.0) > 0.0:
        return density_noise(shape, w["noise"], w["seed"])
    return np.ones(shape)


# The batched 1D scan: 256 instances of batch_scan(seed 0), delta = lambda_p/128,
# D = 1, open boundaries, 4096 steps.
BATCH_SCAN = dict(n_inst=256, seed=0, delta=LAMBDA_P / 128, dvel=1.0, steps=4096)


def batch_instances(n_inst=None, seed=None):
    """Instance descriptors of the batched scan (keys of the batch binding)."""
    n_inst = BATCH_SCAN["n_inst"] if n_inst is None else n_inst
    seed = BATCH_SCAN["seed"] if seed is None else seed
    delta = BATCH_SCAN["delta"]
    out = []
    for d in batch_scan(n_inst, seed):
        out.append(dict(d, delta=delta, dt=0.1 * delta, tau_tilde=0.52, dvel=BATCH_SCAN["dvel"],
                        bc="open", z0=6.0 * d["sigma_z"]))
    return out
