"""Hand-written discrete adjoint of the 2D local-equilibrium step: gradient of
the witness E_z with respect to the driver's slice weights, against central
finite differences of the FP64 oracle and of the FP64 kernel forward, an
exact identity of the linear regime, and itself (checkpoint interval,
storage precision, the autograd wrapper)."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

LP = 2 * math.pi


def _small(**kw):
    d = LP / 32
    cfg = dict(nz=64, nx=24, delta=d, dt=0.1 * d, tau_tilde=0.53, storage="fp64", mu=1e-2, alpha=0.5,
               sigma_z=0.5, sigma_x=0.5, z0=3.0, slice_zmin=-1.5, slice_zmax=1.5, steps=120,
               witness_behind=0.5 * LP)
    cfg.update(kw)
    return cfg


def _weights(n, seed=1):
    from paper_2309_04872_amd import workloads

    return workloads.slice_weights(n, 0.5, 1.5, seed)


def _oracle_loss(cfg, w):
    from paper_2309_04872_amd.adjoint import witness_slot

    o = oracle.Oracle(2, cfg["nz"], cfg["nx"], delta=cfg["delta"], dt=cfg["dt"], tau_tilde=cfg["tau_tilde"],
                      closure=oracle.LEC, dvel=3.0, mu=cfg["mu"], alpha=cfg["alpha"], sigma_z=cfg["sigma_z"],
                      sigma_x=cfg["sigma_x"], z0=cfg["z0"], slice_w=w, slice_zmin=cfg["slice_zmin"],
                      slice_zmax=cfg["slice_zmax"])
    o.init()
    o.step(cfg["steps"])
    ez = o.get("ez_yee")
    i, j0 = witness_slot(cfg)
    return 0.5 * (ez[j0, i] + ez[j0 + 1, i])


def _fd(loss, w, h=1e-4, which=None):
    g = np.zeros(len(w))
    for s in (range(len(w)) if which is None else which):
        e = np.zeros(len(w))
        e[s] = h
        g[s] = (loss(w + e) - loss(w - e)) / (2 * h)
    return g


def test_adjoint_matches_oracle_fd():
    from paper_2309_04872_amd.adjoint import loss_and_grad

    cfg = _small()
    w = _weights(8)
    loss, g = loss_and_grad(cfg, w, every=50)
    lo = _oracle_loss(cfg, w)
    g_fd = _fd(lambda v: _oracle_loss(cfg, v), w)
    print("loss", loss, "oracle", lo, flush=True)
    print("adjoint", g, "\nfd     ", g_fd, flush=True)
    assert abs(loss - lo) <= 1e-10 * abs(lo)
    assert np.max(np.abs(g)) > 1e-4
    assert np.max(np.abs(g - g_fd)) <= 1e-6 * np.max(np.abs(g_fd))


def test_adjoint_matches_kernel_fd_periodic_and_open():
    """Both boundary rules (periodic along z, open along x) and a driver strong
    enough for the recovery's nonlinearity to matter."""
    from paper_2309_04872_amd.adjoint import forward_loss, loss_and_grad

    cfg = _small(alpha=2.0, bc_z="periodic", steps=90)
    w = _weights(8, seed=2)
    _, g = loss_and_grad(cfg, w, every=30)
    g_fd = _fd(lambda v: forward_loss(cfg, v), w)
    print("adjoint", g, "\nfd     ", g_fd, flush=True)
    assert np.max(np.abs(g - g_fd)) <= 1e-6 * np.max(np.abs(g_fd))


@pytest.mark.parametrize("nslices", [8, 2000])
def test_adjoint_linear_regime_identity(nslices):
    """For a weak driver the witness field is linear and homogeneous in the
    weights (a plasma at rest without driver stays at rest), so
    loss(w) = sum_s w_s d loss / d w_s up to O(alpha^2). 2000 slices: more
    slices than columns in the bunch window, most of them empty."""
    from paper_2309_04872_amd.adjoint import loss_and_grad

    cfg = _small(alpha=1e-6)
    w = _weights(nslices, seed=3)
    loss, g = loss_and_grad(cfg, w, every=40)
    print("loss", loss, "w.g", float(w @ g), flush=True)
    assert abs(loss - w @ g) <= 1e-6 * abs(loss)


def test_adjoint_checkpoint_interval_bitwise():
    from paper_2309_04872_amd.adjoint import loss_and_grad

    cfg = _small(steps=70)
    w = _weights(8, seed=4)
    _, g1 = loss_and_grad(cfg, w, every=70)
    _, g2 = loss_and_grad(cfg, w, every=9)
    assert np.array_equal(g1, g2)


def test_autograd_function():
    import torch

    from paper_2309_04872_amd.adjoint import loss_and_grad, witness_field

    cfg = _small(steps=60)
    w = _weights(8, seed=5)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    loss = witness_field(wt, cfg, 25)
    (3.0 * loss).backward()
    ref_loss, ref_g = loss_and_grad(cfg, w, every=25)
    assert float(loss.detach()) == ref_loss
    # the seed 3 * 1/2 instead of 1/2 rounds differently along the way
    assert np.allclose(wt.grad.numpy(), 3.0 * ref_g, rtol=1e-12, atol=0)


def test_adjoint_full_size():
    """The differentiable workload: 1024 x 256, 2000 steps, 64 slices,
    checkpoints every 100 steps. FP64 adjoint against central differences of
    the FP64 forward on sampled slices; the FP32-forward gradient against the
    FP64 one."""
    from paper_2309_04872_amd import workloads
    from paper_2309_04872_amd.adjoint import adjoint_config, forward_loss, loss_and_grad

    w = workloads.slice_weights(64, 0.5, 1.5, 0)
    c64 = adjoint_config(storage="fp64")
    loss64, g64 = loss_and_grad(c64, w, every=100)
    c32 = adjoint_config(storage="fp32")
    loss32, g32 = loss_and_grad(c32, w, every=100)
    rel = np.linalg.norm(g32 - g64) / np.linalg.norm(g64)
    print("loss fp64", loss64, "fp32", loss32, "grad rel-L2 fp32 vs fp64", rel, flush=True)
    assert rel <= 1e-3
    top = list(np.argsort(-np.abs(g64))[:2]) + [0, 63]
    g_fd = _fd(lambda v: forward_loss(c64, v), w, which=top)
    for s in top:
        print("slice", s, "adjoint", g64[s], "fd", g_fd[s], flush=True)
        assert abs(g64[s] - g_fd[s]) <= 1e-6 * np.max(np.abs(g64))


@pytest.mark.parametrize("storage,bc_z", [("fp64", "open"), ("fp32", "periodic"), ("fp16dev", "open")])
def test_adjoint_post_records_bitwise(storage, bc_z):
    """The recompute from post-collision records (lbw_step_record_post, the
    reverse kernels streaming the populations themselves) gives the loss and
    the gradient of the canonical records bit for bit."""
    from paper_2309_04872_amd.adjoint import loss_and_grad

    cfg = _small(storage=storage, bc_z=bc_z, steps=70, alpha=2.0)
    w = _weights(8, seed=7)
    l1, g1 = loss_and_grad(cfg, w, every=30)
    l2, g2 = loss_and_grad(cfg, w, every=30, records="canonical")
    assert l1 == l2
    assert np.array_equal(g1, g2), (g1, g2)
    assert np.max(np.abs(g1)) > 0
