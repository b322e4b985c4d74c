"""Gradient of the accelerating field at a witness point behind the driver
with respect to the driver's per-slice current weights, by the hand-written
discrete adjoint of the 2D local-equilibrium step (lbw_adjoint_step in the C
ABI) with checkpoint-and-recompute. Argument marshalling and bookkeeping
only: every forward and adjoint step runs in the HIP library.

The loss is E_z on the Yee grid at the witness: the mean of the two E_z
values of the axial pair of rows x = -delta/2, +delta/2 at the slot whose
centre (i + 1/2) delta is nearest to z_driver(T) - distance.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib, trace
from .sim import LbwError, Sim


def witness_slot(cfg):
    """(i, j0): E_z slot along z and the lower of the two axial rows."""
    t_end = cfg["steps"] * cfg["dt"]
    zw = cfg["z0"] + t_end - cfg["witness_behind"]
    i = int(round(zw / cfg["delta"] - 0.5))
    if not 0 <= i < cfg["nz"] - 1:
        raise ValueError("witness point outside the grid")
    return i, cfg["nx"] // 2 - 1


class _Run:
    """One configured simulation plus its checkpoint storage."""

    def __init__(self, cfg, weights):
        self.cfg = cfg
        self.w = np.ascontiguousarray(weights, dtype=np.float64)
        self.sim = Sim(2, cfg["nz"], cfg["nx"], delta=cfg["delta"], dt=cfg["dt"], tau_tilde=cfg["tau_tilde"],
                       closure="lec", dvel=3.0, storage=cfg["storage"], bc_z=cfg.get("bc_z", "open"),
                       bc_x=cfg.get("bc_x", "open"))

    def start(self):
        c = self.cfg
        self.sim.init_plasma(c["mu"])
        self.sim.init_driver(c["alpha"], c["sigma_z"], c["sigma_x"], z0=c["z0"], slice_w=self.w,
                             slice_zmin=c["slice_zmin"], slice_zmax=c["slice_zmax"])
        return self

    def loss(self):
        i, j0 = witness_slot(self.cfg)
        ez = self.sim.field("ez", at_nodes=False)
        return 0.5 * (ez[j0, i] + ez[j0 + 1, i])


def forward_loss(cfg, weights):
    """The loss alone (no checkpoints)."""
    r = _Run(cfg, weights).start()
    r.sim.step(cfg["steps"])
    return r.loss()


_TIMING = {}


def last_timing():
    """Phase times (ms) of the last loss_and_grad(..., timing=True)."""
    return dict(_TIMING)


def loss_and_grad(cfg, weights, every=100, grad_out=1.0, timing=False, records="post"):
    """Loss and d loss / d weights (numpy), checkpoints every ``every`` steps.
    timing: record HIP events on the simulation's stream around the forward,
    the recompute and the reverse steps (last_timing()). records: "post"
    recomputes a segment recording each fused launch's output
    (lbw_step_record_post, no per-step canonicalisation) for
    lbw_adjoint_step_post; "canonical" records canonical states
    (lbw_step_record) for lbw_adjoint_step. Both give the same bits."""
    if records not in ("post", "canonical"):
        raise ValueError("records must be 'post' or 'canonical'")
    import torch

    r = _Run(cfg, weights).start()
    sim, lib, h = r.sim, r.sim._lib, r.sim._h
    steps = cfg["steps"]
    sb = sim.state_device_bytes()
    ev = {}

    def mark(name):
        if timing:
            e = torch.cuda.Event(enable_timing=True)
            e.record(sim.stream)
            ev.setdefault(name, []).append(e)

    ckpt = {}
    mark("fwd0")
    with trace.marker("adjoint forward"):
        for n0 in range(0, steps, every):
            ckpt[n0] = sim.save_state_device()
            sim.step(min(every, steps - n0))
    mark("fwd1")
    loss = r.loss()

    dev = sim.device
    nc = sim.ncell
    adj = torch.zeros(lib.lbw_adjoint_bytes(h) // 8, dtype=torch.float64, device=dev)
    K = (adj.numel() // nc) - 3
    i, j0 = witness_slot(cfg)
    ez_off = K * nc
    adj[ez_off + j0 * cfg["nz"] + i] = 0.5 * grad_out
    adj[ez_off + (j0 + 1) * cfg["nz"] + i] = 0.5 * grad_out
    grad = torch.zeros(len(r.w), dtype=torch.float64, device=dev)
    scratch = torch.empty(lib.lbw_adjoint_workspace_bytes(h), dtype=torch.uint8, device=dev)
    buf = torch.empty((every + 1) * sb, dtype=torch.uint8, device=dev)
    vp = ctypes.c_void_p

    def check(rc):
        if rc != 0:
            raise LbwError(rc, lib.lbw_last_error(h).decode())

    for n0 in sorted(ckpt, reverse=True):
        n1 = min(n0 + every, steps)
        mark("rec0")
        with trace.marker("adjoint recompute"):
            sim.load_state_device(ckpt[n0], n0)
            if records == "post":
                sim.step_record_post(n1 - n0, buf, sb)
            else:
                sim.save_state_device(buf[0:sb])
                sim.step_record(n1 - n0, buf[sb:], sb)
        mark("rec1")
        mark("adj0")
        with trace.marker("adjoint reverse"):
            for n in range(n1 - 1, n0 - 1, -1):
                m = n - n0
                if records == "post":
                    # state n's populations: the checkpoint, or record m - 1 (post-collision)
                    pops_n = ckpt[n0] if m == 0 else buf[(m - 1) * sb:]
                    check(lib.lbw_adjoint_step_post(h, vp(pops_n.data_ptr()), int(m > 0),
                                                    vp(buf[m * sb:].data_ptr()), n, vp(adj.data_ptr()),
                                                    vp(grad.data_ptr()), vp(scratch.data_ptr())))
                else:
                    check(lib.lbw_adjoint_step(h, vp(buf[m * sb:].data_ptr()), vp(buf[(m + 1) * sb:].data_ptr()),
                                               n, vp(adj.data_ptr()), vp(grad.data_ptr()), vp(scratch.data_ptr())))
        mark("adj1")
    check(lib.lbw_adjoint_init_fields(h, vp(adj.data_ptr()), vp(grad.data_ptr()), vp(scratch.data_ptr())))
    torch.cuda.synchronize(dev)
    if timing:
        def total(a, b):
            return sum(x.elapsed_time(y) for x, y in zip(ev[a], ev[b]))
        _TIMING.clear()
        _TIMING.update(forward_ms=total("fwd0", "fwd1"), recompute_ms=total("rec0", "rec1"),
                       adjoint_ms=total("adj0", "adj1"), adjoint_steps=steps)
    g = grad.cpu().numpy()
    sim.close()
    return loss, g


def _autograd_function():
    import torch

    class WitnessField(torch.autograd.Function):
        """loss = E_z at the witness; input: slice weights (CPU or device
        tensor), cfg: the workload dict, every: checkpoint interval."""

        @staticmethod
        def forward(ctx, weights, cfg, every):
            w = weights.detach().cpu().numpy().astype(np.float64)
            ctx.cfg, ctx.every, ctx.w = cfg, every, w
            ctx.device, ctx.dtype = weights.device, weights.dtype
            return torch.tensor(forward_loss(cfg, w), dtype=weights.dtype, device=weights.device)

        @staticmethod
        def backward(ctx, gout):
            _, g = loss_and_grad(ctx.cfg, ctx.w, ctx.every, grad_out=float(gout))
            return torch.tensor(g, dtype=ctx.dtype, device=ctx.device), None, None

    return WitnessField


_WF = None


def witness_field(weights, cfg, every=100):
    """Differentiable loss: torch.autograd.Function over the slice weights."""
    global _WF
    if _WF is None:
        _WF = _autograd_function()
    return _WF.apply(weights, cfg, every)


def adjoint_config(storage=None, **overrides):
    """The differentiable wake workload (1024 x 256, 2000 steps, 64 slices over
    zeta in [-3 sigma_z, 3 sigma_z), witness 1.5 lambda_p behind the driver)."""
    from . import workloads

    w = workloads.workload("wake2d_lec_adjoint")
    cfg = dict(nz=w["nz"], nx=w["nx"], delta=w["delta"], dt=w["dt"], tau_tilde=w["tau_tilde"],
               storage=storage or w["storage"], mu=w["mu"], alpha=w["alpha"], sigma_z=w["sigma_z"],
               sigma_x=w["sigma_x"], z0=w["z0"], slice_zmin=-3.0 * w["sigma_z"],
               slice_zmax=3.0 * w["sigma_z"], steps=w["steps"], witness_behind=1.5 * 2 * math.pi)
    cfg.update(overrides)
    return cfg
