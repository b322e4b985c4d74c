"""Benchmark of the fused LB + field step on one MI355X.

Workload (default): the 2D warm-closure wake, 4096 x 1024 nodes,
delta = lambda_p/64, FP64 populations, mu = 5e-2, bi-Gaussian driver
(sigma_z = 1, sigma_x = 0.5, n_b/n0 = 2): the largest configuration, at the
paper's presumed precision. One "step" is one pass of the whole hot path over
the grid: streaming, moments, recovery, forcing, collision and the Yee field
update, i.e. one fused kernel launch. Inputs are synthetic (uniform plasma,
analytic bunch) and resident in HBM before the timed region. Without --steps
it runs 400 steps: the warm closure's temperature theta^zz first turns
negative near t = 4.5 (step ~459) in this strongly driven case, in the oracle
as in the kernels.

Prints one JSON line: MLUPS of the whole job, the HBM roofline of the fused
kernel (algorithmic bytes per lattice update over its HIP-event-measured
average duration), the CPU oracle timed on the host's cores, and for the
default workload the FP32 and FP16-deviation storage variants: their fused
kernel time and the relative L2 error of density perturbation, momentum and
E_z against the FP64 run after 400 steps.

Other workloads (--workload): wake2d_lec_fp32, wake1d_lec_fp64, wake2d_warmc
(--storage fp64 | fp32 | fp16dev), batch1d_scan, wake2d_lec_adjoint, and wake_axi_lec /
wake_axi_warmc, the paper's own axisymmetric production case (3000 x 600
nodes, 30 000 steps, FP64), the one workload for which the paper states a
throughput: there vs_baseline is the ratio to it (a 96-core CPU cluster;
context, not target).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per lattice update of the fused step: every population
# read once and written once, the three Yee arrays (FP64) read once and
# written once, the warm closure's lagged values read and written in place.
def bytes_per_lu(dims, closure, storage):
    K = (1 + dims) if closure == "lec" else (4 if dims == 1 else 8)
    Q = 3 if dims == 1 else 9
    sb = {"fp64": 8, "fp32": 4, "fp16dev": 2}[storage]
    nf = 1 if dims == 1 else 3
    nlag = 0 if closure == "lec" else (3 if dims == 1 else 5)
    return 2 * K * Q * sb + 2 * nf * 8 + 2 * nlag * 8


# HBM-side bytes per launch of the fused kernel, measured with rocprofv3
# --pmc FETCH_SIZE and WRITE_SIZE and scaled by a 1 GiB copy
# (the summaries and commands are in profiles/k_step2d_*.md). FETCH_SIZE
# counts the L2's requests to memory, and the 256 MB last-level cache (MALL)
# sits behind that point: for grids whose state exceeds it (wake2d_warmc,
# 5.4 GB in FP64) the bytes are HBM bytes up to the re-reads that hit the
# MALL. Valid for the kernel as profiled; remove an entry when it changes.
TRAFFIC_BYTES_PER_LAUNCH = {
    ("wake2d_lec_fp32", "fp32"): 297.6e6,
    ("wake2d_lec_fp32", "fp64"): 552.5e6,
    ("wake2d_lec_fp32", "fp16dev"): 170.4e6,
    ("wake2d_warmc", "fp64"): 6081.6e6,
    ("wake2d_warmc", "fp32"): 3254.3e6,
    ("wake2d_warmc", "fp16dev"): 1876.7e6,
    ("wake_axi_lec", "fp64"): 1022.2e6,
    ("wake_axi_lec", "fp32"): 530.2e6,
    ("wake_axi_lec", "fp16dev"): 307.1e6,
    ("wake_axi_warmc", "fp64"): 2969.7e6,
    ("wake_axi_warmc", "fp32"): 1420.4e6,
    ("wake_axi_warmc", "fp16dev"): 861.7e6,
}


# The paper's own throughput on its 3D3V production case (Sec. 5): 3000 x 600
# nodes, 3e4 steps in about 182 min (LEC-LB) and 368 min (WARMC-LB) on 96 Xeon
# E5-2695 cores with MPI (precision not stated, FP64 presumed).
PAPER_MINUTES = {"wake_axi_lec": 182, "wake_axi_warmc": 368}
PAPER_MLUPS = {k: 3000 * 600 * 30000 / (m * 60) / 1e6 for k, m in PAPER_MINUTES.items()}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_bandwidth_gbs(stream, nbytes=1 << 30, reps=10):
    """Practical HBM ceiling: read + write bytes over the duration of the
    library's streaming copy (lbw_stream_copy: one 16-byte non-temporal load
    and store per thread) of nbytes, HIP events on ``stream``."""
    import ctypes

    import torch

    from paper_2309_04872_amd import _lib

    L = _lib.load()
    with torch.cuda.stream(stream):
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
    args = (ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(x.data_ptr()), nbytes, ctypes.c_void_p(stream.cuda_stream))
    if L.lbw_stream_copy(*args) != 0:
        raise RuntimeError("lbw_stream_copy failed")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        L.lbw_stream_copy(*args)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    if not torch.equal(x, y):
        raise RuntimeError("lbw_stream_copy produced a wrong copy")
    del x, y
    return 2 * nbytes / (ms / 1e3) / 1e9


def one_thread(fn, seconds):
    """MLUPS of fn(cells_steps_counter) on one oracle thread."""
    import oracle

    n0 = oracle.num_threads()
    oracle.set_threads(1)
    try:
        return fn(seconds)
    finally:
        oracle.set_threads(n0)


def cpu_baseline(w, budget_s=12.0):
    """The CPU oracle (test infrastructure, FP64) on a bounded sample of the
    same workload: the full grid for as many steps as fit the budget."""
    import oracle

    o = oracle.Oracle(w["dims"], w["nz"], w["nx"], delta=w["delta"], dt=w["dt"],
                      tau_tilde=w["tau_tilde"], closure=0 if w["closure"] == "lec" else 1,
                      dvel=w["dvel"], mu=w["mu"], alpha=w["alpha"], sigma_z=w["sigma_z"],
                      sigma_x=w["sigma_x"], z0=w["z0"], geom=1 if w["geom"] == "axi" else 0)
    o.init()
    o.step(1)  # first touch of the arrays
    cells = w["nz"] * w["nx"]

    def run(seconds):
        t0 = time.perf_counter()
        n = 0
        while True:
            o.step(1)
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        return n, time.perf_counter() - t0

    n, dt = run(budget_s)
    n1, dt1 = one_thread(run, budget_s / 4)
    return {"value": cells * n / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle", "value_1core": cells * n1 / dt1 / 1e6, "cpu_model": cpu_model(),
            "sample": f"full {w['nx']}x{w['nz']} grid, {n} FP64 steps ({dt:.1f} s) of the same workload; "
                      f"{n1} steps on one thread ({dt1:.1f} s)"}


def cpu_baseline_adjoint(cfg, weights, budget_s=12.0):
    """The CPU oracle's route to the same gradient: central differences over
    the 64 slice weights need 2 x 64 forward runs of the whole workload. A
    bounded sample of one forward run (the full grid with the sliced driver,
    as many steps as fit the budget) is timed; the gradient rate is that
    forward rate over 128."""
    import oracle

    o = oracle.Oracle(2, cfg["nz"], cfg["nx"], delta=cfg["delta"], dt=cfg["dt"], tau_tilde=cfg["tau_tilde"],
                      closure=0, dvel=3.0, mu=cfg["mu"], alpha=cfg["alpha"], sigma_z=cfg["sigma_z"],
                      sigma_x=cfg["sigma_x"], z0=cfg["z0"], slice_w=weights, slice_zmin=cfg["slice_zmin"],
                      slice_zmax=cfg["slice_zmax"])
    o.init()
    o.step(1)
    cells = cfg["nz"] * cfg["nx"]
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        o.step(1)
        n += 1
    dt = time.perf_counter() - t0
    fwd = cells * n / dt / 1e6
    return {"value": fwd / 128, "unit": "MLUPS", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "forward_mlups": fwd,
            "sample": f"full {cfg['nx']}x{cfg['nz']} grid with the sliced driver, {n} FP64 forward steps "
                      f"({dt:.1f} s); a central-difference gradient over 64 slices takes 128 forward runs"}


def fd_fp64_gpu(cfg, weights):
    """The plain FP64 route on the GPU: central differences over the 64 slices
    with FP64 forward runs. One 2000-step FP64 forward run is timed (HIP
    events around lbw_step) and scaled by the 128 runs a gradient needs."""
    import torch

    from paper_2309_04872_amd import adjoint

    c = dict(cfg, storage="fp64")
    r = adjoint._Run(c, weights).start()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r.sim.step(c["steps"])
    e1.record()
    torch.cuda.synchronize()
    fwd_s = e0.elapsed_time(e1) / 1e3
    r.sim.close()
    cells = c["nz"] * c["nx"]
    return {"value": cells * c["steps"] / (128 * fwd_s) / 1e6, "unit": "MLUPS", "forward_s": fwd_s, "runs": 128,
            "kind": "central differences of FP64 forward runs on the GPU (one run timed, x 128)"}


# Steps a workload runs when --steps is not given, where its full length
# leaves the closure's range of validity: the strongly driven warm wake's
# temperature theta^zz first turns negative near t = 4.5 (step ~459), in the
# oracle as in the kernels, independently of dt and delta.
VALID_WINDOW_STEPS = {"wake2d_warmc": 400}


def precision_variants(w, steps=400):
    """The same workload with FP64, FP32 and FP16-deviation population
    storage: each run for ``steps`` steps from t = 0 (fused kernel timed with
    HIP events on the simulation's stream), then the relative L2 error of the
    density perturbation n - 1, the momentum densities n gamma u_z,
    n gamma u_x and the node E_z against the FP64 run."""
    import torch

    from paper_2309_04872_amd.sim import Sim

    cells = w["nz"] * w["nx"]
    out, ref = {}, None
    for storage in ("fp64", "fp32", "fp16dev"):
        s = Sim(w["dims"], w["nz"], w["nx"], delta=w["delta"], dt=w["dt"], tau_tilde=w["tau_tilde"],
                closure=w["closure"], dvel=w["dvel"], storage=storage, geom=w["geom"])
        s.init_plasma(w["mu"])
        s.init_driver(w["alpha"], w["sigma_z"], w["sigma_x"], z0=w["z0"])
        s.set_timing(True)
        s.step(steps)
        k_ms, k_n = s.get_timing()
        s.set_timing(False)
        got = {"n-1": s.read("n") - 1.0, "mz": s.read("mz"), "mx": s.read("mx"), "ez": s.field("ez")}
        s.close()
        del s
        torch.cuda.empty_cache()
        k_s = k_ms / k_n / 1e3
        blu = bytes_per_lu(w["dims"], w["closure"], storage)
        rec = {"kernel_avg_us": k_s * 1e6, "mlups_kernel": cells / k_s / 1e6, "bytes_per_lu": blu,
               "frac": blu * cells / k_s / 1e9 / HBM_PEAK_GBS, "steps": steps}
        if ref is None:
            ref = got
        else:
            rec["rel_l2_vs_fp64"] = {q: float(np.linalg.norm(got[q] - ref[q]) / np.linalg.norm(ref[q]))
                                     for q in got}
            rec["speedup_vs_fp64"] = out["fp64"]["kernel_avg_us"] / rec["kernel_avg_us"]
        out[storage] = rec
    return out


def batch_bytes_per_step(insts):
    """Algorithmic bytes of one step of the batched scan: per instance
    bytes_per_lu(1, closure, FP64) times its node count."""
    return sum(d["nz"] * bytes_per_lu(1, d["closure"], "fp64") for d in insts)


BATCH_TRAFFIC_PER_STEP = 30.97e6  # profiles/k_batch1d_batch1d_scan.md
BATCH_PASS_DEPTH = 16


def batch_sweeps(steps, depth=BATCH_PASS_DEPTH):
    """Sweeps of the whole state in one batched launch of ``steps`` steps:
    the first step alone, passes of ``depth`` steps, pairs, a last single
    step, and the closing canonicalisation (the kernel's pass schedule)."""
    if steps <= 0:
        return 0
    rest = steps - 1
    tail = rest % depth
    return 1 + rest // depth + tail // 2 + tail % 2 + 1


def sequential_fp64(insts, steps):
    """The same scan as plain single runs: every instance as its own 1D FP64
    simulation (lbw_create / lbw_step), one after another on the GPU; only the
    lbw_step calls are timed (HIP events), so allocation and initialisation
    stay outside."""
    import torch

    from paper_2309_04872_amd.sim import Sim

    total_ms = 0.0
    for d in insts:
        delta = 2 * np.pi / 128
        s = Sim(1, d["nz"], delta=delta, dt=0.1 * delta, tau_tilde=0.52, closure=d["closure"], dvel=1.0)
        s.init_plasma(d["mu"])
        if d["alpha"] != 0.0:
            s.init_driver(d["alpha"], d["sigma_z"], z0=6.0 * d["sigma_z"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        total_ms += e0.elapsed_time(e1)
        s.close()
    cells = sum(d["nz"] for d in insts)
    return {"value": cells * steps / (total_ms / 1e3) / 1e6, "unit": "MLUPS", "seconds": total_ms / 1e3,
            "kind": "single FP64 runs in sequence (lbw_step per instance)"}


def cpu_baseline_batch(insts, budget_s=12.0):
    """The CPU oracle on a bounded sample of the scan: its first instances in
    turn (alternating closures), 256 steps each, until the budget is spent."""
    import oracle

    cells_steps = 0
    used = []
    t0 = time.perf_counter()
    for d in insts:
        o = oracle.Oracle(1, d["nz"], 1, delta=d["delta"], dt=d["dt"], tau_tilde=d["tau_tilde"],
                          closure=0 if d["closure"] == "lec" else 1, dvel=d["dvel"], mu=d["mu"],
                          alpha=d["alpha"], sigma_z=d["sigma_z"], z0=d["z0"])
        o.init()
        o.step(256)
        cells_steps += d["nz"] * 256
        used.append(d["nz"])
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0

    def first(seconds):
        d = insts[0]
        o = oracle.Oracle(1, d["nz"], 1, delta=d["delta"], dt=d["dt"], tau_tilde=d["tau_tilde"],
                          closure=0 if d["closure"] == "lec" else 1, dvel=d["dvel"], mu=d["mu"],
                          alpha=d["alpha"], sigma_z=d["sigma_z"], z0=d["z0"])
        o.init()
        t1 = time.perf_counter()
        k = 0
        while time.perf_counter() - t1 < seconds:
            o.step(64)
            k += 64
        return d["nz"] * k / (time.perf_counter() - t1) / 1e6

    return {"value": cells_steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle", "value_1core": one_thread(first, budget_s / 4), "cpu_model": cpu_model(),
            "sample": f"first {len(used)} instances of the scan ({sum(used)} nodes), 256 FP64 steps each, "
                      f"{dt:.1f} s; one thread: the first instance"}


def bench_batch(args):
    import torch

    from paper_2309_04872_amd import workloads
    from paper_2309_04872_amd.batch import Batch

    insts = workloads.batch_instances()
    steps = args.steps if args.steps is not None else workloads.BATCH_SCAN["steps"]
    cells = sum(d["nz"] for d in insts)
    b = Batch(insts).init()
    if args.batch_config:
        # a fixed launch configuration instead of the autotuner (for profiled runs)
        threads, cpt = (int(v) for v in args.batch_config.split(","))
        b.set_config(threads, cpt)
    else:
        threads, cpt = b.autotune(probe_steps=20)
    sched = b.schedule()
    if args.warmup:
        b.step(args.warmup, graph=True)
    torch.cuda.synchronize()
    b.init()  # timed region: the scan from t = 0, inputs resident in HBM
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(b.stream)
    t0 = time.perf_counter()
    b.step(steps, graph=True)
    ev1.record(b.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    k_ms = b.last_ms()  # HIP events on the batch's stream around the one launch
    copy_gbs = copy_bandwidth_gbs(b.stream)
    bad = b.nonfinite()
    bps = batch_bytes_per_step(insts)
    # HBM-side bytes per step measured with rocprofv3 (FETCH_SIZE, WRITE_SIZE,
    # calibrated by a 1 GiB copy) for this kernel; the summary is in
    # profiles/k_batch1d_batch1d_scan.md
    traffic_per_step = BATCH_TRAFFIC_PER_STEP
    # the blocked algorithm reads and writes the state once per sweep, not
    # once per step: its algorithmic bytes per launch are bps x sweeps
    sweeps = batch_sweeps(steps)
    achieved = bps * sweeps / (k_ms / 1e3) / 1e9
    per_step_equiv = bps * steps / (k_ms / 1e3) / 1e9
    line = {
        "metric": "MLUPS (LB+field)",
        "value": cells * steps / (ms_total / 1e3) / 1e6,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_total / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "batch1d_scan", "instances": len(insts), "total_nodes": cells,
            "nz_range": [min(d["nz"] for d in insts), max(d["nz"] for d in insts)],
            "closures": "alternating lec / warmc", "populations": "fp64", "delta": "lambda_p/128",
            "steps_per_run": steps, "launches": 1, "hip_graph": True,
            "launch_config": {"threads": threads, "nodes_per_thread": cpt, "split": sched[2],
                              "workgroups": sched[3], "autotuned": not args.batch_config},
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            # measured on the full 4096-step launch (the pass schedule depends on the step count)
            "traffic": (traffic_per_step * steps
                        if traffic_per_step and steps == workloads.BATCH_SCAN["steps"] else None),
            "kernel": "k_batch1d",
            "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
            "kernel_avg_us": k_ms * 1e3, "bytes_per_step": bps, "sweeps": sweeps, "launches": 1,
            "per_step_equivalent_gbs": per_step_equiv,
            "note": "16 steps per pass: the state is read and written once per sweep, so achieved "
                    "counts bytes_per_step x sweeps; HBM is far from bounding the launch, which the "
                    "latency of the longest instance's passes on one compute unit does",
        },
        "wall_s": wall,
        "diagnostics": {"nonfinite_instances": int((bad > 0).sum())},
        # the same launch counting only the instances that stayed finite (the
        # strongly driven warm-closure ones that lose validity still cost
        # their full arithmetic)
        "value_finite_instances": sum(d["nz"] for d, k in zip(insts, bad) if k == 0) * steps
                                  / (ms_total / 1e3) / 1e6,
    }
    if not args.no_sequential:
        line["sequential_fp64"] = sequential_fp64(insts, steps)
    b.close()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_batch(insts, args.cpu_budget)
    print(json.dumps(line), flush=True)


# Algorithmic bytes per node of one reverse step of the adjoint: the FP64
# adjoint of the canonical state (K*Q = 27 population planes and the three
# Yee arrays) read once and written once, and the two saved forward states
# (steps n and n + 1: populations in the storage type, three FP64 Yee arrays)
# read once. 744 B with FP32 populations.
def adjoint_bytes_per_node(storage):
    sb = {"fp64": 8, "fp32": 4, "fp16dev": 2}[storage]
    P = 27
    return 2 * (P + 3) * 8 + 2 * (P * sb + 3 * 8)


# What the implementation's eight reverse-step kernels read and write per node
# (full planes), for comparison with the algorithmic bytes above.
def adjoint_impl_bytes_per_node(storage):
    sb = {"fp64": 8, "fp32": 4, "fp16dev": 2}[storage]
    P = 27
    maxwell = 3 * 8 + P * sb + 2 * P * 8 + 8       # adj E, B; f^{n+1}; adj f (+=); adj B'
    stream = P * 8 + P * 8 + 2 * 8                  # adj f -> adj f*, adj F
    collide = P * sb + 3 * 8 + P * 8 + 2 * 8 + P * 8 + 3 * 8
    bh = 2 * 8 + 8                                  # adj Bh from adj B' and adj Bn_y
    xsum = 2 * 8 + 8
    fields = 6 * 8 + 3 * 8                          # adj E^n, B^{n-1/2}
    return maxwell + stream + collide + bh + xsum + fields


def bench_adjoint(args):
    import torch

    from paper_2309_04872_amd import adjoint, workloads

    storage = args.storage or "fp32"
    cfg = adjoint.adjoint_config(storage=storage)
    if args.steps is not None:
        cfg["steps"] = args.steps
    w = workloads.slice_weights(64, 0.5, 1.5, 0)
    cells = cfg["nz"] * cfg["nx"]
    if args.warmup:  # one untimed gradient of the same workload
        adjoint.loss_and_grad(cfg, w, every=100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss, g = adjoint.loss_and_grad(cfg, w, every=100, timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = adjoint.last_timing()
    step_s = tm["adjoint_ms"] / tm["adjoint_steps"] / 1e3
    bpn = adjoint_bytes_per_node(storage)
    achieved = bpn * cells / step_s / 1e9
    line = {
        "metric": "MLUPS (LB+field)",
        "value": cells * cfg["steps"] / wall / 1e6,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": cfg["steps"],
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / cfg["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16"}[storage],
        "data": "synthetic",
        "config": {
            "workload": "wake2d_lec_adjoint", "nz": cfg["nz"], "nx": cfg["nx"], "closure": "lec",
            "populations": storage, "adjoint": "f64", "slices": 64, "checkpoint_every": 100,
            "what": "one gradient: forward with checkpoints, recompute, reverse steps",
            "delta": "lambda_p/64", "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "reverse step (8 kernels)",
            "kernel_avg_us": step_s * 1e6, "bytes_per_node": bpn,
            "impl_bytes_per_node": adjoint_impl_bytes_per_node(storage),
        },
        "wall_s": wall,
        "phases_ms": tm,
        "loss": loss, "grad_norm": float(np.linalg.norm(g)),
        "fd_fp64": fd_fp64_gpu(cfg, w),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_adjoint(cfg, w, args.cpu_budget)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="wake2d_warmc")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32 / FP16-dev comparison of the default workload")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch1d_scan: skip the single-run FP64 comparison")
    ap.add_argument("--batch-config", default=None,
                    help="batch1d_scan: threads,nodes_per_thread instead of the autotuner")
    ap.add_argument("--storage", default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the scheme is built and measured per GPU); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch1d_scan":
        return bench_batch(args)
    if args.workload == "wake2d_lec_adjoint":
        return bench_adjoint(args)

    import torch

    from paper_2309_04872_amd import workloads
    from paper_2309_04872_amd.sim import Sim

    over = {"storage": args.storage} if args.storage else {}
    w = workloads.workload(args.workload, **over)
    default_steps = VALID_WINDOW_STEPS.get(args.workload, w["steps"])
    steps = args.steps if args.steps is not None else default_steps
    cells = w["nz"] * w["nx"]

    def build():
        s = Sim(w["dims"], w["nz"], w["nx"], delta=w["delta"], dt=w["dt"], tau_tilde=w["tau_tilde"],
                closure=w["closure"], dvel=w["dvel"], storage=w["storage"], geom=w["geom"])
        s.init_plasma(w["mu"], n=workloads.initial_density(w) if w.get("noise") else None)
        s.init_driver(w["alpha"], w["sigma_z"], w["sigma_x"], z0=w["z0"])
        return s

    s = build()
    if args.warmup:
        s.step(args.warmup)
    torch.cuda.synchronize()
    # timed region: the workload from t = 0, inputs resident in HBM
    s.init_plasma(w["mu"], n=workloads.initial_density(w) if w.get("noise") else None)
    s.init_driver(w["alpha"], w["sigma_z"], w["sigma_x"], z0=w["z0"])
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    t0 = time.perf_counter()
    s.step(steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    dg = s.diagnostics()
    # kernel duration: the same workload again, one event pair around the
    # back-to-back fused launches (HIP events on the simulation's stream)
    s.init_plasma(w["mu"], n=workloads.initial_density(w) if w.get("noise") else None)
    s.init_driver(w["alpha"], w["sigma_z"], w["sigma_x"], z0=w["z0"])
    s.set_timing(True)
    s.step(steps)
    k_ms, k_n = s.get_timing()
    s.set_timing(False)
    k_avg_s = k_ms / max(k_n, 1) / 1e3
    copy_gbs = copy_bandwidth_gbs(s.stream)
    blu = bytes_per_lu(w["dims"], w["closure"], w["storage"])
    achieved = blu * cells / k_avg_s / 1e9
    traffic = TRAFFIC_BYTES_PER_LAUNCH.get((args.workload, w["storage"]))
    mlups = cells * steps / (ms_total / 1e3) / 1e6
    paper = PAPER_MLUPS.get(args.workload)
    # against the paper's number only on its own workload at its precision
    vs = mlups / paper if paper and w["storage"] == "fp64" and steps == w["steps"] else None
    line = {
        "metric": "MLUPS (LB+field)",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_total / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": vs,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16"}[w["storage"]],
        "data": "synthetic",
        "config": {
            "workload": args.workload, "nz": w["nz"], "nx": w["nx"], "closure": w["closure"],
            "geometry": w["geom"], "populations": w["storage"], "recovery": "f64", "steps_per_run": steps,
            "delta": "lambda_p/%d" % round(2 * np.pi / w["delta"]), "delta_kp": w["delta"], "mu": w["mu"],
            "alpha": w["alpha"], "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
            "kernel": "k_step2d" if w["dims"] == 2 else "k_step1d_persist",
            "kernel_avg_us": k_avg_s * 1e6, "bytes_per_lu": blu, "launches": k_n,
        },
        "wall_s": wall,
        "diagnostics": {"sum_n": dg[0], "field_energy": dg[1], "max_lattice_mach": dg[4],
                        "recovery_fallbacks": dg[6]},
    }
    if w["dims"] == 1:
        line["roofline"]["note"] = (
            "one cooperative launch runs every step (kernel_avg_us and launches count steps); the 1D "
            "state stays in the L2 cache, so the step is bound by the latency of its recovery chain "
            "and grid barriers (24 steps per pass), not by HBM")
    if paper:
        line["paper_baseline"] = {
            "value": paper, "unit": "MLUPS", "hardware": "96 cores, Intel Xeon E5-2695 @ 2.40 GHz, MPI",
            "source": "Sec. 5: about %d min for 3e4 %s steps on the 3000 x 600 axisymmetric grid"
                      % (PAPER_MINUTES[args.workload], "LEC-LB" if w["closure"] == "lec" else "WARMC-LB")}
    s.close()
    del s
    if args.workload == "wake2d_warmc" and w["storage"] == "fp64" and not args.no_variants:
        line["precision_variants"] = precision_variants(w)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
