"""Precision variants at full grid size: FP32 and FP16 deviation storage
against the FP64 run on the same GPU (the FP64 kernel matches the oracle to
1e-10 on prefixes, see the parity tests; the oracle itself would need hours
for these runs). Reported: per-field relative L2 of the density perturbation
n - 1, the momentum densities and E_z. These are stated errors: each test
guards the measured value (a regression bound about 1.5x above it); the
FP32 parity tolerance of 1e-4 against the oracle applies to the parity tests.

The warm-closure wake (4096 x 1024, n_b/n0 = 2, mu = 0.05) is compared over
its first 400 steps (t = 3.9): near t = 4.5 (step ~459) its temperature
theta^zz first turns negative on the axis behind the bunch head, and later
the run diverges (non-finite near step 1400), in the FP64 kernel and in the
oracle alike. On a reduced grid the oracle puts that onset at t = 4.5 for
dt and dt / 2 (LB diffusion held fixed) and for delta / 2, so 400 steps is
inside the closure's range of validity at every resolution tried. The
local-equilibrium wake runs its full 8000 steps."""
import json
import os

import numpy as np
import pytest

from paper_2309_04872_amd import workloads

pytestmark = pytest.mark.gpu

FIELDS = ("dn", "mz", "mx", "ez")


def _report(name, report):
    """Write the error report as JSON into $LBW_REPORT_DIR when it is set."""
    d = os.environ.get("LBW_REPORT_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, name), "w") as f:
            json.dump(report, f)


def _run(w, storage, steps, extra=()):
    from paper_2309_04872_amd.sim import Sim

    s = Sim(2, w["nz"], w["nx"], delta=w["delta"], closure=w["closure"], dvel=w["dvel"],
            storage=storage, geom=w["geom"])
    s.init_plasma(w["mu"])
    s.init_driver(w["alpha"], w["sigma_z"], w["sigma_x"], z0=w["z0"])
    s.step(steps)
    out = {q: s.read(q) for q in ("mz", "mx", *extra)}
    out["dn"] = s.read("n") - 1.0
    out["ez"] = s.field("ez")
    dg = s.diagnostics()
    del s
    return out, dg


WARM_STABLE_STEPS = 400

# Stated errors (relative L2 against the FP64 run, measured on MI355X); the
# tests guard each at 1.5x the measured value.
MEASURED = {
    "wake2d_warmc": {"fp32": {"dn": 3.8e-6, "mz": 2.0e-6, "mx": 1.1e-6, "ez": 1.4e-6},
                     "fp16dev": {"dn": 1.34e-3, "mz": 8.4e-4, "mx": 6.6e-4, "ez": 2.1e-4}},
    "wake2d_lec_fp32": {"fp32": {"dn": 7.3e-5, "mz": 5.8e-5, "mx": 7.4e-5, "ez": 7.7e-5},
                        "fp16dev": {"dn": 2.3e-3, "mz": 1.66e-3, "mx": 1.64e-3, "ez": 1.68e-3}},
    "wake_axi_lec": {"fp32": {"dn": 8.7e-5, "mz": 1.0e-4, "mx": 1.03e-4, "ez": 9.7e-5},
                     "fp16dev": {"dn": 1.19e-3, "mz": 9.9e-4, "mx": 9.8e-4, "ez": 7.2e-4}},
    "wake_axi_warmc": {"fp32": {"dn": 8.5e-5, "mz": 9.1e-5, "mx": 1.04e-4, "ez": 9.4e-5},
                       "fp16dev": {"dn": 3.2e-3, "mz": 6.1e-3, "mx": 5.8e-3, "ez": 4.1e-3}},
}


def _guard(name, storage, errs):
    ref = MEASURED[name][storage]
    bad = {q: (e, ref[q]) for q, e in errs.items() if not e <= 1.5 * ref[q]}
    assert not bad, (name, storage, "error above 1.5x the stated value", bad)


def test_warm_wake_precision_variants():
    w = workloads.workload("wake2d_warmc")
    steps = WARM_STABLE_STEPS
    ref, dref = _run(w, "fp64", steps, extra=("thzz",))
    assert ref["thzz"].min() > 0.0
    report = {"workload": "wake2d_warmc", "steps": steps}
    for storage in ("fp32", "fp16dev"):
        got, dg = _run(w, storage, steps)
        assert dg[5] == 0
        errs = {q: float(np.linalg.norm(got[q] - ref[q]) / np.linalg.norm(ref[q])) for q in FIELDS}
        report[storage] = errs
        print(storage, errs, flush=True)
        _guard("wake2d_warmc", storage, errs)
    _report("precision_wake2d_warmc.json", report)


def test_lec_wake_precision_variants_full_length():
    """The benchmark workload (2048 x 512, 8000 steps) in FP32 and FP16
    deviation storage against FP64."""
    w = workloads.workload("wake2d_lec_fp32")
    ref, _ = _run(w, "fp64", w["steps"])
    report = {"workload": "wake2d_lec_fp32", "steps": w["steps"]}
    for storage in ("fp32", "fp16dev"):
        got, dg = _run(w, storage, w["steps"])
        assert dg[5] == 0
        errs = {q: float(np.linalg.norm(got[q] - ref[q]) / np.linalg.norm(ref[q])) for q in FIELDS}
        report[storage] = errs
        print(storage, errs, flush=True)
        _guard("wake2d_lec_fp32", storage, errs)
    _report("precision_wake2d_lec.json", report)


@pytest.mark.parametrize("closure", ["lec", "warmc"])
def test_axi_production_precision_variants(closure):
    """The paper's axisymmetric production run (3000 x 600, mu = 0.04,
    Q~ = 0.5, all 30 000 steps) in FP32 and FP16 deviation storage against
    FP64. Over 30 000 steps the FP32 rounding reaches about 1e-4 in the
    momenta (stated errors in MEASURED)."""
    w = workloads.workload("wake_axi_" + closure)
    print("axi precision", closure, flush=True)
    ref, _ = _run(w, "fp64", w["steps"])
    report = {"workload": "wake_axi_" + closure, "steps": w["steps"]}
    for storage in ("fp32", "fp16dev"):
        got, dg = _run(w, storage, w["steps"])
        assert dg[5] == 0
        errs = {q: float(np.linalg.norm(got[q] - ref[q]) / np.linalg.norm(ref[q])) for q in FIELDS}
        report[storage] = errs
        print(storage, errs, flush=True)
        _guard("wake_axi_" + closure, storage, errs)
    _report(f"precision_wake_axi_{closure}.json", report)
