"""Precision variants at full grid size: FP32 and FP16 deviation storage
against the FP64 run on the same GPU (the FP64 kernel matches the oracle to
1e-10 on prefixes, see the parity tests; the oracle itself would need hours
for these runs). Reported: per-field relative L2 of density, momentum and
E_z.

The warm-closure wake (4096 x 1024, n_b/n0 = 2, mu = 0.05) is compared over
its first 400 steps: by step 500 the longitudinal pressure theta^zz has turned
negative on the axis behind the bunch head and the run diverges (non-finite
by step ~1400), in the FP64 kernel and in the oracle alike (the oracle's
minimum theta^zz at steps 200 / 400 is 0.0109 / 0.00225, the kernel's the
same). The local-equilibrium wake runs its full 8000 steps."""
import json
import os

import numpy as np
import pytest

from paper_2309_04872_amd import workloads

pytestmark = pytest.mark.gpu

FIELDS = ("n", "mz", "mx", "ez")


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
    out = {q: s.read(q) for q in ("n", "mz", "mx", *extra)}
    out["ez"] = s.field("ez")
    dg = s.diagnostics()
    del s
    return out, dg


WARM_STABLE_STEPS = 400


def test_warm_wake_precision_variants():
    w = workloads.workload("wake2d_warmc")
    steps = WARM_STABLE_STEPS
    ref, dref = _run(w, "fp64", steps, extra=("thzz",))
    assert ref["thzz"].min() > 0.0
    report = {"workload": "wake2d_warmc", "steps": steps}
    for storage, bound in (("fp32", 1e-4), ("fp16dev", 5e-2)):
        got, dg = _run(w, storage, steps)
        assert dg[5] == 0
        errs = {q: float(np.linalg.norm(got[q] - ref[q]) / np.linalg.norm(ref[q])) for q in FIELDS}
        report[storage] = errs
        print(storage, errs, flush=True)
        assert all(e <= bound for e in errs.values()), (storage, errs)
    _report("precision_wake2d_warmc.json", report)


def test_lec_wake_precision_variants_full_length():
    """The benchmark workload (2048 x 512, 8000 steps) in FP32 and FP16
    deviation storage against FP64."""
    w = workloads.workload("wake2d_lec_fp32")
    ref, _ = _run(w, "fp64", w["steps"])
    report = {"workload": "wake2d_lec_fp32", "steps": w["steps"]}
    for storage, bound in (("fp32", 1e-4), ("fp16dev", 5e-2)):
        got, dg = _run(w, storage, w["steps"])
        assert dg[5] == 0
        errs = {q: float(np.linalg.norm(got[q] - ref[q]) / np.linalg.norm(ref[q])) for q in FIELDS}
        report[storage] = errs
        print(storage, errs, flush=True)
        assert all(e <= bound for e in errs.values()), (storage, errs)
    _report("precision_wake2d_lec.json", report)


@pytest.mark.parametrize("closure", ["lec", "warmc"])
def test_axi_production_precision_variants(closure):
    """The paper's axisymmetric production run (3000 x 600, mu = 0.04,
    Q~ = 0.5, all 30 000 steps) in FP32 and FP16 deviation storage against
    FP64. Over 30 000 steps the FP32 rounding reaches about 1e-4 in the
    momenta (1.0e-4 measured for the local-equilibrium closure), so the FP32
    bound here is 3e-4."""
    w = workloads.workload("wake_axi_" + closure)
    print("axi precision", closure, flush=True)
    ref, _ = _run(w, "fp64", w["steps"])
    report = {"workload": "wake_axi_" + closure, "steps": w["steps"]}
    for storage, bound in (("fp32", 3e-4), ("fp16dev", 5e-2)):
        got, dg = _run(w, storage, w["steps"])
        assert dg[5] == 0
        errs = {q: float(np.linalg.norm(got[q] - ref[q]) / np.linalg.norm(ref[q])) for q in FIELDS}
        report[storage] = errs
        print(storage, errs, flush=True)
        assert all(e <= bound for e in errs.values()), (storage, errs)
    _report(f"precision_wake_axi_{closure}.json", report)
