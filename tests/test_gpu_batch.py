"""Batched 1D parameter scans (one persistent launch for many 1D runs)
against the CPU oracle, the single-run library path and themselves
(graph replay, split calls, autotuner state restore, non-finite flags)."""
import numpy as np
import pytest

import oracle
from _pairs import rel_l2

pytestmark = pytest.mark.gpu

LP = 2 * np.pi  # plasma wavelength in units of c / omega_p
CL = {"lec": oracle.LEC, "warmc": oracle.WARMC}
BC = {"open": oracle.OPEN, "periodic": oracle.PERIODIC}
CONFIGS = [(256, 1), (256, 2), (512, 1), (512, 2), (1024, 1)]
SPLIT_CONFIGS = [(256, 2), (512, 1), (512, 2), (1024, 1)]


def _mixed_instances():
    """Both closures, both boundaries, D = 1 and 3, sizes from one partial
    pass to several passes of every configuration, with and without driver."""
    d = LP / 128
    return [
        dict(nz=300, closure="lec", mu=1e-3, alpha=0.5, sigma_z=0.5, delta=d),
        dict(nz=513, closure="warmc", mu=1e-2, alpha=0.3, sigma_z=0.7, delta=d),
        dict(nz=128, closure="lec", mu=2e-2, alpha=0.0, bc="periodic", delta=LP / 32),
        dict(nz=200, closure="warmc", mu=5e-3, alpha=0.0, bc="periodic", delta=LP / 40),
        dict(nz=700, closure="lec", mu=5e-2, alpha=2.0, sigma_z=0.6, dvel=3.0, delta=d),
        dict(nz=1100, closure="warmc", mu=1e-4, alpha=3.0, sigma_z=0.3, delta=d),
        dict(nz=2500, closure="lec", mu=1e-1, alpha=2.5, sigma_z=1.5, delta=d, tau_tilde=0.55),
    ]


def _densities(insts, seed=3):
    rng = np.random.default_rng(seed)
    return [1.0 + 1e-3 * rng.uniform(-1, 1, d["nz"]) for d in insts]


def _oracle(d, n=None):
    delta = d.get("delta", LP / 128)
    o = oracle.Oracle(1, d["nz"], 1, delta=delta, dt=d.get("dt", 0.1 * delta),
                      tau_tilde=d.get("tau_tilde", 0.52), closure=CL[d["closure"]],
                      dvel=d.get("dvel", 1.0), bc_z=BC[d.get("bc", "open")], mu=d["mu"],
                      alpha=d.get("alpha", 0.0), sigma_z=d.get("sigma_z", 1.0),
                      z0=d.get("z0", 6.0 * d.get("sigma_z", 1.0)))
    o.init(n=n, fields_from_driver=d.get("alpha", 0.0) != 0.0)
    return o


def _batch(insts, n=None):
    from paper_2309_04872_amd.batch import Batch

    return Batch(insts).init(n)


def _snapshot(b, which=("n", "uz", "ez", "gamma")):
    return [np.concatenate([b.read(i, q) for q in which]) for i in range(b.n)]


@pytest.mark.parametrize("cfg", CONFIGS)
def test_batch_matches_oracle(cfg):
    insts = _mixed_instances()
    dens = _densities(insts)
    b = _batch(insts, dens)
    b.set_config(*cfg)
    print("config", cfg, flush=True)
    b.step(120).step(80)
    assert b.step_count == 200
    assert not b.nonfinite().any()
    for i, d in enumerate(insts):
        o = _oracle(d, dens[i]).step(200)
        errs = {}
        for q in ("n", "uz", "gamma", "ez"):
            g, r = b.read(i, q), o.get(q)
            assert np.all(np.isfinite(g))
            errs[q] = rel_l2(g, r)
        if d["closure"] == "warmc":
            errs["thzz"] = rel_l2(b.read(i, "thzz"), o.get("thzz"))
        print(i, d["closure"], d["nz"], {k: float("%.3g" % v) for k, v in errs.items()}, flush=True)
        assert max(errs.values()) <= 1e-10, (i, errs)


def test_batch_matches_single_runs():
    """Instance i of a batch and the same run through lbw_step (one launch
    per step) execute the same per-node arithmetic; they agree to rounding
    (the compiler may contract the shared expressions differently in the
    two kernels)."""
    from paper_2309_04872_amd.sim import Sim

    insts = _mixed_instances()
    dens = _densities(insts, seed=5)
    b = _batch(insts, dens).step(150)
    for i, d in enumerate(insts):
        delta = d.get("delta", LP / 128)
        s = Sim(1, d["nz"], delta=delta, closure=d["closure"], dvel=d.get("dvel", 1.0),
                tau_tilde=d.get("tau_tilde", 0.52), bc_z=d.get("bc", "open"))
        s.init_plasma(d["mu"], n=dens[i])
        if d.get("alpha", 0.0):
            s.init_driver(d["alpha"], d["sigma_z"], z0=d.get("z0", 6.0 * d["sigma_z"]))
        s.step(150)
        for q in ("n", "uz", "ez"):
            g = b.read(i, q)
            r = s.field("ez") if q == "ez" else s.read(q)
            e = rel_l2(g, r)
            assert e <= 1e-10, (i, q, e)


def test_batch_full_scan_sampled():
    """The 256-instance scan at full size and length (4096 steps) in the
    launch configuration the benchmark times (autotuned, one graph-replayed
    launch). Sampled against the oracle: the longest, the shortest and the
    most strongly driven local-equilibrium instances, and the longest
    warm-closure instance with n_b/n0 < 0.1. Strongly driven warm-closure
    instances turn non-finite before the end in the oracle as well; the
    shortest one the kernel flags is run on the oracle to the same step and
    must be non-finite there too, and no local-equilibrium instance may be
    flagged."""
    from paper_2309_04872_amd import workloads

    insts = workloads.batch_instances()
    steps = workloads.BATCH_SCAN["steps"]
    b = _batch(insts)
    cfg = b.autotune(probe_steps=10)
    print("autotuned", cfg, flush=True)
    assert cfg in CONFIGS
    print("schedule", b.schedule(), flush=True)
    b.step(steps, graph=True)
    bad = b.nonfinite()
    nz = np.array([d["nz"] for d in insts])
    alpha = np.array([d["alpha"] for d in insts])
    lec = np.array([d["closure"] == "lec" for d in insts])
    print("non-finite instances", np.flatnonzero(bad).tolist(), flush=True)
    assert not bad[lec].any()
    pick = {int(np.flatnonzero(lec)[np.argmax(nz[lec])]), int(np.flatnonzero(lec)[np.argmin(nz[lec])]),
            int(np.flatnonzero(lec)[np.argmax(alpha[lec])])}
    weak = np.flatnonzero(~lec & (alpha < 0.1))
    pick.add(int(weak[np.argmax(nz[weak])]))
    for i in sorted(pick):
        assert bad[i] == 0
        o = _oracle(insts[i]).step(steps)
        errs = {q: rel_l2(b.read(i, q), o.get(q)) for q in ("n", "uz", "ez")}
        print(i, insts[i]["closure"], insts[i]["nz"], "alpha %.3g" % insts[i]["alpha"],
              {k: float("%.3g" % v) for k, v in errs.items()}, flush=True)
        assert max(errs.values()) <= 1e-10, (i, errs)
    flagged = np.flatnonzero(bad)
    if flagged.size:
        j = int(flagged[np.argmin(nz[flagged])])
        o = _oracle(insts[j]).step(steps)
        assert not np.all(np.isfinite(o.get("n")) & np.isfinite(o.get("uz")) & np.isfinite(o.get("ez"))), j


def test_batch_graph_replay_matches_eager():
    insts = _mixed_instances()
    dens = _densities(insts, seed=7)
    a = _batch(insts, dens)
    g = _batch(insts, dens)
    for _ in range(3):
        a.step(40)
        g.step(40, graph=True)
        # eager work and a synchronisation between replays
        sa, sg = _snapshot(a), _snapshot(g)
        for x, y in zip(sa, sg):
            assert np.array_equal(x, y)
    assert g.step_count == 120


def test_batch_split_calls_bitwise():
    insts = _mixed_instances()
    dens = _densities(insts, seed=11)
    one = _batch(insts, dens).step(100)
    four = _batch(insts, dens)
    for k in (25, 25, 24, 26):
        four.step(k)
    for x, y in zip(_snapshot(one, ("n", "uz", "ez", "thzz")), _snapshot(four, ("n", "uz", "ez", "thzz"))):
        assert np.array_equal(x, y)


def test_batch_autotune_restores_state():
    insts = _mixed_instances()
    dens = _densities(insts, seed=13)
    b = _batch(insts, dens).step(30)
    before = _snapshot(b, ("n", "uz", "ez", "thzz", "lambda"))
    cfg = b.autotune(probe_steps=7)
    assert cfg in CONFIGS and b.config() == cfg
    assert b.step_count == 30
    after = _snapshot(b, ("n", "uz", "ez", "thzz", "lambda"))
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    b.step(30)
    ref = _batch(insts, dens).step(30).step(30)
    for x, y in zip(_snapshot(b), _snapshot(ref)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("split", [False, True])
def test_batch_nonfinite_flags(split):
    """An instance whose pressure term overflows (n = 1e200: n0^3 is not
    representable) turns non-finite and is counted; the other instances
    are unaffected. Under the split schedule the count is summed over the
    instance's workgroups."""
    k = 10 if split else 1  # long enough to be shared by several workgroups
    insts = [dict(nz=300 * k, closure="lec", mu=1e-3, alpha=0.2, sigma_z=0.5),
             dict(nz=260 * k, closure="lec", mu=1e-3, alpha=0.0),
             dict(nz=310 * k, closure="warmc", mu=1e-3, alpha=0.2, sigma_z=0.5)]
    dens = [np.ones(300 * k), np.full(260 * k, 1e200), np.ones(310 * k)]
    b = _batch(insts, dens)
    if split:
        b.set_schedule(256, 2, split=True)
        assert b.schedule()[3] > len(insts)
    b.step(5)
    bad = b.nonfinite()
    assert bad[0] == 0 and bad[2] == 0 and bad[1] == 260 * k, bad
    ref = _batch([insts[0], insts[2]], [dens[0], dens[2]]).step(5)
    assert np.array_equal(b.read(0, "n"), ref.read(0, "n"))
    assert np.array_equal(b.read(2, "ez"), ref.read(1, "ez"))


def test_batch_errors():
    from paper_2309_04872_amd.batch import Batch
    from paper_2309_04872_amd.sim import LbwError

    insts = _mixed_instances()[:2]
    b = Batch(insts)
    with pytest.raises(LbwError, match="STATE"):
        b.step(1)
    b.init()
    with pytest.raises(LbwError, match="ARG"):
        b.set_config(1024, 2)
    with pytest.raises(LbwError, match="ARG"):
        b.read(2, "n")
    with pytest.raises(LbwError, match="NONFINITE"):
        b.init([np.ones(300), -np.ones(513)])
    with pytest.raises(LbwError, match="UNSTABLE"):
        Batch([dict(nz=64, closure="lec", mu=1e-3, tau_tilde=0.5)])


# ---------------------------------------------------------------------------
# Split schedule: long instances shared by several co-resident workgroups
# (cooperative launch), short ones packed into one workgroup's list.

@pytest.mark.parametrize("cfg", SPLIT_CONFIGS)
def test_batch_split_schedule_bitwise(cfg):
    """Every node runs the same arithmetic under every schedule, so the split
    schedule's results are the bits of one workgroup per instance, through
    single steps, pairs, deep passes and a second call."""
    insts = _mixed_instances()
    dens = _densities(insts, seed=17)
    ref = _batch(insts, dens)
    ref.set_config(*cfg)
    ref.step(120).step(81)
    b = _batch(insts, dens)
    b.set_schedule(*cfg, split=True)
    t, c, split, wg = b.schedule()
    print("split schedule", cfg, "workgroups", wg, flush=True)
    assert (t, c) == cfg and split and wg > len(insts)
    b.step(120).step(81)
    assert b.step_count == 201
    for x, y in zip(_snapshot(ref, ("n", "uz", "ez", "thzz", "lambda")), _snapshot(b, ("n", "uz", "ez", "thzz", "lambda"))):
        assert np.array_equal(x, y)
    assert np.array_equal(ref.nonfinite(), b.nonfinite())


def test_batch_split_graph_replay():
    """The split schedule captured in a HIP graph and replayed, with eager
    work between the replays, equals eager launches bit for bit."""
    insts = _mixed_instances()
    dens = _densities(insts, seed=19)
    a = _batch(insts, dens)
    g = _batch(insts, dens)
    for x in (a, g):
        x.set_schedule(1024, 1, split=True)
    for _ in range(3):
        a.step(40)
        g.step(40, graph=True)
        for x, y in zip(_snapshot(a), _snapshot(g)):
            assert np.array_equal(x, y)


def test_batch_split_full_scan_matches_whole():
    """The 256-instance scan, 200 steps: the split schedule (the longest
    instances shared, the short ones packed) against one workgroup per
    instance, bit for bit on every instance."""
    from paper_2309_04872_amd import workloads

    insts = workloads.batch_instances()
    ref = _batch(insts).step(200)
    b = _batch(insts)
    b.set_schedule(1024, 1, split=True)
    print("scan split schedule", b.schedule(), flush=True)
    b.step(200)
    for i in range(len(insts)):
        for q in ("n", "uz", "ez"):
            assert np.array_equal(ref.read(i, q), b.read(i, q)), (i, q)
