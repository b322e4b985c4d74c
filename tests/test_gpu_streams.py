"""The library on a caller's stream: a simulation and a batch bound to a side
stream (default priority) give the same bits as on the current stream, and
the binding's device outputs are written in that stream's order."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LP = 2 * np.pi


def _sim(stream=None):
    from paper_2309_04872_amd.sim import Sim

    s = Sim(2, 256, 64, delta=LP / 64, closure="lec", storage="fp32", stream=stream)
    s.init_plasma(1e-2)
    s.init_driver(1.0, 1.0, 0.5, z0=6.0)
    return s


def test_sim_on_side_stream_bitwise():
    import torch

    side = torch.cuda.Stream()
    ref = _sim()
    ref.step(40)
    a = _sim(side)
    a.step(40)
    dn = a.read_device("n")           # written on the side stream
    side.synchronize()
    for q in ("n", "uz", "ux"):
        np.testing.assert_array_equal(a.read(q), ref.read(q))
    np.testing.assert_array_equal(a.field("ez"), ref.field("ez"))
    np.testing.assert_array_equal(dn.cpu().numpy(), ref.read("n"))
    ck = a.save_state_device()
    a.step(5)
    a.load_state_device(ck, 40)
    a.step(5)
    ref.step(5)
    side.synchronize()
    np.testing.assert_array_equal(a.read("n"), ref.read("n"))
    a.close()
    ref.close()


def test_batch_on_side_stream_bitwise():
    import torch

    from paper_2309_04872_amd.batch import Batch

    insts = [dict(nz=300, closure="lec", mu=1e-3, alpha=0.5, sigma_z=0.5),
             dict(nz=513, closure="warmc", mu=1e-2, alpha=0.3, sigma_z=0.7)]
    side = torch.cuda.Stream()
    ref = Batch(insts).init()
    ref.step(37)
    b = Batch(insts, stream=side).init()
    b.step(37, graph=True)
    side.synchronize()
    for i in range(2):
        for q in ("n", "uz", "ez"):
            np.testing.assert_array_equal(b.read(i, q), ref.read(i, q))
    b.close()
    ref.close()


@pytest.mark.gpu
def test_stream_copy_exact():
    """The streaming-copy reference copies bit for bit, a ragged size (not a
    multiple of the workgroup's 4096 bytes) on a side stream."""
    import ctypes

    import torch

    from paper_2309_04872_amd import _lib

    L = _lib.load()
    st = torch.cuda.Stream()
    n = 16 * 1000003
    g = torch.Generator(device="cpu").manual_seed(7)
    x = torch.randint(0, 256, (n,), dtype=torch.uint8, generator=g).cuda()
    y = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    rc = L.lbw_stream_copy(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(x.data_ptr()), n,
                           ctypes.c_void_p(st.cuda_stream))
    assert rc == 0
    st.synchronize()
    assert torch.equal(y[:n], x)
    assert int(y[n:].count_nonzero()) == 0


@pytest.mark.gpu
def test_library_loaded_before_torch():
    """A fresh process that loads the library through the binding before it
    imports torch itself still finds the GPU."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2309_04872_amd import _lib\n"
            "L = _lib.load()\n"
            "from paper_2309_04872_amd.sim import Sim\n"
            "s = Sim(2, 64, 16, closure='lec', storage='fp32')\n"
            "s.init_plasma(1e-2); s.step(3); s.close()\n"
            "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]


def test_device_buffer_refusals_leave_state_unchanged():
    """load_state_device / save_state_device / step_record refuse a device
    tensor that is too small, not contiguous or not 256-byte aligned with
    ValueError before any call reaches the C side; the simulation then steps
    on exactly as one that never saw the refused calls."""
    import torch

    ref = _sim()
    ref.step(10)
    a = _sim()
    a.step(10)
    n = a.state_device_bytes()
    ok = a.save_state_device()
    small = torch.zeros(n - 256, dtype=torch.uint8, device=a.device)
    strided = torch.zeros(2 * n, dtype=torch.uint8, device=a.device)[::2]
    shifted = torch.zeros(n + 256, dtype=torch.uint8, device=a.device)[1:n + 1]
    for buf, msg in ((small, "needed"), (strided, "contiguous"), (shifted, "aligned")):
        with pytest.raises(ValueError, match=msg):
            a.load_state_device(buf, 10)
        with pytest.raises(ValueError, match=msg):
            a.save_state_device(out=buf)
        with pytest.raises(ValueError, match=msg):
            a.step_record(1, buf)
    with pytest.raises(ValueError, match="tensor on"):
        a.load_state_device(ok.cpu(), 10)
    torch.cuda.synchronize()
    assert a.step_count == 10
    a.step(5)
    ref.step(5)
    for q in ("n", "uz", "ux"):
        np.testing.assert_array_equal(a.read(q), ref.read(q))
    np.testing.assert_array_equal(a.field("ez"), ref.field("ez"))
