"""lbw_diagnostics_static, the allocation-free variant of lbw_diagnostics
(its reduction scratch in a static device array of the library), against
lbw_diagnostics through the C ABI: two calls in a row on driven states, the
second on a smaller grid, and the refusal of a grid above the array's limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _static_diag(s):
    import torch

    from paper_2309_04872_amd import _lib

    lib = _lib.load()
    out = torch.full((8,), -1.0, dtype=torch.float64, device=s.device)
    rc = lib.lbw_diagnostics_static(s._h, ctypes.c_void_p(out.data_ptr()))
    return rc, out


def _driven(nz, nx, closure, storage):
    from paper_2309_04872_amd.sim import Sim

    s = Sim(2, nz, nx, delta=2 * np.pi / 32, closure=closure, storage=storage)
    s.init_plasma(0.03)
    s.init_driver(0.8, 1.0, 0.5, z0=4.0)
    s.step(30)
    return s


def test_static_diagnostics_match_two_calls():
    import torch

    for nz, nx, closure, storage in ((300, 120, "warmc", "fp64"), (96, 40, "lec", "fp32")):
        print("static diagnostics", nz, nx, closure, storage, flush=True)
        s = _driven(nz, nx, closure, storage)
        ref = s.diagnostics()
        rc, out = _static_diag(s)
        assert rc == 0, s._lib.lbw_last_error(s._h).decode()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # same kernels and order: the sums are the same bits; the rms Gauss
        # residual's square root is taken on the device instead of the host
        for i in (0, 1, 2, 4, 5, 6, 7):
            assert got[i] == ref[i], (i, got[i], ref[i])
        assert abs(got[3] - ref[3]) <= 1e-15 * abs(ref[3]), (got[3], ref[3])
        s.close()


def test_static_diagnostics_rejects_large_grid():
    from paper_2309_04872_amd.sim import Sim

    s = Sim(2, 4096, 1400, delta=2 * np.pi / 64, closure="lec", storage="fp16dev")
    s.init_plasma(0.01)
    rc, _ = _static_diag(s)
    assert rc == -7, rc
    assert "static scratch" in s._lib.lbw_last_error(s._h).decode()
    s.close()
