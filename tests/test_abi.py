"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/lbwake.h declares, and rejects invalid grids before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_2309_04872_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbwake.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbw_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.SO_PATH):
        from paper_2309_04872_amd import build

        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert len(declared) >= 15
    assert sorted(_lib.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_version(lib):
    assert b"gfx950" in lib.lbw_version()


def _grid(**kw):
    g = dict(dims=2, nz=64, nx=16, delta=0.1, dt=0.01, tau_tilde=0.53, closure=0, dvel=3.0,
             storage=0, bc_z=0, bc_x=0)
    g.update(kw)
    return _lib.GridDesc(**g)


def test_workspace_bytes(lib):
    g = _grid()
    n = lib.lbw_workspace_bytes(ctypes.byref(g))
    nc = 64 * 16
    # two FP64 population buffers of 3 x 9 planes plus six field planes at least
    assert n >= 2 * 27 * nc * 8 + 6 * nc * 8
    g32 = _grid(storage=1)
    assert lib.lbw_workspace_bytes(ctypes.byref(g32)) < n
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(dims=3))) == 0
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(nz=2))) == 0
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(dims=1, nx=4))) == 0
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(closure=5))) == 0


def test_grid_size_limit(lib):
    """Node offsets inside a population plane and every plane offset times
    72 planes stay below 2^31: grids beyond 2e9 / 72 nodes are rejected, the
    largest accepted one needs its full workspace (no overflow in the size)."""
    limit = int(2.0e9 / 72)
    nx = 1024
    nz_ok = limit // nx
    g_ok = _grid(nz=nz_ok, nx=nx, closure=1)
    n_ok = lib.lbw_workspace_bytes(ctypes.byref(g_ok))
    assert n_ok >= 2 * 72 * nz_ok * nx * 8
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(nz=nz_ok + 2, nx=nx))) == 0
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(nz=4, nx=4))) > 0  # smallest 2D grid


def test_geometry_validation(lib):
    """The axisymmetric geometry is 2D with an open outer radius, for both
    closures; it needs the workspace of the slab grid."""
    for closure in (0, 1):
        assert lib.lbw_workspace_bytes(ctypes.byref(_grid(geom=1, closure=closure))) == \
            lib.lbw_workspace_bytes(ctypes.byref(_grid(closure=closure)))
        rc, h = _create(lib, _grid(geom=1, closure=closure))
        assert rc == 0
        lib.lbw_destroy(h)
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(geom=2))) == 0
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(geom=1, bc_x=1))) == 0
    assert lib.lbw_workspace_bytes(ctypes.byref(_grid(geom=1, dims=1, nx=1))) == 0
    nb = lib.lbw_workspace_bytes(ctypes.byref(_grid()))
    assert _create(lib, _grid(geom=1, bc_x=1), nbytes=nb)[0] == -1


def _create(lib, g, ws=256 * 1024, nbytes=None):
    h = ctypes.c_void_p()
    if nbytes is None:
        nbytes = lib.lbw_workspace_bytes(ctypes.byref(g))
    rc = lib.lbw_create(ctypes.byref(g), ctypes.c_void_p(ws), nbytes, None, ctypes.byref(h))
    return rc, h


def test_create_validation(lib):
    # a fake, aligned workspace address: lbw_create only records it
    rc, h = _create(lib, _grid())
    assert rc == 0 and h.value
    assert lib.lbw_step_count(h) == 0
    assert lib.lbw_step(h, 1) == -6  # LBW_ERR_STATE: step before init
    assert b"init" in lib.lbw_last_error(h)
    assert lib.lbw_step_record(h, 1, ctypes.c_void_p(512 * 1024), 1 << 20) == -6
    assert lib.lbw_step_record(None, 1, ctypes.c_void_p(512 * 1024), 1 << 20) == -1
    # argument checks that come before any device work
    A = (ctypes.c_double * 3)()
    assert lib.lbw_init_moments(h, -1e-3, A, None, None) == -1   # mu < 0
    assert b"mu" in lib.lbw_last_error(h)
    drv = _lib.DriverDesc(alpha=0.5, sigma_z=0.5, sigma_x=0.5)
    assert lib.lbw_init_driver(h, ctypes.byref(drv), 1) == -6     # before init
    lib.lbw_destroy(h)
    assert _create(lib, _grid(tau_tilde=0.5))[0] == -4           # BGK stability
    assert _create(lib, _grid(dt=0.1))[0] == -4                  # 2D Courant
    assert _create(lib, _grid(dims=1, nx=1, dt=0.1))[0] == 0      # 1D Courant limit dt = delta
    assert _create(lib, _grid(), ws=256 * 1024 + 8)[0] == -2      # misaligned workspace
    assert _create(lib, _grid(), nbytes=1024)[0] == -2            # too small
    assert _create(lib, _grid(nz=1))[0] == -1


def _inst(**kw):
    d = dict(nz=1000, closure=0, dvel=1.0, mu=1e-3, delta=0.05, dt=0.005, tau_tilde=0.52, bc=0,
             alpha=0.5, sigma_z=0.5, z0=3.0)
    d.update(kw)
    return _lib.InstanceDesc(**d)


def _insts(*ds):
    return (_lib.InstanceDesc * len(ds))(*ds)


def test_batch_workspace_bytes(lib):
    one = _insts(_inst())
    n1 = lib.lbw_batch_workspace_bytes(one, 1)
    # two LEC population buffers (2 x 3 planes of 1024 padded nodes) and E_z at least
    assert n1 >= 2 * 6 * 1024 * 8 + 1024 * 8
    two = _insts(_inst(), _inst(closure=1, nz=3000))
    assert lib.lbw_batch_workspace_bytes(two, 2) >= n1 + 2 * 12 * 3008 * 8
    assert lib.lbw_batch_workspace_bytes(_insts(_inst(nz=3)), 1) == 0
    assert lib.lbw_batch_workspace_bytes(_insts(_inst(closure=4)), 1) == 0
    assert lib.lbw_batch_workspace_bytes(_insts(_inst(alpha=1.0, sigma_z=0.0)), 1) == 0
    assert lib.lbw_batch_workspace_bytes(one, 0) == 0


def test_batch_create_validation(lib):
    def create(arr, n, ws=256 * 1024, nbytes=None):
        h = ctypes.c_void_p()
        if nbytes is None:
            nbytes = lib.lbw_batch_workspace_bytes(arr, n)
        rc = lib.lbw_batch_create(arr, n, ctypes.c_void_p(ws), nbytes, None, ctypes.byref(h))
        return rc
    # every check below returns before any device call
    assert create(_insts(_inst(tau_tilde=0.5)), 1) == -4
    assert create(_insts(_inst(dt=0.06)), 1) == -4                 # dt > delta
    assert create(_insts(_inst(nz=2)), 1, nbytes=1 << 20) == -1
    assert create(_insts(_inst()), 1, ws=256 * 1024 + 8) == -2      # misaligned
    assert create(_insts(_inst()), 1, nbytes=64) == -2              # too small
    assert create(_insts(_inst()), 0, nbytes=1 << 20) == -1


def test_stream_copy_host_checks(lib):
    """lbw_stream_copy refuses, on the host and before any launch, NULL
    pointers, misalignment, overlap and sizes not a multiple of 16; an empty
    copy launches nothing."""
    vp = ctypes.c_void_p
    a, b = 1 << 20, 1 << 24  # addresses only; never dereferenced on these paths
    assert lib.lbw_stream_copy(None, vp(a), 16, None) == -1
    assert lib.lbw_stream_copy(vp(b), None, 16, None) == -1
    assert lib.lbw_stream_copy(vp(b + 8), vp(a), 16, None) == -1
    assert lib.lbw_stream_copy(vp(b), vp(a + 4), 16, None) == -1
    assert lib.lbw_stream_copy(vp(b), vp(a), 24, None) == -1
    assert lib.lbw_stream_copy(vp(a + 16), vp(a), 64, None) == -1  # overlap
    assert lib.lbw_stream_copy(vp(a), vp(a + 16), 64, None) == -1
    assert lib.lbw_stream_copy(vp(b), vp(a), 0, None) == 0


def test_diagnostics_every_null_sim(lib):
    assert lib.lbw_set_diagnostics_every(None, 10, None, 4) == -1
    assert lib.lbw_diagnostics_rows(None) == -1


def test_exports_only_the_declared_interface(lib):
    """The library exports the declared C ABI and nothing else (kernel handles
    and helpers stay local), where nm is available."""
    import shutil
    import subprocess

    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.SO_PATH], capture_output=True, text=True,
                         check=True).stdout
    names = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    assert names == set(_declared()), sorted(names ^ set(_declared()))[:10]


def test_binding_refuses_host_buffers_for_device_calls():
    """The binding's device-buffer calls (load_state_device, save_state_device,
    step_record, step_record_post) hand a raw pointer to the C side, which reads
    or writes lbw_state_device_bytes() bytes there: anything but a tensor on the
    simulation's device is refused before the call, and a checkpoint into host
    memory needs a pinned uint8 tensor of lbw_state_bytes() bytes."""
    import types

    import torch

    from paper_2309_04872_amd.sim import Sim

    fake = types.SimpleNamespace(device=torch.device("cuda", 0), _h=None,
                                 _lib=types.SimpleNamespace(lbw_state_bytes=lambda h: 4096))
    for bad in (torch.zeros(4096, dtype=torch.uint8), bytearray(4096), None):
        with pytest.raises(ValueError, match="tensor on cuda:0"):
            Sim._device_buffer(fake, bad, 4096, "load_state_device")
    with pytest.raises(ValueError, match="pinned"):
        Sim.save_state_async(fake, torch.zeros(4096, dtype=torch.uint8))
    for bad in (torch.zeros(4096, dtype=torch.float32), torch.zeros(8192, dtype=torch.uint8)[::2]):
        with pytest.raises(ValueError, match="contiguous uint8 CPU tensor"):
            Sim.save_state_async(fake, bad)
