"""Python binding of the C ABI: one ``Sim`` per simulation. PyTorch provides
the device workspace and the stream; the binding only marshals arguments."""
from __future__ import annotations

import ctypes
import sys

import numpy as np

from . import _lib, trace


class LbwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.STATUS.get(code, code)}: {msg}")
        self.code = code


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Sim:
    """A 1D or 2D simulation bound to a torch-allocated workspace on ``device``.

    Parameters mirror ``lbw_grid_desc``: ``closure`` in {'lec', 'warmc'},
    ``storage`` in {'fp64', 'fp32', 'fp16dev'}, ``bc_z``/``bc_x`` in
    {'open', 'periodic'}, ``geom`` in {'slab', 'axi'} (2D: Cartesian (z, x)
    or the axisymmetric (z, r) geometry of App. A, where x runs over
    r_j = (j + 1/2) delta). ``dt`` defaults to delta / 10 and ``tau_tilde``
    to 0.52 (1D) / 0.53 (2D), the paper's choices (Sec. 5).
    """

    def __init__(self, dims, nz, nx=1, delta=2 * np.pi / 128, dt=None, tau_tilde=None,
                 closure="lec", dvel=None, storage="fp64", bc_z="open", bc_x="open",
                 geom="slab", device="cuda:0", stream=None):
        import torch

        self._lib = _lib.load()
        if dt is None:
            dt = 0.1 * delta
        if tau_tilde is None:
            tau_tilde = 0.52 if dims == 1 else 0.53
        if dvel is None:
            dvel = 1.0 if dims == 1 else 3.0
        self.dims, self.nz, self.nx = dims, nz, nx
        self.shape = (nx, nz)
        self.ncell = nx * nz
        self.closure = closure
        self.grid = _lib.GridDesc(dims, nz, nx, delta, dt, tau_tilde, _lib.CLOSURES[closure],
                                  float(dvel), _lib.STORAGE[storage], _lib.BCS[bc_z], _lib.BCS[bc_x],
                                  _lib.GEOMS[geom])
        self.geom = geom
        nbytes = self._lib.lbw_workspace_bytes(ctypes.byref(self.grid))
        if nbytes == 0:
            h = ctypes.c_void_p()
            rc = self._lib.lbw_create(ctypes.byref(self.grid), None, 0, None, ctypes.byref(h))
            raise LbwError(rc if rc != 0 else -1, "invalid or unsupported grid descriptor")
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        # allocated on the simulation's stream: once freed, the caching
        # allocator reuses the block only in that stream's order, after the
        # work queued there
        with torch.cuda.stream(stream):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        rc = self._lib.lbw_create(ctypes.byref(self.grid), ctypes.c_void_p(self.workspace.data_ptr()),
                                  nbytes, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise LbwError(rc, "lbw_create rejected the grid")
        self._h = h

    # ------------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise LbwError(rc, self._lib.lbw_last_error(self._h).decode())

    def _arr(self, a):
        if a is None:
            return None
        return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), self.shape))

    def close(self):
        """Release the library handle (and its HIP events). Call it before the
        interpreter shuts down; the workspace tensor stays torch's."""
        if getattr(self, "_h", None):
            self._lib.lbw_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter shutdown the HIP runtime (or a profiler's hooks
        # around it) may already be gone: leave the handle to the process exit
        # (module globals such as sys may be None by then, hence the default)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _device_buffer(self, buf, nbytes, what):
        """Refuse a buffer the C side could not use safely: it reads or writes
        nbytes at buf.data_ptr() on this simulation's device."""
        import torch

        if not isinstance(buf, torch.Tensor) or not buf.is_cuda or buf.device != self.device:
            raise ValueError(f"{what}: a tensor on {self.device} is required")
        if not buf.is_contiguous():
            raise ValueError(f"{what}: the tensor must be contiguous")
        if buf.numel() * buf.element_size() < nbytes:
            raise ValueError(f"{what}: {buf.numel() * buf.element_size()} bytes, {nbytes} needed")
        if buf.data_ptr() % 256:
            raise ValueError(f"{what}: the buffer must be 256-byte aligned")
        return ctypes.c_void_p(buf.data_ptr())

    # ------------------------------------------------------------------
    def init_plasma(self, mu, n=None, uz=None, ux=None):
        n, uz, ux = self._arr(n), self._arr(uz), self._arr(ux)
        p = _lib.PlasmaDesc(mu, _dp(n), _dp(uz), _dp(ux))
        self._check(self._lib.lbw_init_plasma(self._h, ctypes.byref(p)))
        return self

    def init_moments(self, mu, A, uz=None, ux=None):
        K = {("lec", 1): 2, ("lec", 2): 3, ("warmc", 1): 4, ("warmc", 2): 8}[(self.closure, self.dims)]
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(K, *self.shape))
        uz, ux = self._arr(uz), self._arr(ux)
        self._check(self._lib.lbw_init_moments(self._h, mu, _dp(A), _dp(uz), _dp(ux)))
        return self

    def init_driver(self, alpha, sigma_z, sigma_x=1.0, z0=None, x0=0.0, slice_w=None,
                    slice_zmin=0.0, slice_zmax=0.0, init_fields=True):
        if z0 is None:
            z0 = 6.0 * sigma_z
        w = None if slice_w is None else np.ascontiguousarray(slice_w, dtype=np.float64)
        d = _lib.DriverDesc(alpha, sigma_z, sigma_x, z0, x0, 0 if w is None else len(w), _dp(w),
                            slice_zmin, slice_zmax)
        self._check(self._lib.lbw_init_driver(self._h, ctypes.byref(d), int(bool(init_fields))))
        return self

    def set_field(self, which, values):
        v = self._arr(values)
        self._check(self._lib.lbw_set_field(self._h, _lib.FIELDS[which], _dp(v), v.size))
        return self

    def step(self, nsteps=1):
        with trace.marker("lbw_step"):
            self._check(self._lib.lbw_step(self._h, int(nsteps)))
        return self

    def set_nonfinite_check(self, every):
        """Check the state for NaN / Inf after every ``every`` steps inside
        step() (0: off); step() then raises LbwError(LBW_ERR_NONFINITE)."""
        self._check(self._lib.lbw_set_nonfinite_check(self._h, int(every)))
        return self

    def record_diagnostics(self, every, capacity=1024):
        """Record the 8 values of diagnostics() after every ``every`` steps of
        step() into a device tensor of ``capacity`` rows (every = 0: stop).
        Asynchronous: nothing is copied to the host while stepping."""
        import torch

        ptr = None
        if every > 0:
            with torch.cuda.stream(self.stream):
                self._diag_series = torch.full((capacity, 8), float("nan"), dtype=torch.float64,
                                               device=self.device)
            ptr = ctypes.c_void_p(self._diag_series.data_ptr())
        self._check(self._lib.lbw_set_diagnostics_every(self._h, int(every), ptr,
                                                        int(capacity) if every > 0 else 0))
        return self

    def diagnostics_series(self):
        """The rows recorded since record_diagnostics() (numpy, rows x 8:
        sum n, field energy, kinetic energy, Gauss residual, max lattice Mach,
        non-finite nodes, recovery fallbacks, step); synchronises the stream."""
        rows = int(self._lib.lbw_diagnostics_rows(self._h))
        series = getattr(self, "_diag_series", None)
        if series is None:
            return np.zeros((0, 8))
        self.stream.synchronize()
        return series[:min(rows, series.shape[0])].cpu().numpy()

    @property
    def step_count(self):
        return int(self._lib.lbw_step_count(self._h))

    def read(self, which):
        out = np.empty(self.shape, dtype=np.float64)
        self._check(self._lib.lbw_read_moment(self._h, _lib.MOMENTS[which], _dp(out), out.size))
        return out if self.dims == 2 else out[0]

    def read_device(self, which):
        """The observable as a device tensor, written on the simulation's
        stream (work on another stream must wait for it)."""
        import torch

        with torch.cuda.stream(self.stream):
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check(self._lib.lbw_read_moment_device(self._h, _lib.MOMENTS[which],
                                                     ctypes.c_void_p(out.data_ptr())))
        return out

    def field(self, which, at_nodes=True):
        out = np.empty(self.shape, dtype=np.float64)
        self._check(self._lib.lbw_read_field(self._h, _lib.FIELDS[which], int(bool(at_nodes)),
                                             _dp(out), out.size))
        return out if self.dims == 2 else out[0]

    def diagnostics(self, check=True):
        out = np.zeros(8)
        rc = self._lib.lbw_diagnostics(self._h, _dp(out))
        if check:
            self._check(rc)
        return out

    def set_timing(self, enable=True):
        self._check(self._lib.lbw_set_timing(self._h, int(bool(enable))))
        return self

    def get_timing(self):
        """(summed fused-kernel milliseconds, launches) since set_timing(True)."""
        ms, n = ctypes.c_double(), ctypes.c_long()
        self._check(self._lib.lbw_get_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # device-side checkpoints (torch uint8 tensors on the simulation's device)
    def state_device_bytes(self):
        return int(self._lib.lbw_state_device_bytes(self._h))

    def save_state_device(self, out=None):
        import torch

        n = self.state_device_bytes()
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._check(self._lib.lbw_save_state_device(self._h, self._device_buffer(out, n, "save_state_device")))
        return out

    def step_record(self, nsteps, buf, stride=None):
        """Advance nsteps steps, writing the canonical state after each into
        ``buf`` (a uint8 device tensor) at offsets 0, stride, 2 stride, ..."""
        stride = self.state_device_bytes() if stride is None else int(stride)
        p = self._device_buffer(buf, nsteps * stride, "step_record")
        self._check(self._lib.lbw_step_record(self._h, int(nsteps), p, stride))
        return self

    def step_record_post(self, nsteps, buf, stride=None):
        """Advance nsteps steps, writing each fused launch's output (the
        post-collision populations and the fields) into ``buf`` at offsets
        0, stride, 2 stride, ... (lbw_step_record_post)."""
        stride = self.state_device_bytes() if stride is None else int(stride)
        p = self._device_buffer(buf, nsteps * stride, "step_record_post")
        self._check(self._lib.lbw_step_record_post(self._h, int(nsteps), p, stride))
        return self

    def load_state_device(self, buf, step):
        p = self._device_buffer(buf, self.state_device_bytes(), "load_state_device")
        self._check(self._lib.lbw_load_state_device(self._h, p, int(step)))
        return self

    def save_state(self) -> bytes:
        n = self._lib.lbw_state_bytes(self._h)
        buf = ctypes.create_string_buffer(n)
        self._check(self._lib.lbw_save_state(self._h, ctypes.cast(buf, ctypes.c_void_p), n))
        return buf.raw

    def save_state_async(self, buf):
        """Queue a checkpoint into ``buf``, a pinned uint8 CPU tensor of
        lbw_state_bytes() bytes, on the simulation's stream and return at once;
        synchronise the stream before reading it (bytes(buf.numpy()))."""
        import torch

        n = self._lib.lbw_state_bytes(self._h)
        if not isinstance(buf, torch.Tensor) or buf.is_cuda or buf.dtype != torch.uint8 or not buf.is_contiguous():
            raise ValueError("save_state_async: a contiguous uint8 CPU tensor is required")
        if not buf.is_pinned():
            raise ValueError("save_state_async: the tensor must be pinned (pin_memory=True)")
        if buf.numel() < n:
            raise ValueError(f"save_state_async: {buf.numel()} bytes, {n} needed")
        self._check(self._lib.lbw_save_state_async(self._h, ctypes.c_void_p(buf.data_ptr()), n))
        return buf

    def load_state(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        self._check(self._lib.lbw_load_state(self._h, ctypes.cast(buf, ctypes.c_void_p), len(data)))
        return self
