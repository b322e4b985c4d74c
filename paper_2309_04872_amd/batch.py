"""Python binding of the batched 1D interface of the C ABI: many independent
1D runs advanced by one persistent kernel launch. Argument marshalling only;
PyTorch provides the device workspace and the stream."""
from __future__ import annotations

import ctypes
import sys

import numpy as np

from . import _lib, trace
from .sim import LbwError


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Batch:
    """``instances``: a list of dicts with keys nz, closure ('lec' | 'warmc'),
    mu, alpha, sigma_z and optionally dvel (1), delta (lambda_p / 128),
    dt (delta / 10), tau_tilde (0.52), bc ('open'), z0 (6 sigma_z)."""

    def __init__(self, instances, device="cuda:0", stream=None):
        import torch

        self._lib = _lib.load()
        descs = []
        for d in instances:
            delta = d.get("delta", 2 * np.pi / 128)
            descs.append(_lib.InstanceDesc(
                int(d["nz"]), _lib.CLOSURES[d["closure"]], float(d.get("dvel", 1.0)), float(d["mu"]),
                delta, d.get("dt", 0.1 * delta), d.get("tau_tilde", 0.52), _lib.BCS[d.get("bc", "open")],
                float(d.get("alpha", 0.0)), float(d.get("sigma_z", 1.0)),
                float(d.get("z0", 6.0 * d.get("sigma_z", 1.0)))))
        self.n = len(descs)
        self.nz = [d.nz for d in descs]
        arr = (_lib.InstanceDesc * self.n)(*descs)
        self._descs = arr
        nbytes = self._lib.lbw_batch_workspace_bytes(arr, self.n)
        if nbytes == 0:
            raise LbwError(-1, "invalid instance descriptor")
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        # allocated on the batch's stream, so that a freed workspace is reused
        # only after the work queued there
        with torch.cuda.stream(stream):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        rc = self._lib.lbw_batch_create(arr, self.n, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                        ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise LbwError(rc, "lbw_batch_create rejected the instances")
        self._h = h

    def _check(self, rc):
        if rc != 0:
            raise LbwError(rc, self._lib.lbw_batch_last_error(self._h).decode())

    def close(self):
        """Release the library handle (its HIP events and graphs). Call it
        before the interpreter shuts down."""
        if getattr(self, "_h", None):
            self._lib.lbw_batch_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter shutdown the HIP runtime may already be gone
        # (module globals such as sys may be None by then, hence the default)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def init(self, n=None):
        """Plasma at rest; ``n``: list of per-instance density arrays, or None."""
        flat = None
        if n is not None:
            flat = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.float64) for v in n]))
            if flat.size != sum(self.nz):
                raise ValueError("densities must cover every instance")
        self._check(self._lib.lbw_batch_init(self._h, _dp(flat)))
        return self

    def step(self, nsteps=1, graph=False):
        with trace.marker("lbw_batch_step"):
            self._check(self._lib.lbw_batch_step(self._h, int(nsteps), int(bool(graph))))
        return self

    @property
    def step_count(self):
        return int(self._lib.lbw_batch_step_count(self._h))

    def set_config(self, threads, nodes_per_thread=1):
        self._check(self._lib.lbw_batch_set_config(self._h, int(threads), int(nodes_per_thread)))
        return self

    def config(self):
        t, c = ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.lbw_batch_get_config(self._h, ctypes.byref(t), ctypes.byref(c)))
        return t.value, c.value

    def set_schedule(self, threads, nodes_per_thread=1, split=False):
        """Launch shape and schedule; split=True shares long instances among
        several co-resident workgroups (cooperative launch)."""
        self._check(self._lib.lbw_batch_set_schedule(self._h, int(threads), int(nodes_per_thread), int(bool(split))))
        return self

    def schedule(self):
        """(threads, nodes per thread, split, workgroups of a launch)."""
        v = [ctypes.c_int() for _ in range(4)]
        self._check(self._lib.lbw_batch_get_schedule(self._h, *[ctypes.byref(x) for x in v]))
        t, c, sp, wg = (x.value for x in v)
        return t, c, bool(sp), wg

    def autotune(self, probe_steps=20):
        t, c = ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.lbw_batch_autotune(self._h, int(probe_steps), ctypes.byref(t), ctypes.byref(c)))
        return t.value, c.value

    def read(self, i, which):
        out = np.empty(self.nz[i] if 0 <= i < self.n else 1, dtype=np.float64)
        code = _lib.BATCH_EZ if which == "ez" else _lib.MOMENTS[which]
        self._check(self._lib.lbw_batch_read(self._h, int(i), code, _dp(out), out.size))
        return out

    def nonfinite(self):
        out = np.zeros(self.n, dtype=np.int32)
        self._check(self._lib.lbw_batch_nonfinite(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return out

    def last_ms(self):
        """Milliseconds of the last step launch (HIP events on the batch's stream)."""
        ms = ctypes.c_double()
        self._check(self._lib.lbw_batch_get_timing(self._h, ctypes.byref(ms)))
        return ms.value
