"""Plain FP64 CPU oracle of the moment-matching lattice Boltzmann scheme for
warm relativistic plasma wakes (Simeoni et al., arXiv 2309.04872).

TEST INFRASTRUCTURE. Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no
code with the GPU library ``paper_2309_04872_amd``; the C source is
``oracle/lbw_oracle.c`` (every function cites the passage of the paper it
follows).

Parity status (the ``-m "not gpu"`` tests under ``tests/test_oracle_*.py``):
- pinned against closed forms of the paper and of the mathematics: the
  equilibrium's moment identities, both recoveries (round trips, mass-shell
  identities), the pressure read-out (double boost), the bare ADE (Gaussian
  advection-diffusion with kappa = nu^2 (tau - dt/2)), number conservation,
  the rest state, the k = 0 oscillation (exact discrete recurrence and the
  continuum frequency, 1D and 2D, with and without a uniform B_y), the
  finite-k Langmuir dispersion along z and x, the transverse electromagnetic
  wave along z and x, the cold linear wake and the warm wake wavelength, the
  relativistic and warm nonlinear uniform oscillations (exact periods, energy
  and trace-condition invariants), the initial fields, mirror symmetry, and
  rotation covariance in the (x, z) plane (a large-amplitude wave travelling
  obliquely against the same wave along z, converging with resolution), which
  pins the 2D-only nonlinear cross terms of the warm closure (products of two
  perturbations, e.g. theta^{xz} d_x(lambda u_z));
- axisymmetric geometry (``tests/test_oracle_axi.py``): pinned by the
  cylindrical Gauss law, the local cold wake, an exact nonlinear breathing
  column, the column's Langmuir modes, and a breathing column carrying a
  shear temperature theta^{rz} = b(t) r, whose b' = -4 a b at order a b pins
  the nonlinear source -u_r lambda theta^{rz} / r of the warm closure;
- diagnostics (``tests/test_oracle_diagnostics.py``): the field and kinetic
  energies against the conserved energy of uniform cold oscillations and the
  closed-form energy of the bunch's initial field, the axisymmetric volume
  weights against exact column sums, max |u| / Lambda against the imposed
  flow.
The diagnostics pins and the theta^{rz} pin are shown to fail for planted
mistakes compiled by ``variant()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblbw_oracle.so")
_SRC = os.path.join(_HERE, "lbw_oracle.c")

LEC, WARMC = 0, 1
OPEN, PERIODIC = 0, 1

OBS = {
    "n": 0, "uz": 1, "ux": 2, "gamma": 3, "n0": 4, "p0": 5, "lambda": 6,
    "thzz": 7, "thxx": 8, "thyy": 9, "thxz": 10, "ppar": 11,
    "ez": 12, "ex": 13, "by": 14, "ez_yee": 15, "ex_yee": 16, "by_yee": 17,
    "mz": 18, "mx": 19,
}


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liblbw_oracle.so`` (gcc, -O2, OpenMP,
    no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


SLAB, AXI = 0, 1  # geometries: Cartesian (z, x) | axisymmetric (z, r)


class _Params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int), ("nz", ctypes.c_int), ("nx", ctypes.c_int),
        ("delta", ctypes.c_double), ("dt", ctypes.c_double),
        ("tau_tilde", ctypes.c_double), ("closure", ctypes.c_int),
        ("dvel", ctypes.c_double), ("bc_z", ctypes.c_int), ("bc_x", ctypes.c_int),
        ("mu", ctypes.c_double), ("alpha", ctypes.c_double),
        ("sigma_z", ctypes.c_double), ("sigma_x", ctypes.c_double),
        ("z0", ctypes.c_double), ("x0", ctypes.c_double),
        ("nslices", ctypes.c_int), ("slice_zmin", ctypes.c_double),
        ("slice_zmax", ctypes.c_double), ("slice_w", ctypes.POINTER(ctypes.c_double)),
        ("geom", ctypes.c_int),
    ]


_lib = None


def _configure(L):
    """Argument and result types of the oracle's C entry points."""
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_create.restype = ctypes.c_void_p
    L.orc_create.argtypes = [ctypes.POINTER(_Params)]
    L.orc_destroy.argtypes = [ctypes.c_void_p]
    L.orc_init.argtypes = [ctypes.c_void_p, dp, dp, dp, ctypes.c_int]
    L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.orc_step_count.restype = ctypes.c_long
    L.orc_step_count.argtypes = [ctypes.c_void_p]
    L.orc_get.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    L.orc_diagnostics.argtypes = [ctypes.c_void_p, dp]
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_feq.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, ctypes.c_double, dp]
    L.orc_lec_recover.restype = ctypes.c_int
    L.orc_lec_recover.argtypes = [ctypes.c_double] * 5 + [dp]
    L.orc_warmc_recover.argtypes = [ctypes.c_int, dp, dp]
    L.orc_ppar.restype = ctypes.c_double
    L.orc_ppar.argtypes = [ctypes.c_double] * 6
    L.orc_lambda0.restype = ctypes.c_double
    L.orc_lambda0.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_init_moments.argtypes = [ctypes.c_void_p, dp, dp, dp]
    L.orc_set_yee.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    L.orc_num_scalars.restype = ctypes.c_int
    L.orc_num_scalars.argtypes = [ctypes.c_void_p]
    L.orc_ade_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_int,
                              ctypes.c_double, ctypes.c_double, dp, ctypes.c_int, dp]
    L.orc_bunch.restype = ctypes.c_double
    L.orc_bunch.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = _configure(ctypes.CDLL(_SO))
    return _lib


def variant(tag, replacements):
    """A copy of the oracle with planted mistakes, for tests showing that a
    pin fails when the arithmetic it covers is wrong. ``replacements`` is a
    list of (old, new) source strings; each ``old`` must occur exactly once in
    ``lbw_oracle.c``. The copy is compiled with the same flags into a
    temporary directory and returned as a loaded library, to be passed to
    ``Oracle(..., library=...)``."""
    import tempfile

    src = open(_SRC).read()
    for old, new in replacements:
        if src.count(old) != 1:
            raise ValueError(f"planted mistake {tag!r}: {old!r} occurs {src.count(old)} times")
        src = src.replace(old, new)
    d = os.path.join(tempfile.gettempdir(), f"lbw_oracle_variant_{os.getpid()}")
    os.makedirs(d, exist_ok=True)
    c, so = os.path.join(d, f"{tag}.c"), os.path.join(d, f"lib{tag}.so")
    with open(c, "w") as fh:
        fh.write(src)
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-I", _HERE, "-w", c, "-o", so, "-lm"], check=True)
    return _configure(ctypes.CDLL(so))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


class Oracle:
    """One simulation on the CPU oracle. Keyword arguments mirror the C
    ``orc_params`` fields; arrays are [nx][nz] with z fastest. ``library``: a
    planted-mistake copy from ``variant()`` (default: the oracle itself)."""

    def __init__(self, dims, nz, nx=1, delta=2 * np.pi / 128, dt=None, tau_tilde=None,
                 closure=LEC, dvel=None, bc_z=OPEN, bc_x=OPEN, mu=1e-3, alpha=0.0,
                 sigma_z=1.0, sigma_x=1.0, z0=None, x0=0.0, slice_w=None,
                 slice_zmin=0.0, slice_zmax=0.0, geom=0, library=None):
        if dt is None:
            dt = 0.1 * delta
        if tau_tilde is None:
            tau_tilde = 0.52 if dims == 1 else 0.53
        if dvel is None:
            dvel = 1.0 if dims == 1 else 3.0
        if z0 is None:
            z0 = 6.0 * sigma_z
        self._L = library if library is not None else lib()
        self._keep = None
        p = _Params(dims, nz, nx, delta, dt, tau_tilde, closure, float(dvel), bc_z, bc_x,
                    mu, alpha, sigma_z, sigma_x, z0, x0, 0, slice_zmin, slice_zmax, None, int(geom))
        if slice_w is not None:
            w = np.ascontiguousarray(slice_w, dtype=np.float64)
            self._keep = w
            p.nslices = len(w)
            p.slice_w = _dp(w)
        self.params = p
        self.dims, self.nz, self.nx = dims, nz, nx
        self.shape = (nx, nz)
        h = self._L.orc_create(ctypes.byref(p))
        if not h:
            raise ValueError("oracle rejected the parameters")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and getattr(self, "_L", None) is not None:
            self._L.orc_destroy(h)
            self._h = None

    def _arr(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), self.shape))
        return a

    def init(self, n=None, uz=None, ux=None, fields_from_driver=True):
        n, uz, ux = self._arr(n), self._arr(uz), self._arr(ux)
        self._init_keep = (n, uz, ux)
        self._L.orc_init(self._h, _dp(n) if n is not None else None,
                         _dp(uz) if uz is not None else None,
                         _dp(ux) if ux is not None else None, int(bool(fields_from_driver)))
        return self

    @property
    def nscalars(self):
        return int(self._L.orc_num_scalars(self._h))

    def init_moments(self, A, uz=None, ux=None):
        """Equilibrium populations of arbitrary scalars A[K][nx][nz] (1D: A[K][nz])."""
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(self.nscalars, *self.shape))
        uz, ux = self._arr(uz), self._arr(ux)
        self._init_keep = (A, uz, ux)
        self._L.orc_init_moments(self._h, _dp(A), _dp(uz) if uz is not None else None,
                                 _dp(ux) if ux is not None else None)
        return self

    def set_yee(self, which, v):
        """Overwrite a raw Yee array: 'ez', 'ex' (E^n) or 'by' (B^{n-1/2})."""
        v = self._arr(v)
        self._L.orc_set_yee(self._h, {"ez": 0, "ex": 1, "by": 2}[which], _dp(v))
        return self

    def step(self, nsteps=1):
        self._L.orc_step(self._h, int(nsteps))
        return self

    @property
    def step_count(self):
        return int(self._L.orc_step_count(self._h))

    def get(self, which):
        out = np.empty(self.shape, dtype=np.float64)
        rc = self._L.orc_get(self._h, OBS[which], _dp(out))
        if rc != 0:
            raise ValueError(which)
        return out if self.dims == 2 else out[0]

    def diagnostics(self):
        out = np.zeros(8)
        self._L.orc_diagnostics(self._h, _dp(out))
        return out

    def bunch(self, z, x, t):
        return self._L.orc_bunch(self._h, z, x, t)


def feq(dims, A, uz, ux, lattice_speed):
    out = np.zeros(3 if dims == 1 else 9)
    lib().orc_feq(dims, A, uz, ux, lattice_speed, _dp(out))
    return out


def lec_recover(n, A1z, A1x, D, mu):
    out = np.zeros(4)
    lib().orc_lec_recover(n, A1z, A1x, D, mu, _dp(out))
    return out


def warmc_recover(dims, A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.zeros(12)
    lib().orc_warmc_recover(dims, _dp(A), _dp(out))
    return out


def ppar(thxx, thyy, thzz, th00, ux, uz):
    return lib().orc_ppar(thxx, thyy, thzz, th00, ux, uz)


def ade_run(dims, A, delta, dt, tau_tilde, uz, ux=0.0, nsteps=1, bc=PERIODIC):
    """Bare moment-matching ADE run (constant u, no forcing) of one scalar."""
    A = np.ascontiguousarray(np.atleast_2d(np.asarray(A, dtype=np.float64)))
    nx, nz = A.shape
    out = np.empty_like(A)
    rc = lib().orc_ade_run(dims, nz, nx, delta, dt, tau_tilde, bc, uz, ux, _dp(A),
                           int(nsteps), _dp(out))
    if rc != 0:
        raise ValueError("ade_run rejected the parameters")
    return out if dims == 2 else out[0]


def lambda0(mu, D):
    return lib().orc_lambda0(mu, D)
