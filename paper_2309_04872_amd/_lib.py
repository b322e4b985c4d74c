"""ctypes declarations of the C ABI in ``include/lbwake.h`` (argument
marshalling only; every step of the method runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "liblbwake.so")

LBW_OK = 0
STATUS = {
    0: "LBW_OK", -1: "LBW_ERR_ARG", -2: "LBW_ERR_WORKSPACE", -3: "LBW_ERR_HIP",
    -4: "LBW_ERR_UNSTABLE", -5: "LBW_ERR_NONFINITE", -6: "LBW_ERR_STATE", -7: "LBW_ERR_UNSUPPORTED",
}
CLOSURES = {"lec": 0, "warmc": 1}
STORAGE = {"fp64": 0, "fp32": 1, "fp16dev": 2}
BCS = {"open": 0, "periodic": 1}
GEOMS = {"slab": 0, "axi": 1}
MOMENTS = {
    "n": 0, "uz": 1, "ux": 2, "gamma": 3, "n0": 4, "p0": 5, "lambda": 6, "thzz": 7, "thxx": 8,
    "thyy": 9, "thxz": 10, "ppar": 11, "mz": 12, "mx": 13,
}
FIELDS = {"ez": 0, "ex": 1, "by": 2, "wake_x": 3}

# Every symbol include/lbwake.h declares.
EXPORTS = [
    "lbw_workspace_bytes", "lbw_create", "lbw_init_plasma", "lbw_init_moments", "lbw_init_driver",
    "lbw_set_field", "lbw_step", "lbw_set_nonfinite_check", "lbw_set_diagnostics_every", "lbw_diagnostics_rows", "lbw_read_moment", "lbw_read_moment_device", "lbw_read_field",
    "lbw_diagnostics", "lbw_diagnostics_static", "lbw_step_count", "lbw_set_timing", "lbw_get_timing", "lbw_state_bytes", "lbw_save_state", "lbw_save_state_async", "lbw_load_state",
    "lbw_last_error", "lbw_version", "lbw_destroy",
    "lbw_state_device_bytes", "lbw_save_state_device", "lbw_load_state_device", "lbw_step_record",
    "lbw_step_record_post", "lbw_adjoint_step_post",
    "lbw_adjoint_bytes", "lbw_adjoint_workspace_bytes", "lbw_adjoint_step", "lbw_adjoint_init_fields",
    "lbw_batch_workspace_bytes", "lbw_batch_create", "lbw_batch_init", "lbw_batch_step",
    "lbw_batch_set_config", "lbw_batch_get_config", "lbw_batch_set_schedule", "lbw_batch_get_schedule",
    "lbw_batch_autotune", "lbw_batch_read",
    "lbw_batch_nonfinite", "lbw_batch_step_count", "lbw_batch_get_timing", "lbw_batch_last_error",
    "lbw_batch_destroy", "lbw_stream_copy",
]
BATCH_EZ = 100


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int), ("nz", ctypes.c_int), ("nx", ctypes.c_int),
        ("delta", ctypes.c_double), ("dt", ctypes.c_double), ("tau_tilde", ctypes.c_double),
        ("closure", ctypes.c_int), ("dvel", ctypes.c_double), ("storage", ctypes.c_int),
        ("bc_z", ctypes.c_int), ("bc_x", ctypes.c_int), ("geom", ctypes.c_int),
    ]


_dp = ctypes.POINTER(ctypes.c_double)


class InstanceDesc(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int), ("closure", ctypes.c_int), ("dvel", ctypes.c_double),
        ("mu", ctypes.c_double), ("delta", ctypes.c_double), ("dt", ctypes.c_double),
        ("tau_tilde", ctypes.c_double), ("bc", ctypes.c_int), ("alpha", ctypes.c_double),
        ("sigma_z", ctypes.c_double), ("z0", ctypes.c_double),
    ]


class PlasmaDesc(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("n_init", _dp), ("uz_init", _dp), ("ux_init", _dp)]


class DriverDesc(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double), ("sigma_z", ctypes.c_double), ("sigma_x", ctypes.c_double),
        ("z0", ctypes.c_double), ("x0", ctypes.c_double), ("nslices", ctypes.c_int),
        ("slice_w", _dp), ("slice_zmin", ctypes.c_double), ("slice_zmax", ctypes.c_double),
    ]


_LIB = None


class LibraryMissing(RuntimeError):
    pass


def load(path: str | None = None):
    """Load ``liblbwake.so``; raises LibraryMissing (no fallback of any kind)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or SO_PATH
    if not os.path.exists(p):
        raise LibraryMissing(
            f"{p} is missing: build the HIP library first (python -m paper_2309_04872_amd.build)")
    # torch (and the HIP runtime it brings) before the library: a process
    # that loaded the library first and torch afterwards found no GPU at the
    # library's first HIP call
    import torch  # noqa: F401

    L = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    L.lbw_workspace_bytes.restype = ctypes.c_size_t
    L.lbw_workspace_bytes.argtypes = [ctypes.POINTER(GridDesc)]
    L.lbw_create.restype = ctypes.c_int
    L.lbw_create.argtypes = [ctypes.POINTER(GridDesc), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.lbw_init_plasma.restype = ctypes.c_int
    L.lbw_init_plasma.argtypes = [vp, ctypes.POINTER(PlasmaDesc)]
    L.lbw_init_moments.restype = ctypes.c_int
    L.lbw_init_moments.argtypes = [vp, ctypes.c_double, _dp, _dp, _dp]
    L.lbw_init_driver.restype = ctypes.c_int
    L.lbw_init_driver.argtypes = [vp, ctypes.POINTER(DriverDesc), ctypes.c_int]
    L.lbw_set_field.restype = ctypes.c_int
    L.lbw_set_field.argtypes = [vp, ctypes.c_int, _dp, ctypes.c_size_t]
    L.lbw_step.restype = ctypes.c_int
    L.lbw_step.argtypes = [vp, ctypes.c_int]
    L.lbw_set_nonfinite_check.restype = ctypes.c_int
    L.lbw_set_nonfinite_check.argtypes = [vp, ctypes.c_int]
    L.lbw_set_diagnostics_every.restype = ctypes.c_int
    L.lbw_set_diagnostics_every.argtypes = [vp, ctypes.c_int, vp, ctypes.c_long]
    L.lbw_diagnostics_rows.restype = ctypes.c_long
    L.lbw_diagnostics_rows.argtypes = [vp]
    L.lbw_read_moment.restype = ctypes.c_int
    L.lbw_read_moment.argtypes = [vp, ctypes.c_int, _dp, ctypes.c_size_t]
    L.lbw_read_moment_device.restype = ctypes.c_int
    L.lbw_read_moment_device.argtypes = [vp, ctypes.c_int, vp]
    L.lbw_read_field.restype = ctypes.c_int
    L.lbw_read_field.argtypes = [vp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_size_t]
    L.lbw_diagnostics.restype = ctypes.c_int
    L.lbw_diagnostics.argtypes = [vp, _dp]
    L.lbw_diagnostics_static.restype = ctypes.c_int
    L.lbw_diagnostics_static.argtypes = [vp, vp]
    L.lbw_step_count.restype = ctypes.c_long
    L.lbw_step_count.argtypes = [vp]
    L.lbw_set_timing.restype = ctypes.c_int
    L.lbw_set_timing.argtypes = [vp, ctypes.c_int]
    L.lbw_get_timing.restype = ctypes.c_int
    L.lbw_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long)]
    L.lbw_state_bytes.restype = ctypes.c_size_t
    L.lbw_state_bytes.argtypes = [vp]
    L.lbw_save_state.restype = ctypes.c_int
    L.lbw_save_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbw_save_state_async.restype = ctypes.c_int
    L.lbw_save_state_async.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbw_load_state.restype = ctypes.c_int
    L.lbw_load_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbw_last_error.restype = ctypes.c_char_p
    L.lbw_last_error.argtypes = [vp]
    L.lbw_version.restype = ctypes.c_char_p
    L.lbw_version.argtypes = []
    L.lbw_destroy.restype = None
    L.lbw_destroy.argtypes = [vp]
    L.lbw_step_record.restype = ctypes.c_int
    L.lbw_step_record.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t]
    L.lbw_step_record_post.restype = ctypes.c_int
    L.lbw_step_record_post.argtypes = [vp, ctypes.c_int, vp, ctypes.c_size_t]
    L.lbw_adjoint_step_post.restype = ctypes.c_int
    L.lbw_adjoint_step_post.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_long, vp, vp, vp]
    L.lbw_state_device_bytes.restype = ctypes.c_size_t
    L.lbw_state_device_bytes.argtypes = [vp]
    L.lbw_save_state_device.restype = ctypes.c_int
    L.lbw_save_state_device.argtypes = [vp, vp]
    L.lbw_load_state_device.restype = ctypes.c_int
    L.lbw_load_state_device.argtypes = [vp, vp, ctypes.c_long]
    L.lbw_adjoint_bytes.restype = ctypes.c_size_t
    L.lbw_adjoint_bytes.argtypes = [vp]
    L.lbw_adjoint_workspace_bytes.restype = ctypes.c_size_t
    L.lbw_adjoint_workspace_bytes.argtypes = [vp]
    L.lbw_adjoint_step.restype = ctypes.c_int
    L.lbw_adjoint_step.argtypes = [vp, vp, vp, ctypes.c_long, vp, vp, vp]
    L.lbw_adjoint_init_fields.restype = ctypes.c_int
    L.lbw_adjoint_init_fields.argtypes = [vp, vp, vp, vp]
    ip = ctypes.POINTER(ctypes.c_int)
    L.lbw_batch_workspace_bytes.restype = ctypes.c_size_t
    L.lbw_batch_workspace_bytes.argtypes = [ctypes.POINTER(InstanceDesc), ctypes.c_int]
    L.lbw_batch_create.restype = ctypes.c_int
    L.lbw_batch_create.argtypes = [ctypes.POINTER(InstanceDesc), ctypes.c_int, vp, ctypes.c_size_t, vp,
                                   ctypes.POINTER(vp)]
    L.lbw_batch_init.restype = ctypes.c_int
    L.lbw_batch_init.argtypes = [vp, _dp]
    L.lbw_batch_step.restype = ctypes.c_int
    L.lbw_batch_step.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.lbw_batch_set_config.restype = ctypes.c_int
    L.lbw_batch_set_config.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.lbw_batch_get_config.restype = ctypes.c_int
    L.lbw_batch_get_config.argtypes = [vp, ip, ip]
    L.lbw_batch_set_schedule.restype = ctypes.c_int
    L.lbw_batch_set_schedule.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.lbw_batch_get_schedule.restype = ctypes.c_int
    L.lbw_batch_get_schedule.argtypes = [vp, ip, ip, ip, ip]
    L.lbw_batch_autotune.restype = ctypes.c_int
    L.lbw_batch_autotune.argtypes = [vp, ctypes.c_int, ip, ip]
    L.lbw_batch_read.restype = ctypes.c_int
    L.lbw_batch_read.argtypes = [vp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_size_t]
    L.lbw_batch_nonfinite.restype = ctypes.c_int
    L.lbw_batch_nonfinite.argtypes = [vp, ip]
    L.lbw_batch_step_count.restype = ctypes.c_long
    L.lbw_batch_step_count.argtypes = [vp]
    L.lbw_batch_get_timing.restype = ctypes.c_int
    L.lbw_batch_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.lbw_batch_last_error.restype = ctypes.c_char_p
    L.lbw_batch_last_error.argtypes = [vp]
    L.lbw_batch_destroy.restype = None
    L.lbw_batch_destroy.argtypes = [vp]
    L.lbw_stream_copy.restype = ctypes.c_int
    L.lbw_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    if path is None:
        _LIB = L
    return L
