"""ctypes view of include/pwbf.h and the loader of libpwbf.so.

The loader never falls back to anything: if the HIP library is not built it
raises, so no result can come from a CPU path by accident.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpwbf.so")

ABI_VERSION = 6
OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_DEVICE, E_BUSY, E_TIMEOUT = 0, -1, -2, -3, -4, -5, -6
FK_STOLT, FK_LU = 0, 1
I16, F16, F32, C32 = 0, 1, 2, 3
DAS, DMAS, PDAS, IQDAS, BBDMAS = 0, 1, 2, 3, 4
APOD_HANN, APOD_BOXCAR, APOD_NONE = 0, 1, 2
MAX_ANGLES, MAX_CHANNELS, MAX_NZ_POST = 32, 256, 4096
NOALLOC_ENV_PIXELS = 1 << 22

ERROR_NAMES = {E_INVALID: "PWBF_E_INVALID", E_UNSUPPORTED: "PWBF_E_UNSUPPORTED",
               E_NOMEM: "PWBF_E_NOMEM", E_DEVICE: "PWBF_E_DEVICE", E_BUSY: "PWBF_E_BUSY",
               E_TIMEOUT: "PWBF_E_TIMEOUT"}


class Geometry(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("n_angles", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("n_samples", ctypes.c_int32),
        ("elem_x", ctypes.POINTER(ctypes.c_double)),
        ("angle_rad", ctypes.POINTER(ctypes.c_double)),
        ("t0", ctypes.POINTER(ctypes.c_double)),
        ("c", ctypes.c_double),
        ("fs", ctypes.c_double),
        ("f0", ctypes.c_double),
        ("nx", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("x0", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("z0", ctypes.c_double),
        ("dz", ctypes.c_double),
        ("f_number", ctypes.c_double),
        ("apod", ctypes.c_int32),
        ("bandpass", ctypes.c_int32),
        ("log_floor_db", ctypes.c_double), ("pdas_p", ctypes.c_double),
        ("iq_decimation", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class Outputs(ctypes.Structure):
    _fields_ = [("rf", ctypes.c_void_p), ("filtered", ctypes.c_void_p),
                ("env", ctypes.c_void_p), ("logimg", ctypes.c_void_p), ("imag", ctypes.c_void_p)]


class Tile(ctypes.Structure):
    _fields_ = [("cpw", ctypes.c_int32), ("lz", ctypes.c_int32), ("wz", ctypes.c_int32),
                ("wx", ctypes.c_int32), ("chunk", ctypes.c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [("geom", ctypes.POINTER(Geometry)), ("rf", ctypes.c_void_p),
                ("rf_dtype", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("angle", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("out", Outputs), ("tile", Tile)]


class BatchInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("n_frames", "n_items", "n_columns", "blocks",
                                               "blocks_per_cu", "lds_bytes", "graph_nodes",
                                               "kernels", "branches")]


BATCH_TUNE = 1


class Disc(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("z", ctypes.c_double), ("r", ctypes.c_double)]


class Cyst(ctypes.Structure):
    _fields_ = [("inside", Disc), ("out", Disc)]


class Contrast(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("mu_in", "mu_out", "sigma_in", "sigma_out",
                                               "cr_db", "cnr")] + \
               [("n_in", ctypes.c_int32), ("n_out", ctypes.c_int32)]


class Resolution(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("peak", "fwhm_x", "fwhm_z")] + \
               [("ix", ctypes.c_int32), ("iz", ctypes.c_int32)]


MAX_METRIC_REGIONS = 32


class Probe(ctypes.Structure):
    _fields_ = [("geom", ctypes.POINTER(Geometry)), ("mode", ctypes.c_int32),
                ("angle", ctypes.c_int32), ("want_env", ctypes.c_int32),
                ("want_log", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("want_quality", ctypes.c_int32), ("quality_region", Cyst),
                ("quality_max_cr_db", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("probe", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double),
                ("rf", ctypes.c_void_p), ("env", ctypes.c_void_p), ("logimg", ctypes.c_void_p),
                ("status", ctypes.c_int32), ("quality_ok", ctypes.c_int32),
                ("frame_max", ctypes.c_float), ("cr_db", ctypes.c_float),
                ("cnr", ctypes.c_float)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("mean_batch", ctypes.c_double), ("budget_bytes", ctypes.c_size_t),
                ("budget_in_use", ctypes.c_size_t), ("budget_peak", ctypes.c_size_t),
                ("expired", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("cpw", ctypes.c_int32), ("lz", ctypes.c_int32), ("wz", ctypes.c_int32),
        ("wx", ctypes.c_int32), ("chunk", ctypes.c_int32), ("tile_z", ctypes.c_int32),
        ("tile_x", ctypes.c_int32), ("win", ctypes.c_int32), ("off_t", ctypes.c_int32),
        ("off_r", ctypes.c_int32), ("tiles_z", ctypes.c_int32),
        ("tiles_x", ctypes.c_int32), ("threads_per_block", ctypes.c_int32),
        ("blocks", ctypes.c_int32), ("n_angles_used", ctypes.c_int32),
        ("lds_bytes", ctypes.c_int64),
        ("X0", ctypes.c_float), ("DX", ctypes.c_float), ("Z0", ctypes.c_float),
        ("DZ", ctypes.c_float), ("X0l", ctypes.c_float), ("DXl", ctypes.c_float),
        ("Z0l", ctypes.c_float), ("DZl", ctypes.c_float), ("ap_k", ctypes.c_float),
        ("sa", ctypes.c_float * MAX_ANGLES), ("sal", ctypes.c_float * MAX_ANGLES),
        ("ca", ctypes.c_float * MAX_ANGLES), ("cal", ctypes.c_float * MAX_ANGLES),
        ("to", ctypes.c_float * MAX_ANGLES), ("tol", ctypes.c_float * MAX_ANGLES),
        ("xe", ctypes.c_float * MAX_CHANNELS), ("xel", ctypes.c_float * MAX_CHANNELS),
    ]


_lib = None


def lib():
    """Load libpwbf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2311_00482_amd.build)")
    try:
        # torch first: libpwbf then binds to the HIP runtime torch already holds
        # (same soname), so device pointers and streams are shared
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    G, O, T, PI = (ctypes.POINTER(Geometry), ctypes.POINTER(Outputs), ctypes.POINTER(Tile),
                   ctypes.POINTER(PlanInfo))
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    L.pwbf_abi_version.restype = ctypes.c_uint32
    L.pwbf_abi_version.argtypes = []
    L.pwbf_last_error.restype = ctypes.c_char_p
    L.pwbf_last_error.argtypes = []
    L.pwbf_workspace_bytes.restype = sz
    L.pwbf_workspace_bytes.argtypes = [G, O]
    for name in ("pwbf_beamform_das", "pwbf_beamform_dmas", "pwbf_beamform_pdas"):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [G, vp, i32, i32, O, vp, sz, vp]
    L.pwbf_contrast_metrics.restype = ctypes.c_int
    L.pwbf_contrast_metrics.argtypes = [G, vp, ctypes.POINTER(Cyst), i32, vp, vp]
    L.pwbf_resolution_metrics.restype = ctypes.c_int
    L.pwbf_resolution_metrics.argtypes = [G, vp, ctypes.POINTER(Disc), i32, vp, vp]
    L.pwbf_iq_demodulate.restype = ctypes.c_int
    L.pwbf_iq_demodulate.argtypes = [G, vp, i32, vp, vp]
    L.pwbf_fk_workspace_bytes.restype = sz
    L.pwbf_fk_workspace_bytes.argtypes = [G, i32, i32, O]
    L.pwbf_fk_migrate.restype = ctypes.c_int
    L.pwbf_fk_migrate.argtypes = [G, vp, i32, i32, i32, O, vp, sz, vp]
    for name in ("pwbf_beamform_iqdas", "pwbf_beamform_bbdmas"):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [G, vp, i32, O, vp, sz, vp]
    L.pwbf_compound.restype = ctypes.c_int
    L.pwbf_compound.argtypes = [G, vp, i32, i32, O, vp, sz, vp]
    L.pwbf_compound_noalloc.restype = ctypes.c_int
    L.pwbf_compound_noalloc.argtypes = [G, vp, i32, i32, O, vp]
    L.pwbf_beamform_ex.restype = ctypes.c_int
    L.pwbf_beamform_ex.argtypes = [G, vp, i32, i32, i32, T, O, vp, sz, vp]
    L.pwbf_validate_call.restype = ctypes.c_int
    L.pwbf_validate_call.argtypes = [G, vp, i32, i32, i32, T, O, vp, sz]
    L.pwbf_describe_plan.restype = ctypes.c_int
    L.pwbf_describe_plan.argtypes = [G, i32, i32, T, PI]
    F, BI = ctypes.POINTER(Frame), ctypes.POINTER(BatchInfo)
    L.pwbf_batch_create.restype = ctypes.c_int
    L.pwbf_batch_create.argtypes = [F, i32, i32, vp, ctypes.POINTER(vp)]
    L.pwbf_batch_update.restype = ctypes.c_int
    L.pwbf_batch_update.argtypes = [vp, F, i32, vp]
    L.pwbf_batch_launch.restype = ctypes.c_int
    L.pwbf_batch_launch.argtypes = [vp, vp]
    L.pwbf_batch_describe.restype = ctypes.c_int
    L.pwbf_batch_describe.argtypes = [vp, BI]
    L.pwbf_batch_destroy.restype = ctypes.c_int
    L.pwbf_batch_destroy.argtypes = [vp]
    L.pwbf_tune.restype = ctypes.c_int
    L.pwbf_tune.argtypes = [G, vp, i32, i32, i32, O, i32, vp, T, ctypes.POINTER(ctypes.c_float)]
    for name in ("pwbf_tune_save", "pwbf_tune_load"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [ctypes.c_char_p]
    L.pwbf_tune_clear.restype = ctypes.c_int
    L.pwbf_tune_clear.argtypes = []
    L.pwbf_server_create.restype = ctypes.c_int
    L.pwbf_server_create.argtypes = [ctypes.POINTER(Probe), i32, sz, i32, ctypes.POINTER(vp)]
    L.pwbf_server_submit.restype = ctypes.c_int
    L.pwbf_server_submit.argtypes = [vp, i32, vp, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_uint64)]
    L.pwbf_server_submit_ex.restype = ctypes.c_int
    L.pwbf_server_submit_ex.argtypes = [vp, i32, vp, ctypes.c_double, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_uint64)]
    L.pwbf_server_poll.restype = ctypes.c_int
    L.pwbf_server_poll.argtypes = [vp, ctypes.POINTER(Result), i32, ctypes.POINTER(i32), i32]
    L.pwbf_server_release.restype = ctypes.c_int
    L.pwbf_server_release.argtypes = [vp, ctypes.c_uint64]
    L.pwbf_server_stats_get.restype = ctypes.c_int
    L.pwbf_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.pwbf_server_now.restype = ctypes.c_double
    L.pwbf_server_now.argtypes = [vp]
    L.pwbf_server_destroy.restype = ctypes.c_int
    L.pwbf_server_destroy.argtypes = [vp]
    if L.pwbf_abi_version() != ABI_VERSION:
        raise ImportError(f"libpwbf ABI {L.pwbf_abi_version()} != binding {ABI_VERSION}")
    _lib = L
    return L


class PwbfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc: int) -> None:
    if rc != OK:
        raise PwbfError(rc, lib().pwbf_last_error().decode())
