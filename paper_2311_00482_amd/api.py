"""Python binding of libpwbf with the C ABI's names.

Argument marshalling only: geometry objects become ``pwbf_geometry``, torch
tensors become device pointers, the current torch stream becomes the HIP
stream. Every step of the beamformer runs in the HIP kernels of libpwbf.so;
torch provides device memory and streams.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Dict, Iterable, Optional, Tuple

import numpy as np

from . import _abi

_DTYPES = {"int16": _abi.I16, "float16": _abi.F16, "float32": _abi.F32, "complex64": _abi.C32}
_MODES = {"das": _abi.DAS, "dmas": _abi.DMAS, "pdas": _abi.PDAS, "iqdas": _abi.IQDAS,
          "bbdmas": _abi.BBDMAS}
_APODS = {"hann": _abi.APOD_HANN, "boxcar": _abi.APOD_BOXCAR, "none": _abi.APOD_NONE}
PLANES = ("rf", "filtered", "env", "log", "imag")


class GeometryArg:
    """A ``pwbf_geometry`` plus the host arrays it points to.

    ``g`` is any object with the attributes elem_x, angles_rad, n_samples, c,
    fs, f0, nx, nz, x0, dx, z0, dz, f_number and apod (name) or apod_code;
    t0_s (per-angle time of sample 0) is optional. ``pdas_p`` is the pDAS root
    order (used by mode "pdas" only); ``iq_decimation`` the decimation of
    baseband records (IQ demodulation and the IQ beamformers only).
    """

    def __init__(self, g, bandpass: bool = False, log_floor_db: float = -70.0,
                 pdas_p: float = 2.0, iq_decimation: int = 1):
        self.elem_x = np.ascontiguousarray(g.elem_x, dtype=np.float64)
        self.angles = np.ascontiguousarray(g.angles_rad, dtype=np.float64)
        t0 = getattr(g, "t0_s", None)
        self.t0 = None if t0 is None else np.ascontiguousarray(t0, dtype=np.float64)
        apod = getattr(g, "apod_code", None)
        if apod is None:
            apod = _APODS[g.apod]
        dp = ctypes.POINTER(ctypes.c_double)
        self.s = _abi.Geometry(
            _abi.ABI_VERSION, len(self.angles), len(self.elem_x), int(g.n_samples),
            self.elem_x.ctypes.data_as(dp), self.angles.ctypes.data_as(dp),
            self.t0.ctypes.data_as(dp) if self.t0 is not None else None,
            float(g.c), float(g.fs), float(g.f0), int(g.nx), int(g.nz), float(g.x0),
            float(g.dx), float(g.z0), float(g.dz), float(g.f_number), int(apod),
            1 if bandpass else 0, float(log_floor_db), float(pdas_p), int(iq_decimation), 0)
        self.nx, self.nz = int(g.nx), int(g.nz)
        self.shape_rf = (len(self.angles), len(self.elem_x), int(g.n_samples))
        # baseband records: decimated by iq_decimation along samples
        self.shape_iq = (len(self.angles), len(self.elem_x),
                         int(g.n_samples) // max(1, int(iq_decimation)))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _as_geom(g, bandpass=False, log_floor_db=-70.0) -> GeometryArg:
    return g if isinstance(g, GeometryArg) else GeometryArg(g, bandpass, log_floor_db)


def _stream_ptr(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(int(stream.cuda_stream))


def _rf_code(rf) -> int:
    name = str(rf.dtype).replace("torch.", "")
    if name not in _DTYPES:
        raise TypeError(f"RF dtype {rf.dtype} not supported (int16, float16, float32, "
                        "complex64 IQ)")
    return _DTYPES[name]


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


@dataclass
class Tile:
    """Launch shape (see pwbf_tile): lane groups, lanes along depth, waves, chunk."""
    cpw: int = 0
    lz: int = 0
    wz: int = 0
    wx: int = 0
    chunk: int = 0

    def c(self) -> _abi.Tile:
        return _abi.Tile(self.cpw, self.lz, self.wz, self.wx, self.chunk)


def workspace_bytes(g, want: Iterable[str] = ("rf",), bandpass=False) -> int:
    ga = _as_geom(g, bandpass)
    want = set(want)
    o = _abi.Outputs(1, 1 if "filtered" in want else None, 1 if "env" in want else None,
                     1 if "log" in want else None)
    n = _abi.lib().pwbf_workspace_bytes(ga.ref, ctypes.byref(o))
    err = _abi.lib().pwbf_last_error().decode()
    if err:
        raise _abi.PwbfError(_abi.E_INVALID, err)
    return int(n)


def describe_plan(g, mode: str = "das", angle: int = -1, tile: Optional[Tile] = None,
                  bandpass: bool = False) -> Dict:
    """The resolved launch shape and float32 constants of a call (no device work)."""
    ga = _as_geom(g, bandpass)
    info = _abi.PlanInfo()
    t = tile.c() if tile is not None else None
    _abi.check(_abi.lib().pwbf_describe_plan(ga.ref, _MODES[mode], angle,
                                             ctypes.byref(t) if t is not None else None,
                                             ctypes.byref(info)))
    out = {k: getattr(info, k) for k, _ in _abi.PlanInfo._fields_}
    for k in ("sa", "sal", "ca", "cal", "to", "tol", "xe", "xel"):
        out[k] = np.array(out[k][:], dtype=np.float32)
    return out


def alloc_outputs(g, want: Iterable[str], device) -> Dict[str, "object"]:
    import torch
    ga = _as_geom(g)
    return {k: torch.empty((ga.nx, ga.nz), dtype=torch.float32, device=device) for k in want}


def _prepare(g, rf, want, out, workspace, bandpass, log_floor_db, p, workspace_needed=True):
    """Marshal one frame's call: geometry, output planes (allocated when not
    given), workspace; returns (geometry, outputs struct, planes, ws ptr, ws bytes)."""
    import torch
    ga = _as_geom(g, bandpass, log_floor_db)
    if bandpass and not ga.s.bandpass:
        ga.s.bandpass = 1
    if p is not None:
        ga.s.pdas_p = float(p)
    if not rf.is_cuda or not rf.is_contiguous():
        raise ValueError("rf must be a contiguous CUDA tensor")
    shape = ga.shape_iq if rf.dtype == torch.complex64 else ga.shape_rf
    if tuple(rf.shape) != shape:
        raise ValueError(f"rf shape {tuple(rf.shape)} != {shape}")
    want = set(want) | {"rf"}
    unknown = want - set(PLANES)
    if unknown:
        raise ValueError(f"unknown output planes {sorted(unknown)}")
    out = dict(out or {})
    for k in want:
        if k not in out:
            out[k] = torch.empty((ga.nx, ga.nz), dtype=torch.float32, device=rf.device)
    o = _abi.Outputs(_ptr(out.get("rf")), _ptr(out.get("filtered")), _ptr(out.get("env")),
                     _ptr(out.get("log")), _ptr(out.get("imag")))
    need = _abi.lib().pwbf_workspace_bytes(ga.ref, ctypes.byref(o)) if workspace_needed else 0
    if need and workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=rf.device)
    ws_ptr = _ptr(workspace)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    return ga, o, out, ws_ptr, ws_bytes


def beamform(g, rf, mode: str = "das", angle: int = -1, tile: Optional[Tile] = None,
             want: Iterable[str] = ("rf",), out: Optional[Dict] = None, workspace=None,
             stream=None, bandpass: bool = False, log_floor_db: float = -70.0,
             p: Optional[float] = None) -> Dict:
    """pwbf_beamform_ex: one frame through libpwbf with an optional explicit
    launch shape. angle -1 = compound over all angles.
    ``mode``: "das", "dmas" or "pdas" (root order ``p``, else the geometry's) on
    RF; "iqdas" or "bbdmas" on complex64 IQ data from ``iq_demodulate`` (planes
    "rf" = real part, "imag", "env" = magnitude, "log").

    ``rf``: CUDA tensor [n_angles, n_channels, n_samples] of int16/float16/float32.
    ``want``: planes among "rf", "filtered", "env", "log" (rf is always made).
    ``out``: preallocated planes (float32 [nx, nz] CUDA tensors) by name.
    Returns the dict of output planes. Work is enqueued on ``stream`` (default:
    torch's current stream) and not waited for.
    """
    ga, o, out, ws_ptr, ws_bytes = _prepare(g, rf, want, out, workspace, bandpass,
                                            log_floor_db, p)
    t = tile.c() if tile is not None else None
    rc = _abi.lib().pwbf_beamform_ex(ga.ref, _ptr(rf), _rf_code(rf), _MODES[mode], angle,
                                     ctypes.byref(t) if t is not None else None, ctypes.byref(o),
                                     ws_ptr, ws_bytes, _stream_ptr(stream, rf.device))
    _abi.check(rc)
    return out


def _named(symbol, g, rf, angle, want=("rf",), out=None, workspace=None, stream=None,
           bandpass=False, log_floor_db=-70.0, p=None, mode=None, iq=False):
    """One of the named single-frame entry points (pwbf_beamform_das, ...)."""
    ga, o, out, ws_ptr, ws_bytes = _prepare(g, rf, want, out, workspace, bandpass,
                                            log_floor_db, p)
    fn = getattr(_abi.lib(), symbol)
    st = _stream_ptr(stream, rf.device)
    if mode is not None:  # pwbf_compound
        rc = fn(ga.ref, _ptr(rf), _rf_code(rf), _MODES[mode], ctypes.byref(o), ws_ptr, ws_bytes,
                st)
    elif iq:
        rc = fn(ga.ref, _ptr(rf), angle, ctypes.byref(o), ws_ptr, ws_bytes, st)
    else:
        rc = fn(ga.ref, _ptr(rf), _rf_code(rf), angle, ctypes.byref(o), ws_ptr, ws_bytes, st)
    _abi.check(rc)
    return out


def beamform_das(g, rf, angle: int, **kw) -> Dict:
    """pwbf_beamform_das: DAS (Eq. 1) for one steering angle."""
    if angle < 0:
        raise ValueError("angle must be >= 0")
    return _named("pwbf_beamform_das", g, rf, angle, **kw)


def beamform_dmas(g, rf, angle: int, **kw) -> Dict:
    """pwbf_beamform_dmas: RF DMAS for one steering angle."""
    if angle < 0:
        raise ValueError("angle must be >= 0")
    return _named("pwbf_beamform_dmas", g, rf, angle, **kw)


def iq_demodulate(g, rf, out=None, stream=None):
    """pwbf_iq_demodulate: baseband IQ records (complex64 [A, N, Ns / D]) of the
    RF, demodulated at the geometry's f0 and decimated by its iq_decimation D."""
    import torch
    ga = _as_geom(g)
    if not rf.is_cuda or not rf.is_contiguous() or tuple(rf.shape) != ga.shape_rf:
        raise ValueError(f"rf must be a contiguous CUDA tensor {ga.shape_rf}")
    if out is None:
        out = torch.empty(ga.shape_iq, dtype=torch.complex64, device=rf.device)
    if out.dtype != torch.complex64 or not out.is_contiguous() or tuple(out.shape) != ga.shape_iq:
        raise ValueError(f"out must be a contiguous complex64 tensor {ga.shape_iq}")
    _abi.check(_abi.lib().pwbf_iq_demodulate(ga.ref, _ptr(rf), _rf_code(rf), _ptr(out),
                                             _stream_ptr(stream, rf.device)))
    return out


_FK_METHODS = {"stolt": _abi.FK_STOLT, "lu": _abi.FK_LU}


def fk_workspace_bytes(g, want: Iterable[str] = ("rf",), angle: int = -1,
                       method: str = "stolt") -> int:
    """pwbf_fk_workspace_bytes: device workspace of an f-k migration call."""
    ga = _as_geom(g)
    want = set(want)
    o = _abi.Outputs(1, None, 1 if "env" in want else None, 1 if "log" in want else None,
                     1 if "imag" in want else None)
    n = _abi.lib().pwbf_fk_workspace_bytes(ga.ref, _FK_METHODS[method], angle, ctypes.byref(o))
    if n == 0:
        raise _abi.PwbfError(_abi.E_UNSUPPORTED, _abi.lib().pwbf_last_error().decode())
    return int(n)


def fk_migrate(g, rf, angle: int = -1, want: Iterable[str] = ("rf", "imag", "env"),
               out: Optional[Dict] = None, workspace=None, stream=None,
               log_floor_db: float = -70.0, method: str = "stolt") -> Dict:
    """pwbf_fk_migrate: Stolt's ("stolt") or Lu's ("lu") f-k migration of RF
    [A, N, Ns] (int16/float16/float32), one angle or (angle -1) the complex sum
    over all angles. Planes "rf" (real part), "imag", "env" (magnitude), "log"."""
    import torch
    ga = _as_geom(g, False, log_floor_db)
    if not rf.is_cuda or not rf.is_contiguous() or tuple(rf.shape) != ga.shape_rf:
        raise ValueError(f"rf must be a contiguous CUDA tensor {ga.shape_rf}")
    want = set(want) | {"rf"}
    unknown = want - {"rf", "imag", "env", "log"}
    if unknown:
        raise ValueError(f"unknown output planes {sorted(unknown)}")
    out = dict(out or {})
    for k in want:
        if k not in out:
            out[k] = torch.empty((ga.nx, ga.nz), dtype=torch.float32, device=rf.device)
    o = _abi.Outputs(_ptr(out.get("rf")), None, _ptr(out.get("env")), _ptr(out.get("log")),
                     _ptr(out.get("imag")))
    need = _abi.lib().pwbf_fk_workspace_bytes(ga.ref, _FK_METHODS[method], angle,
                                              ctypes.byref(o))
    if need == 0:
        raise _abi.PwbfError(_abi.E_UNSUPPORTED, _abi.lib().pwbf_last_error().decode())
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=rf.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _abi.check(_abi.lib().pwbf_fk_migrate(ga.ref, _ptr(rf), _rf_code(rf), _FK_METHODS[method],
                                          angle, ctypes.byref(o), _ptr(workspace), ws_bytes,
                                          _stream_ptr(stream, rf.device)))
    return out


def _metric_out(torch, n, struct, dev):
    return torch.empty(n * ctypes.sizeof(struct), dtype=torch.uint8, device=dev)


def _read_structs(buf, struct, n):
    raw = bytes(buf.cpu().numpy().tobytes())
    arr = (struct * n).from_buffer_copy(raw)
    return [{k: getattr(a, k) for k, _ in struct._fields_} for a in arr]


def contrast_metrics(g, env, cysts, stream=None):
    """pwbf_contrast_metrics: CR (Eq. 5) and CNR (Eq. 6) of cysts on an envelope
    image (float32 CUDA [nx, nz]). ``cysts``: ((x, z, r) inside, (x, z, r)
    background) in metres. Waits for the stream and returns one dict per cyst."""
    import torch
    ga = _as_geom(g)
    n = len(cysts)
    arr = (_abi.Cyst * max(1, n))(*[_abi.Cyst(_abi.Disc(*c[0]), _abi.Disc(*c[1])) for c in cysts])
    out = _metric_out(torch, max(1, n), _abi.Contrast, env.device)
    _abi.check(_abi.lib().pwbf_contrast_metrics(ga.ref, _ptr(env), arr, n, _ptr(out),
                                                _stream_ptr(stream, env.device)))
    torch.cuda.synchronize(env.device)
    res = _read_structs(out, _abi.Contrast, n)
    for r in res:
        r["mu_in"], r["mu_out"] = float(r["mu_in"]), float(r["mu_out"])
    return res


def resolution_metrics(g, env, targets, stream=None):
    """pwbf_resolution_metrics: peak and lateral / axial FWHM (m) of point
    targets searched inside discs (x, z, r) in metres. Waits for the stream."""
    import torch
    ga = _as_geom(g)
    n = len(targets)
    arr = (_abi.Disc * max(1, n))(*[_abi.Disc(*t) for t in targets])
    out = _metric_out(torch, max(1, n), _abi.Resolution, env.device)
    _abi.check(_abi.lib().pwbf_resolution_metrics(ga.ref, _ptr(env), arr, n, _ptr(out),
                                                  _stream_ptr(stream, env.device)))
    torch.cuda.synchronize(env.device)
    return _read_structs(out, _abi.Resolution, n)


def beamform_iqdas(g, iq, angle: int, **kw) -> Dict:
    """pwbf_beamform_iqdas: DAS of the delay-compensated IQ samples for one angle."""
    if angle < 0:
        raise ValueError("angle must be >= 0")
    return _named("pwbf_beamform_iqdas", g, iq, angle, iq=True, **kw)


def beamform_bbdmas(g, iq, angle: int, **kw) -> Dict:
    """pwbf_beamform_bbdmas: BB-DMAS (Eq. 4) for one angle."""
    if angle < 0:
        raise ValueError("angle must be >= 0")
    return _named("pwbf_beamform_bbdmas", g, iq, angle, iq=True, **kw)


def beamform_pdas(g, rf, angle: int, p: float = 2.0, **kw) -> Dict:
    """pwbf_beamform_pdas: pDAS (Eqs. 2-3) of root order p for one steering angle."""
    if angle < 0:
        raise ValueError("angle must be >= 0")
    return _named("pwbf_beamform_pdas", g, rf, angle, p=p, **kw)


def compound(g, rf, mode: str = "das", **kw) -> Dict:
    """pwbf_compound: coherent sum over all angles of the per-angle images
    (DAS, DMAS, pDAS; complex IQ-DAS, BB-DMAS)."""
    return _named("pwbf_compound", g, rf, -1, mode=mode, **kw)


def compound_noalloc(g, rf, mode: str = "das", want: Iterable[str] = ("rf",),
                     out: Optional[Dict] = None, stream=None, bandpass: bool = False,
                     log_floor_db: float = -70.0, p: Optional[float] = None) -> Dict:
    """pwbf_compound_noalloc: pwbf_compound without a workspace (the library's
    own per-GPU scratch array); planes not given in ``out`` are allocated here,
    by torch, before the call."""
    ga, o, out, _, _ = _prepare(g, rf, want, out, None, bandpass, log_floor_db, p,
                                workspace_needed=False)
    rc = _abi.lib().pwbf_compound_noalloc(ga.ref, _ptr(rf), _rf_code(rf), _MODES[mode],
                                          ctypes.byref(o), _stream_ptr(stream, rf.device))
    _abi.check(rc)
    return out


# ------------------------------------------------------------------- tuning
def tune(g, rf, mode: str = "das", angle: int = -1, waves: int = 0, out_rf=None, stream=None,
         bandpass: bool = False):
    """pwbf_tune: time launch shapes for this frame and remember the fastest.
    Returns (Tile, milliseconds). ``out_rf`` (float32 [nx, nz]) is overwritten."""
    import torch
    ga = _as_geom(g, bandpass)
    if out_rf is None:
        out_rf = torch.empty((ga.nx, ga.nz), dtype=torch.float32, device=rf.device)
    o = _abi.Outputs(_ptr(out_rf), None, None, None)
    best = _abi.Tile()
    ms = ctypes.c_float()
    _abi.check(_abi.lib().pwbf_tune(ga.ref, _ptr(rf), _rf_code(rf), _MODES[mode], angle,
                                    ctypes.byref(o), waves, _stream_ptr(stream, rf.device),
                                    ctypes.byref(best), ctypes.byref(ms)))
    return Tile(best.cpw, best.lz, best.wz, best.wx, best.chunk), float(ms.value)


def tune_save(path: str) -> None:
    _abi.check(_abi.lib().pwbf_tune_save(path.encode()))


def tune_load(path: str) -> None:
    _abi.check(_abi.lib().pwbf_tune_load(path.encode()))


def tune_clear() -> None:
    _abi.check(_abi.lib().pwbf_tune_clear())


# ------------------------------------------------------------------- batches
@dataclass
class FrameSpec:
    """One frame of a batch: geometry object, CUDA RF tensor, mode, angle
    (-1 = compound), output planes (dict name -> float32 [nx, nz] CUDA tensor),
    band-pass flag and optional launch shape."""
    geom: object
    rf: object
    mode: str = "das"
    angle: int = -1
    out: Optional[Dict] = None
    bandpass: bool = False
    tile: Optional[Tile] = None
    p: Optional[float] = None  # pDAS root order (mode "pdas"); None: the geometry's


class Batch:
    """pwbf_batch: uneven frames in one graph-captured launch (up to four branches)."""

    def __init__(self, frames, tune: bool = False, stream=None):
        self._keep = []
        arr = self._frames(frames)
        handle = ctypes.c_void_p()
        dev = frames[0].rf.device
        _abi.check(_abi.lib().pwbf_batch_create(arr, len(frames), _abi.BATCH_TUNE if tune else 0,
                                                _stream_ptr(stream, dev), ctypes.byref(handle)))
        self.handle = handle
        self.device = dev
        self.frames = list(frames)

    def _frames(self, frames):
        arr = (_abi.Frame * len(frames))()
        keep = []
        for i, f in enumerate(frames):
            ga = _as_geom(f.geom, f.bandpass)
            if f.p is not None:
                ga.s.pdas_p = float(f.p)
            keep.append(ga)
            if not f.rf.is_cuda or not f.rf.is_contiguous() or tuple(f.rf.shape) != ga.shape_rf:
                raise ValueError(f"frame {i}: rf must be a contiguous CUDA tensor {ga.shape_rf}")
            out = f.out or {}
            if "rf" not in out:
                raise ValueError(f"frame {i}: out['rf'] is required")
            t = f.tile.c() if f.tile is not None else _abi.Tile()
            arr[i] = _abi.Frame(ctypes.pointer(ga.s), _ptr(f.rf), _rf_code(f.rf), _MODES[f.mode],
                                f.angle, 0, _abi.Outputs(_ptr(out.get("rf")),
                                                         _ptr(out.get("filtered")),
                                                         _ptr(out.get("env")),
                                                         _ptr(out.get("log"))), t)
        self._keep = keep
        return arr

    def update(self, frames, stream=None) -> None:
        arr = self._frames(frames)
        _abi.check(_abi.lib().pwbf_batch_update(self.handle, arr, len(frames),
                                                _stream_ptr(stream, self.device)))
        self.frames = list(frames)

    def launch(self, stream=None) -> None:
        _abi.check(_abi.lib().pwbf_batch_launch(self.handle, _stream_ptr(stream, self.device)))

    def describe(self) -> Dict:
        info = _abi.BatchInfo()
        _abi.check(_abi.lib().pwbf_batch_describe(self.handle, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in _abi.BatchInfo._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            _abi.check(_abi.lib().pwbf_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class ProbeSpec:
    """One probe of a serving loop (pwbf_probe): geometry, beamformer, planes."""
    geom: object
    mode: str = "das"
    angle: int = -1
    want: Iterable[str] = ("rf", "env", "log")
    slots: int = 4
    bandpass: bool = False
    p: Optional[float] = None  # pDAS root order (mode "pdas")
    # a quality check of every served frame: ((x, z, r) inside, (x, z, r)
    # background) in m; passes when the frame maximum is > 0 and the CR of that
    # region (Eq. (5)) is at most quality_max_cr_db
    quality_region: Optional[Tuple] = None
    quality_max_cr_db: float = -10.0


@dataclass
class Completed:
    """A finished request (pwbf_result); the planes stay valid until release()."""
    id: int
    probe: int
    slot: int
    t_arrival: float
    t_admit: float
    t_launch: float
    t_done: float
    rf: Optional[int]
    env: Optional[int]
    logimg: Optional[int]
    status: int = 0          # 0, or E_TIMEOUT: dropped at its deadline (no planes)
    quality_ok: bool = False  # the probe's quality check (when it has one)
    frame_max: float = 0.0
    cr_db: float = 0.0
    cnr: float = 0.0


class Server:
    """pwbf_server: continuous batching of int16 frames over resident HBM rings.

    ``submit`` takes a pinned host int16 tensor [angles, channels, samples] and
    keeps a reference to it until the request is released. ``planes(result)``
    views the slot's device planes as torch tensors (no copy)."""

    def __init__(self, probes, hbm_budget_bytes: int = 0, max_queue: int = 0):
        self._geoms = [_as_geom(p.geom, p.bandpass) for p in probes]
        for p, ga in zip(probes, self._geoms):
            if p.p is not None:
                ga.s.pdas_p = float(p.p)
        arr = (_abi.Probe * len(probes))()
        for i, (p, ga) in enumerate(zip(probes, self._geoms)):
            want = set(p.want)
            q = _abi.Cyst()
            if p.quality_region is not None:
                q = _abi.Cyst(_abi.Disc(*p.quality_region[0]), _abi.Disc(*p.quality_region[1]))
            arr[i] = _abi.Probe(ctypes.pointer(ga.s), _MODES[p.mode], p.angle,
                                1 if "env" in want else 0, 1 if "log" in want else 0,
                                p.slots, 0 if p.quality_region is None else 1, q,
                                float(p.quality_max_cr_db))
        handle = ctypes.c_void_p()
        _abi.check(_abi.lib().pwbf_server_create(arr, len(probes), hbm_budget_bytes, max_queue,
                                                 ctypes.byref(handle)))
        self.handle = handle
        self.probes = list(probes)
        self._pending = {}

    def submit(self, probe: int, host_rf, t_arrival: float = -1.0,
               deadline: float = -1.0) -> int:
        """Queue a frame; ``deadline`` >= 0 is the server time (``now()``) by
        which it must be admitted, else it comes back expired (status E_TIMEOUT)."""
        import torch
        ga = self._geoms[probe]
        if (host_rf.dtype != torch.int16 or host_rf.is_cuda or not host_rf.is_contiguous()
                or tuple(host_rf.shape) != ga.shape_rf):
            raise ValueError(f"host_rf must be a contiguous host int16 tensor {ga.shape_rf}")
        rid = ctypes.c_uint64()
        _abi.check(_abi.lib().pwbf_server_submit_ex(self.handle, probe, host_rf.data_ptr(),
                                                    t_arrival, deadline, ctypes.byref(rid)))
        self._pending[rid.value] = host_rf
        return rid.value

    def poll(self, max_results: int = 64, wait_ms: int = 0):
        res = (_abi.Result * max_results)()
        n = ctypes.c_int32()
        _abi.check(_abi.lib().pwbf_server_poll(self.handle, res, max_results, ctypes.byref(n),
                                               wait_ms))
        return [Completed(r.id, r.probe, r.slot, r.t_arrival, r.t_admit, r.t_launch, r.t_done,
                          r.rf, r.env, r.logimg, r.status, bool(r.quality_ok), r.frame_max,
                          r.cr_db, r.cnr) for r in res[:n.value]]

    def planes(self, result: Completed) -> Dict:
        """Copies of a completed request's device planes as [nx, nz] float32 tensors."""
        import torch
        ga = self._geoms[result.probe]
        out = {}
        for name, ptr in (("rf", result.rf), ("env", result.env), ("log", result.logimg)):
            if ptr:
                t = torch.empty((ga.nx, ga.nz), dtype=torch.float32, device="cuda")
                rc = _hip().hipMemcpy(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(ptr),
                                      ctypes.c_size_t(t.numel() * 4), 3)
                if rc != 0:
                    raise _abi.PwbfError(_abi.E_DEVICE, f"hipMemcpy of the {name} plane: {rc}")
                out[name] = t
        return out

    def release(self, rid: int) -> None:
        _abi.check(_abi.lib().pwbf_server_release(self.handle, rid))
        self._pending.pop(rid, None)

    def stats(self) -> Dict:
        st = _abi.ServerStats()
        _abi.check(_abi.lib().pwbf_server_stats_get(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _abi.ServerStats._fields_}

    def now(self) -> float:
        return float(_abi.lib().pwbf_server_now(self.handle))

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            _abi.check(_abi.lib().pwbf_server_destroy(self.handle))
            self.handle = None
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _hip():
    """The HIP runtime torch loaded (only for copying library-owned planes)."""
    import torch  # noqa: F401
    return ctypes.CDLL("libamdhip64.so.7")
