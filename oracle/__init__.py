"""FP64 reference beamformer (the oracle).

TEST INFRASTRUCTURE ONLY. This package is what the GPU path is checked against:
only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
it. It shares no code with the GPU library and never imports it.

The per-pixel beamformers (DAS, compound, RF DMAS in two forms, pDAS, IQ-DAS and
BB-DMAS on baseband data) are plain C in
``pwbf_oracle.c``, FP64, single-threaded (or, with ``parallel=True``, the same
source built with OpenMP over the pixel loop, bitwise the same values); the column post-processing along depth
(band-pass, Hilbert envelope, log compression) is NumPy FP64 with ``numpy.fft``
as the transform. Geometry objects are duck-typed: anything with the attributes
of ``synth.Geometry`` (elem_x, angles_rad, t0_s, c, fs, nx, nz, x0, dx, z0, dz,
f_number, apod_code, n_samples, f0).

Image metrics (FWHM, Eq. (5) CR, Eq. (6) CNR) are in ``oracle/metrics.py``.

Paper passages followed: Eq. (1) and the delay text after it (DAS); Eq. (2) and
Eq. (4) for the signed-root compression and the squared-sum form of DMAS;
Eqs. (2)-(3) for pDAS (p-th root before the sum, signed p-th power after);
Eq. (4) for BB-DMAS on IQ data, with IQ-DAS as Eq. (1) on the same data; the
absolute value of the analytic signal for the image; the -70 dB display range
(Fig. 3 caption). Every function is pinned by CPU tests against closed forms,
invariants and an independent brute-force evaluation; none is "parity unpinned".
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pwbf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_libs = {}


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc -O2, no fast-math): the single-threaded library
    and, from the same source with -fopenmp, the one that shares the pixel loop
    among threads (bitwise the same values)."""
    for lib, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            tmp = lib + f".tmp{os.getpid()}"
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC",
                                   "-shared", "-fno-fast-math", *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, lib)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("n_angles", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("n_samples", ctypes.c_int32), ("elem_x", ctypes.c_void_p),
                ("angle", ctypes.c_void_p), ("t0", ctypes.c_void_p),
                ("c", ctypes.c_double), ("fs", ctypes.c_double),
                ("nx", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("x0", ctypes.c_double), ("dx", ctypes.c_double),
                ("z0", ctypes.c_double), ("dz", ctypes.c_double),
                ("f_number", ctypes.c_double), ("apod", ctypes.c_int32)]


def _load(parallel: bool = False):
    """The oracle library: single-threaded, or (parallel) the OpenMP build."""
    key = bool(parallel)
    if key not in _libs:
        path = _LIB_OMP if key else _LIB
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER(_Geom)
        lib.ora_tof_samples.restype = ctypes.c_double
        lib.ora_tof_samples.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double]
        lib.ora_apod_weight.restype = ctypes.c_double
        lib.ora_apod_weight.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        lib.ora_interp.restype = ctypes.c_double
        lib.ora_interp.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double]
        lib.ora_das.restype = ctypes.c_int
        lib.ora_das.argtypes = [P, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_int64, ctypes.c_void_p]
        lib.ora_dmas.restype = ctypes.c_int
        lib.ora_dmas.argtypes = [P, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.ora_iq.restype = ctypes.c_int
        lib.ora_iq.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_void_p]
        lib.ora_pdas.restype = ctypes.c_int
        lib.ora_pdas.argtypes = [P, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.ora_threads.restype = ctypes.c_int
        lib.ora_threads.argtypes = []
        _libs[key] = lib
    return _libs[key]


def threads(parallel: bool = True) -> int:
    """Threads the (parallel or single-threaded) build shares a call among."""
    return int(_load(parallel).ora_threads())


class _Bound:
    """A ctypes geometry plus the arrays it points into (kept alive together)."""

    def __init__(self, g, decimation: int = 1):
        # records decimated by D are records at the rate fs / D, n_samples / D long
        self.elem_x = np.ascontiguousarray(g.elem_x, dtype=np.float64)
        self.angle = np.ascontiguousarray(g.angles_rad, dtype=np.float64)
        self.t0 = np.ascontiguousarray(g.t0_s, dtype=np.float64)
        self.s = _Geom(len(self.angle), len(self.elem_x), int(g.n_samples) // decimation,
                       self.elem_x.ctypes.data, self.angle.ctypes.data, self.t0.ctypes.data,
                       float(g.c), float(g.fs) / decimation, int(g.nx), int(g.nz), float(g.x0),
                       float(g.dx), float(g.z0), float(g.dz), float(g.f_number),
                       int(g.apod_code))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _rf64(g, rf) -> np.ndarray:
    rf = np.ascontiguousarray(rf, dtype=np.float64)
    if rf.ndim == 2:
        rf = rf[None]
    assert rf.shape == (len(g.angles_rad), len(g.elem_x), g.n_samples), rf.shape
    return rf


def _pix(g, pix) -> Optional[np.ndarray]:
    if pix is None:
        return None
    return np.ascontiguousarray(pix, dtype=np.int64)


def tof_samples(g, a: int, e: int, x: float, z: float) -> float:
    """Time of flight (samples) for angle a, element e, point (x, z)."""
    b = _Bound(g)
    return _load().ora_tof_samples(b.ref, a, e, x, z)


def apod_weight(g, e: int, x: float, z: float) -> float:
    b = _Bound(g)
    return _load().ora_apod_weight(b.ref, e, x, z)


def interp(u: np.ndarray, s: float) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    return _load().ora_interp(u.ctypes.data, len(u), s)


def das(g, rf, angle: int = -1, pix=None, parallel: bool = False) -> np.ndarray:
    """DAS (Eq. 1). angle -1 = coherent compound over all angles. Returns [nx, nz]
    when ``pix`` is None, else the values at the flat pixel indices ``pix``.
    ``parallel`` runs the OpenMP build of the same source (same values)."""
    b = _Bound(g)
    rf = _rf64(g, rf)
    p = _pix(g, pix)
    n = g.nx * g.nz if p is None else len(p)
    out = np.empty(n, dtype=np.float64)
    rc = _load(parallel).ora_das(b.ref, rf.ctypes.data, angle, None if p is None else p.ctypes.data, n,
                         out.ctypes.data)
    if rc != 0:
        raise ValueError("ora_das rejected its arguments")
    return out.reshape(g.nx, g.nz) if p is None else out


def dmas(g, rf, angle: int = -1, form: str = "identity", pix=None,
         parallel: bool = False) -> np.ndarray:
    """RF DMAS with signed square-root compression; form "pairs" or "identity"."""
    b = _Bound(g)
    rf = _rf64(g, rf)
    p = _pix(g, pix)
    n = g.nx * g.nz if p is None else len(p)
    out = np.empty(n, dtype=np.float64)
    f = {"pairs": 0, "identity": 1}[form]
    rc = _load(parallel).ora_dmas(b.ref, rf.ctypes.data, angle, f, None if p is None else p.ctypes.data,
                          n, out.ctypes.data)
    if rc != 0:
        raise ValueError("ora_dmas rejected its arguments")
    return out.reshape(g.nx, g.nz) if p is None else out


def pdas(g, rf, angle: int = -1, p: float = 2.0, pix=None,
         parallel: bool = False) -> np.ndarray:
    """pDAS (Eqs. 2-3): sum of w sign(v)|v|^(1/p), then its signed p-th power;
    angle -1 sums the per-angle pDAS values."""
    b = _Bound(g)
    rf = _rf64(g, rf)
    q = _pix(g, pix)
    n = g.nx * g.nz if q is None else len(q)
    out = np.empty(n, dtype=np.float64)
    rc = _load(parallel).ora_pdas(b.ref, rf.ctypes.data, angle, float(p),
                          None if q is None else q.ctypes.data, n, out.ctypes.data)
    if rc != 0:
        raise ValueError("ora_pdas rejected its arguments")
    return out.reshape(g.nx, g.nz) if q is None else out


def band_keep(ns: int, fs: float, fd: float, decimation: int) -> np.ndarray:
    """Boolean [ns]: the DFT bins the decimating demodulation keeps, the positive
    bins (0..ns/2) whose frequency k fs / ns lies within fs / (2 D) of fd; every
    bin when D = 1."""
    if decimation <= 1:
        return np.ones(ns, dtype=bool)
    k = np.arange(ns)
    return (k <= ns // 2) & (np.abs(k * fs / ns - fd) < fs / (2.0 * decimation))


def iq_demodulate(g, rf, fd: Optional[float] = None, decimation: int = 1) -> np.ndarray:
    """Baseband (IQ) channel records (Section II-B's IQ signals; the paper does
    not give the demodulation, its filter or the decimation, so this is a
    reading): the analytic signal of each record (one-sided spectrum along
    samples: 1 at DC and Nyquist, 2 on positive bins, 0 on negative ones) times
    exp(-2 pi i fd n / fs), fd = f0 by default. Decimation by D keeps, before the
    inverse transform, only the bins of ``band_keep`` (an ideal low-pass of the
    baseband signal to the band of the rate fs / D), then every D-th sample.
    Returns complex128 [n_angles][n_channels][n_samples / D]; n_samples even."""
    rf = _rf64(g, rf)
    ns = rf.shape[-1]
    assert ns % 2 == 0 and ns % decimation == 0
    fd = float(g.f0 if fd is None else fd)
    h = np.zeros(ns)
    h[0] = 1.0
    h[1:ns // 2] = 2.0
    h[ns // 2] = 1.0
    h = h * band_keep(ns, float(g.fs), fd, decimation)
    analytic = np.fft.ifft(np.fft.fft(rf, axis=-1) * h, axis=-1)
    n = np.arange(ns)
    return (analytic * np.exp(-2j * np.pi * fd * n / g.fs))[..., ::decimation]


def iq_beamform(g, iq, form: str = "iqdas", angle: int = -1, fd: Optional[float] = None,
                pix=None, parallel: bool = False, decimation: int = 1) -> np.ndarray:
    """IQ-DAS ("iqdas") or BB-DMAS ("bbdmas", Eq. 4) from baseband records ``iq``
    demodulated at fd (f0 by default); complex, [nx, nz] or at ``pix``. angle -1
    sums the complex per-angle values. Records decimated by D are read at their
    own rate: the delay of s samples at fs is s / D samples of the record, and
    the phase rotation uses the same time."""
    b = _Bound(g, decimation)
    iq = np.asarray(iq)
    if iq.ndim == 2:
        iq = iq[None]
    assert iq.shape == (len(g.angles_rad), len(g.elem_x), g.n_samples // decimation), iq.shape
    re = np.ascontiguousarray(iq.real, dtype=np.float64)
    im = np.ascontiguousarray(iq.imag, dtype=np.float64)
    q = _pix(g, pix)
    n = g.nx * g.nz if q is None else len(q)
    out_re = np.empty(n)
    out_im = np.empty(n)
    fd = float(g.f0 if fd is None else fd)
    rc = _load(parallel).ora_iq(b.ref, re.ctypes.data, im.ctypes.data, fd,
                        {"iqdas": 0, "bbdmas": 1}[form], angle,
                        None if q is None else q.ctypes.data, n, out_re.ctypes.data,
                        out_im.ctypes.data)
    if rc != 0:
        raise ValueError("ora_iq rejected its arguments")
    y = out_re + 1j * out_im
    return y.reshape(g.nx, g.nz) if q is None else y


def compound(g, rf, mode: str = "das", pix=None, p: float = 2.0) -> np.ndarray:
    """Coherent compounding: the unweighted sum over angles of the per-angle image."""
    if mode == "das":
        return das(g, rf, -1, pix)
    if mode == "pdas":
        return pdas(g, rf, -1, p, pix)
    return dmas(g, rf, -1, "identity", pix)


# ---------------------------------------------------------------- post-processing
def band_bins(nz: int, dz: float, c: float, f0: float) -> np.ndarray:
    """Boolean mask over FFT bins of a depth column whose round-trip frequency
    f_k = |k'| c / (2 nz dz) lies in [f0, 3 f0] (k' the signed bin index)."""
    k = np.fft.fftfreq(nz) * nz  # signed integer bins
    f = np.abs(k) * c / (2.0 * nz * dz)
    return (f >= f0) & (f <= 3.0 * f0)


def bandpass_z(img: np.ndarray, dz: float, c: float, f0: float) -> np.ndarray:
    """Zero-phase brick-wall band-pass along depth (axis 1) keeping [f0, 3 f0]."""
    img = np.asarray(img, dtype=np.float64)
    X = np.fft.fft(img, axis=-1)
    H = band_bins(img.shape[-1], dz, c, f0)
    return np.real(np.fft.ifft(X * H, axis=-1))


def hilbert_weights(nz: int) -> np.ndarray:
    """One-sided spectrum weights: 1 at DC and Nyquist, 2 for positive bins, 0 else."""
    h = np.zeros(nz)
    h[0] = 1.0
    if nz % 2 == 0:
        h[nz // 2] = 1.0
        h[1:nz // 2] = 2.0
    else:
        h[1:(nz + 1) // 2] = 2.0
    return h


def envelope_z(img: np.ndarray) -> np.ndarray:
    """Magnitude of the analytic signal along depth (axis 1)."""
    img = np.asarray(img, dtype=np.float64)
    X = np.fft.fft(img, axis=-1)
    return np.abs(np.fft.ifft(X * hilbert_weights(img.shape[-1]), axis=-1))


def log_compress(env: np.ndarray, floor_db: float = -70.0) -> np.ndarray:
    """20 log10(env / max env), clipped below at ``floor_db`` (floor everywhere if
    the envelope is identically zero)."""
    env = np.asarray(env, dtype=np.float64)
    m = float(np.max(env)) if env.size else 0.0
    if m <= 0.0:
        return np.full(env.shape, floor_db)
    with np.errstate(divide="ignore"):
        out = 20.0 * np.log10(env / m)
    return np.maximum(out, floor_db)


def beamform(g, rf, mode: str = "das", angle: int = -1, bandpass: bool = False,
             floor_db: float = -70.0, p: float = 2.0, parallel: bool = False) -> dict:
    """The whole path for one frame: raw image, optional band-pass, envelope, log."""
    if mode == "das":
        raw = das(g, rf, angle, parallel=parallel)
    elif mode == "pdas":
        raw = pdas(g, rf, angle, p, parallel=parallel)
    else:
        raw = dmas(g, rf, angle, "identity", parallel=parallel)
    out = {"rf": raw}
    src = raw
    if bandpass:
        src = bandpass_z(raw, g.dz, g.c, g.f0)
        out["filtered"] = src
    out["env"] = envelope_z(src)
    out["log"] = log_compress(out["env"], floor_db)
    return out
