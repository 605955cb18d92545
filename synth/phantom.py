"""Seeded scatterer phantoms and the plane-wave channel RF they produce.

Forward model (2-D, no attenuation, no element directivity): a plane wave
steered by angle theta leaves the array at t = 0 from the first-firing element,
reaches a scatterer at (x, z) after (x sin theta + z cos theta - d) / c with
d = min_e(x_e sin theta), and the echo reaches element e after a further
sqrt((x - x_e)^2 + z^2) / c. Each scatterer adds ``amp * p(t - t_arrival)`` to
the channel, where ``p`` is a Gaussian-windowed cosine whose envelope spans two
cycles at half maximum, truncated at 3.5 sigma.

Random draws use ``numpy.random.default_rng(seed)`` in a fixed order: point
targets, cysts, speckle positions, speckle amplitudes, noise.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

from .configs import Geometry

PULSE_TRUNC_SIGMAS = 3.5


@dataclasses.dataclass
class Phantom:
    x: np.ndarray  # scatterer lateral positions, m
    z: np.ndarray  # scatterer depths, m
    amp: np.ndarray  # scatterer amplitudes
    points: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 2)))
    cysts: List[Tuple[float, float, float]] = dataclasses.field(default_factory=list)


def pulse_sigma(f0: float) -> float:
    """Gaussian sigma of an envelope whose full width at half maximum is two cycles."""
    return (2.0 / f0) / (2.0 * math.sqrt(2.0 * math.log(2.0)))


def _snap(v: np.ndarray, v0: float, dv: float, n: int) -> np.ndarray:
    idx = np.clip(np.rint((v - v0) / dv), 0, n - 1)
    return v0 + idx * dv


def point_phantom(points_xz, amp: float = 1.0) -> Phantom:
    pts = np.atleast_2d(np.asarray(points_xz, dtype=np.float64))
    return Phantom(x=pts[:, 0].copy(), z=pts[:, 1].copy(), amp=np.full(len(pts), amp),
                   points=pts.copy())


def _speckle(rng, n, x_lo, x_hi, z_lo, z_hi):
    xs = rng.uniform(x_lo, x_hi, n)
    zs = rng.uniform(z_lo, z_hi, n)
    return xs, zs


def phantom_c1(g: Geometry, rng: np.random.Generator, n_points: int = 5,
               n_speckle: int = 2000, point_amp: float = 10.0) -> Phantom:
    """Points at z = 10, 15, 20, 25, 30 mm with x ~ U[-5, 5] mm, snapped to pixel
    centres of ``g``; uniform Gaussian-amplitude speckle over the field of view."""
    zp = np.array([10e-3, 15e-3, 20e-3, 25e-3, 30e-3])[:n_points]
    xp = rng.uniform(-5e-3, 5e-3, n_points)
    xp = _snap(xp, g.x0, g.dx, g.nx)
    zp = _snap(zp, g.z0, g.dz, g.nz)
    xs, zs = _speckle(rng, n_speckle, g.x_min, g.x_max, g.z_min, g.z_max)
    amps = rng.standard_normal(n_speckle)
    pts = np.stack([xp, zp], 1)
    return Phantom(x=np.concatenate([xp, xs]), z=np.concatenate([zp, zs]),
                   amp=np.concatenate([np.full(n_points, point_amp), amps]), points=pts)


def phantom_scaled(g: Geometry, rng: np.random.Generator, point_amp: float = 10.0) -> Phantom:
    """The single-frame recipe scaled to ``g``'s field of view: five points spread
    over depth, speckle at the same areal density (2000 per 19 mm x 40 mm)."""
    w = g.x_max - g.x_min
    h = g.z_max - g.z_min
    zp = g.z_min + h * np.array([0.2, 0.35, 0.5, 0.65, 0.8])
    xp = rng.uniform(-0.25 * w, 0.25 * w, 5) + 0.5 * (g.x_min + g.x_max)
    xp = _snap(xp, g.x0, g.dx, g.nx)
    zp = _snap(zp, g.z0, g.dz, g.nz)
    n_speckle = int(round(2000 * (w * h) / (19e-3 * 40e-3)))
    xs, zs = _speckle(rng, n_speckle, g.x_min, g.x_max, g.z_min, g.z_max)
    amps = rng.standard_normal(n_speckle)
    return Phantom(x=np.concatenate([xp, xs]), z=np.concatenate([zp, zs]),
                   amp=np.concatenate([np.full(5, point_amp), amps]),
                   points=np.stack([xp, zp], 1))


def phantom_c3(g: Geometry, rng: np.random.Generator, n_points: int = 20, n_cysts: int = 3,
               n_speckle: int = 20000, point_amp: float = 10.0) -> Phantom:
    """20 points and 3 anechoic cysts (radius U[2, 4] mm, non-overlapping, no point
    within 3 mm of a cyst), speckle uniform over the field of view and removed
    inside the cysts."""
    # points first (draw order), placed after the cysts are known by rejection
    pts_raw = np.stack([rng.uniform(-17e-3, 17e-3, 4 * n_points),
                        rng.uniform(7e-3, 43e-3, 4 * n_points)], 1)
    cysts: List[Tuple[float, float, float]] = []
    while len(cysts) < n_cysts:
        r = rng.uniform(2e-3, 4e-3)
        cx = rng.uniform(-14e-3, 14e-3)
        cz = rng.uniform(12e-3, 40e-3)
        if all(math.hypot(cx - a, cz - b) > r + rb + 1e-3 for a, b, rb in cysts):
            cysts.append((cx, cz, r))

    def inside(x, z, margin=0.0):
        m = np.zeros(np.shape(x), dtype=bool)
        for cx, cz, r in cysts:
            m |= (x - cx) ** 2 + (z - cz) ** 2 < (r + margin) ** 2
        return m

    # points stay 3 mm (several lateral widths of the point response, side
    # lobes included) outside every cyst, so no cyst reads a point's energy
    keep = ~inside(pts_raw[:, 0], pts_raw[:, 1], 3e-3)
    pts = pts_raw[keep][:n_points]
    assert len(pts) == n_points
    xp = _snap(pts[:, 0], g.x0, g.dx, g.nx)
    zp = _snap(pts[:, 1], g.z0, g.dz, g.nz)
    xs, zs = _speckle(rng, n_speckle, g.x_min, g.x_max, g.z_min, g.z_max)
    amps = rng.standard_normal(n_speckle)
    out = ~inside(xs, zs)
    xs, zs, amps = xs[out], zs[out], amps[out]
    return Phantom(x=np.concatenate([xp, xs]), z=np.concatenate([zp, zs]),
                   amp=np.concatenate([np.full(n_points, point_amp), amps]),
                   points=np.stack([xp, zp], 1), cysts=cysts)


def cyst_regions(g: Geometry, ph: Phantom, inside: float = 0.8, offset: float = 2.2):
    """The contrast regions of each cyst (Section II-D): the inside disc of
    radius inside * r at the cyst's centre, and a background disc of the same
    radius offset * r away, on whichever of the four sides (left, right, above,
    below) that stays on the grid and clear of every cyst lies farthest from the
    point targets. Returns [((x, z, r_in), (x, z, r_in)), ...] in metres."""
    out = []
    pts = np.asarray(ph.points, dtype=np.float64).reshape(-1, 2)
    for cx, cz, r in ph.cysts:
        best = None
        for ox, oz in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            bx, bz = cx + ox * offset * r, cz + oz * offset * r
            if not (g.x_min + r < bx < g.x_max - r and g.z_min + r < bz < g.z_max - r):
                continue
            if any(math.hypot(bx - ax, bz - az) < ar + inside * r for ax, az, ar in ph.cysts):
                continue
            clear = (float(np.hypot(pts[:, 0] - bx, pts[:, 1] - bz).min()) if len(pts)
                     else math.inf) - inside * r
            if best is None or clear > best[0]:
                best = (clear, bx, bz)
        out.append(((cx, cz, inside * r), (best[1], best[2], inside * r)))
    return out


def echo_times(g: Geometry, angle_index: int, xs: np.ndarray, zs: np.ndarray,
               elem: Optional[np.ndarray] = None) -> np.ndarray:
    """Arrival time (s, relative to the time of sample 0) of each scatterer's echo
    at each element: array [n_elem, n_scat]."""
    th = g.angles_rad[angle_index]
    ex = g.elem_x if elem is None else g.elem_x[elem]
    first = np.min(g.elem_x * math.sin(th))
    t_in = (xs * math.sin(th) + zs * math.cos(th) - first) / g.c
    t_out = np.hypot(xs[None, :] - ex[:, None], zs[None, :]) / g.c
    return t_in[None, :] + t_out - g.t0_s[angle_index]


def simulate_clean(g: Geometry, ph: Phantom) -> np.ndarray:
    """Noise-free channel RF, float64 array [n_angles][n_channels][n_samples]."""
    from . import _native
    sigma = pulse_sigma(g.f0)
    rf = np.empty((g.n_angles, g.n_channels, g.n_samples))
    for a in range(g.n_angles):
        t = echo_times(g, a, ph.x, ph.z)
        rf[a] = _native.accumulate(t, ph.amp, g.n_samples, g.fs, g.f0, sigma,
                                   PULSE_TRUNC_SIGMAS * sigma)
    return rf


def simulate_clean_numpy(g: Geometry, ph: Phantom, chunk: int = 16) -> np.ndarray:
    """The same RF as :func:`simulate_clean`, evaluated tap by tap in NumPy (slow;
    kept to cross-check the C core)."""
    A, N, Ns = g.n_angles, g.n_channels, g.n_samples
    rf = np.zeros((A, N, Ns))
    sigma = pulse_sigma(g.f0)
    half = int(math.ceil(PULSE_TRUNC_SIGMAS * sigma * g.fs))
    taps = np.arange(-half, half + 1)
    # cos(2 pi f0 (k/fs + d)) = cos(w k) cos(w' d) - sin(w k) sin(w' d)
    wk = 2.0 * math.pi * g.f0 * taps / g.fs
    cos_k, sin_k = np.cos(wk), np.sin(wk)
    for a in range(A):
        for e0 in range(0, N, chunk):
            e1 = min(N, e0 + chunk)
            t = echo_times(g, a, ph.x, ph.z, np.arange(e0, e1))  # [E, S]
            nc = np.rint(t * g.fs)
            d = nc / g.fs - t  # in [-0.5/fs, 0.5/fs]
            dt = d[..., None] + taps / g.fs  # [E, S, K]
            env = np.exp(-0.5 * (dt / sigma) ** 2)
            env[np.abs(dt) > PULSE_TRUNC_SIGMAS * sigma] = 0.0
            ph_d = 2.0 * math.pi * g.f0 * d
            osc = np.cos(ph_d)[..., None] * cos_k - np.sin(ph_d)[..., None] * sin_k
            val = env * osc * ph.amp[None, :, None]
            n = nc[..., None].astype(np.int64) + taps
            ok = (n >= 0) & (n < Ns)
            flat = (np.arange(e1 - e0)[:, None, None] * Ns + n)[ok]
            acc = np.bincount(flat, weights=val[ok], minlength=(e1 - e0) * Ns)
            rf[a, e0:e1] += acc.reshape(e1 - e0, Ns)
    return rf


def simulate_rf(g: Geometry, ph: Phantom, rng: Optional[np.random.Generator] = None,
                snr_db: Optional[float] = 30.0, quantize: bool = True,
                max_abs: float = 511.0) -> dict:
    """Channel RF for ``ph`` under ``g``.

    Returns a dict with ``master`` (float64, the values the oracle sees) and the
    storage forms: ``i16`` (10-bit quantised, when ``quantize``) or ``f32`` and
    ``f16`` (scaled so max |RF| = ``max_abs``). White Gaussian noise at ``snr_db``
    relative to the global RMS of the clean RF is added before scaling.
    """
    clean = simulate_clean(g, ph)
    rf = clean
    if snr_db is not None:
        assert rng is not None
        rms = math.sqrt(float(np.mean(clean ** 2)))
        rf = clean + rng.standard_normal(clean.shape) * rms * 10.0 ** (-snr_db / 20.0)
    peak = float(np.max(np.abs(rf)))
    scale = max_abs / peak if peak > 0 else 1.0
    out = {"scale": scale}
    if quantize:
        q = np.clip(np.rint(rf * scale), -512, 511).astype(np.int16)
        out["i16"] = q
        out["master"] = q.astype(np.float64)
    else:
        m = rf * scale
        out["master"] = m
        out["f32"] = m.astype(np.float32)
        out["f16"] = m.astype(np.float16)
    return out


def make_frame(spec_geom: Geometry, seed: int, kind: str = "c1", quantize: bool = True,
               snr_db: Optional[float] = 30.0) -> dict:
    """Phantom + RF for one frame of a named recipe ("c1", "c3" or "scaled")."""
    rng = np.random.default_rng(seed)
    if kind == "c1":
        ph = phantom_c1(spec_geom, rng)
    elif kind == "c3":
        ph = phantom_c3(spec_geom, rng)
    elif kind == "scaled":
        ph = phantom_scaled(spec_geom, rng)
    else:
        raise ValueError(kind)
    out = simulate_rf(spec_geom, ph, rng, snr_db=snr_db, quantize=quantize)
    out["phantom"] = ph
    out["geom"] = spec_geom
    return out
