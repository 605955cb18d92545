"""FP64 reference image metrics (the oracle's part for image quality).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: it checks the GPU
metrics kernels and shares no code with them.

Paper passages (Section II-D, "Evaluation Metrics"):
 - FWHM of point targets, measured at -6 dB on the lateral and the axial
   profile: here the full width at half the peak amplitude of the envelope
   (20 log10 0.5 = -6.02 dB), each crossing located by linear interpolation
   between the last pixel at or above half the peak and the first below it;
   NaN when a profile does not fall below half within the image.
 - Eq. (5): CR = 20 log10(mu_in / mu_out).
 - Eq. (6): CNR = (mu_in - mu_out) / sqrt(s), where the printed denominator
   sqrt(sigma_in^2 + sigma_out^2 / 2) is read as sqrt((sigma_in^2 + sigma_out^2) / 2);
   mu and sigma are the mean and the (population) standard deviation of the
   envelope over the pixels inside the cyst and inside a background disc.

A pixel belongs to a disc when the distance from its centre to the disc's
centre is at most the radius, decided here in float64 from the grid
convention (pixel (ix, iz) centred at (x0 + ix dx, z0 + iz dz)).
``disc_distance`` also gives the distance in radii, so a caller can tell
which pixels lie so close to the boundary that a float32 evaluation may
decide them either way.
"""

from __future__ import annotations

import math

import numpy as np


def pixel_centres(g):
    """(X [nx, 1], Z [1, nz]) pixel-centre coordinates of grid g, float64."""
    X = (g.x0 + np.arange(g.nx, dtype=np.float64) * g.dx)[:, None]
    Z = (g.z0 + np.arange(g.nz, dtype=np.float64) * g.dz)[None, :]
    return X, Z


def disc_distance(g, x: float, z: float, r: float) -> np.ndarray:
    """[nx, nz]: distance of every pixel centre from (x, z), in units of r."""
    X, Z = pixel_centres(g)
    return np.hypot(X - x, Z - z) / r


def disc_mask(g, x: float, z: float, r: float) -> np.ndarray:
    """Boolean [nx, nz]: the pixels of grid g whose centres lie in the disc."""
    return disc_distance(g, x, z, r) <= 1.0


def region_stats(env: np.ndarray, mask: np.ndarray):
    """(count, mean, population standard deviation) of env over the mask, float64."""
    vals = np.asarray(env, dtype=np.float64)[mask]
    n = vals.size
    if n == 0:
        return 0, float("nan"), float("nan")
    mu = vals.sum() / n
    return n, float(mu), float(math.sqrt(((vals - mu) ** 2).sum() / n))


def contrast_from_masks(env, mask_in, mask_out) -> dict:
    """CR (Eq. 5) and CNR (Eq. 6) of env between two pixel sets."""
    n_in, mu_in, sd_in = region_stats(env, mask_in)
    n_out, mu_out, sd_out = region_stats(env, mask_out)
    cr = 20.0 * math.log10(mu_in / mu_out) if mu_in > 0 and mu_out > 0 else float("nan")
    den = math.sqrt((sd_in ** 2 + sd_out ** 2) / 2.0)
    cnr = (mu_in - mu_out) / den if den > 0 else float("nan")
    return {"n_in": n_in, "n_out": n_out, "mu_in": mu_in, "mu_out": mu_out, "sigma_in": sd_in,
            "sigma_out": sd_out, "cr_db": cr, "cnr": cnr}


def contrast(g, env, cyst_in, cyst_out) -> dict:
    """CR (Eq. 5) and CNR (Eq. 6) for one cyst: ``cyst_in`` and ``cyst_out`` are
    (x, z, r) discs in metres for the inside and the background."""
    return contrast_from_masks(env, disc_mask(g, *cyst_in), disc_mask(g, *cyst_out))


def _half_width(profile: np.ndarray, i0: int, half: float):
    """Distance (in samples) from the left to the right half-level crossing around
    the peak at i0, linear interpolation; NaN if a side never falls below half."""
    p = np.asarray(profile, dtype=np.float64)
    n = len(p)
    i = i0
    while i >= 0 and p[i] >= half:
        i -= 1
    if i < 0:
        return float("nan")
    left = i + (half - p[i]) / (p[i + 1] - p[i])
    j = i0
    while j < n and p[j] >= half:
        j += 1
    if j >= n:
        return float("nan")
    right = (j - 1) + (p[j - 1] - half) / (p[j - 1] - p[j])
    return right - left


def resolution(g, env, target, mask=None) -> dict:
    """Peak inside the disc ``target`` = (x, z, r) (first flat index among equal
    maxima; ``mask`` overrides the disc's pixels) and the lateral / axial FWHM
    through it, in metres, all in float64."""
    env = np.asarray(env, dtype=np.float64)
    if mask is None:
        mask = disc_mask(g, *target)
    if not mask.any():
        return {"peak": float("nan"), "ix": -1, "iz": -1, "fwhm_x": float("nan"),
                "fwhm_z": float("nan")}
    masked = np.where(mask, env, -np.inf)
    k = int(np.argmax(masked))  # numpy returns the first maximum
    ix, iz = divmod(k, g.nz)
    peak = float(env[ix, iz])
    half = 0.5 * peak
    return {"peak": peak, "ix": ix, "iz": iz,
            "fwhm_x": _half_width(env[:, iz], ix, half) * g.dx,
            "fwhm_z": _half_width(env[ix, :], iz, half) * g.dz}
