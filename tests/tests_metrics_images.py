"""Synthetic envelope images with exactly known metrics (shared by CPU and GPU tests)."""

import numpy as np

from synth import Geometry


def grid(nx=81, nz=91, pitch=0.1e-3):
    return Geometry(n_channels=8, n_samples=64, angles_deg=(0.0,), nx=nx, nz=nz,
                    x_min=-nx * pitch / 2, x_max=nx * pitch / 2, z_min=5e-3,
                    z_max=5e-3 + nz * pitch)


def cone_image():
    """A cone of half-widths 8 (x) and 6 (z) pixels at (40, 45): FWHM 8 dx, 6 dz."""
    g = grid()
    ix0, iz0 = 40, 45
    X = (np.arange(g.nx) - ix0)[:, None] * g.dx
    Z = (np.arange(g.nz) - iz0)[None, :] * g.dz
    env = np.maximum(0.0, 1.0 - np.maximum(np.abs(X) / (8 * g.dx), np.abs(Z) / (6 * g.dz)))
    return g, env.astype(np.float32), (g.x_pix[ix0], g.z_pix[iz0], 1.03e-3), 8 * g.dx, 6 * g.dz


def two_level_image():
    """A dark disc (0.5) and a background disc alternating 1.5 / 2.5 along z (radii
    off the pixel lattice, so no pixel centre lies on a boundary)."""
    from oracle import metrics
    g = grid()
    cyst = (g.x_pix[30], g.z_pix[40], 1.03e-3)
    back = (g.x_pix[60], g.z_pix[40], 1.03e-3)
    env = np.full((g.nx, g.nz), 2.0, dtype=np.float32)
    env[metrics.disc_mask(g, *cyst)] = 0.5
    bm = metrics.disc_mask(g, *back)
    alt = np.where((np.arange(g.nz) % 2)[None, :] == 0, 1.5, 2.5).astype(np.float32)
    env = np.where(bm, alt, env).astype(np.float32)
    return g, env, cyst, back
