"""Pins of the oracle's image metrics (FWHM, Eq. (5) CR, Eq. (6) CNR) against
closed forms: disc membership by counting, moments of two-level images, the
FWHM of a triangle (exact under linear interpolation) and of a Gaussian."""

import math

import numpy as np
import pytest

from oracle import metrics
from synth import Geometry


def grid(nx=81, nz=91, pitch=0.1e-3):
    return Geometry(n_channels=8, n_samples=64, angles_deg=(0.0,), nx=nx, nz=nz,
                    x_min=-nx * pitch / 2, x_max=nx * pitch / 2, z_min=5e-3,
                    z_max=5e-3 + nz * pitch)


def test_disc_of_radius_one_and_a_half_pixels_holds_nine_pixels():
    g = grid()
    ix, iz = 40, 45
    m = metrics.disc_mask(g, g.x_pix[ix], g.z_pix[iz], 1.5 * g.dx)
    assert m.sum() == 9
    assert m[ix - 1:ix + 2, iz - 1:iz + 2].all()


def test_disc_area_and_symmetry():
    # a radius off the pixel lattice: no pixel centre lies within 1e-3 pixel of
    # the boundary, so rounding cannot decide any pixel
    g = grid(nx=301, nz=301, pitch=0.05e-3)
    r = 4.013e-3
    d = metrics.disc_distance(g, g.x_pix[150], g.z_pix[150], r)
    assert np.abs(d - 1.0).min() * r / g.dx > 1e-3
    m = metrics.disc_mask(g, g.x_pix[150], g.z_pix[150], r)
    area = m.sum() * g.dx * g.dz
    assert abs(area / (math.pi * r * r) - 1.0) < 0.01
    assert np.array_equal(m, m[::-1, :]) and np.array_equal(m, m[:, ::-1])


def test_region_stats_of_two_level_region():
    # n1 pixels at v1, n2 at v2: mean (n1 v1 + n2 v2)/n, variance n1 n2 (v1 - v2)^2 / n^2
    g = grid()
    mask = metrics.disc_mask(g, g.x_pix[40], g.z_pix[45], 1.2e-3)
    env = np.zeros((g.nx, g.nz), dtype=np.float32)
    idx = np.argwhere(mask)
    env[mask] = 3.0
    for k in range(0, len(idx), 3):
        env[tuple(idx[k])] = 7.0
    n = int(mask.sum())
    n2 = len(range(0, len(idx), 3))
    n1 = n - n2
    cnt, mu, sd = metrics.region_stats(env, mask)
    assert cnt == n
    assert mu == pytest.approx((n1 * 3.0 + n2 * 7.0) / n, rel=1e-14)
    assert sd == pytest.approx(math.sqrt(n1 * n2 * 16.0) / n, rel=1e-12)


def test_contrast_of_a_dark_cyst():
    g = grid()
    cyst = (g.x_pix[30], g.z_pix[40], 1.0e-3)
    back = (g.x_pix[60], g.z_pix[40], 1.0e-3)
    env = np.full((g.nx, g.nz), 2.0, dtype=np.float32)
    env[metrics.disc_mask(g, *cyst)] = 0.5
    # background: alternate 1.5 / 2.5 along z
    bm = metrics.disc_mask(g, *back)
    alt = np.where((np.arange(g.nz) % 2)[None, :] == 0, 1.5, 2.5).astype(np.float32)
    env = np.where(bm, alt, env)
    c = metrics.contrast(g, env, cyst, back)
    vals = env[bm].astype(np.float64)
    n1 = int((vals == 1.5).sum())
    n2 = int((vals == 2.5).sum())
    mu_out = (1.5 * n1 + 2.5 * n2) / (n1 + n2)
    sd_out = math.sqrt(n1 * n2) / (n1 + n2)  # |v1 - v2| = 1
    assert c["mu_in"] == pytest.approx(0.5) and c["sigma_in"] == pytest.approx(0.0, abs=1e-12)
    assert c["mu_out"] == pytest.approx(mu_out, rel=1e-12)
    assert c["cr_db"] == pytest.approx(20 * math.log10(0.5 / mu_out), rel=1e-12)
    assert c["cnr"] == pytest.approx((0.5 - mu_out) / math.sqrt(sd_out ** 2 / 2), rel=1e-12)


def test_fwhm_of_a_triangle_is_exact():
    # a cone of base half-width L = 8 pixels: half maximum at exactly L / 2
    g = grid()
    ix0, iz0 = 40, 45
    X = (np.arange(g.nx) - ix0)[:, None] * g.dx
    Z = (np.arange(g.nz) - iz0)[None, :] * g.dz
    env = np.maximum(0.0, 1.0 - np.maximum(np.abs(X) / (8 * g.dx), np.abs(Z) / (6 * g.dz)))
    r = metrics.resolution(g, env.astype(np.float32), (g.x_pix[ix0], g.z_pix[iz0], 1e-3))
    assert (r["ix"], r["iz"]) == (ix0, iz0) and r["peak"] == 1.0
    assert r["fwhm_x"] == pytest.approx(8 * g.dx, rel=1e-12)
    assert r["fwhm_z"] == pytest.approx(6 * g.dz, rel=1e-12)


def test_fwhm_of_a_gaussian():
    g = grid(nx=201, nz=201, pitch=0.02e-3)
    sx, sz = 0.2e-3, 0.12e-3
    X = (g.x_pix - g.x_pix[100])[:, None]
    Z = (g.z_pix - g.z_pix[90])[None, :]
    env = np.exp(-X ** 2 / (2 * sx ** 2) - Z ** 2 / (2 * sz ** 2)).astype(np.float32)
    r = metrics.resolution(g, env, (g.x_pix[100], g.z_pix[90], 0.5e-3))
    k = 2 * math.sqrt(2 * math.log(2))
    assert r["fwhm_x"] == pytest.approx(k * sx, rel=2e-3)
    assert r["fwhm_z"] == pytest.approx(k * sz, rel=2e-3)


def test_peak_ties_take_the_first_index_and_flat_profiles_give_nan():
    g = grid()
    env = np.ones((g.nx, g.nz), dtype=np.float32)
    r = metrics.resolution(g, env, (g.x_pix[40], g.z_pix[45], 0.35e-3))
    m = metrics.disc_mask(g, g.x_pix[40], g.z_pix[45], 0.35e-3)
    first = int(np.flatnonzero(m.ravel())[0])
    assert (r["ix"], r["iz"]) == divmod(first, g.nz)
    assert math.isnan(r["fwhm_x"]) and math.isnan(r["fwhm_z"])


def test_disc_membership_is_the_distance_definition():
    # brute force, one pixel at a time with math.hypot, on an off-centre disc
    g = grid(nx=23, nz=19)
    x, z, r = g.x_pix[7] + 0.37e-4, g.z_pix[11] - 0.21e-4, 0.52e-3
    m = metrics.disc_mask(g, x, z, r)
    for ix in range(g.nx):
        for iz in range(g.nz):
            xp, zp = g.x0 + ix * g.dx, g.z0 + iz * g.dz
            assert m[ix, iz] == (math.hypot(xp - x, zp - z) <= r)
    assert 0 < m.sum() < g.nx * g.nz
