"""Pins of the oracle's Stolt f-k migration: point scatterers from the independent
forward model focus at their own pixel, and a brute-force evaluation with
explicit DFT sums (no FFT) reproduces the migrated image on a tiny problem."""

import cmath
import math

import numpy as np
import pytest

from oracle import fk
from synth import Geometry, point_phantom, simulate_rf


def _geom(deg):
    angles = deg if isinstance(deg, tuple) else (deg,)
    return Geometry(n_channels=64, n_samples=2048, angles_deg=angles, nx=128, nz=256,
                    x_min=-9.6e-3, x_max=9.6e-3, z_min=5e-3, z_max=35e-3)


@pytest.mark.parametrize("deg,tol_px", [(0.0, 0), (-6.0, 2), (8.0, 2)])
def test_point_scatterer_focuses_at_its_pixel(deg, tol_px):
    g = _geom(deg)
    ix, iz = 70, 150
    rf = simulate_rf(g, point_phantom([(g.x_pix[ix], g.z_pix[iz])]), snr_db=None,
                     quantize=False)["master"]
    env = np.abs(fk.fk_migrate(g, rf))
    kx, kz = np.unravel_index(np.argmax(env), env.shape)
    assert abs(kx - ix) <= tol_px and kz == iz
    # focused: the peak stands well above the image away from the point
    far = env.copy()
    far[ix - 15:ix + 16, iz - 15:iz + 16] = 0
    assert far.max() < 0.1 * env.max()


def test_compound_focuses_two_points():
    g = _geom((-8.0, 0.0, 8.0))
    pts = [(40, 80), (90, 200)]
    rf = simulate_rf(g, point_phantom([(g.x_pix[a], g.z_pix[b]) for a, b in pts]), snr_db=None,
                     quantize=False)["master"]
    env = np.abs(fk.fk_migrate(g, rf))
    for a, b in pts:
        win = env[a - 6:a + 7, b - 6:b + 7]
        ka, kb = np.unravel_index(np.argmax(win), win.shape)
        assert abs(ka - 6) <= 1 and abs(kb - 6) <= 1


def _brute_migrate(g, rf_a, a):
    """Steps 1-4 with explicit sums (cmath, Python loops): the migrated image."""
    th = math.radians(g.angles_deg[a])
    v = g.c / (math.sqrt(2.0) * math.cos(th) ** 2)
    N, Nt = rf_a.shape
    Nx = 1
    while Nx < 2 * N:
        Nx *= 2
    p = (g.elem_x[-1] - g.elem_x[0]) / (N - 1)
    fire = [g.elem_x[e] * math.sin(th) for e in range(N)]
    K = Nt // 2 + 1
    df = g.fs / Nt
    S = [[0j] * K for _ in range(N)]
    for e in range(N):
        tau = (fire[e] - min(fire)) / g.c
        for k in range(K):
            acc = 0j
            for n in range(Nt):
                acc += rf_a[e, n] * cmath.exp(-2j * math.pi * k * n / Nt)
            S[e][k] = acc * cmath.exp(2j * math.pi * k * df * (tau - g.t0_s[a]))
    Psi = [[sum(S[e][k] * cmath.exp(-2j * math.pi * m * e / Nx) for e in range(N))
            for k in range(K)] for m in range(Nx)]
    I = [[0j] * K for _ in range(Nx)]
    for m in range(Nx):
        kx = (m if m < Nx // 2 else m - Nx) / (Nx * p)
        for j in range(K):
            kz = j * df / v
            rho = math.hypot(kx, kz)
            if rho == 0:
                continue
            u = v * rho / df
            i0 = math.floor(u)
            if i0 > Nt // 2:
                continue
            w = u - i0
            nxt = Psi[m][i0 + 1] if i0 + 1 <= Nt // 2 else 0j  # zero past the last bin
            I[m][j] = ((1 - w) * Psi[m][i0] + w * nxt) * kz / rho
    M = np.zeros((Nx, Nt), dtype=complex)
    for xe in range(Nx):
        for l in range(Nt):
            acc = 0j
            for m in range(Nx):
                for j in range(K):
                    acc += I[m][j] * cmath.exp(2j * math.pi * (m * xe / Nx + j * l / Nt))
            M[xe, l] = acc / (Nx * Nt)
    return M


@pytest.mark.parametrize("deg", [0.0, 7.0])
def test_migration_matches_explicit_sums(deg):
    g = Geometry(n_channels=3, n_samples=16, angles_deg=(deg,), nx=4, nz=4, x_min=-0.6e-3,
                 x_max=0.6e-3, z_min=0.2e-3, z_max=0.8e-3, t0=(0.05e-6,))
    rf = np.random.default_rng(3).standard_normal((1, 3, 16))
    got = fk.migrate_angle(g, rf[0], 0)
    ref = _brute_migrate(g, rf[0], 0)
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("deg", [-9.0, 0.0, 7.0])
def test_stolt_map_is_continuous_at_the_band_edge(deg):
    """The source bin of the (kx = 0, Nyquist) cell is exactly Nt / 2; a change of
    the angle far below any physical meaning (1e-12 rad) moves it across that
    bin by rounding and must not change the migrated image."""
    g = Geometry(n_channels=16, n_samples=1024, angles_deg=(deg,), nx=8, nz=8,
                 x_min=-1e-3, x_max=1e-3, z_min=5e-3, z_max=7e-3)
    rf = np.random.default_rng(5).standard_normal((16, 1024))
    a = fk.migrate_angle(g, rf, 0)
    eps = math.degrees(1e-12)
    for d in (-eps, eps):
        b = fk.migrate_angle(g.replace(angles_deg=(deg + d,)), rf, 0)
        assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()
