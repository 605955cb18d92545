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


# ---- Lu's migration -------------------------------------------------------

@pytest.mark.parametrize("deg", [0.0, -6.0, 8.0, 15.0])
def test_lu_point_scatterer_focuses_at_its_pixel(deg):
    g = _geom(deg)
    ix, iz = 70, 150
    rf = simulate_rf(g, point_phantom([(g.x_pix[ix], g.z_pix[iz])]), snr_db=None,
                     quantize=False)["master"]
    env = np.abs(fk.fk_migrate(g, rf, method="lu"))
    kx, kz = np.unravel_index(np.argmax(env), env.shape)
    assert (kx, kz) == (ix, iz)  # exact model of the plane wave: no lateral drift
    far = env.copy()
    far[ix - 15:ix + 16, iz - 15:iz + 16] = 0
    assert far.max() < 0.1 * env.max()


def test_lu_compound_focuses_two_points():
    g = _geom((-8.0, 0.0, 8.0))
    pts = [(40, 80), (90, 200)]
    rf = simulate_rf(g, point_phantom([(g.x_pix[a], g.z_pix[b]) for a, b in pts]), snr_db=None,
                     quantize=False)["master"]
    env = np.abs(fk.fk_migrate(g, rf, method="lu"))
    for a, b in pts:
        win = env[a - 6:a + 7, b - 6:b + 7]
        assert np.unravel_index(np.argmax(win), win.shape) == (6, 6)


@pytest.mark.parametrize("method", ["lu", "stolt"])
def test_fk_agrees_with_das_on_speckle(method):
    """Agreement with DAS images: on a speckle phantom both reconstruct the same
    scatterers, so the envelopes (DAS without apodization, along-depth Hilbert
    envelope) correlate (0.79 for Lu's, 0.76 for Stolt's here), far more than
    with a copy shifted by 4 pixels along either axis (< 0.2)."""
    import oracle
    from synth import Phantom
    g = Geometry(n_channels=32, n_samples=1024, angles_deg=(6.0,), nx=32, nz=64,
                 x_min=-2.4e-3, x_max=2.4e-3, z_min=8e-3, z_max=14e-3, apod="none")
    rng = np.random.default_rng(21)
    n = 150
    ph = Phantom(x=rng.uniform(-3e-3, 3e-3, n), z=rng.uniform(7e-3, 15e-3, n),
                 amp=rng.standard_normal(n))
    rf = simulate_rf(g, ph, snr_db=None, quantize=False)["master"]
    das = oracle.envelope_z(oracle.das(g, rf, -1).reshape(g.nx, g.nz))
    img = np.abs(fk.fk_migrate(g, rf, method=method))

    def corr(a, b):
        a = a - a.mean()
        b = b - b.mean()
        return float((a * b).sum() / np.sqrt((a * a).sum() * (b * b).sum()))
    assert corr(das, img) > 0.7
    for axis in (0, 1):
        assert corr(das, np.roll(img, 4, axis=axis)) < 0.3


def _lu_brute(g, rf_a, a):
    """Lu's steps 1-4 with explicit sums and loops (cmath)."""
    th = math.radians(g.angles_deg[a])
    sn, cs = math.sin(th), math.cos(th)
    N, Nt = rf_a.shape
    Nx = 1
    while Nx < 4 * N:
        Nx *= 2
    p = (g.elem_x[-1] - g.elem_x[0]) / (N - 1)
    fire = [g.elem_x[e] * sn for e in range(N)]
    tau_first = (fire[0] - min(fire)) / g.c
    K = Nt // 2 + 1
    df = g.fs / Nt
    S = [[0j] * K for _ in range(N)]
    for e in range(N):
        for k in range(K):
            acc = sum(rf_a[e, n] * cmath.exp(-2j * math.pi * k * n / Nt) for n in range(Nt))
            S[e][k] = acc * cmath.exp(2j * math.pi * k * df * (tau_first - g.t0_s[a]))
    Psi = [[sum(S[e][k] * cmath.exp(-2j * math.pi * m * e / Nx) for e in range(N))
            for k in range(K)] for m in range(Nx)]

    def psi(m, k):  # periodic in m, zero past the last frequency bin
        return Psi[m % Nx][k] if 0 <= k < K else 0j
    I = [[0j] * K for _ in range(Nx)]
    for m in range(Nx):
        kxp = (m if m < Nx // 2 else m - Nx) / (Nx * p)
        for j in range(K):
            kzp = 2.0 * j * df / g.c
            den = kxp * sn + kzp * cs
            if den <= 0:
                continue
            k = (kxp * kxp + kzp * kzp) / (2.0 * den)
            kzr = kzp - k * cs
            if kzr < 0:
                continue
            mf = (kxp - k * sn) * Nx * p
            uf = k * g.c / df
            if uf >= K:
                continue
            m0, i0 = math.floor(mf), math.floor(uf)
            wm, wu = mf - m0, uf - i0
            v = ((1 - wm) * (1 - wu) * psi(m0, i0) + (1 - wm) * wu * psi(m0, i0 + 1)
                 + wm * (1 - wu) * psi(m0 + 1, i0) + wm * wu * psi(m0 + 1, i0 + 1))
            I[m][j] = v * kzr / den
    M = np.zeros((Nx, Nt), dtype=complex)
    for xe in range(Nx):
        for l in range(Nt):
            acc = 0j
            for m in range(Nx):
                for j in range(K):
                    acc += I[m][j] * cmath.exp(2j * math.pi * (m * xe / Nx + j * l / Nt))
            M[xe, l] = acc / (Nx * Nt)
    return M


@pytest.mark.parametrize("deg", [0.0, 7.0, -12.0])
def test_lu_migration_matches_explicit_sums(deg):
    g = Geometry(n_channels=3, n_samples=16, angles_deg=(deg,), nx=4, nz=4, x_min=-0.6e-3,
                 x_max=0.6e-3, z_min=0.2e-3, z_max=0.8e-3, t0=(0.05e-6,))
    rf = np.random.default_rng(4).standard_normal((1, 3, 16))
    got = fk.lu_migrate_angle(g, rf[0], 0)
    ref = _lu_brute(g, rf[0], 0)
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("deg,c", [(-9.0, 1540.0), (0.0, 1540.0), (7.0, 1540.0),
                                   (0.0, 1500.0)])
def test_lu_remap_is_continuous(deg, c):
    """Cells on the branch boundary (grazing receive wave) and on the band edge
    take values that a 1e-12 rad change of the angle must not move. With
    c = 1500 m/s the kz' step is exactly twice the kx' step here, so at 0 deg
    the boundary kz' = |kx'| runs through grid cells and a hard cut there would
    flip with the sign of the perturbation."""
    g = Geometry(n_channels=16, n_samples=1024, angles_deg=(deg,), nx=8, nz=8,
                 x_min=-1e-3, x_max=1e-3, z_min=5e-3, z_max=7e-3, c=c)
    rf = np.random.default_rng(6).standard_normal((16, 1024))
    a = fk.lu_migrate_angle(g, rf, 0)
    eps = math.degrees(1e-12)
    for d in (-eps, eps):
        b = fk.lu_migrate_angle(g.replace(angles_deg=(deg + d,)), rf, 0)
        assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()
