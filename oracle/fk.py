"""FP64 reference f-k migrations (Stolt's and Lu's) for steered plane waves
(test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: it checks the GPU f-k
kernels and shares no code with them.

The paper lists Stolt's f-k migration among its beamformers (Section II-B)
without a formula. What is computed here, per steering angle th, for a linear
array of uniform pitch p (element e at x_e = x_first + e p):

 1. Time shift. Sample n of trace e was recorded at t0 + n / fs; the trace is
    advanced by the element's firing delay tau_e = (x_e sin th - min_k x_k sin th) / c
    so that a scatterer at (x0, z0) lies on t'(x) = ((x0 - x) sin th + z0 cos th
    + sqrt((x - x0)^2 + z0^2)) / c. In the temporal spectrum (length Nt = Ns,
    e^{-2 pi i f t}) that is a factor exp(2 pi i f (tau_e - t0)) on the bins
    f_k = k fs / Nt, 0 <= k <= Nt / 2 (the positive half: the result is the
    analytic, complex image).
 2. Spatial spectrum along the array, zero-padded to Nx = the power of two >= 2 N:
    kx_m = m / (Nx p) for m < Nx / 2, (m - Nx) / (Nx p) otherwise.
 3. Stolt mapping with an exploding-reflector velocity v: the image spectrum at
    (kx_m, kz_j = j df / v), 0 <= j <= Nt / 2, is the data spectrum at
    f = v sqrt(kx^2 + kz^2), linearly interpolated between bins of the one-sided
    spectrum extended by zeros past bin Nt / 2 (so it falls linearly to zero
    between bins Nt / 2 and Nt / 2 + 1 and is zero beyond; the value is then
    continuous in f, and rounding of f at exactly Nt / 2 cannot change it),
    times kz / sqrt(kx^2 + kz^2) (the Jacobian; 0 at the origin).
    v and the coordinate map are chosen so that the exploding-reflector
    hyperbola matches t'(x) at its apex in position, time and curvature: the
    apex is at x0 + z0 tan th, t' = 2 z0 cos th / c, curvature cos^3 th / (z0 c),
    giving v = c / (sqrt(2) cos^2 th) and the migrated point at
    (x1, z1) = (x0 + z0 tan th, sqrt(2) z0 / cos th). At th = 0 this is the
    classic v = c / sqrt(2).
 4. Inverse transforms: along kx (length Nx), then along kz with the one-sided
    spectrum zero-filled to Nt (numpy's ifft conventions, 1/(Nx Nt) overall),
    giving the migrated complex image on x1 = x_first + e' p, z1 = l v / fs.
 5. Each output pixel (x0, z0) reads the migrated image at (x1, z1) by bilinear
    interpolation (zero outside). Compounding sums the complex per-angle images.

Lu's migration (the scattering model; Section II-B names it beside Stolt's) maps
the data spectrum to the image spectrum exactly for a plane wave in a uniform
medium, without an exploding-reflector velocity. With coordinates relative to
the first element (x_rel = x - x_first, z) and time relative to the moment the
transmitted wave crosses it (tau_first = (x_first sin th - min_k x_k sin th) / c),
a scatterer at (x0, z0) lies on t(x) = (x0_rel sin th + z0 cos th
+ sqrt((x - x0)^2 + z0^2)) / c, and the spectra (e^{-2 pi i (kx x + f t)}, all
wavenumbers in cycles per metre, k = f / c) satisfy
    R(kx, f) ~ F(kx + k sin th, k cos th + sqrt(k^2 - kx^2)).
 1. Temporal spectrum as above, every trace times exp(2 pi i f (tau_first - t0)).
 2. Spatial spectrum as above, but zero-padded to Nx = the power of two >= 4 N:
    step 3 reads it at fractional spatial bins, and over an aperture of N p
    its phase turns by up to pi per bin at 2 N padding (pi / 2 at 4 N); linear
    interpolation across the coarser sampling leaves a ghost of the point
    (18% of the peak at 8 degrees with 64 channels, 4% at 4 N).
 3. Image spectrum on kx'_m (as kx) and kz'_j = 2 j df / c, 0 <= j <= Nt / 2:
    inverting the map, k = (kx'^2 + kz'^2) / (2 (kx' sin th + kz' cos th)),
    kx = kx' - k sin th and kz_r = kz' - k cos th (the receive wavenumber, which
    must be >= 0: the other root of the squared relation is not a wave towards
    the array); the data spectrum at (kx, f = k c) by bilinear interpolation,
    periodic in the spatial bin (the DFT is) and along frequency on the one-sided
    spectrum extended by zeros past bin Nt / 2, times the Jacobian of the change
    of variables (kx, k) -> (kx', kz'), which is kz_r / (kx' sin th + kz' cos th)
    (it vanishes where the receive wave turns grazing, so the remap is
    continuous there). Zero at the origin and wherever kz_r < 0.
 4. Inverse transforms as above: the migrated image on x1 = x_first + e' p,
    z1 = l c / (2 fs) (true coordinates: no per-angle map).
 5. Pixel (x0, z0) reads it at (x0, z0) bilinearly; angles add (complex).
"""

from __future__ import annotations

import math

import numpy as np


def fk_params(g, a: int):
    th = float(g.angles_rad[a])
    v = g.c / (math.sqrt(2.0) * math.cos(th) ** 2)
    return th, v


def uniform_pitch(g) -> float:
    x = np.asarray(g.elem_x, dtype=np.float64)
    p = (x[-1] - x[0]) / (len(x) - 1)
    assert p > 0 and np.allclose(np.diff(x), p, rtol=0, atol=1e-9 * p), "f-k needs uniform pitch"
    return float(p)


def nx_padded(n: int, factor: int = 2) -> int:
    """The power of two >= factor * n (2 for Stolt's migration, 4 for Lu's)."""
    m = 1
    while m < factor * n:
        m *= 2
    return m


def migrate_angle(g, rf_a: np.ndarray, a: int) -> np.ndarray:
    """Steps 1-4 for one angle: the migrated complex image [Nx, Nt] on (x1, z1)."""
    th, v = fk_params(g, a)
    p = uniform_pitch(g)
    N, Nt = rf_a.shape
    Nx = nx_padded(N)
    x = np.asarray(g.elem_x, dtype=np.float64)
    t0 = float(g.t0_s[a])
    tau = (x * math.sin(th) - (x * math.sin(th)).min()) / g.c
    k = np.arange(Nt // 2 + 1)
    f = k * g.fs / Nt
    S = np.fft.fft(np.asarray(rf_a, dtype=np.float64), axis=1)[:, :Nt // 2 + 1]  # [N, K]
    S = S * np.exp(2j * math.pi * f[None, :] * (tau[:, None] - t0))
    Sp = np.zeros((Nx, Nt // 2 + 1), dtype=complex)
    Sp[:N] = S
    Psi = np.fft.fft(Sp, axis=0)  # [Nx, K]
    m = np.arange(Nx)
    kx = np.where(m < Nx // 2, m, m - Nx) / (Nx * p)
    df = g.fs / Nt
    kz = np.arange(Nt // 2 + 1) * df / v
    # Stolt mapping, elementwise over (kx_m, kz_j)
    rho = np.hypot(kx[:, None], kz[None, :])
    u = v * rho / df
    i0 = np.floor(u).astype(np.int64)
    ok = (rho > 0) & (i0 <= Nt // 2)
    i0c = np.where(ok, i0, 0)
    w = u - i0
    # the spectrum extended by one zero bin past Nt / 2
    Psi_z = np.concatenate([Psi, np.zeros((Nx, 1), dtype=complex)], axis=1)
    lo = np.take_along_axis(Psi_z, i0c, axis=1)
    hi = np.take_along_axis(Psi_z, i0c + 1, axis=1)
    jac = np.divide(kz[None, :], rho, out=np.zeros_like(rho), where=rho > 0)
    I = np.where(ok, ((1.0 - w) * lo + w * hi) * jac, 0.0)
    img_kz = np.fft.ifft(I, axis=0)  # back to x1 positions
    full = np.zeros((Nx, Nt), dtype=complex)
    full[:, :Nt // 2 + 1] = img_kz
    return np.fft.ifft(full, axis=1)  # [Nx, Nt] on (x1, z1)


def lu_migrate_angle(g, rf_a: np.ndarray, a: int) -> np.ndarray:
    """Lu's steps 1-4 for one angle: the migrated complex image [Nx, Nt] on (x1, z1)."""
    th = float(g.angles_rad[a])
    sn, cs = math.sin(th), math.cos(th)
    p = uniform_pitch(g)
    N, Nt = rf_a.shape
    Nx = nx_padded(N, 4)
    x = np.asarray(g.elem_x, dtype=np.float64)
    t0 = float(g.t0_s[a])
    tau_first = (x[0] * sn - (x * sn).min()) / g.c
    K = Nt // 2 + 1
    df = g.fs / Nt
    f = np.arange(K) * df
    S = np.fft.fft(np.asarray(rf_a, dtype=np.float64), axis=1)[:, :K]  # [N, K]
    S = S * np.exp(2j * math.pi * f[None, :] * (tau_first - t0))
    Sp = np.zeros((Nx, K), dtype=complex)
    Sp[:N] = S
    Psi = np.fft.fft(Sp, axis=0)  # [Nx, K], spatial bin m, frequency bin k
    Psi_z = np.concatenate([Psi, np.zeros((Nx, 1), dtype=complex)], axis=1)
    m = np.arange(Nx)
    kxp = (np.where(m < Nx // 2, m, m - Nx) / (Nx * p))[:, None]  # kx'
    kzp = (2.0 * np.arange(K) * df / g.c)[None, :]                # kz'
    den = kxp * sn + kzp * cs
    num = kxp ** 2 + kzp ** 2
    k = np.divide(num, 2.0 * den, out=np.zeros(np.broadcast(kxp, kzp).shape), where=den > 0)
    kz_r = kzp - k * cs
    ok = (den > 0) & (kz_r >= 0)
    mf = (kxp - k * sn) * (Nx * p)   # fractional spatial bin of kx
    uf = k * g.c / df                # fractional frequency bin
    ok &= uf < K
    m0 = np.floor(mf).astype(np.int64)
    wm = mf - m0
    i0 = np.where(ok, np.floor(uf), 0).astype(np.int64)
    wu = uf - i0
    val = np.zeros_like(k, dtype=complex)
    for dm, w1 in ((0, 1.0 - wm), (1, wm)):
        for di, w2 in ((0, 1.0 - wu), (1, wu)):
            mm = np.mod(m0 + dm, Nx)
            ii = np.where(ok, i0 + di, 0)
            val += w1 * w2 * Psi_z[mm, ii]
    jac = np.divide(kz_r, den, out=np.zeros_like(k), where=ok)
    I = np.where(ok, val * jac, 0.0)
    img_kz = np.fft.ifft(I, axis=0)
    full = np.zeros((Nx, Nt), dtype=complex)
    full[:, :K] = img_kz
    return np.fft.ifft(full, axis=1)


def bilinear(M: np.ndarray, ux: np.ndarray, uz: np.ndarray) -> np.ndarray:
    """M at fractional indices (ux, uz) (arrays of one shape), zero outside."""
    Nx, Nt = M.shape
    i0, j0 = np.floor(ux).astype(np.int64), np.floor(uz).astype(np.int64)
    fx, fz = ux - i0, uz - j0
    out = np.zeros(np.shape(ux), dtype=complex)
    for di, wx in ((0, 1.0 - fx), (1, fx)):
        for dj, wz in ((0, 1.0 - fz), (1, fz)):
            i, j = i0 + di, j0 + dj
            ok = (i >= 0) & (i < Nx) & (j >= 0) & (j < Nt)
            out += np.where(ok, wx * wz * M[np.clip(i, 0, Nx - 1), np.clip(j, 0, Nt - 1)], 0.0)
    return out


def fk_migrate(g, rf, angle: int = -1, method: str = "stolt") -> np.ndarray:
    """Complex f-k image [nx, nz] by Stolt's ("stolt") or Lu's ("lu") migration;
    angle -1 sums all angles."""
    rf = np.asarray(rf, dtype=np.float64)
    if rf.ndim == 2:
        rf = rf[None]
    p = uniform_pitch(g)
    x_first = float(np.asarray(g.elem_x)[0])
    out = np.zeros((g.nx, g.nz), dtype=complex)
    x0 = (g.x0 + np.arange(g.nx) * g.dx)[:, None]
    z0 = (g.z0 + np.arange(g.nz) * g.dz)[None, :]
    for a in range(rf.shape[0]):
        if angle >= 0 and a != angle:
            continue
        if method == "stolt":
            th, v = fk_params(g, a)
            M = migrate_angle(g, rf[a], a)
            dz1 = v / g.fs
            x1 = x0 + z0 * math.tan(th)
            z1 = math.sqrt(2.0) * z0 / math.cos(th) + 0.0 * x0
        elif method == "lu":
            M = lu_migrate_angle(g, rf[a], a)
            dz1 = g.c / (2.0 * g.fs)
            x1 = x0 + 0.0 * z0
            z1 = z0 + 0.0 * x0
        else:
            raise ValueError(method)
        out += bilinear(M, (x1 - x_first) / p, z1 / dz1)
    return out
