"""FP64 reference Stolt f-k migration for steered plane waves (test infrastructure).

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


def nx_padded(n: int) -> int:
    m = 1
    while m < 2 * n:
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


def fk_migrate(g, rf, angle: int = -1) -> np.ndarray:
    """Complex f-k image [nx, nz]; angle -1 sums all angles."""
    rf = np.asarray(rf, dtype=np.float64)
    if rf.ndim == 2:
        rf = rf[None]
    p = uniform_pitch(g)
    x_first = float(np.asarray(g.elem_x)[0])
    out = np.zeros((g.nx, g.nz), dtype=complex)
    for a in range(rf.shape[0]):
        if angle >= 0 and a != angle:
            continue
        th, v = fk_params(g, a)
        M = migrate_angle(g, rf[a], a)
        dz1 = v / g.fs
        x0 = (g.x0 + np.arange(g.nx) * g.dx)[:, None]
        z0 = (g.z0 + np.arange(g.nz) * g.dz)[None, :]
        x1 = x0 + z0 * math.tan(th)
        z1 = math.sqrt(2.0) * z0 / math.cos(th) + 0.0 * x0
        out += bilinear(M, (x1 - x_first) / p, z1 / dz1)
    return out
