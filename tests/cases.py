"""Small geometries shared by the GPU parity tests and the CPU window-bound check."""

import numpy as np

from synth import Geometry


def geom(**kw):
    base = dict(n_channels=16, n_samples=600, angles_deg=(0.0,), nx=37, nz=100,
                x_min=-3e-3, x_max=3e-3, z_min=3e-3, z_max=12e-3, f_number=1.2)
    base.update(kw)
    return Geometry(**base)


def rand_rf(g, seed, kind="f32", white=False):
    """Seeded random channel data. By default band-limited like ultrasound RF:
    white Gaussian noise filtered by the transmitted pulse (a two-cycle Gaussian
    burst at f0), i.e. fully developed speckle. ``white=True`` keeps the raw
    white noise (content up to Nyquist), the harshest input for interpolation.
    kind "i16" scales to the 10-bit range and rounds, "f32" returns float32."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((g.n_angles, g.n_channels, g.n_samples))
    if not white:
        sigma = (2.0 / g.f0) / (2.0 * np.sqrt(2.0 * np.log(2.0)))
        t = np.arange(-int(np.ceil(3.5 * sigma * g.fs)), int(np.ceil(3.5 * sigma * g.fs)) + 1) / g.fs
        pulse = np.exp(-0.5 * (t / sigma) ** 2) * np.cos(2 * np.pi * g.f0 * t)
        x = np.apply_along_axis(lambda r: np.convolve(r, pulse, mode="same"), -1, x)
        x /= x.std()
    if kind == "i16":
        return np.clip(np.rint(x * 511.0 / np.abs(x).max()), -512, 511).astype(np.int16)
    return x.astype(np.float32)


SMALL = [
    # name, geometry kwargs, mode, angle, tile, dtype
    ("das_1ch", dict(n_channels=1), "das", 0, None, "f32"),
    ("das_ragged_cpw1", dict(nx=37, nz=100), "das", 0, (1, 16, 1, 2, 0), "f32"),
    ("das_ragged_cpw2", dict(nx=13, nz=257), "das", 0, (2, 8, 2, 2, 6), "i16"),
    ("das_ragged_cpw4", dict(nx=9, nz=33, n_channels=7), "das", 0, (4, 8, 1, 1, 4), "f32"),
    ("das_one_pixel", dict(nx=1, nz=1), "das", 0, None, "f32"),
    # lane groups of 8 and 4 pixels (the shapes coarse grids fall back to)
    ("das_cpw8", dict(nx=37, nz=100, angles_deg=(-5.0, 0.0, 5.0)), "das", -1, (8, 8, 1, 2, 0),
     "f32"),
    ("dmas_cpw16", dict(nx=21, nz=77, n_channels=20), "dmas", 0, (16, 2, 2, 2, 0), "i16"),
    ("das_one_column", dict(nx=1, nz=300), "das", 0, (1, 64, 1, 1, 0), "f32"),
    ("das_boxcar", dict(apod="boxcar"), "das", 0, None, "f32"),
    ("das_no_apod_near_array", dict(apod="none", z_min=-1e-3, z_max=4e-3), "das", 0, None, "f32"),
    ("das_hann_near_array_cpw1", dict(z_min=-1e-3, z_max=4e-3), "das", 0, (1, 16, 1, 2, 0), "f32"),
    ("compound_3a_boxcar_cpw1", dict(apod="boxcar", angles_deg=(-12.0, 0.0, 9.0)), "das", -1,
     (1, 16, 1, 2, 0), "f32"),
    ("das_record_too_short", dict(n_samples=120), "das", 0, None, "f32"),
    # a coarse grid (pixels of 15.6 x 2 samples) whose default tile does not
    # fit the window limit: the plan falls back to the largest tile that does
    ("das_coarse_grid_fallback", dict(nz=64, z_min=3e-3, z_max=13e-3, nx=5), "das", 0, None,
     "f32"),
    ("compound_3a_coarse_grid_fallback", dict(nz=64, z_min=3e-3, z_max=13e-3, nx=5,
                                              angles_deg=(-10.0, 0.0, 10.0)), "das", -1, None,
     "i16"),
    # the longest window the kernels accept (64 entries)
    ("das_window_at_limit", dict(nx=21, nz=77), "das", 0, (2, 16, 1, 4, 4), "f32"),
    ("compound_3a", dict(angles_deg=(-12.0, 0.0, 9.0)), "das", -1, None, "f32"),
    ("compound_7a_t0", dict(angles_deg=(-15., -10., -5., 0., 5., 10., 15.),
                            t0=(0.5e-6, 0.0, -0.3e-6, 1e-6, 0.0, 0.2e-6, 0.0)), "das", -1,
     (1, 16, 1, 2, 0), "f32"),
    ("compound_17a_generic", dict(angles_deg=tuple(range(-16, 18, 2)), nx=11, nz=70), "das",
     -1, None, "f32"),
    ("compound_32a_generic", dict(angles_deg=tuple(np.linspace(-20, 20, 32)), nx=6, nz=40,
                                  n_channels=8), "das", -1, None, "f32"),
    ("angle_slab", dict(angles_deg=(-8.0, 4.0, 11.0)), "das", 2, None, "i16"),
    ("dmas_2ch", dict(n_channels=2), "dmas", 0, None, "f32"),
    ("dmas_coarse_grid_fallback", dict(nz=64, z_min=3e-3, z_max=13e-3, nx=5), "dmas", 0, None,
     "f32"),
    ("dmas_ragged_cpw2", dict(nx=63, nz=231, n_channels=12), "dmas", 0, (2, 16, 1, 4, 4),
     "f32"),
    ("dmas_compound_5a", dict(angles_deg=(-10., -5., 0., 5., 10.)), "dmas", -1, None, "i16"),
    # a DMAS window of 40 entries: delays are measured from each
    # wavefront's centre pixel, so the window's length does not enter them
    ("dmas_window_40", dict(), "dmas", 0, (16, 2, 1, 8, 0), "f32"),
    ("dmas_compound_generic", dict(angles_deg=tuple(range(-18, 18, 2)), nx=7, nz=40,
                                   n_channels=6), "dmas", -1, (8, 4, 1, 1, 0), "f32"),
]


# Launch shapes whose LDS windows exceed the 64-entry limit: every call with
# them is refused before anything is enqueued.
REFUSED = [
    # name, geometry kwargs, mode, angle, tile
    ("das_64_deep_column", dict(nz=64, z_min=3e-3, z_max=13e-3, nx=5), "das", 0,
     (1, 64, 1, 1, 0)),
    ("compound_3a_64_deep_column", dict(nz=64, z_min=3e-3, z_max=13e-3, nx=5,
                                        angles_deg=(-10.0, 0.0, 10.0)), "das", -1,
     (1, 64, 1, 1, 0)),
    ("dmas_64_deep_column", dict(nz=64, z_min=3e-3, z_max=13e-3, nx=5), "dmas", 0,
     (1, 64, 1, 1, 0)),
    ("das_ragged_64x16", dict(nx=37, nz=100), "das", 0, (1, 64, 1, 4, 0)),
    ("compound_7a_32x8", dict(angles_deg=(-15., -10., -5., 0., 5., 10., 15.)), "das", -1,
     (1, 16, 2, 2, 0)),
    ("dmas_generic_4x8", dict(angles_deg=tuple(range(-18, 18, 2)), nx=7, nz=40, n_channels=6),
     "dmas", -1, (4, 4, 1, 2, 0)),
    ("pdas_64_deep_column", dict(nz=64, z_min=3e-3, z_max=13e-3, nx=5), "pdas", 0,
     (1, 64, 1, 1, 0)),
]


TILE_SWEEP = geom(angles_deg=(-6.0, 0.0, 6.0, 12.0), nx=40, nz=140, n_channels=24)
_SWEEP_ALL = [(cpw, lz, wz, wx, chunk) for cpw in (1, 2, 4)
              for lz in sorted({64 // cpw, 16, 4})
              for wz, wx in ((1, 1), (1, 8), (2, 4), (8, 1))
              for chunk in (0, cpw, 3 * cpw)]


def tile_sweep_shapes():
    """The sweep's launch shapes whose LDS windows fit (the others are rejected)."""
    from paper_2311_00482_amd import PwbfError, Tile, describe_plan
    ok = []
    for sh in _SWEEP_ALL:
        try:
            describe_plan(TILE_SWEEP, "das", -1, Tile(*sh))
            ok.append(sh)
        except PwbfError:
            pass
    return ok
