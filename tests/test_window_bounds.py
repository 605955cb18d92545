"""The kernel's LDS windows contain every gather, shown on the CPU.

Using the float32 constants the library hands its kernel (pwbf_describe_plan),
this re-evaluates in float32 the kernel's per-tile window origins and every
pixel's interpolation index for the shapes the tests and the benchmark launch,
and checks 0 <= floor(s) <= win - 1 with a margin for the one-ulp hardware
square root. A window index outside that range would read a neighbouring
window, so this is checked before the kernel ever runs.
"""

import numpy as np
import pytest

from cases import REFUSED, SMALL, TILE_SWEEP, geom, tile_sweep_shapes
from paper_2311_00482_amd.api import Tile, describe_plan
from synth import (Geometry, config_c1, config_c2, config_c3, config_c4_frames, config_c5_probes,
                   paper_geometry)

f32 = np.float32


def fma(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64)
            + np.asarray(c, np.float64)).astype(f32)


def window_index_range(g, mode="das", angle=-1, tile=None, channels=None, margin=2e-3):
    """(min, max) of the window entry read over every pixel, angle and listed
    channel, and the window length, following the kernel's arithmetic: tile
    (DMAS, pDAS: wavefront) constants in float-float (emulated in float64),
    per-pixel offsets in float32."""
    p = describe_plan(g, mode, angle, tile)
    win = p["win"]
    TZ, TX = p["tile_z"], p["tile_x"]
    ix = np.arange(p["tiles_x"] * TX)
    iz = np.arange(p["tiles_z"] * TZ)
    IX, IZ = np.meshgrid(ix, iz, indexing="ij")
    ix0 = (IX // TX) * TX
    iz0 = (IZ // TZ) * TZ
    ixe = np.minimum(ix0 + TX - 1, g.nx - 1)  # tiles stop at the grid edge
    ize = np.minimum(iz0 + TZ - 1, g.nz - 1)
    ixq = (ix0 + ixe) >> 1
    izq = (iz0 + ize) >> 1
    DX, DZ = f32(p["DX"]), f32(p["DZ"])
    X0d = float(p["X0"]) + float(p["X0l"])
    Z0d = float(p["Z0"]) + float(p["Z0l"])
    DXd = float(p["DX"]) + float(p["DXl"])
    DZd = float(p["DZ"]) + float(p["DZl"])
    # DMAS and pDAS take each wavefront's centre pixel as the reference of the
    # per-gather offsets; the others take the tile's
    wref = mode in ("dmas", "pdas")
    if wref:
        lz = p["lz"]
        lx = 64 // p["cpw"] // lz
        bx0 = ix0 + ((IX - ix0) // lx) * lx
        bz0 = iz0 + ((IZ - iz0) // lz) * lz
        ixr = (bx0 + np.minimum(bx0 + lx - 1, ixe)) >> 1
        izr = (bz0 + np.minimum(bz0 + lz - 1, ize)) >> 1
    else:
        ixr, izr = ixq, izq
    dx = ((np.minimum(IX, ixe) - ixr).astype(f32) * DX).astype(f32)
    dz = ((np.minimum(IZ, ize) - izr).astype(f32) * DZ).astype(f32)
    dxlo = ((ix0 - ixq).astype(f32) * DX).astype(f32)
    dxhi = ((ixe - ixq).astype(f32) * DX).astype(f32)
    dzlo = ((iz0 - izq).astype(f32) * DZ).astype(f32)
    dzhi = ((ize - izq).astype(f32) * DZ).astype(f32)
    Xq = X0d + ixq * DXd  # float64 stands in for the kernel's float-float
    Zq = Z0d + izq * DZd
    Zqf = Zq.astype(f32)
    Xr = X0d + ixr * DXd
    Zr = Z0d + izr * DZd
    cp = fma(2 * Zr.astype(f32), dz, fma(dx, dx, (dz * dz).astype(f32)))
    dx2 = (2 * dx).astype(f32)
    chans = range(g.n_channels) if channels is None else channels
    lo, hi = np.inf, -np.inf
    for a in range(p["n_angles_used"]):
        sah, cah = f32(p["sa"][a]), f32(p["ca"][a])
        sa = float(p["sa"][a]) + float(p["sal"][a])
        ca = float(p["ca"][a]) + float(p["cal"][a])
        to = float(p["to"][a]) + float(p["tol"][a])
        txq = Xq * sa + Zq * ca - to
        dmin = (np.minimum(dxlo * sah, dxhi * sah) + np.minimum(dzlo * cah, dzhi * cah))
        lt = np.floor(txq + dmin.astype(np.float64)) - 1
        ot, orr = p["off_t"], p["off_r"]
        if wref:  # the reference's delay split into an integer kT and a fraction
            trel = Xr * sa + Zr * ca - to - lt - ot
            kt = np.rint(trel)
            txl = ((trel - kt).astype(f32) + fma(dx, sah, (dz * cah).astype(f32))).astype(f32)
        else:
            kt = 0
            txl = ((txq - lt - ot).astype(f32) + fma(dx, sah, (dz * cah).astype(f32))).astype(f32)
        for e in chans:
            xe = float(p["xe"][e]) + float(p["xel"][e])
            dq = Xq - xe
            rq2 = dq * dq + Zq * Zq
            rq = np.sqrt(rq2)
            dqf = dq.astype(f32)
            ddx = np.maximum(np.maximum(dqf + dxlo, -(dqf + dxhi)), f32(0))
            zlo = (Zqf + dzlo).astype(f32)
            zhi = (Zqf + dzhi).astype(f32)
            ddz = np.where(zlo > 0, zlo, np.where(zhi < 0, -zhi, f32(0))).astype(f32)
            rmin = np.sqrt(fma(ddx, ddx, (ddz * ddz).astype(f32))).astype(f32)
            lr = np.floor(rmin).astype(np.float64) - 1
            if wref:
                dw = Xr - xe
                rw2 = dw * dw + Zr * Zr
                rw = np.sqrt(rw2)
                rrel = rw - lr - orr
                kr = np.rint(rrel)
                num = fma(dx2, dw.astype(f32), cp)
                den = (np.sqrt((rw2.astype(f32) + num).astype(f32)) + rw.astype(f32)).astype(f32)
                rxl = fma(num, (1 / den.astype(np.float64)).astype(f32), (rrel - kr).astype(f32))
            else:
                kr = 0
                num = fma(dx2, dqf, cp)
                den = (np.sqrt((rq2.astype(f32) + num).astype(f32)) + rq.astype(f32)).astype(f32)
                rxl = fma(num, (1 / den.astype(np.float64)).astype(f32),
                          (rq - lr - orr).astype(f32))
            s = (txl + rxl).astype(f32)  # centred; the entry read is floor(s) + ot + orr (+ kT + kR)
            lo = min(lo, float((np.floor(s - margin) + kt + kr).min()) + ot + orr)
            hi = max(hi, float((np.floor(s + margin) + kt + kr).max()) + ot + orr)
    return lo, hi, win


def edge_channels(n):
    return sorted({0, 1, n // 3, n // 2, n - 2, n - 1})


CASES = [
    ("c1", config_c1(), "das", 0, None),
    ("c1_cpw4", config_c1(), "das", 0, Tile(4, 8, 1, 4, 0)),
    ("c2", config_c2(), "dmas", 0, None),
    ("c3", config_c3(), "das", -1, None),
    ("c3_tall", config_c3(), "das", -1, Tile(1, 32, 1, 2, 0)),
    ("c3_cpw2", config_c3(), "das", -1, Tile(2, 16, 2, 4, 8)),
    ("c3_wide", config_c3(), "das", -1, Tile(1, 4, 2, 4, 0)),
    ("near_array", Geometry(n_channels=32, n_samples=1024, angles_deg=(-20.0, 0.0, 25.0),
                            nx=70, nz=90, x_min=-8e-3, x_max=8e-3, z_min=-2e-3, z_max=6e-3,
                            t0=(1e-6, 0.0, -2e-6)), "das", -1, Tile(2, 8, 2, 2, 0)),
]


@pytest.mark.parametrize("name,g,mode,angle,tile", CASES, ids=[c[0] for c in CASES])
def test_every_gather_inside_its_window(name, g, mode, angle, tile):
    lo, hi, win = window_index_range(g, mode, angle, tile, edge_channels(g.n_channels))
    assert lo >= 0, (name, lo)
    assert hi <= win - 1, (name, hi, win)


@pytest.mark.parametrize("name,kw,mode,angle,tile,kind", SMALL, ids=[s[0] for s in SMALL])
def test_small_gpu_cases_inside_windows(name, kw, mode, angle, tile, kind):
    g = geom(**kw)
    t = Tile(*tile) if tile else None
    lo, hi, win = window_index_range(g, mode, angle, t)
    assert lo >= 0 and hi <= win - 1, (name, lo, hi, win)


def test_tile_sweep_inside_windows():
    shapes = tile_sweep_shapes()
    assert len(shapes) >= 40
    for shape in shapes:
        lo, hi, win = window_index_range(TILE_SWEEP, "das", -1, Tile(*shape))
        assert lo >= 0 and hi <= win - 1, (shape, lo, hi, win)


@pytest.mark.parametrize("nx,nz", [(128, 32), (256, 32), (512, 64), (1024, 64), (1750, 64)])
def test_paper_grids_inside_windows(nx, nz):
    g = paper_geometry(nx, nz)
    lo, hi, win = window_index_range(g, "das", 0, None, edge_channels(g.n_channels))
    assert lo >= 0 and hi <= win - 1


@pytest.mark.slow
def test_batch_and_serving_shapes_inside_windows():
    seen = set()
    for spec in config_c4_frames() + config_c5_probes():
        g = spec.geom
        key = (g.n_channels, g.n_angles, g.nx, g.nz, g.z_min, spec.mode)
        if key in seen:
            continue
        seen.add(key)
        lo, hi, win = window_index_range(g, spec.mode, -1, None, edge_channels(g.n_channels))
        assert lo >= 0 and hi <= win - 1, (g.name, lo, hi, win)


def _tuner_shapes():
    # Of the candidates the tuner times for batch blocks (8 wavefronts), the ones
    # with the extreme tile extents: deepest (64 x 8), widest (8 x 64), default.
    return [(1, 32, 2, 4, 0), (1, 8, 1, 8, 0), (1, 16, 1, 8, 0), (4, 16, 1, 8, 0)]


@pytest.mark.slow
def test_tuner_shapes_inside_windows_on_batch_workload():
    from paper_2311_00482_amd import PwbfError
    seen = set()
    for spec in config_c4_frames() + config_c5_probes():
        g = spec.geom
        key = (g.n_channels, g.n_angles, g.nx, g.nz, g.z_min, spec.mode)
        if key in seen:
            continue
        seen.add(key)
        for shape in _tuner_shapes():
            try:
                lo, hi, win = window_index_range(g, spec.mode, -1, Tile(*shape),
                                                 [0, g.n_channels - 1])
            except PwbfError:
                continue  # a shape whose windows do not fit is rejected, never launched
            assert lo >= 0 and hi <= win - 1, (g.name, shape, lo, hi, win)


def test_batch_test_shapes_inside_windows():
    import torch  # noqa: F401  (mixed_frames builds tensors; run on the CPU here)
    specs = [
        (geom(angles_deg=(-8.0, 0.0, 8.0), nx=80, nz=128), "das", -1, (1, 16, 1, 8, 0)),
        (geom(n_channels=32, nx=66, nz=128), "dmas", 0, (4, 8, 1, 8, 0)),
        (geom(angles_deg=(-10., -5., 0., 5., 10.), nx=21, nz=256, n_channels=24), "das", -1,
         (4, 16, 1, 8, 0)),
        (geom(angles_deg=(0.0, 4.0), n_channels=20, nx=128, nz=512, z_min=10e-3,
              z_max=10e-3 + 512 * 25e-6), "dmas", -1, (1, 16, 2, 4, 0)),
        (geom(angles_deg=tuple(range(-6, 8, 2)), nx=68, nz=128), "das", 3, (1, 8, 2, 4, 0)),
        (geom(angles_deg=(-5.0, 5.0), n_channels=20, nx=90, nz=128), "pdas", -1,
         (4, 8, 1, 8, 0)),
    ]
    for g, mode, angle, shape in specs:
        lo, hi, win = window_index_range(g, mode, angle, Tile(*shape))
        assert lo >= 0 and hi <= win - 1, (shape, lo, hi, win)


MAX_WINDOW = 64  # PWBF_MAX_WINDOW


@pytest.mark.parametrize("name,kw,mode,angle,tile", REFUSED, ids=[c[0] for c in REFUSED])
def test_long_windows_are_refused(name, kw, mode, angle, tile):
    # a shape whose windows exceed 64 entries would put float32 delay offsets
    # past 32 samples: the host refuses it, and the default plan of the same
    # call picks a shape that fits
    from paper_2311_00482_amd import PwbfError
    from paper_2311_00482_amd._abi import E_UNSUPPORTED
    g = geom(**kw)
    with pytest.raises(PwbfError) as ei:
        describe_plan(g, mode, angle, Tile(*tile))
    assert ei.value.code == E_UNSUPPORTED
    assert "window" in str(ei.value)
    assert describe_plan(g, mode, angle, None)["win"] <= MAX_WINDOW


def test_every_workload_default_fits_the_window_limit():
    specs = [(config_c1(), "das"), (config_c2(), "dmas"), (config_c3(), "das"),
             (config_c3(), "iqdas"), (config_c3(), "pdas")]
    specs += [(s.geom, s.mode) for s in config_c4_frames() + config_c5_probes()]
    specs += [(paper_geometry(nx, nz), "das") for nx, nz in
              [(128, 32), (256, 32), (512, 64), (1024, 64), (1750, 64)]]
    for g, mode in specs:
        for angle in (-1, 0):
            assert describe_plan(g, mode, angle, None)["win"] <= MAX_WINDOW, (g.name, mode)
    # batch blocks (8 wavefronts) as well
    from paper_2311_00482_amd import lib
    assert lib() is not None


def _root_offset_bound(g, angle, cpw, lz):
    """Largest distance (samples) of a DMAS / pDAS gather's delay from its
    wavefront's reference pixel for lane groups of lz x (64 / cpw / lz)
    pixels: twice the depth reach plus the lateral reach times the largest
    transmit sine plus the sine of the widest apodized receive angle."""
    lx = 64 // cpw // lz
    scale = g.fs / g.c
    dx = (g.x_max - g.x_min) / max(g.nx - 1, 1) * scale
    dz = (g.z_max - g.z_min) / max(g.nz - 1, 1) * scale
    angles = g.angles_deg if angle < 0 else (g.angles_deg[angle],)
    smax = max(abs(np.sin(np.deg2rad(a))) for a in angles)
    sphi = 1.0 if g.apod == "none" else 1.0 / np.sqrt(1.0 + 4.0 * g.f_number ** 2)
    return 2.0 * (lz // 2) * dz + (lx // 2) * dx * (smax + sphi)


def test_root_modes_pick_compact_lane_groups():
    # the shapes DMAS and pDAS plans pick themselves keep every gather within
    # 4 samples of its wavefront's reference pixel (re-derived here from the
    # geometry) when some shape does; an explicit tall shape is taken as given;
    # a grid on which no shape is that compact still plans (the best fitting)
    specs = [(config_c2(), "dmas"), (config_c2(), "pdas"), (config_c3(), "pdas"),
             (config_c3(), "dmas")]
    specs += [(s.geom, s.mode) for s in config_c4_frames() if s.mode != "das"]
    for g, mode in specs:
        p = describe_plan(g, mode, -1, None)
        assert _root_offset_bound(g, -1, p["cpw"], p["lz"]) <= 4.0 + 1e-9, (g.name, p)
    f21 = config_c4_frames()[21].geom
    assert _root_offset_bound(f21, -1, 1, 32) > 10.0
    p = describe_plan(f21, "dmas", -1, Tile(1, 32, 1, 8, 0))
    assert (p["cpw"], p["lz"]) == (1, 32)
    # a small grid whose default shape (4 lane groups of 16 x 1 pixels, what DAS
    # takes) fits the window but reaches 7.3 samples: DMAS plans a flatter one
    small = geom(n_channels=32, nx=64, nz=256)
    assert describe_plan(small, "das", 0, None)["lz"] == 16
    assert _root_offset_bound(small, 0, 4, 16) > 4.0
    describe_plan(small, "dmas", 0, Tile(4, 16, 1, 8, 0))  # accepted when explicit
    p = describe_plan(small, "dmas", 0, None)
    assert _root_offset_bound(small, 0, p["cpw"], p["lz"]) <= 4.0
    coarse = geom(n_channels=12, nx=21, nz=77)  # pixels 3.7 x 1.5 samples
    p = describe_plan(coarse, "dmas", 0, None)
    assert _root_offset_bound(coarse, 0, p["cpw"], p["lz"]) > 0


def test_too_coarse_grid_is_refused():
    # pixels of ~40 x 40 samples: no launch shape keeps a window within 64 entries
    from paper_2311_00482_amd import PwbfError
    from paper_2311_00482_amd._abi import E_UNSUPPORTED
    g = geom(nx=5, nz=5, x_min=-6e-3, x_max=6e-3, z_min=5e-3, z_max=20e-3)
    with pytest.raises(PwbfError) as ei:
        describe_plan(g, "das", 0, None)
    assert ei.value.code == E_UNSUPPORTED
