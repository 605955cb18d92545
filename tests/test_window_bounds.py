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

from cases import SMALL, TILE_SWEEP, geom, tile_sweep_shapes
from paper_2311_00482_amd.api import Tile, describe_plan
from synth import (Geometry, config_c1, config_c2, config_c3, config_c4_frames, config_c5_probes,
                   paper_geometry)

f32 = np.float32


def fma(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64)
            + np.asarray(c, np.float64)).astype(f32)


def window_index_range(g, mode="das", angle=-1, tile=None, channels=None, margin=2e-3):
    p = describe_plan(g, mode, angle, tile)
    cpw, wz, wx, win = p["cpw"], p["wz"], p["wx"], p["win"]
    TZ, TX = (64 // cpw) * wz, wx
    ix = np.arange(p["tiles_x"] * TX)
    iz = np.arange(p["tiles_z"] * TZ)
    IX, IZ = np.meshgrid(ix, iz, indexing="ij")
    ix0 = (IX // TX) * TX
    iz0 = (IZ // TZ) * TZ
    ixe = np.minimum(ix0 + TX - 1, g.nx - 1)  # tiles stop at the grid edge
    ize = np.minimum(iz0 + TZ - 1, g.nz - 1)
    X0, DX, Z0, DZ = f32(p["X0"]), f32(p["DX"]), f32(p["Z0"]), f32(p["DZ"])
    X = fma(np.minimum(IX, ixe).astype(f32), DX, X0)
    Z = fma(np.minimum(IZ, ize).astype(f32), DZ, Z0)
    Z2 = (Z * Z).astype(f32)
    Xlo = fma(ix0.astype(f32), DX, X0)
    Xhi = fma(ixe.astype(f32), DX, X0)
    Zlo = fma(iz0.astype(f32), DZ, Z0)
    Zhi = fma(ize.astype(f32), DZ, Z0)
    N = g.n_channels
    chans = range(N) if channels is None else channels
    lo, hi = np.inf, -np.inf
    for a in range(p["n_angles_used"]):
        sa, ca, to = f32(p["sa"][a]), f32(p["ca"][a]), f32(p["to"][a])
        t = fma(X, sa, fma(Z, ca, -to))
        xc = Xlo if sa >= 0 else Xhi
        zc = Zlo if ca >= 0 else Zhi
        lt = (np.floor(fma(xc, sa, fma(zc, ca, -to))) - 1).astype(f32)
        txl = (t - lt).astype(f32)
        for e in chans:
            xe = f32(p["xe"][e])
            dxm = np.maximum(np.maximum(Xlo - xe, xe - Xhi), f32(0))
            dzm = np.where(Zlo > 0, Zlo, np.where(Zhi < 0, -Zhi, f32(0))).astype(f32)
            rmin = np.sqrt(fma(dxm, dxm, (dzm * dzm).astype(f32))).astype(f32)
            lr = (np.floor(rmin) - 1).astype(f32)
            dxe = (X - xe).astype(f32)
            rx = np.sqrt(fma(dxe, dxe, Z2)).astype(f32)
            s = (txl + (rx - lr).astype(f32)).astype(f32)
            lo = min(lo, float(np.floor(s - margin).min()))
            hi = max(hi, float(np.floor(s + margin).max()))
    return lo, hi, win


def edge_channels(n):
    return sorted({0, 1, n // 3, n // 2, n - 2, n - 1})


CASES = [
    ("c1", config_c1(), "das", 0, None),
    ("c1_cpw4", config_c1(), "das", 0, Tile(4, 1, 4, 0)),
    ("c2", config_c2(), "dmas", 0, None),
    ("c3", config_c3(), "das", -1, None),
    ("c3_tall", config_c3(), "das", -1, Tile(1, 4, 2, 0)),
    ("c3_cpw2", config_c3(), "das", -1, Tile(2, 2, 4, 8)),
    ("near_array", Geometry(n_channels=32, n_samples=1024, angles_deg=(-20.0, 0.0, 25.0),
                            nx=70, nz=90, x_min=-8e-3, x_max=8e-3, z_min=-2e-3, z_max=6e-3,
                            t0=(1e-6, 0.0, -2e-6)), "das", -1, Tile(2, 2, 2, 0)),
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
