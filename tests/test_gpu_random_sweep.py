"""Seeded random geometries against the FP64 oracle, every beamforming mode.

Each case draws, from its own seeded generator, an acquisition (channel
count, record length, transmit angles and their per-angle time offsets), a
pixel grid (every other case coarse, from one pixel upward, or fine, with
the pixel pitch of imaging grids; lateral span and offset, a depth range that
may start behind the array face), the receive F-number and
apodization, the mode (DAS, DMAS, pDAS with p in [1, 2], IQ-DAS, BB-DMAS),
the storage type and either compounding or one angle. The library plans its
own launch shape; a geometry on which no shape keeps its LDS windows within
the limit is refused (PWBF_E_UNSUPPORTED) and counted, never compared. Every
other image is compared whole with the oracle at the FP32 bar, 1e-5 of the
oracle image's maximum (complex planes for the IQ modes), on band-limited
speckle RF like the fixed cases.

Boxcar apodization decides each (pixel, channel) pair's membership by a
threshold, |x - x_e| < z / (2 F#), and its weight jumps from 0 to 1 there: a
pair within float32 rounding of the edge may fall on either side in the
kernel (float32) and in the oracle (float64), and either image is the
definition at the edge. For boxcar cases each pixel is therefore compared
with the closest of the oracle images at F# and F# (1 +- 2e-6), which moves
only pairs within 2e-6 of the edge (the kernel's decision is accurate to a
few float32 roundings, ~3e-7).
"""

import dataclasses

import numpy as np
import pytest

import oracle
from synth import Geometry

from cases import rand_rf

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
N_CASES = 120
BOXCAR_EDGE = 2e-6
MODES = ("das", "dmas", "pdas", "iqdas", "bbdmas")


def draw_case(i: int, with_decimation: bool = False):
    """Case i: (geometry, mode, angle, storage kind, pDAS p), and with
    with_decimation the IQ decimation drawn after them (1, 2 or 4 for the IQ
    modes, 1 otherwise)."""
    rng = np.random.default_rng(7000 + i)
    mode = MODES[i % len(MODES)]
    iq = mode in ("iqdas", "bbdmas")
    n_ch = int(rng.integers(2 if mode in ("dmas", "pdas", "bbdmas") else 1, 97))
    n_ang = int(rng.choice([1, 2, 3, 5, 7]))
    angles = tuple(float(a) for a in np.sort(rng.uniform(-15.0, 15.0, n_ang)).round(3))
    t0 = tuple(float(t) for t in rng.uniform(0.0, 1.5e-6, n_ang)) if rng.random() < 0.3 else ()
    ns = int(rng.choice([512, 1024, 2048])) if iq else int(rng.integers(300, 1600))
    if i % 2:
        # fine grid: pixel pitch 20-80 um across, 15-60 um in depth
        nx, nz = int(rng.integers(16, 257)), int(rng.integers(32, 513))
        half = nx * float(rng.uniform(20e-6, 80e-6)) / 2.0
        span = nz * float(rng.uniform(15e-6, 60e-6))
    else:
        # coarse grid: up to 90 x 220 pixels over up to 16 x 15 mm
        nx, nz = int(rng.integers(1, 91)), int(rng.integers(1, 221))
        half = float(rng.uniform(1e-3, 8e-3))
        span = float(rng.uniform(2e-3, 15e-3))
    xc = float(rng.uniform(-2e-3, 2e-3))
    z0 = float(rng.uniform(-1e-3, 6e-3))
    g = Geometry(n_channels=n_ch, n_samples=ns, angles_deg=angles, nx=nx, nz=nz,
                 x_min=xc - half, x_max=xc + half, z_min=z0, z_max=z0 + span,
                 f_number=float(rng.uniform(0.8, 2.5)),
                 apod=str(rng.choice(["hann", "boxcar", "none"])), t0=t0,
                 name=f"random_{i:02d}_{mode}")
    angle = -1 if rng.random() < 0.6 else int(rng.integers(0, n_ang))
    kind = str(rng.choice(["f32", "i16"]))
    p = float(rng.uniform(1.0, 2.0)) if mode == "pdas" and rng.random() < 0.5 else 2.0
    if with_decimation:
        return g, mode, angle, kind, p, (int(rng.choice([1, 2, 4])) if iq else 1)
    return g, mode, angle, kind, p


def _cerr(gpu, ora):
    m = np.abs(ora).max()
    return float(np.abs(gpu - ora).max() / m) if m > 0 else float(np.abs(gpu).max())


def oracle_image(g, mode, angle, p, rf64):
    if mode in ("iqdas", "bbdmas"):
        return oracle.iq_beamform(g, oracle.iq_demodulate(g, rf64), mode, angle)
    if mode == "das":
        return oracle.das(g, rf64, angle, parallel=True)
    if mode == "dmas":
        return oracle.dmas(g, rf64, angle, "identity", parallel=True)
    return oracle.pdas(g, rf64, angle, p, parallel=True)


def sweep_error(g, mode, angle, p, rf64, got):
    """Max-normalised error against the oracle; for boxcar apodization per
    pixel against the closest of the images at F# and F# (1 +- BOXCAR_EDGE)."""
    ref = oracle_image(g, mode, angle, p, rf64)
    m = np.abs(ref).max()
    d = np.abs(got - ref)
    if g.apod == "boxcar":
        for s in (-1.0, 1.0):
            gs = dataclasses.replace(g, f_number=g.f_number * (1.0 + s * BOXCAR_EDGE))
            d = np.minimum(d, np.abs(got - oracle_image(gs, mode, angle, p, rf64)))
    return float(d.max() / m) if m > 0 else float(np.abs(got).max())


@pytest.mark.parametrize("i", range(N_CASES))
def test_random_geometry_whole_image(i):
    import torch
    from paper_2311_00482_amd import GeometryArg, PwbfError, beamform, describe_plan, iq_demodulate
    assert torch.cuda.is_available(), "these tests need the GPU"
    g, mode, angle, kind, p = draw_case(i)
    ga = GeometryArg(g, pdas_p=p)
    try:
        plan = describe_plan(ga, mode, angle)
    except PwbfError as e:
        assert "window" in str(e) or "launch shape" in str(e), str(e)
        pytest.skip(f"{g.name}: refused ({e})")
    rf = rand_rf(g, 100 + i, kind)
    rf_t = torch.from_numpy(np.ascontiguousarray(rf)).cuda()
    if mode in ("iqdas", "bbdmas"):
        out = beamform(ga, iq_demodulate(ga, rf_t), mode, angle, want=("rf", "imag"))
        torch.cuda.synchronize()
        got = out["rf"].cpu().numpy().astype(np.float64) + 1j * out["imag"].cpu().numpy()
    else:
        out = beamform(ga, rf_t, mode, angle, want=("rf",))
        torch.cuda.synchronize()
        got = out["rf"].cpu().numpy().astype(np.float64)
    e = sweep_error(g, mode, angle, p, rf.astype(np.float64), got)
    shape = (plan["cpw"], plan["lz"], plan["wz"], plan["wx"])
    print(f"{g.name}: {g.n_channels} ch, {g.n_angles} angles (angle {angle}), "
          f"{g.nx} x {g.nz}, {g.apod}, {kind}, p {p:.3f}, shape {shape}: {e:.2e}")
    assert e <= TOL32, (g.name, e)


DECIMATED = [i for i in range(N_CASES)
             if draw_case(i, True)[1] in ("iqdas", "bbdmas") and draw_case(i, True)[5] > 1]


@pytest.mark.parametrize("i", DECIMATED)
def test_random_geometry_decimated_iq(i):
    import torch
    from paper_2311_00482_amd import GeometryArg, beamform, iq_demodulate
    g, mode, angle, kind, p, dec = draw_case(i, True)
    ga = GeometryArg(g, iq_decimation=dec)
    rf = rand_rf(g, 100 + i, kind)
    rf_t = torch.from_numpy(np.ascontiguousarray(rf)).cuda()
    out = beamform(ga, iq_demodulate(ga, rf_t), mode, angle, want=("rf", "imag"))
    torch.cuda.synchronize()
    got = out["rf"].cpu().numpy().astype(np.float64) + 1j * out["imag"].cpu().numpy()
    rf64 = rf.astype(np.float64)
    ref = oracle.iq_beamform(g, oracle.iq_demodulate(g, rf64, decimation=dec), mode, angle,
                             decimation=dec)
    m = np.abs(ref).max()
    d = np.abs(got - ref)
    if g.apod == "boxcar":
        for s in (-1.0, 1.0):
            gs = dataclasses.replace(g, f_number=g.f_number * (1.0 + s * BOXCAR_EDGE))
            alt = oracle.iq_beamform(gs, oracle.iq_demodulate(gs, rf64, decimation=dec), mode,
                                     angle, decimation=dec)
            d = np.minimum(d, np.abs(got - alt))
    assert float(d.max() / m) <= TOL32, (g.name, dec)
