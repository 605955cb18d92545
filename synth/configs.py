"""Acquisition geometries and image grids of the synthetic workloads.

Units are SI (metres, seconds, hertz, radians). The linear array lies on z = 0
with element centres ``x_e = (e - (N-1)/2) * pitch``. Image grids are
cell-centred: pixel ``i`` along x sits at ``x_min + (i + 0.5) * dx`` with
``dx = (x_max - x_min) / nx``, and likewise along z.

The workloads follow the paper's acquisition (a linear array with 0.3 mm pitch
and plane-wave transmit, Table I and the experimental-setup subsection) with the
parameters of the five synthetic benchmark configurations: a 5 MHz pulse sampled
at 20 MHz, c = 1540 m/s, Hann receive apodization at f-number 1.5.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

C_SOUND = 1540.0
F0 = 5e6
FS = 20e6
PITCH = 0.3e-3
F_NUMBER = 1.5

APOD_CODES = {"hann": 0, "boxcar": 1, "none": 2}


@dataclasses.dataclass(frozen=True)
class Geometry:
    """One acquisition (array, transmit angles, sampling) plus its pixel grid."""

    n_channels: int
    n_samples: int
    angles_deg: Tuple[float, ...]
    nx: int
    nz: int
    x_min: float
    x_max: float
    z_min: float
    z_max: float
    pitch: float = PITCH
    c: float = C_SOUND
    fs: float = FS
    f0: float = F0
    f_number: float = F_NUMBER
    apod: str = "hann"
    t0: Tuple[float, ...] = ()  # per-angle time of sample 0, s; empty = all 0
    name: str = ""

    @property
    def n_angles(self) -> int:
        return len(self.angles_deg)

    @property
    def elem_x(self) -> np.ndarray:
        n = self.n_channels
        return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * self.pitch

    @property
    def angles_rad(self) -> np.ndarray:
        return np.deg2rad(np.asarray(self.angles_deg, dtype=np.float64))

    @property
    def t0_s(self) -> np.ndarray:
        if len(self.t0) == 0:
            return np.zeros(self.n_angles)
        assert len(self.t0) == self.n_angles
        return np.asarray(self.t0, dtype=np.float64)

    @property
    def dx(self) -> float:
        return (self.x_max - self.x_min) / self.nx

    @property
    def dz(self) -> float:
        return (self.z_max - self.z_min) / self.nz

    @property
    def x0(self) -> float:
        """Centre of pixel column 0."""
        return self.x_min + 0.5 * self.dx

    @property
    def z0(self) -> float:
        """Centre of pixel row 0."""
        return self.z_min + 0.5 * self.dz

    @property
    def x_pix(self) -> np.ndarray:
        return self.x0 + np.arange(self.nx) * self.dx

    @property
    def z_pix(self) -> np.ndarray:
        return self.z0 + np.arange(self.nz) * self.dz

    @property
    def apod_code(self) -> int:
        return APOD_CODES[self.apod]

    @property
    def gathers(self) -> int:
        """Pixel x channel x angle samples gathered for one frame."""
        return self.nx * self.nz * self.n_channels * self.n_angles

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


def config_c1() -> Geometry:
    """Single-frame DAS: 64 elements, 0 deg, int16 64x2048, grid 128x256 over 19x40 mm."""
    return Geometry(n_channels=64, n_samples=2048, angles_deg=(0.0,), nx=128, nz=256,
                    x_min=-9.5e-3, x_max=9.5e-3, z_min=0.0, z_max=40e-3, name="c1_das_64ch")


def config_c2() -> Geometry:
    """DMAS: 128 elements, 0 deg, int16 128x4096, grid 512x512 with dz = 25 um.

    The band-pass at 2 f0 keeps the band [f0, 3 f0]; along z the pixel grid
    samples the round-trip signal at 2 dz / c, so the band only fits below the
    grid's Nyquist when dz <= c / (12 f0) = 25.7 um.
    """
    return Geometry(n_channels=128, n_samples=4096, angles_deg=(0.0,), nx=512, nz=512,
                    x_min=-9.5e-3, x_max=9.5e-3, z_min=13.6e-3, z_max=26.4e-3,
                    name="c2_dmas_128ch")


C3_ANGLES = tuple(float(a) for a in range(-10, 11, 2))


def config_c3() -> Geometry:
    """Coherent compounding: 11 angles in [-10, 10] deg, 128x4096 per angle, 1024x1024."""
    return Geometry(n_channels=128, n_samples=4096, angles_deg=C3_ANGLES, nx=1024, nz=1024,
                    x_min=-19.05e-3, x_max=19.05e-3, z_min=5e-3, z_max=45e-3,
                    name="c3_compound_11a_128ch_1024sq")


ANGLE_SETS = {1: (0.0,), 5: (-10.0, -5.0, 0.0, 5.0, 10.0), 11: C3_ANGLES}


@dataclasses.dataclass(frozen=True)
class FrameSpec:
    geom: Geometry
    mode: str  # "das" | "dmas"
    seed: int


def config_c4_frames(n_frames: int = 32, seed: int = 2000) -> List[FrameSpec]:
    """Uneven batch: channels, angles, grid, samples and mode drawn per frame from rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n_frames):
        n_ch = int(rng.choice([64, 128]))
        n_ang = int(rng.choice([1, 5, 11]))
        nx = int(rng.choice([256, 512, 1024]))
        nz = int(rng.choice([256, 512, 1024]))
        ns = int(rng.choice([2048, 4096]))
        mode = "dmas" if rng.random() < 0.5 else "das"
        half = n_ch * PITCH / 2.0
        if mode == "das":
            z_min, z_max = 5e-3, 45e-3
        else:
            z_min, z_max = 10e-3, 10e-3 + nz * 25e-6
        g = Geometry(n_channels=n_ch, n_samples=ns, angles_deg=ANGLE_SETS[n_ang], nx=nx, nz=nz,
                     x_min=-half, x_max=half, z_min=z_min, z_max=z_max,
                     name=f"c4_f{f:02d}_{mode}_{n_ch}ch_{n_ang}a_{nx}x{nz}")
        out.append(FrameSpec(g, mode, seed + f))
    return out


def config_c5_probes() -> List[FrameSpec]:
    """The four simulated probes of the serving loop (geometry and mode; seeds 3100+)."""
    a = Geometry(n_channels=64, n_samples=2048, angles_deg=(0.0,), nx=256, nz=512,
                 x_min=-9.6e-3, x_max=9.6e-3, z_min=5e-3, z_max=45e-3, name="probe_a")
    b = Geometry(n_channels=128, n_samples=4096, angles_deg=ANGLE_SETS[5], nx=512, nz=512,
                 x_min=-19.2e-3, x_max=19.2e-3, z_min=5e-3, z_max=45e-3, name="probe_b")
    c = config_c3().replace(name="probe_c")
    d = Geometry(n_channels=64, n_samples=2048, angles_deg=(0.0,), nx=512, nz=512,
                 x_min=-9.6e-3, x_max=9.6e-3, z_min=10e-3, z_max=10e-3 + 512 * 25e-6,
                 name="probe_d")
    return [FrameSpec(a, "das", 3100), FrameSpec(b, "das", 3200), FrameSpec(c, "das", 3300),
            FrameSpec(d, "dmas", 3400)]


def paper_geometry(nx: int, nz: int) -> Geometry:
    """The paper's own acquisition (Table I; experimental setup): 64-channel receive,
    0.3 mm pitch, 7.5 MHz centre frequency, 50 MHz sampling, one non-steered plane
    wave, 3 cm depth. The imaging grids of its timing study are given as lateral x
    axial pixel counts."""
    n = 64
    half = n * PITCH / 2.0
    depth = 30e-3
    ns = int(2 ** math.ceil(math.log2(2.2 * depth / C_SOUND * 50e6)))
    return Geometry(n_channels=n, n_samples=ns, angles_deg=(0.0,), nx=nx, nz=nz,
                    x_min=-half, x_max=half, z_min=1e-3, z_max=depth, fs=50e6, f0=7.5e6,
                    name=f"paper_{nx}x{nz}")
