"""GPU parity of the f-k migrations (Stolt's and Lu's) against the FP64 oracle.

The oracle transforms with numpy's float64 FFTs; the GPU path runs float32 LDS
FFTs with float-float interpolation positions. The bar is max-normalised over the
complex image, max |gpu - oracle| / max |oracle| <= 1e-5, for one angle and for
compounds, on ragged channel counts, the record-length limits and the largest
padded array; FP16-stored RF meets 1e-5 against the oracle fed the stored values
and 1e-3 against the unrounded data. The magnitude plane is |rf + i imag| and the
log image follows from it within 0.1 dB.
"""

import numpy as np
import pytest

from oracle import fk
from synth import config_c3

from cases import geom, rand_rf

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = 1e-3
TOL_DB = 0.1


def _torch():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch


def cerr(gpu, ora):
    m = np.abs(ora).max()
    return float(np.abs(gpu - ora).max() / m) if m > 0 else float(np.abs(gpu).max())


def run(g, rf, angle=-1, want=("rf", "imag", "env", "log"), workspace=None, method="stolt"):
    from paper_2311_00482_amd import fk_migrate
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(rf)).cuda()
    print(f"fk_migrate {method} {t.shape} {t.dtype} angle {angle} grid {g.nx}x{g.nz}",
          flush=True)
    out = fk_migrate(g, t, angle, want=want, workspace=workspace, method=method)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def cplx(out):
    return out["rf"] + 1j * out["imag"]


FK_SMALL = [
    # name, geometry kwargs, angle, storage
    ("one_angle_0deg", dict(n_samples=512), 0, "f32"),
    ("one_angle_steered_i16", dict(n_samples=512, angles_deg=(-7.0,)), 0, "i16"),
    ("compound_3a_t0", dict(n_samples=1024, angles_deg=(-9.0, 0.0, 7.0),
                            t0=(0.4e-6, 0.0, -0.2e-6), nz=160, z_max=20e-3), -1, "f32"),
    ("slab_of_compound", dict(n_samples=512, angles_deg=(-8.0, 4.0, 11.0)), 2, "i16"),
    ("ragged_channels", dict(n_channels=23, n_samples=256, nx=13, nz=257, z_max=8e-3), -1,
     "f32"),
    ("max_padded_array", dict(n_channels=256, n_samples=128, nx=40, nz=50, x_min=-30e-3,
                              x_max=30e-3, z_min=1e-3, z_max=4e-3,
                              angles_deg=(-5.0, 5.0)), -1, "f32"),
    ("steep_angles", dict(n_samples=512, angles_deg=(-25.0, 30.0)), -1, "f32"),
    ("max_record", dict(n_channels=8, n_samples=4096, nx=9, nz=300, z_max=60e-3), 0, "i16"),
    ("tiny_record", dict(n_channels=2, n_samples=2, nx=3, nz=4, z_min=0.0, z_max=0.1e-3), 0,
     "f32"),
    ("one_pixel", dict(nx=1, nz=1, n_samples=256), 0, "f32"),
    ("grid_beyond_record", dict(n_samples=64, nz=50, z_min=20e-3, z_max=30e-3), 0, "f32"),
]


METHODS = ["stolt", "lu"]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("name,kw,angle,kind", FK_SMALL, ids=[c[0] for c in FK_SMALL])
def test_migration_matches_the_oracle(name, kw, angle, kind, method):
    g = geom(**kw)
    rf = rand_rf(g, 40 + len(name), kind, white=g.n_samples < 64)
    out = run(g, rf, angle, method=method)
    ref = fk.fk_migrate(g, rf.astype(np.float64), angle, method=method)
    if name == "grid_beyond_record":
        # every pixel maps past the end of the migrated image: exactly zero
        assert np.abs(ref).max() == 0 and np.abs(cplx(out)).max() == 0
        return
    assert cerr(cplx(out), ref) <= TOL32, name


@pytest.mark.parametrize("method", METHODS)
def test_fp16_storage(method):
    torch = _torch()
    g = geom(n_samples=1024, angles_deg=(-6.0, 6.0), nz=160, z_max=20e-3)
    rf = rand_rf(g, 7, "f32")
    r16 = torch.from_numpy(rf).to(torch.float16)
    got = cplx(run(g, r16.numpy(), -1, method=method))
    stored = r16.float().numpy().astype(np.float64)
    assert cerr(got, fk.fk_migrate(g, stored, method=method)) <= TOL32
    assert cerr(got, fk.fk_migrate(g, rf.astype(np.float64), method=method)) <= TOL16


def test_planes_and_log_image():
    g = geom(n_samples=512, angles_deg=(-4.0, 3.0))
    rf = rand_rf(g, 9, "i16")
    out = run(g, rf, -1)
    z = cplx(out)
    np.testing.assert_allclose(out["env"], np.abs(z), rtol=1e-6, atol=1e-6 * np.abs(z).max())
    ref = np.abs(fk.fk_migrate(g, rf.astype(np.float64)))
    ref_db = np.maximum(20 * np.log10(np.maximum(ref, 1e-300) / ref.max()), -70.0)
    keep = ref_db > -60.0
    assert np.abs(out["log"][keep] - ref_db[keep]).max() < TOL_DB
    assert out["log"].max() == 0.0 and out["log"].min() >= -70.0
    # the log image alone (no envelope plane): the envelope goes to the workspace
    alone = run(g, rf, -1, want=("rf", "log"))
    np.testing.assert_array_equal(alone["log"], out["log"])


def test_workspace_reuse_between_calls():
    """A single-angle call after a compound on the same workspace starts from a
    cleared accumulator."""
    from paper_2311_00482_amd import fk_workspace_bytes
    torch = _torch()
    g = geom(n_samples=512, angles_deg=(-6.0, 2.0, 8.0))
    rf = rand_rf(g, 11, "f32")
    ws = torch.empty(fk_workspace_bytes(g, ("rf", "imag", "env"), -1), dtype=torch.uint8,
                     device="cuda")
    comp = cplx(run(g, rf, -1, want=("rf", "imag", "env"), workspace=ws))
    one = cplx(run(g, rf, 1, want=("rf", "imag", "env"), workspace=ws))
    assert cerr(comp, fk.fk_migrate(g, rf.astype(np.float64))) <= TOL32
    assert cerr(one, fk.fk_migrate(g, rf.astype(np.float64), 1)) <= TOL32


@pytest.mark.parametrize("method", METHODS)
def test_point_scatterer_focuses_at_its_pixel(method):
    from synth import point_phantom, simulate_rf
    g = geom(n_channels=64, n_samples=2048, angles_deg=(-6.0, 0.0, 8.0), nx=128, nz=256,
             x_min=-9.6e-3, x_max=9.6e-3, z_min=5e-3, z_max=35e-3)
    ix, iz = 70, 150
    rf = simulate_rf(g, point_phantom([(g.x_pix[ix], g.z_pix[iz])]), snr_db=None,
                     quantize=False)["master"].astype(np.float32)
    env = run(g, rf, -1, method=method)["env"]
    kx, kz = np.unravel_index(np.argmax(env), env.shape)
    assert abs(kx - ix) <= 1 and abs(kz - iz) <= 1


@pytest.mark.parametrize("method", METHODS)
def test_full_size_compound_11_angles(method):
    """The measured workload: 11 angles, 128 channels x 4096 samples, 1024 x 1024
    pixels, int16 RF, the launch shape the benchmark times."""
    g = config_c3()
    rf = rand_rf(g, 2024, "i16")
    got = cplx(run(g, rf, -1, want=("rf", "imag", "env"), method=method))
    ref = fk.fk_migrate(g, rf.astype(np.float64), method=method)
    assert cerr(got, ref) <= TOL32
