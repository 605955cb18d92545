"""GPU image metrics (FWHM, Eq. (5) CR, Eq. (6) CNR) against the oracle's metrics
on the same float32 envelope image.

Disc membership and the peak (argmax, first flat index on ties) are float32
decisions both sides take identically, so pixel counts and peak positions must
match exactly; means, deviations and widths are float32 sums and
interpolations on the GPU against float64 in the oracle: relative 1e-5 (CR to
1e-4 dB). The benchmark phantom's anechoic cysts must also read darker than
their background.
"""

import math

import numpy as np
import pytest

from oracle import metrics as om
from synth import config_c3, make_frame

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch


@pytest.fixture(scope="module")
def c3_env():
    from paper_2311_00482_amd import beamform
    torch = _torch()
    g = config_c3()
    fr = make_frame(g, 1003, "c3", quantize=False)
    out = beamform(g, torch.from_numpy(fr["f32"]).cuda(), "das", -1, want=("rf", "env"))
    torch.cuda.synchronize()
    return g, fr["phantom"], out["env"]


def _regions(g, ph):
    cysts = []
    for cx, cz, r in ph.cysts:
        side = 1.0 if cx < 0 else -1.0
        cysts.append(((cx, cz, 0.8 * r), (cx + side * 2.2 * r, cz, 0.8 * r)))
    targets = [(float(x), float(z), 1.0e-3) for x, z in ph.points]
    return cysts, targets


def test_contrast_matches_oracle_and_cysts_are_dark(c3_env):
    from paper_2311_00482_amd import contrast_metrics
    g, ph, env = c3_env
    cysts, _ = _regions(g, ph)
    got = contrast_metrics(g, env, cysts)
    host = env.cpu().numpy()
    for c, r in zip(cysts, got):
        ref = om.contrast(g, host, c[0], c[1])
        assert (r["n_in"], r["n_out"]) == (ref["n_in"], ref["n_out"])
        for k in ("mu_in", "mu_out", "sigma_in", "sigma_out", "cnr"):
            assert r[k] == pytest.approx(ref[k], rel=1e-5), k
        assert abs(r["cr_db"] - ref["cr_db"]) <= 1e-4
        print(f"cyst at ({c[0][0] * 1e3:.1f}, {c[0][1] * 1e3:.1f}) mm: CR {r['cr_db']:.2f} dB, "
              f"CNR {r['cnr']:.2f}")
        assert r["cr_db"] < 0.0  # the anechoic region reads darker than the speckle


def test_resolution_matches_oracle(c3_env):
    from paper_2311_00482_amd import resolution_metrics
    g, ph, env = c3_env
    _, targets = _regions(g, ph)
    got = resolution_metrics(g, env, targets)
    host = env.cpu().numpy()
    n_finite = 0
    for t, r in zip(targets, got):
        ref = om.resolution(g, host, t)
        assert (r["ix"], r["iz"]) == (ref["ix"], ref["iz"])
        assert r["peak"] == ref["peak"]
        for k in ("fwhm_x", "fwhm_z"):
            if math.isnan(ref[k]):
                assert math.isnan(r[k])
            else:
                n_finite += 1
                assert r[k] == pytest.approx(ref[k], rel=1e-5), k
                assert 0.05e-3 < r[k] < 3e-3  # a focused point, not a plateau
    assert n_finite >= len(targets)


def test_metrics_on_exact_images():
    # the cone of the oracle pins: widths exact; a two-level background
    from paper_2311_00482_amd import contrast_metrics, resolution_metrics
    from tests_metrics_images import cone_image, two_level_image
    torch = _torch()
    g, env, t, wx, wz = cone_image()
    r = resolution_metrics(g, torch.from_numpy(env).cuda(), [t])[0]
    assert r["fwhm_x"] == pytest.approx(wx, rel=1e-6) and r["fwhm_z"] == pytest.approx(wz, rel=1e-6)
    g, env, cyst, back = two_level_image()
    got = contrast_metrics(g, torch.from_numpy(env).cuda(), [(cyst, back)])[0]
    ref = om.contrast(g, env, cyst, back)
    assert (got["n_in"], got["n_out"]) == (ref["n_in"], ref["n_out"])
    assert got["cnr"] == pytest.approx(ref["cnr"], rel=1e-6)
