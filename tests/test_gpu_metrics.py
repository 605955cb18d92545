"""GPU image metrics (FWHM, Eq. (5) CR, Eq. (6) CNR) against the float64 oracle
metrics on the same float32 envelope image.

The oracle decides disc membership in float64 (distance of the pixel centre
at most the radius); the GPU decides it in float32. Pixels whose centres lie
within a relative 1e-5 of a boundary (BAND) may go either way: every other
pixel must be decided alike, the GPU's pixel count must lie between the two
extremes, and its statistics must equal the oracle's over some choice of the
boundary pixels that gives that count. Means, deviations and widths are
float32 sums and interpolations on the GPU against float64 in the oracle:
relative 1e-5 (CR to 1e-4 dB). The benchmark phantom's anechoic cysts must read
at least 10 dB darker than their background.
"""

import math

import numpy as np
import pytest

from metric_checks import _contrast_matches, _regions, _split
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


def test_contrast_matches_oracle_and_cysts_are_dark(c3_env):
    from paper_2311_00482_amd import contrast_metrics
    g, ph, env = c3_env
    cysts, _ = _regions(g, ph)
    got = contrast_metrics(g, env, cysts)
    host = env.cpu().numpy()
    for c, r in zip(cysts, got):
        ref = _contrast_matches(g, host, c, r)
        assert ref is not None, (c, r, om.contrast(g, host, c[0], c[1]))
        print(f"cyst at ({c[0][0] * 1e3:.1f}, {c[0][1] * 1e3:.1f}) mm: CR {r['cr_db']:.2f} dB, "
              f"CNR {r['cnr']:.2f}")
        assert r["cr_db"] < -10.0  # the anechoic region reads well below the speckle


def test_resolution_matches_oracle(c3_env):
    from paper_2311_00482_amd import resolution_metrics
    g, ph, env = c3_env
    _, targets = _regions(g, ph)
    got = resolution_metrics(g, env, targets)
    host = env.cpu().numpy()
    n_finite = 0
    for t, r in zip(targets, got):
        sure, band = _split(g, t)
        # the GPU's peak is the first maximum over its own pixel set, which holds
        # every sure pixel and possibly boundary ones
        assert sure[r["ix"], r["iz"]] or band[r["ix"], r["iz"]]
        m = sure.copy()
        m[r["ix"], r["iz"]] = True
        ref = om.resolution(g, host, t, mask=m)
        assert (r["ix"], r["iz"]) == (ref["ix"], ref["iz"])
        assert r["peak"] == ref["peak"]
        assert r["peak"] >= host[sure].max()
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
    # radii off the pixel lattice: no boundary pixel, so the sets agree exactly
    assert not _split(g, cyst)[1].any() and not _split(g, back)[1].any()
    assert (got["n_in"], got["n_out"]) == (ref["n_in"], ref["n_out"])
    assert got["cnr"] == pytest.approx(ref["cnr"], rel=1e-6)
