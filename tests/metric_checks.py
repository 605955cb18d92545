"""Helpers of the metric checks: disc membership with a boundary band, and the
regions of the benchmark phantom's cysts and point targets.

The oracle decides disc membership in float64; the GPU decides it in float32.
Pixels whose centres lie within a relative BAND of a boundary may go either
way: the helpers enumerate the pixel sets the float32 decision may give.
"""

import itertools

import numpy as np
import pytest

from oracle import metrics as om

BAND = 1e-5


def _split(g, disc):
    """Pixels surely inside the disc, and those within BAND of its boundary."""
    d = om.disc_distance(g, *disc)
    return d <= 1.0 - BAND, np.abs(d - 1.0) < BAND


def _masks_with_count(g, disc, n):
    """Every pixel set the float32 decision may give for this disc with n pixels."""
    sure, band = _split(g, disc)
    extra = np.argwhere(band)
    k = n - int(sure.sum())
    assert 0 <= k <= len(extra), (n, int(sure.sum()), len(extra))
    assert len(extra) <= 12, "too many boundary pixels to enumerate"
    for pick in itertools.combinations(range(len(extra)), k):
        m = sure.copy()
        for i in pick:
            m[tuple(extra[i])] = True
        yield m


def _matching_masks(g, env, cyst, got):
    """(oracle contrast, inside mask, background mask) for the first pixel sets
    the float32 decision may give whose float64 statistics match ``got`` (a
    pwbf_contrast as a dict), or None."""
    for mi in _masks_with_count(g, cyst[0], got["n_in"]):
        for mo in _masks_with_count(g, cyst[1], got["n_out"]):
            ref = om.contrast_from_masks(env, mi, mo)
            ok = all(got[k] == pytest.approx(ref[k], rel=1e-5)
                     for k in ("mu_in", "mu_out", "sigma_in", "sigma_out", "cnr"))
            if ok and abs(got["cr_db"] - ref["cr_db"]) <= 1e-4:
                return ref, mi, mo
    return None


def _contrast_matches(g, env, cyst, got):
    m = _matching_masks(g, env, cyst, got)
    return None if m is None else m[0]


def _regions(g, ph):
    """Each cyst's inside and background discs, and a 1 mm disc around each
    point target."""
    from synth.phantom import cyst_regions
    targets = [(float(x), float(z), 1.0e-3) for x, z in ph.points]
    return cyst_regions(g, ph), targets
