"""The synthetic input generator: determinism, pulse shape, storage forms."""

import math

import numpy as np

from synth import (config_c1, config_c3, config_c4_frames, config_c5_probes, make_frame,
                   point_phantom, simulate_rf)
from synth.phantom import phantom_c1, pulse_sigma, simulate_clean, simulate_clean_numpy


def test_c_core_matches_numpy_evaluation():
    g = config_c1().replace(angles_deg=(-7.0, 0.0, 9.0))
    ph = phantom_c1(g, np.random.default_rng(5), n_speckle=300)
    a = simulate_clean(g, ph)
    b = simulate_clean_numpy(g, ph)
    np.testing.assert_allclose(a, b, atol=1e-12 * np.abs(b).max())


def test_pulse_envelope_fwhm_is_two_cycles():
    f0 = 5e6
    s = pulse_sigma(f0)
    half = s * math.sqrt(2 * math.log(2))
    assert 2 * half == pytest_approx(2 / f0)


def pytest_approx(v):
    import pytest
    return pytest.approx(v, rel=1e-12)


def test_single_echo_lands_at_travel_time():
    g = config_c1().replace(n_channels=4, nx=8, nz=8)
    x, z = 0.45e-3, 12e-3
    rf = simulate_rf(g, point_phantom([[x, z]]), snr_db=None, quantize=False)["master"][0]
    for e in range(4):
        t = (z + math.hypot(x - g.elem_x[e], z)) / g.c
        n = int(round(t * g.fs))
        assert np.argmax(np.abs(rf[e])) in (n - 1, n, n + 1)


def test_frames_are_deterministic_and_quantised():
    a = make_frame(config_c1(), 1001, "c1")
    b = make_frame(config_c1(), 1001, "c1")
    np.testing.assert_array_equal(a["i16"], b["i16"])
    q = a["i16"]
    assert q.dtype == np.int16 and q.min() >= -512 and q.max() <= 511
    assert q.shape == (1, 64, 2048)
    c = make_frame(config_c1(), 1002, "c1")
    assert not np.array_equal(a["i16"], c["i16"])


def test_float_storage_forms():
    g = config_c3().replace(n_channels=16, angles_deg=(0.0, 4.0), nx=64, nz=64)
    fr = make_frame(g, 7, "c3", quantize=False)
    m = fr["master"]
    assert np.abs(m).max() == 511.0
    np.testing.assert_array_equal(fr["f32"], m.astype(np.float32))
    assert np.abs(fr["f16"].astype(np.float64) - m).max() <= 0.125 + 1e-12  # half ulp at 256..512


def test_config_shapes():
    assert config_c3().gathers == 1024 * 1024 * 128 * 11
    frames = config_c4_frames()
    assert len(frames) == 32
    assert {f.mode for f in frames} == {"das", "dmas"}
    for f in frames:
        if f.mode == "dmas":
            assert abs(f.geom.dz - 25e-6) < 1e-12
    assert [p.geom.n_angles for p in config_c5_probes()] == [1, 5, 11, 1]
