"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
special-case delays, the impulse response, a point scatterer produced by the
independent forward model, invariants of a linear beamformer, closed forms of
DMAS and pDAS, relations between the beamformers (pDAS at p = 1 is DAS; at
p = 2 with boxcar weights and positive data it is 2 DMAS + DAS), and a
brute-force re-evaluation that interpolates with numpy.interp.
"""

import math

import numpy as np
import pytest

import oracle
from synth import Geometry, point_phantom, simulate_rf


def small_geom(**kw):
    base = dict(n_channels=16, n_samples=512, angles_deg=(0.0,), nx=12, nz=20,
                x_min=-2.4e-3, x_max=2.4e-3, z_min=4e-3, z_max=12e-3, f_number=1.0)
    base.update(kw)
    return Geometry(**base)


# ----------------------------------------------------------------------- delays
def test_interp_matches_numpy_interp_on_zero_padded_record():
    rng = np.random.default_rng(0)
    u = rng.standard_normal(9)
    padded = np.concatenate([[0.0], u, [0.0]])
    grid = np.arange(-1, len(u) + 1, dtype=np.float64)
    for s in [-3.0, -1.0, -0.75, -0.25, 0.0, 0.5, 3.25, 7.999, 8.0, 8.5, 9.0, 12.0]:
        ref = np.interp(s, grid, padded, left=0.0, right=0.0)
        assert oracle.interp(u, s) == pytest.approx(ref, abs=1e-15)


def test_delay_on_axis_is_round_trip():
    # non-steered, pixel straight below element e: down and back along z
    g = small_geom()
    for e in [0, 5, 15]:
        for z in [1e-3, 7.3e-3, 30e-3]:
            s = oracle.tof_samples(g, 0, e, g.elem_x[e], z)
            assert s == pytest.approx(2 * z * g.fs / g.c, rel=1e-14)


def test_delay_3_4_5_triangle():
    g = small_geom()
    e = 3
    x = g.elem_x[e] + 3e-3
    s = oracle.tof_samples(g, 0, e, x, 4e-3)
    assert s == pytest.approx((4e-3 + 5e-3) * g.fs / g.c, rel=1e-14)
    x = g.elem_x[e] - 3e-3  # the receive path is symmetric in x - x_e
    assert oracle.tof_samples(g, 0, e, x, 4e-3) == pytest.approx(s, rel=1e-14)


@pytest.mark.parametrize("deg", [30.0, -30.0])
def test_delay_steered_wave_reaches_each_element_when_it_fires(deg):
    # A plane wave steered by theta is launched by delaying element e by
    # (x_e - x_first) sin(theta) / c; for a point on the array face at element
    # e the receive path is zero, so the total is exactly that firing delay.
    g = small_geom(angles_deg=(deg,))
    first = g.elem_x[0] if deg > 0 else g.elem_x[-1]
    for e in [0, 7, 15]:
        s = oracle.tof_samples(g, 0, e, g.elem_x[e], 0.0)
        expect = (g.elem_x[e] - first) * math.sin(math.radians(deg)) * g.fs / g.c
        assert s == pytest.approx(expect, abs=1e-12)
        assert s >= -1e-12  # nothing fires before time zero


def test_delay_t0_shifts_sample_index():
    g = small_geom(angles_deg=(0.0, 6.0), t0=(0.0, 1.25e-6))
    s_a = oracle.tof_samples(g.replace(t0=(0.0, 0.0)), 1, 4, 1e-3, 8e-3)
    s_b = oracle.tof_samples(g, 1, 4, 1e-3, 8e-3)
    assert s_a - s_b == pytest.approx(1.25e-6 * g.fs, rel=1e-12)


# ----------------------------------------------------------------- apodization
def test_hann_apodization_points():
    g = small_geom(f_number=1.5)
    e = 6
    z = 9e-3
    a = z / (2 * 1.5)  # half-aperture
    xe = g.elem_x[e]
    assert oracle.apod_weight(g, e, xe, z) == pytest.approx(1.0)
    assert oracle.apod_weight(g, e, xe + a / 2, z) == pytest.approx(0.5, abs=1e-15)
    assert oracle.apod_weight(g, e, xe - a / 2, z) == pytest.approx(0.5, abs=1e-15)
    assert oracle.apod_weight(g, e, xe + a, z) == 0.0
    assert oracle.apod_weight(g, e, xe + 1.01 * a, z) == 0.0
    assert oracle.apod_weight(g, e, xe, 0.0) == 0.0
    assert oracle.apod_weight(g, e, xe, -1e-3) == 0.0
    rng = np.random.default_rng(1)
    for d in rng.uniform(0, a, 20):
        # Hann as a squared cosine over the half-aperture: cos^2(pi d / (2 a))
        assert oracle.apod_weight(g, e, xe + d, z) == pytest.approx(
            math.cos(math.pi * d / (2 * a)) ** 2, abs=1e-14)


def test_boxcar_and_none_apodization():
    g = small_geom(apod="boxcar", f_number=2.0)
    z = 8e-3
    assert oracle.apod_weight(g, 2, g.elem_x[2] + 1.9e-3, z) == 1.0
    assert oracle.apod_weight(g, 2, g.elem_x[2] + 2.1e-3, z) == 0.0
    g = small_geom(apod="none")
    assert oracle.apod_weight(g, 2, 50e-3, -3e-3) == 1.0


# ------------------------------------------------------------- impulse response
@pytest.mark.parametrize("deg", [0.0, 7.0])
def test_impulse_response_is_weighted_triangle_on_isodelay_arc(deg):
    g = small_geom(angles_deg=(deg,), nx=10, nz=200, z_min=2e-3, z_max=14e-3)
    e, nstar = 9, 150
    rf = np.zeros((1, g.n_channels, g.n_samples))
    rf[0, e, nstar] = 1.0
    img = oracle.das(g, rf, 0)
    expect = np.zeros_like(img)
    for ix, x in enumerate(g.x_pix):
        for iz, z in enumerate(g.z_pix):
            s = oracle.tof_samples(g, 0, e, x, z)
            expect[ix, iz] = oracle.apod_weight(g, e, x, z) * max(0.0, 1.0 - abs(s - nstar))
    np.testing.assert_allclose(img, expect, atol=1e-14)
    assert np.count_nonzero(img) > 10  # the arc crosses the grid


# ---------------------------------------------------------------- point target
@pytest.mark.parametrize("deg,ix,iz", [(0.0, 20, 30), (8.0, 13, 41), (-8.0, 29, 22),
                                       (0.0, 3, 50)])
def test_point_scatterer_peaks_at_its_own_pixel(deg, ix, iz):
    # The echo is generated by the independent forward model in synth; the
    # beamformed image of one noise-free scatterer placed on a pixel centre must
    # peak at that pixel.
    g = Geometry(n_channels=48, n_samples=1024, angles_deg=(deg,), nx=40, nz=64,
                 x_min=-6e-3, x_max=6e-3, z_min=8e-3, z_max=14.4e-3, f_number=1.0)
    ph = point_phantom([[g.x_pix[ix], g.z_pix[iz]]], amp=1.0)
    rf = simulate_rf(g, ph, snr_db=None, quantize=False)["master"]
    img = np.abs(oracle.das(g, rf, 0))
    assert np.unravel_index(np.argmax(img), img.shape) == (ix, iz)
    env = oracle.envelope_z(oracle.das(g, rf, 0))
    assert np.unravel_index(np.argmax(env), env.shape) == (ix, iz)


def test_point_scatterer_compound_peaks_at_its_own_pixel():
    g = Geometry(n_channels=48, n_samples=1024, angles_deg=(-10.0, -4.0, 2.0, 10.0), nx=40,
                 nz=64, x_min=-6e-3, x_max=6e-3, z_min=8e-3, z_max=14.4e-3, f_number=1.0)
    ph = point_phantom([[g.x_pix[25], g.z_pix[17]]])
    rf = simulate_rf(g, ph, snr_db=None, quantize=False)["master"]
    for a in range(g.n_angles):
        img = np.abs(oracle.das(g, rf, a))
        assert np.unravel_index(np.argmax(img), img.shape) == (25, 17)
    img = np.abs(oracle.das(g, rf, -1))
    assert np.unravel_index(np.argmax(img), img.shape) == (25, 17)


# ------------------------------------------------------------------ invariants
def _rand_rf(g, seed):
    return np.random.default_rng(seed).standard_normal((g.n_angles, g.n_channels, g.n_samples))


def test_das_is_linear_in_rf():
    g = small_geom(angles_deg=(-5.0, 3.0))
    a, b = _rand_rf(g, 1), _rand_rf(g, 2)
    lhs = oracle.das(g, 2.5 * a - 0.75 * b, -1)
    rhs = 2.5 * oracle.das(g, a, -1) - 0.75 * oracle.das(g, b, -1)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11 * np.abs(rhs).max())


def test_das_channel_superposition():
    g = small_geom(n_channels=6)
    rf = _rand_rf(g, 3)
    total = oracle.das(g, rf, 0)
    parts = np.zeros_like(total)
    for e in range(g.n_channels):
        one = np.zeros_like(rf)
        one[:, e] = rf[:, e]
        parts += oracle.das(g, one, 0)
    np.testing.assert_allclose(total, parts, atol=1e-12 * np.abs(total).max())


def test_compound_is_sum_of_angles():
    g = small_geom(angles_deg=(-10.0, 0.0, 4.0))
    rf = _rand_rf(g, 4)
    per = sum(oracle.das(g.replace(angles_deg=(g.angles_deg[a],)), rf[a:a + 1], 0)
              for a in range(3))
    np.testing.assert_allclose(oracle.das(g, rf, -1), per, atol=1e-12 * np.abs(per).max())
    perd = sum(oracle.dmas(g.replace(angles_deg=(g.angles_deg[a],)), rf[a:a + 1], 0)
               for a in range(3))
    np.testing.assert_allclose(oracle.compound(g, rf, "dmas"), perd,
                               atol=1e-12 * np.abs(perd).max())
    perp = sum(oracle.pdas(g.replace(angles_deg=(g.angles_deg[a],)), rf[a:a + 1], 0, 2.5)
               for a in range(3))
    np.testing.assert_allclose(oracle.compound(g, rf, "pdas", p=2.5), perp,
                               atol=1e-12 * np.abs(perp).max())


@pytest.mark.parametrize("mode", ["das", "dmas", "pdas"])
def test_mirror_symmetry(mode):
    # A symmetric array and grid: mirroring x, the steering angle and the element
    # order mirrors the image along x.
    g = small_geom(angles_deg=(6.0,), x_min=-2.4e-3, x_max=2.4e-3)
    gm = g.replace(angles_deg=(-6.0,))
    rf = _rand_rf(g, 5)
    rfm = rf[:, ::-1, :]
    f = {"das": oracle.das, "dmas": oracle.dmas, "pdas": oracle.pdas}[mode]
    img = f(g, rf, 0)
    imgm = f(gm, rfm, 0)
    np.testing.assert_allclose(imgm[::-1, :], img, atol=1e-11 * np.abs(img).max())


# ------------------------------------------------------------------------ DMAS
@pytest.mark.parametrize("apod,deg", [("hann", 0.0), ("none", 5.0), ("boxcar", -3.0)])
def test_dmas_pairs_equal_identity(apod, deg):
    g = small_geom(apod=apod, angles_deg=(deg,), n_channels=24)
    rf = _rand_rf(g, 6)
    p = oracle.dmas(g, rf, 0, "pairs")
    i = oracle.dmas(g, rf, 0, "identity")
    np.testing.assert_allclose(i, p, atol=1e-11 * np.abs(p).max())


def test_dmas_of_equal_signals():
    # every delayed sample equal to u (w = 1): each of the N(N-1)/2 pairs gives |u|
    g = small_geom(apod="none", n_channels=10, n_samples=2048)
    u = -3.7
    rf = np.full((1, g.n_channels, g.n_samples), u)
    img = oracle.dmas(g, rf, 0)
    n = g.n_channels
    np.testing.assert_allclose(img, n * (n - 1) / 2 * abs(u), rtol=1e-13)


def test_dmas_two_channels_closed_form():
    # N = 2: y = w1 w2 sign(v1 v2) sqrt|v1 v2|; the weight stays outside the root
    g = small_geom(n_channels=2, f_number=0.6, x_min=-1.2e-3, x_max=1.2e-3)
    rf = _rand_rf(g, 7)
    gn = g.replace(apod="none")
    v = []
    for e in range(2):
        one = np.zeros_like(rf)
        one[:, e] = rf[:, e]
        v.append(oracle.das(gn, one, 0))
    w = np.zeros((2, g.nx, g.nz))
    for e in range(2):
        for ix, x in enumerate(g.x_pix):
            for iz, z in enumerate(g.z_pix):
                w[e, ix, iz] = oracle.apod_weight(g, e, x, z)
    expect = w[0] * w[1] * np.sign(v[0] * v[1]) * np.sqrt(np.abs(v[0] * v[1]))
    assert np.count_nonzero(w[0] * w[1]) > 10
    np.testing.assert_allclose(oracle.dmas(g, rf, 0), expect, atol=1e-13)


# ------------------------------------------------------------------------ pDAS
@pytest.mark.parametrize("apod,deg", [("hann", 0.0), ("boxcar", 6.0), ("none", -4.0)])
def test_pdas_with_p_one_is_das(apod, deg):
    g = small_geom(apod=apod, angles_deg=(deg, -2.0))
    rf = _rand_rf(g, 21)
    ref = oracle.das(g, rf, -1)
    np.testing.assert_allclose(oracle.pdas(g, rf, -1, 1.0), ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("p", [1.5, 2.0, 3.0])
def test_pdas_single_channel_closed_form(p):
    # one element: sign(w sign(v)|v|^(1/p)) |w |v|^(1/p)|^p = w^p v = w^(p-1) * DAS
    g = small_geom(n_channels=1, x_min=-1.5e-3, x_max=1.5e-3, f_number=2.0)
    rf = _rand_rf(g, 22)
    das = oracle.das(g, rf, 0)
    w = np.array([[oracle.apod_weight(g, 0, x, z) for z in g.z_pix] for x in g.x_pix])
    assert 0 < np.count_nonzero(w) < w.size  # inside and outside the aperture
    np.testing.assert_allclose(oracle.pdas(g, rf, 0, p), w ** (p - 1) * das,
                               atol=1e-12 * np.abs(das).max())


def test_pdas_is_odd_and_homogeneous_of_degree_one():
    g = small_geom(angles_deg=(3.0,), n_channels=12)
    rf = _rand_rf(g, 23)
    base = oracle.pdas(g, rf, 0, 2.7)
    np.testing.assert_allclose(oracle.pdas(g, 3.25 * rf, 0, 2.7), 3.25 * base,
                               atol=1e-11 * np.abs(base).max())
    np.testing.assert_allclose(oracle.pdas(g, -rf, 0, 2.7), -base, atol=1e-13 * np.abs(base).max())


def test_pdas_of_equal_signals():
    # every delayed sample equal to u (w = 1): y = sign(u) |u| N^p
    g = small_geom(apod="none", n_channels=7, n_samples=2048)
    u, p = -2.3, 3.0
    rf = np.full((1, g.n_channels, g.n_samples), u)
    np.testing.assert_allclose(oracle.pdas(g, rf, 0, p), -abs(u) * g.n_channels ** p,
                               rtol=1e-13)


def test_pdas_p2_is_twice_dmas_plus_das_for_boxcar_positive_data():
    # w in {0, 1} and v >= 0: (sum w sqrt v)^2 = 2 sum_{i<j} s_i s_j + sum w v
    g = small_geom(apod="boxcar", angles_deg=(-4.0,), n_channels=20)
    rf = np.abs(_rand_rf(g, 24))
    lhs = oracle.pdas(g, rf, 0, 2.0)
    rhs = 2.0 * oracle.dmas(g, rf, 0) + oracle.das(g, rf, 0)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(rhs).max())


# ------------------------------------------------------------ IQ-DAS, BB-DMAS
def test_iq_das_without_demodulation_is_das_of_the_analytic_signal():
    # fd = 0: the baseband record is the analytic signal itself, so IQ-DAS is the
    # DAS of the record plus i times the DAS of its Hilbert transform (scipy's)
    from scipy.signal import hilbert
    g = small_geom(angles_deg=(-3.0, 5.0), n_samples=512)
    rf = _rand_rf(g, 31)
    iq = oracle.iq_demodulate(g, rf, fd=0.0)
    y = oracle.iq_beamform(g, iq, "iqdas", -1, fd=0.0)
    ref = oracle.das(g, rf, -1) + 1j * oracle.das(g, np.imag(hilbert(rf, axis=-1)), -1)
    np.testing.assert_allclose(y, ref, atol=1e-11 * np.abs(ref).max())


def _tone(g, k, theta):
    n = np.arange(g.n_samples)
    u = np.cos(2 * np.pi * k * n / g.n_samples + theta)
    return np.broadcast_to(u, (g.n_angles, g.n_channels, g.n_samples)).copy()


def test_iq_demodulation_of_an_integer_bin_tone_is_constant():
    g = small_geom(n_samples=512)
    k, theta = 128, 0.7  # fd = k fs / Ns = fs / 4
    iq = oracle.iq_demodulate(g, _tone(g, k, theta), fd=k * g.fs / g.n_samples)
    np.testing.assert_allclose(iq, np.exp(1j * theta), atol=1e-12)


def _tone_sums(g, fd, theta):
    """sum_e w_e exp(i (2 pi fd s_e / fs + theta)) per pixel, from the pinned delay
    and weight functions."""
    out = np.zeros((g.nx, g.nz), dtype=complex)
    for ix, x in enumerate(g.x_pix):
        for iz, z in enumerate(g.z_pix):
            for e in range(g.n_channels):
                s = oracle.tof_samples(g, 0, e, x, z)
                assert 1.0 < s < g.n_samples - 2
                out[ix, iz] += oracle.apod_weight(g, e, x, z) * np.exp(
                    1j * (2 * np.pi * fd * s / g.fs + theta))
    return out


def test_iq_das_and_bb_dmas_of_a_tone_in_closed_form():
    g = small_geom(angles_deg=(4.0,), n_samples=512, nx=6, nz=7, n_channels=9)
    k, theta = 128, -1.1
    fd = k * g.fs / g.n_samples
    iq = oracle.iq_demodulate(g, _tone(g, k, theta), fd=fd)
    sums = _tone_sums(g, fd, theta)
    np.testing.assert_allclose(oracle.iq_beamform(g, iq, "iqdas", 0, fd=fd), sums, atol=1e-9)
    # |q| = 1 everywhere, so the square root leaves every sample unchanged
    np.testing.assert_allclose(oracle.iq_beamform(g, iq, "bbdmas", 0, fd=fd), sums ** 2,
                               atol=1e-8)


def test_bb_dmas_single_channel_closed_form():
    # one element: (w sqrt(a) e^{i phi})^2 = w^2 a e^{2 i phi} = w y_iqdas^2 / |y_iqdas|
    g = small_geom(n_channels=1, x_min=-1.5e-3, x_max=1.5e-3, f_number=2.0, n_samples=512)
    rf = _rand_rf(g, 32)
    iq = oracle.iq_demodulate(g, rf)
    y1 = oracle.iq_beamform(g, iq, "iqdas", 0)
    yb = oracle.iq_beamform(g, iq, "bbdmas", 0)
    w = np.array([[oracle.apod_weight(g, 0, x, z) for z in g.z_pix] for x in g.x_pix])
    assert 0 < np.count_nonzero(w) < w.size
    expect = np.where(np.abs(y1) > 0, w * y1 ** 2 / np.where(y1 == 0, 1, np.abs(y1)), 0)
    np.testing.assert_allclose(yb, expect, atol=1e-12 * np.abs(expect).max())


def test_iq_compound_is_sum_of_angles():
    g = small_geom(angles_deg=(-8.0, 1.0, 6.0), n_samples=512)
    rf = _rand_rf(g, 33)
    iq = oracle.iq_demodulate(g, rf)
    for form in ("iqdas", "bbdmas"):
        per = sum(oracle.iq_beamform(g, iq, form, a) for a in range(3))
        np.testing.assert_allclose(oracle.iq_beamform(g, iq, form, -1), per,
                                   atol=1e-12 * np.abs(per).max())


# ------------------------------------------------------------ IQ decimation
def test_decimation_by_one_is_the_full_rate_demodulation():
    g = small_geom(n_samples=512)
    rf = _rand_rf(g, 41)
    assert np.array_equal(oracle.iq_demodulate(g, rf, decimation=1), oracle.iq_demodulate(g, rf))


@pytest.mark.parametrize("D", [2, 4, 8])
def test_decimated_demodulation_of_an_in_band_tone(D):
    # a tone on bin k within fs / (2 D) of fd (fd off the bin grid): the band
    # limit keeps it whole, so sample m of the decimated record is the baseband
    # exponential at the original sample m D
    g = small_geom(n_samples=512)
    fd = 0.21 * g.fs
    k = int(round(fd * g.n_samples / g.fs)) + 3
    assert abs(k * g.fs / g.n_samples - fd) < g.fs / (2 * D)
    theta = 0.4
    q = oracle.iq_demodulate(g, _tone(g, k, theta), fd=fd, decimation=D)
    assert q.shape[-1] == g.n_samples // D
    n = np.arange(0, g.n_samples, D)
    expect = np.exp(1j * (2 * np.pi * (k / g.n_samples - fd / g.fs) * n + theta))
    np.testing.assert_allclose(q, np.broadcast_to(expect, q.shape), atol=1e-12)


@pytest.mark.parametrize("D", [2, 4, 8])
def test_decimated_demodulation_removes_an_out_of_band_tone(D):
    g = small_geom(n_samples=512)
    fd = 0.21 * g.fs
    k = int(np.ceil((fd + g.fs / (2 * D)) * g.n_samples / g.fs)) + 1  # just past the band
    q = oracle.iq_demodulate(g, _tone(g, k, 1.3), fd=fd, decimation=D)
    assert np.abs(q).max() < 1e-12
    # ... and the bins kept are exactly the positive ones within the band
    keep = oracle.band_keep(g.n_samples, g.fs, fd, D)
    f = np.arange(g.n_samples) * g.fs / g.n_samples
    assert keep.sum() > 0 and np.all(np.abs(f[keep] - fd) < g.fs / (2 * D))
    assert np.all(np.nonzero(keep)[0] <= g.n_samples // 2)


def test_decimated_iq_das_of_a_tone_at_fd_in_closed_form():
    # a tone at fd has a constant baseband record, decimated or not; the
    # beamformer reads it at its own rate and rotates by the delay's time, so the
    # image is the same closed-form phasor sum as at the full rate
    g = small_geom(angles_deg=(4.0,), n_samples=512, nx=6, nz=7, n_channels=9)
    k, theta = 128, -1.1
    fd = k * g.fs / g.n_samples
    sums = _tone_sums(g, fd, theta)
    for D in (2, 4):
        iq = oracle.iq_demodulate(g, _tone(g, k, theta), fd=fd, decimation=D)
        np.testing.assert_allclose(oracle.iq_beamform(g, iq, "iqdas", 0, fd=fd, decimation=D),
                                   sums, atol=1e-9)


def test_decimated_iq_das_reads_the_record_at_its_own_rate():
    # a tone slightly off fd: its baseband record turns slowly, and the decimated
    # IQ-DAS may differ from the full-rate one only by the linear interpolation
    # error at the two rates, |q''| h^2 / 8 per sample with h = D or 1 samples
    # (reading the decimated record at s instead of s / D would be far off)
    g = small_geom(angles_deg=(-3.0,), n_samples=512, nx=6, nz=9, n_channels=12)
    k, theta = 126, 0.3
    fd = 128 * g.fs / g.n_samples
    w_sum = max(sum(oracle.apod_weight(g, e, x, z) for e in range(g.n_channels))
                for x in g.x_pix for z in g.z_pix)
    y1 = oracle.iq_beamform(g, oracle.iq_demodulate(g, _tone(g, k, theta), fd=fd), "iqdas", 0,
                            fd=fd)
    for D in (2, 4):
        iq = oracle.iq_demodulate(g, _tone(g, k, theta), fd=fd, decimation=D)
        yD = oracle.iq_beamform(g, iq, "iqdas", 0, fd=fd, decimation=D)
        dphi = 2 * np.pi * abs(k / g.n_samples - fd / g.fs)  # baseband radians per sample
        bound = (dphi ** 2 / 8) * (D ** 2 + 1) * w_sum
        assert np.abs(yD - y1).max() <= 1.01 * bound
        assert np.abs(y1).max() > 100 * bound  # the check is not vacuous


# ------------------------------------------------------------ brute force 4x4
def brute_das_dmas(g, rf, p=2.5):
    """Independent evaluation: numpy.interp on a zero-padded record, Hann as a
    squared cosine, angle-outer loop order; returns DAS, DMAS (pair sum) and
    pDAS of order p."""
    A, N, Ns = rf.shape
    das = np.zeros((g.nx, g.nz))
    dmas = np.zeros((g.nx, g.nz))
    pdas = np.zeros((g.nx, g.nz))
    grid = np.arange(-1, Ns + 1, dtype=np.float64)
    for a in range(A):
        th = math.radians(g.angles_deg[a])
        fire = g.elem_x * math.sin(th)
        fire = fire - fire.min()  # firing delay of each element, in metres of path
        for ix in range(g.nx):
            x = g.x_min + (ix + 0.5) * (g.x_max - g.x_min) / g.nx
            for iz in range(g.nz):
                z = g.z_min + (iz + 0.5) * (g.z_max - g.z_min) / g.nz
                # transmit path measured from the first-firing element's wavefront
                path_tx = x * math.sin(th) + z * math.cos(th) - (g.elem_x * math.sin(th)).min()
                sh = []
                root_sum = 0.0
                for e in range(N):
                    path_rx = math.hypot(x - g.elem_x[e], z)
                    s = (path_tx + path_rx) / g.c * g.fs - g.t0_s[a] * g.fs
                    padded = np.concatenate([[0.0], rf[a, e], [0.0]])
                    v = float(np.interp(s, grid, padded, left=0.0, right=0.0))
                    half = z / (2 * g.f_number)
                    d = abs(x - g.elem_x[e])
                    w = math.cos(math.pi * d / (2 * half)) ** 2 if (z > 0 and d < half) else 0.0
                    das[ix, iz] += w * v
                    sh.append(w * math.copysign(math.sqrt(abs(v)), v) if v != 0 else 0.0)
                    root_sum += w * math.copysign(abs(v) ** (1.0 / p), v) if v != 0 else 0.0
                for i in range(N):
                    for j in range(i + 1, N):
                        dmas[ix, iz] += sh[i] * sh[j]
                pdas[ix, iz] += math.copysign(abs(root_sum) ** p, root_sum)
    return das, dmas, pdas


def brute_iq(g, rf, fd):
    """Independent IQ path: scipy's analytic signal, numpy.interp on the real and
    imaginary parts of the zero-padded baseband record, cmath rotation, Hann as a
    squared cosine; returns IQ-DAS and BB-DMAS (compound sums)."""
    import cmath
    from scipy.signal import hilbert
    A, N, Ns = rf.shape
    n = np.arange(Ns)
    iq = hilbert(rf, axis=-1) * np.exp(-2j * np.pi * fd * n / g.fs)
    grid = np.arange(-1, Ns + 1, dtype=np.float64)
    yd = np.zeros((g.nx, g.nz), dtype=complex)
    yb = np.zeros((g.nx, g.nz), dtype=complex)
    for a in range(A):
        th = math.radians(g.angles_deg[a])
        for ix in range(g.nx):
            x = g.x_min + (ix + 0.5) * (g.x_max - g.x_min) / g.nx
            for iz in range(g.nz):
                z = g.z_min + (iz + 0.5) * (g.z_max - g.z_min) / g.nz
                path_tx = x * math.sin(th) + z * math.cos(th) - (g.elem_x * math.sin(th)).min()
                sd, sb = 0j, 0j
                for e in range(N):
                    s = (path_tx + math.hypot(x - g.elem_x[e], z)) / g.c * g.fs - g.t0_s[a] * g.fs
                    re = float(np.interp(s, grid, np.concatenate([[0.0], iq[a, e].real, [0.0]])))
                    im = float(np.interp(s, grid, np.concatenate([[0.0], iq[a, e].imag, [0.0]])))
                    v = complex(re, im) * cmath.exp(2j * math.pi * fd * s / g.fs)
                    half = z / (2 * g.f_number)
                    d = abs(x - g.elem_x[e])
                    w = math.cos(math.pi * d / (2 * half)) ** 2 if (z > 0 and d < half) else 0.0
                    sd += w * v
                    sb += w * (math.sqrt(abs(v)) * cmath.exp(1j * cmath.phase(v)) if v != 0 else 0)
                yd[ix, iz] += sd
                yb[ix, iz] += sb * sb
    return yd, yb


@pytest.mark.parametrize("seed,angles", [(11, (0.0,)), (12, (-9.0, 3.0, 10.0))])
def test_brute_force_4x4(seed, angles):
    g = Geometry(n_channels=8, n_samples=400, angles_deg=angles, nx=4, nz=4, x_min=-1e-3,
                 x_max=1.4e-3, z_min=5e-3, z_max=6.2e-3, f_number=0.8, t0=(0.3e-6,) * len(angles))
    rf = _rand_rf(g, seed)
    bd, bm, bp = brute_das_dmas(g, rf, 2.5)
    np.testing.assert_allclose(oracle.das(g, rf, -1), bd, atol=1e-12 * np.abs(bd).max())
    np.testing.assert_allclose(oracle.compound(g, rf, "dmas"), bm, atol=1e-12 * np.abs(bm).max())
    np.testing.assert_allclose(oracle.compound(g, rf, "pdas", p=2.5), bp,
                               atol=1e-12 * np.abs(bp).max())
    assert np.abs(bd).max() > 0 and np.abs(bm).max() > 0 and np.abs(bp).max() > 0
    g2 = g.replace(n_samples=512)
    rf2 = _rand_rf(g2, seed + 100)
    yd, yb = brute_iq(g2, rf2, g2.f0)
    iq = oracle.iq_demodulate(g2, rf2)
    np.testing.assert_allclose(oracle.iq_beamform(g2, iq, "iqdas", -1), yd,
                               atol=1e-10 * np.abs(yd).max())
    np.testing.assert_allclose(oracle.iq_beamform(g2, iq, "bbdmas", -1), yb,
                               atol=1e-10 * np.abs(yb).max())


# ------------------------------------------------------------- post-processing
@pytest.mark.parametrize("nz", [16, 64, 256, 1024])
def test_envelope_of_integer_bin_tone_is_one(nz):
    n = np.arange(nz)
    cols = np.stack([np.cos(2 * np.pi * k * n / nz + ph) for k, ph in
                     [(1, 0.0), (3, 0.4), (nz // 4, 1.0), (nz // 2 - 1, -0.3)]])
    np.testing.assert_allclose(oracle.envelope_z(cols), 1.0, atol=1e-12)


def test_envelope_of_am_tone():
    # Bedrosian: a slow modulation times a faster carrier keeps its modulation as envelope
    nz = 512
    n = np.arange(nz)
    m = 1.0 + 0.5 * np.cos(2 * np.pi * 3 * n / nz)
    col = m * np.cos(2 * np.pi * 40 * n / nz + 0.2)
    np.testing.assert_allclose(oracle.envelope_z(col[None])[0], m, atol=1e-12)


def test_bandpass_keeps_band_and_removes_rest():
    nz, dz, c, f0 = 512, 25e-6, 1540.0, 5e6
    n = np.arange(nz)
    fbin = c / (2 * nz * dz)  # round-trip frequency of one bin
    k_in = int(round(2 * f0 / fbin))  # 2 f0, in band
    k_lo = int(math.floor(0.5 * f0 / fbin))  # below f0
    k_hi = int(math.ceil(3.0 * f0 / fbin)) + 2  # just above 3 f0
    assert k_hi < nz // 2
    tone_in = np.cos(2 * np.pi * k_in * n / nz + 0.3)
    out = oracle.bandpass_z((tone_in + 0.7 * np.cos(2 * np.pi * k_lo * n / nz)
                             + 0.2 * np.sin(2 * np.pi * k_hi * n / nz) + 1.5)[None], dz, c, f0)
    np.testing.assert_allclose(out[0], tone_in, atol=1e-12)
    # the edges of the band are inclusive
    mask = oracle.band_bins(nz, dz, c, f0)
    k = np.arange(nz // 2)
    f = k * fbin
    np.testing.assert_array_equal(mask[:nz // 2], (f >= f0) & (f <= 3 * f0))


def test_log_compress():
    env = np.array([[0.0, 1e-5, 1e-3, 0.1, 2.0], [1.0, 0.5, 2e-4, 2.0, 1.999]])
    out = oracle.log_compress(env, -70.0)
    assert out[0, 4] == 0.0 and out[1, 3] == 0.0
    assert out[0, 0] == -70.0 and out[0, 1] == -70.0
    assert out[0, 2] == pytest.approx(20 * math.log10(1e-3 / 2))
    assert out[1, 1] == pytest.approx(-20 * math.log10(4))
    np.testing.assert_array_equal(oracle.log_compress(np.zeros((3, 4))), -70.0)
    assert oracle.log_compress(env, -40.0).min() == -40.0


def test_openmp_build_gives_the_single_threaded_values_bitwise():
    # the same source built with -fopenmp shares the pixel loop among threads;
    # each pixel is still one thread's literal evaluation, so nothing may change
    g = small_geom(angles_deg=(-6.0, 0.0, 9.0), nx=19, nz=23)
    rng = np.random.default_rng(5)
    rf = rng.standard_normal((g.n_angles, g.n_channels, g.n_samples))
    pix = rng.choice(g.nx * g.nz, 57, replace=False)
    for fn in (lambda **k: oracle.das(g, rf, -1, **k),
               lambda **k: oracle.das(g, rf, 1, pix=pix, **k),
               lambda **k: oracle.dmas(g, rf, -1, "identity", **k),
               lambda **k: oracle.dmas(g, rf, 0, "pairs", pix=pix, **k),
               lambda **k: oracle.pdas(g, rf, -1, 2.5, **k)):
        assert np.array_equal(fn(), fn(parallel=True))
    iq = oracle.iq_demodulate(g, rf)
    for form in ("iqdas", "bbdmas"):
        assert np.array_equal(oracle.iq_beamform(g, iq, form, -1),
                              oracle.iq_beamform(g, iq, form, -1, parallel=True))


def test_dmas_float32_delay_floor_on_incoherent_content():
    # The root of DMAS is steep at near-zero delayed samples, and incoherent
    # content (uniform noise) puts some of its 16.7 M gathers next to zero while
    # its image maximum stays near the incoherent level. Shifting every delay
    # of a 1024 x 256, 64-channel frame by 3e-8 samples (below the resolution of
    # a float32 delay of even one sample) then moves the float64 definition by
    # more than 1e-5 (max-normalised): no float32-delay beamformer meets that
    # bar on such content, which is why the root modes' parity is stated on
    # simulated phantom frames. Their coherent targets move by under 1e-6.
    import dataclasses
    from synth import config_c4_frames, make_frame
    g = config_c4_frames()[21].geom
    shifted = dataclasses.replace(g, t0=(3e-8 / g.fs,))
    rng = np.random.default_rng(2)
    noise = rng.integers(-511, 512, (g.n_angles, g.n_channels, g.n_samples)).astype(np.int16)
    phantom = make_frame(g, config_c4_frames()[21].seed, "scaled")["i16"]
    for rf, lo, hi in ((noise, 1e-5, np.inf), (phantom, 0.0, 1e-6)):
        ref = oracle.dmas(g, rf, -1, "identity", parallel=True)
        moved = oracle.dmas(shifted, rf, -1, "identity", parallel=True)
        e = np.abs(moved - ref).max() / np.abs(ref).max()
        assert lo < e < hi, e
