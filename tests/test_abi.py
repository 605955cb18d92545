"""The C ABI on the CPU: the library loads, exports every declared symbol, and
rejects invalid arguments on the host before any HIP call.

Argument checks go through pwbf_validate_call, which runs every host-side check
of the beamforming entry points and never enqueues work, so the fake device
addresses below are never used. The real entry points are only called with
arguments that fail their very first check.
"""

import ctypes
import os
import re
import threading

import numpy as np
import pytest

from paper_2311_00482_amd import _abi
from paper_2311_00482_amd.api import GeometryArg, Tile, describe_plan
from synth import config_c1, config_c2, config_c3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x10000  # an aligned address that validation accepts but is never used


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"PWBF_API\s+[\w\s\*]+?\b(pwbf_\w+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    names = declared_symbols()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), n
    assert L.pwbf_abi_version() == _abi.ABI_VERSION


def _call(g, rf=FAKE, dtype=_abi.I16, mode=_abi.DAS, angle=-1, tile=None, out=None, ws=None,
          ws_bytes=0):
    if out is None:
        out = _abi.Outputs(FAKE, None, None, None)
    L = _abi.lib()
    t = ctypes.byref(tile) if tile is not None else None
    o = ctypes.byref(out) if out is not False else None
    gref = g.ref if g is not None else None
    rc = L.pwbf_validate_call(gref, rf, dtype, mode, angle, t, o, ws, ws_bytes)
    return rc, L.pwbf_last_error().decode()


def test_entry_points_reject_null_geometry_first():
    L = _abi.lib()
    o = ctypes.byref(_abi.Outputs(FAKE, None, None, None))
    assert L.pwbf_beamform_das(None, FAKE, 0, 0, o, None, 0, None) == _abi.E_INVALID
    assert L.pwbf_beamform_dmas(None, FAKE, 0, 0, o, None, 0, None) == _abi.E_INVALID
    assert L.pwbf_beamform_pdas(None, FAKE, 0, 0, o, None, 0, None) == _abi.E_INVALID
    assert L.pwbf_compound(None, FAKE, 0, 0, o, None, 0, None) == _abi.E_INVALID
    assert L.pwbf_beamform_ex(None, FAKE, 0, 0, -1, None, o, None, 0, None) == _abi.E_INVALID
    assert "NULL" in L.pwbf_last_error().decode()


def test_valid_call_passes_validation():
    assert _call(GeometryArg(config_c1()), angle=0) == (0, "")


def test_null_and_version_errors():
    assert _call(None)[0] == _abi.E_INVALID
    g = GeometryArg(config_c1())
    g.s.abi_version = 99
    rc, msg = _call(g)
    assert rc == _abi.E_INVALID and "abi_version" in msg


@pytest.mark.parametrize("field,value,code", [
    ("n_angles", 0, _abi.E_INVALID), ("n_angles", 33, _abi.E_UNSUPPORTED),
    ("n_channels", 0, _abi.E_INVALID), ("n_channels", 257, _abi.E_UNSUPPORTED),
    ("n_samples", 1, _abi.E_INVALID), ("c", 0.0, _abi.E_INVALID), ("fs", -1.0, _abi.E_INVALID),
    ("nx", 0, _abi.E_INVALID), ("dz", 0.0, _abi.E_INVALID), ("dx", float("nan"), _abi.E_INVALID),
    ("apod", 7, _abi.E_INVALID), ("f_number", 0.0, _abi.E_INVALID),
    ("log_floor_db", 3.0, _abi.E_INVALID), ("bandpass", 2, _abi.E_INVALID),
])
def test_geometry_validation(field, value, code):
    g = GeometryArg(config_c1())
    setattr(g.s, field, value)
    rc, msg = _call(g)
    assert rc == code, msg
    assert msg


def test_far_field_rejected_for_float32_delays():
    g = GeometryArg(config_c1())
    g.s.z0 = 50.0  # 50 m deep: delays beyond what float32 resolves
    assert _call(g)[0] == _abi.E_UNSUPPORTED


def test_angle_validation():
    g = config_c1()
    ga = GeometryArg(g.replace(angles_deg=(0.0, 95.0)))
    assert _call(ga)[0] == _abi.E_INVALID
    ga = GeometryArg(g)
    assert _call(ga, angle=1)[0] == _abi.E_INVALID
    assert _call(ga, angle=-2)[0] == _abi.E_INVALID
    L = _abi.lib()
    o = _abi.Outputs(FAKE, None, None, None)
    # the single-angle entry point rejects a negative angle before anything else
    assert L.pwbf_beamform_das(ga.ref, FAKE, 0, -1, ctypes.byref(o), None, 0, None) == \
        _abi.E_INVALID


def test_call_argument_validation():
    g = GeometryArg(config_c1())
    assert _call(g, rf=None)[0] == _abi.E_INVALID
    assert _call(g, rf=FAKE + 1)[0] == _abi.E_INVALID  # int16 needs 2-byte alignment
    assert _call(g, rf=FAKE + 2, dtype=_abi.F32)[0] == _abi.E_INVALID
    assert _call(g, dtype=9)[0] == _abi.E_INVALID
    assert _call(g, mode=3)[0] == _abi.E_INVALID
    assert _call(g, out=False)[0] == _abi.E_INVALID
    assert _call(g, out=_abi.Outputs(None, None, None, None))[0] == _abi.E_INVALID
    assert _call(g, out=_abi.Outputs(FAKE + 2, None, None, None))[0] == _abi.E_INVALID
    rc, msg = _call(g, out=_abi.Outputs(FAKE, FAKE, None, None))
    assert rc == _abi.E_INVALID and "bandpass" in msg
    one = GeometryArg(config_c1().replace(n_channels=1))
    assert _call(one, mode=_abi.DMAS)[0] == _abi.E_INVALID


@pytest.mark.parametrize("p,code", [(1.0, 0), (1.5, 0), (2.0, 0), (2.01, -2), (3.0, -2),
                                    (16.0, -2), (0.99, -1), (0.0, -1), (float("nan"), -1),
                                    (float("inf"), -1)])
def test_pdas_root_order_validation(p, code):
    g = GeometryArg(config_c1(), pdas_p=p)
    rc, msg = _call(g, mode=_abi.PDAS)
    assert rc == code, msg
    if code:
        assert "pdas_p" in msg
    # other modes ignore the field
    assert _call(g, mode=_abi.DAS)[0] == 0


def test_post_processing_shape_rules():
    g = GeometryArg(config_c1().replace(nz=250))
    assert _call(g, out=_abi.Outputs(FAKE, None, FAKE, None))[0] == _abi.E_UNSUPPORTED
    g = GeometryArg(config_c1().replace(nz=8192, z_max=80e-3))
    assert _call(g, out=_abi.Outputs(FAKE, None, FAKE, None))[0] == _abi.E_UNSUPPORTED
    # band-pass needs dz <= c / (12 f0): C1's 156 um grid is too coarse, C2's 25 um is fine
    g = GeometryArg(config_c1(), bandpass=True)
    rc, msg = _call(g)
    assert rc == _abi.E_UNSUPPORTED and "c / (12 f0)" in msg


def test_workspace_rules():
    L = _abi.lib()
    g = GeometryArg(config_c1())
    assert L.pwbf_workspace_bytes(g.ref, ctypes.byref(_abi.Outputs(FAKE, None, None, None))) == 0
    assert L.pwbf_workspace_bytes(g.ref, ctypes.byref(_abi.Outputs(FAKE, None, FAKE, None))) == 0
    # the frame maximum's 64 slots, one 128-byte line each
    assert L.pwbf_workspace_bytes(g.ref, ctypes.byref(_abi.Outputs(FAKE, None, FAKE, FAKE))) == 8192
    n = L.pwbf_workspace_bytes(g.ref, ctypes.byref(_abi.Outputs(FAKE, None, None, FAKE)))
    assert n == 8192 + 128 * 256 * 4
    log = _abi.Outputs(FAKE, None, FAKE, FAKE)
    assert _call(g, out=log)[0] == _abi.E_INVALID  # no workspace
    assert _call(g, out=log, ws=FAKE, ws_bytes=255)[0] == _abi.E_INVALID
    assert _call(g, out=log, ws=FAKE + 64, ws_bytes=4096)[0] == _abi.E_INVALID  # alignment
    g.s.nx = 0
    assert L.pwbf_workspace_bytes(g.ref, ctypes.byref(log)) == 0
    assert L.pwbf_last_error().decode()


@pytest.mark.parametrize("tile,code", [
    (Tile(cpw=3), _abi.E_INVALID), (Tile(cpw=1, wz=3, wx=3), _abi.E_INVALID),
    (Tile(cpw=2, wz=1, wx=1, chunk=3), _abi.E_INVALID),
    (Tile(cpw=2, lz=64, wz=1, wx=1), _abi.E_INVALID), (Tile(cpw=1, lz=12), _abi.E_INVALID),
    (Tile(cpw=1, wz=1, wx=8, chunk=256), _abi.E_UNSUPPORTED),
])
def test_tile_validation(tile, code):
    g = GeometryArg(config_c3())
    assert _call(g, tile=tile.c())[0] == code


def test_last_error_is_thread_local():
    g = GeometryArg(config_c1())
    g.s.n_samples = 1
    _call(g)
    main_msg = _abi.lib().pwbf_last_error().decode()
    seen = []

    def worker():
        seen.append(_abi.lib().pwbf_last_error().decode())

    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert main_msg and seen == [""]


def test_describe_plan_default_shapes():
    p = describe_plan(config_c3())
    assert p["n_angles_used"] == 11 and p["cpw"] == 1
    assert p["threads_per_block"] == 64 * p["wz"] * p["wx"]
    assert p["blocks"] == p["tiles_z"] * p["tiles_x"]
    assert p["lds_bytes"] <= 64 * 1024
    assert p["chunk"] * 1 >= 1
    p1 = describe_plan(config_c1(), angle=0)
    assert p1["n_angles_used"] == 1
    sc = 20e6 / 1540.0
    g = config_c1()
    assert p1["X0"] == pytest.approx(g.x0 * sc, rel=1e-6)
    assert p1["DZ"] == pytest.approx(g.dz * sc, rel=1e-6)
    np.testing.assert_allclose(p1["xe"][:64], (g.elem_x * sc).astype(np.float32))
    assert p1["xe"][200] == p1["xe"][63]
    p2 = describe_plan(config_c2(), "dmas", bandpass=True)
    assert p2["n_angles_used"] == 1


# ------------------------------------------------------------------- batches
def _frame(g, rf=FAKE, dtype=_abi.I16, mode=_abi.DAS, angle=-1, tile=None, reserved=0):
    t = tile.c() if tile is not None else _abi.Tile()
    return _abi.Frame(ctypes.pointer(g.s), rf, dtype, mode, angle, reserved,
                      _abi.Outputs(FAKE, None, None, None), t)


def _create(frames, flags=0):
    arr = (_abi.Frame * max(1, len(frames)))(*frames)
    h = ctypes.c_void_p()
    rc = _abi.lib().pwbf_batch_create(arr, len(frames), flags, None, ctypes.byref(h))
    return rc, _abi.lib().pwbf_last_error().decode()


def test_iq_mode_and_dtype_rules():
    g = GeometryArg(config_c1())
    C = _abi.C32
    assert _call(g, dtype=C, mode=_abi.IQDAS) == (0, "")
    assert _call(g, dtype=C, mode=_abi.BBDMAS, angle=0) == (0, "")
    for mode, dtype in ((_abi.IQDAS, _abi.F32), (_abi.BBDMAS, _abi.I16), (_abi.DAS, C),
                        (_abi.PDAS, C)):
        rc, msg = _call(g, dtype=dtype, mode=mode)
        assert rc == _abi.E_INVALID and "IQ" in msg
    assert _call(g, dtype=C, mode=5)[0] == _abi.E_INVALID
    assert _call(g, rf=FAKE + 4, dtype=C, mode=_abi.IQDAS)[0] == _abi.E_INVALID  # 8-byte samples
    # the complex image: imag only in the IQ modes, no band-pass there
    assert _call(g, dtype=C, mode=_abi.IQDAS, out=_abi.Outputs(FAKE, None, FAKE, None, FAKE)) \
        == (0, "")
    rc, msg = _call(g, out=_abi.Outputs(FAKE, None, None, None, FAKE))
    assert rc == _abi.E_INVALID and "imag" in msg
    g2 = GeometryArg(config_c2(), bandpass=True)
    rc, msg = _call(g2, dtype=C, mode=_abi.IQDAS)
    assert rc == _abi.E_INVALID and "band-pass" in msg
    # |image| needs no depth FFT: any nz
    g3 = GeometryArg(config_c1().replace(nz=250))
    assert _call(g3, dtype=C, mode=_abi.IQDAS, out=_abi.Outputs(FAKE, None, FAKE, None)) == (0, "")
    g4 = GeometryArg(config_c1().replace(f0=0.0))
    rc, msg = _call(g4, dtype=C, mode=_abi.IQDAS)
    assert rc == _abi.E_INVALID and "f0" in msg


def test_iq_demodulate_argument_errors():
    L = _abi.lib()
    g = GeometryArg(config_c1())
    assert L.pwbf_iq_demodulate(None, FAKE, 0, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_iq_demodulate(g.ref, FAKE, _abi.C32, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_iq_demodulate(g.ref, None, 0, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_iq_demodulate(g.ref, FAKE + 1, 0, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_iq_demodulate(g.ref, FAKE, 0, FAKE + 4, None) == _abi.E_INVALID
    for ns in (600, 8192):
        gb = GeometryArg(config_c1().replace(n_samples=ns))
        assert L.pwbf_iq_demodulate(gb.ref, FAKE, 0, FAKE, None) == _abi.E_UNSUPPORTED
    gf = GeometryArg(config_c1().replace(f0=-1.0))
    assert L.pwbf_iq_demodulate(gf.ref, FAKE, 0, FAKE, None) == _abi.E_INVALID
    o = ctypes.byref(_abi.Outputs(FAKE, None, None, None))
    assert L.pwbf_beamform_iqdas(g.ref, FAKE, -1, o, None, 0, None) == _abi.E_INVALID
    assert L.pwbf_beamform_bbdmas(None, FAKE, 0, o, None, 0, None) == _abi.E_INVALID


def test_metrics_argument_errors():
    L = _abi.lib()
    g = GeometryArg(config_c1())
    d = _abi.Disc(0.0, 20e-3, 1e-3)
    cy = (_abi.Cyst * 1)(_abi.Cyst(d, d))
    tg = (_abi.Disc * 1)(d)
    assert L.pwbf_contrast_metrics(None, FAKE, cy, 1, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_contrast_metrics(g.ref, None, cy, 1, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_contrast_metrics(g.ref, FAKE, cy, 0, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_contrast_metrics(g.ref, FAKE, cy, 33, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_contrast_metrics(g.ref, FAKE, None, 1, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_contrast_metrics(g.ref, FAKE, cy, 1, None, None) == _abi.E_INVALID
    bad = (_abi.Cyst * 1)(_abi.Cyst(_abi.Disc(0.0, 20e-3, 0.0), d))
    assert L.pwbf_contrast_metrics(g.ref, FAKE, bad, 1, FAKE, None) == _abi.E_INVALID
    nan = (_abi.Disc * 1)(_abi.Disc(float("nan"), 20e-3, 1e-3))
    assert L.pwbf_resolution_metrics(g.ref, FAKE, nan, 1, FAKE, None) == _abi.E_INVALID
    assert L.pwbf_resolution_metrics(g.ref, FAKE + 2, tg, 1, FAKE, None) == _abi.E_INVALID


def test_batch_create_rejects_before_touching_the_device():
    g = GeometryArg(config_c1())
    ok = _frame(g)
    assert _create([])[0] == _abi.E_INVALID
    assert _create([ok], flags=8)[0] == _abi.E_INVALID
    assert _create([ok, _frame(g, reserved=1)])[0] == _abi.E_INVALID
    rc, msg = _create([ok, _frame(g, tile=Tile(1, 16, 1, 4, 0))])
    assert rc == _abi.E_INVALID and "wz * wx = 8" in msg
    g20 = GeometryArg(config_c1().replace(angles_deg=tuple(range(-10, 10))))
    rc, msg = _create([_frame(g20)])
    assert rc == _abi.E_UNSUPPORTED and "16 angles" in msg
    rc, msg = _create([_frame(g, dtype=_abi.C32, mode=_abi.IQDAS)])
    assert rc == _abi.E_UNSUPPORTED and "single-frame" in msg
    bad = GeometryArg(config_c1())
    bad.s.dz = -1.0
    assert _create([ok, _frame(bad)])[0] == _abi.E_INVALID
    assert _create([_frame(g, rf=None)])[0] == _abi.E_INVALID
    L = _abi.lib()
    assert L.pwbf_batch_create(None, 1, 0, None, None) == _abi.E_INVALID
    assert L.pwbf_batch_launch(None, None) == _abi.E_INVALID
    assert L.pwbf_batch_update(None, None, 1, None) == _abi.E_INVALID
    assert L.pwbf_batch_destroy(None) == 0


def _probe(g, mode=_abi.DAS, angle=-1, env=1, log=1, slots=2, quality=0, region=None,
           max_cr=-10.0):
    q = _abi.Cyst() if region is None else _abi.Cyst(_abi.Disc(*region[0]), _abi.Disc(*region[1]))
    return _abi.Probe(ctypes.pointer(g.s) if g is not None else None, mode, angle, env, log,
                      slots, quality, q, max_cr)


def _server_create(probes, budget=0, max_queue=0):
    L = _abi.lib()
    arr = (_abi.Probe * max(1, len(probes)))(*probes)
    h = ctypes.c_void_p()
    rc = L.pwbf_server_create(arr, len(probes), budget, max_queue, ctypes.byref(h))
    assert not h.value
    return rc, L.pwbf_last_error().decode()


def test_server_create_rejects_before_touching_the_device():
    g = GeometryArg(config_c1())
    ok = _probe(g)
    assert _server_create([])[0] == _abi.E_INVALID
    assert _server_create([ok], max_queue=-1)[0] == _abi.E_INVALID
    assert _server_create([ok, _probe(g, quality=2)])[0] == _abi.E_INVALID
    good = ((0.0, 0.02, 2e-3), (5e-3, 0.02, 2e-3))
    assert _server_create([_probe(g, quality=1)])[0] == _abi.E_INVALID  # no region
    rc, msg = _server_create([_probe(g, quality=1, region=((0.0, 0.02, 0.0), good[1]))])
    assert rc == _abi.E_INVALID and "quality check" in msg
    rc, _ = _server_create([_probe(g, quality=1, region=good, max_cr=float("nan"))])
    assert rc == _abi.E_INVALID
    rc, _ = _server_create([_probe(g, quality=1, region=((float("inf"), 0.02, 1e-3), good[1]))])
    assert rc == _abi.E_INVALID
    assert _server_create([_probe(g, slots=65)])[0] == _abi.E_INVALID
    assert _server_create([_probe(g, env=2)])[0] == _abi.E_INVALID
    assert _server_create([_probe(None)])[0] == _abi.E_INVALID
    assert _server_create([_probe(g, mode=7)])[0] == _abi.E_INVALID
    assert _server_create([_probe(g, angle=1)])[0] == _abi.E_INVALID
    rc, msg = _server_create([ok, _probe(GeometryArg(config_c1().replace(
        angles_deg=tuple(range(-10, 10)))))])
    assert rc == _abi.E_UNSUPPORTED and "16 angles" in msg and "probe 1" in msg
    rc, msg = _server_create([_probe(GeometryArg(config_c1().replace(nz=300)))])
    assert rc == _abi.E_UNSUPPORTED and "power of two" in msg
    rc, msg = _server_create([_probe(g, mode=_abi.BBDMAS)])
    assert rc == _abi.E_UNSUPPORTED and "single-frame" in msg
    slot = 64 * 2048 * 2 + 3 * 128 * 256 * 4 + 8192  # FP16 RF, rf/env/log planes, max slots
    rc, msg = _server_create([ok], budget=slot - 1)
    assert rc == _abi.E_INVALID and f"needs {slot} bytes" in msg
    L = _abi.lib()
    assert L.pwbf_server_create(None, 1, 0, 0, None) == _abi.E_INVALID
    rid = ctypes.c_uint64()
    assert L.pwbf_server_submit(None, 0, FAKE, -1.0, ctypes.byref(rid)) == _abi.E_INVALID
    assert L.pwbf_server_submit_ex(None, 0, FAKE, -1.0, 1.0, ctypes.byref(rid)) == _abi.E_INVALID
    n = ctypes.c_int32()
    assert L.pwbf_server_poll(None, None, 1, ctypes.byref(n), 0) == _abi.E_INVALID
    assert L.pwbf_server_release(None, 1) == _abi.E_INVALID
    assert L.pwbf_server_stats_get(None, None) == _abi.E_INVALID
    assert L.pwbf_server_now(None) == 0.0
    assert L.pwbf_server_destroy(None) == 0


def test_tune_argument_errors():
    L = _abi.lib()
    g = GeometryArg(config_c1())
    o = _abi.Outputs(FAKE, None, None, None)
    assert L.pwbf_tune(g.ref, FAKE, 0, 0, 0, ctypes.byref(o), 3, None, None, None) == \
        _abi.E_INVALID
    assert L.pwbf_tune(g.ref, FAKE, 0, 0, 0, None, 0, None, None, None) == _abi.E_INVALID
    g.s.n_angles = 0
    assert L.pwbf_tune(g.ref, FAKE, 0, 0, 0, ctypes.byref(o), 0, None, None, None) == \
        _abi.E_INVALID


def test_tuning_table_round_trip_drives_default_plans(tmp_path):
    import math
    from paper_2311_00482_amd import tune_clear, tune_load, tune_save
    g = config_c3()
    sc = g.fs / g.c
    smax = max(abs(math.sin(a)) for a in g.angles_rad)
    # the table key names the shape (see the library's shape_key)
    key = "m0_t2_a11_n128_s4096_x1024_z1024_dx%.4g_dz%.4g_sin%.3g_w0" % (
        g.dx * sc, g.dz * sc, smax)
    path = tmp_path / "tune.json"
    path.write_text('{\n  "%s": [2, 8, 1, 4, 0]\n}\n' % key)
    tune_clear()
    try:
        assert describe_plan(g)["cpw"] == 1
        tune_load(str(path))
        p = describe_plan(g)
        assert (p["cpw"], p["lz"], p["wz"], p["wx"]) == (2, 8, 1, 4)
        # an explicit tile still wins over the table
        assert describe_plan(g, tile=Tile(1, 16, 1, 8, 0))["cpw"] == 1
        out = tmp_path / "saved.json"
        tune_save(str(out))
        assert key in out.read_text()
    finally:
        tune_clear()
    assert describe_plan(g)["cpw"] == 1


def test_fk_workspace_and_argument_errors():
    L = _abi.lib()
    g3 = config_c3()
    g = GeometryArg(g3)
    o = _abi.Outputs(FAKE, None, FAKE, None, FAKE)
    r256 = lambda b: (b + 255) // 256 * 256  # noqa: E731
    W = L.pwbf_fk_workspace_bytes
    ST, LU = _abi.FK_STOLT, _abi.FK_LU

    # T [128][2049 rounded up to blocks of 4096 / Nx bins], P [2049][Nx],
    # U [Nx][2049], M [Nx][4096] per angle, complex float32; Nx = 256 (Stolt)
    # or 512 (Lu)
    def per(a, nx, n=128, nt=4096):
        kb, rows = nt // 2 + 1, 4096 // nx
        kpad = -(-kb // rows) * rows
        return (r256(a * n * kpad * 8) + r256(a * kb * nx * 8) + r256(a * nx * kb * 8)
                + r256(a * nx * nt * 8))
    need = 8192 + per(11, 256)
    assert W(g.ref, ST, -1, ctypes.byref(o)) == need
    assert W(g.ref, ST, 3, ctypes.byref(o)) == 8192 + per(1, 256)
    assert W(g.ref, LU, -1, ctypes.byref(o)) == 8192 + per(11, 512)
    assert W(g.ref, ST, 11, ctypes.byref(o)) == 0 and W(g.ref, ST, -2, ctypes.byref(o)) == 0
    assert W(g.ref, 2, -1, ctypes.byref(o)) == 0 and b"method" in L.pwbf_last_error()
    # a log image without an envelope plane needs the envelope in the workspace
    olog = _abi.Outputs(FAKE, None, None, FAKE)
    assert W(g.ref, ST, -1, ctypes.byref(olog)) == need + 1024 * 1024 * 4
    # unsupported shapes: record length, one channel, non-uniform pitch
    for bad in (g3.replace(n_samples=600), g3.replace(n_samples=8192), g3.replace(n_channels=1)):
        for meth in (ST, LU):
            assert W(GeometryArg(bad).ref, meth, -1, ctypes.byref(o)) == 0
            assert L.pwbf_last_error()
    ga = GeometryArg(g3)
    ga.elem_x[5] += 0.01 * (ga.elem_x[1] - ga.elem_x[0])
    assert W(ga.ref, LU, -1, ctypes.byref(o)) == 0
    assert b"pitch" in L.pwbf_last_error()
    # Lu pads to 4 N: 256 channels need 1024 (supported)
    g256 = GeometryArg(g3.replace(n_channels=256, n_samples=1024))
    assert W(g256.ref, LU, 0, ctypes.byref(o)) == 8192 + per(1, 1024, n=256, nt=1024)
    # every call below fails a host check before any HIP call (workspace is NULL
    # or too small, so none reaches the launches)
    oo = ctypes.byref(o)
    M = L.pwbf_fk_migrate
    assert M(None, FAKE, 0, ST, -1, oo, None, 0, None) == _abi.E_INVALID
    assert M(ga.ref, FAKE, 0, ST, -1, oo, FAKE, need, None) == _abi.E_UNSUPPORTED
    assert M(g.ref, FAKE, 0, 7, -1, oo, FAKE, need, None) == _abi.E_INVALID
    assert M(g.ref, FAKE, _abi.C32, ST, -1, oo, None, 0, None) == _abi.E_INVALID
    assert M(g.ref, None, 0, ST, -1, oo, None, 0, None) == _abi.E_INVALID
    assert M(g.ref, FAKE + 1, 0, LU, -1, oo, None, 0, None) == _abi.E_INVALID
    assert M(g.ref, FAKE, 0, ST, 11, oo, None, 0, None) == _abi.E_INVALID
    assert M(g.ref, FAKE, 0, ST, -2, oo, None, 0, None) == _abi.E_INVALID
    assert M(g.ref, FAKE, 0, ST, -1, None, None, 0, None) == _abi.E_INVALID
    of = _abi.Outputs(FAKE, FAKE, None, None)
    assert M(g.ref, FAKE, 0, ST, -1, ctypes.byref(of), None, 0, None) == _abi.E_INVALID
    assert b"band-pass" in L.pwbf_last_error()
    gb = GeometryArg(g3, bandpass=True)
    assert M(gb.ref, FAKE, 0, LU, -1, oo, None, 0, None) == _abi.E_INVALID
    assert M(g.ref, FAKE, 0, ST, -1, oo, None, 0, None) == _abi.E_INVALID
    assert M(g.ref, FAKE, 0, ST, -1, oo, FAKE + 128, need, None) == _abi.E_INVALID
    assert M(g.ref, FAKE, 0, ST, -1, oo, FAKE, need - 1, None) == _abi.E_INVALID
    assert b"required" in L.pwbf_last_error()
    # the Stolt-sized workspace is too small for Lu
    assert M(g.ref, FAKE, 0, LU, -1, oo, FAKE, need, None) == _abi.E_INVALID


def test_noalloc_entry_refuses_envelope_beyond_its_scratch():
    # a log image without an envelope output on a grid of more than 2^22 pixels
    # needs more scratch than the allocation-free call holds: refused on the
    # host, before any HIP call, with the reason
    L = _abi.lib()
    g = GeometryArg(config_c3().replace(nx=4096, nz=2048))
    o = _abi.Outputs(FAKE, None, None, FAKE, None)
    rc = L.pwbf_compound_noalloc(g.ref, FAKE, _abi.F32, _abi.DAS, ctypes.byref(o), None)
    assert rc == _abi.E_UNSUPPORTED
    assert "scratch" in L.pwbf_last_error().decode()
    assert L.pwbf_compound_noalloc(None, FAKE, _abi.F32, _abi.DAS, ctypes.byref(o),
                                   None) == _abi.E_INVALID
