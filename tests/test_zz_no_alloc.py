"""The allocation-free compound entry point (pwbf_compound_noalloc) against
pwbf_compound with a caller's workspace, through the C ABI, on two calls in a
row, the second on a smaller frame: the same kernels run, so the planes must
agree to the float32 bar (max-normalised 1e-5, log image 0.1 dB), and the
second call must not see the first call's frame maximum left in the shared
scratch array."""

import ctypes

import numpy as np
import pytest

from cases import geom, rand_rf

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_DB = 0.1


def _torch():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch


def _planes(torch, g, names):
    return {k: torch.full((g.nx, g.nz), float("nan"), dtype=torch.float32, device="cuda")
            for k in names}


def _outputs(_abi, planes):
    def ptr(k):
        return planes[k].data_ptr() if k in planes else None
    return _abi.Outputs(ptr("rf"), ptr("filtered"), ptr("env"), ptr("log"), None)


def _call_both(g, rf, mode, names, bandpass=False):
    from paper_2311_00482_amd import _abi
    from paper_2311_00482_amd.api import GeometryArg, _rf_code
    torch = _torch()
    L = _abi.lib()
    ga = GeometryArg(g, bandpass=bandpass)
    rf_t = torch.from_numpy(rf).cuda()
    code = _rf_code(rf_t)
    stream = torch.cuda.current_stream().cuda_stream
    # the allocation-free call
    a = _planes(torch, g, names)
    oa = _outputs(_abi, a)
    rc = L.pwbf_compound_noalloc(ga.ref, rf_t.data_ptr(), code, _abi.DAS if mode == "das"
                                 else _abi.DMAS, ctypes.byref(oa), stream)
    assert rc == 0, L.pwbf_last_error().decode()
    torch.cuda.synchronize()
    # the workspace call
    b = _planes(torch, g, names)
    ob = _outputs(_abi, b)
    need = L.pwbf_workspace_bytes(ga.ref, ctypes.byref(ob))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    rc = L.pwbf_compound(ga.ref, rf_t.data_ptr(), code, _abi.DAS if mode == "das" else _abi.DMAS,
                         ctypes.byref(ob), ws.data_ptr() if need else None, need, stream)
    assert rc == 0, L.pwbf_last_error().decode()
    torch.cuda.synchronize()
    return ({k: v.cpu().numpy().astype(np.float64) for k, v in a.items()},
            {k: v.cpu().numpy().astype(np.float64) for k, v in b.items()})


def _check(a, b):
    for k in a:
        if k == "log":
            assert np.isfinite(a[k]).all()
            assert float(np.abs(a[k] - b[k]).max()) <= TOL_DB, k
            assert a[k].max() == 0.0  # normalised by this frame's own maximum
        else:
            e = float(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max())
            assert e <= TOL32, (k, e)


def test_noalloc_matches_workspace_call_twice_second_smaller():
    # first: 5 angles, 64 channels, 256 x 512, the log image without an
    # envelope output (the envelope lives in the scratch array)
    g1 = geom(angles_deg=(-8.0, -4.0, 0.0, 4.0, 8.0), n_channels=64, n_samples=1024,
              nx=256, nz=512, x_min=-9e-3, x_max=9e-3, z_min=4e-3, z_max=24e-3)
    rf1 = rand_rf(g1, 71, "i16")
    a, b = _call_both(g1, rf1, "das", ("rf", "log"))
    _check(a, b)
    # second, smaller, with a much smaller image maximum: a stale maximum from
    # the first call would put its log image far below 0 dB
    g2 = geom(angles_deg=(0.0,), n_channels=16, n_samples=600, nx=37, nz=64)
    rf2 = (rand_rf(g2, 72, "f32") * 1e-3).astype(np.float32)
    a2, b2 = _call_both(g2, rf2, "dmas", ("rf", "log"))
    _check(a2, b2)
