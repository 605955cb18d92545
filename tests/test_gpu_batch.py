"""GPU: batches of uneven frames in one persistent graph launch, and the tuner.

A batch frame runs the same tile body as a single-frame launch with the same
launch shape. The two kernels are compiled separately, so the compiler may fuse
multiply-adds differently: each plane of a frame must match its single-frame
result to 1e-6 (max-normalised; 1e-3 dB on the log image) - the frame is the
same alone and in the mix, well inside the 1e-5 bar against the oracle. Graph
replays of one batch are bitwise equal. The whole uneven 32-frame workload is
also checked against the FP64 oracle.
"""

import numpy as np
import pytest

import oracle
from synth import config_c4_frames, make_frame

from cases import geom, rand_rf

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def planes(g, want, dev):
    torch = _torch()
    return {k: torch.full((g.nx, g.nz), float("nan"), dtype=torch.float32, device=dev)
            for k in want}


def single(g, rf_t, mode, angle, tile, want, bandpass):
    from paper_2311_00482_amd import beamform
    out = beamform(g, rf_t, mode, angle, tile=tile, want=want, bandpass=bandpass)
    _torch().cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def same(got, ref, key, mode):
    if key == "log":
        return float(np.abs(got - ref).max()) <= 1e-3
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-30)) <= 1e-6


def mixed_frames(dev, seed=0):
    from paper_2311_00482_amd import FrameSpec, Tile
    torch = _torch()
    specs = [
        (geom(angles_deg=(-8.0, 0.0, 8.0), nx=80, nz=128), "das", -1, Tile(1, 16, 1, 8, 0),
         ("rf", "env", "log"), False, "f32"),
        (geom(n_channels=32, nx=66, nz=128), "dmas", 0, Tile(4, 8, 1, 8, 0), ("rf", "env"), False,
         "i16"),
        (geom(angles_deg=(-10., -5., 0., 5., 10.), nx=21, nz=256, n_channels=24), "das", -1,
         Tile(4, 16, 1, 8, 0), ("rf",), False, "f16"),
        (geom(angles_deg=(0.0, 4.0), n_channels=20, nx=128, nz=512, z_min=10e-3,
              z_max=10e-3 + 512 * 25e-6), "dmas", -1, Tile(1, 16, 2, 4, 0),
         ("rf", "filtered", "env", "log"), True, "f32"),
        (geom(angles_deg=tuple(range(-6, 8, 2)), nx=68, nz=128), "das", 3, Tile(1, 8, 2, 4, 0),
         ("rf", "log"), False, "f32"),
        (geom(angles_deg=(-5.0, 5.0), n_channels=20, nx=90, nz=128), "pdas", -1,
         Tile(4, 8, 1, 8, 0), ("rf", "env"), False, "i16"),
    ]
    frames, ref_args = [], []
    for i, (g, mode, angle, tile, want, bp, kind) in enumerate(specs):
        rf = rand_rf(g, 100 + i + seed, "i16" if kind == "i16" else "f32")
        rf_t = torch.from_numpy(rf).to(dev)
        if kind == "f16":
            rf_t = rf_t.to(torch.float16)
        frames.append(FrameSpec(g, rf_t, mode, angle, planes(g, want, dev), bp, tile))
        ref_args.append((g, rf_t, mode, angle, tile, want, bp))
    return frames, ref_args


def test_batch_planes_bitwise_equal_single_frame_launches():
    from paper_2311_00482_amd import Batch
    torch = _torch()
    dev = torch.device("cuda:0")
    frames, args = mixed_frames(dev)
    b = Batch(frames)
    info = b.describe()
    assert info["n_frames"] == len(frames) and info["blocks"] >= 1
    # reset, then per branch one beamform kernel per class of its frames, post, log
    assert 1 <= info["branches"] <= min(4, len(frames))
    assert info["kernels"] >= info["branches"]
    # (a branch launches post-processing and log kernels only for frames that ask)
    assert 1 + info["kernels"] <= info["graph_nodes"] <= 1 + info["kernels"] + 2 * info["branches"]
    b.launch()
    torch.cuda.synchronize()
    for f, a in zip(frames, args):
        ref = single(*a)
        for k, v in f.out.items():
            got = v.cpu().numpy()
            assert same(got, ref[k], k, a[2]), (a[2], k, np.abs(got - ref[k]).max())
    b.close()


def test_batch_graph_replays_and_updates():
    from paper_2311_00482_amd import Batch
    torch = _torch()
    dev = torch.device("cuda:0")
    frames, _ = mixed_frames(dev)
    b = Batch(frames)
    b.launch()
    torch.cuda.synchronize()
    first = [{k: v.cpu().numpy() for k, v in f.out.items()} for f in frames]
    for rep in range(3):
        for f in frames:  # scribble on the outputs between replays
            for v in f.out.values():
                v.fill_(float(rep) - 7.0)
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for f, ref in zip(frames, first):
            for k, v in f.out.items():
                assert np.array_equal(v.cpu().numpy(), ref[k]), (rep, k)
    # new RF and new output buffers of the same shapes
    frames2, args2 = mixed_frames(dev, seed=50)
    b.update(frames2)
    b.launch()
    torch.cuda.synchronize()
    for f, a in zip(frames2, args2):
        ref = single(*a)
        for k, v in f.out.items():
            assert same(v.cpu().numpy(), ref[k], k, a[2]), k
    # the same shapes on another geometry: the grid moved sideways and deeper
    # and a tighter F-number change which channels reach each tile, and the
    # update must follow them (the tiles' channel hulls are recomputed)
    from paper_2311_00482_amd import FrameSpec
    frames3, args3 = [], []
    for f, a in zip(frames2, args2):
        g3 = f.geom.replace(x_min=f.geom.x_min + 1.1e-3, x_max=f.geom.x_max + 1.1e-3,
                            z_min=f.geom.z_min + 0.7e-3, z_max=f.geom.z_max + 0.7e-3,
                            f_number=f.geom.f_number * 1.6)
        frames3.append(FrameSpec(g3, f.rf, f.mode, f.angle, f.out, f.bandpass, f.tile))
        args3.append((g3,) + tuple(a[1:]))
    b.update(frames3)
    b.launch()
    torch.cuda.synchronize()
    for f, a in zip(frames3, args3):
        ref = single(*a)
        for k, v in f.out.items():
            assert same(v.cpu().numpy(), ref[k], k, a[2]), ("moved grid", k)
    # a frame of another shape is refused
    g_other = geom(nx=41, nz=128, angles_deg=(-8.0, 0.0, 8.0))
    frames2[0].geom = g_other
    from paper_2311_00482_amd import PwbfError
    with pytest.raises(PwbfError):
        b.update(frames2)
    b.close()


@pytest.fixture(scope="module")
def c4():
    specs = config_c4_frames()
    return [(s, make_frame(s.geom, s.seed, "scaled")) for s in specs]


def test_uneven_32_frame_batch_matches_oracle(c4):
    from paper_2311_00482_amd import Batch, FrameSpec
    torch = _torch()
    dev = torch.device("cuda:0")
    frames = []
    for s, fr in c4:
        g = s.geom
        rf_t = torch.from_numpy(fr["i16"]).to(dev).to(torch.float16)  # int16 -> FP16 is exact
        want = ("rf", "env", "log")
        frames.append(FrameSpec(g, rf_t, s.mode, -1, planes(g, want, dev), False, None))
    b = Batch(frames, tune=True)
    b.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    worst = 0.0
    for (s, fr), f in zip(c4, frames):
        g = s.geom
        y = f.out["rf"].cpu().numpy().astype(np.float64)
        assert np.isfinite(y).all()
        pix = np.unique(np.concatenate([rng.choice(g.nx * g.nz, 150, replace=False),
                                        [int(np.argmax(np.abs(y)))]]))
        ref = oracle.compound(g, fr["master"], s.mode, pix)
        e = np.abs(y.ravel()[pix] - ref).max() / np.abs(y).max()
        worst = max(worst, e)
        assert e <= 1e-5, (g.name, e)
        lg = f.out["log"].cpu().numpy()
        assert lg.max() == 0.0 and lg.min() >= -70.0
    b.close()
    print(f"32-frame batch: worst sampled max-normalised error {worst:.2e}")


def test_tune_picks_a_shape_and_default_plans_follow_it():
    from paper_2311_00482_amd import describe_plan, tune, tune_clear
    torch = _torch()
    g = geom(angles_deg=(-5.0, 0.0, 5.0), nx=128, nz=256)
    rf_t = torch.from_numpy(rand_rf(g, 9)).cuda()
    tune_clear()
    try:
        t, ms = tune(g, rf_t, "das", -1)
        assert ms > 0 and t.cpw in (1, 2, 4)
        p = describe_plan(g)
        assert (p["cpw"], p["lz"], p["wz"], p["wx"]) == (t.cpw, t.lz, t.wz, t.wx)
        t8, _ = tune(g, rf_t, "das", -1, waves=8)
        assert t8.wz * t8.wx == 8
    finally:
        tune_clear()
