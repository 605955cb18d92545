#!/usr/bin/env python3
"""Throughput of the plane-wave beamformer on the 11-angle compounding workload.

One step = one frame through the whole path: coherent compound DAS of 11
steering angles x 128 channels x 4096 samples onto 1024 x 1024 pixels, then the
depth-wise Hilbert envelope and the -70 dB log image, with RF resident in HBM.
Prints one JSON line (rank 0). Synthetic seeded RF: 20 points, 3 anechoic cysts
and ~19k speckle scatterers, Gaussian 2-cycle 5 MHz pulse, 30 dB SNR.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpixel·ch/s + frames/s (128ch, 11-angle, 1024²); p50/p99 frame latency"
UNIT = "Gpixel·ch/s"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz issue 3.93e13 non-packed
# float32 lane operations per second (the packed-FP32 and FMA doublings of the
# 157.3 TFLOP/s vector figure do not apply to this kernel's instruction mix).
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8e12
# Algorithmic float32 operations of the beamformer (counted once, as defined):
# per gathered sample (pixel, channel, angle): delay add, floor, fraction,
# sample difference, interpolation FMA, accumulate = 6; per (pixel, channel):
# receive offset, squared distance, square root, aperture ratio, cosine, weight
# FMA, window test, weight select, weighted accumulate = 9; per (pixel, angle):
# the transmit delay, 2.
OPS_PER_GATHER, OPS_PER_PIX_CH, OPS_PER_PIX_ANGLE = 6, 9, 2
KERNEL_SOURCES = ["paper_2311_00482_amd/csrc/beamform.hip", "paper_2311_00482_amd/csrc/plan.h"]
COUNTERS = os.path.join(ROOT, "profiles", "k_beamform_c3_compound_f32.counters.json")


def algorithmic_ops(g) -> float:
    P = g.nx * g.nz
    return float(P * g.n_channels * g.n_angles * OPS_PER_GATHER
                 + P * g.n_channels * OPS_PER_PIX_CH + P * g.n_angles * OPS_PER_PIX_ANGLE)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes():
    """HBM bytes per launch of the beamform kernel from committed rocprofv3
    counters, or None when absent or taken on a different kernel source."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return float(c["hbm_bytes_per_dispatch"])


def time_steps(fn, steps, warmup, torch):
    """Warm up, then time exactly `steps` calls bracketed by synchronisation;
    per-step latency from HIP events on the launching stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])  # ms
    span = ev[0][0].elapsed_time(ev[-1][1])  # ms, first start to last end
    return wall, lat, span


def cpu_baseline(g, rf_master, budget_s: float):
    """The FP64 oracle on a bounded sample of whole depth columns, single thread."""
    import oracle
    cols_all = np.arange(g.nx)
    t0 = time.perf_counter()
    oracle.das(g, rf_master, -1, np.arange(g.nz) + (g.nx // 2) * g.nz)
    per_col = time.perf_counter() - t0
    n_cols = int(max(1, min(g.nx, budget_s / max(per_col, 1e-6))))
    cols = cols_all[np.linspace(0, g.nx - 1, n_cols).astype(int)]
    pix = (cols[:, None] * g.nz + np.arange(g.nz)[None, :]).ravel()
    t0 = time.perf_counter()
    oracle.das(g, rf_master, -1, pix)
    dt = time.perf_counter() - t0
    gathers = len(pix) * g.n_channels * g.n_angles
    return {"value": gathers / dt / 1e9, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"{n_cols} of {g.nx} depth columns ({len(pix)} pixels x "
                      f"{g.n_channels} ch x {g.n_angles} angles), compound DAS only, "
                      f"{dt:.1f} s", "seconds": dt,
            "frames_per_s_equiv": gathers / dt / g.gathers}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline sample")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the timed FP32 compound loop (for rocprofv3)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run 3 plain device-to-device copies of this many MiB "
                         "(a reference kernel for calibrating HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(frames would be sharded across GPUs with no exchange); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2311_00482_amd import beamform, describe_plan
    from synth import config_c3, make_frame

    dev = torch.device("cuda:0")
    g = config_c3()
    print(f"[bench] simulating {g.name}", file=sys.stderr, flush=True)
    fr = make_frame(g, 1003, "c3", quantize=False)
    rf32 = torch.from_numpy(fr["f32"]).to(dev)
    rf16 = torch.from_numpy(fr["f16"]).to(dev)
    want = ("rf", "env", "log")
    outs = {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in want}
    ws = torch.empty(4096, dtype=torch.uint8, device=dev)

    def step32():
        beamform(g, rf32, "das", -1, want=want, out=outs, workspace=ws)

    def step16():
        beamform(g, rf16, "das", -1, want=want, out=outs, workspace=ws)

    rf_only = {"rf": outs["rf"]}

    def kernel_only():
        beamform(g, rf32, "das", -1, want=("rf",), out=rf_only)

    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    print("[bench] timing FP32-stored RF (headline)", file=sys.stderr, flush=True)
    wall, lat, span = time_steps(step32, args.steps, args.warmup, torch)
    if args.profile_only:
        print(json.dumps({"profile_only": True, "ms_per_step": wall / args.steps * 1e3}))
        return
    print("[bench] timing FP16-stored RF", file=sys.stderr, flush=True)
    wall16, lat16, _ = time_steps(step16, args.steps, args.warmup, torch)
    print("[bench] timing the beamform kernel alone", file=sys.stderr, flush=True)
    _, _, kspan = time_steps(kernel_only, args.steps, args.warmup, torch)
    k_ms = kspan / args.steps

    gathers = g.gathers
    value = gathers * args.steps / wall / 1e9
    ops = algorithmic_ops(g)
    achieved = ops / (k_ms * 1e-3)
    traffic = traffic_bytes()
    plan = describe_plan(g, "das", -1)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "compound DAS, 11 angles -10..10 deg, 128 ch x 4096 samples, "
                               "1024x1024 pixels, FP32-stored RF, RF + envelope + log per frame",
                   "rf_storage": "f32", "pixels": g.nx * g.nz, "channels": g.n_channels,
                   "angles": g.n_angles, "samples": g.n_samples,
                   "tile": {k: plan[k] for k in ("cpw", "lz", "wz", "wx", "tile_z", "tile_x",
                                                  "chunk", "win")}},
        "frames_per_s": args.steps / wall,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "Tlane-op/s",
                     "frac": achieved / VALU_LANE_OPS_PEAK, "traffic": traffic,
                     "kernel": "k_beamform<11> (compound DAS)", "kernel_ms": k_ms,
                     "ops_per_launch": ops},
        "hbm": {"compulsory_bytes_per_frame": float(rf32.numel() * 4 + 3 * g.nx * g.nz * 4),
                "compulsory_frac": float(rf32.numel() * 4 + 3 * g.nx * g.nz * 4)
                / (wall / args.steps) / HBM_PEAK,
                "gather_effective_GBps": gathers * 2 * 4 / (k_ms * 1e-3) / 1e9,
                "gather_effective_frac": gathers * 2 * 4 / (k_ms * 1e-3) / HBM_PEAK},
        "variants": {"f16_storage": {"value": gathers * args.steps / wall16 / 1e9,
                                     "frames_per_s": args.steps / wall16,
                                     "latency_ms": {"p50": float(np.percentile(lat16, 50)),
                                                    "p99": float(np.percentile(lat16, 99))}}},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        cb = cpu_baseline(g, fr["master"], args.cpu_budget)
        cb["host_cores_available"] = os.cpu_count()
        line["cpu_baseline"] = cb
    print(json.dumps(line))


if __name__ == "__main__":
    main()
