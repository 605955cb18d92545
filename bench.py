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
import gc
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
# the transmit delay, 2. Only (pixel, channel) pairs inside the receive aperture
# (nonzero apodization weight) count: the others add exactly zero to the sum.
OPS_PER_GATHER, OPS_PER_PIX_CH, OPS_PER_PIX_ANGLE = 6, 9, 2
KERNEL_SOURCES = ["paper_2311_00482_amd/csrc/beamform.hip",
                  "paper_2311_00482_amd/csrc/beamform_device.h",
                  "paper_2311_00482_amd/csrc/plan.h"]
COUNTERS = os.path.join(ROOT, "profiles", "k_beamform_c3_compound_f32.counters.json")
# workspace of the single-frame calls timed here (every call that asks for the log
# image also asks for the envelope plane, so the workspace holds only the frame
# maximum's slots); the library checks the size on every call
WS_BYTES = 64 * 1024


def aperture_pairs(g) -> int:
    """(pixel, channel) pairs with a nonzero apodization weight: |x - x_e| < z / (2 F#)."""
    if g.apod == "none":
        return g.nx * g.nz * g.n_channels
    xe = np.sort(np.asarray(g.elem_x, dtype=np.float64))
    h = np.maximum(g.z_pix, 0.0) / (2.0 * g.f_number)
    X = g.x_pix[:, None]
    hi = np.searchsorted(xe, (X + h[None, :]).ravel(), "left")
    lo = np.searchsorted(xe, (X - h[None, :]).ravel(), "right")
    return int(np.maximum(hi - lo, 0).sum())


# The nonlinear beamformers, counted the same way (per gather, per (pixel,
# channel), per (pixel, angle)). DMAS: delay add, floor, fraction,
# interpolation FMA, |v|, square root, signed root, weighted accumulate, |v|
# accumulate = 9; per (pixel, channel) the DAS terms with the weighted
# accumulate replaced by w^2 and its FMA into Q = 10; per (pixel, angle) the
# transmit delay and the square of the angle's sum = 3. pDAS: delay add, floor,
# fraction, interpolation FMA, |v|, log2, times 1/p, exp2, signed root,
# weighted accumulate = 10; per (pixel, channel) the DAS terms without the
# weighted accumulate = 8; per (pixel, angle) the transmit delay and the signed
# p-th power (|t|, log2, times p, exp2, sign, add) = 8. At p = 2 the root is a
# square root and the power t |t|: 8 per gather (delay add, floor, fraction,
# interpolation FMA, |v|, square root, signed root, weighted accumulate), 8 per
# (pixel, channel), 4 per (pixel, angle) (transmit delay, |t|, multiply, add).
# IQ-DAS: delay add, floor, two interpolation FMAs (real and imaginary lines),
# complex multiply-accumulate with the receive phasor (4) = 8 per gather; per
# (pixel, channel) the DAS terms plus the receive phase (multiply, cos, sin,
# complex multiply by the tile's integer-part phasor, weight) = 18; per (pixel,
# angle) the transmit delay, its phasor (multiply, cos, sin, complex multiply),
# the complex multiply of the angle's sum and the add = 14. BB-DMAS adds |q|^2,
# square root, reciprocal square root, a select and two scalings per gather
# (14) and the square of each angle's sum (17 per (pixel, angle)).
MODE_OPS = {"das": (OPS_PER_GATHER, OPS_PER_PIX_CH, OPS_PER_PIX_ANGLE), "dmas": (9, 10, 3),
            "pdas": (10, 8, 8), "pdas2": (8, 8, 4), "iqdas": (8, 18, 14),
            "bbdmas": (14, 18, 17)}


def algorithmic_ops(g, mode: str = "das", p: float = 2.0) -> float:
    key = "pdas2" if mode == "pdas" and p == 2.0 else mode
    per_gather, per_pix_ch, per_pix_angle = MODE_OPS[key]
    P = g.nx * g.nz
    pairs = aperture_pairs(g)
    return float(pairs * g.n_angles * per_gather + pairs * per_pix_ch
                 + P * g.n_angles * per_pix_angle)


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


# The device lowers its clocks within milliseconds of idling (measured on
# MI355X: after 50 ms idle the next steps run 15% slower, after 5 ms 4%) and
# takes a few milliseconds of load to raise them again, longer than a short
# warm-up. Each timed loop therefore first runs its step, untimed, for a ramp
# period, with all host-side preparation (events, garbage collection) done
# before, so the warm-up and timed steps follow the ramp with no idle gap
# (--clock-ramp seconds, 0 to skip, as for profiling runs).
RAMP_S = 0.3


def time_steps(fn, steps, warmup, torch, ramp_s=None):
    """Ramp, warm up, then time exactly `steps` calls bracketed by
    synchronisation; per-step latency from HIP events on the launching stream.
    Python's garbage collector is run before and paused during the ramp, the
    warm-up and the timed loop, so a collection cannot stall the host between
    launches."""
    ramp_s = RAMP_S if ramp_s is None else ramp_s
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    gc.collect()
    gc.disable()
    try:
        return _time_steps(fn, steps, warmup, torch, stream, ev, ramp_s)
    finally:
        gc.enable()


def _time_steps(fn, steps, warmup, torch, stream, ev, ramp_s):
    t_ramp = time.perf_counter()
    while time.perf_counter() - t_ramp < ramp_s:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
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


def cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _columns(g, n_cols):
    """n_cols whole depth columns spread over the grid, and their flat pixel indices."""
    cols = np.unique(np.linspace(0, g.nx - 1, max(1, min(g.nx, n_cols))).astype(int))
    return cols, (cols[:, None] * g.nz + np.arange(g.nz)[None, :]).ravel()


def cpu_baseline(g, rf_master, budget_s: float):
    """The FP64 oracle timed on the host's cores: the OpenMP build of the same
    source over every thread it is given (the reported value), and the
    single-threaded build, each on whole depth columns sized to about budget_s
    seconds (the OpenMP leg takes the whole image when it fits). Returns the
    baseline record and the OpenMP leg's (columns, pixels, values) for the
    accuracy figures."""
    import oracle
    mid = np.arange(g.nz) + (g.nx // 2) * g.nz
    legs = {}
    for parallel in (False, True):
        t0 = time.perf_counter()
        oracle.das(g, rf_master, -1, mid, parallel=parallel)
        per_col = time.perf_counter() - t0
        cols, pix = _columns(g, int(budget_s / max(per_col, 1e-6)))
        t0 = time.perf_counter()
        vals = oracle.das(g, rf_master, -1, pix, parallel=parallel)
        dt = time.perf_counter() - t0
        legs[parallel] = (cols, pix, vals, dt)
    gathers_per_pixel = g.n_channels * g.n_angles

    def rate(leg):
        return len(leg[1]) * gathers_per_pixel / leg[3] / 1e9

    def sample(leg):
        return (f"{len(leg[0])} of {g.nx} depth columns ({len(leg[1])} pixels x "
                f"{g.n_channels} ch x {g.n_angles} angles), compound DAS only, {leg[3]:.1f} s")

    omp, one = legs[True], legs[False]
    threads = oracle.threads(True)
    note = ("the oracle evaluates every channel of every pixel, including those outside "
            "the receive aperture (zero weight); the GPU kernel visits only the in-aperture "
            f"(pixel, channel) pairs, {aperture_pairs(g) / (g.nx * g.nz * g.n_channels):.1%} "
            "of them here. The unit counts all channels for both, as defined.")
    rec = {"value": rate(omp), "unit": UNIT, "cores": threads, "kind": "oracle",
           "sample": sample(omp), "seconds": omp[3],
           "frames_per_s_equiv": len(omp[1]) * gathers_per_pixel / omp[3] / g.gathers,
           "build": f"OpenMP, {threads} threads", "cpu_model": cpu_model(),
           "host_cores_available": os.cpu_count(),
           "single_thread": {"value": rate(one), "unit": UNIT, "cores": 1,
                             "sample": sample(one), "seconds": one[3],
                             "frames_per_s_equiv":
                                 len(one[1]) * gathers_per_pixel / one[3] / g.gathers},
           "channels_note": note}
    return rec, omp[:3]


def _max_norm(gpu, ref) -> float:
    """max |gpu - ref| / max |ref| (the per-pixel max-normalised error)."""
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(np.asarray(gpu, dtype=np.float64) - ref).max()
                 / max(float(np.abs(ref).max()), 1e-300))


def _plane_errors(gpu: dict, ref_rf: np.ndarray, cols=None) -> dict:
    """rf and envelope errors (max-normalised) and the log image's largest dB
    difference where the oracle's log image is at or above -40 dB, over whole
    depth columns (all of them when cols is None)."""
    import oracle
    sel = slice(None) if cols is None else cols
    ref_env = oracle.envelope_z(ref_rf)
    out = {"rf": _max_norm(gpu["rf"][sel], ref_rf)}
    if "env" in gpu:
        out["env"] = _max_norm(gpu["env"][sel], ref_env)
    if "log" in gpu and cols is None:
        ref_log = oracle.log_compress(ref_env)
        m = ref_log >= -40.0
        out["log_db_max_abs"] = float(np.abs(gpu["log"][m] - ref_log[m]).max())
    return out


def error_vs_oracle(gs, fr, sample, gpu32: dict, gpu16: dict) -> dict:
    """The headline frame's planes against the FP64 oracle on the OpenMP
    baseline's sample (whole depth columns), for each RF storage type: FP32
    against the oracle on the simulated (float64) record, FP16 against it too
    (storage rounding included) and against the oracle on the FP16-stored
    samples themselves (the kernel's own arithmetic)."""
    import oracle
    cols, pix, vals = sample
    ref = vals.reshape(len(cols), gs.nz)
    whole = len(cols) == gs.nx
    res = {"sample": f"{len(cols)} of {gs.nx} depth columns", "norm": "max |oracle| over the "
           "sample, per plane", "bar": {"f32": 1e-5, "f16": 1e-3, "log_db": 0.1},
           "f32": _plane_errors(gpu32, ref, None if whole else cols),
           "f16": _plane_errors(gpu16, ref, None if whole else cols)}
    ref16 = oracle.das(gs, fr["f16"], -1, pix, parallel=True).reshape(len(cols), gs.nz)
    res["f16_vs_oracle_on_stored_samples"] = _plane_errors(gpu16, ref16,
                                                           None if whole else cols)
    return res


def _mode_error(gs, fr, mode: str, quant: bool, rf_plane) -> dict:
    """The raw beamformed plane of a DMAS or pDAS (p = 2) frame against the
    oracle on the stored samples: the whole image on 512 x 512 grids, 64 depth
    columns on larger ones."""
    import oracle
    rf_in = fr["i16"] if quant else fr["f32"]
    whole = gs.nx * gs.nz <= 512 * 512
    cols, pix = _columns(gs, gs.nx if whole else 64)
    if mode == "dmas":
        ref = oracle.dmas(gs, rf_in, -1, "identity", pix, parallel=True)
    else:
        ref = oracle.pdas(gs, rf_in, -1, 2.0, pix, parallel=True)
    gpu = rf_plane.cpu().numpy()[cols]
    return {"rf": _max_norm(gpu, ref.reshape(len(cols), gs.nz)),
            "sample": "whole image" if whole else f"{len(cols)} of {gs.nx} depth columns",
            "rf_storage": "int16" if quant else "f32"}


def c1_error(dev, torch) -> dict:
    """The single-frame DAS workload (1 angle, 64 ch x 2048 int16 samples,
    128 x 256 pixels) against the oracle on the whole image."""
    import oracle
    from paper_2311_00482_amd import GeometryArg, beamform
    from synth import config_c1, make_frame
    gs = config_c1()
    fr = make_frame(gs, 1001, "c1", quantize=True)
    g = GeometryArg(gs)
    out = beamform(g, torch.from_numpy(fr["i16"]).to(dev), "das", -1, want=("rf", "env", "log"))
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    ref = oracle.das(gs, fr["i16"], -1, parallel=True)
    res = _plane_errors(gpu, ref)
    res.update({"rf_storage": "int16", "sample": "whole image"})
    return res


def other_modes(dev, torch, steps: int, warmup: int, check: bool = True) -> dict:
    """DMAS and pDAS (p = 2) kernels on the DMAS workload (128 ch, 512 x 512 at
    dz = 25 um, int16 RF) and pDAS on the 11-angle compound workload (FP32 RF):
    kernel time from HIP events, the frame rate of the whole path (band-pass,
    envelope and log for the DMAS workload; envelope and log for compound), and
    the roofline fraction of each kernel with its own algorithmic op count."""
    from paper_2311_00482_amd import GeometryArg, beamform
    from synth import config_c2, config_c3, make_frame

    # the floor under any launch timed this way: a one-element fill kernel
    tiny = torch.zeros(1, device=dev)
    _, flat, _ = time_steps(lambda: tiny.zero_(), 200, 20, torch)
    floor_ms = float(np.mean(flat))
    res = {"launch_floor": {"kernel_ms": floor_ms, "what": "HIP-event duration of a "
                            "one-element fill kernel, timed like the kernels below"}}
    cases = [("dmas_128ch_512x512", config_c2(), "dmas", True, "c1", True),
             ("pdas_p2_128ch_512x512", config_c2(), "pdas", True, "c1", True),
             ("pdas_p2_compound_11a_1024x1024", config_c3(), "pdas", False, "c3", False)]
    for name, gs, mode, bp, kind, quant in cases:
        g = GeometryArg(gs, bandpass=bp, pdas_p=2.0)
        fr = make_frame(gs, 1001 if kind == "c1" else 1003, kind, quantize=quant)
        rf = torch.from_numpy(fr["i16"] if quant else fr["f32"]).to(dev)
        want = ("rf", "filtered", "env", "log") if bp else ("rf", "env", "log")
        outs = {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in want}
        ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
        rf_only = {"rf": outs["rf"]}
        n = max(20, steps // 3)
        wall, lat, _ = time_steps(
            lambda: beamform(g, rf, mode, -1, want=want, out=outs, workspace=ws, bandpass=bp),
            n, max(5, warmup // 3), torch)
        _, klat, _ = time_steps(lambda: beamform(g, rf, mode, -1, want=("rf",), out=rf_only),
                                n, max(5, warmup // 3), torch)
        k_ms = float(np.mean(klat))  # average launch duration (HIP events around each launch)
        ops = algorithmic_ops(gs, mode)
        res[name] = {"frames_per_s": n / wall, "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "kernel_ms": k_ms,
                     "value": gs.gathers / (k_ms * 1e-3) / 1e9, "unit": UNIT,
                     "roofline": {"bound": "alu", "achieved": ops / (k_ms * 1e-3) / 1e12,
                                  "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "Tlane-op/s",
                                  "frac": ops / (k_ms * 1e-3) / VALU_LANE_OPS_PEAK,
                                  "ops_per_launch": ops,
                                  # the same with the launch floor taken off the time
                                  "frac_above_launch_floor":
                                      ops / (max(k_ms - floor_ms, 1e-6) * 1e-3)
                                      / VALU_LANE_OPS_PEAK},
                     "rf_storage": "int16" if quant else "f32"}
        if check:
            res[name]["error_vs_oracle"] = _mode_error(gs, fr, mode, quant, rf_only["rf"])
        print(f"[bench] {name}: {res[name]['kernel_ms']:.3f} ms kernel, "
              f"frac {res[name]['roofline']['frac']:.2f}", file=sys.stderr, flush=True)
    res.update(iq_modes(dev, torch, steps, warmup))
    res.update(fk_mode(dev, torch, steps, warmup))
    return res


def fk_windows(gs, method: str):
    """Per angle, the columns and rows of the migrated image that the pixel grid
    reads (the library's window rule: the floor of the extreme tap positions, one
    more for the upper tap, one more on each side, clipped to the image)."""
    n, nt = gs.n_channels, gs.n_samples
    nx = 1
    while nx < (4 if method == "lu" else 2) * n:
        nx *= 2
    p = (gs.elem_x[-1] - gs.elem_x[0]) / (n - 1)
    xf = gs.elem_x[0]

    def win(v0, di, ni, dk, nk, size):
        vs = [v0, v0 + (ni - 1) * di, v0 + (nk - 1) * dk, v0 + (ni - 1) * di + (nk - 1) * dk]
        a = max(0.0, math.floor(min(vs)) - 1.0)
        b = min(size - 1.0, math.floor(max(vs)) + 2.0)
        return int(b - a) + 1 if a <= b else 0

    out = []
    for th in gs.angles_rad:
        if method == "lu":
            kz = 2.0 * gs.fs / gs.c
            nc = win((gs.x0 - xf) / p, gs.dx / p, gs.nx, 0.0, gs.nz, nx)
        else:
            v = gs.c / (math.sqrt(2.0) * math.cos(th) ** 2)
            kz = math.sqrt(2.0) / math.cos(th) / (v / gs.fs)
            tn = math.tan(th)
            nc = win((gs.x0 + gs.z0 * tn - xf) / p, gs.dx / p, gs.nx, gs.dz * tn / p, gs.nz, nx)
        nr = win(gs.z0 * kz, 0.0, gs.nx, gs.dz * kz, gs.nz, nt)
        out.append((nc, nr) if nc and nr else (0, 0))
    return nx, out


def fk_stage_bytes(gs, rf_bytes: int, method: str = "stolt") -> float:
    """HBM bytes of one f-k call as staged, each stage reading its input and
    writing its output once: the RF; the temporal spectra T (written, read); the
    2-D spectra P (written, read once by the remap); the remapped spectra U of
    the window's columns (written, read); the window of the migrated images M
    (written, read); the three output planes. The array is padded to 2 N
    (Stolt) or 4 N (Lu)."""
    nx, wins = fk_windows(gs, method)
    kb = gs.n_samples // 2 + 1
    t = gs.n_angles * gs.n_channels * kb * 8
    pp = gs.n_angles * kb * nx * 8
    u = sum(nc for nc, _ in wins) * kb * 8
    m = sum(nc * nr for nc, nr in wins) * 8
    return float(rf_bytes + 2 * t + 2 * pp + 2 * u + 2 * m + 3 * gs.nx * gs.nz * 4)


def fk_mode(dev, torch, steps: int, warmup: int) -> dict:
    """Stolt's and Lu's f-k migrations on the 11-angle compound workload (FP32 RF,
    1024 x 1024 pixels): the whole call (six kernels over all angles at once,
    plus the log image), timed with HIP events around each call, with the staged
    traffic per call over the call time as an HBM fraction. That roofline does
    not bind these calls: counter passes put them at 0.56 (Stolt) and 0.71 (Lu)
    of the VALU issue peak over their kernels, Lu's remap at 0.87
    (profiles/fk_c3_compound_f32.sq.md)."""
    from paper_2311_00482_amd import GeometryArg, fk_migrate, fk_workspace_bytes
    from synth import config_c3, make_frame

    gs = config_c3()
    g = GeometryArg(gs)
    rf = torch.from_numpy(make_frame(gs, 1003, "c3", quantize=False)["f32"]).to(dev)
    want = ("rf", "imag", "env", "log")
    outs = {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in want}
    res = {}
    for method in ("stolt", "lu"):
        ws = torch.empty(fk_workspace_bytes(g, want, -1, method), dtype=torch.uint8, device=dev)
        n = max(20, steps // 3)
        wall, lat, _ = time_steps(lambda: fk_migrate(g, rf, -1, want=want, out=outs,
                                                     workspace=ws, method=method),
                                  n, max(5, warmup // 3), torch)
        ms = float(np.mean(lat))
        b = fk_stage_bytes(gs, rf.numel() * 4, method)
        name = f"fk_{method}_compound_11a_1024x1024"
        res[name] = {"frames_per_s": n / wall, "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "call_ms": ms,
                     "roofline": {"bound": "hbm", "achieved": b / (ms * 1e-3) / 1e9,
                                  "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                  "frac": b / (ms * 1e-3) / HBM_PEAK, "bytes_per_call": b,
                                  "scope": "whole call (six kernels + log image)",
                                  "binding": "VALU issue (counter passes in "
                                             "profiles/fk_c3_compound_f32.sq.md), not HBM"},
                     "workspace_bytes": int(ws.numel()), "rf_storage": "f32"}
        print(f"[bench] {name}: {ms:.3f} ms per call, "
              f"frac {res[name]['roofline']['frac']:.2f}", file=sys.stderr, flush=True)
        del ws
    return res


def iq_modes(dev, torch, steps: int, warmup: int) -> dict:
    """The IQ path on the 11-angle compound workload (FP32 RF): the demodulation
    kernel (HBM-bound: reads the RF once, writes 8-byte complex samples), and
    IQ-DAS / BB-DMAS from the demodulated records (kernel time, roofline, and the
    frame rate of demodulation + beamforming + log), and IQ-DAS from records
    decimated by 2 (the same algorithmic operations on half the samples)."""
    from paper_2311_00482_amd import GeometryArg, beamform, iq_demodulate
    from synth import config_c3, make_frame

    gs = config_c3()
    g = GeometryArg(gs)
    rf = torch.from_numpy(make_frame(gs, 1003, "c3", quantize=False)["f32"]).to(dev)
    iq = iq_demodulate(g, rf)
    n = max(20, steps // 3)
    w = max(5, warmup // 3)
    _, dlat, _ = time_steps(lambda: iq_demodulate(g, rf, out=iq), n, w, torch)
    d_ms = float(np.mean(dlat))
    bytes_moved = rf.numel() * 4 + iq.numel() * 8
    res = {"iq_demod_11a_128ch_4096": {
        "kernel_ms": d_ms, "records": gs.n_angles * gs.n_channels,
        "roofline": {"bound": "hbm", "achieved": bytes_moved / (d_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": bytes_moved / (d_ms * 1e-3) / HBM_PEAK,
                     "bytes_per_launch": float(bytes_moved)}}}
    want = ("rf", "imag", "env", "log")
    outs = {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in want}
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    rf_only = {"rf": outs["rf"], "imag": outs["imag"]}
    g2 = GeometryArg(gs, iq_decimation=2)
    iq2 = iq_demodulate(g2, rf)
    for mode, gg, q, tag in (("iqdas", g, iq, ""), ("bbdmas", g, iq, ""),
                             ("iqdas", g2, iq2, "_decim2")):
        def frame():
            iq_demodulate(gg, rf, out=q)
            beamform(gg, q, mode, -1, want=want, out=outs, workspace=ws)
        wall, lat, _ = time_steps(frame, n, w, torch)
        _, klat, _ = time_steps(lambda: beamform(gg, q, mode, -1, want=("rf", "imag"),
                                                 out=rf_only), n, w, torch)
        k_ms = float(np.mean(klat))
        ops = algorithmic_ops(gs, mode)
        name = f"{mode}{tag}_compound_11a_1024x1024"
        res[name] = {"frames_per_s": n / wall, "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "kernel_ms": k_ms,
                     "value": gs.gathers / (k_ms * 1e-3) / 1e9, "unit": UNIT,
                     "roofline": {"bound": "alu", "achieved": ops / (k_ms * 1e-3) / 1e12,
                                  "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "Tlane-op/s",
                                  "frac": ops / (k_ms * 1e-3) / VALU_LANE_OPS_PEAK,
                                  "ops_per_launch": ops},
                     "rf_storage": "f32 -> complex64 IQ" + (", decimated by 2" if tag else "")}
        print(f"[bench] {name}: {k_ms:.3f} ms kernel, frac {res[name]['roofline']['frac']:.2f}",
              file=sys.stderr, flush=True)
    return res


def image_metrics(dev, torch, g, gs, phantom, env32, env16) -> dict:
    """CR / CNR (Eqs. 5-6) of the phantom's anechoic cysts and the FWHM of its
    point targets on the FP32- and FP16-stored frames' envelopes, with the
    metric kernels' time (HIP events, mean of 20 launches each)."""
    from paper_2311_00482_amd import _abi
    from paper_2311_00482_amd import contrast_metrics, resolution_metrics
    import ctypes

    from synth.phantom import cyst_regions
    cysts = cyst_regions(gs, phantom)
    targets = [(float(x), float(z), 1.0e-3) for x, z in phantom.points]
    res = {}
    for name, env in (("f32", env32), ("f16", env16)):
        c = contrast_metrics(g, env, cysts)
        t = resolution_metrics(g, env, targets)
        fx = [v["fwhm_x"] for v in t if v["fwhm_x"] == v["fwhm_x"]]
        fz = [v["fwhm_z"] for v in t if v["fwhm_z"] == v["fwhm_z"]]
        res[name] = {"cr_db": [v["cr_db"] for v in c], "cnr": [v["cnr"] for v in c],
                     "fwhm_x_mm_median": float(np.median(fx)) * 1e3 if fx else None,
                     "fwhm_z_mm_median": float(np.median(fz)) * 1e3 if fz else None}
    # kernel time
    L = _abi.lib()
    arr_c = (_abi.Cyst * len(cysts))(*[_abi.Cyst(_abi.Disc(*a), _abi.Disc(*b)) for a, b in cysts])
    arr_t = (_abi.Disc * len(targets))(*[_abi.Disc(*t) for t in targets])
    out = torch.empty(4096, dtype=torch.uint8, device=dev)
    stream = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    _, lc, _ = time_steps(lambda: L.pwbf_contrast_metrics(g.ref, env32.data_ptr(), arr_c,
                                                          len(cysts), out.data_ptr(), stream),
                          20, 3, torch)
    _, lt, _ = time_steps(lambda: L.pwbf_resolution_metrics(g.ref, env32.data_ptr(), arr_t,
                                                            len(targets), out.data_ptr(), stream),
                          20, 3, torch)
    res["contrast_kernel_ms"] = float(np.mean(lc))
    res["resolution_kernel_ms"] = float(np.mean(lt))
    res["regions"] = {"cysts": len(cysts), "targets": len(targets)}
    return res


def uneven_batch(dev, torch, steps: int, warmup: int, check: bool = False) -> dict:
    """The uneven 32-frame workload (seeded: 64/128 channels, 1/5/11 angles,
    grids 256..1024 per axis, 2048/4096 samples, DAS and DMAS with band-pass,
    int16 RF, RF + envelope + log per frame) as one tuned batch launch, against
    the same frames launched one after another as single frames with default
    launch shapes. The RF is seeded noise of the frames' shapes: the kernels'
    time does not depend on the values. The roofline fraction divides the
    frames' algorithmic operations (the single-frame op model) by the whole
    launch's time, post-processing included. With check, the raw planes of the
    four frames cheapest to evaluate are compared with the oracle."""
    import oracle
    from paper_2311_00482_amd import Batch, FrameSpec, GeometryArg, beamform
    from synth import config_c4_frames

    specs = config_c4_frames()
    want = ("rf", "filtered", "env", "log")
    gen = torch.Generator().manual_seed(2000)
    frames, singles, gathers, ops = [], [], 0, 0.0
    for sp in specs:
        bp = sp.mode == "dmas"
        g = GeometryArg(sp.geom, bandpass=bp)
        w = want if bp else ("rf", "env", "log")
        shape = (sp.geom.n_angles, sp.geom.n_channels, sp.geom.n_samples)
        rf = torch.randint(-511, 512, shape, generator=gen, dtype=torch.int16).to(dev)
        out = {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in w}
        frames.append(FrameSpec(g, rf, sp.mode, -1, out, bp))
        ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
        singles.append((g, rf, sp.mode, w, out, ws, bp))
        gathers += sp.geom.gathers
        ops += algorithmic_ops(sp.geom, sp.mode)
    t0 = time.perf_counter()
    batch = Batch(frames, tune=True)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    info = batch.describe()
    n = max(5, steps // 32)
    wallb, latb, _ = time_steps(batch.launch, n, max(2, warmup // 16), torch)
    ms_b = float(np.mean(latb))
    err = None
    if check:
        err = _uneven_errors(specs, frames, batch, torch)

    def one_by_one():
        for g, rf, mode, w, out, ws, bp in singles:
            beamform(g, rf, mode, -1, want=w, out=out, workspace=ws, bandpass=bp)
    walls, lats, _ = time_steps(one_by_one, n, max(2, warmup // 16), torch)
    batch.close()
    nf = len(specs)
    res = {"frames": nf, "tuned_create_s": t_create, "kernels": info["kernels"],
           "branches": info.get("branches"),
           "batched": {"frames_per_s": nf * n / wallb, "ms_per_launch": ms_b,
                       "value": gathers * n / wallb / 1e9, "unit": UNIT},
           "roofline": {"bound": "alu", "achieved": ops / (ms_b * 1e-3) / 1e12,
                        "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "Tlane-op/s",
                        "frac": ops / (ms_b * 1e-3) / VALU_LANE_OPS_PEAK,
                        "ops_per_launch": ops,
                        "scope": "whole graph launch (beamform, band-pass, envelope, log)"},
           "single_frames": {"frames_per_s": nf * n / walls,
                             "ms_per_32": float(np.mean(lats)),
                             "value": gathers * n / walls / 1e9, "unit": UNIT}}
    if err is not None:
        res["error_vs_oracle"] = err
    return res


def _uneven_errors(specs, frames, batch, torch) -> dict:
    """Raw planes of the four frames cheapest to evaluate against the oracle on
    the same int16 samples: first on the timing run's uniform-noise RF, beside
    how far the float64 definition itself moves when every delay shifts by
    3e-8 samples (below the resolution of a float32 delay: the root of DMAS is
    steep at the near-zero samples that incoherent content has, so that move is
    the float32 floor there); then on the simulated phantom frames of the same
    shapes (the batch relaunched on them)."""
    import dataclasses
    import oracle
    from synth import make_frame
    cheap = sorted(range(len(specs)), key=lambda i: specs[i].geom.gathers)[:4]

    def ref_of(sp, host, g=None):
        g = g or sp.geom
        if sp.mode == "dmas":
            return oracle.dmas(g, host, -1, "identity", parallel=True)
        return oracle.das(g, host, -1, parallel=True)

    def name(i):
        g = specs[i].geom
        return f"frame{i}_{specs[i].mode}_{g.n_angles}a_{g.n_channels}ch_{g.nx}x{g.nz}"

    noise, floor, phantom = {}, {}, {}
    for i in cheap:
        sp = specs[i]
        host = frames[i].rf.cpu().numpy()
        ref = ref_of(sp, host)
        noise[name(i)] = _max_norm(frames[i].out["rf"].cpu().numpy(), ref)
        shifted = dataclasses.replace(sp.geom, t0=tuple(3e-8 / sp.geom.fs for _ in sp.geom.angles_deg))
        floor[name(i)] = _max_norm(ref_of(sp, host, shifted), ref)
    sims = {i: make_frame(specs[i].geom, specs[i].seed, "scaled") for i in cheap}
    for i in cheap:
        frames[i].rf.copy_(torch.from_numpy(sims[i]["i16"]))
    batch.launch()
    torch.cuda.synchronize()
    for i in cheap:
        phantom[name(i)] = _max_norm(frames[i].out["rf"].cpu().numpy(),
                                     ref_of(specs[i], sims[i]["i16"]))
    return {"rf": phantom, "content": "simulated phantom frames (points and cysts in speckle)",
            "white_noise_rf": noise,
            "definition_move_at_3e-8_sample_delay_shift": floor,
            "sample": "whole images of the four frames cheapest to evaluate",
            "rf_storage": "int16"}


def _serve_rate(srv, hosts, n_probes, rate, seconds, warmup, rng, keep=None):
    """Poisson arrivals at rate for warmup + seconds; requests arriving in the
    first warmup seconds are served but not counted. keep(r, srv) may copy a
    result's planes before its release."""
    from paper_2311_00482_amd import PwbfError
    horizon = warmup + seconds
    n = int(rate * horizon * 1.2) + 16
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    arrivals = arrivals[arrivals < horizon]
    n = len(arrivals)
    which = rng.integers(0, n_probes, n)
    t0 = srv.now() + 0.01
    t_measure = t0 + warmup
    before = None
    lat, parts, quality, k, accepted, done = [], [], [], 0, 0, 0
    limit = time.time() + horizon + 60
    while k < n or done < accepted:
        if time.time() > limit:
            raise RuntimeError(f"serving run at {rate}/s did not drain")
        now = srv.now()
        if before is None and now >= t_measure:
            before = srv.stats()
        while k < n and t0 + arrivals[k] <= now:
            try:
                srv.submit(int(which[k]), hosts[which[k]], t0 + arrivals[k])
                accepted += 1
            except PwbfError as e:  # a full probe queue drops the request
                if e.code != -5:
                    raise
            k += 1
        got = srv.poll(64, wait_ms=0 if k < n else 5)
        for r in got:
            done += 1
            if r.t_arrival >= t_measure:
                lat.append(r.t_done - r.t_arrival)
                parts.append((r.t_admit - r.t_arrival, r.t_launch - r.t_admit,
                              r.t_done - r.t_launch))
                if srv.probes[r.probe].quality_region is not None:
                    quality.append(r.quality_ok)
            if keep is not None:
                keep(r, srv)
            srv.release(r.id)
        if not got and k < n:  # sleep only when the next arrival is far off
            gap = t0 + arrivals[k] - srv.now()
            if gap > 3e-3:  # host sleeps can overshoot by a millisecond or more
                time.sleep(gap - 2e-3)
    after = srv.stats()
    before = before or after
    wall = seconds
    pq = np.percentile(np.array(parts) * 1e3, 50, axis=0)
    pq99 = np.percentile(np.array(parts) * 1e3, 99, axis=0)
    return {"offered_per_s": rate, "measured_s": seconds, "warmup_s": warmup,
            "requests": len(lat), "completed_per_s": len(lat) / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "p50_parts_ms": {"queue": float(pq[0]), "upload": float(pq[1]), "gpu": float(pq[2])},
            "p99_parts_ms": {"queue": float(pq99[0]), "upload": float(pq99[1]),
                             "gpu": float(pq99[2])},
            "mean_batch": (after["completed"] - before["completed"])
            / max(1, after["batches"] - before["batches"]),
            "rejected": after["rejected"] - before["rejected"],
            "quality_pass": float(np.mean(quality)) if quality else None}


def systems(dev, torch, steps: int, warmup: int, check: bool = False,
            serve_seconds: float = 10.0, serve_warmup: float = 1.0) -> dict:
    """Single-frame FP32 against batched FP32, batched FP16 and served FP16 on
    the same GPU.

    The RF is the 11-angle frame quantised to 10-bit int16, which FP16 holds
    exactly, so every form computes on identical sample values (equal accuracy
    by construction; the batched planes are checked against the single-frame
    ones). Batched: B frames of the workload (the frame rolled along samples so
    each is distinct) in one graph launch, FP32- and FP16-stored (the FP32
    batch isolates what the storage type contributes). Served: four probes
    (1 angle 64 ch 256x512; 5 angles 128 ch 512x512; the 11-angle 1024x1024
    workload, with a quality check of its first cyst on every frame; DMAS 64 ch
    512x512) under Poisson arrivals at 500, 1000, 2000, 3500 and 5000 frames/s,
    each a measured window after a warm-up, int16 RF uploaded from pinned host
    memory per request; latency = done - arrival.
    """
    import oracle
    from paper_2311_00482_amd import Batch, FrameSpec, GeometryArg, ProbeSpec, Server, beamform
    from synth import config_c3, config_c5_probes, make_frame
    from synth.phantom import cyst_regions

    gs = config_c3()
    g = GeometryArg(gs)
    want = ("rf", "env", "log")
    i16 = torch.from_numpy(make_frame(gs, 1003, "c3", quantize=True)["i16"])

    def planes():
        return {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in want}

    out32 = planes()
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)
    rf32 = i16.to(torch.float32).to(dev)
    wall32, lat32, _ = time_steps(
        lambda: beamform(g, rf32, "das", -1, want=want, out=out32, workspace=ws),
        steps, warmup, torch)
    res = {"single_frame_f32": {"frames_per_s": steps / wall32,
                                "p50_ms": float(np.percentile(lat32, 50)),
                                "p99_ms": float(np.percentile(lat32, 99))}}
    del rf32

    B = 8
    nb = max(10, steps // B)
    for name, dt in (("batched_f32", torch.float32), ("batched_f16", torch.float16)):
        frames = [FrameSpec(g, torch.roll(i16, 17 * k, dims=2).to(dt).to(dev), "das", -1,
                            planes()) for k in range(B)]
        batch = Batch(frames)
        wallb, latb, _ = time_steps(batch.launch, nb, max(2, warmup // B), torch)
        dev_max = max(float((frames[0].out[k] - out32[k]).abs().max()
                            / out32[k].abs().max().clamp_min(1e-30)) for k in ("rf", "env"))
        res[name] = {"frames_per_launch": B, "frames_per_s": B * nb / wallb,
                     "ms_per_launch": float(np.percentile(latb, 50)),
                     "max_rel_diff_vs_single_f32": dev_max}
        batch.close()
        del frames
    res["f16_storage_gain_batched"] = (res["batched_f16"]["frames_per_s"]
                                       / res["batched_f32"]["frames_per_s"])

    res["uneven_batch_32"] = uneven_batch(dev, torch, steps, warmup, check=check)
    ub = res["uneven_batch_32"]
    print(f"[bench] uneven batch: {ub['batched']['ms_per_launch']:.3f} ms per launch, "
          f"frac {ub['roofline']['frac']:.2f}", file=sys.stderr, flush=True)

    specs = config_c5_probes()
    hosts, phantoms = [], []
    for k, sp in enumerate(specs):
        kind = "c3" if sp.geom.name == "probe_c" else "scaled"
        f = make_frame(sp.geom, sp.seed, kind, quantize=True)
        hosts.append(torch.from_numpy(f["i16"]).pin_memory())
        phantoms.append(f["phantom"])
    probe_specs = []
    for sp, ph in zip(specs, phantoms):
        region = cyst_regions(sp.geom, ph)[0] if sp.geom.name == "probe_c" else None
        probe_specs.append(ProbeSpec(sp.geom, sp.mode, -1, want, 8,
                                     bandpass=(sp.mode == "dmas"), quality_region=region,
                                     quality_max_cr_db=-10.0))
    srv = Server(probe_specs)
    rng = np.random.default_rng(42)
    kept = {}

    def keep(r, s):  # the first result of each probe, for the accuracy check
        if check and r.status == 0 and r.probe not in kept:
            kept[r.probe] = {k: v.cpu().numpy() for k, v in s.planes(r).items()}

    served = []
    try:
        for rate in (500.0, 1000.0, 2000.0, 3500.0, 5000.0):
            served.append(_serve_rate(srv, hosts, len(specs), rate, serve_seconds,
                                      serve_warmup, rng, keep))
            print(f"[bench] served {rate:.0f}/s: {served[-1]}", file=sys.stderr, flush=True)
    finally:
        srv.close()
    res["served_f16"] = {"probes": [sp.geom.name for sp in specs], "runs": served,
                         "quality_check": "probe_c: frame maximum > 0 and CR of its first "
                                          "cyst <= -10 dB, per request"}
    if check:
        err = {}
        for i, sp in enumerate(specs):
            if i not in kept:
                continue
            host = hosts[i].numpy()
            whole = sp.geom.nx * sp.geom.nz <= 512 * 512
            cols, pix = _columns(sp.geom, sp.geom.nx if whole else 64)
            if sp.mode == "dmas":
                ref = oracle.dmas(sp.geom, host, -1, "identity", pix, parallel=True)
            else:
                ref = oracle.das(sp.geom, host, -1, pix, parallel=True)
            err[sp.geom.name] = _max_norm(kept[i]["rf"][cols], ref.reshape(len(cols),
                                                                          sp.geom.nz))
        res["served_f16"]["error_vs_oracle"] = {
            "rf": err, "sample": "whole image (64 depth columns for 1024 x 1024)",
            "rf_storage": "int16 uploaded, FP16 on the device"}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--no-systems", action="store_true",
                    help="skip the batched and served FP16 measurements")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the DMAS and pDAS measurements")
    ap.add_argument("--profile-mode", default="das",
                    choices=("das", "pdas", "dmas", "iqdas", "bbdmas", "fk", "fklu", "batch",
                             "uneven"),
                    help="with --profile-only: the beamformer of the timed loop (dmas and "
                         "pdas run on the 128-channel 512 x 512 DMAS workload, pdas also "
                         "takes the compound workload with --profile-compound)")
    ap.add_argument("--profile-compound", action="store_true")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--clock-ramp", type=float, default=RAMP_S,
                    help="seconds of untimed steps before each warm-up, so that the "
                         "device's clocks have settled when the timed steps start")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle: no CPU baseline and no accuracy figures")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="measured seconds per arrival rate of the serving run")
    ap.add_argument("--serve-warmup", type=float, default=1.0,
                    help="seconds of arrivals before each measured serving window")
    ap.add_argument("--cpu-budget", type=float, default=8.0,
                    help="seconds of oracle work per CPU baseline leg")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the timed FP32 compound loop (for rocprofv3)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run 3 plain device-to-device copies of this many MiB "
                         "(a reference kernel for calibrating HBM byte counters)")
    args = ap.parse_args()
    globals()["RAMP_S"] = args.clock_ramp
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(frames would be sharded across GPUs with no exchange); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2311_00482_amd import GeometryArg, beamform, describe_plan
    from synth import config_c3, make_frame

    dev = torch.device("cuda:0")
    g = GeometryArg(config_c3())  # marshalled once, as a caller streaming frames would
    gs = config_c3()
    print(f"[bench] simulating {gs.name}", file=sys.stderr, flush=True)
    fr = make_frame(gs, 1003, "c3", quantize=False)
    rf32 = torch.from_numpy(fr["f32"]).to(dev)
    rf16 = torch.from_numpy(fr["f16"]).to(dev)
    want = ("rf", "env", "log")
    outs = {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in want}
    ws = torch.empty(WS_BYTES, dtype=torch.uint8, device=dev)

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

    if args.profile_only and args.profile_mode == "uneven":
        r = uneven_batch(dev, torch, args.steps * 32, args.warmup * 16)
        print(json.dumps({"profile_only": True, "mode": "uneven",
                          "ms_per_launch": r["batched"]["ms_per_launch"]}))
        return
    if args.profile_only and args.profile_mode == "batch":
        from paper_2311_00482_amd import Batch, FrameSpec
        i16 = torch.from_numpy(fr["i16"]) if "i16" in fr else rf32.cpu().round().to(torch.int16)
        wantb = ("rf", "env", "log")
        frames = [FrameSpec(g, torch.roll(i16, 17 * k, dims=2).to(torch.float16).to(dev), "das",
                            -1, {k2: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev)
                                 for k2 in wantb}) for k in range(8)]
        batch = Batch(frames)
        wall, _, _ = time_steps(batch.launch, args.steps, args.warmup, torch)
        batch.close()
        print(json.dumps({"profile_only": True, "mode": "batch", "frames_per_launch": 8,
                          "ms_per_step": wall / args.steps * 1e3}))
        return
    if args.profile_only and args.profile_mode in ("fk", "fklu"):
        from paper_2311_00482_amd import fk_migrate, fk_workspace_bytes
        meth = "lu" if args.profile_mode == "fklu" else "stolt"
        wantk = ("rf", "imag", "env", "log")
        outk = {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in wantk}
        wsk = torch.empty(fk_workspace_bytes(g, wantk, -1, meth), dtype=torch.uint8, device=dev)
        wall, _, _ = time_steps(lambda: fk_migrate(g, rf32, -1, want=wantk, out=outk,
                                                   workspace=wsk, method=meth),
                                args.steps, args.warmup, torch)
        print(json.dumps({"profile_only": True, "mode": args.profile_mode,
                          "ms_per_step": wall / args.steps * 1e3}))
        return
    if args.profile_only and args.profile_mode in ("iqdas", "bbdmas"):
        from paper_2311_00482_amd import iq_demodulate
        iq = iq_demodulate(g, rf32)
        wantq = ("rf", "imag", "env", "log")
        outq = {k: torch.empty((g.nx, g.nz), dtype=torch.float32, device=dev) for k in wantq}

        def iq_step():
            iq_demodulate(g, rf32, out=iq)
            beamform(g, iq, args.profile_mode, -1, want=wantq, out=outq, workspace=ws)
        wall, _, _ = time_steps(iq_step, args.steps, args.warmup, torch)
        print(json.dumps({"profile_only": True, "mode": args.profile_mode,
                          "ms_per_step": wall / args.steps * 1e3}))
        return
    if args.profile_only and args.profile_mode != "das":
        from synth import config_c2
        if args.profile_mode == "pdas" and args.profile_compound:
            gp, rfp, bp = GeometryArg(gs, pdas_p=2.0), rf32, False
        else:
            g2 = config_c2()
            gp, bp = GeometryArg(g2, bandpass=True, pdas_p=2.0), True
            rfp = torch.from_numpy(make_frame(g2, 1001, "c1")["i16"]).to(dev)
        wantp = ("rf", "filtered", "env", "log") if bp else ("rf", "env", "log")
        outp = {k: torch.empty((gp.nx, gp.nz), dtype=torch.float32, device=dev) for k in wantp}
        wall, _, _ = time_steps(lambda: beamform(gp, rfp, args.profile_mode, -1, want=wantp,
                                                 out=outp, workspace=ws, bandpass=bp),
                                args.steps, args.warmup, torch)
        print(json.dumps({"profile_only": True, "mode": args.profile_mode,
                          "ms_per_step": wall / args.steps * 1e3}))
        return
    print("[bench] timing FP32-stored RF (headline)", file=sys.stderr, flush=True)
    wall, lat, span = time_steps(step32, args.steps, args.warmup, torch)
    if args.profile_only:
        print(json.dumps({"profile_only": True, "ms_per_step": wall / args.steps * 1e3}))
        return
    print("[bench] timing FP16-stored RF", file=sys.stderr, flush=True)
    wall16, lat16, _ = time_steps(step16, args.steps, args.warmup, torch)
    print("[bench] timing the beamform kernel alone", file=sys.stderr, flush=True)
    _, klat, _ = time_steps(kernel_only, args.steps, args.warmup, torch)
    k_ms = float(np.mean(klat))  # average launch duration (HIP events around each launch)

    gathers = gs.gathers
    value = gathers * args.steps / wall / 1e9
    ops = algorithmic_ops(gs)
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
                   "rf_storage": "f32", "pixels": gs.nx * gs.nz, "channels": gs.n_channels,
                   "angles": gs.n_angles, "samples": gs.n_samples,
                   "tile": {k: plan[k] for k in ("cpw", "lz", "wz", "wx", "tile_z", "tile_x",
                                                  "chunk", "win")}},
        "clock_ramp_s": args.clock_ramp,
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
                "gather_effective_frac": gathers * 2 * 4 / (k_ms * 1e-3) / HBM_PEAK,
                # the counters' HBM bytes over the kernel's time: why the VALU
                # roofline, not HBM, is the binding one for this kernel
                "measured_GBps": None if traffic is None else traffic / (k_ms * 1e-3) / 1e9,
                "measured_frac": None if traffic is None else traffic / (k_ms * 1e-3) / HBM_PEAK,
                "binding": "VALU issue: the kernel issues VALU work in every slot (SQ "
                           "counters) while its measured HBM traffic uses a few percent "
                           "of the peak; each RF line is staged once per tile and reread "
                           "from LDS and L2 (85% L2 hits)"},
        "variants": {"f16_storage": {"value": gathers * args.steps / wall16 / 1e9,
                                     "frames_per_s": args.steps / wall16,
                                     "latency_ms": {"p50": float(np.percentile(lat16, 50)),
                                                    "p99": float(np.percentile(lat16, 99))}}},
    }
    print("[bench] image metrics", file=sys.stderr, flush=True)
    env16 = torch.empty_like(outs["env"])
    beamform(g, rf16, "das", -1, want=("rf", "env"), out={"rf": torch.empty_like(env16),
                                                           "env": env16})
    beamform(g, rf32, "das", -1, want=want, out=outs, workspace=ws)
    torch.cuda.synchronize()
    line["image_metrics"] = image_metrics(dev, torch, g, gs, fr["phantom"], outs["env"], env16)
    if not args.no_modes:
        print("[bench] DMAS and pDAS", file=sys.stderr, flush=True)
        line["modes"] = other_modes(dev, torch, args.steps, args.warmup,
                                    check=not args.no_cpu_baseline)
    if not args.no_systems:
        print("[bench] batched and served FP16 vs single-frame FP32", file=sys.stderr, flush=True)
        line["systems"] = systems(dev, torch, args.steps, args.warmup,
                                  check=not args.no_cpu_baseline,
                                  serve_seconds=args.serve_seconds,
                                  serve_warmup=args.serve_warmup)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        cb, sample = cpu_baseline(gs, fr["master"], args.cpu_budget)
        line["cpu_baseline"] = cb
        print("[bench] accuracy against the oracle", file=sys.stderr, flush=True)
        step32()
        gpu32 = {k: v.cpu().numpy() for k, v in outs.items()}
        step16()
        gpu16 = {k: v.cpu().numpy() for k, v in outs.items()}
        err = error_vs_oracle(gs, fr, sample, gpu32, gpu16)
        err["single_frame_64ch_128x256"] = c1_error(dev, torch)
        for name, rec in line.get("modes", {}).items():
            if "error_vs_oracle" in rec:
                err[name] = rec["error_vs_oracle"]
        sysrec = line.get("systems", {})
        if "error_vs_oracle" in sysrec.get("uneven_batch_32", {}):
            err["uneven_batch_32"] = sysrec["uneven_batch_32"]["error_vs_oracle"]
        if "error_vs_oracle" in sysrec.get("served_f16", {}):
            err["served_f16"] = sysrec["served_f16"]["error_vs_oracle"]
        line["error_vs_oracle"] = err
    print(json.dumps(line))


if __name__ == "__main__":
    main()
