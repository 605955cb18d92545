"""GPU: the continuous-batching serving loop.

Every serving batch runs one persistent kernel whose per-frame arithmetic
depends only on the probe's plan, fixed when the server is created, never on
which other frames share the launch: a frame's planes must be bitwise equal
alone and in a mix of probes. int16 RF of 10 bits converts to float16
exactly, so the served planes meet the float32 bars against the FP64 oracle.
Admission holds the slot bytes in use under the HBM budget; a full probe queue
rejects with PWBF_E_BUSY; a request still queued at its deadline comes back
with PWBF_E_TIMEOUT and no planes. A probe's per-frame quality check (frame
maximum, CR and CNR of one region, pass or fail against a CR bound) equals the
metrics of the served envelope, checked against the float64 oracle metrics on
that envelope and on the oracle's own envelope (the check combines float32
partial sums per column chunk, so it agrees with the metrics call to rounding).
"""

import time

import numpy as np
import pytest

import oracle
from synth import config_c5_probes, make_frame

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_DB = 0.1
KINDS = {"probe_a": "scaled", "probe_b": "scaled", "probe_c": "c3", "probe_d": "scaled"}


def _torch():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch


@pytest.fixture(scope="module")
def probes():
    """The four serving probes with one simulated int16 frame each (pinned host)."""
    torch = _torch()
    out = []
    for spec in config_c5_probes():
        fr = make_frame(spec.geom, spec.seed, KINDS[spec.geom.name], quantize=True)
        host = torch.from_numpy(fr["i16"]).pin_memory()
        out.append((spec, fr, host))
    return out


def _server(probes, which=None, slots=4, budget=0, max_queue=0, want=("rf", "env", "log")):
    from paper_2311_00482_amd import ProbeSpec, Server
    sel = probes if which is None else [probes[i] for i in which]
    specs = [ProbeSpec(s.geom, s.mode, -1, want, slots, bandpass=(s.mode == "dmas"))
             for s, _, _ in sel]
    return Server(specs, budget, max_queue)


def _collect(srv, n, timeout_s=30.0, release=True):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < n:
        assert time.time() < t_end, f"only {len(got)} of {n} requests completed"
        for r in srv.poll(64, wait_ms=100):
            planes = {k: v.cpu().numpy() for k, v in srv.planes(r).items()}
            got[r.id] = (r, planes)
            if release:
                srv.release(r.id)
    return got


def _err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def test_each_result_same_alone_and_in_the_mix(probes):
    srv = _server(probes)
    try:
        alone = []
        for i, (_, _, host) in enumerate(probes):
            rid = srv.submit(i, host)
            (r, planes), = _collect(srv, 1).values()
            assert r.id == rid and r.probe == i
            alone.append(planes)
        before = srv.stats()
        order = []
        for _ in range(3):
            for i, (_, _, host) in enumerate(probes):
                order.append((srv.submit(i, host), i))
        got = _collect(srv, len(order))
        after = srv.stats()
        for rid, i in order:
            r, planes = got[rid]
            assert r.probe == i
            for k in ("rf", "env", "log"):
                assert np.array_equal(planes[k], alone[i][k]), (i, k)
        # the twelve requests did share launches
        assert after["batches"] - before["batches"] < len(order)
        assert after["completed"] == before["completed"] + len(order)
    finally:
        srv.close()


def test_served_planes_match_the_oracle(probes):
    srv = _server(probes)
    try:
        for i, (_, _, host) in enumerate(probes):
            srv.submit(i, host)
        got = sorted(_collect(srv, len(probes)).values(), key=lambda t: t[0].probe)
    finally:
        srv.close()
    for (spec, fr, _), (r, planes) in zip(probes, got):
        g = spec.geom
        tol = TOL32
        if g.nx * g.nz <= 512 * 512:
            ref = oracle.beamform(g, fr["master"], spec.mode, -1, bandpass=spec.mode == "dmas")
            assert _err(planes["rf"], ref["rf"]) <= tol, spec.geom.name
            assert _err(planes["env"], ref["env"]) <= tol, spec.geom.name
            m = ref["log"] >= -40.0
            assert float(np.abs(planes["log"][m] - ref["log"][m]).max()) <= TOL_DB
        else:
            # full-size compound probe: sampled pixels and two whole depth columns
            rng = np.random.default_rng(11)
            pix = rng.choice(g.nx * g.nz, 2000, replace=False)
            ref = oracle.das(g, fr["master"], -1, pix)
            norm = np.abs(planes["rf"]).max()
            assert float(np.abs(planes["rf"].ravel()[pix] - ref).max() / norm) <= tol
            cols = [g.nx // 3, g.nx // 2]
            col_pix = np.concatenate([np.arange(g.nz) + ix * g.nz for ix in cols])
            env_ref = oracle.envelope_z(oracle.das(g, fr["master"], -1, col_pix)
                                        .reshape(len(cols), g.nz))
            assert float(np.abs(planes["env"][cols] - env_ref).max()
                         / planes["env"].max()) <= tol


def test_budget_admission_and_queue_limit(probes):
    from paper_2311_00482_amd import PwbfError
    spec, _, host = probes[0]
    g = spec.geom
    plane = g.nx * g.nz * 4
    slot_bytes = g.n_angles * g.n_channels * g.n_samples * 2 + 3 * plane + 8192  # + max slots
    srv = _server(probes, [0], slots=4, budget=2 * slot_bytes, max_queue=3)
    try:
        first = srv.submit(0, host)
        (r, _), = _collect(srv, 1, release=False).values()
        assert r.id == first
        second = srv.submit(0, host)
        (r2, _), = _collect(srv, 1, release=False).values()
        assert r2.id == second
        st = srv.stats()
        assert st["budget_in_use"] == 2 * slot_bytes == st["budget_peak"]
        # both slots the budget allows are held: three wait, the fourth is refused
        waiting = [srv.submit(0, host) for _ in range(3)]
        time.sleep(0.05)
        st = srv.stats()
        assert st["queued"] == 3 and st["budget_in_use"] == 2 * slot_bytes
        with pytest.raises(PwbfError) as ei:
            srv.submit(0, host)
        assert ei.value.code == -5
        assert srv.stats()["rejected"] == 1
        srv.release(first)
        srv.release(second)
        got = _collect(srv, 3)
        assert sorted(got) == sorted(waiting)
        st = srv.stats()
        assert st["budget_peak"] <= 2 * slot_bytes and st["budget_in_use"] == 0
        assert st["queued"] == 0 and st["in_flight"] == 0
        with pytest.raises(PwbfError):
            srv.release(first)  # already released
    finally:
        srv.close()


def test_poisson_arrivals_latency_and_order(probes):
    srv = _server(probes, [0, 1, 3], slots=6)
    rng = np.random.default_rng(5)
    n, rate = 150, 1500.0
    gaps = rng.exponential(1.0 / rate, n)
    which = rng.integers(0, 3, n)
    hosts = [probes[i][2] for i in (0, 1, 3)]
    try:
        ids = []
        t_next = srv.now()
        got = {}
        for k in range(n):
            t_next += gaps[k]
            while srv.now() < t_next:
                for r in srv.poll(64, wait_ms=0):
                    got[r.id] = r
                    srv.release(r.id)
            ids.append(srv.submit(int(which[k]), hosts[which[k]], t_next))
        t_end = time.time() + 30
        while len(got) < n:
            assert time.time() < t_end
            for r in srv.poll(64, wait_ms=100):
                got[r.id] = r
                srv.release(r.id)
        st = srv.stats()
    finally:
        srv.close()
    assert sorted(got) == sorted(ids)
    lat = []
    for r in got.values():
        assert r.t_arrival <= r.t_admit <= r.t_launch <= r.t_done
        lat.append(r.t_done - r.t_arrival)
    assert st["completed"] == n and st["rejected"] == 0
    p50, p99 = np.percentile(lat, [50, 99])
    assert 0 < p50 <= p99 < 1.0


def test_close_with_requests_in_flight(probes):
    srv = _server(probes, [2, 3], slots=2)
    for _ in range(3):
        srv.submit(0, probes[2][2])
        srv.submit(1, probes[3][2])
    srv.close()  # stops the scheduler, waits for the device, frees the rings


def _contrast_of(g, env, region):
    from paper_2311_00482_amd import contrast_metrics
    return contrast_metrics(g, env, [region])[0]


def test_quality_check_matches_the_metrics_and_the_oracle(probes):
    """Probe c (the compound benchmark frame with its cysts) served twice: with a
    CR bound of -10 dB the first cyst passes, with -200 dB it fails."""
    from metric_checks import _matching_masks, _regions
    from oracle import metrics as om
    from paper_2311_00482_amd import ProbeSpec, Server
    torch = _torch()
    spec, fr, host = probes[2]
    g = spec.geom
    region = _regions(g, fr["phantom"])[0][0]
    specs = [ProbeSpec(g, "das", -1, ("rf", "env"), 2, quality_region=region,
                       quality_max_cr_db=bound) for bound in (-10.0, -200.0)]
    srv = Server(specs)
    try:
        for i in range(2):
            srv.submit(i, host)
        got = sorted(_collect(srv, 2).values(), key=lambda t: t[0].probe)
        # the same frame again, three at once: the check's per-slot counters and
        # partial buffers are reused and give the same figures every time
        for _ in range(3):
            srv.submit(0, host)
        again = [r for r, _ in _collect(srv, 3).values()]
    finally:
        srv.close()
    for r in again:
        assert (r.frame_max, r.cr_db, r.cnr, r.quality_ok) == (
            got[0][0].frame_max, got[0][0].cr_db, got[0][0].cnr, got[0][0].quality_ok)
    # the oracle's envelope over the columns both discs touch (full depth)
    X, _ = om.pixel_centres(g)
    cols = np.nonzero(np.any([np.abs(X[:, 0] - d[0]) <= d[2] + g.dx for d in region], 0))[0]
    pix = (cols[:, None] * g.nz + np.arange(g.nz)[None, :]).ravel()
    rf_cols = oracle.das(g, fr["master"], -1, pix, parallel=True).reshape(len(cols), g.nz)
    env_ref = np.zeros((g.nx, g.nz))
    env_ref[cols] = oracle.envelope_z(rf_cols)
    for (r, planes), bound in zip(got, (-10.0, -200.0)):
        env = planes["env"]
        assert r.status == 0
        # the frame maximum is the envelope's, bit for bit
        assert r.frame_max == float(env.max())
        # CR and CNR are those of the metrics call on the same plane (the check
        # sums per column chunk and combines the chunks; float32 rounding apart)
        c = _contrast_of(g, torch.from_numpy(env).cuda(), region)
        assert abs(r.cr_db - c["cr_db"]) <= 1e-4
        assert r.cnr == pytest.approx(c["cnr"], rel=1e-5)
        # ... which are the float64 oracle metrics of that plane
        m = _matching_masks(g, env, region, c)
        assert m is not None, (c, om.contrast(g, env, *region))
        ref, mi, mo = m
        # and, within what the envelope's 1e-5 bar allows, of the oracle's envelope
        o = om.contrast_from_masks(env_ref, mi, mo)
        d_env = TOL32 * float(env.max())
        tol_cr = 1.5 * 20.0 / np.log(10.0) * d_env * (1.0 / o["mu_in"] + 1.0 / o["mu_out"])
        s = np.sqrt((o["sigma_in"] ** 2 + o["sigma_out"] ** 2) / 2.0)
        tol_cnr = 1.5 * (2.0 + abs(o["cnr"])) * d_env / s
        assert abs(r.cr_db - o["cr_db"]) <= tol_cr, (r.cr_db, o["cr_db"], tol_cr)
        assert abs(r.cnr - o["cnr"]) <= tol_cnr, (r.cnr, o["cnr"], tol_cnr)
        assert r.quality_ok == (r.frame_max > 0 and r.cr_db <= bound)
    assert got[0][0].quality_ok and not got[1][0].quality_ok
    assert got[0][0].cr_db < -10.0


def test_deadline_expires_queued_requests(probes):
    from paper_2311_00482_amd import PwbfError
    spec, _, host = probes[0]
    srv = _server(probes, [0], slots=1)
    try:
        first = srv.submit(0, host)
        (r, _), = _collect(srv, 1, release=False).values()  # holds the only slot
        late = srv.submit(0, host, deadline=srv.now() + 0.05)
        time.sleep(0.3)
        (e, planes), = _collect(srv, 1, release=False).values()
        assert e.id == late and e.status == -6 and e.slot == -1 and planes == {}
        assert e.rf is None and e.t_done >= e.t_arrival + 0.05
        st = srv.stats()
        assert st["expired"] == 1 and st["completed"] == 1 and st["queued"] == 0
        srv.release(late)  # frees nothing: the slot is still held
        assert srv.stats()["budget_in_use"] == st["budget_in_use"]
        srv.release(first)
        ok = srv.submit(0, host, deadline=srv.now() + 30.0)
        (r2, planes2), = _collect(srv, 1).values()
        assert r2.id == ok and r2.status == 0 and "rf" in planes2
        with pytest.raises(PwbfError):
            srv.submit(0, host, deadline=float("nan"))
    finally:
        srv.close()
