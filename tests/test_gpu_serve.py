"""The request loop: requests that arrive while others are on the GPU are
admitted as memory and slots free up, and each result is bitwise the result
of solving that grid alone."""
import time

import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx

pytestmark = pytest.mark.gpu


def _requests():
    ws = [G.small_random(900, seed=81, n_bins=42, box=3e21, rate=1e48, n_src=1, dt=3e13,
                         precision=G.SX_FP32_TRANSPORT),
          G.small_random(2500, seed=82, n_bins=84, box=3e21, rate=1e48, n_src=3, dt=3e13,
                         precision=G.SX_FP32_TRANSPORT),
          G.small_random(400, seed=83, n_bins=21, box=3e21, rate=1e48, n_src=2, dt=3e13,
                         precision=G.SX_FP64),
          G.config1(),
          G.small_random(1500, seed=84, n_bins=42, box=3e21, rate=1e48, n_src=4, dt=3e13,
                         precision=G.SX_FP32_TRANSPORT)]
    sweeps = [60, 130, 45, 200, 90]
    return ws, sweeps


def _alone(ws, sweeps):
    out = []
    with sx.Context(0) as ctx:
        for w, s in zip(ws, sweeps):
            gid = ctx.upload(w)
            ctx.solve([gid], s)
            out.append(ctx.state(gid, nin=False))
            ctx.free(gid)
    return out


def _serve(ws, sweeps, gap_s=0.02, **opts):
    got = {}
    with sx.Context(0) as ctx:
        srv = sx.Server(ctx, **opts)
        tickets = []
        try:
            for i, (w, s) in enumerate(zip(ws, sweeps)):
                tickets.append(srv.submit(w, s))
                if i >= 1:
                    time.sleep(gap_s)   # later requests arrive while earlier ones run
            for _ in tickets:
                r = srv.poll(timeout=60.0)
                assert r is not None, "a request did not finish within 60 s"
                x, y = srv.take(r["ticket"])
                got[r["ticket"]] = (r, x, y)
        finally:
            stats = srv.stop()
    return [got[t] for t in tickets], stats


def _check_same(ref, served):
    for i, (a, (r, x, y)) in enumerate(zip(ref, served)):
        assert r["status"] == sx.SX_OK, f"request {i} status {r['status']}"
        assert np.array_equal(a["y"], y), f"request {i}: y differs from the solve alone"
        assert np.array_equal(a["x"], x), f"request {i}: x differs"
        assert r["tallies"] == a["tallies"], f"request {i}: tallies differ"
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_served_results_equal_alone():
    ws, sweeps = _requests()
    print("[case] serve 5 requests, round 20, max_active 3", flush=True)
    ref = _alone(ws, sweeps)
    served, stats = _serve(ws, sweeps, round_sweeps=20, max_active=3, prep_threads=2)
    _check_same(ref, served)
    assert stats["finished"] == 5 and stats["failed"] == 0
    assert 1 <= stats["peak_active"] <= 3
    assert stats["latency_p50_s"] > 0 and stats["latency_p99_s"] >= stats["latency_p50_s"]
    assert stats["updates"] == sum(w.n * w.k * s for w, s in zip(ws, sweeps))


def test_admission_waits_for_memory():
    """A budget that holds about one grid at a time: requests wait for
    retirements, and still every result is the one alone."""
    ws, sweeps = _requests()
    need = max(sx.sx_grid_bytes(w) for w in ws)
    print(f"[case] serve with budget {int(1.3 * need)} bytes", flush=True)
    ref = _alone(ws, sweeps)
    served, stats = _serve(ws, sweeps, round_sweeps=25, max_active=8, prep_threads=3,
                           hbm_budget=int(1.3 * need))
    _check_same(ref, served)
    assert stats["finished"] == 5
    assert stats["peak_active"] <= 2


def test_malformed_request_reports_its_error():
    ws, sweeps = _requests()
    bad = G.with_(ws[0], nbr_idx=np.where(ws[0].nbr_idx == 0, 1, ws[0].nbr_idx)
                  .astype(np.int32))
    print("[case] serve one malformed request among good ones", flush=True)
    served, stats = _serve([ws[2], bad, ws[0]], [10, 10, 10], round_sweeps=5)
    assert served[0][0]["status"] == sx.SX_OK
    assert served[1][0]["status"] == sx.SX_EINVAL
    assert served[2][0]["status"] == sx.SX_OK
    assert stats["finished"] == 2 and stats["failed"] == 1


def test_served_mixed_physics_equal_alone():
    """Requests with combined transport, diffuse radiation and plain
    direction-conserving transport, in both precisions, served together:
    each result is the one of the grid solved alone."""
    base = dict(box=3e21, rate=3e45, dt=3e13)
    ws = [G.with_(G.small_random(1200, seed=86, n_bins=42, n_src=2, **base),
                  transport=G.SX_TRANSPORT_COMBINED, tau_switch=1.0),
          G.with_(G.small_random(900, seed=87, n_bins=21, n_src=1, precision=G.SX_FP32_TRANSPORT,
                                 **base), alpha_A=G.ALPHA_A),
          G.small_random(1500, seed=88, n_bins=42, n_src=3, **base),
          G.with_(G.small_random(700, seed=89, n_bins=42, n_src=2, precision=G.SX_FP32_TRANSPORT,
                                 **base), transport=G.SX_TRANSPORT_COMBINED, tau_switch=0.5,
                  alpha_A=G.ALPHA_A)]
    sweeps = [50, 35, 60, 45]
    print("[case] serve mixed physics", flush=True)
    ref = _alone(ws, sweeps)
    served, stats = _serve(ws, sweeps, round_sweeps=15, max_active=4, prep_threads=2)
    _check_same(ref, served)
    assert stats["finished"] == 4 and stats["failed"] == 0
