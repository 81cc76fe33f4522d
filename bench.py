#!/usr/bin/env python3
"""Throughput of the SimpleX2 direction-conserving transport + hydrogen
chemistry step on one MI355X, in vertex-direction updates per second.

A step is one whole solve of the Stromgren problem on a resident grid:
device-side re-selection of the bin tables and gather lists, state reset,
`--sweeps` radiative-transfer steps (fused gather / chemistry / outgoing
kernel each), and read-back of the ionised fraction and photon tallies.
One update advances one (vertex, bin) pair by one sweep.

Prints one JSON line (see the end of main()).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, GB/s


def _analytic():
    """The analytic references of the tests (front laws, equilibrium
    profiles), imported from tests/analytic.py."""
    p = os.path.join(ROOT, "tests")
    if p not in sys.path:
        sys.path.insert(0, p)
    import analytic
    return analytic


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_update(k: int, photon_bytes: int) -> float:
    """What the method must move per vertex-direction update with perfect
    reuse: read + write one photon word, ~2 B of routing (three 6-bit
    slots), and ~110 B of per-vertex data (neutral fraction read + write,
    transmission, three chemistry coefficients, one CSR row of ~15.5
    neighbours) shared by the K bins."""
    return 2.0 * photon_bytes + 2.0 + 110.0 / k


def combined_bytes_per_step(w, layout, photon_bytes: int) -> float:
    """Algorithmic bytes of one combined-transport step for a given mode
    mix: a direction-conserving vertex moves what it moves in
    direction-conserving transport (K updates); a ballistic vertex reads one
    packet and writes one per incoming edge, with ~1 B of routing per edge,
    plus the same ~110 B of per-vertex data."""
    import numpy as np
    deg = np.diff(w.nbr_ptr)
    lay = np.asarray(layout) != 0
    dct = float(np.count_nonzero(~lay)) * w.k * algorithmic_bytes_per_update(w.k, photon_bytes)
    bal = float(np.sum(deg[lay])) * (2.0 * photon_bytes + 1.0) + 110.0 * float(np.count_nonzero(lay))
    return dct + bal


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_0912_4273_amd", "csrc", "sx_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    e = d.get(workload)
    if not e or e.get("kernel_sha") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def _build(task):
    from paper_0912_4273_amd import gridgen as G
    if task[0] == "batch":
        return G.batch_member(task[1])
    if task[0] == "shadow":
        return G.shadow_test(n=task[1], n_sweeps=task[2])
    return G.serve_pool_grid(task[1], task[2])


def build_grids(n_batch: int, pool_sizes, shadow_n: int = 0, shadow_sweeps: int = 1500):
    """The shadowing grid, the batch members and the serving pool, built on
    the host cores before the GPU is touched (worker processes are forked);
    largest first."""
    import multiprocessing as mp
    tasks = [("shadow", shadow_n, shadow_sweeps)] if shadow_n > 0 else []
    tasks += [("pool", i, n) for i, n in enumerate(pool_sizes)][::-1]
    tasks += [("batch", g) for g in range(n_batch)]
    if not tasks:
        return [], [], None, 0
    workers = max(1, min(16, os.cpu_count() or 1, len(tasks)))
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_build, tasks, chunksize=1)
    shadow = out.pop(0) if shadow_n > 0 else None
    pool_grids = sorted(out[:len(pool_sizes)], key=lambda w: w.n)
    return out[len(pool_sizes):], pool_grids, shadow, workers


def shadow_leg(ctx, w, log, profile):
    """The 1M-vertex shadowing problem in FP32: throughput of the whole
    solve, and the plane-parallel diagnostics (front crossing, ionised depth
    into the clump on its axis against the 1-D Stromgren length, ionisation
    behind the clump against off the shadow)."""
    import numpy as np
    from paper_0912_4273_amd import gridgen as G
    kpc = G.KPC_CM
    t0 = time.perf_counter()
    gid = ctx.upload(w)
    up = time.perf_counter() - t0
    profile(True)
    t0 = time.perf_counter()
    ctx.solve([gid], w.n_sweeps)
    st = ctx.state(gid, nin=False)
    el = time.perf_counter() - t0
    pr = profile(False)
    info = ctx.info(gid)
    ctx.free(gid)
    m = w.meta
    p = w.pos / kpc
    cy = m["clump_c_kpc"][1]
    rperp = np.hypot(p[:, 1] - cy, p[:, 2] - m["clump_c_kpc"][2])
    inclump = np.sum((p - np.array(m["clump_c_kpc"])) ** 2, axis=1) < m["clump_r_kpc"] ** 2
    x = st["x"]
    A = _analytic()
    lit = m["clump_c_kpc"][0] - m["clump_r_kpc"]
    back = m["clump_c_kpc"][0] + m["clump_r_kpc"]
    axis = (rperp < 0.25) & (p[:, 0] >= lit) & (p[:, 0] <= back)
    try:
        depth = float(A.half_crossing(p[axis, 0] - lit, x[axis], 0.05))
    except AssertionError:   # a short run: the front has not reached the clump
        depth = None
    behind = (p[:, 0] > back) & (p[:, 0] < back + 0.3) & (rperp < 0.25)
    off = (p[:, 0] > back) & (p[:, 0] < back + 0.3) & (rperp > 1.5)
    n_c = m["n_H"] * m["contrast"]
    l_s = m["flux"] / (G.ALPHA_B * n_c * n_c) / kpc
    z_ode = A.slab_front(m["flux"], n_c, w.sigma, w.alpha_B) / kpc
    tl = st["tallies"]
    kern = pr["total_ms"] / max(pr["launches"], 1)
    upd = w.n * w.k * w.n_sweeps
    res = dict(
        value=upd / el, unit="vertex·direction updates/s", vertices=w.n, bins=w.k,
        sweeps=w.n_sweeps, ms_per_solve=1e3 * el, upload_s=up, sweep_kernel_us=1e3 * kern,
        algorithmic_hbm_frac=round(algorithmic_bytes_per_update(w.k, 4) * w.n * w.k
                                   / (kern * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        counter_bytes_per_launch=measured_traffic(f"shadow_{w.n}_k{w.k}"),
        device_bytes=info["bytes"],
        clump_axis_depth_kpc=depth, stromgren_length_1d_kpc=l_s,
        clump_depth_over_1d_equilibrium_profile=None if depth is None else round(depth / z_ode, 4),
        x_axis_behind_clump=float(x[behind].mean()), x_off_shadow=float(x[off].mean()),
        conservation_residual=abs(tl["emitted"] - tl["absorbed"] - tl["escaped"]
                                  - tl["in_flight"]) / tl["emitted"])
    log(f"shadow: {res['value']:.3e} updates/s, sweep {1e3 * kern:.1f} us, depth "
        f"{depth} kpc (1-D profile {z_ode:.3f}), axis behind {res['x_axis_behind_clump']:.3f} "
        f"off {res['x_off_shadow']:.3f}")
    return res


def serve_leg(ctx, pool, args, log):
    """Poisson arrivals of solve requests into the library's request loop;
    throughput and submit-to-result latency."""
    import threading
    import numpy as np
    from paper_0912_4273_amd import gridgen as G
    from paper_0912_4273_amd import sx
    arr = G.serve_arrivals(args.serve_rate, args.serve_seconds)
    n_max = max(w.n for w in pool)
    ctx.set_schedule([], graph_sweeps=0)   # the batch changes every round
    srv = sx.Server(ctx, round_sweeps=args.serve_round, max_active=64,
                    prep_threads=args.serve_prep_threads)
    results, errors = [], []

    def poller():
        while len(results) + len(errors) < len(arr):
            r = srv.poll(timeout=5.0)
            if r is None:
                continue
            srv.take(r["ticket"])
            (results if r["status"] == sx.SX_OK else errors).append(r)

    th = threading.Thread(target=poller, daemon=True)
    th.start()
    offered = 0.0
    t0 = time.perf_counter()
    for r, ta in enumerate(arr):
        dt = t0 + ta - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        w = G.serve_request(pool, r, 1e4, n_max)
        offered += w.n * w.k * w.n_sweeps
        srv.submit(w, w.n_sweeps)
        if (r + 1) % 100 == 0:
            log(f"serve: {r + 1}/{len(arr)} submitted, {len(results)} done")
    # drain: the requests still queued or on the GPU, reported as they finish
    deadline = time.perf_counter() + max(600.0, 4 * args.serve_seconds)
    while th.is_alive() and time.perf_counter() < deadline:
        th.join(timeout=30.0)
        if th.is_alive():
            log(f"serve: all {len(arr)} submitted, {len(results)} done")
    wall = time.perf_counter() - t0
    st = srv.stop()
    ctx.set_schedule([], graph_sweeps=args.graph_sweeps)
    lat = np.array([r["t_done"] - r["t_submit"] for r in results])
    q = (lambda f: float(np.quantile(lat, f))) if len(lat) else (lambda f: None)
    return dict(
        value=st["updates"] / st["span_s"] if st["span_s"] > 0 else None,
        unit="vertex·direction updates/s",
        requests=len(arr), finished=int(st["finished"]), failed=int(st["failed"]),
        arrivals=f"Poisson {args.serve_rate}/s for {args.serve_seconds} s (seed 5)",
        vertices=f"log-uniform [1e4, {n_max}] served from a pool of {len(pool)} grids",
        offered_updates_per_s=offered / args.serve_seconds,
        latency_p50_s=q(0.5), latency_p99_s=q(0.99),
        latency_max_s=float(lat.max()) if len(lat) else None,
        queue_wait_p50_s=float(np.median([r["t_admit"] - r["t_submit"] for r in results]))
        if results else None,
        rounds=int(st["rounds"]), peak_active=int(st["peak_active"]),
        gpu_round_frac=st["round_s"] / st["span_s"] if st["span_s"] > 0 else None,
        wall_s=wall, round_sweeps=args.serve_round, prep_threads=args.serve_prep_threads)


def rotation_leg(ctx, w, every: int, log):
    """The same Stromgren solve with the direction bins rotated at random
    every `every` sweeps (seeded rotations): throughput including the
    rebuilds of the routing, their cost, and the ionised-volume radius
    against the analytic front law."""
    import numpy as np
    from paper_0912_4273_amd import gridgen as G
    gid = ctx.upload(w)
    n_rot = (w.n_sweeps + every - 1) // every
    Rs = G.random_rotations(n_rot, seed=2024)
    t_rot = 0.0
    t0 = time.perf_counter()
    done = 0
    for i in range(n_rot):
        n = min(every, w.n_sweeps - done)
        ctx.step([gid], n)
        done += n
        t1 = time.perf_counter()
        ctx.rotate(gid, Rs[i])
        t_rot += time.perf_counter() - t1
    st = ctx.state(gid, nin=False)
    el = time.perf_counter() - t0
    r_s = (3 * w.meta["rate"] / (4 * math.pi * w.alpha_B * w.meta["n_H"] ** 2)) ** (1 / 3)
    t_rec = 1.0 / (w.alpha_B * w.meta["n_H"])
    # the front law over time (untimed repeat of the same rotations, the
    # ionised-volume radius every 50 sweeps) and the equilibrium profile
    A = _analytic()
    ctx.reset(gid)
    dev, done = [], 0
    for i in range(n_rot):
        n = min(every, w.n_sweeps - done)
        ctx.step([gid], n)
        done += n
        ctx.rotate(gid, Rs[i])
        if done % 50 == 0 and done * w.dt >= 100 * 3.15576e13:
            xr = ctx.state(gid, nin=False)["x"]
            dev.append(abs(A.ionised_volume_radius(w.volume, xr)
                           / A.front_radius(done * w.dt, r_s, t_rec) - 1.0))
    ctx.free(gid)
    c = w.pos[w.src_vertex[0]]
    r = np.linalg.norm(w.pos - c, axis=1)
    shell = 1.237 * (w.box ** 3 / w.n) ** (1.0 / 3.0)
    r_half = A.half_crossing(r, st["x"], shell, exclude=w.src_vertex[0])
    r_ode = A.inner_profile_front(w.meta["rate"], w.meta["n_H"], w.sigma, w.alpha_B)
    rv = (3 / (4 * math.pi) * float(np.sum(w.volume * st["x"]))) ** (1 / 3)
    tl = st["tallies"]
    res = dict(value=w.n * w.k * w.n_sweeps / el, unit="vertex·direction updates/s",
               rotate_every=every, rotations=n_rot, ms_per_solve=1e3 * el,
               ms_per_rotation=1e3 * t_rot / n_rot,
               front_radius_over_analytic=round(
                   rv / (r_s * (1 - math.exp(-w.n_sweeps * w.dt / t_rec)) ** (1 / 3)), 4),
               front_law_max_dev_from_100myr=round(max(dev), 4) if dev else None,
               inner_profile_half_crossing_over_ode=round(r_half / r_ode, 4),
               conservation_residual=abs(tl["emitted"] - tl["absorbed"] - tl["escaped"]
                                         - tl["in_flight"]) / tl["emitted"])
    log(f"rotating every {every}: {res['value']:.3e} updates/s, "
        f"{res['ms_per_rotation']:.2f} ms per rotation, front/analytic "
        f"{res['front_radius_over_analytic']}")
    return res


def combined_leg(ctx, w, tau_switch: float, log, prof):
    """The same Stromgren solve with combined transport: ballistic where the
    optical depth is at least tau_switch, direction-conserving elsewhere.
    Throughput in the headline's units (N K per step, the same problem),
    the combined sweep kernel's average time, the share of vertices left
    ballistic, the front radius against the analytic law."""
    import numpy as np
    from paper_0912_4273_amd import gridgen as G
    wc = G.with_(w, transport=G.SX_TRANSPORT_COMBINED, tau_switch=tau_switch)
    t0 = time.perf_counter()
    gid = ctx.upload(wc)
    up = time.perf_counter() - t0
    ctx.solve([gid], 20)           # warm-up: plan, graph, caches
    ctx.reset(gid)
    ctx.sync()
    prof(True)
    t0 = time.perf_counter()
    ctx.step([gid], w.n_sweeps)
    st = ctx.state(gid, nin=False)
    el = time.perf_counter() - t0
    pr = prof(False)
    lay = ctx.edge_state(gid)["layout"]
    # the paper's production mode: the bins rotated before every step
    ctx.reset(gid)
    Rs = G.random_rotations(w.n_sweeps, seed=2025)
    ctx.sync()
    t1 = time.perf_counter()
    for R in Rs:
        ctx.step([gid], 1)
        ctx.rotate(gid, R)
    str_ = ctx.state(gid, nin=False)
    el_rot = time.perf_counter() - t1
    ctx.free(gid)
    rv_rot = (3 / (4 * math.pi) * float(np.sum(w.volume * str_["x"]))) ** (1 / 3)
    r_s = (3 * w.meta["rate"] / (4 * math.pi * w.alpha_B * w.meta["n_H"] ** 2)) ** (1 / 3)
    t_rec = 1.0 / (w.alpha_B * w.meta["n_H"])
    rv = (3 / (4 * math.pi) * float(np.sum(w.volume * st["x"]))) ** (1 / 3)
    tl = st["tallies"]
    kus = 1e3 * pr["total_ms"] / max(pr["launches"], 1)
    bytes_end = combined_bytes_per_step(w, lay, 4)
    res = dict(value=w.n * w.k * w.n_sweeps / el, unit="vertex·direction updates/s",
               tau_switch=tau_switch, ms_per_solve=1e3 * el, upload_s=round(up, 2),
               sweep_kernel_us=kus,
               algorithmic_bytes_per_step_at_end=round(bytes_end),
               hbm_frac_at_end_mix=round(bytes_end / (kus * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
               ballistic_fraction_end=round(float(lay.mean()), 4),
               front_radius_over_analytic=round(
                   rv / (r_s * (1 - math.exp(-w.n_sweeps * w.dt / t_rec)) ** (1 / 3)), 4),
               conservation_residual=abs(tl["emitted"] - tl["absorbed"] - tl["escaped"]
                                         - tl["in_flight"]) / tl["emitted"],
               rotated_every_step=dict(
                   value=w.n * w.k * w.n_sweeps / el_rot, ms_per_solve=1e3 * el_rot,
                   front_radius_over_analytic=round(
                       rv_rot / (r_s * (1 - math.exp(-w.n_sweeps * w.dt / t_rec)) ** (1 / 3)), 4)))
    log(f"combined transport rotated every step: {res['rotated_every_step']['value']:.3e} "
        f"updates/s, front/analytic {res['rotated_every_step']['front_radius_over_analytic']}")
    log(f"combined transport (switch {tau_switch}): {res['value']:.3e} updates/s, "
        f"{res['ms_per_solve']:.1f} ms/solve, sweep {res['sweep_kernel_us']:.1f} us, "
        f"ballistic at end {res['ballistic_fraction_end']}, front/analytic "
        f"{res['front_radius_over_analytic']}")
    return res


def diffuse_leg(ctx, w, log, prof):
    """The same Stromgren solve off the spot: case-A chemistry and the
    ground-level recombination photons transported (direction-conserving
    transport).  Throughput in the headline's units, the kernel's average
    time, the share of recombination photons among those emitted, and the
    front radius against the on-the-spot (case-B) law it should follow."""
    import numpy as np
    from paper_0912_4273_amd import gridgen as G
    wd = G.with_(w, alpha_A=G.ALPHA_A)
    gid = ctx.upload(wd)
    ctx.solve([gid], 20)
    ctx.reset(gid)
    ctx.sync()
    prof(True)
    t0 = time.perf_counter()
    ctx.step([gid], w.n_sweeps)
    st = ctx.state(gid, nin=False)
    el = time.perf_counter() - t0
    pr = prof(False)
    ctx.free(gid)
    r_s = (3 * w.meta["rate"] / (4 * math.pi * w.alpha_B * w.meta["n_H"] ** 2)) ** (1 / 3)
    t_rec = 1.0 / (w.alpha_B * w.meta["n_H"])
    rv = (3 / (4 * math.pi) * float(np.sum(w.volume * st["x"]))) ** (1 / 3)
    tl = st["tallies"]
    src = w.meta["rate"] * w.dt * w.n_sweeps
    res = dict(value=w.n * w.k * w.n_sweeps / el, unit="vertex·direction updates/s",
               alpha_A=G.ALPHA_A, ms_per_solve=1e3 * el,
               sweep_kernel_us=1e3 * pr["total_ms"] / max(pr["launches"], 1),
               recombination_photon_share=round((tl["emitted"] - src) / tl["emitted"], 4),
               front_radius_over_case_b_law=round(
                   rv / (r_s * (1 - math.exp(-w.n_sweeps * w.dt / t_rec)) ** (1 / 3)), 4),
               conservation_residual=abs(tl["emitted"] - tl["absorbed"] - tl["escaped"]
                                         - tl["in_flight"]) / tl["emitted"])
    log(f"diffuse radiation: {res['value']:.3e} updates/s, sweep {res['sweep_kernel_us']:.1f} us, "
        f"recombination photons {res['recombination_photon_share']}, front/case-B "
        f"{res['front_radius_over_case_b_law']}")
    return res


def regrid_leg(ctx, w, passes: int, n_min: int, tau_remove: float, log, prof):
    """Dynamic grid (Sect. 2.1.4): half the Stromgren solve, then `passes`
    thinning passes (vertices with optical depth below tau_remove, down to a
    minimum resolution of n_min^3 over the box), then the second half on the
    thinned grid.  Cost of a pass by part, vertices left, step time before
    and after, front radius against the analytic law at the end."""
    import numpy as np
    from paper_0912_4273_amd import regrid as RG
    half = w.n_sweeps // 2
    spacing = RG.min_spacing_for(w.box, n_min)
    gid = ctx.upload(w)
    prof(True)
    ctx.solve([gid], half)
    k0 = prof(False)
    wc, gc = w, gid
    parts = dict(select_s=0.0, triangulate_s=0.0, upload_s=0.0, remap_s=0.0)
    removed = []
    for _ in range(passes):
        t0 = time.perf_counter()
        rm = ctx.select_removal(gc, tau_remove, spacing)
        t1 = time.perf_counter()
        if not rm.any():
            break
        st = ctx.state(gc, nin=False)
        wn, new_of_old = RG.thinned_workload(wc, ~rm, st["x"])
        t2 = time.perf_counter()
        gn = ctx.upload(wn)
        t3 = time.perf_counter()
        ctx.remap(gc, gn, new_of_old)
        t4 = time.perf_counter()
        ctx.free(gc)
        parts["select_s"] += t1 - t0
        parts["triangulate_s"] += t2 - t1
        parts["upload_s"] += t3 - t2
        parts["remap_s"] += t4 - t3
        removed.append(int(rm.sum()))
        wc, gc = wn, gn
    prof(True)
    ctx.solve([gc], w.n_sweeps - half)
    k1 = prof(False)
    st = ctx.state(gc, nin=False)
    ctx.free(gc)
    r_s = (3 * w.meta["rate"] / (4 * math.pi * w.alpha_B * w.meta["n_H"] ** 2)) ** (1 / 3)
    t_rec = 1.0 / (w.alpha_B * w.meta["n_H"])
    rv = (3 / (4 * math.pi) * float(np.sum(wc.volume * st["x"]))) ** (1 / 3)
    tl = st["tallies"]
    res = dict(passes=len(removed), removed_per_pass=removed, vertices_after=wc.n,
               min_resolution=n_min, tau_remove=tau_remove,
               seconds_per_pass={k: round(v / max(len(removed), 1), 3) for k, v in parts.items()},
               sweep_kernel_us_before=1e3 * k0["total_ms"] / max(k0["launches"], 1),
               sweep_kernel_us_after=1e3 * k1["total_ms"] / max(k1["launches"], 1),
               front_radius_over_analytic=round(
                   rv / (r_s * (1 - math.exp(-w.n_sweeps * w.dt / t_rec)) ** (1 / 3)), 4),
               conservation_residual=abs(tl["emitted"] - tl["absorbed"] - tl["escaped"]
                                         - tl["in_flight"]) / tl["emitted"])
    log(f"dynamic grid: removed {removed} of {w.n}, sweep {res['sweep_kernel_us_before']:.1f} -> "
        f"{res['sweep_kernel_us_after']:.1f} us, per pass {res['seconds_per_pass']}, front/analytic "
        f"{res['front_radius_over_analytic']}")
    return res


def small_leg(ctx, log, prof, graph_sweeps: int):
    """The plain single-source test (4096 vertices, 42 bins, all-FP64, 200
    sweeps over 500 Myr): a grid too small to fill the GPU, so the time per
    sweep is launch and latency bound.  Timed whole (reset, 200 sweeps,
    read-back) under each work split, as HIP-graph replays and as plain
    launches; the sweep launch's time comes from HIP events on the library
    stream, gaps included."""
    from paper_0912_4273_amd import gridgen as G
    w1 = G.config1()
    gid = ctx.upload(w1)
    sweeps = w1.n_sweeps
    out = dict(workload=f"stromgren_{w1.n}_k{w1.k}_{sweeps}sweeps", vertices=w1.n, bins=w1.k,
               sweeps=sweeps, precision="fp64")
    runs = {}
    for split in (1, 2, 4):
        for label, gs in (("graph", graph_sweeps), ("launches", 0)):
            # at most 4 waves per workgroup
            ctx.set_schedule([gid], tiles_per_group=4 // split, graph_sweeps=gs,
                             work_split=split)
            for _ in range(2):   # warm-up (graph instantiation)
                ctx.reset(gid)
                ctx.solve([gid], sweeps)
            reps = 5
            prof(True)
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.reset(gid)
                ctx.solve([gid], sweeps)
                ctx.state(gid, nin=False)
            el = (time.perf_counter() - t0) / reps
            pr = prof(False)
            runs[f"split{split}_{label}"] = dict(
                ms_per_solve=round(1e3 * el, 3),
                sweep_launch_us=round(1e3 * pr["total_ms"] / max(pr["launches"], 1), 2),
                updates_per_s=w1.n * w1.k * sweeps / el)
    ctx.set_schedule([gid], graph_sweeps=graph_sweeps)
    ctx.free(gid)
    best = min(runs, key=lambda r: runs[r]["ms_per_solve"])
    out.update(runs=runs, best=best, value=runs[best]["updates_per_s"],
               unit="vertex·direction updates/s")
    log(f"small grid (fp64, 4096 x 42, 200 sweeps): best {best} "
        f"{runs[best]['ms_per_solve']:.2f} ms/solve, {out['value']:.3e} updates/s; "
        + ", ".join(f"{k} {v['sweep_launch_us']:.1f} us" for k, v in runs.items()))
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, sweeps: int, sweeps_mt: int):
    """The FP64 oracle on the same grid from the initial state, for a bounded
    number of sweeps: sequential (one thread, the parity reference) and its
    pull form on all the host cores this process may use (at most 16, the
    GPU machine's share)."""
    from oracle import Oracle
    o = Oracle(w)
    t0 = time.perf_counter()
    o.run(sweeps)
    dt1 = time.perf_counter() - t0
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                         else (os.cpu_count() or 1)))
    om = Oracle(w)
    om.run_threads(1, threads)       # builds its sender lists
    t0 = time.perf_counter()
    om.run_threads(sweeps_mt, threads)
    dtm = time.perf_counter() - t0
    return dict(value=w.n * w.k * sweeps_mt / dtm, unit="vertex·direction updates/s",
                cores=threads, kind="oracle",
                sample=f"{sweeps_mt} sweeps of the same {w.n}-vertex, {w.k}-bin grid after one "
                       f"from the neutral initial state, FP64, pull form on {threads} threads "
                       f"({dtm:.1f} s)",
                cpu_model=cpu_model(),
                single_thread=dict(value=w.n * w.k * sweeps / dt1, cores=1,
                                   sample=f"{sweeps} sweeps from the neutral initial state, "
                                          f"sequential oracle ({dt1:.1f} s)"))


def _err_stats(got, ref, atol):
    """Max and 99th percentile of |got - ref| / (|ref| + atol)."""
    import numpy as np
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    if got.size == 0:
        return None
    e = np.abs(got - ref) / (np.abs(ref) + atol)
    return dict(max=float(e.max()), p99=float(np.quantile(e, 0.99)))


def precision_stats(got, ref, unit, n_sub_atol=True):
    """Per-result error of a GPU state against the oracle: x, y, y where y
    >= 1e-6 (what FP64 chemistry protects), the photon field (relative to
    the value plus 1e-9 of a photon unit, below which FP32 underflow makes
    relative error meaningless) and the tallies."""
    import numpy as np
    msk = ref["y"] >= 1e-6
    out = dict(x=_err_stats(got["x"], ref["x"], 1e-12), y=_err_stats(got["y"], ref["y"], 1e-12),
               y_ge_1e6=_err_stats(got["y"][msk], ref["y"][msk], 0.0),
               photons=_err_stats(got["photons"], ref["photons"], 1e-9 * unit))
    tl = {}
    for k in ("emitted", "absorbed", "escaped", "in_flight"):
        a, b = got["tallies"][k], ref["tallies"][k]
        tl[k] = abs(a - b) / max(abs(b), 1e-300)
    out["tallies_rel"] = tl
    return out


def precision_leg(ctx, w2, log):
    """Error against the FP64 oracle, per result: the 4096-vertex Stromgren
    test whole (200 sweeps) in both precisions, and one sweep of the
    262144-vertex benchmark grid from the GPU's state after 300 sweeps.
    Also the plain FP64 throughput of the small test (the launch-bound
    configuration) with graph replays and with single launches."""
    from paper_0912_4273_amd import gridgen as G
    from oracle import Oracle
    w1 = G.config1()
    ora = Oracle(w1)
    ora.run(w1.n_sweeps)
    ref1 = ora.state()
    ora.close()
    out = dict(stromgren_4096_200_sweeps={}, stromgren_262144_one_sweep={})
    for prec, name in ((G.SX_FP64, "fp64"), (G.SX_FP32_TRANSPORT, "fp32")):
        gid = ctx.upload(G.with_(w1, precision=prec))
        ctx.solve([gid], w1.n_sweeps)
        got = ctx.state(gid, photons=True)
        unit = ctx.info(gid)["photon_unit"]
        out["stromgren_4096_200_sweeps"][name] = precision_stats(got, ref1, unit)
        # throughput of the small grid (64 tiles: one wave per tile leaves
        # most of the GPU idle): graph replays, single launches, and each
        # tile's bins split over four waves
        for label, kw in (("graph50", dict(graph_sweeps=50)),
                          ("graph0", dict(graph_sweeps=0)),
                          ("graph50_split4", dict(tiles_per_group=1, work_split=4,
                                                  graph_sweeps=50))):
            ctx.set_schedule([gid], **kw)
            ctx.reset(gid)
            ctx.solve([gid], 20)
            ctx.reset(gid)
            ctx.sync()
            ctx.profile(True)
            ctx.profile_read()
            t0 = time.perf_counter()
            ctx.solve([gid], w1.n_sweeps)
            el = time.perf_counter() - t0
            pr = ctx.profile_read()
            ctx.profile(False)
            f = out["stromgren_4096_200_sweeps"][name]
            f[f"updates_per_s_{label}"] = w1.n * w1.k * w1.n_sweeps / el
            f[f"sweep_us_{label}"] = 1e3 * pr["total_ms"] / max(pr["launches"], 1)
        ctx.free(gid)
    # one sweep at the benchmark's size, both precisions, from the GPU state
    ora2 = Oracle(w2)
    for prec, name in ((G.SX_FP32_TRANSPORT, "fp32"), (G.SX_FP64, "fp64")):
        gid = ctx.upload(G.with_(w2, precision=prec))
        ctx.solve([gid], 300)
        s1 = ctx.state(gid, photons=True)
        ctx.solve([gid], 1)
        s2 = ctx.state(gid, photons=True)
        unit = ctx.info(gid)["photon_unit"]
        ctx.free(gid)
        ora2.set_state(y=s1["y"], photons=s1["photons"], tallies=s1["tallies"])
        ora2.run(1)
        out["stromgren_262144_one_sweep"][name] = precision_stats(s2, ora2.state(), unit)
    ora2.close()
    f1 = out["stromgren_4096_200_sweeps"]
    log(f"precision: 4096 whole fp32 x max {f1['fp32']['x']['max']:.2e}, fp64 x max "
        f"{f1['fp64']['x']['max']:.2e}; small fp64 {f1['fp64']['updates_per_s_graph50']:.3e} "
        f"updates/s (graphs) / {f1['fp64']['updates_per_s_graph0']:.3e} (single launches) / "
        f"{f1['fp64']['updates_per_s_graph50_split4']:.3e} (four waves per tile)")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--bins", type=int, default=84)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--cpu-sweeps", type=int, default=25)
    ap.add_argument("--cpu-sweeps-mt", type=int, default=100,
                    help="sweeps of the all-cores oracle baseline")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the per-result error statement against the oracle")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 4096-vertex all-FP64 leg")
    ap.add_argument("--batch-grids", type=int, default=64,
                    help="grids in the batched leg (0 = skip it)")
    ap.add_argument("--batch-sweeps", type=int, default=200)
    ap.add_argument("--autotune-trials", type=int, default=2)
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="arrival window of the serving leg (0 = skip it)")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-max-n", type=int, default=2000000,
                    help="largest pool grid (the request range is [1e4, 2e6])")
    ap.add_argument("--serve-round", type=int, default=50)
    ap.add_argument("--serve-prep-threads", type=int, default=12)
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg")
    ap.add_argument("--shadow-n", type=int, default=1048576,
                    help="vertices of the shadowing leg (0 = skip it)")
    ap.add_argument("--shadow-sweeps", type=int, default=1500)
    ap.add_argument("--rotate-every", type=int, default=1,
                    help="sweeps between random rotations of the bins in the rotation leg "
                         "(0 = skip the leg)")
    ap.add_argument("--combined-tau", type=float, default=1.0,
                    help="switch of the combined-transport leg (negative: skip the leg)")
    ap.add_argument("--no-diffuse", action="store_true",
                    help="skip the diffuse-recombination-radiation leg")
    ap.add_argument("--regrid-passes", type=int, default=2,
                    help="thinning passes of the dynamic-grid leg (0: skip the leg)")
    ap.add_argument("--regrid-min-res", type=int, default=32)
    ap.add_argument("--graph-sweeps", type=int, default=50,
                    help="sweeps per replayed HIP graph (0: one launch per sweep)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent grids would shard across GPUs with no exchange; one grid "
              "larger than a GPU would need a ghost exchange per step, not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_0912_4273_amd import gridgen as G

    # host-side grid construction first: the batch is built by forked
    # workers, which must not inherit an initialised GPU runtime
    if args.serve_only:
        args.batch_grids = 0
        args.shadow_n = 0
    pool_sizes = (G.serve_pool_sizes(1e4, args.serve_max_n, 8)
                  if args.serve_seconds > 0 else [])
    t = time.perf_counter()
    batch, pool, shadow, nw = build_grids(max(args.batch_grids, 0), pool_sizes,
                                          max(args.shadow_n, 0), args.shadow_sweeps)
    if batch or pool:
        log(f"built {len(batch)} batch grids ({sum(b.n for b in batch)} vertices) and "
            f"{len(pool)} pool grids (up to {max([0] + [w.n for w in pool])} vertices) in "
            f"{time.perf_counter() - t:.1f} s on {nw} processes")
    t = time.perf_counter()
    w = G.stromgren_test(args.n, seed=2, n_bins=args.bins, bins_seed=102,
                         n_sweeps=args.sweeps, precision=G.SX_FP32_TRANSPORT,
                         name=f"stromgren_{args.n}_k{args.bins}")
    log(f"grid {w.n} vertices, {w.n_edges} directed edges, built in "
        f"{time.perf_counter() - t:.1f} s")

    import torch
    from paper_0912_4273_amd import sx

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.init()
    workload = f"stromgren_{w.n}_k{w.k}_{args.sweeps}sweeps"

    stream = torch.cuda.Stream(device=dev)
    ctx = sx.Context(device=0, stream=stream.cuda_stream, use_torch_allocator=True)
    ctx.set_schedule([], graph_sweeps=args.graph_sweeps)

    def upload(wl):
        t0 = time.perf_counter()
        gid = ctx.upload(wl)
        return gid, time.perf_counter() - t0

    def one_step(gid):
        ctx.reset(gid)
        ctx.step([gid], args.sweeps)
        return ctx.state(gid, nin=False)

    def timed(gid, steps, warmup):
        for _ in range(warmup):
            one_step(gid)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        st = None
        for _ in range(steps):
            st = one_step(gid)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile(False)
        return el, prof, st

    served = None
    if args.serve_only:
        served = serve_leg(ctx, pool, args, log)
        print(json.dumps({"served": served}), flush=True)
        ctx.close()
        return

    # ---- FP32 transport + FP64 chemistry (headline)
    gid, up_s = upload(w)
    log(f"uploaded fp32 grid in {up_s:.2f} s")
    el, prof, st32 = timed(gid, args.steps, args.warmup)
    ups = w.n * w.k * args.sweeps * args.steps / el
    ms_step = 1e3 * el / args.steps
    kern_ms = prof["total_ms"] / max(prof["launches"], 1)
    log(f"fp32: {ms_step:.1f} ms/step, {ups:.3e} updates/s, sweep kernel "
        f"{1e3 * kern_ms:.1f} us avg over {prof['launches']} launches")
    t32 = st32["tallies"]
    resid = abs(t32["emitted"] - (t32["absorbed"] + t32["escaped"] + t32["in_flight"])) \
        / t32["emitted"]
    ctx.free(gid)

    # ---- plain single-grid FP64 on the same GPU
    fp64 = None
    if not args.no_fp64:
        w64 = G.with_(w, precision=G.SX_FP64)
        gid64, _ = upload(w64)
        el64, prof64, st64 = timed(gid64, 1, 1)
        ups64 = w.n * w.k * args.sweeps / el64
        k64 = prof64["total_ms"] / max(prof64["launches"], 1)
        fp64 = dict(value=ups64, ms_per_step=1e3 * el64, sweep_kernel_us=1e3 * k64)
        ctx.free(gid64)

    # ---- batched: many uneven grids in one launch per sweep, autotuned
    batched = None
    if batch:
        t0 = time.perf_counter()
        ids = [ctx.upload(b) for b in batch]
        up_b = time.perf_counter() - t0
        nsw = [args.batch_sweeps] * len(ids)
        ctx.autotune(args.autotune_trials)
        ctx.solve(ids, nsw)            # tunes the schedule on its first sweeps
        ctx.autotune(0)
        sched = ctx.get_schedule(ids)
        for gid in ids:
            ctx.reset(gid)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        ctx.solve(ids, nsw)
        sts = [ctx.state(gid, nin=False) for gid in ids]
        el_b = time.perf_counter() - t0
        pb = ctx.profile_read()
        ctx.profile(False)
        upd_b = sum(b.n * b.k for b in batch) * args.batch_sweeps
        kb = pb["total_ms"] / max(pb["launches"], 1)
        # front radius against the analytic law, per grid (4 t_rec: 0.9937 r_S)
        ratios = []
        for b, st in zip(batch, sts):
            rv = (3 / (4 * math.pi) * float(np.sum(b.volume * st["x"]))) ** (1 / 3)
            ratios.append(rv / (b.meta["r_s"] * (1 - math.exp(-4.0)) ** (1 / 3)))
        # FP32 against all-FP64 on a few members, alone
        dx = []
        for b, st in list(zip(batch, sts))[:4]:
            g64 = ctx.upload(G.with_(b, precision=G.SX_FP64))
            ctx.solve([g64], args.batch_sweeps)
            dx.append(float(np.max(np.abs(ctx.state(g64, nin=False)["x"] - st["x"]))))
            ctx.free(g64)
        for gid in ids:
            ctx.free(gid)
        bpu_b = algorithmic_bytes_per_update(42, 4)
        batched = dict(
            value=upd_b / el_b, unit="vertex·direction updates/s",
            ms_per_step=1e3 * el_b, grids=len(batch),
            vertices=int(sum(b.n for b in batch)), bins=42, sweeps=args.batch_sweeps,
            upload_s=up_b, sweep_kernel_us=1e3 * kb,
            algorithmic_hbm_frac=round(bpu_b * upd_b / args.batch_sweeps
                                       / (kb * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            counter_bytes_per_launch=measured_traffic(f"batched_{len(batch)}_k42"),
            schedule=sched,
            front_radius_over_analytic=dict(min=round(min(ratios), 4),
                                            median=round(float(np.median(ratios)), 4),
                                            max=round(max(ratios), 4)),
            fp32_vs_fp64_max_abs_x_4_grids=max(dx))
        log(f"batched: {batched['value']:.3e} updates/s, {1e3 * el_b:.1f} ms/solve, "
            f"sweep launch {1e3 * kb:.1f} us, schedule {sched}")

    rotated = None
    if args.rotate_every > 0:
        rotated = rotation_leg(ctx, w, args.rotate_every, log)

    def prof(on):
        if on:
            ctx.profile(True)
            ctx.profile_read()
            return None
        r = ctx.profile_read()
        ctx.profile(False)
        return r

    small = None
    if not args.no_small:
        small = small_leg(ctx, log, prof, args.graph_sweeps)

    combined = None
    if args.combined_tau >= 0:
        combined = combined_leg(ctx, w, args.combined_tau, log, prof)

    regridded = None
    if args.regrid_passes > 0:
        regridded = regrid_leg(ctx, w, args.regrid_passes, args.regrid_min_res, 0.5, log, prof)

    diffused = None
    if not args.no_diffuse:
        diffused = diffuse_leg(ctx, w, log, prof)

    shadowed = None
    if shadow is not None:
        shadowed = shadow_leg(ctx, shadow, log, prof)

    precision = None
    if not args.no_precision:
        precision = precision_leg(ctx, w, log)
        ctx.set_schedule([], graph_sweeps=args.graph_sweeps)

    if pool:
        served = serve_leg(ctx, pool, args, log)
        log(f"served: {served['finished']}/{served['requests']} requests, "
            f"{served['value']:.3e} updates/s, p50 {served['latency_p50_s']:.2f} s, "
            f"p99 {served['latency_p99_s']:.2f} s")

    bpu = algorithmic_bytes_per_update(w.k, 4)
    bytes_launch = bpu * w.n * w.k
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_traffic(workload))

    # ---- physics / accuracy of the fp32 run
    box = w.box
    r_s = (3 * w.meta["rate"] / (4 * math.pi * w.alpha_B * w.meta["n_H"] ** 2)) ** (1 / 3)
    t_rec = 1.0 / (w.alpha_B * w.meta["n_H"])
    t_end = args.sweeps * w.dt
    rv32 = (3 / (4 * math.pi) * float(np.sum(w.volume * st32["x"]))) ** (1 / 3)
    acc = dict(front_radius_over_analytic=round(rv32 / (r_s * (1 - math.exp(-t_end / t_rec)) ** (1 / 3)), 4),
               conservation_residual=resid)
    if fp64 is not None:
        rv64 = (3 / (4 * math.pi) * float(np.sum(w.volume * st64["x"]))) ** (1 / 3)
        acc["fp32_vs_fp64_front_radius_rel"] = abs(rv32 / rv64 - 1)
        acc["fp32_vs_fp64_max_abs_x"] = float(np.max(np.abs(st32["x"] - st64["x"])))

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 1 GiB")

    cpu = None
    if not args.no_cpu:
        log(f"cpu oracle: {args.cpu_sweeps} sweeps")
        cpu = cpu_baseline(G.with_(w, precision=G.SX_FP64), args.cpu_sweeps, args.cpu_sweeps_mt)

    ctx.close()
    out = {
        "metric": "vertex·direction updates/s (batched FP32 vs plain FP64) + p50/p99 solve latency",
        "value": ups,
        "unit": "vertex·direction updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 transport, f64 chemistry",
        "data": "synthetic",
        "config": {"workload": workload, "vertices": w.n, "bins": w.k,
                   "sweeps_per_step": args.sweeps, "precision": "fp32_transport",
                   "physics": "Stromgren test: n_H 1e-3, 5e48 photons/s, 13.2 kpc box, 500 Myr"},
        "fp64_plain": fp64,
        "small_fp64": small,
        "batched": batched,
        "served": served,
        "shadow": shadowed,
        "rotated": rotated,
        "combined": combined,
        "diffuse": diffused,
        "dynamic_grid": regridded,
        "upload_s": up_s,
        "sweep_kernel_us": 1e3 * kern_ms,
        "roofline": roof,
        "algorithmic_bytes_per_update": bpu,
        "accuracy": acc,
        "precision_vs_oracle": precision,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
