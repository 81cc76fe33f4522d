"""Edge cases of the method and of the limits, GPU against the oracle: the
largest bin count in both precisions, a single bin, fewer than three
neighbours per bin, a vertex of very high degree, and the limits just past
the supported ones."""
import math

import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx
from oracle import Oracle
from parity import assert_state_close

pytestmark = pytest.mark.gpu


def _compare(ctx, w, sweeps, what):
    print(f"[case] {what}: n={w.n} k={w.k} mpb={w.max_per_bin} prec={w.precision}", flush=True)
    gid = ctx.upload(w)
    try:
        ctx.solve([gid], sweeps)
        got = ctx.state(gid, photons=True)
        tab = ctx.tables(gid)
        unit = ctx.info(gid)["photon_unit"]
    finally:
        ctx.free(gid)
    ora = Oracle(w)
    ot = ora.tables()
    ora.run(sweeps)
    ref = ora.state()
    ora.close()
    assert np.array_equal(tab["sel_m"], ot["sel_m"]), what
    assert np.array_equal(tab["sel_nbr"][:, :, :w.max_per_bin], ot["sel_nbr"]), what
    assert np.array_equal(tab["edge_bin"], ot["edge_bin"]), what
    assert_state_close(got, ref, w.precision, unit, what)


def _hub(n_leaves, precision=G.SX_FP64):
    """A centre vertex linked to n_leaves vertices on a sphere (Fibonacci
    lattice), the leaves also linked in a ring; the source sits at the
    centre."""
    i = np.arange(n_leaves) + 0.5
    phi = np.arccos(1 - 2 * i / n_leaves)
    th = math.pi * (1 + 5 ** 0.5) * i
    leaves = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    pos = np.vstack([np.zeros((1, 3)), leaves]) * 3e20
    rows = [list(range(1, n_leaves + 1))]
    for a in range(n_leaves):
        rows.append(sorted({0, 1 + (a + 1) % n_leaves, 1 + (a - 1) % n_leaves}))
    ptr = np.zeros(n_leaves + 2, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in r], np.int32)
    n = n_leaves + 1
    return G.Workload(
        name=f"hub{n_leaves}", pos=pos, nbr_ptr=ptr, nbr_idx=idx,
        n_H=np.full(n, 1e-3), volume=np.full(n, 1e61), bin_dirs=G.icosahedral_bins_42(),
        src_vertex=np.array([0], np.int32), src_rate=np.array([1e48]), dt=3e12,
        n_sweeps=10, precision=precision, box=6e20)


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_largest_bin_count(sxctx, prec):
    w = G.small_random(1500, seed=91, n_bins=96, box=3e21, rate=1e48, n_src=2,
                       dt=3e13, precision=prec)
    _compare(sxctx, w, 20, "96 bins")


def test_single_bin(sxctx):
    w = G.small_random(600, seed=92, n_bins=1, box=3e21, rate=1e48, n_src=3, dt=3e13)
    _compare(sxctx, w, 15, "one bin")


@pytest.mark.parametrize("mpb", [1, 2])
def test_fewer_neighbours_per_bin(sxctx, mpb):
    w = G.small_random(900, seed=93, n_bins=42, box=3e21, rate=1e48, n_src=2, dt=3e13)
    _compare(sxctx, G.with_(w, max_per_bin=mpb), 15, f"{mpb} per bin")


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_high_degree_vertex(sxctx, prec):
    _compare(sxctx, _hub(120, prec), 10, "hub of degree 120")


def test_limits_just_past_supported(sxctx):
    with pytest.raises(sx.SxError) as e:
        sxctx.upload(_hub(sx.SX_MAX_DEGREE + 1))
    assert e.value.code == sx.SX_ENOTSUP
    w = G.small_random(300, seed=94, n_bins=sx.SX_MAX_BINS + 1)
    with pytest.raises(sx.SxError) as e:
        sxctx.upload(w)
    assert e.value.code == sx.SX_ENOTSUP
    with pytest.raises(sx.SxError) as e:
        sxctx.upload(G.with_(G.small_random(300, seed=95), max_per_bin=4))
    assert e.value.code == sx.SX_EINVAL



@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_thick_cells_pass_their_tiny_share(sxctx, prec):
    """Cells of optical depth ~40: what they pass on (~e^-40 of what comes
    in) is kept, not rounded away, so the escaped tally agrees with the
    oracle relative to its own size."""
    w = G.with_(G.stromgren_test(512, seed=11, n_bins=21, bins_seed=5, n_sweeps=20,
                                 t_end_myr=50.0, name="thick"), precision=prec)
    gid = sxctx.upload(w)
    try:
        sxctx.solve([gid], w.n_sweeps)
        got = sxctx.state(gid)["tallies"]
    finally:
        sxctx.free(gid)
    o = Oracle(w)
    tau = o.tables()["tau"]
    o.run(w.n_sweeps)
    ref = o.state()["tallies"]
    o.close()
    assert np.median(tau) > 20
    assert ref["escaped"] > 0
    rel = 1e-9 if prec == G.SX_FP64 else 1e-4
    for key in ("emitted", "absorbed", "escaped", "in_flight"):
        assert abs(got[key] - ref[key]) <= rel * abs(ref[key]), (key, got[key], ref[key])
