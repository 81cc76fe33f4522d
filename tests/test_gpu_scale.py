"""Parity at the sizes the benchmark runs: the routing tables of the
262144-vertex and the 1M-vertex grids bit for bit, one sweep of the 1M-vertex
shadowing problem (photon planes larger than the last-level cache, beam
sources) from the GPU's own state, and members of the 64-grid batch run
inside the batch's tile map against the oracle run alone."""
import multiprocessing as mp
import os

import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx
from oracle import Oracle
from parity import assert_state_close

pytestmark = pytest.mark.gpu


def _tables_equal(tab, ot, w, what):
    assert np.array_equal(tab["sel_m"], ot["sel_m"]), f"{what}: m(i,k) differs"
    sel = tab["sel_nbr"][:, :, : w.max_per_bin]
    assert np.array_equal(sel, ot["sel_nbr"]), f"{what}: selected neighbours differ"
    assert np.array_equal(tab["edge_bin"], ot["edge_bin"]), f"{what}: edge bins differ"
    np.testing.assert_array_equal(tab["dL"], ot["dL"])
    np.testing.assert_array_equal(tab["tau"], ot["tau"])


def test_tables_262144(sxctx):
    """The Stromgren benchmark grid (262144 vertices, 84 bins)."""
    print("[case] tables 262144 x 84: building grid and oracle", flush=True)
    w = G.config2(precision=G.SX_FP32_TRANSPORT)
    ora = Oracle(w)
    gid = sxctx.upload(w)
    try:
        tab = sxctx.tables(gid)
    finally:
        sxctx.free(gid)
    _tables_equal(tab, ora.tables(), w, "262144")
    ora.close()


@pytest.fixture(scope="module")
def shadow_full():
    print("[case] building the 1,048,576-vertex shadowing grid", flush=True)
    w = G.shadow_test()
    print(f"[case] built: {w.n} vertices, {w.n_edges} edges, {len(w.src_vertex)} beam "
          "sources; oracle tables", flush=True)
    ora = Oracle(w)
    yield w, ora
    ora.close()


def test_tables_shadow_full_size(sxctx, shadow_full):
    w, ora = shadow_full
    gid = sxctx.upload(w)
    try:
        tab = sxctx.tables(gid)
    finally:
        sxctx.free(gid)
    _tables_equal(tab, ora.tables(), w, "shadow 1M")


def test_shadow_full_size_one_sweep(shadow_full):
    """300 sweeps on the GPU under the benchmark's schedule (its photon
    planes, 704 MB, exceed the 256 MB last-level cache, so the in-words are
    loaded without the non-temporal hint), then one sweep on each side from
    the GPU's state."""
    w, ora = shadow_full
    with sx.Context(0) as ctx:
        ctx.set_schedule([], tiles_per_group=4, order=sx.SX_ORDER_GRID, xcd_contiguous=1,
                         graph_sweeps=50)
        gid = ctx.upload(w)
        print("[case] shadow 1M: 300 sweeps on the GPU", flush=True)
        ctx.solve([gid], 300)
        s1 = ctx.state(gid, photons=True)
        ctx.solve([gid], 1)
        s2 = ctx.state(gid, photons=True)
        unit = ctx.info(gid)["photon_unit"]
    print("[case] shadow 1M: one oracle sweep from the GPU state", flush=True)
    ora.set_state(y=s1["y"], photons=s1["photons"], tallies=s1["tallies"])
    ora.run(1)
    ref = ora.state()
    assert_state_close(s2, ref, G.SX_FP32_TRANSPORT, unit, "shadow 1M one sweep")
    assert np.count_nonzero(s2["x"] > 0.5) > 10000


def _member(g):
    return G.batch_member(g)


def test_batch_members_against_oracle(sxctx):
    """The 64-grid batch (vertex counts log-uniform in [4096, 262144], 42
    bins, FP32 transport) runs 20 sweeps as one batch under the benchmark's
    schedule; four members are compared element by element with the oracle
    running each alone."""
    workers = max(1, min(16, os.cpu_count() or 1))
    print(f"[case] building the 64 batch grids on {workers} processes", flush=True)
    with mp.get_context("fork").Pool(workers) as pool:
        ws = pool.map(_member, range(64), chunksize=1)
    print(f"[case] batch: {sum(w.n for w in ws)} vertices", flush=True)
    with sx.Context(0) as ctx:
        ids = [ctx.upload(w) for w in ws]
        ctx.set_schedule(ids, tiles_per_group=4, order=sx.SX_ORDER_GRID, xcd_contiguous=1,
                         graph_sweeps=10)
        ctx.solve(ids, [20] * len(ids))
        picks = [0, 17, 42, 63]
        got = {g: ctx.state(ids[g], photons=True) for g in picks}
        units = {g: ctx.info(ids[g])["photon_unit"] for g in picks}
    for g in picks:
        print(f"[case] batch member {g}: {ws[g].n} vertices, oracle 20 sweeps", flush=True)
        o = Oracle(ws[g])
        o.run(20)
        assert_state_close(got[g], o.state(), G.SX_FP32_TRANSPORT, units[g], f"batch member {g}")
        o.close()
