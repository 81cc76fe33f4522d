"""Parity at the benchmark's full size and for the shadowing problem.

The 262144-vertex, 84-bin grid is too large for the oracle to replay a whole
solve, so the check is per sweep: the GPU runs 300 sweeps under the
benchmark's launch schedule, its state is handed to the oracle, and one more
sweep on each side is compared element by element.  The shadowing problem
(dense clump, plane source as beam sources) is compared whole at a size the
oracle finishes in seconds."""
import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx
from oracle import Oracle
from parity import assert_edges_close, assert_state_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full_grid():
    print("[case] building the 262144-vertex grid and its oracle tables", flush=True)
    w = G.config2(precision=G.SX_FP32_TRANSPORT)
    ora = Oracle(w)
    print("[case] built", flush=True)
    yield w, ora
    ora.close()


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_full_size_one_sweep(full_grid, prec):
    w0, ora = full_grid
    w = G.with_(w0, precision=prec)
    with sx.Context(0) as ctx:
        ctx.set_schedule([], tiles_per_group=4, order=sx.SX_ORDER_GRID, xcd_contiguous=1,
                         graph_sweeps=50)
        gid = ctx.upload(w)
        print(f"[case] full size prec={prec}: 300 sweeps on the GPU", flush=True)
        ctx.solve([gid], 300)
        s1 = ctx.state(gid, photons=True)
        ctx.solve([gid], 1)
        s2 = ctx.state(gid, photons=True)
        unit = ctx.info(gid)["photon_unit"]
    print(f"[case] full size prec={prec}: one oracle sweep from the GPU state", flush=True)
    ora.set_state(y=s1["y"], photons=s1["photons"], tallies=s1["tallies"])
    ora.run(1)
    ref = ora.state()
    assert_state_close(s2, ref, prec, unit, f"full size one sweep, prec {prec}")
    # the front has moved well into the grid: the comparison covers lit cells
    assert np.count_nonzero(s2["x"] > 0.5) > 1000


@pytest.mark.parametrize("prec", [G.SX_FP32_TRANSPORT, G.SX_FP64])
def test_full_size_one_sweep_combined(full_grid, prec):
    """Combined transport (switch at optical depth 1) at the benchmark's size
    and launch configuration: 300 steps on the GPU, then one step on each
    side from the GPU's state, bins and per-edge packets."""
    w0, ora = full_grid
    w = G.with_(w0, precision=prec, transport=G.SX_TRANSPORT_COMBINED, tau_switch=1.0)
    with sx.Context(0) as ctx:
        ctx.set_schedule([], graph_sweeps=50)
        gid = ctx.upload(w)
        print(f"[case] full size combined prec={prec}: 300 sweeps on the GPU", flush=True)
        ctx.solve([gid], 300)
        s1, e1 = ctx.state(gid, photons=True), ctx.edge_state(gid)
        ctx.solve([gid], 1)
        s2, e2 = ctx.state(gid, photons=True), ctx.edge_state(gid)
        unit = ctx.info(gid)["photon_unit"]
    lay = e1["layout"]
    assert np.count_nonzero(lay == 0) > 1000 and np.count_nonzero(lay == 1) > 1000
    print(f"[case] full size combined prec={prec}: one oracle sweep", flush=True)
    ora.set_transport(True, 1.0)
    try:
        ora.set_state(y=s1["y"], photons=s1["photons"], tallies=s1["tallies"])
        ora.set_edge_state(photons_e=e1["photons_e"], layout=lay.astype(np.int8))
        ora.run(1)
        ref, ref_e = ora.state(), ora.edge_state()
    finally:
        ora.set_transport(False)
    assert_state_close(s2, ref, prec, unit, f"full size combined, prec {prec}")
    assert_edges_close(e2, ref_e, prec, unit, f"full size combined, prec {prec}")


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_shadow_problem_small(prec):
    """Dense clump, plane-parallel source as beams along +x, points drawn
    with density proportional to n_H^(1/3)."""
    w = G.shadow_test(n=12000, n_sweeps=150, precision=prec)
    print(f"[case] shadow n={w.n} sources={len(w.src_vertex)} prec={prec}", flush=True)
    with sx.Context(0) as ctx:
        gid = ctx.upload(w)
        ctx.solve([gid], 60)
        got = ctx.state(gid, photons=True)
        unit = ctx.info(gid)["photon_unit"]
    ora = Oracle(w)
    ora.run(60)
    ref = ora.state()
    ora.close()
    assert_state_close(got, ref, prec, unit, f"shadow prec {prec}")
