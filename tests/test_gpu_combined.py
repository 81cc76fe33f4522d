"""Combined ballistic / direction-conserving transport on the GPU against
the oracle: the ballistic tables bit for bit, whole solves where the mode
decisions cannot differ, one step from a shared state at the benchmark's
size, the exact straight-line lattice, batches that mix transport modes,
checkpoint restore and the refused rotation."""
import math

import numpy as np
import pytest

import oracle_pins as P
from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx
from oracle import Oracle
from parity import assert_edges_close, assert_state_close

pytestmark = pytest.mark.gpu

CT = G.SX_TRANSPORT_COMBINED


def _work(n=2000, seed=61, k=42, prec=G.SX_FP64, tau_switch=1.0, rate=3e45):
    w = G.small_random(n, seed=seed, n_bins=k, box=3e21, rate=rate, n_src=3, dt=3e13,
                       precision=prec)
    sd = np.zeros((3, 3))
    sd[1] = [0.0, 0.6, 0.8]   # one beam source
    return G.with_(w, src_dir=sd, transport=CT, tau_switch=tau_switch)


def _gpu_run(ctx, w, sweeps):
    gid = ctx.upload(w)
    try:
        ctx.solve([gid], sweeps)
        st = ctx.state(gid, photons=True)
        es = ctx.edge_state(gid)
        unit = ctx.info(gid)["photon_unit"]
    finally:
        ctx.free(gid)
    return st, es, unit


def _oracle_run(w, sweeps):
    o = Oracle(w)
    o.run(sweeps)
    st, es = o.state(), o.edge_state()
    o.close()
    return st, es


def test_ballistic_tables_bit_exact(sxctx):
    for w in (_work(800, seed=62), G.with_(_work(600, seed=63), max_per_bin=2)):
        print(f"[case] ballistic tables n={w.n} mpb={w.max_per_bin}", flush=True)
        gid = sxctx.upload(w)
        try:
            got = sxctx.ballistic(gid)
            tab = sxctx.tables(gid)
        finally:
            sxctx.free(gid)
        o = Oracle(w)
        ref = o.ballistic()
        ot = o.tables()
        o.close()
        assert np.array_equal(got["bm"], ref["bm"])
        assert np.array_equal(got["bsel"][:, :w.max_per_bin], ref["bsel"])
        assert np.array_equal(tab["sel_m"], ot["sel_m"])


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_all_ballistic_solve(sxctx, prec):
    """Switch 0: every vertex ballistic in every step (no decision can differ
    between the two sides), whole solve compared."""
    w = _work(prec=prec, tau_switch=0.0)
    print(f"[case] all ballistic prec={prec}", flush=True)
    st, es, unit = _gpu_run(sxctx, w, 40)
    rs, re_ = _oracle_run(w, 40)
    assert es["layout"].all()
    assert_state_close(st, rs, prec, unit, "all ballistic")
    assert_edges_close(es, re_, prec, unit, "all ballistic")


def test_combined_solve_fp64(sxctx):
    """The paper's switch (optical depth 1): ionised vertices turn
    direction-conserving as the fronts pass; fp64 on both sides."""
    w = _work(tau_switch=1.0)
    print("[case] combined fp64, switch 1", flush=True)
    st, es, unit = _gpu_run(sxctx, w, 60)
    rs, re_ = _oracle_run(w, 60)
    lay = es["layout"]
    assert lay.any() and (lay == 0).any(), "both modes in use"
    assert_state_close(st, rs, G.SX_FP64, unit, "combined fp64")
    assert_edges_close(es, re_, G.SX_FP64, unit, "combined fp64")


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_combined_one_step_from_shared_state(sxctx, prec):
    """Mixed modes in both precisions: the GPU's state after 50 steps is
    handed to the oracle and one more step is compared (both sides take the
    mode decisions from the same neutral fractions)."""
    w = _work(3000, seed=64, prec=prec, tau_switch=1.0)
    print(f"[case] combined one step prec={prec}", flush=True)
    _one_step_after(sxctx, w, prec, 50, f"one step prec {prec}")


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_combined_largest_bin_count(sxctx, prec):
    """96 bins: selection masks and per-edge bin lists past bin 64, and in
    fp64 all 48 bin blocks of a vertex (the per-block flags of photons from
    ballistic senders).  Mixed modes, one step from a shared state."""
    w = _work(3000, seed=65, k=96, prec=prec, tau_switch=1.0)
    print(f"[case] combined 96 bins prec={prec}", flush=True)
    _one_step_after(sxctx, w, prec, 50, f"96 bins prec {prec}")


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_bin_lists_longer_than_the_lds_stage(sxctx, prec):
    """cos_min -0.99 on a chain: every bin of a vertex selects both
    neighbours, so each in-edge's bin list holds all 96 bins, and the lists
    of one workgroup (256 x 96 bytes) exceed the LDS stage of the list fill,
    which then writes them directly.  Mixed modes, one step from a shared
    state."""
    kpc = G.KPC_CM
    w = G.chain_graph(600, 0.02 * kpc, 1e-2, 1e62, bins=G.random_bins(96, 7))
    w = G.with_(w, cos_min=-0.99, transport=CT, tau_switch=1.0, dt=3e13,
                src_rate=np.array([1e48]), precision=prec)
    print(f"[case] long bin lists prec={prec}", flush=True)
    _one_step_after(sxctx, w, prec, 40, f"long bin lists prec {prec}")


def _one_step_after(sxctx, w, prec, steps, label):
    gid = sxctx.upload(w)
    try:
        sxctx.solve([gid], steps)
        s1, e1 = sxctx.state(gid, photons=True), sxctx.edge_state(gid)
        sxctx.solve([gid], 1)
        s2, e2 = sxctx.state(gid, photons=True), sxctx.edge_state(gid)
        unit = sxctx.info(gid)["photon_unit"]
    finally:
        sxctx.free(gid)
    assert e1["layout"].any() and (e1["layout"] == 0).any()
    o = Oracle(w)
    o.set_state(y=s1["y"], photons=s1["photons"], tallies=s1["tallies"])
    o.set_edge_state(photons_e=e1["photons_e"], layout=e1["layout"].astype(np.int8))
    o.run(1)
    rs, re_ = o.state(), o.edge_state()
    o.close()
    assert_state_close(s2, rs, prec, unit, label)
    assert_edges_close(e2, re_, prec, unit, label)


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_lattice_straight_lines_exact(sxctx, prec):
    """Both conversions on the lattice where every path is straight: exact
    photon counts, layouts and escapes."""
    w = G.with_(P.lattice_two_regions(), precision=prec)
    print(f"[case] lattice prec={prec}", flush=True)
    st, es, unit = _gpu_run(sxctx, w, w.n_sweeps)
    O, Oe, layout, escaped = P.lattice_expected(w)
    assert np.array_equal(es["layout"].astype(np.int8), layout)
    assert np.array_equal(st["photons"], O)
    assert np.array_equal(es["photons_e"], Oe)
    t = st["tallies"]
    assert t["emitted"] == 18.0 * w.n_sweeps
    assert t["escaped"] == escaped
    assert t["in_flight"] == O.sum() + Oe.sum()


def test_batches_mix_transport_modes():
    """DCT and combined grids of both precisions solved in one batch give
    each grid's result alone, bit for bit."""
    ws = [_work(900, seed=65, tau_switch=1.0),
          G.small_random(700, seed=66, n_bins=21, box=3e21, rate=1e47, n_src=2, dt=3e13),
          _work(1100, seed=67, prec=G.SX_FP32_TRANSPORT, tau_switch=0.5),
          G.small_random(500, seed=68, n_bins=42, box=3e21, rate=1e47, n_src=1, dt=3e13,
                         precision=G.SX_FP32_TRANSPORT)]
    sweeps = [30, 25, 40, 20]
    print("[case] mixed batch of 4 grids", flush=True)
    with sx.Context(0) as ctx:
        alone = []
        for w, s in zip(ws, sweeps):
            gid = ctx.upload(w)
            ctx.solve([gid], s)
            alone.append(ctx.state(gid, photons=True))
            ctx.free(gid)
        gids = [ctx.upload(w) for w in ws]
        ctx.solve(gids, sweeps)
        for a, gid, w in zip(alone, gids, ws):
            b = ctx.state(gid, photons=True)
            assert np.array_equal(a["y"], b["y"]), w.name
            assert np.array_equal(a["photons"], b["photons"]), w.name
            assert a["tallies"] == b["tallies"], w.name


def test_checkpoint_restore_edges(sxctx):
    """State and per-edge state read back, restored into a fresh grid, and
    both continued: the same evolution to the photon tolerance."""
    w = _work(1500, seed=69, tau_switch=1.0)
    print("[case] restore with edges", flush=True)
    a = sxctx.upload(w)
    b = sxctx.upload(w)
    try:
        sxctx.solve([a], 30)
        st, es = sxctx.state(a, photons=True), sxctx.edge_state(a)
        sxctx.restore(b, y=st["y"], photons=st["photons"], tallies=st["tallies"])
        sxctx.restore_edges(b, es["photons_e"], es["layout"])
        e2 = sxctx.edge_state(b)
        assert np.array_equal(e2["layout"], es["layout"])
        sxctx.solve([a], 10)
        sxctx.solve([b], 10)
        sa, sb = sxctx.state(a, photons=True), sxctx.state(b, photons=True)
        unit = sxctx.info(a)["photon_unit"]
        assert_state_close(sb, sa, G.SX_FP64, unit, "restored")
        assert_edges_close(sxctx.edge_state(b), sxctx.edge_state(a), G.SX_FP64, unit,
                           "restored")
    finally:
        sxctx.free(a)
        sxctx.free(b)


@pytest.mark.parametrize("prec,k", [(G.SX_FP64, 42), (G.SX_FP32_TRANSPORT, 42),
                                    (G.SX_FP32_TRANSPORT, 96)])
def test_combined_rotated(sxctx, prec, k):
    """Combined transport with the bins rotated between steps (as the
    paper does for its direction-conserving part): the bin selection, the
    edge bins and the per-edge lists are rebuilt on the device.  fp64: whole
    solve; fp32: one step from the GPU's state after the rotations.  96
    bins: the selection's pass over bins 64..95 and mask bits past 64."""
    w = _work(2000, seed=75, k=k, prec=prec, tau_switch=1.0)
    Rs = G.random_rotations(3, seed=11)
    print(f"[case] combined rotated prec={prec} k={k}", flush=True)
    gid = sxctx.upload(w)
    o = Oracle(w)
    try:
        for R in Rs:
            sxctx.solve([gid], 15)
            sxctx.rotate(gid, R)
            o.run(15)
            o.rotate(R)
        tab = sxctx.tables(gid)
        ot = o.tables()
        assert np.array_equal(tab["sel_m"], ot["sel_m"])
        assert np.array_equal(tab["edge_bin"], ot["edge_bin"])
        if prec == G.SX_FP32_TRANSPORT:
            s1, e1 = sxctx.state(gid, photons=True), sxctx.edge_state(gid)
            o.set_state(y=s1["y"], photons=s1["photons"], tallies=s1["tallies"])
            o.set_edge_state(photons_e=e1["photons_e"], layout=e1["layout"].astype(np.int8))
            sxctx.solve([gid], 1)
            o.run(1)
        else:
            sxctx.solve([gid], 15)
            o.run(15)
        st, es = sxctx.state(gid, photons=True), sxctx.edge_state(gid)
        unit = sxctx.info(gid)["photon_unit"]
        ref, ref_e = o.state(), o.edge_state()
    finally:
        sxctx.free(gid)
        o.close()
    assert es["layout"].any() and (es["layout"] == 0).any()
    assert_state_close(st, ref, prec, unit, f"combined rotated prec {prec} k {k}")
    assert_edges_close(es, ref_e, prec, unit, f"combined rotated prec {prec} k {k}")


def test_combined_limits(sxctx):
    d = sxctx.upload(G.small_random(300, seed=71, n_bins=21))
    try:
        with pytest.raises(sx.SxError) as e:
            sxctx.edge_state(d)
        assert e.value.code == sx.SX_EINVAL
    finally:
        sxctx.free(d)


# ------------------------------------------- edge reference of the bins ---

def _edge_ref(n=1500, seed=72, prec=G.SX_FP64, k=42):
    w = G.small_random(n, seed=seed, n_bins=k, box=3e21, rate=3e45, n_src=3, dt=3e13,
                       precision=prec)
    return G.with_(w, dct_reference=G.SX_DCT_REF_EDGE)


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_edge_reference_tables_and_solve(sxctx, prec):
    """Bins tied to their closest edge: selection bit for bit, whole solve."""
    w = _edge_ref(prec=prec)
    print(f"[case] edge reference prec={prec}", flush=True)
    gid = sxctx.upload(w)
    try:
        tab = sxctx.tables(gid)
        sxctx.solve([gid], 40)
        st = sxctx.state(gid, photons=True)
        unit = sxctx.info(gid)["photon_unit"]
    finally:
        sxctx.free(gid)
    o = Oracle(w)
    ot = o.tables()
    o.run(40)
    ref = o.state()
    o.close()
    assert np.array_equal(tab["sel_m"], ot["sel_m"])
    assert np.array_equal(tab["sel_nbr"][:, :, :w.max_per_bin], ot["sel_nbr"])
    assert_state_close(st, ref, prec, unit, f"edge reference prec {prec}")


def test_edge_reference_rotated(sxctx):
    """The edge reference after a rotation of the bins (rebuilt on the
    device) against the oracle's rotation.  The rotation comes after an odd
    number of steps and needs a larger overflow pool than the upload: the
    step count and buffer parity on the device survive the rebuild."""
    w = _edge_ref(1200, seed=73)
    R = G.random_rotations(1, seed=7)[0]
    print("[case] edge reference rotated", flush=True)
    gid = sxctx.upload(w)
    try:
        sxctx.solve([gid], 11)
        before = sxctx.info(gid)["bytes"]
        sxctx.rotate(gid, R)
        # the rotated routing needs more overflow records: the pool grew
        assert sxctx.info(gid)["bytes"] > before
        tab = sxctx.tables(gid)
        sxctx.solve([gid], 9)
        st = sxctx.state(gid, photons=True)
        unit = sxctx.info(gid)["photon_unit"]
    finally:
        sxctx.free(gid)
    o = Oracle(w)
    o.run(11)
    o.rotate(R)
    ot = o.tables()
    o.run(9)
    ref = o.state()
    o.close()
    assert st["tallies"]["sweeps"] == 20
    assert np.array_equal(tab["sel_m"], ot["sel_m"])
    assert np.array_equal(tab["sel_nbr"], ot["sel_nbr"])
    assert_state_close(st, ref, G.SX_FP64, unit, "edge reference rotated")


def test_edge_reference_combined(sxctx):
    """Combined transport with the edge reference for its
    direction-conserving part."""
    w = G.with_(_work(1500, seed=74, tau_switch=1.0), dct_reference=G.SX_DCT_REF_EDGE)
    print("[case] edge reference + combined", flush=True)
    st, es, unit = _gpu_run(sxctx, w, 50)
    rs, re_ = _oracle_run(w, 50)
    assert_state_close(st, rs, G.SX_FP64, unit, "edge reference combined")
    assert_edges_close(es, re_, G.SX_FP64, unit, "edge reference combined")


def _knn_workload(n=1500, k=28, seed=5, **kw):
    """A symmetric k-nearest-neighbour graph (not a Delaunay graph): about
    32 neighbours per vertex, so a 64-vertex tile has ~2000 incoming edges,
    more than the combined-transport kernel sums through LDS."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    box = 3e21
    pos = rng.random((n, 3)) * box
    _, nn = cKDTree(pos).query(pos, k=k + 1)
    rows = [set() for _ in range(n)]
    for i in range(n):
        for j in nn[i, 1:]:
            rows[i].add(int(j))
            rows[int(j)].add(i)
    ptr = np.zeros(n + 1, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in sorted(r)], np.int32)
    src = np.array([0, n // 2], np.int32)
    w = G.Workload(name="knn", pos=pos, nbr_ptr=ptr, nbr_idx=idx, n_H=np.full(n, 1e-3),
                   volume=np.full(n, box ** 3 / n), bin_dirs=G.icosahedral_bins_42(),
                   src_vertex=src, src_rate=np.full(2, 3e45), dt=3e13, n_sweeps=40, box=box)
    return G.with_(w, **kw)


@pytest.mark.parametrize("kw", [dict(transport=G.SX_TRANSPORT_COMBINED, tau_switch=1.0),
                                dict(transport=G.SX_TRANSPORT_COMBINED, tau_switch=1.0,
                                     alpha_A=G.ALPHA_A)])
def test_tiles_with_many_incoming_edges(sxctx, kw):
    """Tiles whose incoming edges exceed what the kernel sums through LDS take
    the per-lane path; the result is the same as the oracle's."""
    w = _knn_workload(**kw)
    assert 64 * np.diff(w.nbr_ptr).mean() > 1536
    print(f"[case] many incoming edges {kw}", flush=True)
    st, es, unit = _gpu_run(sxctx, w, 40)
    rs, re_ = _oracle_run(w, 40)
    assert es["layout"].any() and (es["layout"] == 0).any()
    assert_state_close(st, rs, G.SX_FP64, unit, "many incoming edges")
    assert_edges_close(es, re_, G.SX_FP64, unit, "many incoming edges")
