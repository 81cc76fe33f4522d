"""Pins of the oracle's dynamic-grid step (Sect. 2.1.4): the removal set and
the state moved onto the thinned grid."""
import numpy as np

from paper_0912_4273_amd import gridgen as G
from oracle import Oracle
from oracle.regrid import remap, select_removal


def _field(w, seed=3):
    """A neutral fraction low inside a sphere around the box centre."""
    c = w.pos.mean(axis=0)
    r = np.linalg.norm(w.pos - c, axis=1)
    rng = np.random.default_rng(seed)
    return np.where(r < 0.3 * w.box, 10 ** rng.uniform(-4, -1, w.n), 1.0)


def test_removal_set_rule():
    w = G.small_random(1500, seed=31, n_bins=21, box=3e21, n_src=2)
    t = Oracle(w).tables()
    y = _field(w)
    spacing = 1.2 * float(np.median(t["dL"]))
    rm = select_removal(w, y, t["tau"], t["dL"], 0.5, spacing)
    od = y * t["tau"]
    cand = (od < 0.5) & (t["dL"] < spacing)
    cand[w.src_vertex] = False
    assert rm.any() and not rm[w.src_vertex].any()
    assert np.all(cand[rm])                                   # only candidates go
    for i in np.nonzero(rm)[0]:                               # no two neighbours
        assert not rm[w.nbr_idx[w.nbr_ptr[i]:w.nbr_ptr[i + 1]]].any()
    for i in np.nonzero(cand & ~rm)[0]:                       # maximal: blocked
        nb = w.nbr_idx[w.nbr_ptr[i]:w.nbr_ptr[i + 1]]
        assert rm[nb].any(), i
    # the thinnest candidate always goes
    assert rm[np.nonzero(cand)[0][np.argmin(od[cand])]]


def test_remap_conserves_photons():
    w = G.small_random(800, seed=32, n_bins=21, box=3e21, rate=1e47, n_src=2, dt=3e13)
    o = Oracle(w)
    o.run(15)
    st, t = o.state(), o.tables()
    rm = select_removal(w, st["y"], t["tau"], t["dL"], 0.5, 2.0 * float(np.max(t["dL"])))
    assert rm.any()
    keep = ~rm
    new_of_old = np.full(w.n, -1, np.int32)
    new_of_old[keep] = np.arange(int(keep.sum()))
    pts = w.pos[keep]
    ptr, idx, simp = G.delaunay(pts)
    wn = G.with_(w, pos=pts, nbr_ptr=ptr, nbr_idx=idx, n_H=w.n_H[keep],
                 volume=G.dual_volumes(pts, simp), src_vertex=new_of_old[w.src_vertex])
    m_new = Oracle(wn).tables()["sel_m"]
    y_new, ph_new, lost = remap(w, st["y"], st["photons"], t["sel_m"], new_of_old, m_new)
    before = float(np.sum(st["photons"] * t["sel_m"]))
    after = float(np.sum(ph_new * m_new)) + lost
    assert abs(after - before) <= 1e-12 * before
    assert np.array_equal(y_new, st["y"][keep])


def test_remap_hands_to_nearest_kept():
    """Chain 0-1-2-3-4 along x with 2 closer to 3: removing 2 hands its
    photons to 3, in the same bin."""
    x = np.array([0.0, 1.0, 2.0, 2.6, 3.6])
    pos = np.zeros((5, 3))
    pos[:, 0] = x
    rows = [[1], [0, 2], [1, 3], [2, 4], [3]]
    ptr = np.zeros(6, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in r], np.int32)
    w = G.Workload(name="chain5", pos=pos, nbr_ptr=ptr, nbr_idx=idx, n_H=np.ones(5),
                   volume=np.ones(5), bin_dirs=G.axis_bins(), src_vertex=np.array([0], np.int32),
                   src_rate=np.array([1.0]), dt=1.0, n_sweeps=1)
    ph = np.zeros((5, 6))
    ph[2, 0] = 5.0      # vertex 2 holds 5 photons in +x (one neighbour selected)
    ph[3, 0] = 1.0
    m_old = np.zeros((5, 6), np.int32)
    m_old[:, 0] = [1, 1, 1, 1, 0]
    m_old[:, 1] = [0, 1, 1, 1, 1]
    new_of_old = np.array([0, 1, -1, 2, 3], np.int32)
    m_new = np.zeros((4, 6), np.int32)
    m_new[:, 0] = [1, 1, 1, 0]
    y_new, ph_new, lost = remap(w, np.ones(5), ph, m_old, new_of_old, m_new)
    assert ph_new[2, 0] == 6.0 and ph_new.sum() == 6.0 and lost == 0.0


def _chain5():
    x = np.array([0.0, 1.0, 2.0, 2.6, 3.6])
    pos = np.zeros((5, 3))
    pos[:, 0] = x
    rows = [[1], [0, 2], [1, 3], [2, 4], [3]]
    ptr = np.zeros(6, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in r], np.int32)
    return G.Workload(name="chain5", pos=pos, nbr_ptr=ptr, nbr_idx=idx, n_H=np.ones(5),
                      volume=np.ones(5), bin_dirs=G.axis_bins(),
                      src_vertex=np.array([0], np.int32), src_rate=np.array([1.0]),
                      dt=1.0, n_sweeps=1)


def test_edge_holdings_filed_in_the_bin_of_their_edge():
    """Vertex 2 of the chain holds edges: the packet that came from 1 (along
    +x, bin 0) and the one from 3 (along -x, bin 1), sent to 1 and 2 chosen
    neighbours.  Vertex 1 holds bins, so its per-edge entries count for
    nothing.  Directed edges in row order point +x -> bin 0, -x -> bin 1."""
    w = _chain5()
    edge_bin = np.array([0, 1, 0, 1, 0, 1, 0, 1], np.int32)
    pe = np.zeros(8)
    bm = np.ones(8, np.int32)
    pe[3] = 3.0                 # row 2, slot of neighbour 1
    pe[4], bm[4] = 2.0, 2       # row 2, slot of neighbour 3
    pe[1] = 7.0                 # row 1: a vertex that holds bins
    layout = np.array([0, 0, 1, 0, 0], np.int8)
    from oracle.regrid import edge_holdings_as_bins
    ex = edge_holdings_as_bins(w, pe, layout, bm, edge_bin)
    assert ex[2, 0] == 3.0 and ex[2, 1] == 4.0 and ex.sum() == 7.0


def test_pending_goes_to_nearest_kept():
    from oracle.regrid import remap_pending
    w = _chain5()
    pend = np.array([0.0, 1.0, 5.0, 2.0, 0.5])
    out, lost = remap_pending(w, pend, np.array([0, 1, -1, 2, 3], np.int32))
    assert np.array_equal(out, [0.0, 1.0, 7.0, 0.5]) and lost == 0.0
    # a removed vertex with no kept neighbour: its photons escape
    out, lost = remap_pending(w, pend, np.array([0, 1, 2, -1, -1], np.int32))
    assert lost == 0.5 and out[2] == 7.0


def _thin(w, st, t, tau_rm):
    rm = select_removal(w, st["y"], t["tau"], t["dL"], tau_rm, 2.0 * float(np.max(t["dL"])))
    assert rm.any()
    keep = ~rm
    new_of_old = np.full(w.n, -1, np.int32)
    new_of_old[keep] = np.arange(int(keep.sum()))
    pts = w.pos[keep]
    ptr, idx, simp = G.delaunay(pts)
    wn = G.with_(w, pos=pts, nbr_ptr=ptr, nbr_idx=idx, n_H=w.n_H[keep],
                 volume=G.dual_volumes(pts, simp), src_vertex=new_of_old[w.src_vertex],
                 dL=None, x_init=None)
    return wn, new_of_old


def _conserved(tl):
    return abs(tl["emitted"] - tl["absorbed"] - tl["escaped"] - tl["in_flight"]) / tl["emitted"]


def test_remap_combined_and_diffuse_conserve_photons():
    """Combined transport with diffuse radiation: the photons held in bins
    and on edges plus those waiting to be re-emitted are the oracle's own
    in-flight tally; thinning moves all of them (or counts them escaped),
    and the solve continued on the thinned grid keeps conserving them."""
    from oracle.regrid import edge_holdings_as_bins, remap_pending
    w = G.small_random(900, seed=34, n_bins=21, box=3e21, rate=1e47, n_src=2, dt=3e13)
    w = G.with_(w, transport=G.SX_TRANSPORT_COMBINED, tau_switch=0.3, alpha_A=G.ALPHA_A)
    o = Oracle(w)
    o.run(15)
    st, es, t, bal = o.state(), o.edge_state(), o.tables(), o.ballistic()
    pend = o.diffuse_pending()
    o.close()
    assert es["layout"].any() and (es["layout"] == 0).any() and pend.sum() > 0
    ex = edge_holdings_as_bins(w, es["photons_e"], es["layout"], bal["bm"], t["edge_bin"])
    bins = float(np.sum(st["photons"] * t["sel_m"]))
    fly = st["tallies"]["in_flight"]
    assert abs(bins + ex.sum() + pend.sum() - fly) <= 1e-12 * fly
    wn, new_of_old = _thin(w, st, t, 0.5)
    on = Oracle(wn)
    m_new = on.tables()["sel_m"]
    y_new, ph_new, lost = remap(w, st["y"], st["photons"], t["sel_m"], new_of_old, m_new,
                                extra=ex)
    pn, lost_p = remap_pending(w, pend, new_of_old)
    after = float(np.sum(ph_new * m_new)) + pn.sum()
    assert abs(after + lost + lost_p - fly) <= 1e-12 * fly
    tl = dict(st["tallies"])
    tl["escaped"] += lost + lost_p
    tl["in_flight"] = after
    on.set_state(y=y_new, photons=ph_new, tallies=tl)
    on.set_edge_state(photons_e=np.zeros(wn.n_edges), layout=np.zeros(wn.n, np.int8))
    on.set_diffuse_pending(pn)
    assert _conserved(tl) <= 1e-12
    on.run(10)
    s2 = on.state()
    on.close()
    assert s2["tallies"]["sweeps"] == tl["sweeps"] + 10
    assert _conserved(s2["tallies"]) <= 1e-12
