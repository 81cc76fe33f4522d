"""Dynamic grid between solves on the GPU against the oracle: the removal
set bit for bit from the same state, the state moved onto the thinned grid,
and the solve continued on it; also with combined transport and diffuse
recombination radiation (edge holdings filed in bins, pending photons
moved)."""
import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import regrid as RG
from paper_0912_4273_amd import sx
from oracle import Oracle
from oracle.regrid import edge_holdings_as_bins, remap, remap_pending, select_removal
from parity import TOL, assert_edges_close, assert_state_close, close

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_regrid_matches_oracle(sxctx, prec):
    w = G.small_random(3000, seed=41, n_bins=42, box=3e21, rate=3e45, n_src=2, dt=3e13,
                       precision=prec)
    tau_rm, spacing = 0.5, None
    print(f"[case] regrid prec={prec}", flush=True)
    gid = sxctx.upload(w)
    gn = None
    try:
        sxctx.solve([gid], 60)
        st = sxctx.state(gid, photons=True)
        tab = sxctx.tables(gid)
        spacing = 1.3 * float(np.median(tab["dL"]))
        rm = sxctx.select_removal(gid, tau_rm, spacing)
        wn, gn, new_of_old = RG.regrid(sxctx, gid, w, tau_rm, spacing)
        s_after = sxctx.state(gn, photons=True)
        unit = sxctx.info(gn)["photon_unit"]
        m_new_gpu = sxctx.tables(gn)["sel_m"]
        sxctx.solve([gn], 20)
        s_end = sxctx.state(gn, photons=True)
    finally:
        sxctx.free(gid)
        if gn is not None:
            sxctx.free(gn)
    assert 0 < rm.sum() < w.n
    # the oracle's own removal set from the same neutral fractions
    o = Oracle(w)
    ot = o.tables()
    o.close()
    rm_o = select_removal(w, st["y"], ot["tau"], ot["dL"], tau_rm, spacing)
    assert np.array_equal(rm, rm_o)
    assert np.array_equal(new_of_old >= 0, ~rm_o)
    # the thinned grid (same points, same triangulation) and the moved state
    keep = ~rm_o
    pts = w.pos[keep]
    ptr, idx, simp = G.delaunay(pts)
    assert np.array_equal(ptr, wn.nbr_ptr) and np.array_equal(idx, wn.nbr_idx)
    ora = Oracle(wn)
    m_new = ora.tables()["sel_m"]
    assert np.array_equal(m_new, m_new_gpu)
    y_new, ph_new, lost = remap(w, st["y"], st["photons"], tab["sel_m"], new_of_old, m_new)
    tl = dict(st["tallies"])
    tl["escaped"] += lost
    tl["in_flight"] = float(np.sum(ph_new * m_new))
    ref = dict(y=y_new, x=1.0 - y_new, photons=ph_new, nin=None, tallies=tl)
    assert_state_close(dict(s_after, nin=None), ref, prec, unit, f"remapped prec {prec}")
    ora.set_state(y=y_new, photons=ph_new, tallies=tl)
    ora.run(20)
    ref_end = ora.state()
    ora.close()
    assert_state_close(s_end, ref_end, prec, unit, f"after regrid prec {prec}")


@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_regrid_combined_diffuse_matches_oracle(sxctx, prec):
    """Combined transport (ballistic where y tau >= 0.3, so vertices that may
    be removed can hold edges) with diffuse radiation: the moved state
    against the oracle's rule applied to the GPU's own state, then one step
    from it on both sides."""
    w = G.small_random(3000, seed=42, n_bins=42, box=3e21, rate=3e45, n_src=2, dt=3e13,
                       precision=prec)
    w = G.with_(w, transport=G.SX_TRANSPORT_COMBINED, tau_switch=0.3, alpha_A=G.ALPHA_A)
    tau_rm = 0.5
    print(f"[case] regrid combined diffuse prec={prec}", flush=True)
    gid = sxctx.upload(w)
    gn = None
    try:
        sxctx.solve([gid], 60)
        st = sxctx.state(gid, photons=True)
        es = sxctx.edge_state(gid)
        pend = sxctx.diffuse_pending(gid)
        tab = sxctx.tables(gid)
        bal = sxctx.ballistic(gid)
        spacing = 1.3 * float(np.median(tab["dL"]))
        wn, gn, new_of_old = RG.regrid(sxctx, gid, w, tau_rm, spacing)
        s_after = sxctx.state(gn, photons=True)
        e_after = sxctx.edge_state(gn)
        p_after = sxctx.diffuse_pending(gn)
        unit = sxctx.info(gn)["photon_unit"]
        m_new_gpu = sxctx.tables(gn)["sel_m"]
        sxctx.solve([gn], 1)
        s_end, e_end, p_end = (sxctx.state(gn, photons=True), sxctx.edge_state(gn),
                               sxctx.diffuse_pending(gn))
    finally:
        sxctx.free(gid)
        if gn is not None:
            sxctx.free(gn)
    rm = new_of_old < 0
    assert 0 < rm.sum() < w.n
    assert es["layout"].any() and (es["layout"] == 0).any() and pend.sum() > 0
    o = Oracle(w)
    ot, ob = o.tables(), o.ballistic()
    o.close()
    assert np.array_equal(ot["edge_bin"], tab["edge_bin"]) and np.array_equal(ob["bm"], bal["bm"])
    ex = edge_holdings_as_bins(w, es["photons_e"], es["layout"], ob["bm"], ot["edge_bin"])
    ora = Oracle(wn)
    m_new = ora.tables()["sel_m"]
    assert np.array_equal(m_new, m_new_gpu)
    y_new, ph_new, lost = remap(w, st["y"], st["photons"], tab["sel_m"], new_of_old, m_new,
                                extra=ex)
    pn, lost_p = remap_pending(w, pend, new_of_old)
    tl = dict(st["tallies"])
    tl["escaped"] += lost + lost_p
    tl["in_flight"] = float(np.sum(ph_new * m_new)) + float(pn.sum())
    ref = dict(y=y_new, x=1.0 - y_new, photons=ph_new, nin=None, tallies=tl)
    what = f"combined diffuse remapped prec {prec}"
    assert_state_close(dict(s_after, nin=None), ref, prec, unit, what)
    assert not e_after["layout"].any()
    rt, at = TOL[prec]["ph"]
    ok, nbad, worst = close(p_after, pn, rt, at * unit)
    assert ok, f"{what} pending: {nbad} off, worst rel {worst:.3e}"
    ora.set_state(y=y_new, photons=ph_new, tallies=tl)
    ora.set_edge_state(photons_e=np.zeros(wn.n_edges), layout=np.zeros(wn.n, np.int8))
    ora.set_diffuse_pending(pn)
    ora.run(1)
    ref_end, ref_e, ref_p = ora.state(), ora.edge_state(), ora.diffuse_pending()
    ora.close()
    what = f"combined diffuse after regrid prec {prec}"
    assert_state_close(s_end, ref_end, prec, unit, what)
    assert_edges_close(e_end, ref_e, prec, unit, what)
    ok, nbad, worst = close(p_end, ref_p, rt, at * unit)
    assert ok, f"{what} pending: {nbad} off, worst rel {worst:.3e}"


def test_regrid_refuses_mixed_physics(sxctx):
    """The two grids must carry the same transport and radiation."""
    w = G.small_random(600, seed=43, n_bins=21, box=3e21, rate=3e45, n_src=1, dt=3e13)
    wc = G.with_(w, transport=G.SX_TRANSPORT_COMBINED, tau_switch=0.3)
    a = sxctx.upload(w)
    b = sxctx.upload(wc)
    try:
        with pytest.raises(sx.SxError) as ei:
            sxctx.remap(a, b, np.arange(w.n, dtype=np.int32))
        assert ei.value.code == sx.SX_EINVAL
    finally:
        sxctx.free(a)
        sxctx.free(b)
