"""Dynamic grid between solves on the GPU against the oracle: the removal
set bit for bit from the same state, the state moved onto the thinned grid,
and the solve continued on it."""
import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import regrid as RG
from oracle import Oracle
from oracle.regrid import remap, select_removal
from parity import assert_state_close

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
