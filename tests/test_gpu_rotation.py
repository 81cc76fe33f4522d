"""Rotation of the direction bins on the GPU against the oracle: the
rebuilt routing is bit-exact, the photons in flight are re-split as in the
oracle, and the grid state follows it within the parity tolerances."""
import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx
from oracle import Oracle
from parity import assert_state_close

pytestmark = pytest.mark.gpu


def _conserved(t, tol):
    r = t["emitted"] - (t["absorbed"] + t["escaped"] + t["in_flight"])
    assert abs(r) <= tol * t["emitted"], r


@pytest.mark.parametrize("prec,k", [(G.SX_FP64, 42), (G.SX_FP32_TRANSPORT, 42),
                                    (G.SX_FP64, 96), (G.SX_FP32_TRANSPORT, 21)])
def test_rotations_match_oracle(sxctx, prec, k):
    """Tables bit for bit after each rotation and the state at the end.
    96 bins take the selection's pass over bins 64..95; 21 bins leave three
    padding bins in the last fp32 block, whose in-words keep their upload
    value through the rebuilds."""
    w = G.small_random(1500, seed=41, n_bins=k, box=3e21, rate=1e48, n_src=3,
                       dt=3e13, precision=prec)
    Rs = G.random_rotations(3, seed=5)
    plan = [(6, Rs[0]), (9, Rs[1]), (5, Rs[2]), (7, None)]
    print(f"[case] rotations prec={prec} k={k}", flush=True)
    gid = sxctx.upload(w)
    ora = Oracle(w)
    try:
        for n, R in plan:
            sxctx.solve([gid], n)
            ora.run(n)
            if R is not None:
                sxctx.rotate(gid, R)
                ora.rotate(R)
                tab, ot = sxctx.tables(gid), ora.tables()
                assert np.array_equal(tab["sel_m"], ot["sel_m"])
                assert np.array_equal(tab["sel_nbr"][:, :, :w.max_per_bin], ot["sel_nbr"])
                assert np.array_equal(tab["edge_bin"], ot["edge_bin"])
            got = sxctx.state(gid, photons=True)
            _conserved(got["tallies"], 1e-9 if prec == G.SX_FP64 else 1e-4)
        unit = sxctx.info(gid)["photon_unit"]
        assert_state_close(got, ora.state(), prec, unit, f"rotations prec {prec} k {k}")
    finally:
        sxctx.free(gid)
        ora.close()


def test_identity_rotation_changes_nothing(sxctx):
    w = G.with_(G.config1(), precision=G.SX_FP32_TRANSPORT)
    outs = []
    for rot in (False, True):
        gid = sxctx.upload(w)
        sxctx.solve([gid], 30)
        if rot:
            sxctx.rotate(gid, np.eye(3))
        sxctx.solve([gid], 20)
        outs.append(sxctx.state(gid, photons=True))
        sxctx.free(gid)
    assert np.array_equal(outs[0]["y"], outs[1]["y"])
    assert np.array_equal(outs[0]["photons"], outs[1]["photons"])
    assert outs[0]["tallies"] == outs[1]["tallies"]


def test_reset_restores_the_given_bins(sxctx):
    w = G.small_random(900, seed=42, n_bins=21, box=3e21, rate=1e48, n_src=2, dt=3e13)
    gid = sxctx.upload(w)
    try:
        sxctx.solve([gid], 15)
        ref = sxctx.state(gid, photons=True)
        t0 = sxctx.tables(gid)
        sxctx.rotate(gid, G.random_rotations(1, seed=3)[0])
        sxctx.solve([gid], 4)
        sxctx.reset(gid)
        assert np.array_equal(sxctx.tables(gid)["sel_m"], t0["sel_m"])
        sxctx.solve([gid], 15)
        again = sxctx.state(gid, photons=True)
        assert np.array_equal(ref["y"], again["y"])
        assert np.array_equal(ref["photons"], again["photons"])
    finally:
        sxctx.free(gid)


def test_rotation_errors(sxctx):
    w = G.small_random(200, seed=43, n_bins=21)
    gid = sxctx.upload(w)
    try:
        for bad in (np.diag([1.0, 1.0, -1.0]), 2 * np.eye(3), np.full((3, 3), np.nan)):
            with pytest.raises(sx.SxError) as e:
                sxctx.rotate(gid, bad)
            assert e.value.code == sx.SX_EINVAL
    finally:
        sxctx.free(gid)
