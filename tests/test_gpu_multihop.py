"""Multi-hop steps on the GPU against the oracle (Sect. 4.6: photons cross up
to H edges per step, the neutral fraction is updated once per step): whole
solves in both precisions, the chain, Test 1 at a 25 Myr step, checkpoint
restore at a step boundary, batches mixing hop counts, and the limits."""
import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx
from oracle import Oracle
from parity import assert_state_close

pytestmark = pytest.mark.gpu


def _conserved(t, tol):
    r = t["emitted"] - (t["absorbed"] + t["escaped"] + t["in_flight"])
    assert abs(r) <= tol * t["emitted"], r / t["emitted"]


def _solve(ctx, w, sweeps):
    gid = ctx.upload(w)
    try:
        ctx.solve([gid], sweeps)
        st = ctx.state(gid, photons=True)
        unit = ctx.info(gid)["photon_unit"]
    finally:
        ctx.free(gid)
    return st, unit


def _oracle(w, sweeps):
    o = Oracle(w)
    o.run(sweeps)
    ref = o.state()
    o.close()
    return ref


@pytest.mark.parametrize("H", [2, 5])
@pytest.mark.parametrize("prec", [G.SX_FP64, G.SX_FP32_TRANSPORT])
def test_multihop_solve(sxctx, prec, H):
    """Random grid with isotropic and beam sources, 6 steps of H hops."""
    w = G.small_random(900, seed=91, n_bins=42, box=3e21, rate=1e48, n_src=3,
                       dt=1.2e14, precision=prec)
    sd = np.zeros((3, 3))
    sd[2] = [1.0, 0.0, 0.0]
    w = G.with_(w, src_dir=sd, hops=H)
    print(f"[case] multi-hop solve prec={prec} H={H}", flush=True)
    st, unit = _solve(sxctx, w, 6 * H)
    ref = _oracle(w, 6 * H)
    assert_state_close(st, ref, prec, unit, f"multi-hop H={H}")
    _conserved(st["tallies"], 1e-9 if prec == G.SX_FP64 else 1e-4)
    assert st["tallies"]["sweeps"] == 6 * H


def test_multihop_mid_step(sxctx):
    """Read back in the middle of a step: the photons in flight and the
    tallies after each hop, y still that of the step's start."""
    H = 4
    w = G.with_(G.small_random(600, seed=92, n_bins=21, box=3e21, rate=1e48, n_src=2,
                               dt=1.2e14), hops=H)
    print("[case] multi-hop mid-step", flush=True)
    gid = sxctx.upload(w)
    o = Oracle(w)
    try:
        for n in (3, 2, 4, 1):
            sxctx.solve([gid], n)
            o.run(n)
            st = sxctx.state(gid, photons=True)
            unit = sxctx.info(gid)["photon_unit"]
            ref = o.state()
            ref["nin"] = st["nin"] = None
            assert_state_close(st, ref, G.SX_FP64, unit, f"after {n} more hops")
    finally:
        sxctx.free(gid)
        o.close()


def test_multihop_chain(sxctx):
    """The oracle's chain case: photons of every hop reach up to H edges."""
    n, sp, H = 14, 3e21, 3
    rng = np.random.default_rng(2)
    nH = 10 ** rng.uniform(-4, -2.5, n)
    w = G.chain_graph(n, sp, 1e-3, sp ** 3)
    w = G.with_(w, n_H=nH, src_rate=np.array([1e30]), dt=1e10, hops=H)
    print("[case] multi-hop chain", flush=True)
    st, unit = _solve(sxctx, w, 5 * H)
    ref = _oracle(w, 5 * H)
    assert_state_close(st, ref, G.SX_FP64, unit, "chain")


def test_multihop_front_law_solve(sxctx):
    """Test 1 with a 25 Myr step and 10 hops per step, whole solve in fp32
    transport, against the oracle."""
    base = G.config1()
    w = G.with_(base, dt=25.0 * G.MYR_S, n_sweeps=200, hops=10,
                precision=G.SX_FP32_TRANSPORT)
    print("[case] multi-hop Test 1, 20 steps of 10 hops", flush=True)
    st, unit = _solve(sxctx, w, 200)
    ref = _oracle(w, 200)
    assert_state_close(st, ref, G.SX_FP32_TRANSPORT, unit, "Test 1 multi-hop")


def test_multihop_restore_at_step_boundary(sxctx):
    """A checkpoint taken between steps restores into a fresh grid and the
    two runs continue bit for bit; a restore in the middle of a step is
    refused."""
    H = 3
    w = G.with_(G.small_random(500, seed=93, n_bins=42, box=3e21, rate=1e48, n_src=2,
                               dt=1.2e14), hops=H)
    print("[case] multi-hop restore", flush=True)
    a = sxctx.upload(w)
    b = sxctx.upload(w)
    try:
        sxctx.solve([a], 2 * H)
        ck = sxctx.state(a, photons=True)
        sxctx.restore(b, y=ck["y"], photons=ck["photons"], tallies=ck["tallies"])
        sxctx.solve([a], 2 * H)
        sxctx.solve([b], 2 * H)
        sa = sxctx.state(a, photons=True)
        sb = sxctx.state(b, photons=True)
        sxctx.solve([a], 1)
        with pytest.raises(sx.SxError) as e:
            sxctx.restore(a, y=ck["y"])
        assert e.value.code == sx.SX_EINVAL
    finally:
        sxctx.free(a)
        sxctx.free(b)
    assert np.array_equal(sa["y"], sb["y"])
    assert np.array_equal(sa["photons"], sb["photons"])
    for k in ("sweeps", "emitted", "absorbed", "escaped", "in_flight"):
        assert abs(sa["tallies"][k] - sb["tallies"][k]) <= 1e-12 * abs(sa["tallies"][k]), k


def test_multihop_in_a_batch(sxctx):
    """A multi-hop grid and a one-hop grid in one launch: each bit for bit
    as alone."""
    w1 = G.with_(G.small_random(700, seed=94, n_bins=42, box=3e21, rate=1e48, n_src=2,
                                dt=1.2e14), hops=4)
    w2 = G.small_random(900, seed=95, n_bins=42, box=3e21, rate=1e48, n_src=2, dt=3e13)
    print("[case] multi-hop in a batch", flush=True)
    alone = [_solve(sxctx, w, 24)[0] for w in (w1, w2)]
    ids = [sxctx.upload(w) for w in (w1, w2)]
    try:
        sxctx.solve(ids, [24, 24])
        both = [sxctx.state(g, photons=True) for g in ids]
    finally:
        for g in ids:
            sxctx.free(g)
    for a, b in zip(alone, both):
        assert np.array_equal(a["y"], b["y"])
        assert np.array_equal(a["photons"], b["photons"])


def test_multihop_limits(sxctx):
    w = G.small_random(300, seed=96, n_bins=21, box=3e21, rate=1e48)
    for bad, code in ((G.with_(w, hops=2, transport=G.SX_TRANSPORT_COMBINED), sx.SX_ENOTSUP),
                      (G.with_(w, hops=2, alpha_A=G.ALPHA_A), sx.SX_ENOTSUP),
                      (G.with_(w, hops=sx.SX_MAX_HOPS + 1), sx.SX_EINVAL),
                      (G.with_(w, hops=-1), sx.SX_EINVAL)):
        with pytest.raises(sx.SxError) as e:
            sxctx.upload(bad)
        assert e.value.code == code
