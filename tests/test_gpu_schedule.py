"""Launch schedules, graph replays and the autotuner change only the order in
which independent tiles run: every result is bitwise the one of plain
single launches."""
import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx

pytestmark = pytest.mark.gpu

PLAIN = dict(tiles_per_group=4, order=sx.SX_ORDER_GRID, xcd_contiguous=1, graph_sweeps=0)
# (tiles per workgroup, waves per tile)
SHAPES = [(4, 1), (2, 1), (1, 1), (2, 2), (1, 2), (1, 4)]


def _mixed_batch():
    """Uneven grids, both precisions, one grid with every tile on the
    direct-gather path."""
    ws = [G.small_random(700, seed=71, n_bins=42, box=3e21, rate=1e48, n_src=2,
                         dt=3e13, precision=G.SX_FP32_TRANSPORT),
          G.small_random(2100, seed=72, n_bins=42, box=3e21, rate=1e48, n_src=1,
                         dt=3e13, precision=G.SX_FP32_TRANSPORT),
          G.small_random(1300, seed=73, n_bins=21, box=3e21, rate=1e48, n_src=3,
                         dt=3e13, precision=G.SX_FP64)]
    return ws


def _upload(ctx, ws, monkeypatch, direct_index=1):
    ids = []
    for i, w in enumerate(ws):
        if i == direct_index:
            monkeypatch.setenv("SX_FORCE_DIRECT", "1")
        ids.append(ctx.upload(w))
        monkeypatch.delenv("SX_FORCE_DIRECT", raising=False)
    return ids


def _states(ctx, ids):
    return [ctx.state(g, photons=True) for g in ids]


def _same(a, b, what):
    for i, (sa, sb) in enumerate(zip(a, b)):
        assert np.array_equal(sa["y"], sb["y"]), f"{what}: grid {i} y"
        assert np.array_equal(sa["photons"], sb["photons"]), f"{what}: grid {i} photons"
        assert sa["tallies"] == sb["tallies"], f"{what}: grid {i} tallies"


def test_every_schedule_gives_the_same_bits(monkeypatch):
    ws = _mixed_batch()
    sweeps = [23, 31, 17]
    with sx.Context(0) as ctx:
        ids = _upload(ctx, ws, monkeypatch)
        ctx.set_schedule(ids, **PLAIN)
        ctx.solve(ids, sweeps)
        ref = _states(ctx, ids)
        for tpb, split in SHAPES:
            for order in (sx.SX_ORDER_GRID, sx.SX_ORDER_DIRECT_FIRST):
                for xcd in (0, 1):
                    for gsw in (0, 7):
                        what = f"tpb={tpb} split={split} order={order} xcd={xcd} graph={gsw}"
                        print("[case]", what, flush=True)
                        for g in ids:
                            ctx.reset(g)
                        ctx.set_schedule(ids, tiles_per_group=tpb, order=order,
                                         xcd_contiguous=xcd, graph_sweeps=gsw,
                                         work_split=split)
                        ctx.solve(ids, sweeps)
                        _same(ref, _states(ctx, ids), what)


def test_work_split_with_fewer_blocks_than_waves():
    """Grids with fewer bin blocks than waves per tile (1, 2 and 3 bins, 5
    in FP64): the waves past the last block hand over zeros."""
    ws = [G.small_random(500, seed=75 + k, n_bins=k, box=3e21, rate=1e48, n_src=2, dt=3e13,
                         precision=G.SX_FP32_TRANSPORT if k < 5 else G.SX_FP64)
          for k in (1, 2, 3, 5)]
    with sx.Context(0) as ctx:
        ids = [ctx.upload(w) for w in ws]
        ctx.set_schedule(ids, **PLAIN)
        ctx.solve(ids, 25)
        ref = _states(ctx, ids)
        for tpb, split in SHAPES[1:]:
            print(f"[case] few bins tpb={tpb} split={split}", flush=True)
            for g in ids:
                ctx.reset(g)
            ctx.set_schedule(ids, tiles_per_group=tpb, order=sx.SX_ORDER_GRID,
                             xcd_contiguous=1, graph_sweeps=0, work_split=split)
            ctx.solve(ids, 25)
            _same(ref, _states(ctx, ids), f"few bins tpb={tpb} split={split}")


def test_invalid_work_split_is_refused():
    with sx.Context(0) as ctx:
        for tpb, split in ((4, 2), (2, 4), (1, 3), (1, 8), (1, -1)):
            with pytest.raises(sx.SxError):
                ctx.set_schedule([], tiles_per_group=tpb, order=sx.SX_ORDER_GRID,
                                 xcd_contiguous=1, graph_sweeps=0, work_split=split)


def test_single_grid_schedules(monkeypatch):
    w = G.with_(G.config1(), precision=G.SX_FP32_TRANSPORT)
    with sx.Context(0) as ctx:
        gid = ctx.upload(w)
        ctx.set_schedule([gid], **PLAIN)
        ctx.solve([gid], 40)
        ref = _states(ctx, [gid])
        for tpb, split in ((1, 1), (2, 1), (2, 2), (1, 4)):
            for gsw in (0, 3, 40):
                print(f"[case] single tpb={tpb} split={split} graph={gsw}", flush=True)
                ctx.reset(gid)
                ctx.set_schedule([gid], tiles_per_group=tpb, order=sx.SX_ORDER_DIRECT_FIRST,
                                 xcd_contiguous=0, graph_sweeps=gsw, work_split=split)
                ctx.solve([gid], 40)
                _same(ref, _states(ctx, [gid]), f"tpb={tpb} split={split} graph={gsw}")


def test_graph_replays_with_eager_work_between(monkeypatch):
    """A graph replayed many times, with state reads (host syncs and
    copies) and single launches between the replays, matches every
    intermediate state of plain launches."""
    ws = _mixed_batch()[:2]
    with sx.Context(0) as ctx:
        ids = _upload(ctx, ws, monkeypatch, direct_index=-1)
        ctx.set_schedule(ids, **PLAIN)
        ref = []
        for _ in range(5):
            ctx.step(ids, 9)
            ref.append(_states(ctx, ids))
        for g in ids:
            ctx.reset(g)
        ctx.set_schedule(ids, tiles_per_group=4, order=sx.SX_ORDER_GRID,
                         xcd_contiguous=1, graph_sweeps=4)
        for r in range(5):
            print(f"[case] replay round {r}", flush=True)
            ctx.step(ids, 9)     # two replays and one single launch
            _same(ref[r], _states(ctx, ids), f"round {r}")


def test_autotune_keeps_results_and_reports(monkeypatch):
    ws = _mixed_batch()
    sweeps = [120, 150, 90]
    with sx.Context(0) as ctx:
        ids = _upload(ctx, ws, monkeypatch)
        ctx.set_schedule(ids, **PLAIN)
        ctx.solve(ids, sweeps)
        ref = _states(ctx, ids)
        for g in ids:
            ctx.free(g)
        ids = _upload(ctx, ws, monkeypatch)
        ctx.autotune(2)
        ctx.solve(ids, sweeps)
        got = _states(ctx, ids)
        s = ctx.get_schedule(ids)
        print("[case] tuned", s, flush=True)
        assert s["tiles_per_group"] in (1, 2, 4)
        assert s["us_per_sweep"] > 0
        assert s["graph_sweeps"] == 50
        _same(ref, got, "autotuned")


def test_schedule_errors():
    with sx.Context(0) as ctx:
        with pytest.raises(sx.SxError) as e:
            ctx.set_schedule([], tiles_per_group=3)
        assert e.value.code == sx.SX_EINVAL
        with pytest.raises(sx.SxError) as e:
            ctx.set_schedule([], graph_sweeps=sx.SX_MAX_GRAPH_SWEEPS + 1)
        assert e.value.code == sx.SX_EINVAL
        with pytest.raises(sx.SxError) as e:
            ctx.set_schedule([12345])
        assert e.value.code == sx.SX_ENOTFOUND
        with pytest.raises(sx.SxError) as e:
            ctx.autotune(-1)
        assert e.value.code == sx.SX_EINVAL
        d = ctx.get_schedule([])
        assert d["tiles_per_group"] == 4 and d["graph_sweeps"] == 50
