"""sx_step_noalloc against sx_step: the same kernels from tables kept in a
static device array, so the results must be bit for bit those of sx_step,
call after call, also when a later call lists a smaller set of grids."""
import numpy as np
import pytest

from paper_0912_4273_amd import gridgen as G
from paper_0912_4273_amd import sx

pytestmark = pytest.mark.gpu


def _grids():
    kw = dict(box=3e21, rate=1e48, dt=3e13)
    return [
        G.small_random(3000, seed=91, n_bins=42, n_src=2, precision=G.SX_FP32_TRANSPORT, **kw),
        G.small_random(1500, seed=92, n_bins=21, n_src=1, precision=G.SX_FP64, **kw),
        G.with_(G.small_random(2000, seed=93, n_bins=42, n_src=3,
                               precision=G.SX_FP32_TRANSPORT, **kw),
                transport=G.SX_TRANSPORT_COMBINED, tau_switch=1.0),
    ]


def _same(ctx, ga, gb, w, what):
    sa, sb = ctx.state(ga, photons=True), ctx.state(gb, photons=True)
    for key in ("x", "y", "photons", "nin"):
        assert np.array_equal(sa[key], sb[key]), f"{what}: {key} differs"
    assert sa["tallies"] == sb["tallies"], f"{what}: tallies differ"
    if w.transport == G.SX_TRANSPORT_COMBINED:
        ea, eb = ctx.edge_state(ga), ctx.edge_state(gb)
        assert np.array_equal(ea["photons_e"], eb["photons_e"]), f"{what}: edge photons"
        assert np.array_equal(ea["layout"], eb["layout"]), f"{what}: layouts"


def _free_device_bytes():
    """Free device memory as the HIP runtime that libsx runs on reports it."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def test_noalloc_step_equals_step():
    ws = _grids()
    print("[case] no-alloc step: 3 grids x 7 sweeps, then 1 grid x 5 sweeps", flush=True)
    with sx.Context(0) as ctx:
        a = [ctx.upload(w) for w in ws]
        b = [ctx.upload(w) for w in ws]
        ctx.step(a, 7)
        ctx.step_noalloc(b, 7)
        ctx.sync()
        for i, w in enumerate(ws):
            _same(ctx, a[i], b[i], w, f"call 1 grid {i}")
        assert ctx.state(b[0])["tallies"]["sweeps"] == 7
        # a second call with a smaller input: one grid, fewer tiles
        ctx.step(a[1:2], 5)
        ctx.step_noalloc(b[1:2], 5)
        ctx.sync()
        for i, w in enumerate(ws):
            _same(ctx, a[i], b[i], w, f"call 2 grid {i}")
        assert ctx.state(b[1])["tallies"]["sweeps"] == 12
        # no device memory is taken by further calls
        free0 = _free_device_bytes()
        for _ in range(5):
            ctx.step_noalloc(b, 2)
        ctx.sync()
        assert _free_device_bytes() == free0
        # beyond the grid limit: an error, nothing launched
        with pytest.raises(sx.SxError) as e:
            ctx.step_noalloc([b[0]] * (sx.SX_NOALLOC_MAX_GRIDS + 1), 1)
        assert e.value.code == sx.SX_EINVAL
        assert ctx.state(b[0])["tallies"]["sweeps"] == 17
