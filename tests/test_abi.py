"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/sx.h declares, the ctypes structs match the C
layout, and the oracle and the library stay separate."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_0912_4273_amd import sx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sx.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(sx_\w+)\s*\(", txt, re.M)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("sx_grid_upload", "sx_step", "sx_solve", "sx_read_state"):
        assert must in names
    assert set(names) == set(sx.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = sx.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", sx.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sx_\w+)", out))
    assert set(declared_functions()) <= exported


def test_binding_constants_match_header():
    txt = open(HEADER).read()
    defs = dict(re.findall(r"^#define (SX_\w+)\s+\(?(-?\d+)\)?", txt, re.M))
    for name in ("SX_OK", "SX_EINVAL", "SX_ENOMEM", "SX_EDEVICE", "SX_ENOTFOUND",
                 "SX_ENOTSUP", "SX_EAGAIN", "SX_FP64", "SX_FP32_TRANSPORT",
                 "SX_ORDER_GRID", "SX_ORDER_DIRECT_FIRST", "SX_MAX_GRAPH_SWEEPS",
                 "SX_MAX_DEGREE", "SX_TRANSPORT_DCT", "SX_TRANSPORT_COMBINED",
                 "SX_DCT_REF_BIN", "SX_DCT_REF_EDGE", "SX_MAX_HOPS"):
        assert int(defs[name]) == getattr(sx, name), name
    assert sx.SX_MAX_BINS == int(defs["SX_MAX_BINS_FP32"]) == int(defs["SX_MAX_BINS_FP64"])


def test_error_strings():
    lib = sx.load()
    assert lib.sx_strerror(sx.SX_EINVAL) == b"invalid argument"
    assert lib.sx_strerror(sx.SX_ENOMEM).startswith(b"out of device memory")
    assert lib.sx_last_error(None) == b"null context"


def test_null_arguments_rejected_without_device():
    lib = sx.load()
    assert lib.sx_init(None, None) == sx.SX_EINVAL
    assert lib.sx_step(None, None, 0, 1) == sx.SX_EINVAL
    assert lib.sx_autotune(None, 1) == sx.SX_EINVAL
    assert lib.sx_serve_start(None, None, None) == sx.SX_EINVAL
    assert lib.sx_serve_stop(None, None) == sx.SX_OK
    assert lib.sx_prepared_free(None) == sx.SX_OK
    assert lib.sx_grid_commit(None, None, None) == sx.SX_EINVAL
    assert lib.sx_set_schedule(None, None, 0, None) == sx.SX_EINVAL
    assert lib.sx_get_schedule(None, None, 0, None, None) == sx.SX_EINVAL
    assert lib.sx_finalize(None) == sx.SX_OK
    assert lib.sx_read_edge_state(None, 1, None, None) == sx.SX_EINVAL
    assert lib.sx_grid_restore_edges(None, 1, None, None) == sx.SX_EINVAL
    assert lib.sx_read_ballistic(None, 1, None, None) == sx.SX_EINVAL
    assert lib.sx_read_diffuse(None, 1, None) == sx.SX_EINVAL
    b = C.c_uint64()
    assert lib.sx_grid_bytes(None, C.byref(b)) == sx.SX_EINVAL


def _c_layout():
    """offsetof/sizeof of the ABI structs as the C compiler sees them."""
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "sx.h"
#define P(s, f) printf(#s "." #f " %zu\n", offsetof(s, f));
int main(void) {
  printf("sx_grid_desc %zu\n", sizeof(sx_grid_desc));
  printf("sx_ctx_opts %zu\n", sizeof(sx_ctx_opts));
  printf("sx_state_out %zu\n", sizeof(sx_state_out));
  printf("sx_tally %zu\n", sizeof(sx_tally));
  printf("sx_schedule %zu\n", sizeof(sx_schedule));
  P(sx_schedule, order) P(sx_schedule, graph_sweeps) P(sx_schedule, work_split)
  printf("sx_serve_opts %zu\n", sizeof(sx_serve_opts));
  printf("sx_serve_result %zu\n", sizeof(sx_serve_result));
  printf("sx_serve_stats %zu\n", sizeof(sx_serve_stats));
  P(sx_serve_opts, hbm_budget) P(sx_serve_result, n_vertices) P(sx_serve_result, t_submit)
  P(sx_serve_result, tally) P(sx_serve_stats, updates) P(sx_serve_stats, latency_max_s)
  P(sx_grid_desc, kappa) P(sx_grid_desc, n_bins) P(sx_grid_desc, cos_min)
  P(sx_grid_desc, src_dir) P(sx_grid_desc, dt) P(sx_grid_desc, precision)
  P(sx_grid_desc, transport) P(sx_grid_desc, dct_reference) P(sx_grid_desc, tau_switch)
  P(sx_grid_desc, alpha_A)
  P(sx_ctx_opts, stream) P(sx_ctx_opts, alloc_user)
  return 0;
}
"""
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    return dict(line.rsplit(" ", 1) for line in out.strip().splitlines())


def test_ctypes_struct_layout_matches_c():
    lay = {k: int(v) for k, v in _c_layout().items()}
    assert C.sizeof(sx.SxGridDesc) == lay["sx_grid_desc"]
    assert C.sizeof(sx.SxCtxOpts) == lay["sx_ctx_opts"]
    assert C.sizeof(sx.SxStateOut) == lay["sx_state_out"]
    assert C.sizeof(sx.SxTally) == lay["sx_tally"]
    assert C.sizeof(sx.SxSchedule) == lay["sx_schedule"]
    for f in ("order", "graph_sweeps", "work_split"):
        assert getattr(sx.SxSchedule, f).offset == lay[f"sx_schedule.{f}"], f
    for name, cls, fields in (
            ("sx_serve_opts", sx.SxServeOpts, ("hbm_budget",)),
            ("sx_serve_result", sx.SxServeResult, ("n_vertices", "t_submit", "tally")),
            ("sx_serve_stats", sx.SxServeStats, ("updates", "latency_max_s"))):
        assert C.sizeof(cls) == lay[name], name
        for f in fields:
            assert getattr(cls, f).offset == lay[f"{name}.{f}"], (name, f)
    for f in ("kappa", "n_bins", "cos_min", "src_dir", "dt", "precision", "transport",
              "dct_reference", "tau_switch", "alpha_A"):
        assert getattr(sx.SxGridDesc, f).offset == lay[f"sx_grid_desc.{f}"], f
    for f in ("stream", "alloc_user"):
        assert getattr(sx.SxCtxOpts, f).offset == lay[f"sx_ctx_opts.{f}"], f


def test_oracle_and_library_share_no_code():
    """The oracle is independent of the HIP path: neither includes or
    imports the other."""
    csrc = os.path.join(ROOT, "paper_0912_4273_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "oracle" not in txt.lower(), f
    for f in ("sx_oracle.c", "sx_oracle.h", "oracle.py"):
        txt = open(os.path.join(ROOT, "oracle", f)).read()
        assert "sx.h" not in txt and "sx_internal" not in txt
        assert "paper_0912_4273_amd" not in txt
    for f in os.listdir(os.path.join(ROOT, "paper_0912_4273_amd")):
        if f.endswith(".py"):
            txt = open(os.path.join(ROOT, "paper_0912_4273_amd", f)).read()
            assert "import oracle" not in txt and "from oracle" not in txt, f


def test_product_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError, match="libsx.so not found"):
        sx.load(str(tmp_path / "libsx.so"))


def test_gridgen_has_no_method_arithmetic():
    """The shared input generator holds no transport or chemistry step."""
    txt = open(os.path.join(ROOT, "paper_0912_4273_amd", "gridgen.py")).read()
    for word in ("expm1", "exp(-", "argmax", "most_straightforward"):
        assert word not in txt


def test_prepare_is_host_only():
    """sx_grid_prepare (the host half of an upload) needs no device: it
    accepts a valid grid, rejects a malformed one with a message, and its
    handle reports a positive byte estimate."""
    from paper_0912_4273_amd import gridgen as G
    w = G.small_random(300, seed=5, n_bins=21)
    h = sx.sx_grid_prepare(w)
    try:
        assert sx.sx_prepared_bytes(h) > 0
    finally:
        sx.sx_prepared_free(h)
    bad = G.with_(w, nbr_idx=np.where(w.nbr_idx == 0, 1, w.nbr_idx).astype(np.int32))
    with pytest.raises(sx.SxError) as e:
        sx.sx_grid_prepare(bad)
    assert e.value.code == sx.SX_EINVAL


def test_prepare_combined_transport_host_only():
    """Combined transport is prepared on the host: a valid request gets a
    larger byte estimate (per-edge state and lists); an unknown mode or a NaN
    switch is rejected."""
    from paper_0912_4273_amd import gridgen as G
    w = G.small_random(300, seed=6, n_bins=21)
    sizes = []
    for ww in (w, G.with_(w, transport=G.SX_TRANSPORT_COMBINED, tau_switch=1.0)):
        h = sx.sx_grid_prepare(ww)
        try:
            sizes.append(sx.sx_prepared_bytes(h))
        finally:
            sx.sx_prepared_free(h)
    assert sizes[1] > sizes[0]
    for bad in (G.with_(w, transport=2),
                G.with_(w, transport=G.SX_TRANSPORT_COMBINED, tau_switch=float("nan"))):
        with pytest.raises(sx.SxError) as e:
            sx.sx_grid_prepare(bad)
        assert e.value.code == sx.SX_EINVAL
