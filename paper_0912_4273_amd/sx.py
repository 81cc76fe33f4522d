"""Python binding of libsx (include/sx.h): argument marshalling only.

Every function below has the name of the C entry point it calls.  All
transport and chemistry run inside libsx's HIP kernels; this module only
packs host arrays into the C structs and unpacks results.  PyTorch is used
(optionally) for the HIP stream and as the device-memory allocator.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsx.so")

SX_OK = 0
SX_EINVAL = -1
SX_ENOMEM = -2
SX_EDEVICE = -3
SX_ENOTFOUND = -4
SX_ENOTSUP = -5
SX_EAGAIN = -6
SX_FP64 = 0
SX_FP32_TRANSPORT = 1
SX_ORDER_GRID = 0
SX_ORDER_DIRECT_FIRST = 1
SX_MAX_GRAPH_SWEEPS = 4096
SX_NOALLOC_MAX_GRIDS = 256
SX_NOALLOC_MAX_TILES = 131072
SX_MAX_BINS = 96
SX_MAX_DEGREE = 127
SX_MAX_HOPS = 1024
SX_TRANSPORT_DCT = 0
SX_TRANSPORT_COMBINED = 1
SX_DCT_REF_BIN = 0
SX_DCT_REF_EDGE = 1

EXPORTED = [
    "sx_init", "sx_finalize", "sx_grid_bytes", "sx_grid_upload",
    "sx_grid_reset", "sx_grid_restore", "sx_grid_free", "sx_step", "sx_step_noalloc",
    "sx_solve", "sx_sync", "sx_read_state", "sx_read_tables",
    "sx_grid_info", "sx_mem_info", "sx_stream", "sx_profile",
    "sx_profile_read", "sx_set_schedule", "sx_get_schedule", "sx_autotune",
    "sx_rotate_bins", "sx_read_edge_state", "sx_grid_restore_edges", "sx_read_ballistic",
    "sx_read_diffuse", "sx_grid_select_removal", "sx_grid_remap",
    "sx_grid_prepare", "sx_prepared_bytes", "sx_grid_commit", "sx_prepared_free",
    "sx_serve_start", "sx_serve_submit", "sx_serve_poll", "sx_serve_take",
    "sx_serve_stop", "sx_strerror", "sx_last_error",
]

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class SxCtxOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("reserved0", C.c_int32),
                ("hbm_budget", C.c_uint64), ("stream", C.c_void_p),
                ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_user", C.c_void_p)]


class SxGridDesc(C.Structure):
    _fields_ = [
        ("n_vertices", C.c_int64), ("pos", C.c_void_p),
        ("nbr_ptr", C.c_void_p), ("nbr_idx", C.c_void_p),
        ("n_H", C.c_void_p), ("volume", C.c_void_p), ("dL", C.c_void_p),
        ("kappa", C.c_double), ("x_init", C.c_void_p),
        ("n_bins", C.c_int32), ("max_per_bin", C.c_int32),
        ("bin_dirs", C.c_void_p), ("cos_min", C.c_double),
        ("n_src", C.c_int32), ("n_subcycles", C.c_int32),
        ("src_vertex", C.c_void_p), ("src_rate", C.c_void_p),
        ("src_dir", C.c_void_p), ("sigma", C.c_double),
        ("alpha_B", C.c_double), ("dt", C.c_double),
        ("precision", C.c_int32), ("transport", C.c_int32),
        ("dct_reference", C.c_int32), ("tau_switch", C.c_double),
        ("alpha_A", C.c_double), ("hops", C.c_int32)]


class SxTally(C.Structure):
    _fields_ = [("sweeps", C.c_double), ("emitted", C.c_double),
                ("absorbed", C.c_double), ("escaped", C.c_double),
                ("in_flight", C.c_double)]


class SxStateOut(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p),
                ("photons", C.c_void_p), ("nin", C.c_void_p),
                ("tally", C.POINTER(SxTally))]


class SxStateIn(C.Structure):
    _fields_ = [("y", C.c_void_p), ("photons", C.c_void_p),
                ("tally", C.POINTER(SxTally))]


class SxSchedule(C.Structure):
    _fields_ = [("tiles_per_group", C.c_int32), ("order", C.c_int32),
                ("xcd_contiguous", C.c_int32), ("graph_sweeps", C.c_int32),
                ("work_split", C.c_int32)]


class SxServeOpts(C.Structure):
    _fields_ = [("round_sweeps", C.c_int32), ("max_active", C.c_int32),
                ("prep_threads", C.c_int32), ("reserved", C.c_int32),
                ("hbm_budget", C.c_uint64)]


class SxServeResult(C.Structure):
    _fields_ = [("ticket", C.c_int64), ("status", C.c_int32), ("n_bins", C.c_int32),
                ("n_vertices", C.c_int64), ("n_sweeps", C.c_int32), ("reserved", C.c_int32),
                ("t_submit", C.c_double), ("t_prepared", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("tally", SxTally)]


class SxServeStats(C.Structure):
    _fields_ = [("finished", C.c_int64), ("failed", C.c_int64), ("rounds", C.c_int64),
                ("peak_active", C.c_int32), ("reserved", C.c_int32),
                ("updates", C.c_double), ("span_s", C.c_double), ("round_s", C.c_double),
                ("latency_p50_s", C.c_double), ("latency_p99_s", C.c_double),
                ("latency_max_s", C.c_double)]


class SxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load(path: Optional[str] = None):
    """Load libsx.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"libsx.so not found at {p}; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(p)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "sx_init": (C.c_int, [C.POINTER(P), C.POINTER(SxCtxOpts)]),
        "sx_finalize": (C.c_int, [P]),
        "sx_grid_bytes": (C.c_int, [C.POINTER(SxGridDesc), C.POINTER(C.c_uint64)]),
        "sx_grid_upload": (C.c_int, [P, C.POINTER(SxGridDesc), C.POINTER(I64)]),
        "sx_grid_reset": (C.c_int, [P, I64]),
        "sx_grid_restore": (C.c_int, [P, I64, C.POINTER(SxStateIn)]),
        "sx_grid_free": (C.c_int, [P, I64]),
        "sx_step": (C.c_int, [P, P, I32, I32]),
        "sx_step_noalloc": (C.c_int, [P, P, I32, I32]),
        "sx_solve": (C.c_int, [P, P, I32, P]),
        "sx_sync": (C.c_int, [P]),
        "sx_read_state": (C.c_int, [P, I64, C.POINTER(SxStateOut)]),
        "sx_read_tables": (C.c_int, [P, I64, P, P, P, P, P]),
        "sx_grid_info": (C.c_int, [P, I64, P, P, P, P, P, P]),
        "sx_mem_info": (C.c_int, [P, P, P]),
        "sx_stream": (P, [P]),
        "sx_profile": (C.c_int, [P, I32]),
        "sx_profile_read": (C.c_int, [P, P, P, P, P]),
        "sx_set_schedule": (C.c_int, [P, P, I32, C.POINTER(SxSchedule)]),
        "sx_get_schedule": (C.c_int, [P, P, I32, C.POINTER(SxSchedule), P]),
        "sx_autotune": (C.c_int, [P, I32]),
        "sx_rotate_bins": (C.c_int, [P, I64, P]),
        "sx_read_edge_state": (C.c_int, [P, I64, P, P]),
        "sx_grid_restore_edges": (C.c_int, [P, I64, P, P]),
        "sx_read_ballistic": (C.c_int, [P, I64, P, P]),
        "sx_read_diffuse": (C.c_int, [P, I64, P]),
        "sx_grid_select_removal": (C.c_int, [P, I64, C.c_double, C.c_double, P, P]),
        "sx_grid_remap": (C.c_int, [P, I64, I64, P]),
        "sx_grid_prepare": (C.c_int, [C.POINTER(SxGridDesc), C.POINTER(P), C.c_char_p,
                                      C.c_size_t]),
        "sx_prepared_bytes": (C.c_int, [P, C.POINTER(C.c_uint64)]),
        "sx_grid_commit": (C.c_int, [P, P, C.POINTER(I64)]),
        "sx_prepared_free": (C.c_int, [P]),
        "sx_serve_start": (C.c_int, [P, C.POINTER(SxServeOpts), C.POINTER(P)]),
        "sx_serve_submit": (C.c_int, [P, C.POINTER(SxGridDesc), I32, C.POINTER(I64)]),
        "sx_serve_poll": (C.c_int, [P, C.c_double, C.POINTER(SxServeResult)]),
        "sx_serve_take": (C.c_int, [P, I64, P, P]),
        "sx_serve_stop": (C.c_int, [P, C.POINTER(SxServeStats)]),
        "sx_strerror": (C.c_char_p, [C.c_int]),
        "sx_last_error": (C.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(ctx, rc):
    if rc != SX_OK:
        lib = load()
        msg = lib.sx_last_error(ctx).decode() if ctx else lib.sx_strerror(rc).decode()
        raise SxError(rc, msg or lib.sx_strerror(rc).decode())


# ------------------------------------------------------------- desc ----

class _Desc:
    """An SxGridDesc plus the numpy arrays its pointers refer to."""

    def __init__(self, w):
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
        self.arrays = dict(
            pos=f64(w.pos), ptr=np.ascontiguousarray(w.nbr_ptr, np.int64),
            idx=np.ascontiguousarray(w.nbr_idx, np.int32), nH=f64(w.n_H),
            vol=f64(w.volume), dL=f64(w.dL), x0=f64(w.x_init),
            bins=f64(w.bin_dirs), sv=np.ascontiguousarray(w.src_vertex, np.int32),
            sr=f64(w.src_rate), sd=f64(w.src_dir))
        a = self.arrays
        self.c = SxGridDesc(
            n_vertices=w.n, pos=_ptr(a["pos"]), nbr_ptr=_ptr(a["ptr"]),
            nbr_idx=_ptr(a["idx"]), n_H=_ptr(a["nH"]), volume=_ptr(a["vol"]),
            dL=_ptr(a["dL"]), kappa=float(w.kappa), x_init=_ptr(a["x0"]),
            n_bins=w.k, max_per_bin=int(w.max_per_bin), bin_dirs=_ptr(a["bins"]),
            cos_min=float(w.cos_min), n_src=int(a["sv"].shape[0]),
            n_subcycles=int(w.n_subcycles), src_vertex=_ptr(a["sv"]),
            src_rate=_ptr(a["sr"]), src_dir=_ptr(a["sd"]), sigma=float(w.sigma),
            alpha_B=float(w.alpha_B), dt=float(w.dt), precision=int(w.precision),
            transport=int(getattr(w, "transport", SX_TRANSPORT_DCT)),
            dct_reference=int(getattr(w, "dct_reference", SX_DCT_REF_BIN)),
            tau_switch=float(getattr(w, "tau_switch", 1.0)),
            alpha_A=float(getattr(w, "alpha_A", 0.0)),
            hops=int(getattr(w, "hops", 1)))


# ------------------------------------------------------ C entry points ----

def sx_init(device: int = 0, hbm_budget: int = 0, stream: Optional[int] = None,
            use_torch_allocator: bool = False):
    """Create a context.  Returns (ctx_handle, keepalive)."""
    lib = load()
    keep = []
    opts = SxCtxOpts(device=device, reserved0=0, hbm_budget=hbm_budget,
                     stream=stream, alloc=ALLOC_FN(), free=FREE_FN(),
                     alloc_user=None)
    if use_torch_allocator:
        import torch
        # blocks are tagged with the stream the library's kernels run on, so
        # that the caching allocator orders their reuse after that stream's
        # work (the context's stream is known once sx_init returns; blocks
        # allocated during sx_init are tagged with the current stream)
        on = {"stream": None}

        def _alloc(nbytes, _user):
            try:
                s = on["stream"] or torch.cuda.current_stream(device)
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), device, s))
            except Exception:
                return None

        def _free(ptr, _user):
            torch.cuda.caching_allocator_delete(int(ptr))

        fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
        keep += [fa, ff]
        opts.alloc, opts.free = fa, ff
    h = C.c_void_p()
    rc = lib.sx_init(C.byref(h), C.byref(opts))
    _check(None, rc)
    if use_torch_allocator:
        on["stream"] = torch.cuda.ExternalStream(int(lib.sx_stream(h) or 0), device=device)
        keep.append(on)
    return h, keep


def sx_finalize(ctx) -> None:
    load().sx_finalize(ctx)


def sx_grid_bytes(w) -> int:
    d = _Desc(w)
    b = C.c_uint64()
    _check(None, load().sx_grid_bytes(C.byref(d.c), C.byref(b)))
    return int(b.value)


def sx_grid_upload(ctx, w) -> int:
    d = _Desc(w)
    gid = C.c_int64()
    _check(ctx, load().sx_grid_upload(ctx, C.byref(d.c), C.byref(gid)))
    return int(gid.value)


def sx_grid_prepare(w):
    """Host part of an upload (no context); returns an opaque handle."""
    d = _Desc(w)
    h = C.c_void_p()
    err = C.create_string_buffer(256)
    rc = load().sx_grid_prepare(C.byref(d.c), C.byref(h), err, 256)
    if rc != SX_OK:
        raise SxError(rc, err.value.decode() or load().sx_strerror(rc).decode())
    return h


def sx_prepared_bytes(p) -> int:
    b = C.c_uint64()
    rc = load().sx_prepared_bytes(p, C.byref(b))
    if rc != SX_OK:
        raise SxError(rc, load().sx_strerror(rc).decode())
    return int(b.value)


def sx_grid_commit(ctx, p) -> int:
    gid = C.c_int64()
    _check(ctx, load().sx_grid_commit(ctx, p, C.byref(gid)))
    return int(gid.value)


def sx_prepared_free(p) -> None:
    load().sx_prepared_free(p)


def sx_rotate_bins(ctx, gid: int, R) -> None:
    r = np.ascontiguousarray(np.asarray(R, np.float64).reshape(9))
    _check(ctx, load().sx_rotate_bins(ctx, gid, _ptr(r)))


def sx_read_edge_state(ctx, gid: int, n: int, n_edges: int) -> dict:
    """Combined transport: photons per edge slot [E] (caller's CSR order) and
    the layout of every vertex [N] (1: it holds edges)."""
    pe = np.zeros(n_edges)
    lay = np.zeros(n, np.uint8)
    _check(ctx, load().sx_read_edge_state(ctx, gid, _ptr(pe), _ptr(lay)))
    return dict(photons_e=pe, layout=lay)


def sx_grid_restore_edges(ctx, gid: int, photons_e, layout) -> None:
    pe = None if photons_e is None else np.ascontiguousarray(photons_e, np.float64)
    lay = np.ascontiguousarray(layout, np.uint8)
    _check(ctx, load().sx_grid_restore_edges(ctx, gid, _ptr(pe), _ptr(lay)))


def sx_read_ballistic(ctx, gid: int, n_edges: int) -> dict:
    sel = np.zeros((n_edges, 3), np.int32)
    cnt = np.zeros(n_edges, np.int32)
    _check(ctx, load().sx_read_ballistic(ctx, gid, _ptr(sel), _ptr(cnt)))
    return dict(bsel=sel, bm=cnt)


def sx_grid_reset(ctx, gid: int) -> None:
    _check(ctx, load().sx_grid_reset(ctx, gid))


def sx_grid_free(ctx, gid: int) -> None:
    _check(ctx, load().sx_grid_free(ctx, gid))


def sx_step(ctx, ids: Sequence[int], n_sweeps: int) -> None:
    a = np.ascontiguousarray(ids, np.int64)
    _check(ctx, load().sx_step(ctx, _ptr(a), int(a.shape[0]), int(n_sweeps)))


def sx_step_noalloc(ctx, ids: Sequence[int], n_sweeps: int) -> None:
    a = np.ascontiguousarray(ids, np.int64)
    _check(ctx, load().sx_step_noalloc(ctx, _ptr(a), int(a.shape[0]), int(n_sweeps)))


def sx_solve(ctx, ids: Sequence[int], n_sweeps) -> None:
    a = np.ascontiguousarray(ids, np.int64)
    s = np.broadcast_to(np.asarray(n_sweeps, np.int32), a.shape).copy()
    _check(ctx, load().sx_solve(ctx, _ptr(a), int(a.shape[0]), _ptr(s)))


def sx_sync(ctx) -> None:
    _check(ctx, load().sx_sync(ctx))


def sx_read_state(ctx, gid: int, n: int, k: int, photons: bool = False,
                  nin: bool = True) -> dict:
    y = np.zeros(n)
    x = np.zeros(n)
    ph = np.zeros((n, k)) if photons else None
    ni = np.zeros(n) if nin else None
    t = SxTally()
    out = SxStateOut(x=_ptr(x), y=_ptr(y), photons=_ptr(ph), nin=_ptr(ni),
                     tally=C.pointer(t))
    _check(ctx, load().sx_read_state(ctx, gid, C.byref(out)))
    return dict(x=x, y=y, photons=ph, nin=ni,
                tallies=dict(sweeps=t.sweeps, emitted=t.emitted,
                             absorbed=t.absorbed, escaped=t.escaped,
                             in_flight=t.in_flight))


def sx_grid_restore(ctx, gid: int, y=None, photons=None, tallies=None) -> None:
    ya = None if y is None else np.ascontiguousarray(y, np.float64)
    pa = None if photons is None else np.ascontiguousarray(photons, np.float64)
    tp = None
    if tallies is not None:
        tp = C.pointer(SxTally(**{k: float(tallies[k]) for k in
                                  ("sweeps", "emitted", "absorbed", "escaped", "in_flight")}))
    si = SxStateIn(y=_ptr(ya), photons=_ptr(pa), tally=tp)
    _check(ctx, load().sx_grid_restore(ctx, gid, C.byref(si)))


def sx_read_tables(ctx, gid: int, n: int, k: int, n_edges: int) -> dict:
    sel = np.zeros((n, k, 3), np.int32)
    m = np.zeros((n, k), np.int32)
    eb = np.zeros(n_edges, np.int32)
    dL = np.zeros(n)
    tau = np.zeros(n)
    _check(ctx, load().sx_read_tables(ctx, gid, _ptr(sel), _ptr(m), _ptr(eb),
                                      _ptr(dL), _ptr(tau)))
    return dict(sel_nbr=sel, sel_m=m, edge_bin=eb, dL=dL, tau=tau)


def sx_grid_info(ctx, gid: int) -> dict:
    n = C.c_int64()
    k = C.c_int32()
    e = C.c_int64()
    p = C.c_int32()
    u = C.c_double()
    b = C.c_uint64()
    _check(ctx, load().sx_grid_info(ctx, gid, C.byref(n), C.byref(k), C.byref(e),
                                    C.byref(p), C.byref(u), C.byref(b)))
    return dict(n=n.value, k=k.value, n_edges=e.value, precision=p.value,
                photon_unit=u.value, bytes=b.value)


def sx_mem_info(ctx) -> tuple[int, int]:
    u = C.c_uint64()
    b = C.c_uint64()
    _check(ctx, load().sx_mem_info(ctx, C.byref(u), C.byref(b)))
    return int(u.value), int(b.value)


def sx_stream(ctx) -> int:
    return int(load().sx_stream(ctx) or 0)


def sx_profile(ctx, enable: bool) -> None:
    _check(ctx, load().sx_profile(ctx, 1 if enable else 0))


def sx_profile_read(ctx) -> dict:
    n = C.c_int64()
    t = C.c_double()
    lo = C.c_double()
    hi = C.c_double()
    _check(ctx, load().sx_profile_read(ctx, C.byref(n), C.byref(t), C.byref(lo),
                                       C.byref(hi)))
    return dict(launches=n.value, total_ms=t.value, min_ms=lo.value, max_ms=hi.value)


def _ids(ids):
    a = np.ascontiguousarray(np.asarray(ids, dtype=np.int64).reshape(-1))
    return a, (_ptr(a) if a.size else None), int(a.size)


def sx_set_schedule(ctx, ids, tiles_per_group=4, order=SX_ORDER_GRID,
                    xcd_contiguous=1, graph_sweeps=50, work_split=1) -> None:
    a, p, n = _ids(ids)
    s = SxSchedule(tiles_per_group, order, xcd_contiguous, graph_sweeps, work_split)
    _check(ctx, load().sx_set_schedule(ctx, p, n, C.byref(s)))


def sx_get_schedule(ctx, ids) -> dict:
    a, p, n = _ids(ids)
    s = SxSchedule()
    us = C.c_double()
    _check(ctx, load().sx_get_schedule(ctx, p, n, C.byref(s), C.byref(us)))
    return dict(tiles_per_group=s.tiles_per_group, order=s.order,
                xcd_contiguous=s.xcd_contiguous, graph_sweeps=s.graph_sweeps,
                work_split=max(1, s.work_split), us_per_sweep=us.value)


def sx_autotune(ctx, trials: int) -> None:
    _check(ctx, load().sx_autotune(ctx, int(trials)))


class Server:
    """The library's request loop (continuous batching) over a Context.
    While it runs, the context belongs to the server."""

    def __init__(self, ctx: "Context", round_sweeps: int = 50, max_active: int = 64,
                 prep_threads: int = 4, hbm_budget: int = 0):
        o = SxServeOpts(round_sweeps, max_active, prep_threads, 0, hbm_budget)
        h = C.c_void_p()
        rc = load().sx_serve_start(ctx.h, C.byref(o), C.byref(h))
        if rc != SX_OK:
            raise SxError(rc, load().sx_strerror(rc).decode())
        self.h = h
        self.n = {}

    def submit(self, w, n_sweeps: int) -> int:
        d = _Desc(w)
        t = C.c_int64()
        rc = load().sx_serve_submit(self.h, C.byref(d.c), int(n_sweeps), C.byref(t))
        if rc != SX_OK:
            raise SxError(rc, load().sx_strerror(rc).decode())
        self.n[int(t.value)] = w.n
        return int(t.value)

    def poll(self, timeout: float = 1.0):
        r = SxServeResult()
        rc = load().sx_serve_poll(self.h, float(timeout), C.byref(r))
        if rc == SX_EAGAIN:
            return None
        if rc != SX_OK:
            raise SxError(rc, load().sx_strerror(rc).decode())
        t = r.tally
        return dict(ticket=r.ticket, status=r.status, n_vertices=r.n_vertices,
                    n_bins=r.n_bins, n_sweeps=r.n_sweeps, t_submit=r.t_submit,
                    t_prepared=r.t_prepared, t_admit=r.t_admit, t_done=r.t_done,
                    tallies=dict(sweeps=t.sweeps, emitted=t.emitted, absorbed=t.absorbed,
                                 escaped=t.escaped, in_flight=t.in_flight))

    def take(self, ticket: int):
        n = self.n.pop(ticket)
        x = np.empty(n)
        y = np.empty(n)
        rc = load().sx_serve_take(self.h, int(ticket), _ptr(x), _ptr(y))
        if rc != SX_OK:
            raise SxError(rc, load().sx_strerror(rc).decode())
        return x, y

    def stop(self) -> dict:
        st = SxServeStats()
        if self.h:
            load().sx_serve_stop(self.h, C.byref(st))
            self.h = None
        return {f: getattr(st, f) for f, _ in SxServeStats._fields_ if f != "reserved"}


# ------------------------------------------------------ convenience ----

class Context:
    """RAII wrapper: a context plus uploaded grids keyed by id."""

    def __init__(self, device: int = 0, hbm_budget: int = 0,
                 stream: Optional[int] = None, use_torch_allocator: bool = False):
        self.h, self._keep = sx_init(device, hbm_budget, stream, use_torch_allocator)
        self.shapes = {}

    def upload(self, w) -> int:
        gid = sx_grid_upload(self.h, w)
        self.shapes[gid] = (w.n, w.k, w.n_edges)
        return gid

    def reset(self, gid):
        sx_grid_reset(self.h, gid)

    def rotate(self, gid, R):
        sx_rotate_bins(self.h, gid, R)

    def step(self, ids, n_sweeps):
        sx_step(self.h, ids, n_sweeps)

    def step_noalloc(self, ids, n_sweeps):
        """sx_step with no device allocation (static scratch tables)."""
        sx_step_noalloc(self.h, ids, n_sweeps)

    def solve(self, ids, n_sweeps):
        sx_solve(self.h, ids, n_sweeps)

    def sync(self):
        sx_sync(self.h)

    def state(self, gid, photons=False, nin=True):
        n, k, _ = self.shapes[gid]
        return sx_read_state(self.h, gid, n, k, photons=photons, nin=nin)

    def restore(self, gid, **kw):
        sx_grid_restore(self.h, gid, **kw)

    def edge_state(self, gid) -> dict:
        n, _, e = self.shapes[gid]
        return sx_read_edge_state(self.h, gid, n, e)

    def restore_edges(self, gid, photons_e, layout):
        sx_grid_restore_edges(self.h, gid, photons_e, layout)

    def diffuse_pending(self, gid):
        """Recombination photons each vertex sends at the next step [N]."""
        n, _, _ = self.shapes[gid]
        d = np.zeros(n)
        _check(self.h, load().sx_read_diffuse(self.h, gid, _ptr(d)))
        return d

    def select_removal(self, gid, tau_remove: float, min_spacing: float):
        """Vertices to remove between solves [N] bool (Sect. 2.1.4)."""
        n, _, _ = self.shapes[gid]
        rm = np.zeros(n, np.uint8)
        cnt = C.c_int64()
        _check(self.h, load().sx_grid_select_removal(self.h, gid, float(tau_remove),
                                                     float(min_spacing), _ptr(rm),
                                                     C.byref(cnt)))
        return rm.astype(bool)

    def remap(self, src, dst, new_of_old):
        """Move the state of grid src onto grid dst (new_of_old: -1 removed)."""
        a = np.ascontiguousarray(new_of_old, np.int32)
        _check(self.h, load().sx_grid_remap(self.h, src, dst, _ptr(a)))

    def ballistic(self, gid) -> dict:
        _, _, e = self.shapes[gid]
        return sx_read_ballistic(self.h, gid, e)

    def tables(self, gid):
        n, k, e = self.shapes[gid]
        return sx_read_tables(self.h, gid, n, k, e)

    def info(self, gid):
        return sx_grid_info(self.h, gid)

    def free(self, gid):
        sx_grid_free(self.h, gid)
        self.shapes.pop(gid, None)

    def mem_info(self):
        return sx_mem_info(self.h)

    def profile(self, enable: bool = True):
        sx_profile(self.h, enable)

    def profile_read(self) -> dict:
        return sx_profile_read(self.h)

    def set_schedule(self, ids, **kw):
        sx_set_schedule(self.h, ids, **kw)

    def get_schedule(self, ids) -> dict:
        return sx_get_schedule(self.h, ids)

    def autotune(self, trials: int):
        sx_autotune(self.h, trials)

    @property
    def stream(self) -> int:
        return sx_stream(self.h)

    def close(self):
        if self.h:
            sx_finalize(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
