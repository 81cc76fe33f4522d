"""ctypes wrapper of the C oracle (sx_oracle.c).  Test infrastructure only."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sx_oracle.c")


def oracle_lib_path() -> str:
    return os.path.join(_HERE, "liboracle_sx.so")


def build_oracle(force: bool = False, src: str = _SRC, out: str = None) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, strict IEEE."""
    out = out or oracle_lib_path()
    if force or not os.path.exists(out) or \
            os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
            "-Wall", "-I", _HERE, "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


_libs = {}


def _load(path=None):
    """Load the oracle library (default: the in-tree build).  Another path
    may be given to load a variant built from a modified copy of the source
    (used by the tests that plant mistakes in the oracle)."""
    key = path or oracle_lib_path()
    if key not in _libs:
        if path is None and not os.path.exists(key):
            build_oracle()
        lib = C.CDLL(key)
        P = C.c_void_p
        lib.ora_create.restype = P
        lib.ora_create.argtypes = [
            C.c_int64, P, P, P, P, P, P, C.c_double, P, C.c_int32, P,
            C.c_int32, C.c_double, C.c_int32, P, P, P, C.c_double,
            C.c_double, C.c_double, C.c_int32]
        lib.ora_run.restype = C.c_int
        lib.ora_run.argtypes = [P, C.c_int32, P]
        lib.ora_run_threads.restype = C.c_int
        lib.ora_run_threads.argtypes = [P, C.c_int32, C.c_int32]
        lib.ora_get_state.restype = None
        lib.ora_get_state.argtypes = [P, P, P, P, P, P]
        lib.ora_set_state.restype = None
        lib.ora_set_state.argtypes = [P, P, P, P]
        lib.ora_get_tables.restype = None
        lib.ora_get_tables.argtypes = [P, P, P, P, P, P]
        lib.ora_rotate.restype = C.c_int
        lib.ora_rotate.argtypes = [P, P]
        lib.ora_set_diffuse.restype = C.c_int
        lib.ora_set_diffuse.argtypes = [P, C.c_double]
        lib.ora_get_diffuse.restype = None
        lib.ora_get_diffuse.argtypes = [P, P]
        lib.ora_set_diffuse_pending.restype = None
        lib.ora_set_diffuse_pending.argtypes = [P, P]
        lib.ora_set_hops.restype = C.c_int
        lib.ora_set_hops.argtypes = [P, C.c_int32]
        lib.ora_set_dct_reference.restype = C.c_int
        lib.ora_set_dct_reference.argtypes = [P, C.c_int32]
        lib.ora_set_transport.restype = C.c_int
        lib.ora_set_transport.argtypes = [P, C.c_int32, C.c_double]
        lib.ora_get_edge_state.restype = None
        lib.ora_get_edge_state.argtypes = [P, P, P]
        lib.ora_set_edge_state.restype = None
        lib.ora_set_edge_state.argtypes = [P, P, P]
        lib.ora_get_ballistic.restype = None
        lib.ora_get_ballistic.argtypes = [P, P, P]
        lib.ora_free.restype = None
        lib.ora_free.argtypes = [P]
        lib.ora_chem_cell.restype = C.c_double
        lib.ora_chem_cell.argtypes = [
            C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
            C.c_double, C.c_int32, P, P]
        lib.ora_last_error.restype = C.c_char_p
        _libs[key] = lib
    return _libs[key]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def chem_cell(y, n_in, dt, nHV, tau, b, n_sub, lib_path=None):
    """(y_new, absorbed, transmitted) for one cell over one step."""
    lib = _load(lib_path)
    A = C.c_double()
    T = C.c_double()
    yn = lib.ora_chem_cell(float(y), float(n_in), float(dt), float(nHV),
                           float(tau), float(b), int(n_sub), C.byref(A),
                           C.byref(T))
    return yn, A.value, T.value


class Oracle:
    """One grid held by the C oracle.  Takes a gridgen.Workload."""

    def __init__(self, w, lib_path=None):
        lib = _load(lib_path)
        self._lib = lib
        self.w = w
        self.n = w.n
        self.k = w.k
        self.mpb = int(w.max_per_bin)
        self._keep = dict(
            pos=np.ascontiguousarray(w.pos, np.float64),
            ptr=np.ascontiguousarray(w.nbr_ptr, np.int64),
            idx=np.ascontiguousarray(w.nbr_idx, np.int32),
            nH=np.ascontiguousarray(w.n_H, np.float64),
            vol=np.ascontiguousarray(w.volume, np.float64),
            dL=None if w.dL is None else np.ascontiguousarray(w.dL, np.float64),
            x0=None if w.x_init is None else np.ascontiguousarray(w.x_init, np.float64),
            bins=np.ascontiguousarray(w.bin_dirs, np.float64),
            sv=np.ascontiguousarray(w.src_vertex, np.int32),
            sr=np.ascontiguousarray(w.src_rate, np.float64),
            sd=None if w.src_dir is None else np.ascontiguousarray(w.src_dir, np.float64),
        )
        k = self._keep
        h = lib.ora_create(
            self.n, _p(k["pos"]), _p(k["ptr"]), _p(k["idx"]), _p(k["nH"]),
            _p(k["vol"]), _p(k["dL"]), float(w.kappa), _p(k["x0"]), self.k,
            _p(k["bins"]), self.mpb, float(w.cos_min), int(k["sv"].shape[0]),
            _p(k["sv"]), _p(k["sr"]), _p(k["sd"]), float(w.sigma),
            float(w.alpha_B), float(w.dt), int(w.n_subcycles))
        if not h:
            raise ValueError("oracle: " + lib.ora_last_error().decode())
        self._h = h
        if float(getattr(w, "alpha_A", 0.0)) > 0.0:
            if lib.ora_set_diffuse(h, float(w.alpha_A)) != 0:
                raise ValueError("oracle: " + lib.ora_last_error().decode())
        if int(getattr(w, "dct_reference", 0)) == 1:
            lib.ora_set_dct_reference(h, 1)
        self.combined = int(getattr(w, "transport", 0)) == 1
        if self.combined:
            lib.ora_set_transport(h, 1, float(w.tau_switch))
        if int(getattr(w, "hops", 1)) > 1:
            self.set_hops(int(w.hops))

    def run(self, n_sweeps: int, history: bool = False):
        hist = np.zeros((n_sweeps, 4)) if history else None
        self._lib.ora_run(self._h, int(n_sweeps), _p(hist))
        return hist

    def run_threads(self, n_sweeps: int, threads: int):
        """Timing-only pull form of run() on `threads` OpenMP threads
        (direction-conserving, on the spot)."""
        if self._lib.ora_run_threads(self._h, int(n_sweeps), int(threads)) != 0:
            raise ValueError("oracle: threaded run covers direction-conserving, on-the-spot grids")

    def state(self):
        n, k = self.n, self.k
        y = np.zeros(n)
        x = np.zeros(n)
        ph = np.zeros((n, k))
        nin = np.zeros(n)
        t = np.zeros(5)
        self._lib.ora_get_state(self._h, _p(y), _p(x), _p(ph), _p(nin), _p(t))
        return dict(y=y, x=x, photons=ph, nin=nin,
                    tallies=dict(sweeps=t[0], emitted=t[1], absorbed=t[2],
                                 escaped=t[3], in_flight=t[4]))

    def set_state(self, y=None, photons=None, tallies=None):
        y = None if y is None else np.ascontiguousarray(y, np.float64)
        ph = None if photons is None else np.ascontiguousarray(photons, np.float64)
        t = None
        if tallies is not None:
            t = np.array([tallies["sweeps"], tallies["emitted"],
                          tallies["absorbed"], tallies["escaped"],
                          tallies["in_flight"]], np.float64)
        self._lib.ora_set_state(self._h, _p(y), _p(ph), _p(t))

    def diffuse_pending(self):
        """Recombination photons each vertex sends at the next sweep [N]."""
        d = np.zeros(self.n)
        self._lib.ora_get_diffuse(self._h, _p(d))
        return d

    def set_diffuse_pending(self, pending):
        self._lib.ora_set_diffuse_pending(self._h, _p(np.ascontiguousarray(pending, np.float64)))

    def set_hops(self, hops: int):
        """Hops per step (multi-hop steps, Sect. 4.6); every sweep is a hop."""
        if self._lib.ora_set_hops(self._h, int(hops)) != 0:
            raise ValueError("oracle: " + self._lib.ora_last_error().decode())

    def set_transport(self, combined: bool, tau_switch: float = 1.0):
        """Switch between direction-conserving and combined transport."""
        self._lib.ora_set_transport(self._h, 1 if combined else 0, float(tau_switch))
        self.combined = bool(combined)

    def edge_state(self):
        """Combined transport: photons per edge slot [E] and the layout of
        every vertex [N] (0 bins, 1 edges)."""
        pe = np.zeros(self.w.n_edges)
        lay = np.zeros(self.n, np.int8)
        self._lib.ora_get_edge_state(self._h, _p(pe), _p(lay))
        return dict(photons_e=pe, layout=lay)

    def set_edge_state(self, photons_e=None, layout=None):
        pe = None if photons_e is None else np.ascontiguousarray(photons_e, np.float64)
        lay = None if layout is None else np.ascontiguousarray(layout, np.int8)
        self._lib.ora_set_edge_state(self._h, _p(pe), _p(lay))

    def ballistic(self):
        """Ballistic tables: chosen neighbours [E, mpb] (-1 padding), counts [E]."""
        sel = np.zeros((self.w.n_edges, self.mpb), np.int32)
        cnt = np.zeros(self.w.n_edges, np.int32)
        self._lib.ora_get_ballistic(self._h, _p(sel), _p(cnt))
        return dict(bsel=sel, bm=cnt)

    def rotate(self, R):
        """Rotate the direction bins to R u_k (Sect. 2.2.3)."""
        r = np.ascontiguousarray(np.asarray(R, np.float64).reshape(9))
        self._lib.ora_rotate(self._h, _p(r))

    def tables(self):
        n, k, m = self.n, self.k, self.mpb
        sel = np.zeros((n, k, m), np.int32)
        cnt = np.zeros((n, k), np.int32)
        eb = np.zeros(self.w.n_edges, np.int32)
        dL = np.zeros(n)
        tau = np.zeros(n)
        self._lib.ora_get_tables(self._h, _p(sel), _p(cnt), _p(eb), _p(dL), _p(tau))
        return dict(sel_nbr=sel, sel_m=cnt, edge_bin=eb, dL=dL, tau=tau)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ora_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
