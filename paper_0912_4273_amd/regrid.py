"""Dynamic grid between solves (Sect. 2.1.4): thin the grid where the
optical depth has dropped, down to a minimum resolution.

The library chooses the vertices (sx_grid_select_removal), the host
triangulates the rest (Qhull, as when the grid was made), the new grid is
uploaded with the same bins and the state is moved over on the library side
(sx_grid_remap)."""
from __future__ import annotations

import numpy as np

from . import gridgen as G


def min_spacing_for(box: float, n_min: int) -> float:
    """Spacing of a minimum resolution of n_min^3 points over the box."""
    return box / float(n_min)


def thinned_workload(w, keep: np.ndarray, x_now: np.ndarray):
    """The workload on the kept vertices: their positions, densities and
    sources, a fresh Delaunay graph and cell volumes, the current ionised
    fraction as the initial state.  Returns (workload, new_of_old)."""
    keep = np.asarray(keep, bool)
    new_of_old = np.full(w.n, -1, np.int32)
    new_of_old[keep] = np.arange(int(keep.sum()), dtype=np.int32)
    pts = np.ascontiguousarray(w.pos[keep])
    ptr, idx, simp = G.delaunay(pts)
    vol = G.dual_volumes(pts, simp)
    src = new_of_old[np.asarray(w.src_vertex)]
    if np.any(src < 0):
        raise ValueError("a source vertex was removed")
    wn = G.with_(w, name=w.name + "_thinned", pos=pts, nbr_ptr=ptr, nbr_idx=idx,
                 n_H=np.asarray(w.n_H)[keep], volume=vol, dL=None,
                 x_init=np.asarray(x_now)[keep], src_vertex=src.astype(np.int32))
    return wn, new_of_old


def regrid(ctx, gid: int, w, tau_remove: float, min_spacing: float):
    """One thinning pass of grid gid (workload w).  Returns (new workload,
    new grid id, new_of_old); the old grid stays uploaded."""
    rm = ctx.select_removal(gid, tau_remove, min_spacing)
    st = ctx.state(gid, nin=False)
    wn, new_of_old = thinned_workload(w, ~rm, st["x"])
    gn = ctx.upload(wn)
    ctx.remap(gid, gn, new_of_old)
    return wn, gn, new_of_old
