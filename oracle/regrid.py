"""Dynamic grid between solves (Sect. 2.1.4) for the oracle: which vertices
to remove, and the state moved onto the thinned grid.  Test infrastructure
only; numpy, written from the rule, sharing nothing with the library.

Rule (the paper gives no more detail): a vertex is a candidate when its
optical depth y tau is below tau_remove, its path length dL below the
minimum-resolution spacing, and it holds no source; candidates are taken in
ascending optical depth (ties: lower id), skipping those next to one already
taken.  State: kept vertices keep y; the photons a vertex holds per bin (m O)
stay in that bin with the vertex (or, for a removed one, with its nearest
kept former neighbour, ties to the lower id), split over the new selection;
with no selection they escape.

Combined transport: a vertex that holds its photons per incoming edge (the
packet that came along i -> j, bm O_e in all) files them in the bin of that
edge, the rule by which a direction-conserving vertex takes photons from a
ballistic sender (Sect. 2.2.4), and they move as bin holdings; every vertex
of the thinned grid starts holding bins.  Diffuse recombination radiation:
the photons a vertex has made and sends at the next step move with it (or
to a removed vertex's nearest kept neighbour) and are sent from there; with
no kept neighbour they escape."""
import numpy as np


def select_removal(w, y, tau, dL, tau_remove, min_spacing):
    """Boolean [N]: the vertices to remove."""
    od = np.asarray(y) * np.asarray(tau)
    is_src = np.zeros(w.n, bool)
    is_src[np.asarray(w.src_vertex)] = True
    cand = np.nonzero((od < tau_remove) & (np.asarray(dL) < min_spacing) & ~is_src)[0]
    order = sorted(cand.tolist(), key=lambda i: (od[i], i))
    taken = np.zeros(w.n, bool)
    near = np.zeros(w.n, bool)
    for i in order:
        if near[i]:
            continue
        taken[i] = True
        near[w.nbr_idx[w.nbr_ptr[i]:w.nbr_ptr[i + 1]]] = True
    return taken


def edge_holdings_as_bins(w, photons_e, layout, bm, edge_bin):
    """[N, K]: what vertices holding edges hold, filed per bin.  photons_e
    [E] is each in-edge's share per chosen neighbour (bm of them); in-edge
    p of row j comes from i = nbr_idx[p] and goes in the bin of the edge
    i -> j (edge_bin, by directed edge in row order)."""
    K = w.k
    out = np.zeros((w.n, K))
    for j in range(w.n):
        if not layout[j]:
            continue
        for p in range(w.nbr_ptr[j], w.nbr_ptr[j + 1]):
            i = int(w.nbr_idx[p])
            row = w.nbr_idx[w.nbr_ptr[i]:w.nbr_ptr[i + 1]]
            q = int(w.nbr_ptr[i] + np.nonzero(row == j)[0][0])
            out[j, int(edge_bin[q])] += photons_e[p] * bm[p]
    return out


def _nearest_kept(w_old, i, new_of_old):
    nb = w_old.nbr_idx[w_old.nbr_ptr[i]:w_old.nbr_ptr[i + 1]]
    best, bo = None, -1
    for o in nb:
        if new_of_old[o] < 0:
            continue
        d = w_old.pos[o] - w_old.pos[i]
        ln = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        if bo < 0 or ln < best or (ln == best and o < bo):
            best, bo = ln, int(o)
    return int(new_of_old[bo]) if bo >= 0 else -1


def remap_pending(w_old, pending, new_of_old):
    """(pending_new, photons that escape): the recombination photons each
    vertex sends at the next step, moved with it or to a removed vertex's
    nearest kept neighbour, added in ascending old id."""
    n_new = int(np.max(new_of_old)) + 1
    out = np.zeros(n_new)
    lost = 0.0
    for i in range(w_old.n):
        j = int(new_of_old[i])
        if j < 0:
            j = _nearest_kept(w_old, i, new_of_old)
        if j >= 0:
            out[j] += pending[i]
        else:
            lost += float(pending[i])
    return out, lost


def remap(w_old, y_old, photons_old, m_old, new_of_old, m_new, extra=None):
    """(y_new, photons_new, photons that escape) after thinning.  extra
    [N, K]: more holdings per bin (edge holdings of combined transport)."""
    n_new = int(np.max(new_of_old)) + 1
    K = photons_old.shape[1]
    held = np.zeros((n_new, K))
    y_new = np.ones(n_new)
    lost = 0.0
    for i in range(w_old.n):
        j = int(new_of_old[i])
        if j >= 0:
            y_new[j] = y_old[i]
        else:
            j = _nearest_kept(w_old, i, new_of_old)
        h = photons_old[i] * m_old[i]
        if extra is not None:
            h = h + extra[i]
        if j >= 0:
            held[j] += h
        else:
            lost += float(np.sum(h))
    ph = np.zeros((n_new, K))
    sel = m_new > 0
    ph[sel] = held[sel] / m_new[sel]
    lost += float(np.sum(held[~sel]))
    return y_new, ph, lost
