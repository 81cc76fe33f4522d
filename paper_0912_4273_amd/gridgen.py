"""Seeded synthetic workloads shaped like the SimpleX2 test problems.

This module builds *inputs* only: point sets, their Delaunay neighbour graph,
cell volumes, direction-bin sets and source lists.  It holds none of the
transport or chemistry arithmetic (no edge directions, no bin selection, no
optical depths, no rate equation); both the GPU library and the CPU oracle
receive exactly the arrays produced here.

Grid construction follows the paper's recipe (Sect. 2.1): a (homogeneous or
non-homogeneous) Poisson point process, then the Delaunay triangulation by
Qhull (scipy.spatial.Delaunay wraps Qhull).  Units are CGS throughout.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

KPC_CM = 3.0857e21          # 1 kpc in cm
MYR_S = 3.15576e13          # 1 Myr (Julian years) in s

# Physics of the isothermal H II region test (Sect. 5.1): monochromatic
# 13.6 eV photons, T = 1e4 K, case-B recombination.
SIGMA_H = 6.3e-18           # cm^2, Eq. (cross_section) at the Lyman limit
ALPHA_B = 2.59e-13          # cm^3 s^-1, case B at 1e4 K
ALPHA_A = 4.18e-13          # cm^3 s^-1, case A (all levels) at 1e4 K

SX_FP64 = 0
SX_FP32_TRANSPORT = 1

SX_TRANSPORT_DCT = 0        # direction-conserving transport everywhere
SX_TRANSPORT_COMBINED = 1   # ballistic where y tau >= tau_switch (Sect. 2.2.4)
SX_DCT_REF_BIN = 0          # bins go by their own direction
SX_DCT_REF_EDGE = 1         # bins go by the vertex's edge closest to them


@dataclass
class Workload:
    """Every input of one solve, in the caller's (original) vertex order."""
    name: str
    pos: np.ndarray                  # [N,3] float64, cm
    nbr_ptr: np.ndarray              # [N+1] int64
    nbr_idx: np.ndarray              # [E] int32, symmetric, rows sorted
    n_H: np.ndarray                  # [N] float64, cm^-3
    volume: np.ndarray               # [N] float64, cm^3
    bin_dirs: np.ndarray             # [K,3] float64 unit vectors
    src_vertex: np.ndarray           # [S] int32
    src_rate: np.ndarray             # [S] float64 photons/s
    dt: float                        # s
    n_sweeps: int
    src_dir: Optional[np.ndarray] = None   # [S,3] or None (isotropic)
    x_init: Optional[np.ndarray] = None    # [N] or None (neutral)
    dL: Optional[np.ndarray] = None        # [N] or None (kappa * mean edge)
    kappa: float = 1.0
    sigma: float = SIGMA_H
    alpha_B: float = ALPHA_B
    n_subcycles: int = 10
    max_per_bin: int = 3
    cos_min: float = 0.0
    precision: int = SX_FP64
    transport: int = SX_TRANSPORT_DCT
    tau_switch: float = 1.0
    dct_reference: int = SX_DCT_REF_BIN
    alpha_A: float = 0.0             # > 0: diffuse recombination radiation
    hops: int = 1                    # edges photons cross per step (multi-hop)
    box: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def k(self) -> int:
        return int(self.bin_dirs.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.nbr_idx.shape[0])

    def updates_per_sweep(self) -> int:
        return self.n * self.k


# ---------------------------------------------------------------- points ---

def poisson_points(n: int, box: float, rng: np.random.Generator) -> np.ndarray:
    """Homogeneous Poisson process conditioned on n points in [0, box]^3."""
    return rng.random((n, 3)) * box


def rejection_points(n: int, box: float, weight, wmax: float,
                     rng: np.random.Generator) -> np.ndarray:
    """Non-homogeneous Poisson process: accept uniform candidates with
    probability weight(p)/wmax until n points are kept (Eq. point_process)."""
    out = []
    have = 0
    while have < n:
        m = max(4096, int(1.3 * (n - have) * 2))
        cand = rng.random((m, 3)) * box
        keep = rng.random(m) * wmax < weight(cand)
        cand = cand[keep]
        out.append(cand)
        have += cand.shape[0]
    return np.concatenate(out)[:n]


# ------------------------------------------------------------- delaunay ---

def delaunay(points: np.ndarray):
    """Delaunay triangulation (Qhull); returns (nbr_ptr int64, nbr_idx int32
    with each row sorted ascending, simplices int32 [T,4])."""
    from scipy.spatial import Delaunay
    tri = Delaunay(points)
    ptr, idx = tri.vertex_neighbor_vertices
    ptr = ptr.astype(np.int64)
    idx = idx.astype(np.int32).copy()
    # canonical row order: ascending neighbour id
    row = np.repeat(np.arange(points.shape[0], dtype=np.int64), np.diff(ptr))
    order = np.lexsort((idx, row))
    idx = idx[order]
    return ptr, idx, tri.simplices.astype(np.int32)


def dual_volumes(points: np.ndarray, simplices: np.ndarray) -> np.ndarray:
    """Cell volume of each vertex: a quarter of the volume of every Delaunay
    tetrahedron it belongs to.  The volumes sum to the hull volume."""
    p = points[simplices]                       # [T,4,3]
    a = p[:, 1] - p[:, 0]
    b = p[:, 2] - p[:, 0]
    c = p[:, 3] - p[:, 0]
    vol = np.abs(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0
    v = np.zeros(points.shape[0])
    np.add.at(v, simplices.ravel(), np.repeat(vol / 4.0, 4))
    return v


# ----------------------------------------------------------------- bins ---

def icosahedral_bins_42() -> np.ndarray:
    """42 unit vectors: the 12 vertices of an icosahedron, (0, +-1, +-phi)
    and its cyclic permutations, followed by the 30 normalised midpoints of
    its edges (a once-subdivided icosahedron).  Fixed order."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    verts = []
    for s1 in (1.0, -1.0):
        for s2 in (phi, -phi):
            verts.append((0.0, s1, s2))
            verts.append((s1, s2, 0.0))
            verts.append((s2, 0.0, s1))
    v = np.array(verts)
    v /= np.linalg.norm(v, axis=1)[:, None]
    # edges: pairs at the minimal distance
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    dmin = d[d > 1e-9].min()
    mids = []
    for i in range(12):
        for j in range(i + 1, 12):
            if abs(d[i, j] - dmin) < 1e-9:
                m = v[i] + v[j]
                mids.append(m / np.linalg.norm(m))
    assert len(mids) == 30
    return np.concatenate([v, np.array(mids)])


def random_bins(k: int, seed: int) -> np.ndarray:
    """k uniform-on-sphere unit vectors from normalised Gaussian triples."""
    g = np.random.default_rng(seed).normal(size=(k, 3))
    return g / np.linalg.norm(g, axis=1)[:, None]


def axis_bins() -> np.ndarray:
    """+x, -x, +y, -y, +z, -z."""
    return np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0],
                     [0, -1.0, 0], [0, 0, 1.0], [0, 0, -1.0]])


# --------------------------------------------------------- test problems ---

def nearest_vertex(points: np.ndarray, p) -> int:
    return int(np.argmin(np.sum((points - np.asarray(p)) ** 2, axis=1)))


def stromgren_test(n: int = 4096, seed: int = 1, n_bins: int = 42,
                   bins_seed: int = 102, box_kpc: float = 13.2,
                   n_H: float = 1e-3, rate: float = 5e48,
                   t_end_myr: float = 500.0, n_sweeps: int = 200,
                   precision: int = SX_FP64, name: str = "") -> Workload:
    """Test 1 of the paper (Sect. 5.1): a single source at the centre of a
    homogeneous, initially neutral box.  n Poisson points; 42 icosahedral
    bins or n_bins random unit vectors from bins_seed."""
    box = box_kpc * KPC_CM
    rng = np.random.default_rng(seed)
    pts = poisson_points(n, box, rng)
    ptr, idx, simp = delaunay(pts)
    vol = dual_volumes(pts, simp)
    bins = icosahedral_bins_42() if n_bins == 42 else random_bins(n_bins, bins_seed)
    src = nearest_vertex(pts, (box / 2, box / 2, box / 2))
    return Workload(
        name=name or f"stromgren_n{n}_k{n_bins}",
        pos=pts, nbr_ptr=ptr, nbr_idx=idx,
        n_H=np.full(n, n_H), volume=vol, bin_dirs=bins,
        src_vertex=np.array([src], np.int32), src_rate=np.array([rate]),
        dt=t_end_myr * MYR_S / n_sweeps, n_sweeps=n_sweeps,
        precision=precision, box=box,
        meta=dict(seed=seed, box_kpc=box_kpc, n_H=n_H, rate=rate,
                  t_end_myr=t_end_myr))


def config1() -> Workload:
    """4096 Poisson vertices in a 13.2 kpc cube, 42 icosahedral bins,
    200 sweeps over 500 Myr, all-FP64."""
    return stromgren_test(4096, seed=1, n_bins=42, n_sweeps=200,
                          precision=SX_FP64, name="stromgren_4096_k42_fp64")


def config2(precision: int = SX_FP32_TRANSPORT) -> Workload:
    """262144 Poisson vertices in the same box, 84 random bins (seed 102),
    1000 sweeps over 500 Myr."""
    return stromgren_test(262144, seed=2, n_bins=84, bins_seed=102,
                          n_sweeps=1000, precision=precision,
                          name="stromgren_262144_k84")


def shadow_test(n: int = 1048576, seed: int = 3, n_bins: int = 84,
                bins_seed: int = 103, box_kpc: float = 6.6,
                n_H: float = 2e-4, contrast: float = 200.0,
                clump_r_kpc: float = 0.8, clump_c_kpc=(5.0, 3.3, 3.3),
                flux: float = 1e6, t_end_myr: float = 15.0,
                n_sweeps: int = 1500,
                precision: int = SX_FP32_TRANSPORT) -> Workload:
    """Shadowing problem: uniform medium plus a dense sphere, points drawn
    with density proportional to n_H^(1/3), plane-parallel source on the
    x = 0 face.  The face's photon rate F * A is split equally over the
    vertices closer to the face than one local mean spacing; each emits as a
    beam along +x."""
    box = box_kpc * KPC_CM
    rc = clump_r_kpc * KPC_CM
    cc = np.array(clump_c_kpc) * KPC_CM
    rng = np.random.default_rng(seed)

    def dens(p):
        inside = np.sum((p - cc) ** 2, axis=1) < rc * rc
        return np.where(inside, n_H * contrast, n_H)

    wmax = (n_H * contrast) ** (1.0 / 3.0)
    pts = rejection_points(n, box, lambda p: dens(p) ** (1.0 / 3.0), wmax, rng)
    ptr, idx, simp = delaunay(pts)
    vol = dual_volumes(pts, simp)
    nh = dens(pts)
    # local mean spacing of the uniform part: (V_box_uniform / N_uniform)^(1/3)
    n_out = int(np.sum(nh == n_H))
    v_out = box ** 3 - 4.0 / 3.0 * math.pi * rc ** 3
    spacing = (v_out / max(n_out, 1)) ** (1.0 / 3.0)
    src = np.nonzero(pts[:, 0] < spacing)[0].astype(np.int32)
    total = flux * box * box
    bins = random_bins(n_bins, bins_seed)
    return Workload(
        name=f"shadow_{n}_k{n_bins}",
        pos=pts, nbr_ptr=ptr, nbr_idx=idx, n_H=nh, volume=vol, bin_dirs=bins,
        src_vertex=src, src_rate=np.full(src.shape[0], total / src.shape[0]),
        src_dir=np.tile(np.array([1.0, 0.0, 0.0]), (src.shape[0], 1)),
        dt=t_end_myr * MYR_S / n_sweeps, n_sweeps=n_sweeps,
        precision=precision, box=box,
        meta=dict(seed=seed, box_kpc=box_kpc, n_H=n_H, contrast=contrast,
                  clump_r_kpc=clump_r_kpc, clump_c_kpc=tuple(clump_c_kpc),
                  flux=flux, spacing=spacing, t_end_myr=t_end_myr))


def batch_member(g: int, n_min: int = 4096, n_max: int = 262144,
                 n_bins: int = 42, n_sweeps: int = 200,
                 precision: int = SX_FP32_TRANSPORT,
                 n_override: Optional[int] = None) -> Workload:
    """Grid g of the 64-grid batch: N log-uniform in [n_min, n_max], n_H
    log-uniform in [1e-4, 1e-2], rate log-uniform in [1e47, 1e50]; the box is
    2.44 Stromgren radii (the ratio of Test 1) and the run spans 4
    recombination times."""
    rng = np.random.default_rng(4000 + g)
    n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
    if n_override is not None:
        n = n_override
    nh = 10 ** rng.uniform(-4, -2)
    rate = 10 ** rng.uniform(47, 50)
    r_s = (3 * rate / (4 * math.pi * ALPHA_B * nh * nh)) ** (1.0 / 3.0)
    t_rec = 1.0 / (ALPHA_B * nh)
    box = 2.44 * r_s
    pts = poisson_points(n, box, rng)
    ptr, idx, simp = delaunay(pts)
    vol = dual_volumes(pts, simp)
    src = nearest_vertex(pts, (box / 2, box / 2, box / 2))
    return Workload(
        name=f"batch{g}_n{n}", pos=pts, nbr_ptr=ptr, nbr_idx=idx,
        n_H=np.full(n, nh), volume=vol, bin_dirs=icosahedral_bins_42()
        if n_bins == 42 else random_bins(n_bins, 104),
        src_vertex=np.array([src], np.int32), src_rate=np.array([rate]),
        dt=4.0 * t_rec / n_sweeps, n_sweeps=n_sweeps, precision=precision,
        box=box, meta=dict(g=g, n_H=nh, rate=rate, r_s=r_s, t_rec=t_rec))


def chain_graph(n: int, spacing: float, n_H: float, volume: float,
                bins: Optional[np.ndarray] = None) -> Workload:
    """A straight 1-D chain of n vertices along +x (vertex i at x = i*spacing),
    each linked to its predecessor and successor; source at vertex 0."""
    pos = np.zeros((n, 3))
    pos[:, 0] = np.arange(n) * spacing
    rows = []
    for i in range(n):
        r = [j for j in (i - 1, i + 1) if 0 <= j < n]
        rows.append(r)
    ptr = np.zeros(n + 1, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in r], np.int32)
    return Workload(
        name=f"chain{n}", pos=pos, nbr_ptr=ptr, nbr_idx=idx,
        n_H=np.full(n, n_H), volume=np.full(n, volume),
        bin_dirs=axis_bins() if bins is None else bins,
        src_vertex=np.array([0], np.int32), src_rate=np.array([1e40]),
        dt=1e10, n_sweeps=n, box=n * spacing)


def lattice_graph(L: int, spacing: float = 1.0) -> Workload:
    """An L x L x L cubic lattice, vertex (ix, iy, iz) at index
    (ix * L + iy) * L + iz and position spacing * (ix, iy, iz), each linked
    to its (up to) six axis neighbours.  Six axis bins, one source at the
    centre; unit density and volume (callers override the physics)."""
    ids = np.arange(L ** 3).reshape(L, L, L)
    ix, iy, iz = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    pos = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], 1).astype(np.float64) * spacing
    rows = []
    for a, b, c in zip(ix.ravel(), iy.ravel(), iz.ravel()):
        r = []
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            p2 = (a + d[0], b + d[1], c + d[2])
            if all(0 <= q < L for q in p2):
                r.append(int(ids[p2]))
        rows.append(sorted(r))
    ptr = np.zeros(L ** 3 + 1, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in r], np.int32)
    n = L ** 3
    return Workload(
        name=f"lattice{L}", pos=pos, nbr_ptr=ptr, nbr_idx=idx,
        n_H=np.ones(n), volume=np.full(n, spacing ** 3), bin_dirs=axis_bins(),
        src_vertex=np.array([int(ids[L // 2, L // 2, L // 2])], np.int32),
        src_rate=np.array([1.0]), dt=1.0, n_sweeps=L, box=L * spacing)


def star_graph(spacing: float = 1.0) -> Workload:
    """A centre vertex with six neighbours on the +-x, +-y, +-z axes; the
    outer vertices are linked to the centre only.  Six axis bins."""
    pos = np.zeros((7, 3))
    pos[1:] = axis_bins() * spacing
    rows = [list(range(1, 7))] + [[0] for _ in range(6)]
    ptr = np.zeros(8, np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in r], np.int32)
    return Workload(
        name="star7", pos=pos, nbr_ptr=ptr, nbr_idx=idx,
        n_H=np.full(7, 1e-3), volume=np.full(7, spacing ** 3),
        bin_dirs=axis_bins(), src_vertex=np.array([0], np.int32),
        src_rate=np.array([1e40]), dt=1e10, n_sweeps=4, box=2 * spacing)


def small_random(n: int, seed: int, n_bins: int = 21, box: float = 1.0,
                 n_H: float = 1e-3, rate: float = 1e40, n_src: int = 2,
                 dt: float = 3.0e13, precision: int = SX_FP64) -> Workload:
    """A tiny Poisson grid in a unit-ish box for brute-force checks."""
    rng = np.random.default_rng(seed)
    pts = poisson_points(n, box, rng)
    ptr, idx, simp = delaunay(pts)
    vol = dual_volumes(pts, simp)
    src = rng.choice(n, size=n_src, replace=False).astype(np.int32)
    return Workload(
        name=f"small{n}_s{seed}", pos=pts, nbr_ptr=ptr, nbr_idx=idx,
        n_H=np.full(n, n_H), volume=vol,
        bin_dirs=random_bins(n_bins, seed + 7),
        src_vertex=src, src_rate=np.full(n_src, rate),
        dt=dt, n_sweeps=8, precision=precision, box=box)


def with_(w: Workload, **kw) -> Workload:
    """Shallow copy of a workload with some fields replaced."""
    d = dict(w.__dict__)
    d.update(kw)
    return Workload(**d)


# ---------------------------------------------------------------- serving
# Solve requests for the request loop: each request takes a grid from a
# pool built once (live triangulation of up to 2e6 points per request would
# take minutes), and draws its own sources, density field, bin set and
# sweep count.

def serve_pool_sizes(n_min: float = 1e4, n_max: float = 2e6, count: int = 8) -> list:
    """Pool grid sizes, log-spaced over [n_min, n_max]."""
    return [int(round(v)) for v in np.exp(np.linspace(math.log(n_min), math.log(n_max), count))]


def serve_pool_grid(i: int, n: int, box_kpc: float = 13.2) -> Workload:
    """Pool grid i: n Poisson points (seed 6000 + i) in the 13.2 kpc box,
    Delaunay graph and dual volumes; physics is filled in per request."""
    box = box_kpc * KPC_CM
    rng = np.random.default_rng(6000 + i)
    pts = poisson_points(n, box, rng)
    ptr, idx, simp = delaunay(pts)
    vol = dual_volumes(pts, simp)
    return Workload(
        name=f"pool{i}_n{n}", pos=pts, nbr_ptr=ptr, nbr_idx=idx,
        n_H=np.full(n, 1e-3), volume=vol, bin_dirs=icosahedral_bins_42(),
        src_vertex=np.zeros(1, np.int32), src_rate=np.ones(1),
        dt=MYR_S, n_sweeps=1, precision=SX_FP32_TRANSPORT, box=box,
        meta=dict(pool=i))


def serve_arrivals(rate_per_s: float, seconds: float, seed: int = 5) -> np.ndarray:
    """Poisson arrival times in [0, seconds)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= seconds:
            return np.array(out)
        out.append(t)


def serve_request(pool: list, r: int, n_min: float = 1e4, n_max: float = 2e6,
                  t_end_myr: float = 500.0) -> Workload:
    """Request r (seed 5,000,000 + r): N log-uniform in [n_min, n_max]
    (served by the pool grid nearest in log N), 1-32 point sources with rates
    log-uniform in [1e47, 1e50] s^-1, uniform n_H = 1e-3 cm^-3 or a 100x
    clump (a sphere of radius 0.1 box at a random centre), 42 or 84 bins,
    200-1000 sweeps over 500 Myr, FP32 transport."""
    rng = np.random.default_rng(5_000_000 + r)
    n_want = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
    g = min(pool, key=lambda w: abs(math.log(w.n) - math.log(n_want)))
    n_src = int(rng.integers(1, 33))
    src = rng.choice(g.n, size=n_src, replace=False).astype(np.int32)
    rates = 10.0 ** rng.uniform(47.0, 50.0, size=n_src)
    n_H = np.full(g.n, 1e-3)
    clump = bool(rng.integers(0, 2))
    if clump:
        c = rng.uniform(0.0, g.box, size=3)
        inside = np.sum((g.pos - c) ** 2, axis=1) < (0.1 * g.box) ** 2
        n_H[inside] *= 100.0
    k = 42 if rng.integers(0, 2) == 0 else 84
    bins = icosahedral_bins_42() if k == 42 else random_bins(84, 102)
    sweeps = int(rng.integers(200, 1001))
    return with_(g, name=f"req{r}_{g.name}_k{k}", n_H=n_H, bin_dirs=bins,
                 src_vertex=src, src_rate=rates, dt=t_end_myr * MYR_S / sweeps,
                 n_sweeps=sweeps, precision=SX_FP32_TRANSPORT,
                 meta=dict(request=r, pool=g.meta["pool"], n_want=n_want, clump=clump))


# --------------------------------------------------------------- rotations
# Random orientations of the direction bins (the method rotates them between
# steps against preferential directions).  They are inputs: the caller draws
# them and hands the same matrices to every implementation.

def random_rotations(n: int, seed: int) -> np.ndarray:
    """n rotation matrices [n, 3, 3], uniform on SO(3): normalised Gaussian
    quaternions (seed)."""
    q = np.random.default_rng(seed).normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1)[:, None]
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def quarter_turn_z() -> np.ndarray:
    """Rotation by 90 degrees about z (exact entries)."""
    return np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
