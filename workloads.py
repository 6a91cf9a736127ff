"""Seeded synthetic inputs shared by the HIP path's callers and the oracle.

This module holds geometry and random draws only: periodic simplicial meshes
(connectivity plus unwrapped vertex coordinates), the noisy initial density
psi_0 and the per-instance parameter draws.  It computes nothing of the
method itself (no integrals, no matrices, no solver steps), so both sides can
take their inputs from here without sharing arithmetic.

Workload shapes follow the paper's numerical studies (Section 7): periodic
regular simplicial meshes, a constant mean density psibar plus small noise, a
crystalline parameter regime (psibar^2 < -r/3, Lemma 3 and the remark after
it).  The grid spacing is h = (2*pi/sqrt(3))/8, i.e. eight points per half
lattice spacing d/2 with d = 4*pi/sqrt(3) (Section 7 uses d and h ~ d/10).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

# Lattice spacing of the single-mode approximation, d = 4*pi/sqrt(3) (Section 7).
LATTICE_D = 4.0 * math.pi / math.sqrt(3.0)
# Grid spacing used for every synthetic workload: 64 cells span 8 half-lattice
# spacings, L = 64*(2*pi/sqrt(3))/8.
H_DEFAULT = (2.0 * math.pi / math.sqrt(3.0)) / 8.0

# Stream tags so that jitter, noise and parameter draws never share a stream.
_TAG_JITTER = 1
_TAG_PSI = 2
_TAG_PARAMS = 3
_TAG_ARRIVALS = 4
_TAG_SMOOTH = 5


@dataclass
class Mesh:
    """A periodic simplicial mesh.

    dim          2 (triangles) or 3 (tetrahedra)
    n            number of (periodically identified) nodes
    elem_nodes   int32 [n_elem, dim+1] node indices of each simplex
    elem_coords  float64 [n_elem, dim+1, dim] unwrapped vertex coordinates, so
                 that each simplex is a proper simplex even where it crosses
                 the periodic boundary
    N            cells per direction, h the cell size, L = N*h the period
    degree       1: P1, elem_nodes holds the dim+1 vertices; 2: P2,
                 elem_nodes holds the dim+1 vertices and then one node per
                 edge, edges in the order of P2_EDGES[dim] (local vertex pairs)
    """

    dim: int
    n: int
    elem_nodes: np.ndarray
    elem_coords: np.ndarray
    N: int
    h: float
    degree: int = 1

    @property
    def n_elem(self) -> int:
        return int(self.elem_nodes.shape[0])

    @property
    def L(self) -> float:
        return self.N * self.h


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(tag)])


def periodic_mesh_2d(N: int, h: float = H_DEFAULT, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Periodic N x N square grid, each cell split along its (i,j)->(i+1,j+1) diagonal.

    Node (i, j) has index i + N*j.  With jitter > 0 every node coordinate is
    moved by an independent U[-jitter*h, +jitter*h] draw; connectivity stays
    fixed.  Both triangles of a cell are counter-clockwise.
    """
    if N < 2:
        raise ValueError("N must be >= 2")
    n = N * N
    disp = np.zeros((n, 2))
    if jitter > 0.0:
        disp = _rng(seed, _TAG_JITTER).uniform(-jitter * h, jitter * h, size=(n, 2))
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    i = i.ravel(order="F")
    j = j.ravel(order="F")  # cell (i, j) in node order: i fastest

    def vert(di, dj):
        ii, jj = i + di, j + dj
        node = (ii % N) + N * (jj % N)
        xy = np.stack([ii * h, jj * h], axis=1) + disp[node]
        return node, xy

    v00, x00 = vert(0, 0)
    v10, x10 = vert(1, 0)
    v11, x11 = vert(1, 1)
    v01, x01 = vert(0, 1)
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    c1 = np.stack([x00, x10, x11], axis=1)
    c2 = np.stack([x00, x11, x01], axis=1)
    # interleave the two triangles of each cell so element order follows cells
    nodes = np.empty((2 * n, 3), dtype=np.int32)
    nodes[0::2] = t1
    nodes[1::2] = t2
    coords = np.empty((2 * n, 3, 2))
    coords[0::2] = c1
    coords[1::2] = c2
    return Mesh(2, n, nodes, coords, N, h)


def periodic_mesh_3d(N: int, h: float = H_DEFAULT, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Periodic N^3 cube grid, each cube split into the 6 Kuhn (Freudenthal) tetrahedra.

    All six tetrahedra of a cube share its main diagonal (0,0,0)-(1,1,1); the
    split is identical in every cube, so the mesh is translation invariant.
    Node (i, j, k) has index i + N*(j + N*k).
    """
    if N < 2:
        raise ValueError("N must be >= 2")
    n = N ** 3
    disp = np.zeros((n, 3))
    if jitter > 0.0:
        disp = _rng(seed, _TAG_JITTER).uniform(-jitter * h, jitter * h, size=(n, 3))
    idx = np.arange(n)
    ci = idx % N
    cj = (idx // N) % N
    ck = idx // (N * N)
    base = np.stack([ci, cj, ck], axis=1)
    eye = np.eye(3, dtype=np.int64)
    tets_nodes = []
    tets_coords = []
    for perm in itertools.permutations(range(3)):
        offs = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for ax in perm:
            cur = cur + eye[ax]
            offs.append(cur.copy())
        vn = []
        vc = []
        for o in offs:
            p = base + o
            node = (p[:, 0] % N) + N * ((p[:, 1] % N) + N * (p[:, 2] % N))
            vn.append(node)
            vc.append(p * h + disp[node])
        tets_nodes.append(np.stack(vn, axis=1))
        tets_coords.append(np.stack(vc, axis=1))
    nodes = np.stack(tets_nodes, axis=1).reshape(6 * n, 4).astype(np.int32)
    coords = np.stack(tets_coords, axis=1).reshape(6 * n, 4, 3)
    return Mesh(3, n, nodes, coords, N, h)


# Local edges of a simplex in the node order of a P2 element (pairs of local vertices).
P2_EDGES = {2: ((0, 1), (1, 2), (0, 2)),
            3: ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))}


def p2_mesh(mesh: Mesh) -> Mesh:
    """The P2 version of a periodic P1 mesh: one extra node per edge.

    Vertex nodes keep their indices 0..n-1; edge nodes follow, numbered in the
    lexicographic order of their (smaller, larger) vertex index pair.  Needs
    N >= 3, so that distinct edges join distinct vertex pairs.
    """
    if mesh.N < 3:
        raise ValueError("P2 meshes need N >= 3")
    ev = mesh.elem_nodes.astype(np.int64)
    pairs = np.stack([np.stack([ev[:, i], ev[:, j]], axis=1) for i, j in P2_EDGES[mesh.dim]], axis=1)  # [E, ne, 2]
    lo = pairs.min(axis=2)
    hi = pairs.max(axis=2)
    key = lo * mesh.n + hi
    uniq, inv = np.unique(key.reshape(-1), return_inverse=True)
    edge_nodes = (mesh.n + inv).reshape(key.shape)
    nodes = np.concatenate([ev, edge_nodes], axis=1).astype(np.int32)
    return Mesh(mesh.dim, mesh.n + len(uniq), nodes, mesh.elem_coords, mesh.N, mesh.h, degree=2)


def make_mesh(dim: int, N: int, h: float = H_DEFAULT, jitter: float = 0.0, seed: int = 0) -> Mesh:
    if dim == 2:
        return periodic_mesh_2d(N, h, jitter, seed)
    if dim == 3:
        return periodic_mesh_3d(N, h, jitter, seed)
    raise ValueError("dim must be 2 or 3")


def psi0(n: int, psibar: float, amplitude: float = 0.01, seed: int = 0) -> np.ndarray:
    """Noisy constant initial density: psi_0 = psibar + U[-A, A] per node (not re-centred)."""
    return psibar + _rng(seed, _TAG_PSI).uniform(-amplitude, amplitude, size=n)


def node_coords(mesh: Mesh) -> np.ndarray:
    """Coordinates of every node in [0, L)^dim (from the unwrapped element vertices)."""
    out = np.zeros((mesh.n, mesh.dim))
    xy = mesh.elem_coords
    if mesh.degree == 2:  # edge nodes sit at the edge midpoints
        mids = [0.5 * (xy[:, i] + xy[:, j]) for i, j in P2_EDGES[mesh.dim]]
        xy = np.concatenate([xy, np.stack(mids, axis=1)], axis=1)
    flat_nodes = mesh.elem_nodes.reshape(-1)
    flat_xy = xy.reshape(-1, mesh.dim)
    first = np.unique(flat_nodes, return_index=True)[1]
    out[flat_nodes[first]] = flat_xy[first]
    return np.mod(out, mesh.L)


def psi_smooth(mesh: Mesh, psibar: float, amplitude: float = 0.2, kmax: int = 2, seed: int = 0) -> np.ndarray:
    """psibar plus a band-limited periodic perturbation.

    Random-phase cosines of the integer wave vectors m with max |m_i| <= kmax
    (wavelengths >= L/kmax), seeded, scaled so that the largest deviation from
    psibar is `amplitude`.  A smooth state with moderate gradients, for the
    terms that grow with the gradient of mu (the PFC1 mobility derivative).
    """
    x = node_coords(mesh)
    rng = _rng(seed, _TAG_SMOOTH)
    f = np.zeros(mesh.n)
    for m in itertools.product(range(-kmax, kmax + 1), repeat=mesh.dim):
        if not any(m):
            continue
        phase = rng.uniform(0.0, 2.0 * math.pi)
        weight = rng.uniform(0.5, 1.0)
        f += weight * np.cos(2.0 * math.pi * (x @ np.asarray(m, dtype=np.float64)) / mesh.L + phase)
    return psibar + amplitude * f / np.abs(f).max()


@dataclass
class Params:
    r: float
    psibar: float
    tau: float
    seed: int


def draw_params(count: int, base_seed: int) -> list[Params]:
    """Per-instance parameters of the batched and served workloads.

    psibar ~ U[-0.4, -0.2], r ~ U[-0.4, -0.25], tau ~ U[0.05, 1.0], seed = base + i.
    """
    out = []
    for i in range(count):
        g = _rng(base_seed + i, _TAG_PARAMS)
        psibar = g.uniform(-0.4, -0.2)
        r = g.uniform(-0.4, -0.25)
        tau = g.uniform(0.05, 1.0)
        out.append(Params(float(r), float(psibar), float(tau), base_seed + i))
    return out


# Mesh classes of the served stream: (dim, N).
SERVED_CLASSES = [(2, 64), (2, 128), (2, 256), (2, 512), (3, 32), (3, 48)]


def served_stream(n_req: int, rate_hz: float, base_seed: int, classes=SERVED_CLASSES):
    """Poisson arrivals of solve requests.

    Returns a list of (arrival_time_s, class_index, Params) sorted by time.
    Mesh class is uniform over `classes`; parameters as in draw_params.
    """
    g = _rng(base_seed, _TAG_ARRIVALS)
    gaps = g.exponential(1.0 / rate_hz, size=n_req) if rate_hz > 0 else np.zeros(n_req)
    t = np.cumsum(gaps) - gaps[0]
    cls = g.integers(0, len(classes), size=n_req)
    prm = draw_params(n_req, base_seed + 1000)
    return [(float(t[i]), int(cls[i]), prm[i]) for i in range(n_req)]
