"""Seeded synthetic grids for the edge-based metric build.

This module only lays out node coordinates and element connectivity (and the
random loss weights the adjoint tests draw).  It holds none of the metric
arithmetic: no face normals, no volumes, no edge extraction.  Both the CPU
oracle's tests and the GPU path's tests and benchmark take their inputs from
here, so that the two sides never exchange data.

The grids stand in for the paper's unit-square triangle grid and unit-cube
tetrahedral grid (Section 5, the paragraph before Table 3): only their node and
element counts are printed, so the split patterns, jitter and stretching below
are this module's own recipe.

Conventions
-----------
* coordinates: float64, structure of arrays, shape ``[D, Nv]``
* connectivity: int32, shape ``[NE, D+1]``; local vertex order is whatever the
  split produces (both orientations occur on purpose).
* node ids: ``i + n*j (+ n*n*k)`` for a structured ``n^D`` grid.

Random streams: ``numpy.random.Generator(PCG64(SeedSequence(seed)))``; child
streams are spawned in a fixed order (jitter, diagonals, batched sizes,
per-mesh jitter, loss weights, finite-difference nodes) so that adding a draw
to one stream never shifts another.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np

__all__ = [
    "Mesh", "BatchedMesh", "streams", "square_tri", "cube_kuhn", "scale_cube",
    "batched_kuhn", "loss_weights", "fd_nodes", "make", "CONFIGS",
    "kuhn_counts", "tri_counts", "hypercube_kuhn", "kuhn4_counts",
]

_STREAM_NAMES = ("jitter", "diag", "sizes", "permesh", "loss", "fd")


def streams(seed: int) -> dict:
    """Spawn the named child generators for ``seed`` (fixed order)."""
    ss = np.random.SeedSequence(int(seed))
    kids = ss.spawn(len(_STREAM_NAMES))
    return {name: kid for name, kid in zip(_STREAM_NAMES, kids)}


def _gen(seq: np.random.SeedSequence) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seq))


@dataclass
class Mesh:
    dim: int
    coords: np.ndarray          # [D, Nv] float64
    elems: np.ndarray           # [NE, D+1] int32
    name: str = ""
    domain_volume: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[1])

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])


@dataclass
class BatchedMesh(Mesh):
    node_off: np.ndarray = None  # [M+1] int64
    elem_off: np.ndarray = None  # [M+1] int64
    sizes: np.ndarray = None     # [M] nodes per axis of each mesh


# --------------------------------------------------------------------------
# closed-form counts of the structured grids (used to size loss weights)
# --------------------------------------------------------------------------

def tri_counts(n: int) -> dict:
    """Counts of an n x n node grid split into 2 triangles per cell."""
    c = n - 1
    return dict(n_nodes=n * n, n_elems=2 * c * c,
                n_edges=2 * n * c + c * c, n_bfaces=4 * c, n_bnodes=4 * c)


def kuhn_counts(n: int) -> dict:
    """Counts of an n^3 node grid with the 6-tet Kuhn split of every cell."""
    c = n - 1
    return dict(n_nodes=n ** 3, n_elems=6 * c ** 3,
                n_edges=3 * n * n * c + 3 * n * c * c + c ** 3,
                n_bfaces=12 * c * c, n_bnodes=n ** 3 - max(n - 2, 0) ** 3)


# --------------------------------------------------------------------------
# 2D: unit square, 2 triangles per cell, diagonal by coin flip
# --------------------------------------------------------------------------

def _interior_mask_2d(n: int) -> np.ndarray:
    i = np.arange(n)
    ii, jj = np.meshgrid(i, i, indexing="xy")  # ii varies fastest along x
    m = (ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1)
    return m.reshape(-1)


def square_tri(n: int = 33, seed: int = 0, jitter: float = 0.2,
               flip: bool = True) -> Mesh:
    """Unit square, ``n x n`` nodes, each cell split by a seeded diagonal.

    Interior nodes move by U(-jitter*h, jitter*h) per axis; boundary nodes stay,
    so the domain stays the unit square.  Cell (i, j) with corners a=(i,j),
    b=(i+1,j), c=(i,j+1), d=(i+1,j+1) becomes (a,b,d),(a,d,c) when its coin is
    0 and (a,b,c),(b,d,c) when it is 1 (``flip=False`` keeps every coin 0).
    """
    st = streams(seed)
    h = 1.0 / (n - 1)
    i = np.arange(n, dtype=np.float64)
    X, Y = np.meshgrid(i * h, i * h, indexing="xy")
    coords = np.stack([X.reshape(-1), Y.reshape(-1)]).astype(np.float64)
    if jitter:
        r = _gen(st["jitter"]).uniform(-jitter * h, jitter * h,
                                       size=(n * n, 2))
        mask = _interior_mask_2d(n)
        coords[:, mask] += r[mask].T
    c = n - 1
    ci, cj = np.meshgrid(np.arange(c), np.arange(c), indexing="xy")
    ci = ci.reshape(-1)
    cj = cj.reshape(-1)
    a = ci + n * cj
    b = a + 1
    cc = a + n
    d = a + n + 1
    coin = (_gen(st["diag"]).integers(0, 2, size=c * c) if flip
            else np.zeros(c * c, dtype=np.int64))
    t0 = np.where(coin[:, None] == 0, np.stack([a, b, d], 1),
                  np.stack([a, b, cc], 1))
    t1 = np.where(coin[:, None] == 0, np.stack([a, d, cc], 1),
                  np.stack([b, d, cc], 1))
    elems = np.empty((2 * c * c, 3), dtype=np.int32)
    elems[0::2] = t0
    elems[1::2] = t1
    return Mesh(2, np.ascontiguousarray(coords), elems, name=f"square{n}",
                meta=dict(n=n, seed=seed, jitter=jitter))


# --------------------------------------------------------------------------
# 3D: unit cube, 6 tets per cell (Kuhn / Freudenthal split)
# --------------------------------------------------------------------------

_KUHN_PERMS = list(permutations(range(3)))  # lexicographic order


def _kuhn_elems(n: int, node_base: int = 0) -> np.ndarray:
    c = n - 1
    cell = np.arange(c, dtype=np.int64)
    c0 = (cell[None, None, :] + n * cell[None, :, None]
          + n * n * cell[:, None, None]).reshape(-1) + node_base
    step = np.array([1, n, n * n], dtype=np.int64)
    offs = np.empty((6, 4), dtype=np.int64)
    for t, (pa, pb, _) in enumerate(_KUHN_PERMS):
        offs[t] = (0, step[pa], step[pa] + step[pb], step.sum())
    if c0.size and c0[-1] + offs.max() >= 2 ** 31:
        raise OverflowError("node ids exceed int32")
    out = c0.astype(np.int32)[:, None, None] + offs.astype(np.int32)[None]
    return out.reshape(-1, 4)


def _axis_nodes_uniform(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) / (n - 1)


def _cube_coords(xs, ys, zs) -> np.ndarray:
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)])


def _interior_mask_3d(n: int) -> np.ndarray:
    a = np.arange(n)
    k, j, i = np.meshgrid(a, a, a, indexing="ij")
    m = ((i > 0) & (i < n - 1) & (j > 0) & (j < n - 1)
         & (k > 0) & (k < n - 1))
    return m.reshape(-1)


def cube_kuhn(n: int = 41, seed: int = 0, jitter: float = 0.15,
              jitter_stream: np.random.SeedSequence | None = None,
              node_base: int = 0) -> Mesh:
    """Unit cube, ``n^3`` nodes, Kuhn split, interior jitter +-jitter*h."""
    h = 1.0 / (n - 1)
    xs = _axis_nodes_uniform(n)
    coords = _cube_coords(xs, xs, xs)
    if jitter:
        seq = jitter_stream if jitter_stream is not None else streams(seed)["jitter"]
        r = _gen(seq).uniform(-jitter * h, jitter * h, size=(n ** 3, 3))
        mask = _interior_mask_3d(n)
        coords[:, mask] += r[mask].T
    elems = _kuhn_elems(n, node_base)
    return Mesh(3, np.ascontiguousarray(coords), elems, name=f"kuhn{n}",
                meta=dict(n=n, seed=seed, jitter=jitter))


def stretched_z(n: int = 161, first: float = 1e-5, ratio: float = 1.15):
    """Node z-positions: geometric spacing from z=0, then uniform to z=1.

    Spacings are ``first*ratio**i`` for ``i < m`` and then a uniform spacing
    ``delta = (1 - S_m)/(n-1-m)``; ``m`` is the smallest count for which the
    next geometric spacing would reach ``delta``.
    """
    cells = n - 1
    for m in range(1, cells):
        geo = first * ratio ** np.arange(m)
        s_m = geo.sum()
        delta = (1.0 - s_m) / (cells - m)
        if first * ratio ** m >= delta:
            break
    else:  # pragma: no cover - impossible for the configs used
        raise ValueError("stretching never reaches the uniform spacing")
    steps = np.concatenate([geo, np.full(cells - m, delta)])
    z = np.concatenate([[0.0], np.cumsum(steps)])
    z[-1] = 1.0
    return z, m, delta


def scale_cube(n: int = 161, seed: int = 0, jitter: float = 0.1,
               first: float = 1e-5, ratio: float = 1.15) -> Mesh:
    """Unit cube with one-wall z stretching and interior jitter +-0.1 local h.

    x and y are uniform with spacing h; the local z spacing of node layer k is
    min(z_k - z_{k-1}, z_{k+1} - z_k).
    """
    h = 1.0 / (n - 1)
    xs = _axis_nodes_uniform(n)
    zs, m, delta = stretched_z(n, first, ratio)
    coords = _cube_coords(xs, xs, zs)
    if jitter:
        r = _gen(streams(seed)["jitter"]).uniform(-1.0, 1.0, size=(n ** 3, 3))
        dz = np.diff(zs)
        hz = np.empty(n)
        hz[1:-1] = np.minimum(dz[:-1], dz[1:])
        hz[0] = dz[0]
        hz[-1] = dz[-1]
        hz_node = np.repeat(hz, n * n)
        mask = _interior_mask_3d(n)
        coords[0, mask] += jitter * h * r[mask, 0]
        coords[1, mask] += jitter * h * r[mask, 1]
        coords[2, mask] += jitter * hz_node[mask] * r[mask, 2]
    elems = _kuhn_elems(n)
    return Mesh(3, np.ascontiguousarray(coords), elems, name=f"scale{n}",
                meta=dict(n=n, seed=seed, jitter=jitter, m_geo=m,
                          delta=delta))


def batched_kuhn(n_mesh: int = 64, seed: int = 0, lo: int = 9, hi: int = 65,
                 jitter: float = 0.15) -> BatchedMesh:
    """``n_mesh`` independent Kuhn cubes of log-uniform size, concatenated.

    Mesh m has ``n_m^3`` nodes with n_m = clamp(round(exp(U(ln lo, ln hi)))),
    its own jitter stream, and node ids offset by the nodes of meshes before it
    (the batch is one disconnected grid).
    """
    st = streams(seed)
    u = _gen(st["sizes"]).uniform(np.log(lo), np.log(hi), size=n_mesh)
    sizes = np.clip(np.rint(np.exp(u)).astype(np.int64), lo, hi)
    kids = st["permesh"].spawn(n_mesh)
    coords, elems = [], []
    node_off = [0]
    elem_off = [0]
    for m in range(n_mesh):
        mesh = cube_kuhn(int(sizes[m]), jitter=jitter, jitter_stream=kids[m],
                         node_base=node_off[-1])
        coords.append(mesh.coords)
        elems.append(mesh.elems)
        node_off.append(node_off[-1] + mesh.n_nodes)
        elem_off.append(elem_off[-1] + mesh.n_elems)
    return BatchedMesh(3, np.ascontiguousarray(np.concatenate(coords, 1)),
                       np.ascontiguousarray(np.concatenate(elems, 0)),
                       name=f"batched{n_mesh}", domain_volume=float(n_mesh),
                       meta=dict(seed=seed, n_mesh=n_mesh),
                       node_off=np.array(node_off, dtype=np.int64),
                       elem_off=np.array(elem_off, dtype=np.int64),
                       sizes=sizes)


# --------------------------------------------------------------------------
# four dimensions: the Kuhn split of a 4-cube into 24 pentatopes
# --------------------------------------------------------------------------

_KUHN4_PERMS = list(permutations(range(4)))  # lexicographic order


def kuhn4_counts(n: int) -> dict:
    """Counts of an n^4 node grid with the 24-pentatope Kuhn split of every
    cell: edges run from a node to each of the 15 nonempty corner offsets of
    its cell, (2n-1)^4 - n^4 in all; the boundary is 8 cubic facets of
    (n-1)^3 cells, 6 tetrahedra each."""
    c = n - 1
    return dict(n_nodes=n ** 4, n_elems=24 * c ** 4, n_edges=(2 * n - 1) ** 4 - n ** 4,
                n_bfaces=48 * c ** 3, n_bnodes=n ** 4 - max(n - 2, 0) ** 4)


def _kuhn4_elems(n: int) -> np.ndarray:
    c = n - 1
    cell = np.arange(c, dtype=np.int64)
    c0 = (cell[None, None, None, :] + n * cell[None, None, :, None]
          + n * n * cell[None, :, None, None] + n ** 3 * cell[:, None, None, None]).reshape(-1)
    step = np.array([1, n, n * n, n ** 3], dtype=np.int64)
    offs = np.empty((24, 5), dtype=np.int64)
    for t, (pa, pb, pc, _) in enumerate(_KUHN4_PERMS):
        offs[t] = (0, step[pa], step[pa] + step[pb], step[pa] + step[pb] + step[pc], step.sum())
    if c0.size and c0[-1] + offs.max() >= 2 ** 31:
        raise OverflowError("node ids exceed int32")
    out = c0.astype(np.int32)[:, None, None] + offs.astype(np.int32)[None]
    return out.reshape(-1, 5)


def hypercube_kuhn(n: int = 9, seed: int = 0, jitter: float = 0.1) -> Mesh:
    """Unit 4-cube, ``n^4`` nodes (id = i + n j + n^2 k + n^3 l), each cell
    split along its main diagonal into the 24 pentatopes (c0, c0+e_a,
    c0+e_a+e_b, c0+e_a+e_b+e_c, c0+(1,1,1,1)) over the permutations (a,b,c,d)
    of the axes (odd ones have negative signed measure), interior nodes
    jittered uniformly +-jitter*h per axis.  With jitter 0.1 a node moves at
    most 0.2h, and two at most 0.4h closer, below the smallest height h/sqrt 2
    of the split's pentatopes, so none is inverted."""
    h = 1.0 / (n - 1)
    xs = _axis_nodes_uniform(n)
    L, K, J, I = np.meshgrid(xs, xs, xs, xs, indexing="ij")
    coords = np.stack([I.reshape(-1), J.reshape(-1), K.reshape(-1), L.reshape(-1)])
    if jitter:
        r = _gen(streams(seed)["jitter"]).uniform(-jitter * h, jitter * h, size=(n ** 4, 4))
        a = np.arange(n)
        l, k, j, i = np.meshgrid(a, a, a, a, indexing="ij")
        inner = ((i > 0) & (i < n - 1) & (j > 0) & (j < n - 1) & (k > 0) & (k < n - 1)
                 & (l > 0) & (l < n - 1)).reshape(-1)
        coords[:, inner] += r[inner].T
    return Mesh(4, np.ascontiguousarray(coords), _kuhn4_elems(n), name=f"kuhn4d{n}",
                meta=dict(n=n, seed=seed, jitter=jitter))


# --------------------------------------------------------------------------
# adjoint inputs
# --------------------------------------------------------------------------

def loss_weights(seed: int, dim: int, n_edges: int, n_nodes: int,
                 n_bnodes: int = 0):
    """w_e ~ N(0,1)^D as [D, Ne]; c_j ~ U(0,1) as [Nv]; beta ~ N(0,1)^D."""
    g = _gen(streams(seed)["loss"])
    w = g.standard_normal(size=(dim, n_edges))
    c = g.uniform(0.0, 1.0, size=n_nodes)
    beta = g.standard_normal(size=(dim, n_bnodes)) if n_bnodes else None
    return w, c, beta


def fd_nodes(seed: int, n_nodes: int, count: int = 64) -> np.ndarray:
    return np.sort(_gen(streams(seed)["fd"]).choice(n_nodes, count,
                                                    replace=False))


# --------------------------------------------------------------------------
# named configurations
# --------------------------------------------------------------------------

CONFIGS = {
    "2d": lambda seed=0: square_tri(33, seed),
    "3d": lambda seed=0: cube_kuhn(41, seed),
    "3d-scale": lambda seed=0: scale_cube(161, seed),
    "3d-adjoint": lambda seed=0: cube_kuhn(81, seed),
    "batched": lambda seed=0: batched_kuhn(64, seed),
    "4d": lambda seed=0: hypercube_kuhn(9, seed),
}


def make(config: str, seed: int = 0) -> Mesh:
    return CONFIGS[config](seed)
