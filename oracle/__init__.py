"""CPU oracle for the edge-based grid metrics — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this package.  It computes the lumped directed-area vectors,
boundary dual-face normals and median-dual volumes by the traditional route
(median dual formed element by element: edge midpoints, face and element
centroids; Sections 3.1 and 4 of the paper) in FP64 with compensated sums, and
builds its own topology with ``std::sort``.  See ``oracle.cpp`` for the full
statement.  It shares no code with the GPU library.

Functions
---------
``topology(dim, coords, elems)``        -> dict of int arrays: the edge array,
                                          element->edge map, incidence CSRs and
                                          boundary elements, each uniquely
                                          defined (the GPU must match them bit
                                          for bit)
``metrics(topo, coords, elems)``        -> (n [D,Ne], b [D,Nbn], V [Nv])
``element_pieces(dim, coords, elems)``  -> per-element dual pieces
``bface_piece(dim, coords, face, opp)`` -> per-vertex boundary pieces
``node_grad(topo, coords, elems, w, c, beta, nodes)`` -> (L_j, dL/dx_j)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

STATUS = {0: "ok", -1: "invalid argument", -2: "node id out of range",
          -3: "degenerate element", -4: "non-manifold face",
          -6: "size overflow"}

TOPO_ARRAYS = ("edge", "node_edge_off", "elem_edge", "elem_edge_sign",
               "edge_inc_off", "edge_inc", "node_inc_off", "node_inc",
               "node_in_off", "node_in_edge", "bface", "bface_owner",
               "bface_edge", "bnode", "node_bnode", "bnode_face_off",
               "bnode_face")


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"oracle {what}: {STATUS.get(code, code)} ({code})")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int
        L.oracle_topo_new.restype = P
        L.oracle_topo_free.argtypes = [P]
        L.oracle_topology.argtypes = [P, i32, i64, i64, P, P]
        L.oracle_topo_sizes.argtypes = [P, P]
        L.oracle_topo_get.argtypes = [P, ctypes.c_char_p, P]
        L.oracle_topo_get.restype = i64
        L.oracle_metrics.argtypes = [P, P, P, P, P, P]
        L.oracle_element_pieces.argtypes = [i32, i64, P, i64, i64, P, P, P]
        L.oracle_bface_piece.argtypes = [i32, i64, P, P, ctypes.c_int32, P]
        L.oracle_node_grad.argtypes = [P, P, P, P, P, P, P, i64, P, P]
        L.oracle_num_threads.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


class Topology:
    """Oracle-side topology: owns the native handle plus numpy copies."""

    def __init__(self, dim, coords, elems):
        L = lib()
        coords = _f64(coords)
        elems = _i32(elems)
        self.dim = int(dim)
        self._h = L.oracle_topo_new()
        rc = L.oracle_topology(self._h, self.dim, coords.shape[1],
                               elems.shape[0], _ptr(elems), _ptr(coords))
        if rc != 0:
            L.oracle_topo_free(self._h)
            self._h = None
            raise OracleError(rc, "topology")
        s = np.zeros(6, dtype=np.int64)
        L.oracle_topo_sizes(self._h, _ptr(s))
        (_, self.n_nodes, self.n_elems, self.n_edges, self.n_bfaces,
         self.n_bnodes) = (int(x) for x in s)
        self.arrays = {}
        for name in TOPO_ARRAYS:
            cnt = L.oracle_topo_get(self._h, name.encode(), None)
            dt = np.int8 if name == "elem_edge_sign" else np.int32
            a = np.empty(cnt, dtype=dt)
            L.oracle_topo_get(self._h, name.encode(), _ptr(a))
            self.arrays[name] = a
        ne = self.dim * (self.dim + 1) // 2
        a = self.arrays
        a["edge"] = a["edge"].reshape(2, self.n_edges)
        a["elem_edge"] = a["elem_edge"].reshape(self.n_elems, ne)
        a["elem_edge_sign"] = a["elem_edge_sign"].reshape(self.n_elems, ne)
        a["bface"] = a["bface"].reshape(self.n_bfaces, self.dim)
        nbe = self.dim * (self.dim - 1) // 2
        a["bface_edge"] = a["bface_edge"].reshape(self.n_bfaces, nbe)

    def __getitem__(self, k):
        return self.arrays[k]

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.oracle_topo_free(self._h)
            self._h = None


def topology(dim, coords, elems) -> Topology:
    return Topology(dim, coords, elems)


def metrics(topo: Topology, coords, elems, want_b=True, want_v=True):
    """(n [D,Ne], b [D,Nbn] | None, V [Nv] | None) by the traditional route."""
    coords = _f64(coords)
    elems = _i32(elems)
    D = topo.dim
    n = np.empty((D, topo.n_edges))
    b = np.empty((D, topo.n_bnodes)) if want_b else None
    V = np.empty(topo.n_nodes) if want_v else None
    rc = lib().oracle_metrics(topo._h, _ptr(coords), _ptr(elems), _ptr(n),
                              _ptr(b), _ptr(V))
    if rc != 0:
        raise OracleError(rc, "metrics")
    return n, b, V


def element_pieces(dim, coords, elems, e0=0, e1=None):
    """Traditional per-element pieces for elements [e0, e1).

    Returns npiece [NE, ne, D] (dual-face area vector of each local edge,
    oriented from the smaller to the larger global id) and vpiece [NE, D+1]
    (sub-cell volume of each local vertex).
    """
    coords = _f64(coords)
    elems = _i32(elems)
    e1 = elems.shape[0] if e1 is None else e1
    ne = dim * (dim + 1) // 2
    npc = np.empty((e1 - e0, ne, dim))
    vpc = np.empty((e1 - e0, dim + 1))
    rc = lib().oracle_element_pieces(dim, coords.shape[1], _ptr(coords), e0,
                                     e1, _ptr(elems), _ptr(npc), _ptr(vpc))
    if rc != 0:
        raise OracleError(rc, "element_pieces")
    return npc, vpc


def bface_piece(dim, coords, face, opp):
    """Outward boundary dual pieces [D(vertex), D] of one boundary face."""
    coords = _f64(coords)
    face = _i32(face)
    out = np.empty((dim, dim))
    rc = lib().oracle_bface_piece(dim, coords.shape[1], _ptr(coords),
                                  _ptr(face), int(opp), _ptr(out))
    if rc != 0:
        raise OracleError(rc, "bface_piece")
    return out


def node_grad(topo: Topology, coords, elems, w=None, c=None, beta=None,
              nodes=None):
    """Per-node patch loss L_j and exact dL/dx_j (forward-mode dual numbers).

    L = sum_e w_e.n_e + sum_i c_i V_i + sum_i beta_i.b_i restricted to the
    terms that depend on x_j.  ``w`` is [D, Ne], ``c`` [Nv], ``beta`` [D, Nbn].
    """
    coords = _f64(coords)
    elems = _i32(elems)
    nodes = _i32(np.arange(topo.n_nodes) if nodes is None else nodes)
    loss = np.empty(nodes.size)
    g = np.empty((nodes.size, topo.dim))
    rc = lib().oracle_node_grad(topo._h, _ptr(coords), _ptr(elems),
                                _ptr(_f64(w)), _ptr(_f64(c)), _ptr(_f64(beta)),
                                _ptr(nodes), nodes.size, _ptr(loss), _ptr(g))
    if rc != 0:
        raise OracleError(rc, "node_grad")
    return loss, g
