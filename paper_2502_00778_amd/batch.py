"""Batches of grids, the fused forward + adjoint, graphs and the launch-shape
tuner (the ``eb_batch_*``, ``eb_graph_*`` and ``eb_autotune`` calls of
``include/eb.h``; argument marshalling only).

A batch is one grid whose meshes are concatenated with offset node ids
(:func:`concat_host` assembles one from per-mesh host arrays).  Everything in
:mod:`.api` works on it unchanged; :func:`batch_offsets` gives each mesh's
range of edges, boundary nodes and boundary faces, and :meth:`Batch.split`
cuts any output into per-mesh views.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import api
from ._lib import EbTuning, check, lib

__all__ = ["concat_host", "Batch", "batch_offsets", "forward_backward", "ForwardBackwardGraph",
           "set_fused_shape", "get_fused_shape", "set_fused_mode", "get_fused_mode",
           "set_fused_wait_limit", "autotune"]

FUSED_MODE = {"persistent": 0, "separate": 1, "persistent_atomic": 2, "separate_atomic": 3}


def concat_host(meshes):
    """Concatenate per-mesh host arrays ``[(coords [D, n_m], elems [E_m, D+1]), ...]``
    into one grid: returns ``(coords, elems, node_off, elem_off)`` (numpy)."""
    if not meshes:
        raise ValueError("no meshes")
    dim = int(np.asarray(meshes[0][0]).shape[0])
    node_off = [0]
    elem_off = [0]
    for X, E in meshes:
        X, E = np.asarray(X), np.asarray(E)
        if X.shape[0] != dim or E.shape[1] != dim + 1:
            raise ValueError("all meshes must have the same dimension")
        node_off.append(node_off[-1] + X.shape[1])
        elem_off.append(elem_off[-1] + E.shape[0])
    if node_off[-1] >= 2 ** 31:
        raise ValueError("too many nodes for int32 ids")
    coords = np.concatenate([np.asarray(X, np.float64) for X, _ in meshes], axis=1)
    elems = np.concatenate([np.asarray(E, np.int64) + o for (_, E), o in
                            zip(meshes, node_off[:-1])]).astype(np.int32)
    return (np.ascontiguousarray(coords), np.ascontiguousarray(elems),
            np.array(node_off, np.int64), np.array(elem_off, np.int64))


@dataclass
class Batch:
    """Per-mesh ranges of a batch (numpy int64 arrays of n_mesh+1 offsets)."""
    node_off: np.ndarray
    elem_off: np.ndarray
    edge_off: np.ndarray
    bnode_off: np.ndarray
    bface_off: np.ndarray

    @property
    def n_mesh(self):
        return len(self.node_off) - 1

    def split(self, t: torch.Tensor, kind: str):
        """Per-mesh views of an output: kind is 'edge' (n, grad_n: [D, Ne]),
        'node' (V, grad_x: [..., Nv]), 'bnode' (b) or 'bface' (bface rows)."""
        off = {"edge": self.edge_off, "node": self.node_off, "bnode": self.bnode_off,
               "bface": self.bface_off, "elem": self.elem_off}[kind]
        if kind in ("bface", "elem"):
            return [t[int(a):int(b)] for a, b in zip(off[:-1], off[1:])]
        return [t[..., int(a):int(b)] for a, b in zip(off[:-1], off[1:])]


def batch_offsets(topo: api.Topology, elems: torch.Tensor, node_off, elem_off,
                  stream=None) -> Batch:
    """eb_batch_offsets: per-mesh edge / boundary-node / boundary-face ranges;
    raises if an element references another mesh's nodes."""
    node_off = np.ascontiguousarray(node_off, dtype=np.int64)
    elem_off = np.ascontiguousarray(elem_off, dtype=np.int64)
    n_mesh = node_off.size - 1
    if elem_off.size != n_mesh + 1 or n_mesh < 1:
        raise ValueError("node_off and elem_off must both hold n_mesh+1 offsets")
    outs = [np.empty(n_mesh + 1, np.int64) for _ in range(3)]
    P = ctypes.POINTER(ctypes.c_int64)
    check(lib().eb_batch_offsets(ctypes.byref(topo.sizes), ctypes.byref(topo.struct),
                                 api._ptr(elems), n_mesh, node_off.ctypes.data_as(P),
                                 elem_off.ctypes.data_as(P), *(o.ctypes.data_as(P) for o in outs),
                                 api._ptr(topo.ws), topo.ws.numel(), api._stream_ptr(stream)),
          "eb_batch_offsets")
    return Batch(node_off, elem_off, *outs)


def _fb_args(coords, topo, elems, grad_n, grad_b, grad_vol, out):
    D = topo.dim
    api._need(coords, "coords", torch.float64, (D, topo.n_nodes))
    api._need(elems, "elems", torch.int32, (topo.n_elems, D + 1))
    if grad_n is not None:
        api._need(grad_n, "grad_n", torch.float64, (D, topo.n_edges))
    if grad_b is not None:
        api._need(grad_b, "grad_b", torch.float64, (D, topo.n_bnodes))
    if grad_vol is not None:
        api._need(grad_vol, "grad_vol", torch.float64, (topo.n_nodes,))
    out = out or {}
    n = api._out((D, topo.n_edges), coords, out.get("n"))
    b = api._out((D, topo.n_bnodes), coords, out.get("b"))
    V = api._out((topo.n_nodes,), coords, out.get("V"))
    g = api._out((D, topo.n_nodes), coords, out.get("g"))
    P = api._ptr
    args = (ctypes.byref(topo.sizes), ctypes.byref(topo.struct), P(elems), P(coords), P(grad_n),
            P(grad_b), P(grad_vol), P(n), P(b), P(V), P(g), P(topo.ws), topo.ws.numel())
    return args, (n, b, V, g)


def forward_backward(coords: torch.Tensor, topo: api.Topology, elems: torch.Tensor,
                     grad_n=None, grad_b=None, grad_vol=None, out=None, stream=None):
    """eb_batch_forward_backward: (n, b, V, dL/dx) in one persistent launch."""
    args, res = _fb_args(coords, topo, elems, grad_n, grad_b, grad_vol, out)
    check(lib().eb_batch_forward_backward(*args, api._stream_ptr(stream)),
          "eb_batch_forward_backward")
    return res


class ForwardBackwardGraph:
    """eb_batch_graph_create: the fused enqueue captured once; ``launch``
    replays it on the current contents of the inputs."""

    def __init__(self, coords, topo, elems, grad_n=None, grad_b=None, grad_vol=None,
                 out=None):
        args, res = _fb_args(coords, topo, elems, grad_n, grad_b, grad_vol, out)
        # keep every buffer the graph points at alive as long as the graph
        self._keep = (coords, topo, elems, grad_n, grad_b, grad_vol) + res
        self.n, self.b, self.V, self.g = res
        h = ctypes.c_void_p()
        check(lib().eb_batch_graph_create(*args, ctypes.byref(h)), "eb_batch_graph_create")
        self._h = h

    def launch(self, stream=None):
        check(lib().eb_graph_launch(self._h, api._stream_ptr(stream)), "eb_graph_launch")
        return self.n, self.b, self.V, self.g

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().eb_graph_destroy(self._h), "eb_graph_destroy")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_fused_shape(tile: int, unroll: int, blocks_per_cu: int = 0):
    check(lib().eb_set_fused_shape(tile, unroll, blocks_per_cu), "eb_set_fused_shape")


def get_fused_shape():
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib().eb_get_fused_shape(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def set_fused_mode(mode: str):
    """eb_set_fused_mode: 'persistent' (one persistent kernel, gather adjoint),
    'separate' (the gather kernels in sequence), 'persistent_atomic' (one
    persistent kernel, FP64-atomic adjoint: grad_coords not bitwise
    reproducible) or 'separate_atomic' (the gather forward and the atomic
    adjoint's kernels in sequence)."""
    check(lib().eb_set_fused_mode(FUSED_MODE[mode]), "eb_set_fused_mode")


def get_fused_mode() -> str:
    return {v: k for k, v in FUSED_MODE.items()}[int(lib().eb_get_fused_mode())]


def set_fused_wait_limit(spins: int):
    check(lib().eb_set_fused_wait_limit(int(spins)), "eb_set_fused_wait_limit")


def _cache_key(topo):
    name = torch.cuda.get_device_name(torch.cuda.current_device())
    # the atomic modes are tuned apart from the gather ones
    kind = "atomic" if get_fused_mode().endswith("atomic") else "gather"
    return (f"{name}|D{topo.dim}|v{topo.n_nodes}|E{topo.n_elems}|e{topo.n_edges}"
            f"|p{int(topo.sizes.plan_bytes)}|{kind}")


def autotune(coords, topo, elems, grad_n=None, grad_b=None, grad_vol=None, reps: int = 3,
             cache: str | None = None, out=None, stream=None) -> dict:
    """eb_autotune, with an optional JSON cache file keyed by device and grid
    sizes: a cached entry is applied without timing anything."""
    key = _cache_key(topo)
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
        if key in db:
            r = db[key]
            api.set_gather_shape(r["gather_tile"], r["gather_unroll"], r["gather_xcd_remap"])
            set_fused_shape(r["fused_tile"], r["fused_unroll"], r["fused_blocks_per_cu"])
            atomic = get_fused_mode().endswith("atomic")
            set_fused_mode(("separate" if r.get("fused_separate") else "persistent")
                           + ("_atomic" if atomic else ""))
            return dict(r, cached=True)
    args, _ = _fb_args(coords, topo, elems, grad_n, grad_b, grad_vol, out)
    t = EbTuning()
    check(lib().eb_autotune(*args, int(reps), api._stream_ptr(stream), ctypes.byref(t)),
          "eb_autotune")
    r = {k: getattr(t, k) for k, _ in EbTuning._fields_}
    if cache:
        db[key] = r
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(r, cached=False)
