"""Python binding of the C ABI in ``include/eb.h`` (same names).

Argument marshalling only: torch provides device memory and the current HIP
stream; every step of the computation runs in the library's HIP kernels.
Inputs must be CUDA(HIP) tensors: coordinates float64 ``[D, Nv]``,
connectivity int32 ``[NE, D+1]``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import EbSizes, EbTopology, check, lib

__all__ = ["Topology", "build_edges", "directed_areas", "dual_volumes",
           "directed_areas_backward", "check_errors", "set_gather_shape",
           "get_gather_shape", "workspace_bytes", "time_next_launch", "time_next_call",
           "edge_residual",
           "directed_areas_variant", "dual_volumes_noalloc", "REDUCE", "VOL_MODE", "BFLUX",
           "VARIANT"]

REDUCE = {"atomic": _lib.EB_REDUCE_ATOMIC, "gather": _lib.EB_REDUCE_GATHER}
VOL_MODE = {"element": _lib.EB_VOL_ELEMENT, "edge": _lib.EB_VOL_EDGE}
BFLUX = {"node": 0, "linear": 1}
VARIANT = {"node_normals": 0, "edge_normals": 1, "dual_faces": 2}


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def workspace_bytes(dim: int, n_nodes: int, n_elems: int) -> int:
    return int(lib().eb_workspace_bytes(dim, n_nodes, n_elems))


@dataclass
class Topology:
    """Device-resident topology of one grid (all arrays int32 unless noted)."""
    dim: int
    n_nodes: int
    n_elems: int
    n_edges: int
    n_bfaces: int
    n_bnodes: int
    arrays: dict
    ws: torch.Tensor
    sizes: EbSizes = field(repr=False, default=None)
    struct: EbTopology = field(repr=False, default=None)

    def __getitem__(self, name):
        return self.arrays[name]

    @property
    def ne(self):
        return self.dim * (self.dim + 1) // 2

    def to_numpy(self):
        """Host copies of the topology arrays (the opaque plan excluded)."""
        return {k: v.cpu().numpy() for k, v in self.arrays.items()
                if v is not None and k != "plan"}

    def plan_view(self):
        """eb_plan_describe: host copies of the kernel plan's arrays, for
        tests that check the plan against the topology (its encoding is the
        library's private one, stated in csrc/eb_plan.h)."""
        v = _lib.EbPlanView()
        plan = self.arrays["plan"]
        check(lib().eb_plan_describe(ctypes.byref(self.sizes), _ptr(plan), ctypes.byref(v)),
              "eb_plan_describe")
        host, base = plan.cpu().numpy(), plan.data_ptr()

        def part(ptr, count, dtype):
            if not ptr:
                return None
            off = ptr - base
            return host[off: off + count * np.dtype(dtype).itemsize].view(dtype)

        return dict(slice_off=part(v.slice_off, (self.n_nodes + 63) // 64 + 1, np.int32),
                    entry=part(v.entry, v.n_slots * v.words, np.uint64),
                    step=part(v.step, v.n_slots, np.uint32),
                    inc_slot=part(v.inc_slot, (self.dim + 1) * self.n_elems, np.int32),
                    n_slots=int(v.n_slots), words=int(v.words))


def build_edges(elems: torch.Tensor, coords: torch.Tensor, edge_inc: bool = True,
                adjoint: bool = True, stream=None) -> Topology:
    """Edge extraction and boundary elements (eb_build_edges + _emit).

    ``adjoint`` also sizes the workspace for the gather adjoint
    (eb_backward_workspace_bytes)."""
    if elems.dim() != 2 or elems.shape[1] not in (3, 4, 5):
        raise ValueError("elems must be [NE, D+1] with D in {2, 3, 4}")
    dim = int(elems.shape[1]) - 1
    _need(elems, "elems", torch.int32)
    _need(coords, "coords", torch.float64)
    if coords.dim() != 2 or coords.shape[0] != dim:
        raise ValueError(f"coords must be [{dim}, Nv]")
    nv, nel = int(coords.shape[1]), int(elems.shape[0])
    dev = coords.device
    L = lib()
    wsb = workspace_bytes(dim, nv, nel)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    node_inc_off = torch.empty(nv + 1, **i32)
    node_inc = torch.empty(max((dim + 1) * nel, 1), **i32)
    sizes = EbSizes()
    s = _stream_ptr(stream)
    check(L.eb_build_edges(dim, nv, nel, _ptr(elems), _ptr(coords), _ptr(node_inc_off),
                           _ptr(node_inc), _ptr(ws), wsb, ctypes.byref(sizes), s),
          "eb_build_edges")
    ne_, nb, nbn = int(sizes.n_edges), int(sizes.n_bfaces), int(sizes.n_bnodes)
    ne = dim * (dim + 1) // 2
    nbe = dim * (dim - 1) // 2
    arr = dict(
        edge=torch.empty(2, ne_, **i32),
        node_edge_off=torch.empty(nv + 1, **i32),
        elem_edge=torch.empty(nel, ne, **i32),
        elem_edge_sign=torch.empty(nel, ne, dtype=torch.int8, device=dev),
        edge_inc_off=torch.empty(ne_ + 1, **i32) if edge_inc else None,
        edge_inc=torch.empty(max(ne * nel, 1), **i32) if edge_inc else None,
        node_inc_off=node_inc_off,
        node_inc=node_inc,
        node_in_off=torch.empty(nv + 1, **i32),
        node_in_edge=torch.empty(max(ne_, 1), **i32),
        bface=torch.empty(nb, dim, **i32),
        bface_owner=torch.empty(nb, **i32),
        bface_edge=torch.empty(nb, nbe, **i32),
        bnode=torch.empty(nbn, **i32),
        node_bnode=torch.empty(nv, **i32),
        bnode_face_off=torch.empty(nbn + 1, **i32),
        bnode_face=torch.empty(max(dim * nb, 1), **i32),
        plan=torch.empty(int(sizes.plan_bytes), dtype=torch.uint8, device=dev),
    )
    st = EbTopology(**{k: (v.data_ptr() if v is not None else None) for k, v in arr.items()})
    check(L.eb_build_edges_emit(ctypes.byref(sizes), _ptr(elems), _ptr(coords),
                                ctypes.byref(st), _ptr(ws), wsb, s), "eb_build_edges_emit")
    if adjoint:
        # after the emit pass only the status block of ws is live; the gather
        # adjoint needs a larger workspace (eb_backward_workspace_bytes)
        wsb2 = int(L.eb_backward_workspace_bytes(ctypes.byref(sizes)))
        if wsb2 > wsb:
            with torch.cuda.stream(stream if stream is not None
                                   else torch.cuda.current_stream()):
                ws2 = torch.empty(wsb2, dtype=torch.uint8, device=dev)
                ws2[:256].copy_(ws[:256])
            ws, wsb = ws2, wsb2
    # trim the placeholder lengths used for empty arrays
    arr["node_inc"] = arr["node_inc"][: (dim + 1) * nel]
    arr["node_in_edge"] = arr["node_in_edge"][:ne_]
    arr["bnode_face"] = arr["bnode_face"][: dim * nb]
    if edge_inc:
        arr["edge_inc"] = arr["edge_inc"][: ne * nel]
    return Topology(dim, nv, nel, ne_, nb, nbn, arr, ws, sizes, st)


def _out(shape, like, out):
    if out is not None:
        return _need(out, "out", torch.float64, shape)
    return torch.empty(shape, dtype=torch.float64, device=like.device)


def directed_areas(coords: torch.Tensor, topo: Topology, elems: torch.Tensor,
                   reduce: str = "gather", volumes: bool = True, boundary: bool = True,
                   n_out=None, b_out=None, v_out=None, stream=None):
    """(n [D, Ne], b [D, Nbn] | None, V [Nv] | None) via eb_directed_areas."""
    D = topo.dim
    _need(coords, "coords", torch.float64, (D, topo.n_nodes))
    _need(elems, "elems", torch.int32, (topo.n_elems, D + 1))
    n = _out((D, topo.n_edges), coords, n_out)
    b = _out((D, topo.n_bnodes), coords, b_out) if boundary else None
    V = _out((topo.n_nodes,), coords, v_out) if volumes else None
    check(lib().eb_directed_areas(ctypes.byref(topo.sizes), ctypes.byref(topo.struct),
                                  _ptr(elems), _ptr(coords), REDUCE[reduce], _ptr(n), _ptr(b),
                                  _ptr(V), _ptr(topo.ws), topo.ws.numel(), _stream_ptr(stream)),
          "eb_directed_areas")
    return n, b, V


def dual_volumes(coords: torch.Tensor, topo: Topology, elems: torch.Tensor,
                 mode: str = "element", n: torch.Tensor | None = None,
                 reduce: str = "gather", out=None, stream=None):
    D = topo.dim
    _need(coords, "coords", torch.float64, (D, topo.n_nodes))
    _need(elems, "elems", torch.int32, (topo.n_elems, D + 1))
    if n is not None:
        _need(n, "n", torch.float64, (D, topo.n_edges))
    V = _out((topo.n_nodes,), coords, out)
    check(lib().eb_dual_volumes(ctypes.byref(topo.sizes), ctypes.byref(topo.struct),
                                _ptr(elems), _ptr(coords), VOL_MODE[mode], _ptr(n),
                                REDUCE[reduce], _ptr(V), _ptr(topo.ws), topo.ws.numel(),
                                _stream_ptr(stream)), "eb_dual_volumes")
    return V


def dual_volumes_noalloc(coords: torch.Tensor, topo: Topology, n: torch.Tensor,
                         reduce: str = "gather", out=None, stream=None):
    """eb_dual_volumes_noalloc: the edge-loop V_j without a workspace (the
    library's fixed device array holds the per-edge terms)."""
    D = topo.dim
    _need(coords, "coords", torch.float64, (D, topo.n_nodes))
    _need(n, "n", torch.float64, (D, topo.n_edges))
    V = _out((topo.n_nodes,), coords, out)
    check(lib().eb_dual_volumes_noalloc(ctypes.byref(topo.sizes), ctypes.byref(topo.struct),
                                        _ptr(coords), _ptr(n), REDUCE[reduce], _ptr(V),
                                        _stream_ptr(stream)), "eb_dual_volumes_noalloc")
    return V


def directed_areas_backward(coords: torch.Tensor, topo: Topology, elems: torch.Tensor,
                            grad_n=None, grad_b=None, grad_vol=None,
                            reduce: str = "atomic", out=None, stream=None):
    """dL/dx [D, Nv] given dL/dn, dL/db, dL/dV (eb_directed_areas_backward)."""
    D = topo.dim
    _need(coords, "coords", torch.float64, (D, topo.n_nodes))
    _need(elems, "elems", torch.int32, (topo.n_elems, D + 1))
    if grad_n is not None:
        _need(grad_n, "grad_n", torch.float64, (D, topo.n_edges))
    if grad_b is not None:
        _need(grad_b, "grad_b", torch.float64, (D, topo.n_bnodes))
    if grad_vol is not None:
        _need(grad_vol, "grad_vol", torch.float64, (topo.n_nodes,))
    g = _out((D, topo.n_nodes), coords, out)
    check(lib().eb_directed_areas_backward(
        ctypes.byref(topo.sizes), ctypes.byref(topo.struct), _ptr(elems), _ptr(coords),
        _ptr(grad_n), _ptr(grad_b), _ptr(grad_vol), REDUCE[reduce], _ptr(g), _ptr(topo.ws),
        topo.ws.numel(), _stream_ptr(stream)), "eb_directed_areas_backward")
    return g


def check_errors(topo: Topology, stream=None) -> int:
    """Synchronize and raise if a kernel recorded an error (eb_check_errors)."""
    rc = lib().eb_check_errors(_ptr(topo.ws), _stream_ptr(stream))
    check(rc, "eb_check_errors")
    return rc


def set_gather_shape(tile: int, unroll: int, xcd_remap: int = 1):
    check(lib().eb_set_gather_shape(tile, unroll, xcd_remap), "eb_set_gather_shape")


def get_gather_shape():
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib().eb_get_gather_shape(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def time_next_launch(start, stop):
    """Arm two ``torch.cuda.Event(enable_timing=True)`` for the principal
    kernel of the next metric / volume / adjoint call (eb_time_next_launch).
    The events must already exist on the device (record each once)."""
    check(lib().eb_time_next_launch(ctypes.c_void_p(start.cuda_event),
                                    ctypes.c_void_p(stop.cuda_event)), "eb_time_next_launch")


def time_next_call(start, stop):
    """Arm two ``torch.cuda.Event(enable_timing=True)`` to bracket the
    kernels of the next eb_directed_areas call (eb_time_next_call)."""
    check(lib().eb_time_next_call(ctypes.c_void_p(start.cuda_event),
                                  ctypes.c_void_p(stop.cuda_event)), "eb_time_next_call")


def edge_residual(coords: torch.Tensor, topo: Topology, elems: torch.Tensor, n: torch.Tensor,
                  flux: torch.Tensor, b: torch.Tensor | None = None, bflux: str = "linear",
                  out=None, stream=None):
    """eb_edge_residual: res [Nv] of the edge loop with nodal flux [D, Nv]."""
    D = topo.dim
    _need(coords, "coords", torch.float64, (D, topo.n_nodes))
    _need(elems, "elems", torch.int32, (topo.n_elems, D + 1))
    _need(n, "n", torch.float64, (D, topo.n_edges))
    _need(flux, "flux", torch.float64, (D, topo.n_nodes))
    if b is not None:
        _need(b, "b", torch.float64, (D, topo.n_bnodes))
    res = _out((topo.n_nodes,), coords, out)
    check(lib().eb_edge_residual(ctypes.byref(topo.sizes), ctypes.byref(topo.struct),
                                 _ptr(elems), _ptr(coords), _ptr(n), _ptr(b), _ptr(flux),
                                 BFLUX[bflux], _ptr(res), _ptr(topo.ws), topo.ws.numel(),
                                 _stream_ptr(stream)), "eb_edge_residual")
    return res


def directed_areas_variant(coords: torch.Tensor, topo: Topology, elems: torch.Tensor,
                           variant: str, n_out=None, b_out=None, v_out=None, stream=None):
    """eb_directed_areas_variant: (n, b, V) by the chosen construction."""
    D = topo.dim
    _need(coords, "coords", torch.float64, (D, topo.n_nodes))
    _need(elems, "elems", torch.int32, (topo.n_elems, D + 1))
    n = _out((D, topo.n_edges), coords, n_out)
    b = _out((D, topo.n_bnodes), coords, b_out)
    V = _out((topo.n_nodes,), coords, v_out)
    check(lib().eb_directed_areas_variant(ctypes.byref(topo.sizes), ctypes.byref(topo.struct),
                                          _ptr(elems), _ptr(coords), VARIANT[variant], _ptr(n),
                                          _ptr(b), _ptr(V), _ptr(topo.ws), topo.ws.numel(),
                                          _stream_ptr(stream)), "eb_directed_areas_variant")
    return n, b, V
