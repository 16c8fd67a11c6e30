"""ctypes loader for ``libeb.so`` — argument marshalling only.

The library must have been built (``python -m paper_2502_00778_amd.build`` or
``__graft_entry__.build()``); there is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeb.so")

EB_OK = 0
EB_REDUCE_ATOMIC, EB_REDUCE_GATHER = 0, 1
EB_VOL_ELEMENT, EB_VOL_EDGE = 0, 1
STATUS_NAMES = {0: "EB_OK", -1: "EB_EINVAL", -2: "EB_ERANGE", -3: "EB_EDEGENERATE",
                -4: "EB_ENONMANIFOLD", -5: "EB_EWORKSPACE", -6: "EB_EOVERFLOW",
                -7: "EB_EHIP", -8: "EB_ECAPACITY", -9: "EB_ETIMEOUT"}

# every symbol declared in include/eb.h
EXPORTS = ("eb_workspace_bytes", "eb_backward_workspace_bytes", "eb_build_edges", "eb_build_edges_emit",
           "eb_directed_areas", "eb_dual_volumes", "eb_directed_areas_backward",
           "eb_set_gather_shape", "eb_get_gather_shape", "eb_time_next_launch", "eb_check_errors",
           "eb_status_string", "eb_last_error_detail", "eb_version",
           "eb_batch_offsets", "eb_batch_forward_backward", "eb_batch_graph_create",
           "eb_graph_launch", "eb_graph_destroy", "eb_set_fused_shape", "eb_get_fused_shape",
           "eb_set_fused_wait_limit", "eb_autotune", "eb_edge_residual",
           "eb_directed_areas_variant", "eb_set_fused_mode", "eb_get_fused_mode",
           "eb_plan_describe", "eb_dual_volumes_noalloc", "eb_time_next_call")

TOPO_FIELDS = ("edge", "node_edge_off", "elem_edge", "elem_edge_sign",
               "edge_inc_off", "edge_inc", "node_inc_off", "node_inc",
               "node_in_off", "node_in_edge", "bface", "bface_owner",
               "bface_edge", "bnode", "node_bnode", "bnode_face_off",
               "bnode_face", "plan")


class EbSizes(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_nodes", ctypes.c_int64),
                ("n_elems", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("n_bfaces", ctypes.c_int64), ("n_bnodes", ctypes.c_int64),
                ("plan_bytes", ctypes.c_int64), ("plan_param", ctypes.c_int64 * 2)]


class EbTopology(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in TOPO_FIELDS]


class EbPlanView(ctypes.Structure):
    _fields_ = [("slice_off", ctypes.c_void_p), ("entry", ctypes.c_void_p),
                ("step", ctypes.c_void_p), ("inc_slot", ctypes.c_void_p),
                ("n_slots", ctypes.c_int64), ("words", ctypes.c_int32)]


class EbTuning(ctypes.Structure):
    _fields_ = [("gather_tile", ctypes.c_int32), ("gather_unroll", ctypes.c_int32),
                ("gather_xcd_remap", ctypes.c_int32), ("gather_ms", ctypes.c_float),
                ("fused_tile", ctypes.c_int32), ("fused_unroll", ctypes.c_int32),
                ("fused_blocks_per_cu", ctypes.c_int32), ("fused_ms", ctypes.c_float),
                ("n_tried", ctypes.c_int32), ("fused_separate", ctypes.c_int32),
                ("separate_ms", ctypes.c_float)]


class EbError(RuntimeError):
    def __init__(self, code: int, call: str, detail: str = ""):
        name = STATUS_NAMES.get(code, str(code))
        super().__init__(f"{call} failed: {name}"
                         + (f" ({detail})" if detail else ""))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2502_00778_amd.build); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                       ctypes.c_size_t)
    L.eb_workspace_bytes.argtypes = [i32, i64, i64]
    L.eb_workspace_bytes.restype = sz
    L.eb_backward_workspace_bytes.argtypes = [ctypes.POINTER(EbSizes)]
    L.eb_backward_workspace_bytes.restype = sz
    L.eb_build_edges.argtypes = [i32, i64, i64, P, P, P, P, P, sz,
                                 ctypes.POINTER(EbSizes), P]
    L.eb_build_edges_emit.argtypes = [ctypes.POINTER(EbSizes), P, P,
                                      ctypes.POINTER(EbTopology), P, sz, P]
    L.eb_directed_areas.argtypes = [ctypes.POINTER(EbSizes),
                                    ctypes.POINTER(EbTopology), P, P, i32, P,
                                    P, P, P, sz, P]
    L.eb_dual_volumes.argtypes = [ctypes.POINTER(EbSizes),
                                  ctypes.POINTER(EbTopology), P, P, i32, P,
                                  i32, P, P, sz, P]
    L.eb_directed_areas_backward.argtypes = [ctypes.POINTER(EbSizes),
                                             ctypes.POINTER(EbTopology), P, P,
                                             P, P, P, i32, P, P, sz, P]
    L.eb_set_gather_shape.argtypes = [i32, i32, i32]
    L.eb_get_gather_shape.argtypes = [ctypes.POINTER(ctypes.c_int)] * 3
    L.eb_get_gather_shape.restype = None
    L.eb_check_errors.argtypes = [P, P]
    L.eb_time_next_launch.argtypes = [P, P]
    L.eb_time_next_call.argtypes = [P, P]
    SZ, TP = ctypes.POINTER(EbSizes), ctypes.POINTER(EbTopology)
    I64P = ctypes.POINTER(ctypes.c_int64)
    L.eb_batch_offsets.argtypes = [SZ, TP, P, i32, I64P, I64P, I64P, I64P, I64P, P, sz, P]
    L.eb_batch_forward_backward.argtypes = [SZ, TP, P, P, P, P, P, P, P, P, P, P, sz, P]
    L.eb_batch_graph_create.argtypes = [SZ, TP, P, P, P, P, P, P, P, P, P, P, sz,
                                        ctypes.POINTER(ctypes.c_void_p)]
    L.eb_graph_launch.argtypes = [P, P]
    L.eb_graph_destroy.argtypes = [P]
    L.eb_set_fused_shape.argtypes = [i32, i32, i32]
    L.eb_get_fused_shape.argtypes = [ctypes.POINTER(ctypes.c_int)] * 3
    L.eb_get_fused_shape.restype = None
    L.eb_set_fused_wait_limit.argtypes = [i64]
    L.eb_set_fused_mode.argtypes = [i32]
    L.eb_get_fused_mode.restype = i32
    L.eb_autotune.argtypes = [SZ, TP, P, P, P, P, P, P, P, P, P, P, sz, i32, P,
                              ctypes.POINTER(EbTuning)]
    L.eb_edge_residual.argtypes = [SZ, TP, P, P, P, P, P, i32, P, P, sz, P]
    L.eb_directed_areas_variant.argtypes = [SZ, TP, P, P, i32, P, P, P, P, sz, P]
    L.eb_plan_describe.argtypes = [SZ, P, ctypes.POINTER(EbPlanView)]
    L.eb_dual_volumes_noalloc.argtypes = [SZ, TP, P, P, i32, P, P]
    L.eb_status_string.argtypes = [i32]
    L.eb_status_string.restype = ctypes.c_char_p
    L.eb_last_error_detail.restype = ctypes.c_char_p
    L.eb_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(rc: int, call: str):
    if rc != EB_OK:
        detail = lib().eb_last_error_detail().decode(errors="replace")
        raise EbError(rc, call, detail)
