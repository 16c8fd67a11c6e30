// C-ABI entry points for the metric, volume and adjoint calls: host-side
// validation, argument packing, launch-shape choice.
#include "eb_kernels.h"

namespace eb {

namespace {
LaunchCfg g_cfg;  // process-wide launch shape of the gather kernels
}

LaunchCfg default_cfg() { return g_cfg; }
void set_gather_cfg(const LaunchCfg &c) { g_cfg = c; }

namespace {
FusedCfg g_fused;  // process-wide launch shape of the fused kernel
}
FusedCfg fused_cfg() { return g_fused; }
void set_fused_cfg(const FusedCfg &c) { g_fused = c; }

namespace {
thread_local TimedLaunch t_armed;       // set by eb_time_next_launch
thread_local TimedLaunch t_current;     // the events of the call in progress
thread_local TimedLaunch t_span_armed;  // set by eb_time_next_call
thread_local TimedLaunch t_span;        // the span events of the call in progress
thread_local bool t_span_started = false;
}  // namespace

// The armed events move to the call in progress; whatever the call does not
// consume is dropped when it returns.
void principal_begin() {
  t_current = t_armed;
  t_armed = TimedLaunch{};
  t_span = t_span_armed;
  t_span_armed = TimedLaunch{};
  t_span_started = false;
}
void principal_end() {
  t_current = TimedLaunch{};
  t_span = TimedLaunch{};
}
void clear_armed_events() {
  t_armed = TimedLaunch{};
  t_span_armed = TimedLaunch{};
}

TimedLaunch take_principal_events() {
  const TimedLaunch t = t_current;
  t_current = TimedLaunch{};
  return t;
}

// Span events of the next launch of the call: the start event on its first
// launch only, the stop event on every launch (each overwrites it, so it
// ends at the last kernel).
TimedLaunch take_span_events() {
  TimedLaunch t = t_span;
  if (t.stop) {
    if (t_span_started) t.start = nullptr;
    t_span_started = true;
  }
  return t;
}

int pack(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem, const double *coords,
         void *ws, size_t ws_bytes, FwdArgs &a) {
  EB_TRY(check_sizes(sz));
  EB_TRY(check_ws(sz->dim, sz->n_nodes, sz->n_elems, ws, ws_bytes));
  EB_TRY(pack_arrays(sz, tp, elem, coords, true, a));
  a.st = ws_at<StatusBlock>(ws, 0);
  return EB_OK;
}

int pack_arrays(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem,
                const double *coords, bool need_elem, FwdArgs &a) {
  if (!tp || !coords || (need_elem && sz->n_elems > 0 && !elem)) {
    set_detail("null pointer");
    return EB_EINVAL;
  }
  if (!aligned16(elem) || !aligned16(coords)) {
    set_detail("arrays must be 16-byte aligned");
    return EB_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(tp->plan) & 255u) != 0) {
    set_detail("the plan must be 256-byte aligned");
    return EB_EINVAL;
  }
  a = FwdArgs{};
  a.nv = sz->n_nodes;
  a.nelem = sz->n_elems;
  a.nedge = sz->n_edges;
  a.nbface = sz->n_bfaces;
  a.nbnode = sz->n_bnodes;
  a.elem = elem;
  a.X = coords_rows(coords, sz->dim, sz->n_nodes);
  a.elem_edge = tp->elem_edge;
  a.node_inc_off = tp->node_inc_off;
  a.node_inc = tp->node_inc;
  const PlanPtrs pl = plan_ptrs(sz, tp->plan);
  a.node_sell_off = pl.slice_off;
  a.node_sell = pl.entry;
  a.inc_sell = pl.inc_slot;
  a.node_step = pl.step;
  a.sell_wide = plan_wide(sz);  // (1 for both wide formats)
  a.node_edge_off = tp->node_edge_off;
  a.edge_tail = tp->edge;
  a.edge_head = tp->edge ? tp->edge + sz->n_edges : nullptr;
  a.node_in_off = tp->node_in_off;
  a.node_in_edge = tp->node_in_edge;
  a.bface = tp->bface;
  a.bface_edge = tp->bface_edge;
  a.node_bnode = tp->node_bnode;
  a.bnode = tp->bnode;
  a.bnode_face_off = tp->bnode_face_off;
  a.bnode_face = tp->bnode_face;
  return EB_OK;
}

int need(bool ok, const char *what) {
  if (ok) return EB_OK;
  set_detail("missing topology array for this call: %s", what);
  return EB_EINVAL;
}

void rows(double *p, int dim, int64_t n, double *&x, double *&y, double *&z) {
  x = p;
  y = p ? p + n : nullptr;
  z = (p && dim == 3) ? p + 2 * n : nullptr;
}
void crows(const double *p, int dim, int64_t n, const double *&x, const double *&y,
           const double *&z) {
  x = p;
  y = p ? p + n : nullptr;
  z = (p && dim == 3) ? p + 2 * n : nullptr;
}

int check_fwd_gather(const eb_sizes *sizes, const FwdArgs &a) {
  EB_TRY(need(a.node_inc_off && a.node_sell_off && a.node_edge_off && a.edge_head &&
                  a.bnode_face_off,
              "node_inc_off, plan, node_edge_off, edge, bnode_face_off"));
  if (sizes->n_bfaces > 0) EB_TRY(need(a.bface && a.bnode && a.bnode_face, "bface, bnode, bnode_face"));
  return EB_OK;
}

// the adjoint's element pieces read a tet's six edge ids as three 8-byte words
int check_elem_edge_aligned(const eb_sizes *sizes, const FwdArgs &a) {
  if (a.w_x && sizes->dim == 3 && !aligned8(a.elem_edge)) {
    set_detail("elem_edge must be 8-byte aligned");
    return EB_EINVAL;
  }
  return EB_OK;
}

int check_bwd_gather(const eb_sizes *sizes, FwdArgs &a, void *ws, size_t ws_bytes) {
  const int D = sizes->dim;
  if (a.w_x) EB_TRY(need(a.elem_edge != nullptr, "elem_edge"));
  EB_TRY(check_elem_edge_aligned(sizes, a));
  EB_TRY(need(a.node_inc_off && a.node_sell_off, "node_inc_off, plan"));
  if (!aligned16(a.node_sell_off)) {
    set_detail("the plan must be 256-byte aligned");
    return EB_EINVAL;
  }
  if (sizes->n_bfaces > 0 && (a.w_x || a.be_x))
    EB_TRY(need(a.bface && a.bface_edge && a.node_bnode && a.bnode && a.bnode_face_off &&
                    a.bnode_face,
                "bface, bface_edge, node_bnode, bnode, bnode_face"));
  const size_t want = backward_ws_total(D, sizes->n_nodes, sizes->n_elems, plan_slots(sizes));
  if (ws_bytes < want) {
    set_detail("the gather adjoint needs %zu workspace bytes, got %zu", want, ws_bytes);
    return EB_EWORKSPACE;
  }
  a.gpiece = ws_at<double>(ws, gpiece_offset(D, sizes->n_nodes, sizes->n_elems));
  a.gstride = plan_slots(sizes);
  return EB_OK;
}

}  // namespace eb

using namespace eb;

extern "C" {

int eb_directed_areas(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                      const double *coords, int reduce, double *n_edge, double *b_node,
                      double *vol, void *ws, size_t ws_bytes, hipStream_t stream) {
  PrincipalScope scope;
  clear_detail();
  if (sizes && sizes->dim == 4)
    return forward4(sizes, topo, elem, coords, reduce, n_edge, b_node, vol, ws, ws_bytes, stream);
  FwdArgs a;
  EB_TRY(pack(sizes, topo, elem, coords, ws, ws_bytes, a));
  if (reduce != EB_REDUCE_ATOMIC && reduce != EB_REDUCE_GATHER) {
    set_detail("reduce must be EB_REDUCE_ATOMIC or EB_REDUCE_GATHER");
    return EB_EINVAL;
  }
  if (no_elements(sizes)) return vol ? fill_f64(vol, sizes->n_nodes, 0.0, stream) : EB_OK;
  if (!n_edge) {
    set_detail("n_edge is required");
    return EB_EINVAL;
  }
  const int D = sizes->dim;
  rows(n_edge, D, sizes->n_edges, a.n_x, a.n_y, a.n_z);
  rows(sizes->n_bnodes > 0 ? b_node : nullptr, D, sizes->n_bnodes, a.b_x, a.b_y, a.b_z);
  a.vol = vol;
  if (reduce == EB_REDUCE_ATOMIC) {
    EB_TRY(need(a.elem_edge != nullptr, "elem_edge"));
    if (sizes->n_bfaces > 0) EB_TRY(need(a.bface && a.bface_edge && a.node_bnode, "bface, bface_edge, node_bnode"));
  } else {
    EB_TRY(check_fwd_gather(sizes, a));
  }
  const LaunchCfg cfg = default_cfg();
  a.xcd_remap = cfg.xcd_remap;
  return D == 2 ? forward_impl<2>(a, reduce, cfg, stream) : forward_impl<3>(a, reduce, cfg, stream);
}

int eb_directed_areas_variant(const eb_sizes *sizes, const eb_topology *topo,
                              const int32_t *elem, const double *coords, int variant,
                              double *n_edge, double *b_node, double *vol, void *ws,
                              size_t ws_bytes, hipStream_t stream) {
  PrincipalScope scope;
  clear_detail();
  EB_TRY(only_dims23(sizes));
  FwdArgs a;
  EB_TRY(pack(sizes, topo, elem, coords, ws, ws_bytes, a));
  if (variant < EB_VARIANT_NODE_NORMALS || variant > EB_VARIANT_DUAL_FACES) {
    set_detail("variant must be 0, 1 or 2");
    return EB_EINVAL;
  }
  if (no_elements(sizes)) return vol ? fill_f64(vol, sizes->n_nodes, 0.0, stream) : EB_OK;
  if (!n_edge) {
    set_detail("n_edge is required");
    return EB_EINVAL;
  }
  const int D = sizes->dim;
  rows(n_edge, D, sizes->n_edges, a.n_x, a.n_y, a.n_z);
  rows(sizes->n_bnodes > 0 ? b_node : nullptr, D, sizes->n_bnodes, a.b_x, a.b_y, a.b_z);
  a.vol = vol;
  EB_TRY(check_fwd_gather(sizes, a));
  const LaunchCfg cfg = default_cfg();
  a.xcd_remap = cfg.xcd_remap;
  return D == 2 ? forward_variant_impl<2>(a, variant, cfg, stream)
                : forward_variant_impl<3>(a, variant, cfg, stream);
}

int eb_dual_volumes(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                    const double *coords, int mode, const double *n_edge, int reduce,
                    double *vol, void *ws, size_t ws_bytes, hipStream_t stream) {
  PrincipalScope scope;
  clear_detail();
  if (sizes && sizes->dim == 4)
    return volumes4(sizes, topo, elem, coords, mode, n_edge, reduce, vol, ws, ws_bytes, stream);
  FwdArgs a;
  EB_TRY(pack(sizes, topo, elem, coords, ws, ws_bytes, a));
  if ((mode != EB_VOL_ELEMENT && mode != EB_VOL_EDGE) ||
      (reduce != EB_REDUCE_ATOMIC && reduce != EB_REDUCE_GATHER) || !vol) {
    set_detail("bad mode / reduce, or vol is null");
    return EB_EINVAL;
  }
  if (no_elements(sizes)) return fill_f64(vol, sizes->n_nodes, 0.0, stream);
  if (mode == EB_VOL_EDGE) {
    if (!n_edge) {
      set_detail("EB_VOL_EDGE needs n_edge");
      return EB_EINVAL;
    }
    EB_TRY(need(a.edge_tail && a.edge_head, "edge"));
    if (reduce == EB_REDUCE_GATHER) {
      EB_TRY(need(a.node_edge_off && a.node_in_off && a.node_in_edge, "node_edge_off, node_in"));
      // per-edge terms in the workspace's incidence-row region (8 bytes per
      // edge fit: it holds 16 (dim+1) bytes per element)
      a.vterm = ws_at<double>(ws, ws_layout(sizes->dim, sizes->n_nodes, sizes->n_elems).rows4);
    }
  } else if (reduce == EB_REDUCE_GATHER) {
    EB_TRY(need(a.node_inc_off && a.node_inc, "node_inc"));
  }
  a.vol = vol;
  return sizes->dim == 2 ? volumes_impl<2>(a, mode, reduce, n_edge, stream)
                         : volumes_impl<3>(a, mode, reduce, n_edge, stream);
}

int eb_edge_residual(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                     const double *coords, const double *n_edge, const double *b_node,
                     const double *flux, int bflux, double *res, void *ws, size_t ws_bytes,
                     hipStream_t stream) {
  PrincipalScope scope;
  clear_detail();
  EB_TRY(only_dims23(sizes));
  FwdArgs a;
  EB_TRY(pack(sizes, topo, elem, coords, ws, ws_bytes, a));
  if (!flux || !res || (bflux != EB_BFLUX_NODE && bflux != EB_BFLUX_LINEAR)) {
    set_detail("n_edge, flux and res are required; b_node for EB_BFLUX_NODE; bflux 0 or 1");
    return EB_EINVAL;
  }
  if (no_elements(sizes)) return fill_f64(res, sizes->n_nodes, 0.0, stream);
  if (!n_edge || (bflux == EB_BFLUX_NODE && sizes->n_bnodes > 0 && !b_node)) {
    set_detail("n_edge, flux and res are required; b_node for EB_BFLUX_NODE; bflux 0 or 1");
    return EB_EINVAL;
  }
  EB_TRY(need(a.edge_tail && a.edge_head && a.node_edge_off && a.node_in_off && a.node_in_edge,
              "edge, node_edge_off, node_in"));
  if (sizes->n_bnodes > 0)
    EB_TRY(need(a.bnode && (bflux == EB_BFLUX_NODE || (a.bnode_face_off && a.bnode_face && a.bface)),
                "bnode, bnode_face, bface"));
  const int D = sizes->dim;
  rows(sizes->n_bnodes > 0 ? const_cast<double *>(b_node) : nullptr, D, sizes->n_bnodes, a.b_x,
       a.b_y, a.b_z);
  a.vterm = ws_at<double>(ws, ws_layout(D, sizes->n_nodes, sizes->n_elems).rows4);
  return D == 2 ? residual_impl<2>(a, n_edge, flux, bflux, res, stream)
                : residual_impl<3>(a, n_edge, flux, bflux, res, stream);
}

int eb_directed_areas_backward(const eb_sizes *sizes, const eb_topology *topo,
                               const int32_t *elem, const double *coords, const double *grad_n,
                               const double *grad_b, const double *grad_vol, int reduce,
                               double *grad_coords, void *ws, size_t ws_bytes,
                               hipStream_t stream) {
  PrincipalScope scope;
  clear_detail();
  EB_TRY(only_dims23(sizes));
  FwdArgs a;
  EB_TRY(pack(sizes, topo, elem, coords, ws, ws_bytes, a));
  if ((reduce != EB_REDUCE_ATOMIC && reduce != EB_REDUCE_GATHER) || !grad_coords) {
    set_detail("bad reduce, or grad_coords is null");
    return EB_EINVAL;
  }
  const int D = sizes->dim;
  if (no_elements(sizes)) return fill_f64(grad_coords, D * sizes->n_nodes, 0.0, stream);
  crows(grad_n, D, sizes->n_edges, a.w_x, a.w_y, a.w_z);
  crows(sizes->n_bnodes > 0 ? grad_b : nullptr, D, sizes->n_bnodes, a.be_x, a.be_y, a.be_z);
  a.c = grad_vol;
  rows(grad_coords, D, sizes->n_nodes, a.g_x, a.g_y, a.g_z);
  if (a.w_x) EB_TRY(need(a.elem_edge != nullptr, "elem_edge"));
  EB_TRY(check_elem_edge_aligned(sizes, a));
  if (sizes->n_bfaces > 0 && (a.w_x || a.be_x))
    EB_TRY(need(a.bface && a.bface_edge && a.node_bnode, "bface, bface_edge, node_bnode"));
  if (reduce == EB_REDUCE_GATHER) EB_TRY(check_bwd_gather(sizes, a, ws, ws_bytes));
  const LaunchCfg cfg = default_cfg();
  a.xcd_remap = cfg.xcd_remap;
  return D == 2 ? backward_impl<2>(a, reduce, cfg, stream) : backward_impl<3>(a, reduce, cfg, stream);
}

int eb_time_next_call(hipEvent_t start, hipEvent_t stop) {
  clear_detail();
  if ((start == nullptr) != (stop == nullptr)) {
    set_detail("start and stop must both be set or both be null");
    return EB_EINVAL;
  }
  t_span_armed.start = start;
  t_span_armed.stop = stop;
  return EB_OK;
}

int eb_time_next_launch(hipEvent_t start, hipEvent_t stop) {
  clear_detail();
  if ((start == nullptr) != (stop == nullptr)) {
    set_detail("start and stop must both be set or both be null");
    return EB_EINVAL;
  }
  t_armed.start = start;
  t_armed.stop = stop;
  return EB_OK;
}

int eb_set_gather_shape(int tile, int unroll, int xcd_remap) {
  clear_detail();
  if ((tile != 64 && tile != 128 && tile != 256) || (unroll != 1 && unroll != 2 && unroll != 4) ||
      (xcd_remap != 0 && xcd_remap != 1)) {
    set_detail("tile must be 64/128/256, unroll 1/2/4, xcd_remap 0/1");
    return EB_EINVAL;
  }
  g_cfg.tile = tile;
  g_cfg.unroll = unroll;
  g_cfg.xcd_remap = xcd_remap;
  return EB_OK;
}

void eb_get_gather_shape(int *tile, int *unroll, int *xcd_remap) {
  if (tile) *tile = g_cfg.tile;
  if (unroll) *unroll = g_cfg.unroll;
  if (xcd_remap) *xcd_remap = g_cfg.xcd_remap;
}

}  // extern "C"
