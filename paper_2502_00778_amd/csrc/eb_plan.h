// The kernel plan: the node-centred kernels' private view of a grid's
// incidences, written by eb_build_edges_emit into the caller's plan buffer
// (eb_topology.plan, eb_sizes.plan_bytes) and read by the gather forward,
// the gather adjoint and the fused kernel.  Callers never interpret it; its
// layout is fixed here only.
//
// Sections, each starting on a 256-byte line:
//   slice_off [ceil(n_nodes/64)+1] int32
//             nodes are taken in slices of 64 (node j is lane j%64 of slice
//             j/64, one wavefront); slice s holds L_s = its longest node_inc
//             row, column-major: entry (r, lane) of slice s is at slot
//             slice_off[s] + 64 r + lane for r < L_s (entries past a node's
//             row are zero).  n_slots = slice_off[last].
//   entry     [n_slots * words] uint64
//             the entries of node j are its node_inc row's incidences.  A row
//             of at most 32 is stored as a strip: first its smallest
//             incidence, then repeatedly, of those not yet stored in
//             ascending order, the first sharing at least dim-1 distinct
//             other vertices with the last stored (a face of the node's
//             link), else the first sharing the most; a longer row is stored
//             ascending.  For incidence (element E, local l) the other
//             vertices in local order are p_m = elem[E][m] for m < dim,
//             except p_l = elem[E][dim].  In a strip they take places: a
//             vertex the previous entry holds keeps its place there (place k
//             is matched to the first unmatched p_m equal to it), the rest
//             fill the free places in local order; the first entry, and every
//             entry of a longer row, keep local order.  o_m = the vertex in
//             place m; slot_m = the position of edge (j, o_m) among j's
//             out-edges (node_edge_off order), or the field's all-ones value
//             when o_m < j; code = sum_m slot_m << (B m).
//             Narrow (words = 1): B = 5, bits 16m..16m+15 = o_m - j as int16,
//             bits 48..62 = code.  Wide (words = 2, chosen when some
//             |o_m - j| > 32767 or some node has more than 31 out-edges):
//             B = 10, word 0 = o_0 | o_1 << 32, word 1 = o_2 | code << 32
//             (o_2 = 0 in 2D).  Consecutive entries of a strip differ in one
//             place, so a reader walking a row keeps the other points.
//   step      [n_slots] uint32, present unless the format is wide without
//             steps (below): the step from entry c-1 of node j's row to entry
//             c, at entry c's slot.  When exactly one place k changes: bits
//             0..19 = o_k - j as a 20-bit two's complement value, bits 20..21
//             = k, bits 22..26 = slot_k (31 = none); otherwise (c = 0, or
//             several or no places change) bit 27 set and the rest 0.  Past a
//             row's end 0.  The gather forward reads 4 bytes per incidence
//             instead of 8 or 16.
//   inc_slot  [(dim+1)*n_elems] int32: slot of incidence elem*(dim+1)+local
//             in the layout above with rows in ascending order, i.e.
//             slice_off[j/64] + 64 r + j%64 for the incidence's rank r in node
//             j's node_inc row (the gather adjoint's per-incidence gradient
//             pieces live at these slots).
//
// Formats (eb_sizes.plan_param[1]): 0 narrow entries with step words (every
// |o_m - j| <= 32767 and at most 31 out-edges per node); 2 wide entries with
// step words (every |o_m - j| <= 2^19 - 1 and at most 31 out-edges: large
// grids numbered with locality); 1 wide entries alone (any grid).
//
// Limits: a node's row has at most 65535 entries (its ranks are 16-bit in
// the build) and at most 1023 out-edges (10-bit slot fields); the build
// reports EB_ECAPACITY beyond either.
#pragma once

#include "eb_internal.h"

namespace eb {

constexpr int MAX_OUT_EDGES = EB_MAX_OUT_EDGES;  // wide slot fields hold 0..1022, 1023 = none
constexpr int MAX_NODE_ELEMS = EB_MAX_NODE_ELEMS;
static_assert(MAX_OUT_EDGES == 1023 && MAX_NODE_ELEMS == 65535, "plan field widths");

struct PlanLayout {
  size_t slice_off, entry, step, inc_slot, total;
};

constexpr int PLAN_NARROW = 0, PLAN_WIDE = 1, PLAN_WIDE_STEPS = 2;
// step words: delta bits, the place's and the slot's shifts, the flag of an
// entry read whole
constexpr int STEP_DBITS = 20, STEP_PLACE = 20, STEP_SLOT = 22;
constexpr uint32_t STEP_WHOLE = 1u << 27;
constexpr int32_t STEP_MAX_DELTA = (1 << (STEP_DBITS - 1)) - 1;

inline PlanLayout plan_layout(int dim, int64_t n_nodes, int64_t n_elems, int64_t n_slots,
                              int format) {
  const bool wide = format != PLAN_NARROW, steps = format != PLAN_WIDE;
  PlanLayout P{};
  if (dim == 4) {  // no plan in four dimensions: one placeholder line
    P.total = 256;
    return P;
  }
  size_t off = 0;
  P.slice_off = off;
  off += align256(sizeof(int32_t) * (size_t)(n_slices(n_nodes) + 1));
  P.entry = off;
  off += align256(sizeof(uint64_t) * (size_t)n_slots * (wide ? 2 : 1));
  P.step = off;
  off += steps ? align256(sizeof(uint32_t) * (size_t)n_slots) : 0;
  P.inc_slot = off;
  off += align256(sizeof(int32_t) * (size_t)(dim + 1) * (size_t)n_elems);
  P.total = off;
  return P;
}

// the plan's layout parameters as eb_build_edges records them in eb_sizes
inline int64_t plan_slots(const eb_sizes *s) { return s->plan_param[0]; }
inline int plan_format(const eb_sizes *s) { return (int)s->plan_param[1]; }
inline int plan_wide(const eb_sizes *s) { return plan_format(s) != PLAN_NARROW ? 1 : 0; }
inline size_t plan_bytes_of(const eb_sizes *s) {
  return plan_layout(s->dim, s->n_nodes, s->n_elems, plan_slots(s), plan_format(s)).total;
}

struct PlanPtrs {
  int32_t *slice_off;
  uint64_t *entry;
  uint32_t *step;  // null in the wide format without steps
  int32_t *inc_slot;
};

inline PlanPtrs plan_ptrs(const eb_sizes *s, void *plan) {
  const PlanLayout P = plan_layout(s->dim, s->n_nodes, s->n_elems, plan_slots(s), plan_format(s));
  char *b = static_cast<char *>(plan);
  PlanPtrs p{};
  if (!b || s->dim == 4) return p;
  p.slice_off = reinterpret_cast<int32_t *>(b + P.slice_off);
  p.entry = reinterpret_cast<uint64_t *>(b + P.entry);
  p.step = plan_format(s) == PLAN_WIDE ? nullptr : reinterpret_cast<uint32_t *>(b + P.step);
  p.inc_slot = reinterpret_cast<int32_t *>(b + P.inc_slot);
  return p;
}

// the layout parameters eb_sizes may carry: what a build can produce
inline bool plan_params_valid(const eb_sizes *s) {
  const int64_t n_slots = plan_slots(s);
  return n_slots >= 0 && n_slots % SELL == 0 && n_slots < (int64_t(1) << 31) &&
         (s->plan_param[1] == PLAN_NARROW || s->plan_param[1] == PLAN_WIDE ||
          s->plan_param[1] == PLAN_WIDE_STEPS) &&
         s->plan_bytes == (int64_t)plan_bytes_of(s);
}

}  // namespace eb
