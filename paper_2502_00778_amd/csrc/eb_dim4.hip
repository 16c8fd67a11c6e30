// Metrics of pentatope grids (dim = 4): the general-D formula of Section
// 3.2.3 with D = 4,
//   n_jk = 1/10 sum_{E contains jk} n_j^E + 1/20 sum_{B contains jk} n_B,
//   b_j  = 1/4 sum_{B contains j} n_B,
//   V_j  = sum_{E contains j} |E|/5      or   1/8 sum_k (x_k - x_j).n_jk,
// with n_j^E the outward area vector of the face of E opposite j (a
// tetrahedron) and n_B that of a boundary tetrahedron (eb_geom4.h).  The
// paper derives D = 2 and 3 and leaves D = 4 to future work.
//
// Plain kernels, not tuned: the gather forward walks each node's node_inc
// row (one thread per node, connectivity and points gathered per incidence,
// the node's out-edges found by binary search among its edge heads and
// accumulated in place, in row order), then a boundary pass per boundary
// node; the atomic forward scatters per element and per boundary face.
#include "eb_geom4.h"
#include "eb_kernels.h"

namespace eb {
namespace {

struct Fwd4 {
  int64_t nv, nelem, nedge, nbface, nbnode;
  const int32_t *elem;
  Coords4 X;
  const int32_t *elem_edge, *node_inc_off, *node_inc, *node_edge_off, *edge_tail, *edge_head;
  const int32_t *node_in_off, *node_in_edge;
  const int32_t *bface, *bface_edge, *node_bnode, *bnode, *bnode_face_off, *bnode_face;
  double *n[4];  // [4][n_edges] rows, or null
  double *b[4];  // [4][n_bnodes] rows, or null
  double *vol;   // or null
  double *term;  // per-edge terms of the edge loop
  StatusBlock *st;
};

__device__ __forceinline__ int32_t out_slot(const int32_t *heads, int32_t n, int32_t k) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (heads[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// the other vertices of incidence elem*5 + l, local order, l's place taken
// by vertex 4
__device__ __forceinline__ void others_of4(const int32_t (&v)[5], int l, int32_t (&o)[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) o[m] = l == m ? v[4] : v[m];
}

// gather forward, node pass: n over j's out-edges and V_j
__global__ __launch_bounds__(256) void k4_fwd_node(Fwd4 a) {
  const int64_t j64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j64 >= a.nv) return;
  const int32_t j = (int32_t)j64;
  const int32_t e0 = a.node_edge_off[j], nout = a.node_edge_off[j + 1] - e0;
  const bool want_n = a.n[0] != nullptr;
  if (want_n)
    for (int32_t s = 0; s < nout; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) a.n[c][e0 + s] = 0.0;
  const V4 Pj = load_pt4(a.X, j);
  double V = 0.0;
  for (int32_t r = a.node_inc_off[j]; r < a.node_inc_off[j + 1]; ++r) {
    const int32_t inc = a.node_inc[r];
    int32_t v[5], o[4];
    load_conn4(a.elem, inc / 5, v);
    others_of4(v, inc % 5, o);
    V4 Q[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) Q[m] = load_pt4(a.X, o[m]);
    double d;
    const V4 nj = pent_face(Pj, Q, d);  // d = 4|E|
    if (d == 0.0) raise_status(a.st, EB_EDEGENERATE, inc / 5);
    V += d * (1.0 / 20.0);
    if (want_n) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (o[m] <= j) continue;
        const int32_t e = e0 + out_slot(a.edge_head + e0, nout, o[m]);
#pragma unroll
        for (int c = 0; c < 4; ++c) a.n[c][e] += 0.1 * nj.c[c];
      }
    }
  }
  if (a.vol) a.vol[j] = V;
}

// gather forward, boundary pass: n_B/20 into j's out-edges of each boundary
// face B of j, b_j = sum n_B/4, in bnode_face order
__global__ __launch_bounds__(256) void k4_fwd_boundary(Fwd4 a) {
  const int64_t bj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bj >= a.nbnode) return;
  const int32_t j = a.bnode[bj];
  const int32_t e0 = a.node_edge_off[j], nout = a.node_edge_off[j + 1] - e0;
  double bs[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t r = a.bnode_face_off[bj]; r < a.bnode_face_off[bj + 1]; ++r) {
    const int32_t f = a.bnode_face[r];
    int32_t fv[4];
    V4 Q[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      fv[s] = a.bface[4 * (int64_t)f + s];
      Q[s] = load_pt4(a.X, fv[s]);
    }
    const V4 nB =
        v4_scale(1.0 / 6.0, v4_cross(v4_sub(Q[1], Q[0]), v4_sub(Q[2], Q[0]), v4_sub(Q[3], Q[0])));
#pragma unroll
    for (int c = 0; c < 4; ++c) bs[c] += 0.25 * nB.c[c];
    if (a.n[0]) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (fv[s] <= j) continue;
        const int32_t e = e0 + out_slot(a.edge_head + e0, nout, fv[s]);
#pragma unroll
        for (int c = 0; c < 4; ++c) a.n[c][e] += 0.05 * nB.c[c];
      }
    }
  }
  if (a.b[0])
#pragma unroll
    for (int c = 0; c < 4; ++c) a.b[c][bj] = bs[c];
}

// atomic forward: one thread per element
__global__ __launch_bounds__(256) void k4_fwd_atomic_elem(Fwd4 a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nelem) return;
  int32_t v[5];
  load_conn4(a.elem, e, v);
  V4 P[5], n[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) P[i] = load_pt4(a.X, v[i]);
  double d = 0.0;
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    V4 Q[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) Q[m] = P[t == m ? 4 : m];
    double dt;
    n[t] = pent_face(P[t], Q, dt);
    if (t == 0) d = dt;
  }
  if (d == 0.0) raise_status(a.st, EB_EDEGENERATE, e);
  if (a.n[0]) {
    int k = 0;
#pragma unroll
    for (int p = 0; p < 5; ++p)
#pragma unroll
      for (int q = p + 1; q < 5; ++q) {
        const V4 nt = v[p] < v[q] ? n[p] : n[q];
        const int32_t id = a.elem_edge[e * 10 + k++];
#pragma unroll
        for (int c = 0; c < 4; ++c) unsafeAtomicAdd(&a.n[c][id], 0.1 * nt.c[c]);
      }
  }
  if (a.vol)
#pragma unroll
    for (int i = 0; i < 5; ++i) unsafeAtomicAdd(&a.vol[v[i]], d * (1.0 / 20.0));
}

// atomic forward: one thread per boundary face
__global__ __launch_bounds__(256) void k4_fwd_atomic_bface(Fwd4 a) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= a.nbface) return;
  int32_t fv[4];
  V4 Q[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    fv[s] = a.bface[4 * f + s];
    Q[s] = load_pt4(a.X, fv[s]);
  }
  const V4 nB =
      v4_scale(1.0 / 6.0, v4_cross(v4_sub(Q[1], Q[0]), v4_sub(Q[2], Q[0]), v4_sub(Q[3], Q[0])));
  if (a.n[0])
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int32_t id = a.bface_edge[6 * f + k];
#pragma unroll
      for (int c = 0; c < 4; ++c) unsafeAtomicAdd(&a.n[c][id], 0.05 * nB.c[c]);
    }
  if (a.b[0])
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int32_t bi = a.node_bnode[fv[s]];
#pragma unroll
      for (int c = 0; c < 4; ++c) unsafeAtomicAdd(&a.b[c][bi], 0.25 * nB.c[c]);
    }
}

// edge loop: t_e = (x_head - x_tail).n_e / 8, then each node's ordered sum
// over its out-edges and in-edges (gather) or atomics at both ends
__device__ __forceinline__ double edge_term4(const Fwd4 &a, const double *const *n, int64_t e) {
  const V4 d = v4_sub(load_pt4(a.X, a.edge_head[e]), load_pt4(a.X, a.edge_tail[e]));
  return (d.c[0] * n[0][e] + d.c[1] * n[1][e] + d.c[2] * n[2][e] + d.c[3] * n[3][e]) *
         (1.0 / 8.0);
}

__global__ __launch_bounds__(256) void k4_vol_edge_terms(Fwd4 a, const double *n0,
                                                        const double *n1, const double *n2,
                                                        const double *n3) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nedge) return;
  const double *n[4] = {n0, n1, n2, n3};
  a.term[e] = edge_term4(a, n, e);
}

__global__ __launch_bounds__(256) void k4_vol_edge_sum(Fwd4 a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.nv) return;
  double V = 0.0;
  for (int32_t e = a.node_edge_off[j]; e < a.node_edge_off[j + 1]; ++e) V += a.term[e];
  for (int32_t r = a.node_in_off[j]; r < a.node_in_off[j + 1]; ++r) V += a.term[a.node_in_edge[r]];
  a.vol[j] = V;
}

__global__ __launch_bounds__(256) void k4_vol_edge_atomic(Fwd4 a, const double *n0,
                                                         const double *n1, const double *n2,
                                                         const double *n3) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nedge) return;
  const double *n[4] = {n0, n1, n2, n3};
  const double t = edge_term4(a, n, e);
  unsafeAtomicAdd(&a.vol[a.edge_tail[e]], t);
  unsafeAtomicAdd(&a.vol[a.edge_head[e]], t);
}

int pack4(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem, const double *coords,
          void *ws, size_t ws_bytes, Fwd4 &a) {
  EB_TRY(check_sizes(sz));
  EB_TRY(check_ws(sz->dim, sz->n_nodes, sz->n_elems, ws, ws_bytes));
  if (!tp || !coords || (sz->n_elems > 0 && !elem)) {
    set_detail("null pointer");
    return EB_EINVAL;
  }
  a = Fwd4{};
  a.nv = sz->n_nodes;
  a.nelem = sz->n_elems;
  a.nedge = sz->n_edges;
  a.nbface = sz->n_bfaces;
  a.nbnode = sz->n_bnodes;
  a.elem = elem;
  a.X = coords4_rows(coords, sz->n_nodes);
  a.elem_edge = tp->elem_edge;
  a.node_inc_off = tp->node_inc_off;
  a.node_inc = tp->node_inc;
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
  a.st = ws_at<StatusBlock>(ws, 0);
  return EB_OK;
}

void rows4(double *p, int64_t n, double *(&r)[4]) {
  for (int c = 0; c < 4; ++c) r[c] = p ? p + c * n : nullptr;
}

}  // namespace

int forward4(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem,
             const double *coords, int reduce, double *n_edge, double *b_node, double *vol,
             void *ws, size_t ws_bytes, hipStream_t s) {
  Fwd4 a;
  EB_TRY(pack4(sz, tp, elem, coords, ws, ws_bytes, a));
  if ((reduce != EB_REDUCE_ATOMIC && reduce != EB_REDUCE_GATHER) || !n_edge) {
    set_detail("bad reduce, or n_edge is null");
    return EB_EINVAL;
  }
  rows4(n_edge, sz->n_edges, a.n);
  rows4(sz->n_bnodes > 0 ? b_node : nullptr, sz->n_bnodes, a.b);
  a.vol = vol;
  EB_TRY(need(a.edge_head && a.node_edge_off, "edge, node_edge_off"));
  if (sz->n_bfaces > 0)
    EB_TRY(need(a.bface && a.bface_edge && a.node_bnode && a.bnode && a.bnode_face_off &&
                    a.bnode_face,
                "bface, bface_edge, node_bnode, bnode, bnode_face"));
  if (reduce == EB_REDUCE_ATOMIC) {
    EB_TRY(need(a.elem_edge != nullptr, "elem_edge"));
    for (int c = 0; c < 4; ++c) EB_TRY(fill_f64(a.n[c], sz->n_edges, 0.0, s));
    if (a.b[0])
      for (int c = 0; c < 4; ++c) EB_TRY(fill_f64(a.b[c], sz->n_bnodes, 0.0, s));
    if (a.vol) EB_TRY(fill_f64(a.vol, sz->n_nodes, 0.0, s));
    if (a.nelem > 0) {
      launch_principal(k4_fwd_atomic_elem, dim3(grid_for(a.nelem, 256)), dim3(256), 0, s, a);
      EB_LAUNCH_CHECK();
    }
    if (a.nbface > 0) {
      launch_span(k4_fwd_atomic_bface, dim3(grid_for(a.nbface, 256)), dim3(256), 0, s, a);
      EB_LAUNCH_CHECK();
    }
    return EB_OK;
  }
  EB_TRY(need(a.node_inc_off && a.node_inc, "node_inc"));
  launch_principal(k4_fwd_node, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a);
  EB_LAUNCH_CHECK();
  if (a.nbnode > 0) {
    launch_span(k4_fwd_boundary, dim3(grid_for(a.nbnode, 256)), dim3(256), 0, s, a);
    EB_LAUNCH_CHECK();
  }
  return EB_OK;
}

int volumes4(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem,
             const double *coords, int mode, const double *n_edge, int reduce, double *vol,
             void *ws, size_t ws_bytes, hipStream_t s) {
  Fwd4 a;
  EB_TRY(pack4(sz, tp, elem, coords, ws, ws_bytes, a));
  if ((mode != EB_VOL_ELEMENT && mode != EB_VOL_EDGE) ||
      (reduce != EB_REDUCE_ATOMIC && reduce != EB_REDUCE_GATHER) || !vol ||
      (mode == EB_VOL_EDGE && !n_edge)) {
    set_detail("bad mode / reduce, vol is null, or EB_VOL_EDGE without n_edge");
    return EB_EINVAL;
  }
  a.vol = vol;
  if (mode == EB_VOL_ELEMENT) {
    if (reduce == EB_REDUCE_ATOMIC) {
      EB_TRY(fill_f64(vol, sz->n_nodes, 0.0, s));
      if (a.nelem > 0) {
        launch_principal(k4_fwd_atomic_elem, dim3(grid_for(a.nelem, 256)), dim3(256), 0, s, a);
        EB_LAUNCH_CHECK();
      }
      return EB_OK;
    }
    EB_TRY(need(a.node_inc_off && a.node_inc, "node_inc"));
    launch_principal(k4_fwd_node, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a);
    EB_LAUNCH_CHECK();
    return EB_OK;
  }
  EB_TRY(need(a.edge_tail && a.edge_head, "edge"));
  const double *n[4];
  for (int c = 0; c < 4; ++c) n[c] = n_edge + c * sz->n_edges;
  if (reduce == EB_REDUCE_ATOMIC) {
    EB_TRY(fill_f64(vol, sz->n_nodes, 0.0, s));
    if (a.nedge > 0) {
      launch_principal(k4_vol_edge_atomic, dim3(grid_for(a.nedge, 256)), dim3(256), 0, s, a,
                       n[0], n[1], n[2], n[3]);
      EB_LAUNCH_CHECK();
    }
    return EB_OK;
  }
  EB_TRY(need(a.node_edge_off && a.node_in_off && a.node_in_edge, "node_edge_off, node_in"));
  // per-edge terms in the workspace's incidence-row region (80 bytes per
  // element there, against 8 per edge)
  a.term = ws_at<double>(ws, ws_layout(4, sz->n_nodes, sz->n_elems).rows4);
  if (a.nedge > 0) {
    launch_principal(k4_vol_edge_terms, dim3(grid_for(a.nedge, 256)), dim3(256), 0, s, a, n[0],
                     n[1], n[2], n[3]);
    EB_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k4_vol_edge_sum, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

}  // namespace eb
