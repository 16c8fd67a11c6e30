// Metrics of pentatope grids (dim = 4): the general-D formula of Section
// 3.2.3 with D = 4,
//   n_jk = 1/10 sum_{E contains jk} n_j^E + 1/20 sum_{B contains jk} n_B,
//   b_j  = 1/4 sum_{B contains j} n_B,
//   V_j  = sum_{E contains j} |E|/5      or   1/8 sum_k (x_k - x_j).n_jk,
// with n_j^E the outward area vector of the face of E opposite j (a
// tetrahedron) and n_B that of a boundary tetrahedron (eb_geom4.h).  The
// paper derives D = 2 and 3 and leaves D = 4 to future work.
//
// The gather forward takes tiles of 64 consecutive nodes, one wave each: a
// node's thread walks its node_inc row four incidences at a time (their
// connectivity and points loaded together; the points from a copy of the
// coordinates as 32-byte rows, made first in the workspace), forms the face vector opposite
// the node, and adds it to its out-edges' accumulators in LDS (the tile's
// out-edges are contiguous; a node's edge found among its first 16 heads,
// held in registers, or by binary search beyond), in row order; the tile's
// edges are written once.  A boundary pass, sixteen lanes per boundary
// node, follows.  The atomic forward sums each block's element contributions per
// edge and per node in LDS hash tables first, then adds each sum with one
// FP64 atomic, and its boundary faces likewise.
#include "eb_geom.h"  // (the LDS hash tables of the atomic pass)
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
  const double4 *xa;  // the points as 32-byte rows (node pass), or null
  StatusBlock *st;
};

// a point from the coordinate rows, or from its 32-byte row (two 16-byte
// loads on one line instead of four 8-byte loads on four)
template <bool AOS> __device__ __forceinline__ V4 node_pt4(const Fwd4 &a, int32_t v) {
  if constexpr (AOS) {
    const double4 p = a.xa[v];
    return {{p.x, p.y, p.z, p.w}};
  } else {
    return load_pt4(a.X, v);
  }
}

__global__ __launch_bounds__(256) void k4_points_rows(Coords4 X, int64_t nv, double4 *xa) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < nv) xa[j] = make_double4(X.x[j], X.y[j], X.z[j], X.w[j]);
}

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

// gather forward, node pass by tiles: TN = 64 nodes (one wave), their
// out-edges' raw sums (the face vectors; n = sum / 10) in LDS when the tile
// has at most CAP of them, else in the output itself; V_j = sum d / 20
constexpr int T4_TN = 64, T4_CAP = 1024, T4_HEADS = 16;

// add to a thread-owned LDS accumulator (only the owner adds to it, and a
// wave's LDS operations complete in order: the sum is in program order)
__device__ __forceinline__ void lds_add4(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <bool AOS>
__global__ __launch_bounds__(T4_TN) void k4_fwd_tile(Fwd4 a) {
  __shared__ double acc[4][T4_CAP];
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * T4_TN;
  const int64_t jend = min(j0 + (int64_t)T4_TN, a.nv);
  const bool want_n = a.n[0] != nullptr;
  const int32_t e0 = a.node_edge_off[j0];
  const int32_t cnt = a.node_edge_off[jend] - e0;
  const bool in_lds = want_n && cnt <= T4_CAP;
  if (in_lds)
    for (int i = t; i < cnt; i += T4_TN)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c][i] = 0.0;
  __syncthreads();
  const int64_t j64 = j0 + t;
  if (j64 < a.nv) {
    const int32_t j = (int32_t)j64;
    const int32_t my0 = a.node_edge_off[j], nout = a.node_edge_off[j + 1] - my0;
    const int32_t base = in_lds ? my0 - e0 : my0;
    if (want_n && !in_lds)
      for (int32_t s = 0; s < nout; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) a.n[c][my0 + s] = 0.0;
    // the first heads in registers: an edge's place is the number below it
    int32_t hd[T4_HEADS];
#pragma unroll
    for (int i = 0; i < T4_HEADS; ++i)
      hd[i] = i < nout ? a.edge_head[my0 + i] : INT32_MAX;
    const bool few = nout <= T4_HEADS;
    auto place = [&](int32_t k) __attribute__((always_inline)) {
      if (!few) return out_slot(a.edge_head + my0, nout, k);
      int32_t r = 0;
#pragma unroll
      for (int i = 0; i < T4_HEADS; ++i) r += hd[i] < k ? 1 : 0;
      return r;
    };
    auto add = [&](int32_t s, const V4 &v) __attribute__((always_inline)) {
      if (in_lds) {
#pragma unroll
        for (int c = 0; c < 4; ++c) lds_add4(&acc[c][base + s], v.c[c]);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) a.n[c][base + s] += v.c[c];
      }
    };
    const V4 Pj = node_pt4<AOS>(a, j);
    double V = 0.0;
    const int32_t r0 = a.node_inc_off[j], r1 = a.node_inc_off[j + 1];
    constexpr int U = 4;  // (LDS holds a CU to a few waves: more loads in flight each)
    for (int32_t r = r0; r < r1; r += U) {
      int32_t inc[U], v[U][5], o[U][4];
      V4 Q[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u) inc[u] = a.node_inc[min(r + u, r1 - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) load_conn4(a.elem, inc[u] / 5, v[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        others_of4(v[u], inc[u] % 5, o[u]);
#pragma unroll
        for (int m = 0; m < 4; ++m) Q[u][m] = node_pt4<AOS>(a, o[u][m]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (r + u >= r1) break;
        double d;
        const V4 nj = pent_face(Pj, Q[u], d);  // d = 4|E|
        if (d == 0.0) raise_status(a.st, EB_EDEGENERATE, inc[u] / 5);
        V += d * (1.0 / 20.0);
        if (want_n)
#pragma unroll
          for (int m = 0; m < 4; ++m)
            if (o[u][m] > j) add(place(o[u][m]), nj);
      }
    }
    if (a.vol) a.vol[j] = V;
    if (want_n && !in_lds)
      for (int32_t s = 0; s < nout; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) a.n[c][my0 + s] *= 0.1;
  }
  if (in_lds) {
    __syncthreads();
    for (int i = t; i < cnt; i += T4_TN)
#pragma unroll
      for (int c = 0; c < 4; ++c) a.n[c][e0 + i] = 0.1 * acc[c][i];
  }
}

// gather forward, boundary pass: B4_G lanes per boundary node (64 / B4_G
// nodes a wave).  A node's faces' n_B are formed a lane each, B4_CAP at a
// time staged in LDS; then a lane per out-edge adds n_B/20 of the faces
// holding the edge's head, in face order, and the group's first lane sums
// b_j = sum n_B/4 likewise: every output gets the additions, in the order,
// of a walk over the node's faces.
constexpr int B4_G = 16, B4_CAP = 32;

template <bool AOS>
__global__ __launch_bounds__(64) void k4_fwd_boundary(Fwd4 a) {
  __shared__ double snb[64 / B4_G][B4_CAP][4];
  __shared__ int32_t sfv[64 / B4_G][B4_CAP][4];
  const int t = threadIdx.x, grp = t / B4_G, g = t % B4_G;
  const int64_t bj = (int64_t)blockIdx.x * (64 / B4_G) + grp;
  const bool live = bj < a.nbnode;
  int32_t e0 = 0, nout = 0, f0 = 0, nf = 0;
  if (live) {
    const int32_t j = a.bnode[bj];
    e0 = a.node_edge_off[j];
    nout = a.node_edge_off[j + 1] - e0;
    f0 = a.bnode_face_off[bj];
    nf = a.bnode_face_off[bj + 1] - f0;
  }
  // as many chunks as the block's longest face list needs (every lane takes
  // every barrier)
  int32_t nch = (nf + B4_CAP - 1) / B4_CAP;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) nch = max(nch, __shfl_xor(nch, o, 64));
  const bool want_n = a.n[0] != nullptr;
  double bs[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t ch = 0; ch < nch; ++ch) {
    const int32_t c0 = ch * B4_CAP, m = min(nf - c0, B4_CAP);
    __syncthreads();  // (the previous chunk is used up)
    for (int32_t u = g; u < m; u += B4_G) {
      const int32_t f = a.bnode_face[f0 + c0 + u];
      V4 Q[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int32_t v = a.bface[4 * (int64_t)f + s];
        sfv[grp][u][s] = v;
        Q[s] = node_pt4<AOS>(a, v);
      }
      const V4 nB = v4_scale(
          1.0 / 6.0, v4_cross(v4_sub(Q[1], Q[0]), v4_sub(Q[2], Q[0]), v4_sub(Q[3], Q[0])));
#pragma unroll
      for (int c = 0; c < 4; ++c) snb[grp][u][c] = nB.c[c];
    }
    __syncthreads();
    if (g == 0)
      for (int32_t u = 0; u < m; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) bs[c] += 0.25 * snb[grp][u][c];
    if (want_n)
      for (int32_t s = g; s < nout; s += B4_G) {
        const int32_t h = a.edge_head[e0 + s];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        bool any = false;
        for (int32_t u = 0; u < m; ++u) {
          if (sfv[grp][u][0] != h && sfv[grp][u][1] != h && sfv[grp][u][2] != h &&
              sfv[grp][u][3] != h)
            continue;
          if (!any) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = a.n[c][e0 + s];
            any = true;
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[c] += 0.05 * snb[grp][u][c];
        }
        if (any)
#pragma unroll
          for (int c = 0; c < 4; ++c) a.n[c][e0 + s] = acc[c];
      }
  }
  if (live && g == 0 && a.b[0])
#pragma unroll
    for (int c = 0; c < 4; ++c) a.b[c][bj] = bs[c];
}

// atomic forward: one thread per element; a block's 256 consecutive
// elements sum their contributions per edge and per node in LDS hash tables
// (1024 edge, 256 node slots), then add each sum with one FP64 atomic
constexpr int A4_TB = 256, A4_HE = 1024, A4_HV = 256;

// one element's contributions into the block's tables
template <bool AOS>
__device__ __forceinline__ void elem4_sums(const Fwd4 &a, int64_t e, LdsAcc<A4_HE, 4> &te,
                                           LdsAcc<A4_HV, 1> &tv) {
  int32_t v[5];
  load_conn4(a.elem, e, v);
  V4 P[5], n[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) P[i] = node_pt4<AOS>(a, v[i]);
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
        const double c[4] = {0.1 * nt.c[0], 0.1 * nt.c[1], 0.1 * nt.c[2], 0.1 * nt.c[3]};
        lds_acc_add(te, a.n, id, c);
      }
  }
  if (a.vol) {
    double *const vout[1] = {a.vol};
    const double share[1] = {d * (1.0 / 20.0)};
#pragma unroll
    for (int i = 0; i < 5; ++i) lds_acc_add(tv, vout, v[i], share);
  }
}

template <bool AOS>
__global__ __launch_bounds__(A4_TB) void k4_fwd_atomic_elem(Fwd4 a) {
  __shared__ LdsAcc<A4_HE, 4> te;
  __shared__ LdsAcc<A4_HV, 1> tv;
  const int t = threadIdx.x;
  const bool want_n = a.n[0] != nullptr, want_v = a.vol != nullptr;
  double *const vout[1] = {a.vol};
  if (want_n) lds_acc_init<A4_TB>(te, t);
  if (want_v) lds_acc_init<A4_TB>(tv, t);
  __syncthreads();
  // a wave takes every fourth element of the block: neighbouring elements
  // (in a structured numbering, those of one cell, which share edges and
  // nodes) go to different waves, so fewer lanes of one LDS atomic
  // instruction hit the same slot
  const int64_t e = (int64_t)blockIdx.x * A4_TB + (t & 63) * (A4_TB / 64) + (t >> 6);
  if (e < a.nelem) elem4_sums<AOS>(a, e, te, tv);
  __syncthreads();
  if (want_n) lds_acc_flush<A4_TB>(te, a.n, t);
  if (want_v) lds_acc_flush<A4_TB>(tv, vout, t);
}

// atomic forward, boundary faces: a thread per face; a block's faces (in
// bface order, consecutive ones sharing most vertices) sum their n_B/20 per
// edge and n_B/4 per boundary node in LDS tables first, then add each sum
// with one FP64 atomic
constexpr int AB4_TB = 256, AB4_HE = 1024, AB4_HB = 256;

template <bool AOS>
__global__ __launch_bounds__(AB4_TB) void k4_fwd_atomic_bface(Fwd4 a) {
  __shared__ LdsAcc<AB4_HE, 4> te;
  __shared__ LdsAcc<AB4_HB, 4> tb;
  const int t = threadIdx.x;
  const bool want_n = a.n[0] != nullptr, want_b = a.b[0] != nullptr;
  if (want_n) lds_acc_init<AB4_TB>(te, t);
  if (want_b) lds_acc_init<AB4_TB>(tb, t);
  __syncthreads();
  const int64_t f = (int64_t)blockIdx.x * AB4_TB + t;
  if (f < a.nbface) {
    int32_t fv[4];
    V4 Q[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      fv[s] = a.bface[4 * f + s];
      Q[s] = node_pt4<AOS>(a, fv[s]);
    }
    const V4 nB =
        v4_scale(1.0 / 6.0, v4_cross(v4_sub(Q[1], Q[0]), v4_sub(Q[2], Q[0]), v4_sub(Q[3], Q[0])));
    if (want_n) {
      const double c[4] = {0.05 * nB.c[0], 0.05 * nB.c[1], 0.05 * nB.c[2], 0.05 * nB.c[3]};
#pragma unroll
      for (int k = 0; k < 6; ++k) lds_acc_add(te, a.n, a.bface_edge[6 * f + k], c);
    }
    if (want_b) {
      const double c[4] = {0.25 * nB.c[0], 0.25 * nB.c[1], 0.25 * nB.c[2], 0.25 * nB.c[3]};
#pragma unroll
      for (int s = 0; s < 4; ++s) lds_acc_add(tb, a.b, a.node_bnode[fv[s]], c);
    }
  }
  __syncthreads();
  if (want_n) lds_acc_flush<AB4_TB>(te, a.n, t);
  if (want_b) lds_acc_flush<AB4_TB>(tb, a.b, t);
}

// edge loop: t_e = (x_head - x_tail).n_e / 8, then each node's ordered sum
// over its out-edges and in-edges (gather) or atomics at both ends
template <bool AOS>
__device__ __forceinline__ double edge_term4(const Fwd4 &a, const double *const *n, int64_t e) {
  const V4 d = v4_sub(node_pt4<AOS>(a, a.edge_head[e]), node_pt4<AOS>(a, a.edge_tail[e]));
  return (d.c[0] * n[0][e] + d.c[1] * n[1][e] + d.c[2] * n[2][e] + d.c[3] * n[3][e]) *
         (1.0 / 8.0);
}

template <bool AOS>
__global__ __launch_bounds__(256) void k4_vol_edge_terms(Fwd4 a, const double *n0,
                                                        const double *n1, const double *n2,
                                                        const double *n3) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nedge) return;
  const double *n[4] = {n0, n1, n2, n3};
  a.term[e] = edge_term4<AOS>(a, n, e);
}

__global__ __launch_bounds__(256) void k4_vol_edge_sum(Fwd4 a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.nv) return;
  const double V = sum_terms<false>(0.0, a.term, a.node_edge_off[j], a.node_edge_off[j + 1]);
  a.vol[j] = sum_terms_at<false>(V, a.term, a.node_in_edge, a.node_in_off[j], a.node_in_off[j + 1]);
}

template <bool AOS>
__global__ __launch_bounds__(256) void k4_vol_edge_atomic(Fwd4 a, const double *n0,
                                                         const double *n1, const double *n2,
                                                         const double *n3) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nedge) return;
  const double *n[4] = {n0, n1, n2, n3};
  const double t = edge_term4<AOS>(a, n, e);
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

// the points copied as 32-byte rows into the workspace's incidence-row
// region (80 bytes per element, free once the build is done) when they fit
// there, past its first `skip` bytes (else null, and the kernels read the
// coordinate rows)
const double4 *point_rows4(const eb_sizes *sz, const Fwd4 &a, void *ws, hipStream_t s,
                           size_t skip = 0) {
  const WsLayout L = ws_layout(4, sz->n_nodes, sz->n_elems);
  if (skip + (size_t)32 * (size_t)sz->n_nodes > L.inc_pos - L.rows4) return nullptr;
  double4 *xa = ws_at<double4>(ws, L.rows4 + skip);
  launch_span(k4_points_rows, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a.X, a.nv, xa);
  return xa;
}

// the atomic element pass
int elem_pass4(const eb_sizes *sz, Fwd4 &a, void *ws, hipStream_t s) {
  a.xa = point_rows4(sz, a, ws, s);
  EB_LAUNCH_CHECK();
  if (a.xa)
    launch_principal(k4_fwd_atomic_elem<true>, dim3(grid_for(a.nelem, 256)), dim3(256), 0, s, a);
  else
    launch_principal(k4_fwd_atomic_elem<false>, dim3(grid_for(a.nelem, 256)), dim3(256), 0, s, a);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

// the gather node pass
int node_pass4(const eb_sizes *sz, Fwd4 &a, void *ws, hipStream_t s) {
  a.xa = point_rows4(sz, a, ws, s);
  EB_LAUNCH_CHECK();
  if (a.xa) {
    launch_principal(k4_fwd_tile<true>, dim3(grid_for(a.nv, T4_TN)), dim3(T4_TN), 0, s, a);
  } else {
    launch_principal(k4_fwd_tile<false>, dim3(grid_for(a.nv, T4_TN)), dim3(T4_TN), 0, s, a);
  }
  EB_LAUNCH_CHECK();
  return EB_OK;
}

}  // namespace

int forward4(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem,
             const double *coords, int reduce, double *n_edge, double *b_node, double *vol,
             void *ws, size_t ws_bytes, hipStream_t s) {
  Fwd4 a;
  EB_TRY(pack4(sz, tp, elem, coords, ws, ws_bytes, a));
  if (reduce != EB_REDUCE_ATOMIC && reduce != EB_REDUCE_GATHER) {
    set_detail("bad reduce, or n_edge is null");
    return EB_EINVAL;
  }
  if (no_elements(sz)) return vol ? fill_f64(vol, sz->n_nodes, 0.0, s) : EB_OK;
  if (!n_edge) {
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
    if (a.nelem > 0) EB_TRY(elem_pass4(sz, a, ws, s));
    if (a.nbface > 0) {
      if (a.xa)
        launch_span(k4_fwd_atomic_bface<true>, dim3(grid_for(a.nbface, 256)), dim3(256), 0, s, a);
      else
        launch_span(k4_fwd_atomic_bface<false>, dim3(grid_for(a.nbface, 256)), dim3(256), 0, s, a);
      EB_LAUNCH_CHECK();
    }
    return EB_OK;
  }
  EB_TRY(need(a.node_inc_off && a.node_inc, "node_inc"));
  EB_TRY(node_pass4(sz, a, ws, s));
  EB_LAUNCH_CHECK();
  if (a.nbnode > 0) {
    if (a.xa)
      launch_span(k4_fwd_boundary<true>, dim3(grid_for(a.nbnode, 64 / B4_G)), dim3(64), 0, s, a);
    else
      launch_span(k4_fwd_boundary<false>, dim3(grid_for(a.nbnode, 64 / B4_G)), dim3(64), 0, s, a);
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
      (reduce != EB_REDUCE_ATOMIC && reduce != EB_REDUCE_GATHER) || !vol) {
    set_detail("bad mode / reduce, vol is null, or EB_VOL_EDGE without n_edge");
    return EB_EINVAL;
  }
  if (no_elements(sz)) return fill_f64(vol, sz->n_nodes, 0.0, s);
  if (mode == EB_VOL_EDGE && !n_edge) {
    set_detail("bad mode / reduce, vol is null, or EB_VOL_EDGE without n_edge");
    return EB_EINVAL;
  }
  a.vol = vol;
  if (mode == EB_VOL_ELEMENT) {
    if (reduce == EB_REDUCE_ATOMIC) {
      EB_TRY(fill_f64(vol, sz->n_nodes, 0.0, s));
      if (a.nelem > 0) EB_TRY(elem_pass4(sz, a, ws, s));
      return EB_OK;
    }
    EB_TRY(need(a.node_inc_off && a.node_inc, "node_inc"));
    return node_pass4(sz, a, ws, s);
  }
  EB_TRY(need(a.edge_tail && a.edge_head, "edge"));
  const double *n[4];
  for (int c = 0; c < 4; ++c) n[c] = n_edge + c * sz->n_edges;
  if (reduce == EB_REDUCE_ATOMIC) {
    EB_TRY(fill_f64(vol, sz->n_nodes, 0.0, s));
    if (a.nedge > 0) {
      a.xa = point_rows4(sz, a, ws, s);
      EB_LAUNCH_CHECK();
      if (a.xa)
        launch_principal(k4_vol_edge_atomic<true>, dim3(grid_for(a.nedge, 256)), dim3(256), 0, s,
                         a, n[0], n[1], n[2], n[3]);
      else
        launch_principal(k4_vol_edge_atomic<false>, dim3(grid_for(a.nedge, 256)), dim3(256), 0,
                         s, a, n[0], n[1], n[2], n[3]);
      EB_LAUNCH_CHECK();
    }
    return EB_OK;
  }
  EB_TRY(need(a.node_edge_off && a.node_in_off && a.node_in_edge, "node_edge_off, node_in"));
  // per-edge terms in the workspace's incidence-row region (80 bytes per
  // element there, against 8 per edge), the point rows after them
  a.term = ws_at<double>(ws, ws_layout(4, sz->n_nodes, sz->n_elems).rows4);
  if (a.nedge > 0) {
    a.xa = point_rows4(sz, a, ws, s, align256(sizeof(double) * (size_t)a.nedge));
    EB_LAUNCH_CHECK();
    if (a.xa)
      launch_principal(k4_vol_edge_terms<true>, dim3(grid_for(a.nedge, 256)), dim3(256), 0, s, a,
                       n[0], n[1], n[2], n[3]);
    else
      launch_principal(k4_vol_edge_terms<false>, dim3(grid_for(a.nedge, 256)), dim3(256), 0, s,
                       a, n[0], n[1], n[2], n[3]);
    EB_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k4_vol_edge_sum, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

}  // namespace eb
