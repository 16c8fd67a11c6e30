// Adjoint device code shared by the adjoint kernels and the fused
// forward + adjoint kernel.
//
// For a loss L = sum_e w_e.n_e + sum_j c_j V_j + sum_j beta_j.b_j the
// forward formulas give, per element E (orientation sign s held fixed),
//   L_E = sum_t W_t.n_t + C_E |E|,
//   W_t = 2/(D(D+1)) * sum of w_e over the local edges whose tail is t,
//   C_E = (1/(D+1)) sum_{i in E} c_i,
// and per boundary element B
//   L_B = W_B.n_B,  W_B = 1/(D(D+1)) sum_{e in B} w_e + (1/D) sum_{i in B} beta_i.
// Derivatives (3D, face (a,b,c) in cyclic outward order, N = s/2 (x_b-x_a) x
// (x_c-x_a)):  d(W.N)/dx_a = s/2 (x_b - x_c) x W, and cyclically;
//        (2D, N = s rot(x_c - x_b), rot(d) = (d_y, -d_x)):
//              d(W.N)/dx_c = s R(W), d(W.N)/dx_b = -s R(W), R(W) = (-W_y, W_x);
// and d|E|/dx_i = -n_i/D (moving a vertex against its opposite face's
// outward normal grows the element).
#pragma once

#include "eb_geom.h"
#include "eb_kernels.h"

namespace eb {

template <int D>
__device__ __forceinline__ V3 load_row3(const double *x, const double *y, const double *z,
                                        int64_t i) {
  if (D == 3) return {x[i], y[i], z[i]};
  return {x[i], y[i], 0.0};
}

// W_t for every local vertex t and C_E of element e.  All indices are
// compile-time constants (the tail of each local edge is chosen with a
// select), so nothing lands in scratch memory.
template <int D>
__device__ __forceinline__ void elem_weights(const FwdArgs &a, int64_t e, const int32_t (&v)[D + 1],
                                             V3 (&W)[D + 1], double &C) {
  constexpr int NE = EL<D>::NE;
  constexpr double kN = 2.0 / (D * (D + 1));
#pragma unroll
  for (int t = 0; t <= D; ++t) W[t] = {0.0, 0.0, 0.0};
  if (a.w_x) {
    // the element's edge ids (3D: 24 bytes, 8-byte aligned: three 2-word loads)
    int32_t eid[NE];
    if constexpr (D == 3) {
      const int2 *q2 = reinterpret_cast<const int2 *>(a.elem_edge + e * NE);
#pragma unroll
      for (int k = 0; k < NE / 2; ++k) {
        const int2 x = q2[k];
        eid[2 * k] = x.x;
        eid[2 * k + 1] = x.y;
      }
    } else {
#pragma unroll
      for (int le = 0; le < NE; ++le) eid[le] = a.elem_edge[e * NE + le];
    }
#pragma unroll
    for (int le = 0; le < NE; ++le) {
      const int p = pair_p<D>(le), q = pair_q<D>(le);
      const int32_t ed = eid[le];
      const V3 w = kN * load_row3<D>(a.w_x, a.w_y, a.w_z, ed);
      const V3 z = {0.0, 0.0, 0.0};
      const bool tail_p = v[p] < v[q];
      W[p] = W[p] + (tail_p ? w : z);
      W[q] = W[q] + (tail_p ? z : w);
    }
  }
  C = 0.0;
  if (a.c) {
#pragma unroll
    for (int i = 0; i <= D; ++i) C += a.c[v[i]];
    C *= 1.0 / (D + 1);
  }
}

// dL_E/dx_i for every local vertex i (compile-time indices only)
template <int D>
__device__ __forceinline__ void elem_grad_all(const V3 (&P)[D + 1], const V3 (&n)[D + 1], double det,
                                              const V3 (&W)[D + 1], double C, V3 (&G)[D + 1]) {
#pragma unroll
  for (int i = 0; i <= D; ++i) G[i] = (-C / D) * n[i];
  if constexpr (D == 3) {
    const double hs = det > 0 ? 0.5 : -0.5;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int fa = face3(t, 0), fb = face3(t, 1), fc = face3(t, 2);
      G[fa] = G[fa] + hs * cross(P[fb] - P[fc], W[t]);
      G[fb] = G[fb] + hs * cross(P[fc] - P[fa], W[t]);
      G[fc] = G[fc] + hs * cross(P[fa] - P[fb], W[t]);
    }
  } else {
    const double s = det > 0 ? 1.0 : -1.0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const V3 R = s * rotW(W[t]);
      const int b = (t + 1) % 3, c = (t + 2) % 3;
      G[c] = G[c] + R;
      G[b] = G[b] - R;
    }
  }
}

// the entry of G[] at runtime index l, by masked sums (no indexed access)
template <int N>
__device__ __forceinline__ V3 pick(const V3 (&G)[N], int l) {
  V3 r = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double m = (l == i) ? 1.0 : 0.0;
    r = r + m * G[i];
  }
  return r;
}

template <int D>
__device__ __forceinline__ V3 bface_weight(const FwdArgs &a, int64_t f, const int32_t (&fv)[D]) {
  constexpr int NBE = D == 2 ? 1 : 3;
  V3 W = {0.0, 0.0, 0.0};
  if (a.w_x) {
    constexpr double kB = 1.0 / (D * (D + 1));
#pragma unroll
    for (int i = 0; i < NBE; ++i) {
      const int32_t ed = a.bface_edge[f * NBE + i];
      W = W + kB * load_row3<D>(a.w_x, a.w_y, a.w_z, ed);
    }
  }
  if (a.be_x) {
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int32_t bi = a.node_bnode[fv[s]];
      W = W + (1.0 / D) * load_row3<D>(a.be_x, a.be_y, a.be_z, bi);
    }
  }
  return W;
}

// d(W.n_B)/dx of every face vertex
template <int D>
__device__ __forceinline__ void bface_grad_all(const V3 (&P)[D], V3 W, V3 (&G)[D]) {
  if constexpr (D == 3) {
    G[0] = 0.5 * cross(P[1] - P[2], W);
    G[1] = 0.5 * cross(P[2] - P[0], W);
    G[2] = 0.5 * cross(P[0] - P[1], W);
  } else {
    const V3 R = rotW(W);
    G[1] = R;
    G[0] = -R;
  }
}

// ------------------------------------------------------------- gather path
//
// Two passes, no atomics.  The element pass forms dL_E/dx_i for every vertex
// i of element E once and stores it at the sliced slot of incidence (E, i)
// (inc_sell: column = rank of the incidence in node_inc's row), so the pieces
// of node j's column sit slice-major, 64 lanes side by side.  The node pass
// then sums j's column in node_inc order with coalesced loads, and the
// boundary pass adds j's boundary faces in bnode_face order.

// element pass: the pieces of element e
template <int D>
__device__ __forceinline__ void bwd_elem_piece(const FwdArgs &a, int64_t e) {
  int32_t v[D + 1], pos[D + 1];
  load_conn<D>(a.elem, e, v);
  load_conn<D>(a.inc_sell, e, pos);
  V3 P[D + 1], n[D + 1], W[D + 1];
#pragma unroll
  for (int i = 0; i <= D; ++i) P[i] = load_pt<D>(a.X, v[i]);
  const double det = elem_normals<D>(P, n);
  double C;
  elem_weights<D>(a, e, v, W, C);
  V3 G[D + 1];
  elem_grad_all<D>(P, n, det, W, C, G);
  // one row per component: 8 bytes a slot, no padding
#pragma unroll
  for (int l = 0; l <= D; ++l) {
    double *q = a.gpiece + pos[l];
    q[0] = G[l].x;
    q[a.gstride] = G[l].y;
    if constexpr (D == 3) q[2 * a.gstride] = G[l].z;
  }
}

// node pass: dL/dx_j from the pieces of j's elements
template <int D>
__device__ __forceinline__ void bwd_node_sum(const FwdArgs &a, int64_t j) {
  const int32_t len = a.node_inc_off[j + 1] - a.node_inc_off[j];
  const double *q = a.gpiece + ((int64_t)a.node_sell_off[j / SELL] + (j % SELL));
  const int64_t gs = a.gstride;
  V3 g = {0.0, 0.0, 0.0};
  // one accumulator, fixed order: the result does not depend on unrolling
#pragma unroll 4
  for (int32_t r = 0; r < len; ++r) {
    const int64_t k = (int64_t)SELL * r;
    g = g + V3{q[k], q[gs + k], D == 3 ? q[2 * gs + k] : 0.0};
  }
  a.g_x[j] = g.x;
  a.g_y[j] = g.y;
  if (D == 3) a.g_z[j] = g.z;
}

// boundary pass: the boundary faces of boundary node bj, added after the
// node pass.  Faces are taken two per round with every load of a round issued
// before the first face is formed (an absent weight array is replaced by entry
// 0 of the coordinates, loaded and not used, so no load sits behind a branch);
// the weights and the faces' terms are summed in the same order as face by face.
template <int D>
__device__ __forceinline__ void bwd_boundary_node(const FwdArgs &a, int64_t bj) {
  constexpr int NBE = D == 2 ? 1 : 3, G = 2;
  constexpr double kB = 1.0 / (D * (D + 1));
  const int32_t j = a.bnode[bj];
  const int32_t r0 = a.bnode_face_off[bj], r1 = a.bnode_face_off[bj + 1];
  const bool have_w = a.w_x != nullptr, have_be = a.be_x != nullptr;
  const double *wx = have_w ? a.w_x : a.X.x, *wy = have_w ? a.w_y : a.X.x;
  const double *wz = have_w ? a.w_z : a.X.x;
  const double *bx = have_be ? a.be_x : a.X.x, *by = have_be ? a.be_y : a.X.x;
  const double *bz = have_be ? a.be_z : a.X.x;
  V3 g = {0.0, 0.0, 0.0};
  for (int32_t r = r0; r < r1; r += G) {
    int32_t f[G], fv[G][D], ed[G][NBE], bi[G][D];
#pragma unroll
    for (int u = 0; u < G; ++u) f[u] = a.bnode_face[min(r + u, r1 - 1)];
#pragma unroll
    for (int u = 0; u < G; ++u) {
#pragma unroll
      for (int s = 0; s < D; ++s) fv[u][s] = a.bface[(int64_t)f[u] * D + s];
#pragma unroll
      for (int i = 0; i < NBE; ++i) ed[u][i] = a.bface_edge[(int64_t)f[u] * NBE + i];
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int s = 0; s < D; ++s) bi[u][s] = a.node_bnode[fv[u][s]];
    V3 P[G][D], Wl[G][NBE], Bl[G][D];
#pragma unroll
    for (int u = 0; u < G; ++u) {
#pragma unroll
      for (int s = 0; s < D; ++s) P[u][s] = load_pt<D>(a.X, fv[u][s]);
#pragma unroll
      for (int i = 0; i < NBE; ++i) Wl[u][i] = load_row3<D>(wx, wy, wz, have_w ? ed[u][i] : 0);
#pragma unroll
      for (int s = 0; s < D; ++s) Bl[u][s] = load_row3<D>(bx, by, bz, have_be ? bi[u][s] : 0);
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (r + u >= r1) break;
      V3 W = {0.0, 0.0, 0.0};
      if (have_w)
#pragma unroll
        for (int i = 0; i < NBE; ++i) W = W + kB * Wl[u][i];
      if (have_be)
#pragma unroll
        for (int s = 0; s < D; ++s) W = W + (1.0 / D) * Bl[u][s];
      int p = 0;
#pragma unroll
      for (int s = 0; s < D; ++s)
        if (fv[u][s] == j) p = s;
      V3 Gr[D];
      bface_grad_all<D>(P[u], W, Gr);
      g = g + pick(Gr, p);
    }
  }
  a.g_x[j] += g.x;
  a.g_y[j] += g.y;
  if (D == 3) a.g_z[j] += g.z;
}

// Elements [blk * TB * EPT, (blk + 1) * TB * EPT) by a block of TB threads:
// dL_E/dx_i for each vertex, summed per node in the LDS table T (barriers
// inside: the whole block calls it) and added to the zeroed gradient with
// one FP64 atomic per distinct node and component.
template <int D, int TB, int EPT_, int H>
__device__ __forceinline__ void bwd_atomic_elem_block(const FwdArgs &a, int64_t blk,
                                                      LdsAcc<H, D> &T) {
  const int t = threadIdx.x;
  double *const gout[3] = {a.g_x, a.g_y, a.g_z};
  lds_acc_init<TB>(T, t);
  __syncthreads();
  const int64_t e0 = blk * TB * EPT_;
#pragma unroll
  for (int k = 0; k < EPT_; ++k) {
    const int64_t e = e0 + (int64_t)k * TB + t;
    if (e >= a.nelem) break;
    int32_t v[D + 1];
    load_conn<D>(a.elem, e, v);
    V3 P[D + 1], n[D + 1], W[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) P[i] = load_pt<D>(a.X, v[i]);
    const double det = elem_normals<D>(P, n);
    double C;
    elem_weights<D>(a, e, v, W, C);
    V3 G[D + 1];
    elem_grad_all<D>(P, n, det, W, C, G);
#pragma unroll
    for (int l = 0; l <= D; ++l) {
      double c[D];
      c[0] = G[l].x;
      c[1] = G[l].y;
      if constexpr (D == 3) c[D - 1] = G[l].z;
      lds_acc_add(T, gout, v[l], c);
    }
  }
  __syncthreads();
  lds_acc_flush<TB>(T, gout, t);
}

// One boundary face's adjoint terms G[p] for its vertices fv[p].
template <int D>
__device__ __forceinline__ void bwd_bface_terms(const FwdArgs &a, int64_t f, int32_t (&fv)[D],
                                                V3 (&G)[D]) {
  V3 P[D];
#pragma unroll
  for (int s = 0; s < D; ++s) {
    fv[s] = a.bface[f * D + s];
    P[s] = load_pt<D>(a.X, fv[s]);
  }
  bface_grad_all<D>(P, bface_weight<D>(a, f, fv), G);
}

// One boundary face's adjoint terms, added with FP64 atomics.
template <int D>
__device__ __forceinline__ void bwd_atomic_bface_one(const FwdArgs &a, int64_t f) {
  int32_t fv[D];
  V3 G[D];
  bwd_bface_terms<D>(a, f, fv, G);
#pragma unroll
  for (int p = 0; p < D; ++p) {
    unsafeAtomicAdd(&a.g_x[fv[p]], G[p].x);
    unsafeAtomicAdd(&a.g_y[fv[p]], G[p].y);
    if (D == 3) unsafeAtomicAdd(&a.g_z[fv[p]], G[p].z);
  }
}

}  // namespace eb
