// Device-side geometry helpers for the metric and adjoint kernels.
//
// Face-normal conventions (Section 3.2 of the paper writes the face area
// vectors for the orientation of its figures; here any local vertex order is
// accepted and the orientation comes from the sign s of the element's signed
// measure):
//   3D: s = sign det[x1-x0, x2-x0, x3-x0];
//       n_t = s * (1/2) (x_b - x_a) x (x_c - x_a) for (t,a,b,c) an even
//       permutation of (0,1,2,3): t=0:(1,2,3) t=1:(0,3,2) t=2:(0,1,3)
//       t=3:(0,2,1).  |E| = |det|/6 and sum_t n_t = 0.
//   2D: s = sign cross(x1-x0, x2-x0);
//       n_t = s * rot(x_c - x_b), b=(t+1)%3, c=(t+2)%3, rot(d) = (d_y, -d_x).
//       |E| = |cross|/2.
// n_t is the outward area vector of the face opposite local vertex t.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "eb_internal.h"

namespace eb {

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator-(V3 a) { return {-a.x, -a.y, -a.z}; }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
// V3 arithmetic never contracted into fused multiply-adds, so that it gives
// the same bits in every kernel it is inlined into
__device__ __forceinline__ V3 nc_add(V3 a, V3 b) {
#pragma clang fp contract(off)
  return {a.x + b.x, a.y + b.y, a.z + b.z};
}
__device__ __forceinline__ V3 nc_scale(double s, V3 a) {
#pragma clang fp contract(off)
  return {s * a.x, s * a.y, s * a.z};
}
__device__ __forceinline__ V3 nc_cross(V3 a, V3 b) {
#pragma clang fp contract(off)
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
// 2D: outward-rotated segment normal (d_y, -d_x); z stays 0
__device__ __forceinline__ V3 rot2(V3 d) { return {d.y, -d.x, 0.0}; }
// 2D: R(W) = (-W_y, W_x), the gradient of W.rot2(d) with respect to d
__device__ __forceinline__ V3 rotW(V3 w) { return {-w.y, w.x, 0.0}; }

template <int D> __device__ __forceinline__ V3 load_pt(const Coords &X, int32_t v) {
  if (D == 3) return {X.x[v], X.y[v], X.z[v]};
  return {X.x[v], X.y[v], 0.0};
}

template <int D> __device__ __forceinline__ void load_conn(const int32_t *elem, int64_t e,
                                                           int32_t (&v)[D + 1]) {
  if constexpr (D == 3) {
    int4 c = reinterpret_cast<const int4 *>(elem)[e];
    v[0] = c.x;
    v[1] = c.y;
    v[2] = c.z;
    v[3] = c.w;
  } else {
    const int32_t *p = elem + 3 * e;
    v[0] = p[0];
    v[1] = p[1];
    v[2] = p[2];
  }
}

// even-permutation faces of a tetrahedron: vertex k (0..2) of the face
// opposite local vertex t, ordered (a, b, c) so that (t, a, b, c) is an even
// permutation of (0, 1, 2, 3)
__device__ __forceinline__ int face3(int t, int k) {
  // rows: t=0 (1,2,3)  t=1 (0,3,2)  t=2 (0,1,3)  t=3 (0,2,1)
  const unsigned tab = (1u << 0) | (2u << 2) | (3u << 4) |      // t = 0
                       (0u << 6) | (3u << 8) | (2u << 10) |     // t = 1
                       (0u << 12) | (1u << 14) | (3u << 16) |   // t = 2
                       (0u << 18) | (2u << 20) | (1u << 22);    // t = 3
  return (tab >> (2 * (3 * t + k))) & 3u;
}

// The element's vertices other than local vertex l, in local order with l's
// place taken by the last vertex (o_m = v[m], except o_l = v[D]).  Written
// with selects on l, never an index, so nothing is placed in scratch memory.
template <int D>
__device__ __forceinline__ void others_of(const int32_t (&v)[D + 1], int l, int32_t (&o)[D]) {
#pragma unroll
  for (int m = 0; m < D; ++m) o[m] = (l == m) ? v[D] : v[m];
}

// out-edge slot m of a sliced-ELL slot code: 5-bit fields (narrow entries,
// 31 = none) or 10-bit fields (wide entries, 1023 = none)
template <bool WIDE> __device__ __forceinline__ int slot_of(uint32_t code, int m) {
  return WIDE ? (int)((code >> (10 * m)) & 1023u) : (int)((code >> (5 * m)) & 31u);
}
template <bool WIDE> constexpr int no_slot() { return WIDE ? 1023 : 31; }

template <int D> struct EL {
  static constexpr int NN = D + 1;
  static constexpr int NE = D * (D + 1) / 2;
};

template <int D> __device__ __forceinline__ int pair_p(int le) {
  if constexpr (D == 2) return le < 2 ? 0 : 1;
  else return le < 3 ? 0 : (le < 5 ? 1 : 2);
}
template <int D> __device__ __forceinline__ int pair_q(int le) {
  if constexpr (D == 2) return le == 0 ? 1 : 2;
  else {
    constexpr int q[6] = {1, 2, 3, 2, 3, 3};
    return q[le];
  }
}

// signed measure times D! (det), and the outward face normals n_t (true
// area vectors, i.e. with the 1/2 in 3D)
template <int D>
__device__ __forceinline__ double elem_normals(const V3 (&P)[D + 1], V3 (&n)[D + 1]) {
  if constexpr (D == 3) {
    const V3 a = P[1] - P[0], b = P[2] - P[0], c = P[3] - P[0];
    const double det = dot(a, cross(b, c));
    const double hs = det > 0 ? 0.5 : -0.5;
    n[0] = hs * cross(P[2] - P[1], P[3] - P[1]);
    n[1] = hs * cross(c, b);
    n[2] = hs * cross(a, c);
    n[3] = hs * cross(b, a);
    return det;
  } else {
    const V3 a = P[1] - P[0], b = P[2] - P[0];
    const double det = a.x * b.y - a.y * b.x;
    const double s = det > 0 ? 1.0 : -1.0;
    n[0] = s * rot2(P[2] - P[1]);
    n[1] = s * rot2(P[0] - P[2]);
    n[2] = s * rot2(P[1] - P[0]);
    return det;
  }
}

// ------------------------------------------------ LDS pre-aggregation
// The atomic paths scatter FP64 adds from elements into edges and nodes.  A
// block first sums its own adds per target id in an LDS table (open
// addressing, linear probing from id mod H: ids that arrive in contiguous
// runs, as the edges of consecutive elements do, land in consecutive slots,
// so the final device-scope adds of neighbouring slots go to neighbouring
// addresses), then issues one device-scope atomic per occupied slot and
// component.  An id that finds no slot within PROBES steps (a table filled
// by a block of scattered ids) is added to global memory directly.
// Elements per thread and LDS table sizes of the atomic element passes: a
// block takes ATOMIC_TB * ATOMIC_EPT consecutive elements; its edge table
// holds ATOMIC_HE slots and its node table ATOMIC_HV.
#ifndef EB_ATOMIC_EPT
#define EB_ATOMIC_EPT 2
#endif
constexpr int ATOMIC_TB = 256;
constexpr int ATOMIC_EPT = EB_ATOMIC_EPT;
constexpr int ATOMIC_HE = 1024 * ATOMIC_EPT;
constexpr int ATOMIC_HV = 512 * ATOMIC_EPT;

template <int H, int K> struct LdsAcc {
  static_assert((H & (H - 1)) == 0, "table size is a power of two");
  static constexpr int PROBES = 16;
  int32_t key[H];
  double acc[K][H];
};

template <int TB, int H, int K>
__device__ __forceinline__ void lds_acc_init(LdsAcc<H, K> &T, int t) {
  for (int s = t; s < H; s += TB) {
    T.key[s] = -1;
#pragma unroll
    for (int k = 0; k < K; ++k) T.acc[k][s] = 0.0;
  }
}

// slot of id in the table (inserted if new), or -1 when the probes run out
template <int H, int K>
__device__ __forceinline__ int lds_acc_slot(LdsAcc<H, K> &T, int32_t id) {
  int s = id & (H - 1);
  for (int p = 0; p < LdsAcc<H, K>::PROBES; ++p) {
    const int32_t k = __hip_atomic_load(&T.key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == id) return s;
    if (k == -1) {
      const int32_t old = atomicCAS(&T.key[s], -1, id);
      if (old == -1 || old == id) return s;
    }
    s = (s + 1) & (H - 1);
  }
  return -1;
}

// add v (K components) for id: into the table, or straight to out[k][id]
template <int H, int K>
__device__ __forceinline__ void lds_acc_add(LdsAcc<H, K> &T, double *const *out, int32_t id,
                                            const double (&v)[K]) {
  const int s = lds_acc_slot(T, id);
  if (s >= 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) atomicAdd(&T.acc[k][s], v[k]);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) unsafeAtomicAdd(&out[k][id], v[k]);
  }
}

// the table's sums to global memory (after a barrier)
template <int TB, int H, int K>
__device__ __forceinline__ void lds_acc_flush(const LdsAcc<H, K> &T, double *const *out, int t) {
  for (int s = t; s < H; s += TB) {
    const int32_t id = T.key[s];
    if (id >= 0)
#pragma unroll
      for (int k = 0; k < K; ++k) unsafeAtomicAdd(&out[k][id], T.acc[k][s]);
  }
}

}  // namespace eb
