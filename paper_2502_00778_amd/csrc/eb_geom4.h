// Device-side geometry of pentatopes (dim = 4), the general-D formula of
// Section 3.2.3 one dimension beyond the paper's 2D and 3D derivations.
//
// The area vector of a tetrahedron {a, b, c, d} in R^4 is
// (1/6) N(b-a, c-a, d-a), with N(u, v, w) the four-dimensional cross
// product: the vector with N.x = det[x; u; v; w] for every x (cofactor
// expansion along the first row).  The outward area vector n_t of the face
// of a pentatope opposite local vertex t is that of its other four vertices,
// oriented so that n_t.(x_a - x_t) > 0 for a vertex a of the face; then
// |E| = n_t.(x_a - x_t)/4, sum_t n_t = 0 and det[x1-x0, ..., x4-x0] = +-24|E|.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "eb_internal.h"

namespace eb {

struct V4 {
  double c[4];
};

__device__ __forceinline__ V4 v4_sub(const V4 &a, const V4 &b) {
  return {{a.c[0] - b.c[0], a.c[1] - b.c[1], a.c[2] - b.c[2], a.c[3] - b.c[3]}};
}
__device__ __forceinline__ V4 v4_scale(double s, const V4 &a) {
  return {{s * a.c[0], s * a.c[1], s * a.c[2], s * a.c[3]}};
}
__device__ __forceinline__ V4 v4_add(const V4 &a, const V4 &b) {
  return {{a.c[0] + b.c[0], a.c[1] + b.c[1], a.c[2] + b.c[2], a.c[3] + b.c[3]}};
}
__device__ __forceinline__ double v4_dot(const V4 &a, const V4 &b) {
  return a.c[0] * b.c[0] + a.c[1] * b.c[1] + a.c[2] * b.c[2] + a.c[3] * b.c[3];
}
// determinant of columns (i, j, k) of the rows u, v, w
__device__ __forceinline__ double v4_minor(const V4 &u, const V4 &v, const V4 &w, int i, int j,
                                           int k) {
  return u.c[i] * (v.c[j] * w.c[k] - v.c[k] * w.c[j]) -
         u.c[j] * (v.c[i] * w.c[k] - v.c[k] * w.c[i]) +
         u.c[k] * (v.c[i] * w.c[j] - v.c[j] * w.c[i]);
}
__device__ __forceinline__ V4 v4_cross(const V4 &u, const V4 &v, const V4 &w) {
  return {{v4_minor(u, v, w, 1, 2, 3), -v4_minor(u, v, w, 0, 2, 3), v4_minor(u, v, w, 0, 1, 3),
           -v4_minor(u, v, w, 0, 1, 2)}};
}

struct Coords4 {
  const double *x, *y, *z, *w;
};
inline Coords4 coords4_rows(const double *c, int64_t nv) {
  return Coords4{c, c + nv, c + 2 * nv, c + 3 * nv};
}
__device__ __forceinline__ V4 load_pt4(const Coords4 &X, int32_t v) {
  return {{X.x[v], X.y[v], X.z[v], X.w[v]}};
}
__device__ __forceinline__ void load_conn4(const int32_t *elem, int64_t e, int32_t (&v)[5]) {
  const int32_t *p = elem + 5 * e;
#pragma unroll
  for (int i = 0; i < 5; ++i) v[i] = p[i];
}

// det[x1-x0, x2-x0, x3-x0, x4-x0] = (x1-x0).N(x2-x0, x3-x0, x4-x0)
__device__ __forceinline__ double pent_det(const V4 (&P)[5]) {
  return v4_dot(v4_sub(P[1], P[0]),
                v4_cross(v4_sub(P[2], P[0]), v4_sub(P[3], P[0]), v4_sub(P[4], P[0])));
}

// Outward area vector of the face opposite local vertex t (face vertices
// o[0..3], any order) and d = n_t.(x_{o0} - x_t) = 4|E|.
__device__ __forceinline__ V4 pent_face(const V4 &Pt, const V4 (&Q)[4], double &d) {
  V4 n = v4_scale(1.0 / 6.0, v4_cross(v4_sub(Q[1], Q[0]), v4_sub(Q[2], Q[0]), v4_sub(Q[3], Q[0])));
  d = v4_dot(n, v4_sub(Q[0], Pt));
  if (d < 0) {
    n = v4_scale(-1.0, n);
    d = -d;
  }
  return n;
}

}  // namespace eb
