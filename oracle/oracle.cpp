// CPU ORACLE for the edge-based grid metrics — TEST INFRASTRUCTURE ONLY.
//
// Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
// load this library.  The GPU library never links it, and it shares no code,
// header, table or helper with the GPU kernels.
//
// What it computes: the grid metrics of the node-centred edge-based scheme
// (Nishikawa, "An Efficient Implementation of Edge-Based Discretization
// without Forming Dual Control Volumes", Section 2, eq.
// threed_fv_semidiscrete_system_00), by the TRADITIONAL route that the paper
// replaces: the median dual is formed explicitly, element by element.
//
//   * n_jk  lumped directed-area vector of edge {j,k}, j<k (Section 2: edges
//           run from the smaller node number), = sum over the elements that
//           share the edge of the area vectors of the median-dual faces that
//           separate j's cell from k's cell inside the element:
//             2D: the segment edge midpoint -> element centroid (Section 3.1.1)
//             3D: the two triangles {m, E, L} and {m, R, E} (Section 3.1.2)
//   * V_j   median-dual volume: sum over E containing j of the part of E that
//           is nearer to j in the barycentric sense, cut along midpoints and
//           centroids (Sections 1-2, the median dual control volume).  It is
//           tiled here by triangles (2D) or tetrahedra (3D) fanned from x_j.
//   * b_j   outward area vector of the boundary part of j's dual cell: on
//           every boundary element B containing j, the piece of B cut off by
//           its edge midpoints and centroid (Section 3.2.3, boundary closure).
//
// Every accumulation is a Neumaier-compensated sum taken in a fixed order
// (element ascending, then local index), so serial and threaded runs give the
// same bits.  Orientation is decided by dot products with edge or height
// vectors, never by an assumed vertex order (the paper's formulas assume the
// orientation of its figures; any local order is accepted here).
//
// The scalar type is a template parameter so that the same construction, run
// on forward-mode dual numbers, gives the exact derivative of a linear loss
// with respect to one node's coordinates (reference gradient for the adjoint).
//
// Topology (edges, element->edge map, boundary faces, node->element lists) is
// built with std::sort over explicit keys; it fixes the integer layout the GPU
// library must reproduce bit for bit:
//   edge        [2][Ne]  SoA, tails then heads, ascending (tail, head)
//   elem_edge   [NE][ne] local pairs 2D (0,1)(0,2)(1,2); 3D (0,1)(0,2)(0,3)(1,2)(1,3)(2,3)
//   elem_edge_sign [NE][ne]  +1 iff elem[p] < elem[q]
//   edge_inc    CSR over edges of elem*ne+local, ascending
//   node_inc    CSR over nodes of elem*(D+1)+local, ascending
//   node_edge_off  CSR offsets of edges by tail
//   node_in     CSR over nodes of the ids of edges whose head is the node
//   bface       [NB][D] faces owned by one element, in ascending sorted-id
//               order, vertices ordered so the area vector points out of the
//               domain (3D rotated to put the smallest id first)
//   bface_owner [NB] elem*(D+1)+local index of the vertex opposite the face
//   bface_edge  [NB][D(D-1)/2] ids of edges (v0,v1) | (v0,v1),(v0,v2),(v1,v2)
//   bnode       sorted ids of nodes on boundary faces; node_bnode its inverse
//   bnode_face  CSR over bnodes of bface ids, ascending
//
// Parity pins (tests/test_oracle_pins.py): closure at every node, sum of V
// equals the domain volume, hand-derivable single-triangle / single-tet /
// 6-tet-cube values, the paper's efficient formula evaluated in exact
// rationals, exact-rational recomputation of the construction, invariances.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#include <parallel/algorithm>
#endif

namespace {

enum {
  OR_OK = 0,
  OR_EINVAL = -1,
  OR_ERANGE = -2,
  OR_EDEGENERATE = -3,
  OR_ENONMANIFOLD = -4,
  OR_EOVERFLOW = -6,
};

// ---------------------------------------------------------------- scalars

struct Dual {  // value plus derivative along 3 seeded directions
  double v;
  double d[3];
};
inline Dual mk(double v) { return Dual{v, {0, 0, 0}}; }
inline Dual operator+(Dual a, Dual b) {
  return Dual{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
}
inline Dual operator-(Dual a, Dual b) {
  return Dual{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
}
inline Dual operator-(Dual a) { return Dual{-a.v, {-a.d[0], -a.d[1], -a.d[2]}}; }
inline Dual operator*(Dual a, Dual b) {
  return Dual{a.v * b.v,
              {a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1],
               a.d[2] * b.v + a.v * b.d[2]}};
}
inline Dual operator*(double s, Dual a) {
  return Dual{s * a.v, {s * a.d[0], s * a.d[1], s * a.d[2]}};
}
inline double val(double x) { return x; }
inline double val(const Dual &x) { return x.v; }

template <class T> struct P3 { T x, y, z; };
template <class T> inline P3<T> operator+(P3<T> a, P3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> inline P3<T> operator-(P3<T> a, P3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> inline P3<T> operator-(P3<T> a) { return {-a.x, -a.y, -a.z}; }
template <class T> inline P3<T> scale(double s, P3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> inline P3<T> cross(P3<T> a, P3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> inline T dot(P3<T> a, P3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
// plane rotation by +90 degrees: (a, b) -> (-b, a); z unused in 2D
template <class T> inline P3<T> rot90(P3<T> a) { return {-a.y, a.x, a.z - a.z}; }
template <class T> inline T absval(T x) { return val(x) < 0 ? -x : x; }
template <class T> inline P3<T> orient_along(P3<T> t, P3<T> dir) {
  return val(dot(t, dir)) < 0 ? -t : t;
}

struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double get() const { return s + c; }
};

// ------------------------------------------------------- local numbering

const int PAIR2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
const int PAIR3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int PAIR4[10][2] = {{0, 1}, {0, 2}, {0, 3}, {0, 4}, {1, 2},
                          {1, 3}, {1, 4}, {2, 3}, {2, 4}, {3, 4}};

inline int n_local_edges(int dim) { return dim == 2 ? 3 : (dim == 3 ? 6 : 10); }
inline const int (*local_pairs(int dim))[2] {
  return dim == 2 ? PAIR2 : (dim == 3 ? PAIR3 : PAIR4);
}

template <class T> inline P3<T> point(const T *const *X, int dim, int64_t v) {
  P3<T> p;
  p.x = X[0][v];
  p.y = X[1][v];
  p.z = dim == 3 ? X[2][v] : X[0][v] - X[0][v];
  return p;
}

// -------------------------------------------- traditional element pieces
//
// For one element with vertex positions P[0..D] and global ids id[0..D]:
//   npiece[le]  area vector of the median-dual face inside the element that
//               separates the two ends of local edge le, oriented from the
//               smaller global id to the larger one;
//   vpiece[i]   volume of the part of the element belonging to vertex i.

template <class T>
void tri_pieces(const P3<T> P[3], const int32_t id[3], P3<T> npiece[3], T vpiece[3]) {
  const P3<T> C = scale(1.0 / 3.0, P[0] + P[1] + P[2]);  // element centroid
  for (int le = 0; le < 3; ++le) {
    int p = PAIR2[le][0], q = PAIR2[le][1];
    int j = id[p] < id[q] ? p : q;
    int k = j == p ? q : p;
    P3<T> m = scale(0.5, P[j] + P[k]);          // edge midpoint
    P3<T> t = rot90(C - m);                     // normal of segment m -> C
    npiece[le] = orient_along(t, P[k] - P[j]);  // points from j to k
  }
  for (int i = 0; i < 3; ++i) {
    // j's quadrilateral {x_i, m_ia, C, m_ib} as two triangles fanned from x_i
    T acc = P[0].x - P[0].x;
    for (int a = 0; a < 3; ++a) {
      if (a == i) continue;
      P3<T> m = scale(0.5, P[i] + P[a]);
      P3<T> u = m - P[i], w = C - P[i];
      acc = acc + 0.5 * absval(u.x * w.y - u.y * w.x);
    }
    vpiece[i] = acc;
  }
}

template <class T>
void tet_pieces(const P3<T> P[4], const int32_t id[4], P3<T> npiece[6], T vpiece[4]) {
  const P3<T> C = scale(0.25, P[0] + P[1] + P[2] + P[3]);  // element centroid
  for (int le = 0; le < 6; ++le) {
    int p = PAIR3[le][0], q = PAIR3[le][1];
    int o[2], no = 0;
    for (int r = 0; r < 4; ++r)
      if (r != p && r != q) o[no++] = r;
    int j = id[p] < id[q] ? p : q;
    int k = j == p ? q : p;
    P3<T> m = scale(0.5, P[j] + P[k]);                            // edge midpoint
    P3<T> L = scale(1.0 / 3.0, P[p] + P[q] + P[o[0]]);            // face centroid
    P3<T> R = scale(1.0 / 3.0, P[p] + P[q] + P[o[1]]);            // face centroid
    P3<T> dir = P[k] - P[j];
    P3<T> t1 = orient_along(scale(0.5, cross(C - m, L - m)), dir);  // {m, E, L}
    P3<T> t2 = orient_along(scale(0.5, cross(R - m, C - m)), dir);  // {m, R, E}
    npiece[le] = t1 + t2;
  }
  for (int i = 0; i < 4; ++i) {
    // the sub-cell of vertex i is the cone from x_i over its three interior
    // dual quads {m_ia, F, C, F'}; each quad splits into two triangles
    // {m_ia, F, C}, giving six tetrahedra {x_i, m_ia, F, C}
    T acc = P[0].x - P[0].x;
    for (int a = 0; a < 4; ++a) {
      if (a == i) continue;
      P3<T> m = scale(0.5, P[i] + P[a]);
      for (int b = 0; b < 4; ++b) {
        if (b == i || b == a) continue;
        P3<T> F = scale(1.0 / 3.0, P[i] + P[a] + P[b]);  // face {i,a,b}
        T det = dot(m - P[i], cross(F - P[i], C - P[i]));
        acc = acc + (1.0 / 6.0) * absval(det);
      }
    }
    vpiece[i] = acc;
  }
}

// Boundary piece of vertex s of boundary element B (vertices V[0..D-1], with
// Xo the owner's vertex opposite B): outward area vector of the part of B cut
// off at x_s by the midpoints of B's edges at s and B's centroid.
template <class T>
P3<T> bface_piece(int dim, const P3<T> *V, int s, P3<T> Xo) {
  const P3<T> Xi = V[s];
  const P3<T> out = Xi - Xo;  // any vector from the inside to the face
  if (dim == 2) {
    P3<T> m = scale(0.5, V[0] + V[1]);
    return orient_along(rot90(m - Xi), out);
  }
  P3<T> F = scale(1.0 / 3.0, V[0] + V[1] + V[2]);
  int a = (s + 1) % 3, b = (s + 2) % 3;
  P3<T> ma = scale(0.5, Xi + V[a]);
  P3<T> mb = scale(0.5, Xi + V[b]);
  P3<T> t1 = orient_along(scale(0.5, cross(ma - Xi, F - Xi)), out);
  P3<T> t2 = orient_along(scale(0.5, cross(F - Xi, mb - Xi)), out);
  return t1 + t2;
}

// ------------------------------------------------ four dimensions (D = 4)
//
// The same traditional construction one dimension up (the paper derives the
// efficient formula for general D, Section 3.2.3, and leaves D = 4 to future
// work).  The median dual cuts an element along the barycentres of its
// faces: the part of E where lambda_p = lambda_q >= every other barycentric
// coordinate is the dual face between p and q, and the part where lambda_i
// is largest is i's sub-cell.  Both are unions of simplices of the
// barycentric subdivision, one per chain of faces:
//   dual face (p,q):  {m_pq, F_pqa, T_pqab, C} over ordered pairs (a,b) of
//                     the other three vertices (six tetrahedra, all in the
//                     hyperplane lambda_p = lambda_q);
//   sub-cell of i:    {x_i, m_ia, F_iab, T_iabc, C} over ordered triples
//                     (a,b,c) of the other four (24 pentatopes);
//   boundary piece of vertex s of a boundary tetrahedron B:
//                     {x_s, m_sa, F_sab, C_B} over ordered pairs (a,b) of
//                     B's other vertices (six tetrahedra in B's hyperplane);
// with m, F, T, C the barycentres of edges, triangles, tetrahedra and the
// element.  The area vector of a tetrahedron {y0,y1,y2,y3} in R^4 is
// (1/6) N(y1-y0, y2-y0, y3-y0), where N(u,v,w) is the vector with
// N(u,v,w).x = det[x; u; v; w] for every x (the four-dimensional cross
// product); it is oriented here by a dot product, like the 2D/3D pieces.

struct Q4 {
  double c[4];
};
inline Q4 q4_add(const Q4 &a, const Q4 &b) {
  return {{a.c[0] + b.c[0], a.c[1] + b.c[1], a.c[2] + b.c[2], a.c[3] + b.c[3]}};
}
inline Q4 q4_sub(const Q4 &a, const Q4 &b) {
  return {{a.c[0] - b.c[0], a.c[1] - b.c[1], a.c[2] - b.c[2], a.c[3] - b.c[3]}};
}
inline Q4 q4_scale(double s, const Q4 &a) {
  return {{s * a.c[0], s * a.c[1], s * a.c[2], s * a.c[3]}};
}
inline double q4_dot(const Q4 &a, const Q4 &b) {
  return a.c[0] * b.c[0] + a.c[1] * b.c[1] + a.c[2] * b.c[2] + a.c[3] * b.c[3];
}
// 3x3 determinant of columns (i, j, k) of the rows u, v, w
inline double minor3(const Q4 &u, const Q4 &v, const Q4 &w, int i, int j, int k) {
  return u.c[i] * (v.c[j] * w.c[k] - v.c[k] * w.c[j]) -
         u.c[j] * (v.c[i] * w.c[k] - v.c[k] * w.c[i]) +
         u.c[k] * (v.c[i] * w.c[j] - v.c[j] * w.c[i]);
}
// N(u,v,w): cofactor expansion of det[x; u; v; w] along its first row
inline Q4 q4_cross(const Q4 &u, const Q4 &v, const Q4 &w) {
  return {{minor3(u, v, w, 1, 2, 3), -minor3(u, v, w, 0, 2, 3), minor3(u, v, w, 0, 1, 3),
           -minor3(u, v, w, 0, 1, 2)}};
}
inline double q4_det(const Q4 &a, const Q4 &b, const Q4 &c, const Q4 &d) {
  return q4_dot(a, q4_cross(b, c, d));
}
inline Q4 q4_along(const Q4 &t, const Q4 &dir) {
  return q4_dot(t, dir) < 0 ? q4_scale(-1.0, t) : t;
}
inline Q4 point4(const double *const *X, int64_t v) {
  return {{X[0][v], X[1][v], X[2][v], X[3][v]}};
}
// area vector of the tetrahedron {y0, y1, y2, y3}, up to orientation
inline Q4 tet_area4(const Q4 &y0, const Q4 &y1, const Q4 &y2, const Q4 &y3) {
  return q4_scale(1.0 / 6.0, q4_cross(q4_sub(y1, y0), q4_sub(y2, y0), q4_sub(y3, y0)));
}

void pent_pieces(const Q4 P[5], const int32_t id[5], Q4 npiece[10], double vpiece[5]) {
  const Q4 C = q4_scale(0.2, q4_add(q4_add(q4_add(P[0], P[1]), q4_add(P[2], P[3])), P[4]));
  for (int le = 0; le < 10; ++le) {
    const int p = PAIR4[le][0], q = PAIR4[le][1];
    int o[3], no = 0;
    for (int r = 0; r < 5; ++r)
      if (r != p && r != q) o[no++] = r;
    const int j = id[p] < id[q] ? p : q, k = j == p ? q : p;
    const Q4 m = q4_scale(0.5, q4_add(P[p], P[q]));
    const Q4 dir = q4_sub(P[k], P[j]);
    Q4 sum = {{0, 0, 0, 0}};
    for (int ia = 0; ia < 3; ++ia)
      for (int ib = 0; ib < 3; ++ib) {
        if (ib == ia) continue;
        const int a = o[ia], b = o[ib];
        const Q4 F = q4_scale(1.0 / 3.0, q4_add(q4_add(P[p], P[q]), P[a]));
        const Q4 T = q4_scale(0.25, q4_add(q4_add(P[p], P[q]), q4_add(P[a], P[b])));
        sum = q4_add(sum, q4_along(tet_area4(m, F, T, C), dir));
      }
    npiece[le] = sum;
  }
  for (int i = 0; i < 5; ++i) {
    double acc = 0.0;
    for (int a = 0; a < 5; ++a) {
      if (a == i) continue;
      const Q4 m = q4_scale(0.5, q4_add(P[i], P[a]));
      for (int b = 0; b < 5; ++b) {
        if (b == i || b == a) continue;
        const Q4 F = q4_scale(1.0 / 3.0, q4_add(q4_add(P[i], P[a]), P[b]));
        for (int c = 0; c < 5; ++c) {
          if (c == i || c == a || c == b) continue;
          const Q4 T = q4_scale(0.25, q4_add(q4_add(P[i], P[a]), q4_add(P[b], P[c])));
          const double det = q4_det(q4_sub(m, P[i]), q4_sub(F, P[i]), q4_sub(T, P[i]),
                                    q4_sub(C, P[i]));
          acc += std::fabs(det) / 24.0;
        }
      }
    }
    vpiece[i] = acc;
  }
}

// Boundary piece of vertex s of the boundary tetrahedron V[0..3] (Xo: the
// owner's vertex opposite it), oriented out of the domain.
Q4 bface_piece4(const Q4 V[4], int s, const Q4 &Xo) {
  const Q4 CB = q4_scale(0.25, q4_add(q4_add(V[0], V[1]), q4_add(V[2], V[3])));
  const Q4 out = q4_sub(V[s], Xo);
  Q4 sum = {{0, 0, 0, 0}};
  for (int a = 0; a < 4; ++a) {
    if (a == s) continue;
    const Q4 m = q4_scale(0.5, q4_add(V[s], V[a]));
    for (int b = 0; b < 4; ++b) {
      if (b == s || b == a) continue;
      const Q4 F = q4_scale(1.0 / 3.0, q4_add(q4_add(V[s], V[a]), V[b]));
      sum = q4_add(sum, q4_along(tet_area4(V[s], m, F, CB), out));
    }
  }
  return sum;
}

// --------------------------------------------------------------- topology

struct Topo {
  int dim = 0;
  int64_t nv = 0, nelem = 0, nedge = 0, nbface = 0, nbnode = 0;
  std::vector<int32_t> edge;  // [2][nedge]
  std::vector<int32_t> node_edge_off, elem_edge, edge_inc_off, edge_inc;
  std::vector<int8_t> elem_edge_sign;
  std::vector<int32_t> node_inc_off, node_inc, node_in_off, node_in_edge;
  std::vector<int32_t> bface, bface_owner, bface_edge, bnode, node_bnode;
  std::vector<int32_t> bnode_face_off, bnode_face;
};

template <class It, class Cmp> void sort_range(It b, It e, Cmp c) {
#ifdef _OPENMP
  __gnu_parallel::sort(b, e, c);
#else
  std::sort(b, e, c);
#endif
}

struct KeyPay {
  uint64_t key;
  uint32_t pay;
};
inline bool kp_less(const KeyPay &a, const KeyPay &b) {
  return a.key != b.key ? a.key < b.key : a.pay < b.pay;
}

// CSR of (row, value) pairs, rows in [0, nrow), values ascending within a row
void csr_from_pairs(std::vector<KeyPay> &kp, int64_t nrow, std::vector<int32_t> &off,
                    std::vector<int32_t> &val) {
  sort_range(kp.begin(), kp.end(), kp_less);
  off.assign(nrow + 1, 0);
  val.resize(kp.size());
  for (size_t i = 0; i < kp.size(); ++i) {
    off[kp[i].key + 1]++;
    val[i] = (int32_t)kp[i].pay;
  }
  for (int64_t r = 0; r < nrow; ++r) off[r + 1] += off[r];
}

int32_t find_edge(const Topo &t, int32_t a, int32_t b) {
  int32_t lo = std::min(a, b), hi = std::max(a, b);
  const int32_t *heads = t.edge.data() + t.nedge;
  const int32_t *beg = heads + t.node_edge_off[lo], *end = heads + t.node_edge_off[lo + 1];
  const int32_t *it = std::lower_bound(beg, end, hi);
  if (it == end || *it != hi) return -1;
  return (int32_t)(it - heads);
}

int build_topology(Topo &t, int dim, int64_t nv, int64_t nelem, const int32_t *elem,
                   const double *const *X) {
  const int nn = dim + 1, ne = n_local_edges(dim);
  const int (*pairs)[2] = local_pairs(dim);
  t.dim = dim;
  t.nv = nv;
  t.nelem = nelem;
  // validation: ids in range, nonzero measure
  for (int64_t e = 0; e < nelem; ++e)
    for (int i = 0; i < nn; ++i) {
      int32_t v = elem[e * nn + i];
      if (v < 0 || v >= nv) return OR_ERANGE;
    }
  for (int64_t e = 0; e < nelem; ++e) {
    const int32_t *c = elem + e * nn;
    double det;
    if (dim == 4) {
      Q4 Q[5];
      for (int i = 0; i < 5; ++i) Q[i] = point4(X, c[i]);
      det = q4_det(q4_sub(Q[1], Q[0]), q4_sub(Q[2], Q[0]), q4_sub(Q[3], Q[0]), q4_sub(Q[4], Q[0]));
    } else {
      P3<double> P[4];
      for (int i = 0; i < nn; ++i) P[i] = point(X, dim, c[i]);
      det = dim == 2 ? (P[1].x - P[0].x) * (P[2].y - P[0].y) - (P[1].y - P[0].y) * (P[2].x - P[0].x)
                     : dot(P[1] - P[0], cross(P[2] - P[0], P[3] - P[0]));
    }
    if (det == 0.0) return OR_EDEGENERATE;
  }

  // edges: key (min << 32 | max), payload elem*ne + local
  std::vector<KeyPay> kp((size_t)nelem * ne);
  for (int64_t e = 0; e < nelem; ++e)
    for (int l = 0; l < ne; ++l) {
      int32_t a = elem[e * nn + pairs[l][0]], b = elem[e * nn + pairs[l][1]];
      uint64_t lo = (uint64_t)std::min(a, b), hi = (uint64_t)std::max(a, b);
      kp[e * ne + l] = KeyPay{(lo << 32) | hi, (uint32_t)(e * ne + l)};
    }
  sort_range(kp.begin(), kp.end(), kp_less);
  std::vector<int32_t> tails, heads;
  t.edge_inc.resize(kp.size());
  t.edge_inc_off.clear();
  t.elem_edge.assign((size_t)nelem * ne, -1);
  t.elem_edge_sign.assign((size_t)nelem * ne, 0);
  for (size_t i = 0; i < kp.size(); ++i) {
    if (i == 0 || kp[i].key != kp[i - 1].key) {
      tails.push_back((int32_t)(kp[i].key >> 32));
      heads.push_back((int32_t)(kp[i].key & 0xffffffffu));
      t.edge_inc_off.push_back((int32_t)i);
    }
    t.edge_inc[i] = (int32_t)kp[i].pay;
    t.elem_edge[kp[i].pay] = (int32_t)(tails.size() - 1);
  }
  t.edge_inc_off.push_back((int32_t)kp.size());
  t.nedge = (int64_t)tails.size();
  t.edge.resize(2 * t.nedge);
  std::copy(tails.begin(), tails.end(), t.edge.begin());
  std::copy(heads.begin(), heads.end(), t.edge.begin() + t.nedge);
  for (int64_t e = 0; e < nelem; ++e)
    for (int l = 0; l < ne; ++l)
      t.elem_edge_sign[e * ne + l] = elem[e * nn + pairs[l][0]] < elem[e * nn + pairs[l][1]] ? 1 : -1;
  kp.clear();
  kp.shrink_to_fit();
  t.node_edge_off.assign(nv + 1, 0);
  for (int64_t i = 0; i < t.nedge; ++i) t.node_edge_off[tails[i] + 1]++;
  for (int64_t v = 0; v < nv; ++v) t.node_edge_off[v + 1] += t.node_edge_off[v];

  // edges by head
  {
    std::vector<KeyPay> hp(t.nedge);
    for (int64_t i = 0; i < t.nedge; ++i) hp[i] = KeyPay{(uint64_t)heads[i], (uint32_t)i};
    csr_from_pairs(hp, nv, t.node_in_off, t.node_in_edge);
  }
  // node -> element incidences
  {
    std::vector<KeyPay> np((size_t)nelem * nn);
    for (int64_t e = 0; e < nelem; ++e)
      for (int i = 0; i < nn; ++i)
        np[e * nn + i] = KeyPay{(uint64_t)elem[e * nn + i], (uint32_t)(e * nn + i)};
    csr_from_pairs(np, nv, t.node_inc_off, t.node_inc);
  }

  // faces: sorted vertex ids of the face opposite each local vertex
  struct FaceKey {
    int32_t v[4];  // ascending; unused places -1
    uint32_t pay;
  };
  auto face_less = [](const FaceKey &a, const FaceKey &b) {
    for (int i = 0; i < 4; ++i)
      if (a.v[i] != b.v[i]) return a.v[i] < b.v[i];
    return a.pay < b.pay;
  };
  std::vector<FaceKey> fk((size_t)nelem * nn);
  for (int64_t e = 0; e < nelem; ++e)
    for (int f = 0; f < nn; ++f) {
      FaceKey k{{-1, -1, -1, -1}, (uint32_t)(e * nn + f)};
      int c = 0;
      for (int i = 0; i < nn; ++i)
        if (i != f) k.v[c++] = elem[e * nn + i];
      std::sort(k.v, k.v + dim);
      fk[e * nn + f] = k;
    }
  sort_range(fk.begin(), fk.end(), face_less);
  t.bface.clear();
  t.bface_owner.clear();
  for (size_t i = 0; i < fk.size();) {
    size_t j = i + 1;
    while (j < fk.size() && std::equal(fk[j].v, fk[j].v + 4, fk[i].v)) ++j;
    if (j - i > 2) return OR_ENONMANIFOLD;
    if (j - i == 1) {
      uint32_t pay = fk[i].pay;
      int64_t e = pay / nn;
      int f = pay % nn;
      if (dim == 4) {
        // keep the ascending order when its area vector N(b-a, c-a, d-a)
        // points away from the opposite vertex, else swap the last two (an
        // odd permutation flips it); the smallest id stays first
        const int32_t *v = fk[i].v;
        const Q4 A = point4(X, v[0]), Xo4 = point4(X, elem[e * nn + f]);
        const double s4 = q4_dot(q4_cross(q4_sub(point4(X, v[1]), A), q4_sub(point4(X, v[2]), A),
                                          q4_sub(point4(X, v[3]), A)),
                                 q4_sub(A, Xo4));
        if (s4 == 0) return OR_EDEGENERATE;
        t.bface.push_back(v[0]);
        t.bface.push_back(v[1]);
        t.bface.push_back(s4 > 0 ? v[2] : v[3]);
        t.bface.push_back(s4 > 0 ? v[3] : v[2]);
        t.bface_owner.push_back((int32_t)pay);
        i = j;
        continue;
      }
      P3<double> Xo = point(X, dim, elem[e * nn + f]);
      P3<double> A = point(X, dim, fk[i].v[0]), B = point(X, dim, fk[i].v[1]);
      bool keep;
      if (dim == 2) {
        // outward normal of segment a->b is (dy, -dx): keep a->b when it
        // points away from the opposite vertex
        P3<double> d = B - A, w = A - Xo;
        double s = d.y * w.x - d.x * w.y;
        keep = s > 0;
        if (s == 0) return OR_EDEGENERATE;
      } else {
        P3<double> Cc = point(X, dim, fk[i].v[2]);
        double s = dot(cross(B - A, Cc - A), A - Xo);
        keep = s > 0;
        if (s == 0) return OR_EDEGENERATE;
      }
      if (dim == 2) {
        t.bface.push_back(keep ? fk[i].v[0] : fk[i].v[1]);
        t.bface.push_back(keep ? fk[i].v[1] : fk[i].v[0]);
      } else {
        t.bface.push_back(fk[i].v[0]);
        t.bface.push_back(keep ? fk[i].v[1] : fk[i].v[2]);
        t.bface.push_back(keep ? fk[i].v[2] : fk[i].v[1]);
      }
      t.bface_owner.push_back((int32_t)pay);
    }
    i = j;
  }
  t.nbface = (int64_t)t.bface_owner.size();
  // edges of each boundary element: its vertex pairs in lexicographic order
  const int nbe = dim * (dim - 1) / 2;
  const int (*bpairs)[2] = local_pairs(dim - 1);
  t.bface_edge.resize(t.nbface * nbe);
  for (int64_t f = 0; f < t.nbface; ++f) {
    const int32_t *v = &t.bface[f * dim];
    if (dim == 2) {
      t.bface_edge[f] = find_edge(t, v[0], v[1]);
    } else {
      for (int i = 0; i < nbe; ++i)
        t.bface_edge[f * nbe + i] = find_edge(t, v[bpairs[i][0]], v[bpairs[i][1]]);
    }
  }
  // boundary nodes
  std::vector<int32_t> bn(t.bface);
  std::sort(bn.begin(), bn.end());
  bn.erase(std::unique(bn.begin(), bn.end()), bn.end());
  t.bnode = bn;
  t.nbnode = (int64_t)bn.size();
  t.node_bnode.assign(nv, -1);
  for (int64_t i = 0; i < t.nbnode; ++i) t.node_bnode[bn[i]] = (int32_t)i;
  {
    std::vector<KeyPay> bp(t.nbface * dim);
    for (int64_t f = 0; f < t.nbface; ++f)
      for (int s = 0; s < dim; ++s)
        bp[f * dim + s] = KeyPay{(uint64_t)t.node_bnode[t.bface[f * dim + s]], (uint32_t)f};
    csr_from_pairs(bp, t.nbnode, t.bnode_face_off, t.bnode_face);
  }
  return OR_OK;
}

// ------------------------------------------------------- piece evaluation

void element_pieces_d(int dim, const double *const *X, const int32_t *elem, int64_t e,
                      double *np_out /*[ne][dim]*/, double *vp_out /*[dim+1]*/) {
  const int nn = dim + 1;
  const int32_t *c = elem + e * nn;
  if (dim == 4) {
    Q4 Q[5], nq[10];
    for (int i = 0; i < 5; ++i) Q[i] = point4(X, c[i]);
    pent_pieces(Q, c, nq, vp_out);
    for (int l = 0; l < 10; ++l)
      for (int k = 0; k < 4; ++k) np_out[l * 4 + k] = nq[l].c[k];
    return;
  }
  P3<double> P[4], npc[6];
  double vpc[4];
  for (int i = 0; i < nn; ++i) P[i] = point(X, dim, c[i]);
  if (dim == 2)
    tri_pieces(P, c, npc, vpc);
  else
    tet_pieces(P, c, npc, vpc);
  const int ne = n_local_edges(dim);
  for (int l = 0; l < ne; ++l) {
    np_out[l * dim + 0] = npc[l].x;
    np_out[l * dim + 1] = npc[l].y;
    if (dim == 3) np_out[l * dim + 2] = npc[l].z;
  }
  for (int i = 0; i < nn; ++i) vp_out[i] = vpc[i];
}

void bface_pieces_d(int dim, const double *const *X, const Topo &t, const int32_t *elem,
                    int64_t f, double *out /*[dim][dim]: vertex s, component*/) {
  const int nn = dim + 1;
  if (dim == 4) {
    Q4 V4[4];
    for (int s = 0; s < 4; ++s) V4[s] = point4(X, t.bface[f * 4 + s]);
    const int32_t own4 = t.bface_owner[f];
    const Q4 Xo4 = point4(X, elem[(int64_t)(own4 / nn) * nn + own4 % nn]);
    for (int s = 0; s < 4; ++s) {
      const Q4 p = bface_piece4(V4, s, Xo4);
      for (int k = 0; k < 4; ++k) out[s * 4 + k] = p.c[k];
    }
    return;
  }
  P3<double> V[3];
  for (int s = 0; s < dim; ++s) V[s] = point(X, dim, t.bface[f * dim + s]);
  int32_t own = t.bface_owner[f];
  P3<double> Xo = point(X, dim, elem[(int64_t)(own / nn) * nn + own % nn]);
  for (int s = 0; s < dim; ++s) {
    P3<double> p = bface_piece(dim, V, s, Xo);
    out[s * dim + 0] = p.x;
    out[s * dim + 1] = p.y;
    if (dim == 3) out[s * dim + 2] = p.z;
  }
}

}  // namespace

// =================================================================== C ABI

extern "C" {

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Element pieces of elements [e0, e1): npiece [e1-e0][ne][dim], vpiece [e1-e0][dim+1].
int oracle_element_pieces(int dim, int64_t nv, const double *coords, int64_t e0, int64_t e1,
                          const int32_t *elem, double *npiece, double *vpiece) {
  if (dim < 2 || dim > 4) return OR_EINVAL;
  const double *X[4] = {coords, coords + nv, dim >= 3 ? coords + 2 * nv : coords,
                        dim == 4 ? coords + 3 * nv : coords};
  const int ne = n_local_edges(dim), nn = dim + 1;
#pragma omp parallel for schedule(static)
  for (int64_t e = e0; e < e1; ++e)
    element_pieces_d(dim, X, elem, e, npiece + (e - e0) * ne * dim, vpiece + (e - e0) * nn);
  return OR_OK;
}

// Boundary piece of one boundary face given explicitly: vertices face[dim]
// (outward order), opposite vertex position taken from node `opp`.
int oracle_bface_piece(int dim, int64_t nv, const double *coords, const int32_t *face,
                       int32_t opp, double *out /*[dim][dim]*/) {
  if (dim != 2 && dim != 3) return OR_EINVAL;
  const double *X[4] = {coords, coords + nv, dim >= 3 ? coords + 2 * nv : coords,
                        dim == 4 ? coords + 3 * nv : coords};
  P3<double> V[3];
  for (int s = 0; s < dim; ++s) V[s] = point(X, dim, face[s]);
  P3<double> Xo = point(X, dim, opp);
  for (int s = 0; s < dim; ++s) {
    P3<double> p = bface_piece(dim, V, s, Xo);
    out[s * dim + 0] = p.x;
    out[s * dim + 1] = p.y;
    if (dim == 3) out[s * dim + 2] = p.z;
  }
  return OR_OK;
}

void *oracle_topo_new(void) { return new (std::nothrow) Topo(); }
void oracle_topo_free(void *h) { delete static_cast<Topo *>(h); }

int oracle_topology(void *h, int dim, int64_t nv, int64_t nelem, const int32_t *elem,
                    const double *coords) {
  if (!h || dim < 2 || dim > 4 || nv <= 0 || nelem < 0) return OR_EINVAL;
  if ((int64_t)n_local_edges(dim) * nelem >= ((int64_t)1 << 31)) return OR_EOVERFLOW;
  if (nv >= ((int64_t)1 << 31)) return OR_EOVERFLOW;
  const double *X[4] = {coords, coords + nv, dim >= 3 ? coords + 2 * nv : coords,
                        dim == 4 ? coords + 3 * nv : coords};
  return build_topology(*static_cast<Topo *>(h), dim, nv, nelem, elem, X);
}

// sizes: dim, nv, nelem, nedge, nbface, nbnode
void oracle_topo_sizes(const void *h, int64_t *out) {
  const Topo &t = *static_cast<const Topo *>(h);
  out[0] = t.dim;
  out[1] = t.nv;
  out[2] = t.nelem;
  out[3] = t.nedge;
  out[4] = t.nbface;
  out[5] = t.nbnode;
}

// Copy one named array out; returns element count, or -1 for an unknown name.
// A NULL destination only reports the count.
int64_t oracle_topo_get(const void *h, const char *name, void *dst) {
  const Topo &t = *static_cast<const Topo *>(h);
  struct Item {
    const char *n;
    const void *p;
    size_t count, bytes;
  };
  const Item items[] = {
      {"edge", t.edge.data(), t.edge.size(), 4},
      {"node_edge_off", t.node_edge_off.data(), t.node_edge_off.size(), 4},
      {"elem_edge", t.elem_edge.data(), t.elem_edge.size(), 4},
      {"elem_edge_sign", t.elem_edge_sign.data(), t.elem_edge_sign.size(), 1},
      {"edge_inc_off", t.edge_inc_off.data(), t.edge_inc_off.size(), 4},
      {"edge_inc", t.edge_inc.data(), t.edge_inc.size(), 4},
      {"node_inc_off", t.node_inc_off.data(), t.node_inc_off.size(), 4},
      {"node_inc", t.node_inc.data(), t.node_inc.size(), 4},
      {"node_in_off", t.node_in_off.data(), t.node_in_off.size(), 4},
      {"node_in_edge", t.node_in_edge.data(), t.node_in_edge.size(), 4},
      {"bface", t.bface.data(), t.bface.size(), 4},
      {"bface_owner", t.bface_owner.data(), t.bface_owner.size(), 4},
      {"bface_edge", t.bface_edge.data(), t.bface_edge.size(), 4},
      {"bnode", t.bnode.data(), t.bnode.size(), 4},
      {"node_bnode", t.node_bnode.data(), t.node_bnode.size(), 4},
      {"bnode_face_off", t.bnode_face_off.data(), t.bnode_face_off.size(), 4},
      {"bnode_face", t.bnode_face.data(), t.bnode_face.size(), 4},
  };
  for (const Item &it : items)
    if (std::strcmp(it.n, name) == 0) {
      if (dst && it.count) std::memcpy(dst, it.p, it.count * it.bytes);
      return (int64_t)it.count;
    }
  return -1;
}

// Full metrics by the traditional construction.
//   n  [dim][nedge]   lumped directed-area vectors (tail -> head)
//   b  [dim][nbnode]  boundary dual-face area vectors (may be NULL)
//   V  [nv]           median-dual volumes (may be NULL)
// Sums are compensated and taken in CSR order, so results do not depend on
// the thread count.
int oracle_metrics(const void *h, const double *coords, const int32_t *elem, double *n,
                   double *b, double *V) {
  const Topo &t = *static_cast<const Topo *>(h);
  const int dim = t.dim, ne = n_local_edges(dim), nn = dim + 1;
  const double *X[4] = {coords, coords + t.nv, dim >= 3 ? coords + 2 * t.nv : coords,
                        dim == 4 ? coords + 3 * t.nv : coords};
  std::vector<double> npc, vpc;
  try {
    npc.resize((size_t)t.nelem * ne * dim);
    vpc.resize((size_t)t.nelem * nn);
  } catch (...) {
    return OR_EOVERFLOW;
  }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < t.nelem; ++e)
    element_pieces_d(dim, X, elem, e, &npc[(size_t)e * ne * dim], &vpc[(size_t)e * nn]);
#pragma omp parallel for schedule(static)
  for (int64_t ed = 0; ed < t.nedge; ++ed) {
    Neumaier acc[4];
    for (int32_t r = t.edge_inc_off[ed]; r < t.edge_inc_off[ed + 1]; ++r) {
      const double *p = &npc[(size_t)t.edge_inc[r] * dim];
      for (int c = 0; c < dim; ++c) acc[c].add(p[c]);
    }
    for (int c = 0; c < dim; ++c) n[c * t.nedge + ed] = acc[c].get();
  }
  if (V) {
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < t.nv; ++v) {
      Neumaier acc;
      for (int32_t r = t.node_inc_off[v]; r < t.node_inc_off[v + 1]; ++r) acc.add(vpc[t.node_inc[r]]);
      V[v] = acc.get();
    }
  }
  if (b) {
    std::vector<double> bpc((size_t)t.nbface * dim * dim);
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < t.nbface; ++f) bface_pieces_d(dim, X, t, elem, f, &bpc[(size_t)f * dim * dim]);
#pragma omp parallel for schedule(static)
    for (int64_t bi = 0; bi < t.nbnode; ++bi) {
      Neumaier acc[4];
      int32_t node = t.bnode[bi];
      for (int32_t r = t.bnode_face_off[bi]; r < t.bnode_face_off[bi + 1]; ++r) {
        int32_t f = t.bnode_face[r];
        int s = 0;
        while (t.bface[(size_t)f * dim + s] != node) ++s;
        for (int c = 0; c < dim; ++c) acc[c].add(bpc[((size_t)f * dim + s) * dim + c]);
      }
      for (int c = 0; c < dim; ++c) b[c * t.nbnode + bi] = acc[c].get();
    }
  }
  return OR_OK;
}

// Loss restricted to the terms that depend on node j, and its exact gradient
// with respect to x_j by forward-mode dual numbers through the traditional
// construction:
//   L = sum_e w_e . n_e + sum_i c_i V_i + sum_{boundary nodes i} beta_i . b_i
// Only elements containing j and boundary faces containing j depend on x_j.
// w [dim][nedge], c [nv], beta [dim][nbnode] (each may be NULL).
// For each listed node: loss_out[k] (may be NULL) and grad_out[k][dim].
int oracle_node_grad(const void *h, const double *coords, const int32_t *elem, const double *w,
                     const double *c, const double *beta, const int32_t *nodes, int64_t nlist,
                     double *loss_out, double *grad_out) {
  const Topo &t = *static_cast<const Topo *>(h);
  if (t.dim == 4) return OR_EINVAL;  // reference gradients are for D = 2, 3
  const int dim = t.dim, ne = n_local_edges(dim), nn = dim + 1;
  const int (*pairs)[2] = local_pairs(dim);
  const double *X[4] = {coords, coords + t.nv, dim >= 3 ? coords + 2 * t.nv : coords,
                        dim == 4 ? coords + 3 * t.nv : coords};
  (void)pairs;
  int status = OR_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < nlist; ++q) {
    const int32_t j = nodes[q];
    if (j < 0 || j >= t.nv) {
      status = OR_ERANGE;
      continue;
    }
    Neumaier L;
    Neumaier G[3];
    auto seeded = [&](int32_t v) {
      P3<Dual> p;
      p.x = mk(X[0][v]);
      p.y = mk(X[1][v]);
      p.z = mk(dim == 3 ? X[2][v] : 0.0);
      if (v == j) {
        p.x.d[0] = 1.0;
        p.y.d[1] = 1.0;
        if (dim == 3) p.z.d[2] = 1.0;
      }
      return p;
    };
    auto add_term = [&](Dual term) {
      L.add(term.v);
      for (int k = 0; k < 3; ++k) G[k].add(term.d[k]);
    };
    for (int32_t r = t.node_inc_off[j]; r < t.node_inc_off[j + 1]; ++r) {
      int64_t e = t.node_inc[r] / nn;
      const int32_t *cc = elem + e * nn;
      P3<Dual> P[4], npc[6];
      Dual vpc[4];
      for (int i = 0; i < nn; ++i) P[i] = seeded(cc[i]);
      if (dim == 2)
        tri_pieces(P, cc, npc, vpc);
      else
        tet_pieces(P, cc, npc, vpc);
      if (w)
        for (int l = 0; l < ne; ++l) {
          int32_t ed = t.elem_edge[e * ne + l];
          Dual s = mk(w[0 * t.nedge + ed]) * npc[l].x + mk(w[1 * t.nedge + ed]) * npc[l].y;
          if (dim == 3) s = s + mk(w[2 * t.nedge + ed]) * npc[l].z;
          add_term(s);
        }
      if (c)
        for (int i = 0; i < nn; ++i) add_term(mk(c[cc[i]]) * vpc[i]);
    }
    if (beta && t.node_bnode[j] >= 0) {
      int32_t bj = t.node_bnode[j];
      for (int32_t r = t.bnode_face_off[bj]; r < t.bnode_face_off[bj + 1]; ++r) {
        int32_t f = t.bnode_face[r];
        P3<Dual> V[3];
        for (int s = 0; s < dim; ++s) V[s] = seeded(t.bface[(size_t)f * dim + s]);
        int32_t own = t.bface_owner[f];
        P3<Dual> Xo = seeded(elem[(int64_t)(own / nn) * nn + own % nn]);
        for (int s = 0; s < dim; ++s) {
          int32_t node = t.bface[(size_t)f * dim + s];
          int32_t bi = t.node_bnode[node];
          P3<Dual> p = bface_piece(dim, V, s, Xo);
          Dual term = mk(beta[0 * t.nbnode + bi]) * p.x + mk(beta[1 * t.nbnode + bi]) * p.y;
          if (dim == 3) term = term + mk(beta[2 * t.nbnode + bi]) * p.z;
          add_term(term);
        }
      }
    }
    if (loss_out) loss_out[q] = L.get();
    for (int k = 0; k < dim; ++k) grad_out[q * dim + k] = G[k].get();
  }
  return status;
}

}  // extern "C"
