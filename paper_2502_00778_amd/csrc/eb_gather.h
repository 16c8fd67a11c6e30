// Device code of the deterministic (gather) forward pass, shared by its
// kernels and the fused forward + adjoint kernel.
#pragma once

#include <type_traits>

#include "eb_geom.h"
#include "eb_kernels.h"

namespace eb {

// ------------------------------------------------------------- gather path
//
// Raw accumulator per edge: sum over elements of c = the cross product the
// thread forms (3D: c = 2 n_j^E; 2D: c = n_j^E), plus the boundary term in
// the same units; the final scale kN turns it into n.
//   3D: n = (1/12)[sum c + sum n_B];  2D: n = (1/3)[sum c + (1/2) sum n_B]
//   d = c.(x_a - x_j) = D! |E|;  V_j = sum d * kV, kV = 1/24 (3D), 1/6 (2D)

template <int D> struct GK {
  static constexpr double kN = D == 3 ? 1.0 / 12.0 : 1.0 / 3.0;
  static constexpr double kBraw = D == 3 ? 1.0 : 0.5;  // n_B in raw units
  static constexpr double kV = D == 3 ? 1.0 / 24.0 : 1.0 / 6.0;
};

// Add to a thread-owned LDS accumulator.  Only the owning thread ever adds
// to a slot, and one wave's LDS operations complete in issue order, so the
// sum is taken in program order (deterministic); the atomic form lets the
// add go without waiting for a read.
__device__ __forceinline__ void lds_add(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// position of head k among the out-edges [b, e) of a node (k is present;
// heads ascend, so it is the number of heads below k), eight heads a load
// round
__device__ __forceinline__ int32_t find_head(const int32_t *__restrict__ head, int32_t b, int32_t e,
                                             int32_t k) {
  int32_t r = 0;
  for (int32_t s = b; s < e; s += 8) {
    int32_t h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) h[u] = head[min(s + u, e - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) r += (s + u < e && h[u] < k) ? 1 : 0;
  }
  return r;
}

// One incidence of node j from the sliced-ELL layout: the element's other
// vertices o[] and the out-edge slot code.
template <int D, bool WIDE>
__device__ __forceinline__ void sell_entry(const uint64_t *__restrict__ sell, int64_t pos,
                                           int32_t j, int32_t (&o)[D], uint32_t &code) {
  if constexpr (!WIDE) {
    const uint64_t w = __builtin_nontemporal_load(sell + pos);
#pragma unroll
    for (int m = 0; m < D; ++m) o[m] = j + (int32_t)(int16_t)(uint16_t)(w >> (16 * m));
    code = (uint32_t)(w >> 48) & 0x7fffu;
  } else {
    const uint64_t w0 = __builtin_nontemporal_load(sell + 2 * pos);
    const uint64_t w1 = __builtin_nontemporal_load(sell + 2 * pos + 1);
    o[0] = (int32_t)(uint32_t)w0;
    o[1] = (int32_t)(uint32_t)(w0 >> 32);
    if constexpr (D == 3) o[2] = (int32_t)(uint32_t)w1;
    code = (uint32_t)(w1 >> 32);
  }
}

// One tile of TN consecutive nodes, by a block of TN threads (called by the
// whole block; acc is the block's LDS accumulator).
// How the contribution of element E to an edge (j, k) with tail j is formed
// (all give n to rounding; the alternatives exist to measure what the
// paper's flop counts cost on this hardware):
//   VAR_NODE   one face vector n_j^E per (node, element), reused for every
//              edge leaving j in E (the remark that one area vector serves
//              all edges with the same tail);
//   VAR_EDGE   n_j^E formed again for each such edge, from a rotated vertex
//              order (one normal per local edge, 6 per tet);
//   VAR_DUAL   the traditional median-dual face of the edge in E from the
//              edge midpoint, the face centroids and the element centroid
//              (Section 3.1), oriented from j to k.
enum FwdVariant { VAR_NODE = 0, VAR_EDGE = 1, VAR_DUAL = 2 };

// the traditional dual-face piece of edge (j, P[m]) in the element of j
// whose other vertices are P[] (oriented from j to P[m])
template <int D, int M>
__device__ __forceinline__ V3 dual_piece(const V3 &xj, const V3 (&P)[D]) {
  const V3 xk = P[M];
  const V3 mid = 0.5 * (xj + xk), ejk = xk - xj;
  if constexpr (D == 3) {
    const V3 xa = P[(M + 1) % 3], xb = P[(M + 2) % 3];
    const V3 C = 0.25 * (xj + xk + xa + xb);
    const V3 F1 = (1.0 / 3.0) * (xj + xk + xa), F2 = (1.0 / 3.0) * (xj + xk + xb);
    V3 t1 = 0.5 * cross(F1 - mid, C - mid), t2 = 0.5 * cross(C - mid, F2 - mid);
    if (dot(t1, ejk) < 0.0) t1 = -t1;
    if (dot(t2, ejk) < 0.0) t2 = -t2;
    return t1 + t2;
  } else {
    const V3 C = (1.0 / 3.0) * (xj + xk + P[1 - M]);
    const V3 g = C - mid;
    V3 t = {-g.y, g.x, 0.0};
    if (dot(t, ejk) < 0.0) t = -t;
    return t;
  }
}

// Wait for every vector memory load in flight (s_waitcnt vmcnt(0), the
// other counters left alone).  Ending a rarely taken branch that loads with
// this keeps its loads from looking pending where the branch rejoins, so the
// path that skipped it does not wait there for loads issued for later work.
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0f70); }

// v with its sign bit xor-ed with bit 31 of m (m = 0 or 0x80000000)
__device__ __forceinline__ double flip_sign(double v, uint32_t m) {
  return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) ^ ((uint64_t)m << 32));
}

// Points of the vertices near a tile (a plan with step words: within 2^19 of
// one of its nodes): each row addressed from a tile-uniform base by a 32-bit
// byte offset, so a load needs one offset register instead of a 64-bit
// address per row.
template <int D> struct NearPts {
  using GD = const __attribute__((address_space(1))) double;
  uint64_t bx, by, bz;  // the rows at node `from` (uniform values)
  int64_t from;
  __device__ __forceinline__ NearPts(const Coords &X, int64_t j0)
      : from(j0 - ((int64_t)1 << (STEP_DBITS - 1))) {
    bx = (uint64_t)X.x + (uint64_t)(from * 8);
    by = (uint64_t)X.y + (uint64_t)(from * 8);
    bz = (uint64_t)X.z + (uint64_t)(from * 8);
  }
  __device__ __forceinline__ V3 operator()(int32_t v) const {
    const uint64_t off = (uint64_t)((uint32_t)(v - (int32_t)from) * 8u);
    const double x = *reinterpret_cast<GD *>(bx + off);
    const double y = *reinterpret_cast<GD *>(by + off);
    const double z = D == 3 ? *reinterpret_cast<GD *>(bz + off) : 0.0;
    return V3{x, y, z};
  }
};

// a wide entry's slot code (10-bit fields, 1023 = none) in the step words'
// 5-bit fields (31 = none; a plan with step words has at most 31 out-edges)
template <int D, bool WIDE> __device__ __forceinline__ uint32_t code5(uint32_t c) {
  if constexpr (!WIDE) return c;
  uint32_t r = 0;
#pragma unroll
  for (int m = 0; m < D; ++m) r |= min((c >> (10 * m)) & 1023u, 31u) << (5 * m);
  return r;
}

// the place offset of a step word, sign-extended from its 20 bits
__device__ __forceinline__ int32_t step_delta(uint32_t w) {
  return (int32_t)(w << (32 - STEP_DBITS)) >> (32 - STEP_DBITS);
}

// c ? a : b by component (a select of whole structs can become a select of
// their addresses, which sends both to scratch memory)
__device__ __forceinline__ V3 pick(bool c, const V3 &a, const V3 &b) {
  return V3{c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}

template <int D, int TN, int CAP, int U, bool WIDE, int VAR = VAR_NODE, bool STEP = false>
__device__ __forceinline__ void fwd_node_tile(const FwdArgs &a, int64_t tile,
                                              double (&acc)[D][CAP]) {
  static_assert(TN % SELL == 0, "a tile is whole slices");
  // the slot fields the walk keeps: the entries' own, or the step words' 5-bit
  constexpr bool CW = WIDE && !STEP;
  // accumulator units: cross products (VAR_NODE / VAR_EDGE), pieces (VAR_DUAL)
  constexpr double kOut = VAR == VAR_DUAL ? 1.0 : GK<D>::kN;
  const int t = threadIdx.x;
  const int64_t j0 = tile * TN;
  if (j0 >= a.nv) return;  // whole block leaves together
  const int64_t jend = min(j0 + (int64_t)TN, a.nv);
  const int32_t e0 = a.node_edge_off[j0];
  const int32_t cnt = a.node_edge_off[jend] - e0;
  const bool in_lds = cnt <= CAP;
  if (in_lds)
    for (int i = t; i < cnt; i += TN)
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c][i] = 0.0;
  __syncthreads();
  double *const nx = a.n_x, *const ny = a.n_y, *const nz = a.n_z;
  const int64_t j = j0 + t;
  if (j < a.nv) {
    const int32_t my0 = a.node_edge_off[j], my1 = a.node_edge_off[j + 1];
    // accumulator of slot s: LDS acc[.][base + s], or the output itself
    const int32_t base = in_lds ? my0 - e0 : my0;
    if (!in_lds)
      for (int32_t ed = my0; ed < my1; ++ed) {
        nx[ed] = 0.0;
        ny[ed] = 0.0;
        if (D == 3) nz[ed] = 0.0;
      }
    const V3 xj = load_pt<D>(a.X, (int32_t)j);
    double vs = 0.0;
    const int32_t len = a.node_inc_off[j + 1] - a.node_inc_off[j];
    const int64_t p0 = (int64_t)a.node_sell_off[j / SELL] + (j % SELL);
    // The walk over the row, compiled once for LDS accumulators and once for
    // accumulation in the output (a tile with more out-edges than CAP), so
    // that no add tests which it is.
    auto walk = [&](auto lds_tag) __attribute__((always_inline)) {
      constexpr bool L = decltype(lds_tag)::value;
      auto add = [&](int s, const V3 &c) __attribute__((always_inline)) {
        if constexpr (L) {
          lds_add(&acc[0][base + s], c.x);
          lds_add(&acc[1][base + s], c.y);
          if (D == 3) lds_add(&acc[2][base + s], c.z);
        } else {
          nx[base + s] += c.x;
          ny[base + s] += c.y;
          if (D == 3) nz[base + s] += c.z;
        }
      };
      // One incidence with the points of its other vertices by place.
      auto form = [&](const V3 (&P)[D], uint32_t code) __attribute__((always_inline)) {
        V3 c;
        if constexpr (D == 3)
          c = cross(P[1] - P[0], P[2] - P[0]);
        else
          c = rot2(P[1] - P[0]);
        double d = dot(c, P[0] - xj);
        const bool neg = d < 0.0;
        const double sg = neg ? -1.0 : 1.0;  // the flip applied to c
        if (d == 0.0) raise_status(a.st, EB_EDEGENERATE, j);
        // c and d negated when d < 0, by their sign bits (no branch)
        const uint32_t flip = neg ? 0x80000000u : 0u;
        c = V3{flip_sign(c.x, flip), flip_sign(c.y, flip), flip_sign(c.z, flip)};
        vs += flip_sign(d, flip);
        if constexpr (VAR == VAR_NODE) {
#pragma unroll
          for (int m = 0; m < D; ++m) {
            const int s = slot_of<CW>(code, m);
            if (s != no_slot<CW>()) add(s, c);
          }
        } else {
          auto edge_term = [&](auto mm) {
            constexpr int m = decltype(mm)::value;
            const int s = slot_of<CW>(code, m);
            if (s == no_slot<CW>()) return;
            if constexpr (VAR == VAR_EDGE) {
              // the same face vector from the vertex order rotated by m
              V3 ce;
              if constexpr (D == 3)
                ce = cross(P[(m + 1) % 3] - P[m], P[(m + 2) % 3] - P[m]);
              else
                ce = m == 0 ? rot2(P[1] - P[0]) : -rot2(P[0] - P[1]);
              add(s, sg * ce);
            } else {
              add(s, dual_piece<D, m>(xj, P));
            }
          };
          edge_term(std::integral_constant<int, 0>{});
          edge_term(std::integral_constant<int, 1>{});
          if constexpr (D == 3) edge_term(std::integral_constant<int, 2>{});
        }
      };
      V3 P[D];  // the current entry's points by place
#pragma unroll
      for (int m = 0; m < D; ++m) P[m] = V3{0.0, 0.0, 0.0};
      if constexpr (!STEP) {
        // Chunks of U entries in storage order.  Consecutive entries of a strip
        // differ in one place, whose point alone is loaded (the others stay in
        // registers): each entry loads the point of the first place it changes.
        // A chunk's points load while the chunk before it is formed, and its
        // entries are read one chunk earlier still, so each round of a wave waits
        // once, for loads issued a whole chunk of work before.  An entry that
        // changes more than one place (a row start, a break in the strip)
        // reloads all its points when it is formed, in a branch taken for the
        // wave only when some lane needs it.
        int32_t oB[U][D], oC[U][D];  // the next chunk's entries, the one after
        uint32_t cB[U], cC[U];
        V3 LB[U];                    // the next chunk's loaded points
        bool fB[U][D], xB[U];        // first place each next entry changes; more than one
        auto changes = [&](const int32_t (&prev)[D], const int32_t (&o)[D], bool (&f)[D], bool &x)
            __attribute__((always_inline)) {
          bool seen = false;
          x = false;
#pragma unroll
          for (int m = 0; m < D; ++m) {
            const bool ch = o[m] != prev[m];
            f[m] = ch && !seen;
            x = x || (ch && seen);
            seen = seen || ch;
          }
        };
        auto first_point = [&](const int32_t (&o)[D], const bool (&f)[D]) __attribute__((always_inline)) {
          // by masks: a chain of selects can be turned into an indexed (scratch)
          // access; an unchanged entry reloads place 0
          int32_t rest = 0, id = 0;
#pragma unroll
          for (int m = 1; m < D; ++m) {
            const int32_t k = f[m] ? -1 : 0;
            id |= o[m] & k;
            rest |= k;
          }
          id |= o[0] & ~rest;
          return load_pt<D>(a.X, id);
        };
        if (len > 0) {
#pragma unroll
          for (int u = 0; u < U; ++u)
            sell_entry<D, WIDE>(a.node_sell, p0 + (int64_t)SELL * min(u, len - 1), (int32_t)j, oB[u],
                                cB[u]);
#pragma unroll
          for (int u = 0; u < U; ++u)
            sell_entry<D, WIDE>(a.node_sell, p0 + (int64_t)SELL * min(U + u, len - 1), (int32_t)j,
                                oC[u], cC[u]);
          int32_t none[D];
#pragma unroll
          for (int m = 0; m < D; ++m) none[m] = -1;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            int32_t prev[D];  // (values: a select of arrays would go through memory)
#pragma unroll
            for (int m = 0; m < D; ++m) prev[m] = u == 0 ? none[m] : oB[u > 0 ? u - 1 : 0][m];
            changes(prev, oB[u], fB[u], xB[u]);
            LB[u] = first_point(oB[u], fB[u]);
          }
        }
        // waves whose lanes all end early skip the loop together
        for (int32_t r = 0; r < len; r += U) {
          // this chunk
          int32_t oA[U][D];
          uint32_t cA[U];
          V3 LA[U];
          bool fA[U][D], xA[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            cA[u] = cB[u];
            LA[u] = LB[u];
            xA[u] = xB[u];
#pragma unroll
            for (int m = 0; m < D; ++m) {
              oA[u][m] = oB[u][m];
              fA[u][m] = fB[u][m];
            }
          }
          // the next chunk's points, and the entries of the one after
#pragma unroll
          for (int u = 0; u < U; ++u) {
            cB[u] = cC[u];
#pragma unroll
            for (int m = 0; m < D; ++m) oB[u][m] = oC[u][m];
            int32_t prev[D];
#pragma unroll
            for (int m = 0; m < D; ++m) prev[m] = u == 0 ? oA[U - 1][m] : oB[u > 0 ? u - 1 : 0][m];
            changes(prev, oB[u], fB[u], xB[u]);
            LB[u] = first_point(oB[u], fB[u]);
          }
          // (unconditional, clamped to the row: a load issued on one path only
          // would make the waits below count for both)
#pragma unroll
          for (int u = 0; u < U; ++u)
            sell_entry<D, WIDE>(a.node_sell, p0 + (int64_t)SELL * min(r + 2 * U + u, len - 1),
                                (int32_t)j, oC[u], cC[u]);
          // form this chunk
#pragma unroll
          for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int m = 0; m < D; ++m) P[m] = pick(fA[u][m], LA[u], P[m]);
            if (__builtin_amdgcn_ballot_w64(xA[u]) != 0 && xA[u]) {
#pragma unroll
              for (int m = 0; m < D; ++m) P[m] = load_pt<D>(a.X, oA[u][m]);
              wait_loads();
            }
            if (r + u < len) form(P, cA[u]);
          }
        }
      } else {
        // The same chunk pipeline over the step words (4 bytes per entry): the
        // words are read two chunks ahead, the point each changes one chunk
        // ahead.  A row's first entry is read whole before the loop; an entry
        // that changes several places (a break in the strip) reads its whole
        // entry and all its points when it is formed, in a branch taken for
        // the wave only when some lane needs it.
        uint32_t wB[U], wC[U];
        V3 LB[U];
        uint32_t code = 0;  // the current entry's slot fields by place
        const NearPts<D> near(a.X, j0);
        // this wave's slice of step words from a uniform base, by 32-bit offsets
        using GW = const __attribute__((address_space(1))) uint32_t;
        const uint64_t steps =
            (uint64_t)a.node_step +
            4u * (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(a.node_sell_off[j / SELL]);
        const uint32_t lane = (uint32_t)(j % SELL);
        auto step_word = [&](int32_t c) __attribute__((always_inline)) {
          const uint32_t i = lane + (uint32_t)SELL * (uint32_t)min(c, len - 1);
          return __builtin_nontemporal_load(reinterpret_cast<GW *>(steps + (uint64_t)(i * 4u)));
        };
        auto step_point = [&](uint32_t w) __attribute__((always_inline)) {
          return near((int32_t)j + step_delta(w));
        };
        if (len > 0) {
          int32_t o0[D];
          uint32_t c0;
          sell_entry<D, WIDE>(a.node_sell, p0, (int32_t)j, o0, c0);
          c0 = code5<D, WIDE>(c0);
#pragma unroll
          for (int u = 0; u < U; ++u) wB[u] = step_word(u);
#pragma unroll
          for (int u = 0; u < U; ++u)
            wC[u] = step_word(U + u);
#pragma unroll
          for (int m = 0; m < D; ++m) P[m] = near(o0[m]);
          code = c0;
          // entry 0 is in place already: its word becomes "place 0 keeps its vertex"
          wB[0] = ((uint32_t)(o0[0] - (int32_t)j) & ((1u << STEP_DBITS) - 1u)) |
                  ((c0 & 31u) << STEP_SLOT);
#pragma unroll
          for (int u = 0; u < U; ++u) LB[u] = step_point(wB[u]);
        }
        for (int32_t r = 0; r < len; r += U) {
          uint32_t wA[U];
          V3 LA[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            wA[u] = wB[u];
            LA[u] = LB[u];
          }
          // the words first: the next round's point loads wait for them, and
          // loads complete in order, so they must not queue behind this
          // round's point loads (unconditional, as above)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            wB[u] = wC[u];
            wC[u] = step_word(r + 2 * U + u);
          }
#pragma unroll
          for (int u = 0; u < U; ++u) LB[u] = step_point(wB[u]);
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const bool live = r + u < len;
            const bool multi = (wA[u] & STEP_WHOLE) != 0u && live;
            const uint32_t k = (wA[u] >> STEP_PLACE) & 3u;
#pragma unroll
            for (int m = 0; m < D; ++m) P[m] = pick(!multi && k == (uint32_t)m, LA[u], P[m]);
            const uint32_t sh = 5u * k;
            code = multi ? code : (code & ~(31u << sh)) | (((wA[u] >> STEP_SLOT) & 31u) << sh);
            if (__builtin_amdgcn_ballot_w64(multi) != 0 && multi) {
              int32_t o[D];
              sell_entry<D, WIDE>(a.node_sell, p0 + (int64_t)SELL * (r + u), (int32_t)j, o, code);
              code = code5<D, WIDE>(code);
#pragma unroll
              for (int m = 0; m < D; ++m) P[m] = near(o[m]);
              wait_loads();
            }
            if (live) form(P, code);
          }
        }
      }
    };
    if (in_lds)
      walk(std::true_type{});
    else
      walk(std::false_type{});
    if (a.vol) a.vol[j] = vs * GK<D>::kV;
    if (!in_lds)
      for (int32_t ed = my0; ed < my1; ++ed) {
        nx[ed] *= kOut;
        ny[ed] *= kOut;
        if (D == 3) nz[ed] *= kOut;
      }
  }
  if (in_lds) {
    __syncthreads();
    for (int i = t; i < cnt; i += TN) {
      nx[e0 + i] = acc[0][i] * kOut;
      ny[e0 + i] = acc[1][i] * kOut;
      if (D == 3) nz[e0 + i] = acc[2][i] * kOut;
    }
  }
}

// Boundary elements, after the element pass: for each boundary node j, b_j
// and the boundary correction n_B/(D(D+1)) of the edges of B whose tail is
// j.  Only j's thread touches those edges, and faces are taken in
// bnode_face order, so the result is deterministic.
template <int D>
__device__ __forceinline__ void fwd_boundary_node(const FwdArgs &a, int64_t bj) {
  const int32_t j = a.bnode[bj];
  const int32_t my0 = a.node_edge_off[j], my1 = a.node_edge_off[j + 1];
  constexpr double kB = 1.0 / (D * (D + 1));
  V3 bs = {0.0, 0.0, 0.0};
  // j's out-edge heads, when there are at most 8 (padded with INT32_MAX): an
  // edge's place is then the number of smaller heads, found without a load
  const int32_t nout = my1 - my0;
  const bool few = nout <= 8;
  int32_t hd[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int32_t h = a.edge_head[nout > 0 ? my0 + min(i, nout - 1) : 0];
    hd[i] = i < nout ? h : INT32_MAX;
  }
  auto place = [&](int32_t k) {
    if (!few) return my0 + find_head(a.edge_head, my0, my1, k);
    int32_t r = my0;
#pragma unroll
    for (int i = 0; i < 8; ++i) r += hd[i] < k ? 1 : 0;
    return r;
  };
  // faces in order, three at a time: their ids, vertices and points are all
  // loaded before the first is formed; then the n entries of all the round's
  // edges are loaded together, each edge's additions chained in registers in
  // face order, and stored (no load waits behind an earlier face's store)
  constexpr int G = 3, H = G * (D - 1);  // a face's vertices other than j
  const int32_t r0 = a.bnode_face_off[bj], r1 = a.bnode_face_off[bj + 1];
  for (int32_t r = r0; r < r1; r += G) {
    int32_t f[G], fv[G][D];
#pragma unroll
    for (int u = 0; u < G; ++u) f[u] = a.bnode_face[min(r + u, r1 - 1)];
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int s = 0; s < D; ++s) fv[u][s] = a.bface[(int64_t)f[u] * D + s];
    V3 c[G];
    {
      V3 P[G][D];
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int s = 0; s < D; ++s) P[u][s] = load_pt<D>(a.X, fv[u][s]);
#pragma unroll
      for (int u = 0; u < G; ++u) {
        // (uncontracted: the same bits as k_fwd_boundary_gather's groups)
        V3 nB;
        if constexpr (D == 3)
          nB = nc_scale(0.5, nc_cross(P[u][1] - P[u][0], P[u][2] - P[u][0]));
        else
          nB = rot2(P[u][1] - P[u][0]);
        if (r + u < r1) bs = nc_add(bs, nB);
        c[u] = nc_scale(kB, nB);
      }
    }
    // hit h = (face u, its (h % (D-1))-th vertex other than j, in vertex order)
    int32_t ed[H];
    bool hit[H];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      // the vertices other than j, in vertex order
      int32_t o[D - 1];
#pragma unroll
      for (int m = 0; m < D - 1; ++m) {
        // m-th other vertex: skip j if it comes at or before position m
        const bool j_before = [&] {
          bool b = false;
#pragma unroll
          for (int s = 0; s <= m; ++s) b = b || fv[u][s] == j;
          return b;
        }();
        o[m] = j_before ? fv[u][m + 1] : fv[u][m];
      }
#pragma unroll
      for (int m = 0; m < D - 1; ++m) {
        const int h = u * (D - 1) + m;
        hit[h] = r + u < r1 && o[m] > j && my1 > my0;
        ed[h] = hit[h] ? place(o[m]) : 0;
      }
    }
    V3 val[H];
#pragma unroll
    for (int h = 0; h < H; ++h)  // (entry 0 for no hit: loaded, not used)
      val[h] = V3{a.n_x[ed[h]], a.n_y[ed[h]], D == 3 ? a.n_z[ed[h]] : 0.0};
#pragma unroll
    for (int h = 0; h < H; ++h) {
      // the latest earlier hit on the same edge already holds its partial sum
      V3 base = val[h];
#pragma unroll
      for (int g = 0; g < h; ++g)
        if (hit[g] && ed[g] == ed[h]) base = val[g];
      val[h] = nc_add(base, c[h / (D - 1)]);
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
      if (!hit[h]) continue;
      a.n_x[ed[h]] = val[h].x;
      a.n_y[ed[h]] = val[h].y;
      if (D == 3) a.n_z[ed[h]] = val[h].z;
    }
  }
  if (a.b_x) {
    const V3 bo = nc_scale(1.0 / D, bs);
    a.b_x[bj] = bo.x;
    a.b_y[bj] = bo.y;
    if (D == 3) a.b_z[bj] = bo.z;
  }
}

}  // namespace eb
