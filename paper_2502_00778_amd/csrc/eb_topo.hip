// Edge extraction and boundary elements (the edge array of Section 2 and the
// boundary-element loops of Sections 3.2.1-3.2.3), built on the GPU.
//
// The build is a bucket (counting) sort keyed by node followed by small
// per-bucket sorts, instead of a multi-pass global radix sort of edge keys:
//   1. count the elements of every node (histogram), scan, scatter
//      elem*(D+1)+local into node_inc (a one-digit radix sort with radix
//      n_nodes), then sort every bucket so the order is unique;
//   2. per node j, the edges with tail j are the distinct neighbours k > j in
//      j's elements: collect them sorted and unique in LDS (count pass, scan,
//      emit pass) -> edges come out in ascending (tail, head) order;
//   3. per node j, the faces whose smallest vertex is j are counted in j's
//      elements (each face lies in one or two elements, both containing j);
//      faces met once are boundary faces, three or more is an error;
//   4. element -> edge map by binary search in the tail's head list; the
//      edge -> element and other CSR lists by count / scan / scatter / row
//      sort.
// Every integer output is thus uniquely defined (bit-exact across runs).
#include "eb_geom.h"

namespace eb {

namespace {

// Per-node topology work keeps each node's sorted head list and its
// candidate faces in LDS.  A fast kernel with small per-node capacities
// handles almost every node; nodes beyond them are queued and handled by a
// second kernel with large capacities (a few threads per block).
constexpr int TB = 128;                   // fast kernel: threads per block
constexpr int MAXH = 32;                  //   heads per node
constexpr int MAXF = 64;                  //   candidate faces per node
constexpr int TBS = 32;                   // queued nodes: threads per block
constexpr int MAXH_S = EB_MAX_OUT_EDGES;  //   heads per node
constexpr int MAXF_S = EB_MAX_NODE_FACES; //   candidate faces per node
static_assert(MAXH_S * MAXH_S <= 0x8000, "face codes fit 15 bits");
static_assert(MAXH <= MAXH_S && MAXF <= MAXF_S, "queued capacities are the larger");

// ----------------------------------------------------- node incidences

// Later build kernels do nothing once a kernel has recorded an error: their
// inputs may then be incomplete.
__device__ __forceinline__ bool build_failed(const StatusBlock *st) {
  return *reinterpret_cast<const volatile int32_t *>(&st->status) != 0;
}

template <int D>
__device__ __forceinline__ bool conn_valid(const int32_t (&v)[D + 1], int64_t nv) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i <= D; ++i) ok = ok && v[i] >= 0 && v[i] < nv;
  return ok;
}

template <int D>
__global__ void k_count_nodes(const int32_t *__restrict__ elem, int64_t nelem, int64_t nv,
                              Coords X, int32_t *cnt, StatusBlock *st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nelem) return;
  int32_t v[D + 1];
  load_conn<D>(elem, e, v);
  if (!conn_valid<D>(v, nv)) {
    raise_status(st, EB_ERANGE, e);
    return;
  }
  V3 P[D + 1];
#pragma unroll
  for (int i = 0; i <= D; ++i) P[i] = load_pt<D>(X, v[i]);
  double det;
  if constexpr (D == 3)
    det = dot(P[1] - P[0], cross(P[2] - P[0], P[3] - P[0]));
  else
    det = (P[1].x - P[0].x) * (P[2].y - P[0].y) - (P[1].y - P[0].y) * (P[2].x - P[0].x);
  if (det == 0.0) raise_status(st, EB_EDEGENERATE, e);
#pragma unroll
  for (int i = 0; i <= D; ++i) atomicAdd(&cnt[v[i]], 1);
}

// cur holds inclusive (end) offsets; each slot taken decrements it, so it
// ends as the exclusive (start) offsets
template <int D>
__global__ void k_scatter_nodes(const int32_t *__restrict__ elem, int64_t nelem, int64_t nv,
                                int32_t *cur, int32_t *node_inc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nelem) return;
  int32_t v[D + 1];
  load_conn<D>(elem, e, v);
  if (!conn_valid<D>(v, nv)) return;
#pragma unroll
  for (int i = 0; i <= D; ++i) {
    int32_t pos = atomicSub(&cur[v[i]], 1) - 1;
    node_inc[pos] = (int32_t)(e * (D + 1) + i);
  }
}

// ------------------------------------------------- per-node edge / faces

struct TopoArgs {
  int64_t nv;
  const int32_t *elem;
  Coords X;
  const int32_t *node_inc_off, *node_inc;
  // count pass (workspace)
  int32_t *outdeg, *fmin, *bflag, *bfn, *ein;
  // emit pass
  const int32_t *eoff, *foff;
  int32_t *edge_tail, *edge_head;
  int32_t *bface, *bface_owner;
  int32_t *in_cur, *node_in_edge;
  int32_t *bf_cur, *bnode_face;
  const int32_t *node_sell_off;
  uint64_t *node_sell;
  int32_t *inc_sell;  // optional inverse of the sliced layout
  int sell_wide;
  int32_t *queue;  // nodes beyond the fast kernel's capacities
  StatusBlock *st;
};

// slot of head k in the thread's sorted head column (k must be present)
template <int TBK>
__device__ __forceinline__ int head_slot(const int32_t (*hs)[TBK], int t, int nh, int32_t k) {
  int s = 0;
  while (s < nh - 1 && hs[s][t] != k) ++s;
  return s;
}

template <int D, bool EMIT, int TBK, int MH, int MF, bool SLOW>
__device__ void node_topo_body(const TopoArgs &a, int32_t j, int t, int32_t (*hs)[TBK],
                               uint16_t (*fc)[TBK]) {
  const int32_t r0 = a.node_inc_off[j], r1 = a.node_inc_off[j + 1];

  // 1. distinct higher-numbered neighbours, ascending, and the number of
  //    candidate faces with j as smallest vertex; nothing is written before
  //    both are known to fit (a node beyond the capacities is queued whole).
  //    The count pass also notes the largest |neighbour - j| (sliced-ELL
  //    format).
  int nh = 0, nfc = 0;
  bool overflow = false;
  int32_t maxdelta = 0;
  for (int32_t r = r0; r < r1; ++r) {
    const int32_t inc = a.node_inc[r];
    const int64_t e = inc / (D + 1);
    const int l = inc - (int)(e * (D + 1));
    int32_t v[D + 1];
    load_conn<D>(a.elem, e, v);
    int higher = 0;
#pragma unroll
    for (int q = 0; q <= D; ++q) {
      const int32_t k = v[q];
      if (!EMIT) maxdelta = max(maxdelta, k > j ? k - j : j - k);
      if (q == l || k <= j) continue;
      ++higher;
      int pos = 0;
      while (pos < nh && hs[pos][t] < k) ++pos;
      if (pos < nh && hs[pos][t] == k) continue;
      if (nh == MH) {
        overflow = true;
        continue;
      }
      for (int s = nh; s > pos; --s) hs[s][t] = hs[s - 1][t];
      hs[pos][t] = k;
      ++nh;
    }
    nfc += D == 3 ? higher * (higher - 1) / 2 : higher;
  }
  if (overflow || nfc > MF) {
    if constexpr (SLOW) {
      raise_status(a.st, EB_ECAPACITY, j);
    } else if constexpr (!EMIT) {
      const int32_t q = atomicAdd(&a.st->totals[T_QUEUE], 1);
      a.queue[q] = j;
    }
    return;
  }
  if constexpr (!EMIT) {
    a.outdeg[j] = nh;
    for (int s = 0; s < nh; ++s) atomicAdd(&a.ein[hs[s][t]], 1);
    // only whether some neighbour lies beyond int16 range, or some node has
    // more than 31 out-edges, matters (either selects the wide format)
    if (maxdelta > 32767) atomicMax(&a.st->totals[T_MAXDELTA], maxdelta);
    if (nh > 31) atomicMax(&a.st->totals[T_MAXOUT], nh);
  } else {
    const int32_t e0 = a.eoff[j];
    for (int s = 0; s < nh; ++s) {
      const int32_t k = hs[s][t];
      a.edge_tail[e0 + s] = j;
      a.edge_head[e0 + s] = k;
      const int32_t pos = atomicSub(&a.in_cur[k], 1) - 1;
      a.node_in_edge[pos] = e0 + s;
    }
  }

  // 2. out-edge slot of each other vertex of every element of j (emitted as
  //    in node_sell) and the candidate faces with j as smallest vertex,
  //    coded by the slots of their two other vertices
  int nf = 0;
  for (int32_t r = r0; r < r1; ++r) {
    const int32_t inc = a.node_inc[r];
    const int64_t e = inc / (D + 1);
    const int l = inc - (int)(e * (D + 1));
    int32_t v[D + 1], o[D];
    load_conn<D>(a.elem, e, v);
    others_of<D>(v, l, o);
    // slot of each other vertex among j's out-edges, -1 below j
    const int s0 = o[0] > j ? head_slot<TBK>(hs, t, nh, o[0]) : -1;
    const int s1 = o[1] > j ? head_slot<TBK>(hs, t, nh, o[1]) : -1;
    int s2 = -1;
    if constexpr (D == 3) s2 = o[2] > j ? head_slot<TBK>(hs, t, nh, o[2]) : -1;
    if constexpr (EMIT) {
      const int B = a.sell_wide ? 10 : 5;
      const int none = (1 << B) - 1;
      const uint64_t code = (uint64_t)((s0 < 0 ? none : s0) | ((s1 < 0 ? none : s1) << B) |
                                       (D == 3 ? (s2 < 0 ? none : s2) << (2 * B) : 0));
      const int64_t pos = (int64_t)a.node_sell_off[j / SELL] + (int64_t)SELL * (r - r0) + (j % SELL);
      if (a.inc_sell) a.inc_sell[inc] = (int32_t)pos;
      if (!a.sell_wide) {
        uint64_t w = code << 48;
#pragma unroll
        for (int m = 0; m < D; ++m) w |= (uint64_t)(uint16_t)(int16_t)(o[m] - j) << (16 * m);
        a.node_sell[pos] = w;
      } else {
        a.node_sell[2 * pos] = (uint64_t)(uint32_t)o[0] | ((uint64_t)(uint32_t)o[1] << 32);
        a.node_sell[2 * pos + 1] = (uint64_t)(uint32_t)(D == 3 ? o[D - 1] : 0) | (code << 32);
      }
    }
    auto add_face = [&](int p, int q) {
      if (p < 0 || q < 0) return;
      const int lo = p < q ? p : q, hi = p < q ? q : p;
      fc[nf++][t] = (uint16_t)(lo * MH + hi);
    };
    if constexpr (D == 3) {
      add_face(s0, s1);
      add_face(s0, s2);
      add_face(s1, s2);
    } else {
      if (s0 >= 0) fc[nf++][t] = (uint16_t)s0;
      if (s1 >= 0) fc[nf++][t] = (uint16_t)s1;
    }
  }
  if constexpr (EMIT) {  // zero the slice entries past j's row
    const int32_t sl0 = a.node_sell_off[j / SELL], sl1 = a.node_sell_off[j / SELL + 1];
    const int32_t slen = (sl1 - sl0) / SELL;
    for (int32_t rl = r1 - r0; rl < slen; ++rl) {
      const int64_t pos = (int64_t)sl0 + (int64_t)SELL * rl + (j % SELL);
      if (!a.sell_wide) {
        a.node_sell[pos] = 0;
      } else {
        a.node_sell[2 * pos] = 0;
        a.node_sell[2 * pos + 1] = 0;
      }
    }
  }

  // 3. multiplicity of each candidate: 1 = boundary face, 2 = interior
  int nb = 0;
  for (int i = 0; i < nf; ++i) {
    const uint16_t c = fc[i][t] & 0x7fff;
    int m = 0;
    for (int i2 = 0; i2 < nf; ++i2) m += (fc[i2][t] & 0x7fff) == c;
    if (m > 2) {
      raise_status(a.st, EB_ENONMANIFOLD, j);
      return;
    }
    if (m == 1) {
      fc[i][t] = c | 0x8000;
      ++nb;
    }
  }
  if constexpr (!EMIT) {
    a.fmin[j] = nb;
    for (int i = 0; i < nf; ++i) {
      const uint16_t c = fc[i][t];
      if (!(c & 0x8000)) continue;
      int32_t fv[D];
      fv[0] = j;
      if constexpr (D == 3) {
        fv[1] = hs[(c & 0x7fff) / MH][t];
        fv[2] = hs[(c & 0x7fff) % MH][t];
      } else {
        fv[1] = hs[c & 0x7fff][t];
      }
#pragma unroll
      for (int s = 0; s < D; ++s) {
        a.bflag[fv[s]] = 1;
        atomicAdd(&a.bfn[fv[s]], 1);
      }
    }
  } else {
    // 4. emit boundary faces in ascending code order (= ascending sorted ids)
    int32_t f = a.foff[j];
    int last = -1;
    for (int done = 0; done < nb; ++done) {
      int best = 0x7fff + 1;
      for (int i = 0; i < nf; ++i) {
        const uint16_t c = fc[i][t];
        if (!(c & 0x8000)) continue;
        const int cc = c & 0x7fff;
        if (cc > last && cc < best) best = cc;
      }
      last = best;
      int32_t fv[D];
      fv[0] = j;
      if constexpr (D == 3) {
        fv[1] = hs[best / MH][t];
        fv[2] = hs[best % MH][t];
      } else {
        fv[1] = hs[best][t];
      }
      // owner: the one element of j holding the face; opposite = its other vertex
      int64_t own = -1;
      int opp = -1;
      int32_t vo = -1;
      for (int32_t r = r0; r < r1 && own < 0; ++r) {
        const int32_t inc = a.node_inc[r];
        const int64_t e = inc / (D + 1);
        int32_t v[D + 1];
        load_conn<D>(a.elem, e, v);
        int hit = 0, o = -1;
#pragma unroll
        for (int q = 0; q <= D; ++q) {
          bool in = false;
#pragma unroll
          for (int s = 0; s < D; ++s) in = in || v[q] == fv[s];
          if (in) ++hit;
          else o = q;
        }
        if (hit == D) {
          own = e;
          opp = o;
          vo = v[o];
        }
      }
      if (own < 0) {  // cannot happen for a consistent node_inc
        raise_status(a.st, EB_EINVAL, j);
        return;
      }
      // outward orientation: the expression, operand order and FP64 rounding
      // of the definition in eb.h (v0 = smallest id), without contraction
      {
#pragma clang fp contract(off)
        const V3 A = load_pt<D>(a.X, fv[0]), B = load_pt<D>(a.X, fv[1]);
        const V3 Xo = load_pt<D>(a.X, vo);
        if constexpr (D == 3) {
          const V3 C = load_pt<D>(a.X, fv[2]);
          const V3 u = B - A, v = C - A, w = A - Xo;
          const double cx = u.y * v.z - u.z * v.y;
          const double cy = u.z * v.x - u.x * v.z;
          const double cz = u.x * v.y - u.y * v.x;
          const double s = cx * w.x + cy * w.y + cz * w.z;
          const bool keep = s > 0;
          a.bface[(int64_t)f * 3 + 0] = fv[0];
          a.bface[(int64_t)f * 3 + 1] = keep ? fv[1] : fv[2];
          a.bface[(int64_t)f * 3 + 2] = keep ? fv[2] : fv[1];
        } else {
          const V3 d = B - A, w = A - Xo;
          const double s = d.y * w.x - d.x * w.y;
          const bool keep = s > 0;
          a.bface[(int64_t)f * 2 + 0] = keep ? fv[0] : fv[1];
          a.bface[(int64_t)f * 2 + 1] = keep ? fv[1] : fv[0];
        }
      }
      a.bface_owner[f] = (int32_t)(own * (D + 1) + opp);
#pragma unroll
      for (int s = 0; s < D; ++s) {
        const int32_t pos = atomicSub(&a.bf_cur[fv[s]], 1) - 1;
        a.bnode_face[pos] = f;
      }
      ++f;
    }
  }
}

template <int D, bool EMIT>
__global__ __launch_bounds__(TB) void k_node_topo(TopoArgs a) {
  __shared__ int32_t hs[MAXH][TB];
  __shared__ uint16_t fc[MAXF][TB];
  const int t = threadIdx.x;
  const int64_t j64 = (int64_t)blockIdx.x * TB + t;
  if (build_failed(a.st)) return;
  if (j64 >= a.nv) {
    if constexpr (EMIT) {  // lanes of the last slice past the last node
      if (j64 < n_slices(a.nv) * SELL) {
        const int32_t sl0 = a.node_sell_off[j64 / SELL], sl1 = a.node_sell_off[j64 / SELL + 1];
        const int w = a.sell_wide ? 2 : 1;
        for (int32_t rl = 0; rl < (sl1 - sl0) / SELL; ++rl)
          for (int k = 0; k < w; ++k)
            a.node_sell[w * ((int64_t)sl0 + (int64_t)SELL * rl + (j64 % SELL)) + k] = 0;
      }
    }
    return;
  }
  node_topo_body<D, EMIT, TB, MAXH, MAXF, false>(a, (int32_t)j64, t, hs, fc);
}

// the queued nodes, with the large capacities
template <int D, bool EMIT>
__global__ __launch_bounds__(TBS) void k_node_topo_queued(TopoArgs a) {
  __shared__ int32_t hs[MAXH_S][TBS];
  __shared__ uint16_t fc[MAXF_S][TBS];
  if (build_failed(a.st)) return;
  const int32_t n = *reinterpret_cast<const volatile int32_t *>(&a.st->totals[T_QUEUE]);
  for (int64_t i = (int64_t)blockIdx.x * TBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * TBS)
    node_topo_body<D, EMIT, TBS, MAXH_S, MAXF_S, true>(a, a.queue[i], threadIdx.x, hs, fc);
}

// longest node_inc row of every 64-node slice
__global__ void k_slice_len(const int32_t *__restrict__ node_inc_off, int64_t nv, int32_t *slen) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= n_slices(nv)) return;
  int32_t m = 0;
  const int64_t j1 = min((sl + 1) * SELL, nv);
  for (int64_t j = sl * SELL; j < j1; ++j) m = max(m, node_inc_off[j + 1] - node_inc_off[j]);
  slen[sl] = m;
}

__global__ void k_emit_slices(const int32_t *__restrict__ slen_scan, int64_t nsl,
                              int32_t *node_sell_off, const StatusBlock *st) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl > nsl || build_failed(st)) return;
  node_sell_off[sl] = SELL * slen_scan[sl];
}

// per-node bookkeeping before the emit pass
struct EmitNodeArgs {
  int64_t nv;
  int dim;
  const int32_t *eoff, *bidx, *bfn, *bfn_scan, *ein_scan;
  int32_t *node_edge_off, *node_bnode, *bnode, *bnode_face_off, *node_in_off;
  const StatusBlock *st;
};

__global__ void k_emit_nodes(EmitNodeArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > a.nv || build_failed(a.st)) return;
  a.node_edge_off[j] = a.eoff[j];
  if (j == a.nv) {
    const int32_t nbn = a.bidx[a.nv];
    a.bnode_face_off[nbn] = a.dim * a.st->totals[T_BFACES];
    a.node_in_off[a.nv] = a.eoff[a.nv];
    return;
  }
  const int32_t b0 = a.bidx[j], b1 = a.bidx[j + 1];
  if (b1 > b0) {
    a.node_bnode[j] = b0;
    a.bnode[b0] = (int32_t)j;
    a.bnode_face_off[b0] = a.bfn_scan[j] - a.bfn[j];
  } else {
    a.node_bnode[j] = -1;
  }
  a.node_in_off[j] = a.ein_scan[j];
}

// ------------------------------------------------- element -> edge map

__device__ __forceinline__ int32_t find_edge(const int32_t *__restrict__ node_edge_off,
                                             const int32_t *__restrict__ head, int32_t a,
                                             int32_t b) {
  const int32_t t = a < b ? a : b, h = a < b ? b : a;
  int32_t lo = node_edge_off[t], hi = node_edge_off[t + 1];
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (head[mid] < h) lo = mid + 1;
    else hi = mid;
  }
  return (lo < node_edge_off[t + 1] && head[lo] == h) ? lo : -1;
}

template <int D>
__global__ void k_elem_edge(const int32_t *__restrict__ elem, int64_t nelem,
                            const int32_t *__restrict__ node_edge_off,
                            const int32_t *__restrict__ head, int32_t *elem_edge,
                            int8_t *elem_edge_sign, int32_t *edge_cnt, StatusBlock *st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nelem || build_failed(st)) return;
  int32_t v[D + 1];
  load_conn<D>(elem, e, v);
  constexpr int NE = EL<D>::NE;
#pragma unroll
  for (int le = 0; le < NE; ++le) {
    const int32_t p = v[pair_p<D>(le)], q = v[pair_q<D>(le)];
    const int32_t id = find_edge(node_edge_off, head, p, q);
    elem_edge[e * NE + le] = id;
    elem_edge_sign[e * NE + le] = p < q ? 1 : -1;
    if (id < 0) raise_status(st, EB_EINVAL, e);
    else if (edge_cnt) atomicAdd(&edge_cnt[id], 1);
  }
}

template <int D>
__global__ void k_bface_edge(const int32_t *__restrict__ bface, int64_t nb,
                             const int32_t *__restrict__ node_edge_off,
                             const int32_t *__restrict__ head, int32_t *bface_edge,
                             const StatusBlock *st) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nb || build_failed(st)) return;
  if constexpr (D == 2) {
    bface_edge[f] = find_edge(node_edge_off, head, bface[2 * f], bface[2 * f + 1]);
  } else {
    const int32_t a = bface[3 * f], b = bface[3 * f + 1], c = bface[3 * f + 2];
    bface_edge[3 * f + 0] = find_edge(node_edge_off, head, a, b);
    bface_edge[3 * f + 1] = find_edge(node_edge_off, head, a, c);
    bface_edge[3 * f + 2] = find_edge(node_edge_off, head, b, c);
  }
}

template <int D>
__global__ void k_scatter_edge_inc(int64_t nelem, const int32_t *__restrict__ elem_edge,
                                   int32_t *cur, int32_t *edge_inc, const StatusBlock *st) {
  constexpr int NE = EL<D>::NE;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nelem * NE || build_failed(st)) return;
  const int32_t id = elem_edge[i];
  if (id < 0) return;
  const int32_t pos = atomicSub(&cur[id], 1) - 1;
  edge_inc[pos] = (int32_t)i;
}

template <int D>
int build_edges_impl(int64_t nv, int64_t nelem, const int32_t *elem, const double *coords,
                     int32_t *node_inc_off, int32_t *node_inc, void *ws, eb_sizes *sizes,
                     hipStream_t s) {
  const WsLayout L = ws_layout(D, nv, nelem);
  StatusBlock *st = ws_at<StatusBlock>(ws, 0);
  int32_t *eoff = ws_at<int32_t>(ws, L.eoff), *foff = ws_at<int32_t>(ws, L.foff);
  int32_t *bidx = ws_at<int32_t>(ws, L.bidx), *bfn = ws_at<int32_t>(ws, L.bfn);
  int32_t *bfn_scan = ws_at<int32_t>(ws, L.bfn_scan), *ein = ws_at<int32_t>(ws, L.ein_scan);
  int32_t *tmp = ws_at<int32_t>(ws, L.scan_tmp);
  const Coords X = coords_rows(coords, D, nv);

  EB_TRY(fill_i32(reinterpret_cast<int32_t *>(st), sizeof(StatusBlock) / 4, 0, s));
  // the six per-node arrays are contiguous lines of the workspace
  // the per-node arrays and slice lengths are contiguous lines of the workspace
  EB_TRY(fill_i32(eoff, (int64_t)((L.scan_tmp - L.eoff) / 4), 0, s));
  EB_TRY(fill_i32(node_inc_off, nv + 1, 0, s));

  // node -> element lists
  if (nelem > 0) {
    hipLaunchKernelGGL(k_count_nodes<D>, dim3(grid_for(nelem, 256)), dim3(256), 0, s, elem,
                       nelem, nv, X, node_inc_off, st);
    EB_LAUNCH_CHECK();
  }
  // the row ends must be the scan total of what was counted: elements
  // rejected above are neither counted nor scattered
  EB_TRY(scan_inclusive(node_inc_off, node_inc_off, nv, node_inc_off + nv, tmp, s));
  if (nelem > 0) {
    hipLaunchKernelGGL(k_scatter_nodes<D>, dim3(grid_for(nelem, 256)), dim3(256), 0, s, elem,
                       nelem, nv, node_inc_off, node_inc);
    EB_LAUNCH_CHECK();
  }
  EB_TRY(rowsort(node_inc_off, node_inc, nv, s));

  // per-node counts of edges, boundary faces, boundary nodes
  TopoArgs ta{};
  ta.nv = nv;
  ta.elem = elem;
  ta.X = X;
  ta.node_inc_off = node_inc_off;
  ta.node_inc = node_inc;
  ta.outdeg = eoff;
  ta.fmin = foff;
  ta.bflag = bidx;
  ta.bfn = bfn;
  ta.ein = ein;
  ta.queue = ws_at<int32_t>(ws, L.queue);
  ta.st = st;
  hipLaunchKernelGGL((k_node_topo<D, false>), dim3(grid_for(nv, TB)), dim3(TB), 0, s, ta);
  EB_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_node_topo_queued<D, false>), dim3(256), dim3(TBS), 0, s, ta);
  EB_LAUNCH_CHECK();
  EB_TRY(scan_exclusive(eoff, eoff, nv + 1, &st->totals[T_EDGES], tmp, s));
  EB_TRY(scan_exclusive(foff, foff, nv + 1, &st->totals[T_BFACES], tmp, s));
  EB_TRY(scan_exclusive(bidx, bidx, nv + 1, &st->totals[T_BNODES], tmp, s));
  EB_TRY(scan_inclusive(bfn, bfn_scan, nv + 1, nullptr, tmp, s));
  EB_TRY(scan_inclusive(ein, ein, nv + 1, nullptr, tmp, s));
  const int64_t nsl = n_slices(nv);
  int32_t *slen = ws_at<int32_t>(ws, L.slen);
  hipLaunchKernelGGL(k_slice_len, dim3(grid_for(nsl, 256)), dim3(256), 0, s,
                     (const int32_t *)node_inc_off, nv, slen);
  EB_LAUNCH_CHECK();
  EB_TRY(scan_exclusive(slen, slen, nsl + 1, &st->totals[T_SELL_ROWS], tmp, s));

  StatusBlock h;
  EB_HIP_CHECK(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
  EB_HIP_CHECK(hipStreamSynchronize(s));
  sizes->dim = D;
  sizes->n_nodes = nv;
  sizes->n_elems = nelem;
  sizes->n_edges = h.totals[T_EDGES];
  sizes->n_bfaces = h.totals[T_BFACES];
  sizes->n_bnodes = h.totals[T_BNODES];
  sizes->n_sell = (int64_t)SELL * h.totals[T_SELL_ROWS];
  sizes->sell_wide = (h.totals[T_MAXDELTA] > 32767 || h.totals[T_MAXOUT] > 31) ? 1 : 0;
  if (h.status != EB_OK)
    set_detail("%s at %s %lld", eb_status_string(h.status),
               h.status == EB_ERANGE || h.status == EB_EDEGENERATE ? "element" : "node",
               (long long)h.detail);
  return h.status;
}

template <int D>
int emit_impl(const eb_sizes *sz, const int32_t *elem, const double *coords,
              const eb_topology *tp, void *ws, hipStream_t s) {
  const int64_t nv = sz->n_nodes, nelem = sz->n_elems;
  const WsLayout L = ws_layout(D, nv, nelem);
  StatusBlock *st = ws_at<StatusBlock>(ws, 0);
  int32_t *eoff = ws_at<int32_t>(ws, L.eoff), *foff = ws_at<int32_t>(ws, L.foff);
  int32_t *bidx = ws_at<int32_t>(ws, L.bidx), *bfn = ws_at<int32_t>(ws, L.bfn);
  int32_t *bfn_scan = ws_at<int32_t>(ws, L.bfn_scan), *ein = ws_at<int32_t>(ws, L.ein_scan);
  int32_t *tmp = ws_at<int32_t>(ws, L.scan_tmp);
  constexpr int NE = EL<D>::NE;

  EmitNodeArgs en{nv, D, eoff, bidx, bfn, bfn_scan, ein, tp->node_edge_off, tp->node_bnode,
                  tp->bnode, tp->bnode_face_off, tp->node_in_off, st};
  hipLaunchKernelGGL(k_emit_nodes, dim3(grid_for(nv + 1, 256)), dim3(256), 0, s, en);
  EB_LAUNCH_CHECK();

  const int64_t nsl = n_slices(nv);
  hipLaunchKernelGGL(k_emit_slices, dim3(grid_for(nsl + 1, 256)), dim3(256), 0, s,
                     (const int32_t *)ws_at<int32_t>(ws, L.slen), nsl, tp->node_sell_off,
                     (const StatusBlock *)st);
  EB_LAUNCH_CHECK();

  TopoArgs ta{};
  ta.nv = nv;
  ta.elem = elem;
  ta.X = coords_rows(coords, D, nv);
  ta.node_inc_off = tp->node_inc_off;
  ta.node_inc = tp->node_inc;
  ta.eoff = eoff;
  ta.foff = foff;
  ta.edge_tail = tp->edge;
  ta.edge_head = tp->edge + sz->n_edges;
  ta.bface = tp->bface;
  ta.bface_owner = tp->bface_owner;
  ta.in_cur = tp->node_in_off;
  ta.node_in_edge = tp->node_in_edge;
  ta.bf_cur = bfn_scan;
  ta.bnode_face = tp->bnode_face;
  ta.node_sell_off = tp->node_sell_off;
  ta.node_sell = tp->node_sell;
  ta.inc_sell = tp->inc_sell;
  ta.sell_wide = sz->sell_wide;
  ta.queue = ws_at<int32_t>(ws, L.queue);
  ta.st = st;
  hipLaunchKernelGGL((k_node_topo<D, true>), dim3(grid_for(nv, TB)), dim3(TB), 0, s, ta);
  EB_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_node_topo_queued<D, true>), dim3(256), dim3(TBS), 0, s, ta);
  EB_LAUNCH_CHECK();
  EB_TRY(rowsort(tp->node_in_off, tp->node_in_edge, nv, s));
  EB_TRY(rowsort(tp->bnode_face_off, tp->bnode_face, sz->n_bnodes, s));

  const bool want_inc = tp->edge_inc_off && tp->edge_inc;
  if (want_inc) EB_TRY(fill_i32(tp->edge_inc_off, sz->n_edges + 1, 0, s));
  if (nelem > 0) {
    hipLaunchKernelGGL(k_elem_edge<D>, dim3(grid_for(nelem, 256)), dim3(256), 0, s, elem,
                       nelem, (const int32_t *)tp->node_edge_off,
                       (const int32_t *)(tp->edge + sz->n_edges), tp->elem_edge,
                       tp->elem_edge_sign, want_inc ? tp->edge_inc_off : nullptr, st);
    EB_LAUNCH_CHECK();
  }
  if (sz->n_bfaces > 0) {
    hipLaunchKernelGGL(k_bface_edge<D>, dim3(grid_for(sz->n_bfaces, 256)), dim3(256), 0, s,
                       (const int32_t *)tp->bface, sz->n_bfaces,
                       (const int32_t *)tp->node_edge_off,
                       (const int32_t *)(tp->edge + sz->n_edges), tp->bface_edge, st);
    EB_LAUNCH_CHECK();
  }
  if (want_inc) {
    EB_TRY(scan_inclusive(tp->edge_inc_off, tp->edge_inc_off, sz->n_edges, nullptr, tmp, s));
    EB_TRY(fill_i32(tp->edge_inc_off + sz->n_edges, 1, (int32_t)(NE * nelem), s));
    if (nelem > 0) {
      hipLaunchKernelGGL(k_scatter_edge_inc<D>, dim3(grid_for(nelem * NE, 256)), dim3(256), 0,
                         s, nelem, (const int32_t *)tp->elem_edge, tp->edge_inc_off,
                         tp->edge_inc, st);
      EB_LAUNCH_CHECK();
    }
    EB_TRY(rowsort(tp->edge_inc_off, tp->edge_inc, sz->n_edges, s));
  }
  return EB_OK;
}

}  // namespace
}  // namespace eb

using namespace eb;

extern "C" {

int eb_build_edges(int dim, int64_t n_nodes, int64_t n_elems, const int32_t *elem,
                   const double *coords, int32_t *node_inc_off, int32_t *node_inc, void *ws,
                   size_t ws_bytes, eb_sizes *sizes_host, hipStream_t stream) {
  clear_detail();
  if (dim != 2 && dim != 3) {
    set_detail("dim must be 2 or 3, got %d", dim);
    return EB_EINVAL;
  }
  if (n_nodes <= 0 || n_elems < 0 || !sizes_host || !coords || !node_inc_off ||
      (n_elems > 0 && (!elem || !node_inc))) {
    set_detail("null pointer or negative size");
    return EB_EINVAL;
  }
  const int64_t ne = dim == 2 ? 3 : 6;
  if (ne * n_elems >= (int64_t(1) << 31) || n_nodes >= (int64_t(1) << 31) - 1) {
    set_detail("grid too large for int32 indexing");
    return EB_EOVERFLOW;
  }
  if (!aligned16(elem) || !aligned16(coords) || !aligned16(node_inc_off) ||
      !aligned16(node_inc)) {
    set_detail("arrays must be 16-byte aligned");
    return EB_EINVAL;
  }
  EB_TRY(check_ws(dim, n_nodes, n_elems, ws, ws_bytes));
  return dim == 2 ? build_edges_impl<2>(n_nodes, n_elems, elem, coords, node_inc_off, node_inc,
                                        ws, sizes_host, stream)
                  : build_edges_impl<3>(n_nodes, n_elems, elem, coords, node_inc_off, node_inc,
                                        ws, sizes_host, stream);
}

int eb_build_edges_emit(const eb_sizes *sizes, const int32_t *elem, const double *coords,
                        const eb_topology *topo, void *ws, size_t ws_bytes,
                        hipStream_t stream) {
  clear_detail();
  EB_TRY(check_sizes(sizes));
  if (!topo || !coords || (sizes->n_elems > 0 && !elem)) {
    set_detail("null pointer");
    return EB_EINVAL;
  }
  const eb_topology &t = *topo;
  const bool has_e = sizes->n_edges > 0, has_el = sizes->n_elems > 0;
  const bool has_f = sizes->n_bfaces > 0, has_bn = sizes->n_bnodes > 0;
  if (!t.node_edge_off || !t.node_inc_off || !t.node_in_off || !t.node_bnode ||
      !t.bnode_face_off || (has_e && (!t.edge || !t.node_in_edge)) ||
      (has_el && (!t.elem_edge || !t.elem_edge_sign || !t.node_inc || !t.node_sell)) ||
      !t.node_sell_off ||
      (has_f && (!t.bface || !t.bface_owner || !t.bface_edge)) ||
      (has_bn && (!t.bnode || !t.bnode_face))) {
    set_detail("a required topology array is null");
    return EB_EINVAL;
  }
  if ((t.edge_inc_off == nullptr) != (t.edge_inc == nullptr)) {
    set_detail("edge_inc_off and edge_inc must both be set or both be null");
    return EB_EINVAL;
  }
  EB_TRY(check_ws(sizes->dim, sizes->n_nodes, sizes->n_elems, ws, ws_bytes));
  return sizes->dim == 2 ? emit_impl<2>(sizes, elem, coords, topo, ws, stream)
                         : emit_impl<3>(sizes, elem, coords, topo, ws, stream);
}

}  // extern "C"
