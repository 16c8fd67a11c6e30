// Edge extraction and boundary elements (the edge array of Section 2 and the
// boundary-element loops of Sections 3.2.1-3.2.3), built on the GPU.
//
// The build is a bucket (counting) sort keyed by node followed by small
// per-bucket sorts, instead of a multi-pass global radix sort of edge keys:
//   1. count the elements of every node (histogram, aggregated per block in
//      LDS), scan, scatter elem*(D+1)+local into node_inc (a one-digit radix
//      sort with radix n_nodes), then sort every bucket so the order is
//      unique;
//   2. per node j, the distinct neighbours of j in j's elements, sorted in
//      LDS (count pass, scan, emit pass): those above j are its out-edges,
//      emitted in ascending (tail, head) order, those below its in-edges;
//      the emit pass also writes each element's edge ids for the local edges
//      whose tail is j, and j's sliced incidence entries;
//   3. per node j, the faces whose smallest vertex is j are counted in j's
//      elements (each face lies in one or two elements, both containing j);
//      faces met once are boundary faces, three or more is an error;
//   4. in-edge ids by binary search in each tail's out-edges; the other CSR
//      lists by count / scan / scatter / row sort.
// Every integer output is thus uniquely defined (bit-exact across runs).
#include <type_traits>

#include "eb_geom.h"
#include "eb_geom4.h"
#include "eb_plan.h"

namespace eb {

namespace {

// Per-node topology work: a fast kernel (a thread per node) keeps each
// node's sorted neighbour list in registers and its candidate faces in LDS,
// with small per-node capacities that hold almost every node; the nodes
// beyond them are queued and handled by a general kernel (a wavefront per
// node) that has no capacity at all.
constexpr int TB = 128;                   // fast kernel: threads per block
constexpr int MAXH = NSET;                //   neighbours per node (registers)
constexpr int MAXF = 64;                  //   candidate faces per node
constexpr int MAXR = 32;                  //   incidences per node (emit ranking)
constexpr int RB = 8;                     // row entries a thread reads at once
constexpr int HT_LOG = 5;                 // count pass: hash slots per node
constexpr int HT = 1 << HT_LOG;
static_assert(MAXH * MAXH <= 0x8000, "face codes fit 15 bits");

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

// Incidences are aggregated per block before touching global counters: a
// block of AGG_TB threads takes AGG_EPT * AGG_TB consecutive elements and
// gathers its (node, count) pairs in an LDS hash table (open addressing),
// then adds each node's count once.  Grids numbered with locality (most
// generators, and any cell-by-cell split) see several times fewer global
// atomics; an incidence that finds no free slot within AGG_PROBE probes
// goes to the global counter directly, so any input still works.
constexpr int AGG_TB = 256;
constexpr int AGG_EPT = 4;
constexpr int AGG_LOG = 11;
constexpr int AGG_HT = 1 << AGG_LOG;  // hash slots
constexpr int AGG_PROBE = 16;

// slot of node v in the block's table (inserting it), or -1 if the probe
// sequence is full
__device__ __forceinline__ int agg_slot(int32_t *hk, int32_t v) {
  uint32_t h = ((uint32_t)v * 2654435761u) >> (32 - AGG_LOG);
#pragma unroll 1
  for (int p = 0; p < AGG_PROBE; ++p) {
    const int32_t prev = atomicCAS(&hk[h], -1, v);
    if (prev == -1 || prev == v) return (int)h;
    h = (h + 1) & (AGG_HT - 1);
  }
  return -1;
}

template <int D>
__global__ __launch_bounds__(AGG_TB) void k_count_nodes(const int32_t *__restrict__ elem,
                                                        int64_t nelem, int64_t nv, Coords X,
                                                        int32_t *cnt, StatusBlock *st) {
  __shared__ int32_t hk[AGG_HT], hc[AGG_HT];
  for (int i = threadIdx.x; i < AGG_HT; i += AGG_TB) {
    hk[i] = -1;
    hc[i] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * AGG_TB * AGG_EPT + threadIdx.x;
  // every element's connectivity first, then the points two elements at a
  // time, so that loads overlap instead of one element's chain at a time
  int32_t v[AGG_EPT][D + 1];
  bool ok[AGG_EPT];
#pragma unroll
  for (int k = 0; k < AGG_EPT; ++k) {
    const int64_t e = base + (int64_t)k * AGG_TB;
    ok[k] = e < nelem;
#pragma unroll
    for (int i = 0; i <= D; ++i) v[k][i] = 0;
    if (ok[k]) load_conn<D>(elem, e, v[k]);
  }
#pragma unroll
  for (int k = 0; k < AGG_EPT; ++k) {
    const int64_t e = base + (int64_t)k * AGG_TB;
    if (ok[k] && !conn_valid<D>(v[k], nv)) {
      raise_status(st, EB_ERANGE, e);
      ok[k] = false;
    }
  }
#pragma unroll
  for (int k0 = 0; k0 < AGG_EPT; k0 += 2) {
    V3 P[2][D + 1];
#pragma unroll
    for (int k = k0; k < k0 + 2; ++k)
#pragma unroll
      for (int i = 0; i <= D; ++i) P[k - k0][i] = ok[k] ? load_pt<D>(X, v[k][i]) : V3{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = k0; k < k0 + 2; ++k) {
      if (!ok[k]) continue;
      const V3 *Q = P[k - k0];
      double det;
      if constexpr (D == 3)
        det = dot(Q[1] - Q[0], cross(Q[2] - Q[0], Q[3] - Q[0]));
      else
        det = (Q[1].x - Q[0].x) * (Q[2].y - Q[0].y) - (Q[1].y - Q[0].y) * (Q[2].x - Q[0].x);
      if (det == 0.0) raise_status(st, EB_EDEGENERATE, base + (int64_t)k * AGG_TB);
    }
  }
#pragma unroll
  for (int k = 0; k < AGG_EPT; ++k) {
    if (!ok[k]) continue;
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      const int h = agg_slot(hk, v[k][i]);
      if (h >= 0) atomicAdd(&hc[h], 1);
      else atomicAdd(&cnt[v[k][i]], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < AGG_HT; i += AGG_TB)
    if (hk[i] >= 0) atomicAdd(&cnt[hk[i]], hc[i]);
}

// cur holds inclusive (end) offsets; each block takes its nodes' ranges off
// their ends, so cur ends as the exclusive (start) offsets.  The order inside
// a row depends on scheduling; the rows are sorted afterwards.  Blocks that
// finish earlier (mostly the earlier elements) take ranges nearer the row's
// end, so each range is placed at its mirror image within the row (from the
// row's fixed ends, a copy of cur before the pass): the ranges then come in
// roughly ascending element order and the sort has little to do.
template <int D>
__device__ __forceinline__ int4 inc_entry(const int32_t (&v)[D + 1], int l, int64_t e) {
  int32_t o[D];
  others_of<D>(v, l, o);
  return make_int4((int32_t)(e * (D + 1) + l), o[0], o[1], D == 3 ? o[D - 1] : 0);
}

template <int D>
__global__ __launch_bounds__(AGG_TB) void k_scatter_nodes(const int32_t *__restrict__ elem,
                                                          int64_t nelem, int64_t nv, int32_t *cur,
                                                          const int32_t *__restrict__ ends,
                                                          int4 *rows4, int32_t *inc_pos,
                                                          int32_t *node_inc) {
  // mirror image of range [p, p + c) within node v's row
  auto mirror = [&](int32_t v, int32_t p, int32_t c) {
    const int32_t row0 = v > 0 ? ends[v - 1] : 0;
    return row0 + ends[v] - p - c;
  };
  __shared__ int32_t hk[AGG_HT], hc[AGG_HT];
  for (int i = threadIdx.x; i < AGG_HT; i += AGG_TB) {
    hk[i] = -1;
    hc[i] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * AGG_TB * AGG_EPT + threadIdx.x;
  int32_t slot[AGG_EPT][D + 1], rank[AGG_EPT][D + 1];
  int32_t v[AGG_EPT][D + 1];
#pragma unroll
  for (int k = 0; k < AGG_EPT; ++k) {
    const int64_t e = base + (int64_t)k * AGG_TB;
    bool ok = e < nelem;
    if (ok) {
      load_conn<D>(elem, e, v[k]);
      ok = conn_valid<D>(v[k], nv);
    }
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      slot[k][i] = -1;
      if (!ok) continue;
      const int h = agg_slot(hk, v[k][i]);
      if (h >= 0) {
        slot[k][i] = h;
        rank[k][i] = atomicAdd(&hc[h], 1);
      } else {
        const int32_t pos = mirror(v[k][i], atomicSub(&cur[v[k][i]], 1) - 1, 1);
        rows4[pos] = inc_entry<D>(v[k], i, e);
        inc_pos[e * (D + 1) + i] = pos;
        node_inc[pos] = (int32_t)(e * (D + 1) + i);
      }
    }
  }
  __syncthreads();
  // one range per (block, node): hc becomes the range's first position
  for (int i = threadIdx.x; i < AGG_HT; i += AGG_TB)
    if (hk[i] >= 0) {
      const int32_t c = hc[i];
      hc[i] = mirror(hk[i], atomicSub(&cur[hk[i]], c) - c, c);
    }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < AGG_EPT; ++k) {
    const int64_t e = base + (int64_t)k * AGG_TB;
#pragma unroll
    for (int i = 0; i <= D; ++i)
      if (slot[k][i] >= 0) {
        const int32_t pos = hc[slot[k][i]] + rank[k][i];
        rows4[pos] = inc_entry<D>(v[k], i, e);
        inc_pos[e * (D + 1) + i] = pos;
        node_inc[pos] = (int32_t)(e * (D + 1) + i);
      }
  }
}

// ------------------------------------------------- per-node edge / faces

struct TopoArgs {
  int64_t nv;
  const int32_t *elem;
  Coords X;
  const double *xw;  // fourth coordinate row (dim 4)
  const int32_t *node_inc_off;
  const int32_t *node_inc;
  const int32_t *rows4;  // workspace: Inc4 per incidence, rows of node_inc_off
  int32_t *nset;         // workspace: the fast count pass's neighbour sets (first
                         // slot -1: the node is queued)
  const uint16_t *row_rank;  // workspace: rank of each row entry within its row
  // count pass (workspace)
  int32_t *outdeg, *fmin, *bflag, *bfn, *ein;
  // emit pass
  const int32_t *eoff, *foff;
  const int32_t *ein_scan;  // inclusive scan of the in-degrees (general kernel)
  int32_t *edge_tail, *edge_head;
  int32_t *bface, *bface_owner;
  int32_t *in_cur, *node_in_edge;
  int32_t *bf_cur, *bnode_face;
  const int32_t *node_sell_off;
  uint64_t *node_sell;
  int sell_wide;
  int32_t *queue;  // nodes beyond the fast kernel's capacities
  StatusBlock *st;
};

// A node's distinct neighbours, ascending, kept in registers (a fixed-size
// sorted array updated with predicated moves, no indexed access).
template <int NR>
struct RegSet {
  static constexpr int CAP = NR;
  int32_t a[NR];
  int n = 0;  // entries inserted (the count pass; a loaded set leaves it 0)
  __device__ __forceinline__ RegSet() {
#pragma unroll
    for (int s = 0; s < NR; ++s) a[s] = INT32_MAX;
  }
  // false when full (k not already present)
  __device__ __forceinline__ bool insert(int32_t k) { return insert_upto(k, NR / 8); }
  // insert touching only the first 8 g slots, g uniform across the wave and
  // large enough that no lane's set outgrows them (the others hold
  // INT32_MAX and stay so)
  __device__ __forceinline__ bool insert_upto(int32_t k, int g) {
    bool dup = false;
#pragma unroll
    for (int q = 0; q < NR / 8; ++q)
      if (q < g)
#pragma unroll
        for (int s = 8 * q; s < 8 * q + 8; ++s) dup = dup || a[s] == k;
    if (dup) return true;
    if (a[NR - 1] != INT32_MAX) return false;
#pragma unroll
    for (int q = NR / 8 - 1; q >= 0; --q)
      if (q < g)
#pragma unroll
        for (int s = 8 * q + 7; s >= 8 * q; --s) {
          const int32_t below = s > 0 ? a[s > 0 ? s - 1 : 0] : INT32_MIN;  // (a[0]: nothing below)
          a[s] = a[s] < k ? a[s] : (below < k ? k : below);
        }
    ++n;
    return true;
  }
  // the groups of eight slots that hold every lane's set after m more
  // inserts (uniform)
  __device__ __forceinline__ int groups_after(int m) const {
    int g = 1;
#pragma unroll
    for (int q = 1; q < NR / 8; ++q) g += __builtin_amdgcn_ballot_w64(n + m > 8 * q) != 0 ? 1 : 0;
    return g;
  }
  // entries below k (the slot of k when present)
  __device__ __forceinline__ int rank(int32_t k) const {
    int r = 0;
#pragma unroll
    for (int s = 0; s < NR; ++s) r += a[s] < k ? 1 : 0;
    return r;
  }
  __device__ __forceinline__ int size() const { return rank(INT32_MAX); }
  // rank(k) comparing only the first 8 g slots, g the same in every lane of
  // the wave (a uniform value): enough when no lane's set is larger, since
  // the empty slots hold INT32_MAX, which no vertex id exceeds
  __device__ __forceinline__ int rank_upto(int32_t k, int g) const {
    static_assert(NR % 8 == 0, "slots in groups of eight");
    int r = 0;
#pragma unroll
    for (int q = 0; q < NR / 8; ++q)
      if (q < g)
#pragma unroll
        for (int s = 8 * q; s < 8 * q + 8; ++s) r += a[s] < k ? 1 : 0;
    return r;
  }
  // h[i] = a[by + i] (INT32_MAX past the set), by a barrel shifter of
  // selects (no indexed access)
  __device__ __forceinline__ void window8(int by, int32_t (&h)[8]) const {
    int32_t b[NR];
#pragma unroll
    for (int s = 0; s < NR; ++s) b[s] = a[s];
#pragma unroll
    for (int sh = 16; sh >= 1; sh >>= 1) {
      const bool on = (by & sh) != 0;
#pragma unroll
      for (int s = 0; s < NR; ++s) b[s] = on ? (s + sh < NR ? b[s + sh < NR ? s + sh : 0] : INT32_MAX) : b[s];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) h[i] = b[i];
  }
  // the groups of eight slots every lane's set fits in (uniform)
  __device__ __forceinline__ int groups_used() const {
    const int n = size();
    int g = 1;
#pragma unroll
    for (int q = 1; q < NR / 8; ++q) g += __builtin_amdgcn_ballot_w64(n > 8 * q) != 0 ? 1 : 0;
    return g;
  }
  __device__ __forceinline__ int32_t at(int i) const {
    int32_t r = 0;
#pragma unroll
    for (int s = 0; s < NR; ++s) r = s == i ? a[s] : r;
    return r;
  }
  template <class F> __device__ __forceinline__ void each(int lo, int hi, F f) const {
#pragma unroll
    for (int s = 0; s < NR; ++s)
      if (s >= lo && s < hi) f(s, a[s]);
  }
  // the set as stored by store(): slot s at p[64 s]
  __device__ __forceinline__ void load(const int32_t *p) {
#pragma unroll
    for (int s = 0; s < NR; ++s) a[s] = p[64 * s];
  }
  __device__ __forceinline__ void store(int32_t *p) const {
#pragma unroll
    for (int s = 0; s < NR; ++s) p[64 * s] = a[s];
  }
};

// Ascending sort of N values in registers by a bitonic network: merge
// stage K (sorted runs of K/2 become runs of K), distance H; every index is
// a compile-time constant (no indexed access).
template <int N, int K, int H>
__device__ __forceinline__ void bitonic_step(int32_t (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int p = i ^ H;
    if (p > i) {
      const int32_t x = v[i], y = v[p];
      const bool up = (i & K) == 0;
      v[i] = up ? min(x, y) : max(x, y);
      v[p] = up ? max(x, y) : min(x, y);
    }
  }
  if constexpr (H > 1)
    bitonic_step<N, K, H / 2>(v);
  else if constexpr (K < N)
    bitonic_step<N, 2 * K, K>(v);
}

template <int N>
__device__ __forceinline__ void sort_net(int32_t (&v)[N]) {
  static_assert((N & (N - 1)) == 0 && N >= 2, "a power of two");
  bitonic_step<N, 2, 1>(v);
}

// One incidence as the scatter pass stores it in the workspace: the
// incidence elem*(D+1)+local and the element's other vertices o_m (o_m =
// elem[m] for m < D, except that j's own place is taken by elem[D]); rows are
// in scheduling order until the emit pass ranks them.
struct Inc4 {
  int32_t inc, o0, o1, o2;
};

template <int D>
__device__ __forceinline__ void inc_others(const int4 &q, int32_t (&o)[D]) {
  o[0] = q.y;
  o[1] = q.z;
  if constexpr (D == 3) o[2] = q.w;
}

// Rank of every entry of every row (the number of smaller incidences in the
// row), and node_inc sorted in place (the scatter pass wrote it in row
// order).  A thread per node; rows up to RK_CAP entries are sorted by
// insertion in an LDS column (the scatter pass leaves rows nearly ascending,
// so the cost follows the few inversions), longer ones ranked from the
// workspace rows (which keep the order).
// Two launches, like the strip kernel's: the first sorts the rows of at most
// RK_SHORT entries in smaller LDS columns (more resident waves) and ranks the
// rows longer than RK_CAP; the second sorts the rows in between.
constexpr int RK_TB = 128;
constexpr int RK_CAP = 32;
constexpr int RK_SHORT = 24;

template <int CAP>
__global__ __launch_bounds__(RK_TB) void k_row_rank(int64_t nv, const int32_t *__restrict__ off,
                                                   const int4 *__restrict__ rows4,
                                                   int32_t *node_inc, uint16_t *row_rank,
                                                   const StatusBlock *st) {
  static_assert(CAP == RK_SHORT || CAP == RK_CAP, "the two launches");
  constexpr bool FIRST = CAP < RK_CAP;
  __shared__ int32_t col[CAP][RK_TB];
  __shared__ uint8_t at[CAP][RK_TB];
  const int t = threadIdx.x;
  const int64_t j = (int64_t)blockIdx.x * RK_TB + t;
  if (j >= nv || build_failed(st)) return;
  const int32_t r0 = off[j], len = off[j + 1] - r0;
  if (FIRST ? (len > RK_SHORT && len <= RK_CAP) : (len <= RK_SHORT || len > RK_CAP)) return;
  if (len <= CAP) {
    auto insert = [&](int32_t i, int32_t x) {
      int32_t k = i;
      for (; k > 0; --k) {
        const int32_t y = col[k - 1][t];
        if (y < x) break;
        col[k][t] = y;
        at[k][t] = at[k - 1][t];
      }
      col[k][t] = x;
      at[k][t] = (uint8_t)i;
    };
    // the row read in aligned 16-byte pieces (the array's length is a
    // multiple of four in 3D; otherwise the last piece is read word by word)
    const int32_t r1 = r0 + len, n_all = off[nv];
    for (int32_t q = r0 & ~3; q < r1; q += 4) {
      int32_t w[4];
      if (q + 4 <= n_all) {
        const int4 x = *reinterpret_cast<const int4 *>(node_inc + q);
        w[0] = x.x;
        w[1] = x.y;
        w[2] = x.z;
        w[3] = x.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = q + u < n_all ? node_inc[q + u] : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q + u >= r0 && q + u < r1) insert(q + u - r0, w[u]);
    }
    // the sorted row, in aligned 16-byte pieces inside it and words at its
    // ends (neighbouring rows belong to other threads)
    for (int32_t q = r0 & ~3; q < r1; q += 4) {
      if (q >= r0 && q + 4 <= r1) {
        *reinterpret_cast<int4 *>(node_inc + q) =
            make_int4(col[q - r0][t], col[q - r0 + 1][t], col[q - r0 + 2][t], col[q - r0 + 3][t]);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q + u >= r0 && q + u < r1) node_inc[q + u] = col[q + u - r0][t];
      }
    }
    // ranks by position (col is free now), eight 16-bit ranks a piece
    for (int32_t k = 0; k < len; ++k) col[at[k][t]][t] = k;
    for (int32_t q = r0 & ~7; q < r1; q += 8) {
      if (q >= r0 && q + 8 <= r1) {
        uint32_t w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          w[u] = (uint32_t)col[q - r0 + 2 * u][t] | ((uint32_t)col[q - r0 + 2 * u + 1][t] << 16);
        *reinterpret_cast<uint4 *>(row_rank + q) = make_uint4(w[0], w[1], w[2], w[3]);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (q + u >= r0 && q + u < r1) row_rank[q + u] = (uint16_t)col[q + u - r0][t];
      }
    }
  } else {
    for (int32_t i = 0; i < len; ++i) {
      const int32_t x = rows4[r0 + i].x;
      int32_t rank = 0;
      for (int32_t i2 = 0; i2 < len; ++i2) rank += rows4[r0 + i2].x < x ? 1 : 0;
      row_rank[r0 + i] = (uint16_t)rank;
      node_inc[r0 + rank] = x;
    }
  }
}

// Boundary face f: vertices fv (fv[0] = j, its smallest), owned by element
// `own`, whose vertex off the face is vo.  Writes the face in outward vertex
// order, its owner, and its id into its vertices' bnode_face rows.
template <int D>
__device__ void write_bface(const TopoArgs &a, int32_t f, const int32_t (&fv)[D], int64_t own,
                            int32_t vo) {
  int32_t v[D + 1];
  load_conn<D>(a.elem, own, v);
  int opp = 0;
#pragma unroll
  for (int qq = 0; qq <= D; ++qq) opp = v[qq] == vo ? qq : opp;
  // outward orientation: the expression, operand order and FP64 rounding
  // of the definition in eb.h (v0 = smallest id), without contraction
  {
#pragma clang fp contract(off)
    const V3 A = load_pt<D>(a.X, fv[0]), B = load_pt<D>(a.X, fv[1]);
    const V3 Xo = load_pt<D>(a.X, vo);
    if constexpr (D == 3) {
      const V3 C = load_pt<D>(a.X, fv[2]);
      const V3 u = B - A, w2 = C - A, w = A - Xo;
      const double cx = u.y * w2.z - u.z * w2.y;
      const double cy = u.z * w2.x - u.x * w2.z;
      const double cz = u.x * w2.y - u.y * w2.x;
      const double sg = cx * w.x + cy * w.y + cz * w.z;
      const bool keep = sg > 0;
      a.bface[(int64_t)f * 3 + 0] = fv[0];
      a.bface[(int64_t)f * 3 + 1] = keep ? fv[1] : fv[2];
      a.bface[(int64_t)f * 3 + 2] = keep ? fv[2] : fv[1];
    } else {
      const V3 d = B - A, w = A - Xo;
      const double sg = d.y * w.x - d.x * w.y;
      const bool keep = sg > 0;
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
}

// Per node j: 1. its distinct neighbours and candidate faces; 2. (emit)
// its sorted node_inc row and sliced entries; 3. face multiplicities;
// 4. (emit) its boundary faces.  RC is the longest row the kernel ranks in
// LDS (pr); a node beyond RC, the set's capacity or MF candidate faces is
// queued for the general kernel.
template <int D, bool EMIT, int TBK, class Set, int MF, int RC>
__device__ __forceinline__ void node_topo_body(const TopoArgs &a, int32_t j, int t, Set &hs,
                               uint16_t (*fc)[TBK], uint8_t (*pr)[TBK]) {
  constexpr int MH = Set::CAP;
  const int32_t r0 = a.node_inc_off[j], r1 = a.node_inc_off[j + 1];
  const int4 *__restrict__ row = reinterpret_cast<const int4 *>(a.rows4) + r0;
  const int32_t len = r1 - r0;

  // 1. distinct neighbours (lower and higher), ascending, and the number of
  //    candidate faces with j as smallest vertex; nothing is written before
  //    both are known to fit (a node beyond the capacities is queued whole).
  //    The neighbours below j are j's in-edges, those above its out-edges.
  //    The count pass also notes the largest |neighbour - j| (sliced-ELL
  //    format).
  int nfc = 0;
  bool overflow = len > RC;
  int32_t maxdelta = 0;
  // (count pass) per incidence c, 16 bits at rec[c / 2] >> 16 (c % 2): the
  // table slots of its other vertices (5 bits each), then their ranks in
  // the sorted set; the row is read once
  static_assert(RC % RB == 0 && RC <= 32, "the row fits the records");
  uint32_t rec[RC / 2];
#pragma unroll
  for (int i = 0; i < RC / 2; ++i) rec[i] = 0;
  int32_t *const nset = a.nset + (int64_t)(j / SELL) * NSET * SELL + (j % SELL);
  if constexpr (EMIT) {  // the count pass's set, unless it queued the node
    if (nset[0] == -1) return;
    hs.load(nset);
  }
  if constexpr (!EMIT) {
    // The distinct other vertices go into an open-addressing table of HT
    // slots (empty = INT32_MAX, which no vertex id reaches) held in this
    // thread's wave's part of the face-code LDS, which step 2 only writes
    // once the table has been read out; the table is then sorted by a
    // network.  Slot h of lane l sits in face-code row 2h + l/32, in the
    // two u16 columns of the wave at 2 (l % 32): the 32-bit accesses of a
    // wave fall on distinct banks.
    static_assert(MH <= HT && 2 * HT <= MF, "the table fits the face-code rows");
    const int l = t & 63;
    int32_t *const tab =
        reinterpret_cast<int32_t *>(&fc[l >> 5][(t & ~63) + 2 * (l & 31)]);
    auto slot = [&](uint32_t h) __attribute__((always_inline)) { return tab + (size_t)h * TBK; };
#pragma unroll
    for (int h = 0; h < HT; ++h) *slot(h) = INT32_MAX;
    int cnt = 0;
    bool full = false;
    auto hash = [](int32_t k) __attribute__((always_inline)) {
      return ((uint32_t)k * 0x9E3779B1u) >> (32 - HT_LOG);
    };
    // the slot holding k, k inserted if absent (0 with `full` set when the
    // table has no room)
    auto insert = [&](int32_t k) __attribute__((always_inline)) -> uint32_t {
      uint32_t h = hash(k);
      for (int p = 0; p < HT; ++p) {
        int32_t *const q = slot(h);
        const int32_t x = *q;
        if (x == k) return h;
        if (x == INT32_MAX) {
          *q = k;
          ++cnt;
          return h;
        }
        h = (h + 1) & (HT - 1);
      }
      full = true;
      return 0;
    };
    // (a thread's RB next entries are read together: one 128-byte line is
    // used up at once, before other lanes' rows evict it)
#pragma unroll
    for (int c0 = 0; c0 < RC; c0 += RB) {
      if (c0 < len && !overflow) {
      int4 qb[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) qb[u] = row[min(c0 + u, len - 1)];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int c = c0 + u;
        if (c >= len) continue;
        int32_t o[D];
        inc_others<D>(qb[u], o);
        int higher = 0;
        uint32_t code = 0;
#pragma unroll
        for (int m = 0; m < D; ++m) {
          const int32_t k = o[m];
          maxdelta = max(maxdelta, k > j ? k - j : j - k);
          if (k > j) ++higher;
          code |= insert(k) << (5 * m);
        }
        rec[c >> 1] |= code << (16 * (c & 1));
        nfc += D == 3 ? higher * (higher - 1) / 2 : higher;
      }
      overflow = full || cnt > MH;
      }
    }
    if (!overflow) {
      int32_t v[HT];
#pragma unroll
      for (int h = 0; h < HT; ++h) v[h] = *slot(h);
      sort_net(v);
#pragma unroll
      for (int s2 = 0; s2 < MH; ++s2) hs.a[s2] = v[s2];
      hs.n = cnt;
      // each present value's slot now holds ~rank (negative: no vertex id,
      // so later searches pass over it), then the records' slots become
      // ranks; the table's LDS is free afterwards
#pragma unroll
      for (int r = 0; r < MH; ++r) {
        const int32_t x = v[r];
        if (x != INT32_MAX) {
          uint32_t h = hash(x);
          for (int p = 0; p < HT && *slot(h) != x; ++p) h = (h + 1) & (HT - 1);
          *slot(h) = ~r;
        }
      }
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        if (c >= len) continue;
        const uint32_t code = (rec[c >> 1] >> (16 * (c & 1))) & 0xffffu;
        uint32_t rk = 0;
#pragma unroll
        for (int m = 0; m < D; ++m) rk |= (uint32_t)~*slot((code >> (5 * m)) & 31u) << (5 * m);
        rec[c >> 1] = (rec[c >> 1] & ~(0xffffu << (16 * (c & 1)))) | (rk << (16 * (c & 1)));
      }
    }
  }
  if (overflow || nfc > MF) {
    if constexpr (!EMIT) {
      const int32_t qi = atomicAdd(&a.st->totals[T_QUEUE], 1);
      a.queue[qi] = j;
      nset[0] = -1;
    }
    return;
  }
  if constexpr (!EMIT) hs.store(nset);
  const int nh = hs.size();
  const int nlow = hs.rank(j);  // neighbours below j come first
  const int nout = nh - nlow;
  if constexpr (!EMIT) {
    a.outdeg[j] = nout;
    a.ein[j] = nlow;
    // only whether some neighbour lies beyond int16 range, or some node has
    // more than 31 out-edges, matters (either selects the wide format)
    if (maxdelta > 32767) atomicMax(&a.st->totals[T_MAXDELTA], maxdelta);
    if (nout > 31) atomicMax(&a.st->totals[T_MAXOUT], nout);
  } else {
    const int32_t e0 = a.eoff[j] - nlow;
    hs.each(nlow, nh, [&](int s, int32_t k) {
      a.edge_tail[e0 + s] = j;
      a.edge_head[e0 + s] = k;
    });
    // in-edges: the lower neighbours, ascending (= ascending edge id); their
    // ids are filled in once every tail's edges exist (k_node_in_ids)
    const int32_t i0 = a.in_cur[j] - nlow;
    hs.each(0, nlow, [&](int s, int32_t k) { a.node_in_edge[i0 + s] = k; });
    a.in_cur[j] = i0;
  }

  // 2. slot of each other vertex of every element of j in j's neighbour list
  //    (its out-edge slot is that minus nlow); the emit pass writes the row in
  //    ascending incidence order (rank = number of smaller incidences) and
  //    the sliced entry at that rank; both passes note the candidate faces
  //    with j as smallest vertex, coded by their two other vertices' slots
  int nf = 0;
  const int ngroups = hs.groups_used();
  // When no lane of the wave has more than 8 out-neighbours, a candidate
  // face is a bit of a 64-bit mask (3D: 8 (p - nlow) + q - nlow for slots
  // p < q; 2D: p - nlow), and its multiplicity is tracked by three masks
  // (seen once, twice, three times) instead of comparing every pair of
  // candidates; bit order is code order.  Otherwise the candidates' codes go
  // to LDS (fc) as below.
  const bool by_mask = __builtin_amdgcn_ballot_w64(nh - nlow > 8) == 0;
  uint64_t once = 0, twice = 0, thrice = 0;
  // (by mask) the out-neighbours, at most 8, ascending: a slot above nlow is
  // then found with 8 comparisons instead of one per slot group
  int32_t hi8[8];
  if (by_mask) hs.window8(nlow, hi8);
  auto slot_of_higher = [&](int32_t k) {
    if (by_mask) {
      int r = nlow;
#pragma unroll
      for (int i = 0; i < 8; ++i) r += hi8[i] < k ? 1 : 0;
      return r;
    }
    return hs.rank_upto(k, ngroups);
  };
  const int64_t sbase = (int64_t)a.node_sell_off[j / SELL] + (j % SELL);
  if constexpr (EMIT) {
    // the entry at each rank, so the row is visited in ascending order below
    // (the stores of a wave then fall on one column of the slice)
    for (int32_t i = 0; i < len; ++i) pr[a.row_rank[r0 + i]][t] = (uint8_t)i;
  }
  // the candidate faces of one incidence from its other vertices' slots
  // (-1: the vertex is below j)
  auto faces_of = [&](int s0, int s1, int s2) __attribute__((always_inline)) {
    auto seen = [&](int b) {
      const uint64_t bit = 1ull << b;
      thrice |= twice & bit;
      twice |= once & bit;
      once |= bit;
    };
    auto add_face = [&](int p, int qq) {
      if (p < 0 || qq < 0) return;
      const int lo = p < qq ? p : qq, hi = p < qq ? qq : p;
      if (by_mask)
        seen(8 * (lo - nlow) + hi - nlow);
      else
        fc[nf++][t] = (uint16_t)(lo * MH + hi);
    };
    if constexpr (D == 3) {
      add_face(s0, s1);
      add_face(s0, s2);
      add_face(s1, s2);
    } else if (by_mask) {
      if (s0 >= 0) seen(s0 - nlow);
      if (s1 >= 0) seen(s1 - nlow);
    } else {
      if (s0 >= 0) fc[nf++][t] = (uint16_t)s0;
      if (s1 >= 0) fc[nf++][t] = (uint16_t)s1;
    }
  };
  if constexpr (!EMIT) {
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      if (c >= len) continue;
      const uint32_t rk = (rec[c >> 1] >> (16 * (c & 1))) & 0xffffu;
      int sl[3] = {-1, -1, -1};
#pragma unroll
      for (int m = 0; m < D; ++m) {
        const int r = (int)((rk >> (5 * m)) & 31u);
        sl[m] = r >= nlow ? r : -1;
      }
      faces_of(sl[0], sl[1], sl[2]);
    }
  }
  for (int32_t c0 = 0; EMIT && c0 < len; c0 += RB) {
   int4 qb[RB];
   int32_t ib[RB];
#pragma unroll
   for (int u = 0; u < RB; ++u) {
     ib[u] = pr[min(c0 + u, len - 1)][t];
     qb[u] = row[ib[u]];
   }
#pragma unroll
   for (int u = 0; u < RB; ++u) {
    const int32_t c = c0 + u;
    if (c >= len) break;
    const int4 q = qb[u];
    int32_t o[D];
    inc_others<D>(q, o);
    const int s0 = o[0] > j ? slot_of_higher(o[0]) : -1;
    const int s1 = o[1] > j ? slot_of_higher(o[1]) : -1;
    int s2 = -1;
    if constexpr (D == 3) s2 = o[2] > j ? slot_of_higher(o[2]) : -1;
    {
      const int32_t rank = c;
      const int B = a.sell_wide ? 10 : 5;
      const int none = (1 << B) - 1;
      const int u0 = s0 < 0 ? none : s0 - nlow, u1 = s1 < 0 ? none : s1 - nlow;
      const int u2 = s2 < 0 ? none : s2 - nlow;
      const uint64_t code = (uint64_t)(u0 | (u1 << B) | (D == 3 ? u2 << (2 * B) : 0));
      const int64_t pos = sbase + (int64_t)SELL * rank;
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
    faces_of(s0, s1, s2);
   }
  }
  if constexpr (EMIT) {  // zero the slice entries past j's row
    const int32_t sl0 = a.node_sell_off[j / SELL], sl1 = a.node_sell_off[j / SELL + 1];
    const int32_t slen = (sl1 - sl0) / SELL;
    for (int32_t rl = len; rl < slen; ++rl) {
      const int64_t pos = sbase + (int64_t)SELL * rl;
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
  uint64_t bmask = 0;  // (by mask) the boundary faces
  if (by_mask) {
    if (thrice != 0) {
      raise_status(a.st, EB_ENONMANIFOLD, j);
      return;
    }
    bmask = once & ~twice;
    nb = __builtin_popcountll(bmask);
  }
  // the slots of a boundary face's other vertices from its code or bit
  auto face_slots = [&](int code, int &p, int &q) {
    if (by_mask) {
      p = nlow + (D == 3 ? code / 8 : code);
      q = nlow + code % 8;
    } else {
      p = D == 3 ? code / MH : code;
      q = code % MH;
    }
  };
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
    for (int i = 0; i < (by_mask ? nb : nf); ++i) {
      int code;
      if (by_mask) {
        code = __builtin_ctzll(bmask);
        bmask &= bmask - 1;
      } else {
        const uint16_t c = fc[i][t];
        if (!(c & 0x8000)) continue;
        code = c & 0x7fff;
      }
      int p, q;
      face_slots(code, p, q);
      int32_t fv[D];
      fv[0] = j;
      fv[1] = hs.at(p);
      if constexpr (D == 3) fv[2] = hs.at(q);
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
      if (by_mask) {
        best = __builtin_ctzll(bmask);
        bmask &= bmask - 1;
      } else {
        for (int i = 0; i < nf; ++i) {
          const uint16_t c = fc[i][t];
          if (!(c & 0x8000)) continue;
          const int cc = c & 0x7fff;
          if (cc > last && cc < best) best = cc;
        }
      }
      last = best;
      int p, q;
      face_slots(best, p, q);
      int32_t fv[D];
      fv[0] = j;
      fv[1] = hs.at(p);
      if constexpr (D == 3) fv[2] = hs.at(q);
      // owner: the one element of j holding the face; opposite = its vertex
      // off the face
      int64_t own = -1;
      int32_t vo = -1;
      // (the row read RB entries a round, the first holder in row order kept)
      for (int32_t i0 = 0; i0 < len && own < 0; i0 += RB) {
        int4 qb[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) qb[u] = row[min(i0 + u, len - 1)];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          if (own >= 0 || i0 + u >= len) break;
          const int4 q = qb[u];
          int32_t o[D];
          inc_others<D>(q, o);
          int hit = 0;
          int32_t off = -1;
#pragma unroll
          for (int m = 0; m < D; ++m) {
            bool in = false;
#pragma unroll
            for (int s = 1; s < D; ++s) in = in || o[m] == fv[s];
            if (in) ++hit;
            else off = o[m];
          }
          if (hit == D - 1) {
            own = q.x / (D + 1);
            vo = off;
          }
        }
      }
      if (own < 0) {  // cannot happen for a consistent build
        raise_status(a.st, EB_EINVAL, j);
        return;
      }
      write_bface<D>(a, f, fv, own, vo);
      ++f;
    }
  }
}

template <int D, bool EMIT>
__global__ __launch_bounds__(TB) void k_node_topo(TopoArgs a) {
  __shared__ __align__(16) uint16_t fc[MAXF][TB];
  __shared__ uint8_t pr[EMIT ? MAXR : 1][TB];
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
  RegSet<MAXH> hs;
  node_topo_body<D, EMIT, TB, RegSet<MAXH>, MAXF, MAXR>(a, (int32_t)j64, t, hs, fc, pr);
}

// ------------------------------------------- general per-node kernel
//
// The queued nodes, any number of neighbours and faces: a wavefront per node
// walks the node's row as often as needed and keeps nothing per node but a
// few wave-uniform values.  Distinct neighbours come out in ascending order
// as successive minima over the row (each a wave reduction over the row's
// other vertices above the previous one); candidate faces with the node as
// smallest vertex likewise as successive minima of their keys (the pair of
// other vertices, both above the node), each counted over the row as it
// comes up (1 = boundary face, 2 = interior, more = error).  The cost is
// (neighbours + faces) times the row length over 64 per node, which only
// matters for nodes of very high degree.

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
    const uint64_t w = (uint64_t)hi << 32 | lo;
    v = w < v ? w : v;
  }
  return v;
}

// candidate face keys of one incidence of j: its pairs of other vertices
// both above j (3D, key hi << 32 | lo of the ascending pair), or its other
// vertices above j (2D, key = the vertex); 0 marks no candidate (a real key
// is at least 1, since its vertices exceed j >= 0)
template <int D>
__device__ __forceinline__ void face_keys(const int32_t (&o)[D], int32_t j,
                                          uint64_t (&k)[D == 3 ? 3 : 2]) {
  if constexpr (D == 3) {
    const int P[3][2] = {{0, 1}, {0, 2}, {1, 2}};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int32_t x = o[P[c][0]], y = o[P[c][1]];
      const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
      k[c] = (x > j && y > j) ? ((uint64_t)(uint32_t)lo << 32 | (uint32_t)hi) : 0;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 2; ++c) k[c] = o[c] > j ? (uint64_t)(uint32_t)o[c] : 0;
  }
}

// position of k among the ascending heads[0, n) (k is present)
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t *heads, int32_t n, int32_t k) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (heads[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <int D, bool EMIT>
__device__ void node_topo_general(const TopoArgs &a, int32_t j, int lane) {
  constexpr int NK = D == 3 ? 3 : 2;
  const int32_t r0 = a.node_inc_off[j], r1 = a.node_inc_off[j + 1];
  const int4 *__restrict__ row = reinterpret_cast<const int4 *>(a.rows4) + r0;
  const int32_t len = r1 - r0;

  // 1. distinct neighbours, ascending; the emit pass writes the out-edges
  //    (tail j) and the in-neighbours (ids filled in later by k_node_in_ids)
  int32_t e0 = 0, in_end = 0, nlow_known = 0;
  if constexpr (EMIT) {
    e0 = a.eoff[j];
    in_end = a.in_cur[j];
    nlow_known = a.ein_scan[j] - (j > 0 ? a.ein_scan[j - 1] : 0);
  }
  int32_t last = INT32_MIN, nh = 0, nlow = 0, maxdelta = 0;
  for (;;) {
    int32_t mn = INT32_MAX;
    for (int32_t i = lane; i < len; i += 64) {
      int32_t o[D];
      inc_others<D>(row[i], o);
#pragma unroll
      for (int m = 0; m < D; ++m) {
        if (o[m] > last) mn = min(mn, o[m]);
        if (!EMIT && nh == 0) maxdelta = max(maxdelta, o[m] > j ? o[m] - j : j - o[m]);
      }
    }
    mn = wave_min_i32(mn);
    if (mn == INT32_MAX) break;
    if constexpr (EMIT) {
      if (lane == 0) {
        if (mn < j) {
          a.node_in_edge[in_end - nlow_known + nh] = mn;
        } else {
          a.edge_tail[e0 + nh - nlow] = j;
          a.edge_head[e0 + nh - nlow] = mn;
        }
      }
    }
    if (mn < j) ++nlow;
    ++nh;
    last = mn;
  }
  const int32_t nout = nh - nlow;
  if constexpr (!EMIT) {
    maxdelta = wave_max_i32(maxdelta);
    if (lane == 0) {
      a.outdeg[j] = nout;
      a.ein[j] = nlow;
      if (maxdelta > 32767) atomicMax(&a.st->totals[T_MAXDELTA], maxdelta);
      if (nout > 31) atomicMax(&a.st->totals[T_MAXOUT], nout);
    }
  } else {
    if (lane == 0) a.in_cur[j] = in_end - nlow;
    // the out-edge heads just written are read back below
    __threadfence();
    // 2. each incidence's entry at its rank (rows longer than the strip
    //    length stay in this ascending order), slots by binary search in
    //    the out-edge heads
    const int32_t *heads = a.edge_head + e0;
    const int64_t sbase = (int64_t)a.node_sell_off[j / SELL] + (j % SELL);
    const int B = a.sell_wide ? 10 : 5;
    const int none = (1 << B) - 1;
    for (int32_t i = lane; i < len; i += 64) {
      int32_t o[D];
      inc_others<D>(row[i], o);
      uint64_t code = 0;
#pragma unroll
      for (int m = 0; m < D; ++m) {
        const int u = o[m] > j ? lower_bound_i32(heads, nout, o[m]) : none;
        code |= (uint64_t)u << (B * m);
      }
      const int64_t pos = sbase + (int64_t)SELL * a.row_rank[r0 + i];
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
    // the slice entries past j's row
    const int32_t slen = (a.node_sell_off[j / SELL + 1] - a.node_sell_off[j / SELL]) / SELL;
    for (int32_t rl = len + lane; rl < slen; rl += 64) {
      const int64_t pos = sbase + (int64_t)SELL * rl;
      if (!a.sell_wide) {
        a.node_sell[pos] = 0;
      } else {
        a.node_sell[2 * pos] = 0;
        a.node_sell[2 * pos + 1] = 0;
      }
    }
  }

  // 3. candidate faces in ascending key order, each counted over the row in
  //    the round after it is found (with its first holder in row order)
  int32_t nb = 0, f = EMIT ? a.foff[j] : 0;
  uint64_t cur = 0;
  for (;;) {
    uint64_t mn = ~0ull;
    int32_t cnt = 0, holder = INT32_MAX;
    for (int32_t i = lane; i < len; i += 64) {
      int32_t o[D];
      inc_others<D>(row[i], o);
      uint64_t k[NK];
      face_keys<D>(o, j, k);
#pragma unroll
      for (int c = 0; c < NK; ++c) {
        if (k[c] > cur) mn = k[c] < mn ? k[c] : mn;
        if (cur != 0 && k[c] == cur) {
          ++cnt;
          holder = min(holder, i);
        }
      }
    }
    mn = wave_min_u64(mn);
    if (cur != 0) {
      cnt = wave_sum_i32(cnt);
      holder = wave_min_i32(holder);
      if (cnt > 2) {
        if (lane == 0) raise_status(a.st, EB_ENONMANIFOLD, j);
        return;
      }
      if (cnt == 1) {
        int32_t fv[D];
        fv[0] = j;
        if constexpr (D == 3) {
          fv[1] = (int32_t)(cur >> 32);
          fv[2] = (int32_t)(uint32_t)cur;
        } else {
          fv[1] = (int32_t)cur;
        }
        if (lane == 0) {
          if constexpr (!EMIT) {
#pragma unroll
            for (int s = 0; s < D; ++s) {
              a.bflag[fv[s]] = 1;
              atomicAdd(&a.bfn[fv[s]], 1);
            }
          } else {
            // the owner's vertex off the face
            int32_t o[D];
            const int4 q = row[holder];
            inc_others<D>(q, o);
            int32_t vo = -1;
#pragma unroll
            for (int m = 0; m < D; ++m) {
              bool in = false;
#pragma unroll
              for (int s = 1; s < D; ++s) in = in || o[m] == fv[s];
              if (!in) vo = o[m];
            }
            write_bface<D>(a, f, fv, q.x / (D + 1), vo);
          }
        }
        ++nb;
        ++f;
      }
    }
    if (mn == ~0ull) break;
    cur = mn;
  }
  if constexpr (!EMIT) {
    if (lane == 0) a.fmin[j] = nb;
  }
}

template <int D, bool EMIT>
__global__ __launch_bounds__(64) void k_node_topo_general(TopoArgs a) {
  if (build_failed(a.st)) return;
  const int32_t n = *reinterpret_cast<const volatile int32_t *>(&a.st->totals[T_QUEUE]);
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x)
    node_topo_general<D, EMIT>(a, a.queue[i], (int)threadIdx.x);
}

// longest node_inc row of every 64-node slice, and of the grid
__global__ void k_slice_len(const int32_t *__restrict__ node_inc_off, int64_t nv, int32_t *slen,
                            StatusBlock *st) {
  const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= n_slices(nv)) return;
  int32_t m = 0;
  const int64_t j1 = min((sl + 1) * SELL, nv);
  for (int64_t j = sl * SELL; j < j1; ++j) m = max(m, node_inc_off[j + 1] - node_inc_off[j]);
  slen[sl] = m;
  if (m > MAX_NODE_ELEMS) atomicMax(&st->totals[T_MAXROW], m);
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

// The ids of N edges {a[q], b[q]} (-1: no such edge) by N binary searches
// taken in step: every active search's probe of a round is loaded before any
// is compared, so the searches cost the round trips of the longest one
// rather than their sum.
template <int N>
__device__ __forceinline__ void find_edges(const int32_t *__restrict__ node_edge_off,
                                           const int32_t *__restrict__ head,
                                           const int32_t (&a)[N], const int32_t (&b)[N],
                                           int32_t (&id)[N]) {
  int32_t lo[N], hi[N], end[N], h[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const int32_t t = min(a[q], b[q]);
    h[q] = max(a[q], b[q]);
    lo[q] = node_edge_off[t];
    hi[q] = end[q] = node_edge_off[t + 1];
  }
  for (;;) {
    bool any = false;
    int32_t x[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const bool on = lo[q] < hi[q];
      any = any || on;
      x[q] = on ? head[(lo[q] + hi[q]) >> 1] : 0;
    }
    if (!any) break;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      if (lo[q] >= hi[q]) continue;
      const int32_t mid = (lo[q] + hi[q]) >> 1;
      if (x[q] < h[q]) lo[q] = mid + 1;
      else hi[q] = mid;
    }
  }
  int32_t y[N];
#pragma unroll
  for (int q = 0; q < N; ++q) y[q] = lo[q] < end[q] ? head[lo[q]] : -1;
#pragma unroll
  for (int q = 0; q < N; ++q) id[q] = y[q] == h[q] ? lo[q] : -1;
}

// node_in_edge holds each node's lower neighbours, ascending; replace each
// by the id of the edge (neighbour, node)
__global__ void k_node_in_ids(int64_t nv, const int32_t *__restrict__ node_in_off,
                              const int32_t *__restrict__ node_edge_off,
                              const int32_t *__restrict__ head, int32_t *node_in_edge,
                              StatusBlock *st) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nv || build_failed(st)) return;
  // four neighbours a round: their ids, then their out-edge ranges, then
  // eight heads of each range at a time, so the loads of a round overlap
  // (the edge's position is the number of the tail's heads below j)
  constexpr int G = 4;
  const int32_t r0 = node_in_off[j], r1 = node_in_off[j + 1];
  for (int32_t r = r0; r < r1; r += G) {
    int32_t nb[G], lo[G], hi[G], id[G];
#pragma unroll
    for (int u = 0; u < G; ++u) nb[u] = node_in_edge[min(r + u, r1 - 1)];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      lo[u] = node_edge_off[nb[u]];
      hi[u] = node_edge_off[nb[u] + 1];
    }
    int32_t h[G][8];  // the first eight heads of every range, all in flight
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int v = 0; v < 8; ++v) h[u][v] = head[hi[u] > lo[u] ? min(lo[u] + v, hi[u] - 1) : 0];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      id[u] = -1;
#pragma unroll
      for (int v = 0; v < 8; ++v)
        if (lo[u] + v < hi[u] && h[u][v] == (int32_t)j) id[u] = lo[u] + v;
      for (int32_t s = lo[u] + 8; s < hi[u]; s += 8) {  // longer ranges
        int32_t x[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) x[v] = head[min(s + v, hi[u] - 1)];
#pragma unroll
        for (int v = 0; v < 8; ++v)
          if (s + v < hi[u] && x[v] == (int32_t)j) id[u] = s + v;
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (r + u >= r1) break;
      if (id[u] < 0) raise_status(st, EB_EINVAL, j);  // cannot happen for a consistent build
      node_in_edge[r + u] = id[u];
    }
  }
}

// local edge index of the local vertex pair (p, q), p < q
template <int D> __host__ __device__ constexpr int pair_index(int p, int q) {
  return D == 3 ? (p == 0 ? q - 1 : (p == 1 ? q + 1 : 5)) : p + q - 1;
}

// Per element, once the sliced entries exist: the sliced position of each
// incidence (its node's slice, column = its rank in the node's row, from
// the positions the scatter pass and the ranks the emit pass recorded) ->
// inc_sell; the out-edge slots of that entry -> the ids of the local edges
// whose tail is that vertex; signs from the vertex order.  All writes are
// per element, contiguous across threads.
constexpr int EM_TB = 256;  // element maps: threads (elements) per block

template <int D, bool WIDE>
__global__ __launch_bounds__(EM_TB) void k_elem_maps(
    const int32_t *__restrict__ elem, int64_t nelem, const int32_t *__restrict__ inc_pos,
    const uint16_t *__restrict__ row_rank, const int32_t *__restrict__ node_sell_off,
    const uint64_t *__restrict__ node_sell, const int32_t *__restrict__ node_edge_off,
    int32_t *elem_edge, int8_t *elem_edge_sign, int32_t *inc_sell, const StatusBlock *st) {
  constexpr int NE = EL<D>::NE;
  // the block's rows of elem_edge and elem_edge_sign, staged so that they
  // leave in whole contiguous lines (a thread's own 24 + 6 bytes would be
  // twelve narrow strided stores)
  __shared__ int32_t s_ee[EM_TB * NE];
  __shared__ int8_t s_sg[EM_TB * NE];
  if (build_failed(st)) return;  // (uniform: only earlier kernels set it)
  const int t = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * EM_TB, e = e0 + t;
  const int nb = (int)min((int64_t)EM_TB, nelem - e0);
  if (e < nelem) {
    int32_t v[D + 1], ip[D + 1], ps[D + 1], ee[NE];
    load_conn<D>(elem, e, v);
    load_conn<D>(inc_pos, e, ip);
#pragma unroll
    for (int le = 0; le < NE; ++le) ee[le] = -1;
#pragma unroll
    for (int l = 0; l <= D; ++l) {
      const int32_t j = v[l];
      const int64_t pos =
          (int64_t)node_sell_off[j / SELL] + (int64_t)SELL * row_rank[ip[l]] + (j % SELL);
      ps[l] = (int32_t)pos;
      const uint32_t code = WIDE ? (uint32_t)(node_sell[2 * pos + 1] >> 32)
                                 : (uint32_t)(node_sell[pos] >> 48) & 0x7fffu;
      const int32_t base = node_edge_off[j];
#pragma unroll
      for (int m = 0; m < D; ++m) {
        const int slot = slot_of<WIDE>(code, m);
        const int lm = m == l ? D : m;  // local index of the m-th other vertex
        const int le = pair_index<D>(l < lm ? l : lm, l < lm ? lm : l);
        if (slot != no_slot<WIDE>()) ee[le] = base + slot;
      }
    }
#pragma unroll
    for (int le = 0; le < NE; ++le) {
      s_ee[t * NE + le] = ee[le];
      s_sg[t * NE + le] = (int8_t)(v[pair_p<D>(le)] < v[pair_q<D>(le)] ? 1 : -1);
    }
    if (inc_sell) {
      if constexpr (D == 3)
        reinterpret_cast<int4 *>(inc_sell)[e] = make_int4(ps[0], ps[1], ps[2], ps[3]);
      else
#pragma unroll
        for (int l = 0; l < 3; ++l) inc_sell[e * 3 + l] = ps[l];
    }
  }
  __syncthreads();
  for (int i = t; i < nb * NE; i += EM_TB) elem_edge[e0 * NE + i] = s_ee[i];
  for (int i = t; i < nb * NE; i += EM_TB) elem_edge_sign[e0 * NE + i] = s_sg[i];
}

// ------------------------------------------------ strip order of the rows
//
// Once the element maps have read the rows in ascending order, each row of
// at most STRIP entries is rewritten as a strip: first its smallest
// incidence, then repeatedly, of those not yet taken in ascending order, the
// first that shares at least D-1 distinct other vertices with the last taken
// (a face of the node's link), else the first sharing the most.  Each
// entry's other vertices (and their out-edge slots with them) are then put
// in places: a vertex the previous entry holds keeps its place there, the
// others fill the free places in order.  Consecutive entries of a strip thus
// differ in one place, which the forward pass exploits (it loads only the
// changed point).  inc_sell keeps the ascending positions: it addresses the
// adjoint's per-incidence pieces, whose node sums do not depend on the order
// of the entries.  One thread per node; its row is staged in LDS.

constexpr int SP_TB = 64;
constexpr int STRIP = 32;  // longest row stored as a strip
static_assert(STRIP <= 32, "the taken set is one 32-bit mask");

template <int D, bool WIDE> struct SellEntry {
  int32_t o[D];
  uint32_t code;
  static constexpr int B = WIDE ? 10 : 5;
  __device__ __forceinline__ void decode(const uint64_t *w, int32_t j) {
    if constexpr (WIDE) {
      o[0] = (int32_t)(uint32_t)w[0];
      o[1] = (int32_t)(uint32_t)(w[0] >> 32);
      if constexpr (D == 3) o[2] = (int32_t)(uint32_t)w[1];
      code = (uint32_t)(w[1] >> 32);
    } else {
#pragma unroll
      for (int m = 0; m < D; ++m) o[m] = j + (int32_t)(int16_t)(uint16_t)(w[0] >> (16 * m));
      code = (uint32_t)(w[0] >> 48) & 0x7fffu;
    }
  }
  __device__ __forceinline__ void encode(uint64_t *w, int32_t j) const {
    if constexpr (WIDE) {
      w[0] = (uint64_t)(uint32_t)o[0] | ((uint64_t)(uint32_t)o[1] << 32);
      w[1] = (uint64_t)(uint32_t)(D == 3 ? o[D - 1] : 0) | ((uint64_t)code << 32);
    } else {
      uint64_t x = (uint64_t)code << 48;
#pragma unroll
      for (int m = 0; m < D; ++m) x |= (uint64_t)(uint16_t)(int16_t)(o[m] - j) << (16 * m);
      w[0] = x;
    }
  }
  // places (see above): S holds the previous entry's vertices by place; place
  // k keeps its vertex when an o_m not yet matched (the first such m) equals
  // it, the unmatched o_m fill the other places in ascending order, and the
  // slot fields move with their vertices
  __device__ __forceinline__ void place(const int32_t (&S)[D]) {
    constexpr uint32_t F = (1u << B) - 1u;
    bool mt[D], kp[D];
#pragma unroll
    for (int m = 0; m < D; ++m) mt[m] = false;
    int32_t no[D];
    uint32_t nc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      kp[k] = false;
      no[k] = S[k];
      nc[k] = F;
#pragma unroll
      for (int m = 0; m < D; ++m) {
        const bool hit = !kp[k] && !mt[m] && o[m] == S[k];
        nc[k] = hit ? (code >> (B * m)) & F : nc[k];
        kp[k] = kp[k] || hit;
        mt[m] = mt[m] || hit;
      }
    }
#pragma unroll
    for (int m = 0; m < D; ++m) {
      bool done = mt[m];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const bool put = !done && !kp[k];
        no[k] = put ? o[m] : no[k];
        nc[k] = put ? (code >> (B * m)) & F : nc[k];
        kp[k] = kp[k] || put;
        done = done || put;
      }
    }
    uint32_t c2 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      o[k] = no[k];
      c2 |= nc[k] << (B * k);
    }
    code = c2;
  }
};

// Two launches: the first (CAP = SP_SHORT) does everything except the strips
// of more than SP_SHORT entries, which the second (CAP = STRIP) walks; the
// smaller LDS rows of the first let more of its waves be resident.
constexpr int SP_SHORT = 24;

template <int D, bool WIDE, int CAP>
__global__ __launch_bounds__(SP_TB) void k_strip(int64_t nv, const int32_t *__restrict__ node_inc_off,
                                                 const int32_t *__restrict__ node_sell_off,
                                                 uint64_t *node_sell, uint32_t *node_step,
                                                 const StatusBlock *st) {
  constexpr int W = WIDE ? 2 : 1;
  constexpr bool FIRST = CAP < STRIP;
  static_assert(CAP == SP_SHORT || CAP == STRIP, "the two launches");
  __shared__ uint64_t row[CAP][W][SP_TB];
  __shared__ uint8_t seq[CAP][SP_TB];
  const int t = threadIdx.x;
  const int64_t j64 = (int64_t)blockIdx.x * SP_TB + t;
  static_assert(SP_TB % SELL == 0, "blocks are whole slices");
  if (build_failed(st)) return;
  if (j64 >= nv) {  // a lane of the last slice with no node: its steps are 0
    if (FIRST && node_step && j64 < n_slices(nv) * SELL) {
      const int64_t sl = j64 / SELL;
      const int32_t slen = (node_sell_off[sl + 1] - node_sell_off[sl]) / SELL;
      for (int32_t c = 0; c < slen; ++c)
        node_step[(int64_t)node_sell_off[sl] + j64 % SELL + (int64_t)SELL * c] = 0;
    }
    return;
  }
  const int32_t j = (int32_t)j64;
  const int32_t len = node_inc_off[j + 1] - node_inc_off[j];
  if (!FIRST && (len <= SP_SHORT || len > STRIP)) return;  // the first launch's rows
  const int64_t base = (int64_t)node_sell_off[j / SELL] + (j % SELL);
  using E = SellEntry<D, WIDE>;
  // the step from the previous entry (vertices by place S) to x (the layout
  // in eb_plan.h; a wide slot field past 30 is "none": a plan with step
  // words has at most 31 out-edges per node)
  auto step_of = [&](const int32_t (&S)[D], const E &x) {
    int changed = 0;
    uint32_t w = 0;
#pragma unroll
    for (int m = D - 1; m >= 0; --m)
      if (x.o[m] != S[m]) {
        ++changed;
        const uint32_t sl = min((x.code >> (E::B * m)) & ((1u << E::B) - 1u), 31u);
        w = ((uint32_t)(x.o[m] - j) & ((1u << STEP_DBITS) - 1u)) | ((uint32_t)m << STEP_PLACE) |
            (sl << STEP_SLOT);
      }
    return changed == 1 ? w : STEP_WHOLE;
  };
  if (FIRST && node_step) {  // zero past the row's end
    const int32_t slen = (node_sell_off[j / SELL + 1] - node_sell_off[j / SELL]) / SELL;
    for (int32_t c = len; c < slen; ++c) node_step[base + (int64_t)SELL * c] = 0;
  }
  if (len > STRIP || len < 2) {  // kept as stored: only the steps
    if (!node_step) return;
    int32_t S[D];
#pragma unroll
    for (int m = 0; m < D; ++m) S[m] = -1;
    for (int32_t c = 0; c < len; ++c) {
      uint64_t w[2] = {node_sell[W * (base + (int64_t)SELL * c)],
                       WIDE ? node_sell[W * (base + (int64_t)SELL * c) + W - 1] : 0};
      E x;
      x.decode(w, j);
      node_step[base + (int64_t)SELL * c] = c == 0 ? STEP_WHOLE : step_of(S, x);
#pragma unroll
      for (int m = 0; m < D; ++m) S[m] = x.o[m];
    }
    return;
  }
  if (len > CAP) return;  // the second launch's rows
  // the row into LDS, eight entries in flight (the tail rereads the last)
  for (int32_t c0 = 0; c0 < len; c0 += 8) {
    uint64_t w[8][W];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < W; ++k)
        w[u][k] = node_sell[W * (base + (int64_t)SELL * min(c0 + u, len - 1)) + k];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < W; ++k) row[min(c0 + u, len - 1)][k][t] = w[u][k];
  }
  auto entry = [&](int32_t q) {
    uint64_t w[2] = {row[q][0][t], WIDE ? row[q][W - 1][t] : 0};
    E x;
    x.decode(w, j);
    return x;
  };
  // the strip (vertices compared as stored: offsets from j, or ids)
  struct Key {
    int32_t v[D];
  };
  auto key = [&](int32_t q) {
    Key k;
    if constexpr (WIDE) {
      const uint64_t w0 = row[q][0][t];
      k.v[0] = (int32_t)(uint32_t)w0;
      k.v[1] = (int32_t)(uint32_t)(w0 >> 32);
      if constexpr (D == 3) k.v[2] = (int32_t)(uint32_t)row[q][W - 1][t];
    } else {
      const uint64_t w0 = row[q][0][t];
#pragma unroll
      for (int m = 0; m < D; ++m) k.v[m] = (int32_t)(int16_t)(uint16_t)(w0 >> (16 * m));
    }
    return k;
  };
  // (an element's vertices are distinct: the build has stopped at any
  // element with a repeated vertex, whose measure is zero)
  auto shared = [](const Key &x, const Key &y) {
    int n = 0;
#pragma unroll
    for (int m = 0; m < D; ++m) {
      bool in = false;
#pragma unroll
      for (int k = 0; k < D; ++k) in = in || y.v[k] == x.v[m];
      n += in ? 1 : 0;
    }
    return n;
  };
  Key cur = key(0);
  seq[0][t] = 0;
  uint32_t rest = (len >= 32 ? 0xffffffffu : (1u << len) - 1u) & ~1u;
  for (int32_t c = 1; c < len; ++c) {
    int best = 0, most = -1;
    Key bk = cur;
    // four candidates per round, all read before any is tested (the same
    // choice as testing them one by one in ascending order)
    constexpr int NC = 4;
    bool done = false;
    for (uint32_t it = rest; it != 0u && !done;) {
      int qs[NC];
      bool ok[NC];
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        ok[u] = it != 0u;
        qs[u] = ok[u] ? __builtin_ctz(it) : 0;
        it &= it - 1u;  // (no-op once empty)
      }
      Key xs[NC];
#pragma unroll
      for (int u = 0; u < NC; ++u) xs[u] = key(qs[u]);
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        if (!ok[u] || done) continue;
        const int sh = shared(xs[u], cur);
        if (sh > most) {
          most = sh;
          best = qs[u];
#pragma unroll
          for (int m = 0; m < D; ++m) bk.v[m] = xs[u].v[m];
          done = sh >= D - 1;
        }
      }
    }
    rest &= ~(1u << best);
    cur = bk;
    seq[c][t] = (uint8_t)best;
  }
  // places, written back in strip order
  int32_t S[D];
#pragma unroll
  for (int m = 0; m < D; ++m) S[m] = -1;
  for (int32_t c = 0; c < len; ++c) {
    E x = entry(seq[c][t]);
    x.place(S);
    if (node_step) node_step[base + (int64_t)SELL * c] = c == 0 ? STEP_WHOLE : step_of(S, x);
#pragma unroll
    for (int m = 0; m < D; ++m) S[m] = x.o[m];
    uint64_t w[2];
    x.encode(w, j);
#pragma unroll
    for (int k = 0; k < W; ++k) node_sell[W * (base + (int64_t)SELL * c) + k] = w[k];
  }
}

// elements per edge, for the optional edge -> element lists
template <int D>
__global__ void k_edge_inc_count(int64_t nelem, const int32_t *__restrict__ elem_edge,
                                 int32_t *cnt, const StatusBlock *st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nelem * EL<D>::NE || build_failed(st)) return;
  atomicAdd(&cnt[elem_edge[i]], 1);
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
    // the face's vertex pairs in lexicographic order
    constexpr int NP = D * (D - 1) / 2;
    int32_t v[D], pa[NP], pb[NP], id[NP];
#pragma unroll
    for (int s = 0; s < D; ++s) v[s] = bface[D * f + s];
    int k = 0;
#pragma unroll
    for (int p = 0; p < D; ++p)
#pragma unroll
      for (int q = p + 1; q < D; ++q) {
        pa[k] = v[p];
        pb[k++] = v[q];
      }
    find_edges<NP>(node_edge_off, head, pa, pb, id);
#pragma unroll
    for (int q = 0; q < NP; ++q) bface_edge[(int64_t)NP * f + q] = id[q];
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

// ------------------------------------------------ four dimensions (dim = 4)
//
// Pentatope grids take a plain form of the build: node rows by a counting
// sort (block-aggregated atomics), rows sorted, and every node through one
// wavefront, its row's other vertices staged in LDS and its neighbours and
// candidate faces kept in LDS sets (the general kernel's successive minima
// beyond the sets' limits).  No kernel plan is made: the dim-4 metric
// kernels walk node_inc directly.  The outputs are the same arrays, with the same
// unique definitions; a boundary face (a tetrahedron) lists its vertices
// ascending, with the last two swapped when that order's area vector
// N(b-a, c-a, d-a) points into the domain.

// The node counts and the scatter aggregate per block in LDS like the
// general passes above (AGG_EPT elements a thread, one global atomic per
// distinct node of the block).
__global__ __launch_bounds__(AGG_TB) void k4_count(const int32_t *__restrict__ elem,
                                                   int64_t nelem, int64_t nv, Coords4 X,
                                                   int32_t *cnt, StatusBlock *st) {
  __shared__ int32_t hk[AGG_HT], hc[AGG_HT];
  for (int i = threadIdx.x; i < AGG_HT; i += AGG_TB) {
    hk[i] = -1;
    hc[i] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * AGG_TB * AGG_EPT + threadIdx.x;
#pragma unroll 1
  for (int k = 0; k < AGG_EPT; ++k) {
    const int64_t e = base + (int64_t)k * AGG_TB;
    if (e >= nelem) continue;
    int32_t v[5];
    load_conn4(elem, e, v);
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 5; ++i) ok = ok && v[i] >= 0 && v[i] < nv;
    if (!ok) {
      raise_status(st, EB_ERANGE, e);
      continue;
    }
    V4 P[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) P[i] = load_pt4(X, v[i]);
    if (pent_det(P) == 0.0) raise_status(st, EB_EDEGENERATE, e);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const int h = agg_slot(hk, v[i]);
      if (h >= 0) atomicAdd(&hc[h], 1);
      else atomicAdd(&cnt[v[i]], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < AGG_HT; i += AGG_TB)
    if (hk[i] >= 0) atomicAdd(&cnt[hk[i]], hc[i]);
}

// cur: the rows' end offsets, taken down to their starts (a range per block
// and node; the rows are sorted afterwards)
__global__ __launch_bounds__(AGG_TB) void k4_scatter(const int32_t *__restrict__ elem,
                                                     int64_t nelem, int64_t nv, int32_t *cur,
                                                     int32_t *node_inc) {
  __shared__ int32_t hk[AGG_HT], hc[AGG_HT];
  for (int i = threadIdx.x; i < AGG_HT; i += AGG_TB) {
    hk[i] = -1;
    hc[i] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * AGG_TB * AGG_EPT + threadIdx.x;
  int32_t slot[AGG_EPT][5], rank[AGG_EPT][5];
#pragma unroll
  for (int k = 0; k < AGG_EPT; ++k) {
    const int64_t e = base + (int64_t)k * AGG_TB;
    int32_t v[5];
    bool ok = e < nelem;
    if (ok) {
      load_conn4(elem, e, v);
#pragma unroll
      for (int i = 0; i < 5; ++i) ok = ok && v[i] >= 0 && v[i] < nv;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      slot[k][i] = -1;
      if (!ok) continue;
      const int h = agg_slot(hk, v[i]);
      if (h >= 0) {
        slot[k][i] = h;
        rank[k][i] = atomicAdd(&hc[h], 1);
      } else {
        node_inc[atomicSub(&cur[v[i]], 1) - 1] = (int32_t)(e * 5 + i);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < AGG_HT; i += AGG_TB)
    if (hk[i] >= 0) {
      const int32_t c = hc[i];
      hc[i] = atomicSub(&cur[hk[i]], c) - c;
    }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < AGG_EPT; ++k) {
    const int64_t e = base + (int64_t)k * AGG_TB;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if (slot[k][i] >= 0) node_inc[hc[slot[k][i]] + rank[k][i]] = (int32_t)(e * 5 + i);
  }
}

// the other vertices of incidence elem*5 + l (local order, l's place taken
// by vertex 4)
__device__ __forceinline__ void others4(const int32_t *elem, int32_t inc, int32_t (&o)[4]) {
  int32_t v[5];
  load_conn4(elem, inc / 5, v);
  const int l = inc % 5;
#pragma unroll
  for (int m = 0; m < 4; ++m) o[m] = l == m ? v[4] : v[m];
}

// candidate face keys of one incidence of j: the triples of its other
// vertices all above j, as (p << 32 | q, r) with p < q < r; (~0, ~0) marks
// none
__device__ __forceinline__ void face_keys4(const int32_t (&o)[4], int32_t j, uint64_t (&kh)[4],
                                           uint64_t (&kl)[4]) {
#pragma unroll
  for (int drop = 0; drop < 4; ++drop) {
    int32_t t[3];
    int n = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (m != drop) t[n++] = o[m];
    // sort three
    int32_t a = min(t[0], t[1]), b = max(t[0], t[1]), c = t[2];
    const int32_t lo = min(a, c), hi = max(b, c), mid = max(a, min(b, c));
    const bool ok = lo > j;
    kh[drop] = ok ? ((uint64_t)(uint32_t)lo << 32 | (uint32_t)mid) : ~0ull;
    kl[drop] = ok ? (uint64_t)(uint32_t)hi : ~0ull;
  }
}

__device__ __forceinline__ bool key_less(uint64_t ah, uint64_t al, uint64_t bh, uint64_t bl) {
  return ah < bh || (ah == bh && al < bl);
}

// the 4D outputs of one boundary face (vertices fv ascending, fv[0] the
// node; inc the holding incidence; f its index): vertex order, owner and
// the rows of the face's vertices
__device__ __forceinline__ void emit_bface4(const TopoArgs &a, const Coords4 &X,
                                            const int32_t (&fv)[4], int32_t inc, int32_t f) {
  int32_t v[5];
  load_conn4(a.elem, inc / 5, v);
  // the owner's vertex off the face
  int opp = 0;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    bool on = false;
#pragma unroll
    for (int s = 0; s < 4; ++s) on = on || v[q] == fv[s];
    if (!on) opp = q;
  }
  // outward order: the expression and operand order of the definition, FP64
  // without contraction
  bool keep;
  {
#pragma clang fp contract(off)
    const V4 A = load_pt4(X, fv[0]);
    const V4 N = v4_cross(v4_sub(load_pt4(X, fv[1]), A), v4_sub(load_pt4(X, fv[2]), A),
                          v4_sub(load_pt4(X, fv[3]), A));
    keep = v4_dot(N, v4_sub(A, load_pt4(X, v[opp]))) > 0;
  }
  int32_t *bf = a.bface + (int64_t)4 * f;
  bf[0] = fv[0];
  bf[1] = fv[1];
  bf[2] = keep ? fv[2] : fv[3];
  bf[3] = keep ? fv[3] : fv[2];
  a.bface_owner[f] = (int32_t)((int64_t)(inc / 5) * 5 + opp);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int32_t pos = atomicSub(&a.bf_cur[fv[s]], 1) - 1;
    a.bnode_face[pos] = f;
  }
}

// The per-node passes by successive minima over the row (the form of the
// general kernel): any row length and neighbour count.  ro: the row's other
// vertices staged in LDS, or null to read them from the connectivity.
template <bool EMIT>
__device__ void node_topo4_rounds(const TopoArgs &a, int32_t j, int lane, const int4 *ro) {
  const int32_t r0 = a.node_inc_off[j], r1 = a.node_inc_off[j + 1];
  const int32_t len = r1 - r0;
  const Coords4 X{a.X.x, a.X.y, a.X.z, a.xw};
  auto others_at = [&](int32_t i, int32_t (&o)[4]) __attribute__((always_inline)) {
    if (ro) {
      const int4 q = ro[i];
      o[0] = q.x;
      o[1] = q.y;
      o[2] = q.z;
      o[3] = q.w;
    } else {
      others4(a.elem, a.node_inc[r0 + i], o);
    }
  };

  // 1. distinct neighbours, ascending (as in the general kernel)
  int32_t e0 = 0, in_end = 0, nlow_known = 0;
  if constexpr (EMIT) {
    e0 = a.eoff[j];
    in_end = a.in_cur[j];
    nlow_known = a.ein_scan[j] - (j > 0 ? a.ein_scan[j - 1] : 0);
  }
  int32_t last = INT32_MIN, nh = 0, nlow = 0;
  for (;;) {
    int32_t mn = INT32_MAX;
    for (int32_t i = lane; i < len; i += 64) {
      int32_t o[4];
      others_at(i, o);
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (o[m] > last) mn = min(mn, o[m]);
    }
    mn = wave_min_i32(mn);
    if (mn == INT32_MAX) break;
    if constexpr (EMIT) {
      if (lane == 0) {
        if (mn < j) {
          a.node_in_edge[in_end - nlow_known + nh] = mn;
        } else {
          a.edge_tail[e0 + nh - nlow] = j;
          a.edge_head[e0 + nh - nlow] = mn;
        }
      }
    }
    if (mn < j) ++nlow;
    ++nh;
    last = mn;
  }
  if constexpr (!EMIT) {
    if (lane == 0) {
      a.outdeg[j] = nh - nlow;
      a.ein[j] = nlow;
    }
  } else {
    if (lane == 0) a.in_cur[j] = in_end - nlow;
  }

  // 2. candidate faces with j as smallest vertex in ascending key order,
  //    each counted over the row the round after it is found
  int32_t nb = 0, f = EMIT ? a.foff[j] : 0;
  uint64_t ch = 0, cl = 0;
  bool have = false;
  for (;;) {
    uint64_t bh = ~0ull, bl = ~0ull;
    int32_t cnt = 0, holder = INT32_MAX;
    for (int32_t i = lane; i < len; i += 64) {
      int32_t o[4];
      others_at(i, o);
      uint64_t kh[4], kl[4];
      face_keys4(o, j, kh, kl);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (kh[c] == ~0ull) continue;
        if ((!have || key_less(ch, cl, kh[c], kl[c])) && key_less(kh[c], kl[c], bh, bl)) {
          bh = kh[c];
          bl = kl[c];
        }
        if (have && kh[c] == ch && kl[c] == cl) {
          ++cnt;
          holder = min(holder, i);
        }
      }
    }
    const uint64_t mh = wave_min_u64(bh);
    const uint64_t ml = wave_min_u64(bh == mh ? bl : ~0ull);
    if (have) {
      cnt = wave_sum_i32(cnt);
      holder = wave_min_i32(holder);
      if (cnt > 2) {
        if (lane == 0) raise_status(a.st, EB_ENONMANIFOLD, j);
        return;
      }
      if (cnt == 1) {
        const int32_t fv[4] = {j, (int32_t)(ch >> 32), (int32_t)(uint32_t)ch, (int32_t)cl};
        if (lane == 0) {
          if constexpr (!EMIT) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              a.bflag[fv[s]] = 1;
              atomicAdd(&a.bfn[fv[s]], 1);
            }
          } else {
            emit_bface4(a, X, fv, a.node_inc[r0 + holder], f);
          }
        }
        ++nb;
        ++f;
      }
    }
    if (mh == ~0ull) break;
    ch = mh;
    cl = ml;
    have = true;
  }
  if constexpr (!EMIT) {
    if (lane == 0) a.fmin[j] = nb;
  }
}

// The per-node passes over LDS sets, for rows of at most R4_CAP incidences
// with at most H4/2 distinct neighbours and H4/2 distinct candidate faces:
// the neighbours go into an open-addressing set and are ranked by counting;
// a candidate face is keyed by the ranks of its three vertices above the node
// among those neighbours (8 bits each), counted in a second set together
// with the sum of its holders' row positions (exact when it is held once).
// Ranks keep vertex order, so both orders are those of the rounds form.
// (The sizes keep a block's LDS near 9 KB: four resident waves per SIMD.)
constexpr int R4_CAP = 192;
constexpr int H4_LOG = 8, H4 = 1 << H4_LOG;
constexpr uint32_t H4_EMPTY = ~0u;

struct Topo4Lds {
  int4 ro[R4_CAP];     // the row's other vertices
  ushort4 sl[R4_CAP];  // and their slots in the neighbour set
  int32_t nr[H4];      // a neighbour's rank among the distinct neighbours
  int32_t sn[H4 / 2];  // the distinct neighbours ascending
  // the neighbour set nk [H4]; once ranked, the candidate face set fk [H4]
  // (rank triples) and fc [H4] (count << 16 plus the sum of the holders'
  // row positions)
  uint32_t sets[2 * H4];
  // the distinct neighbours in set order tl [H4/2 + 4] (padded to fours)
  // and their slots ts [H4/2]; later the faces held once bl [H4/2]
  // (key << 8 | position)
  __align__(16) int32_t lists[H4 + 4];
  int32_t n_nb, n_face, over;
};

__device__ __forceinline__ uint32_t h4_slot(uint32_t k) {
  return (k * 2654435761u) >> (32 - H4_LOG);
}

// k's slot in tab, inserted when absent (counting it in *count); -1 and
// *over set when the set is full
__device__ __forceinline__ int h4_insert(uint32_t *tab, uint32_t k, int32_t *count,
                                         int32_t *over) {
  uint32_t h = h4_slot(k);
  for (int p = 0; p < H4; ++p) {
    const uint32_t old = atomicCAS(&tab[h], H4_EMPTY, k);
    if (old == H4_EMPTY) {
      atomicAdd(count, 1);
      return (int)h;
    }
    if (old == k) return (int)h;
    h = (h + 1) & (H4 - 1);
  }
  *over = 1;
  return -1;
}

// false (and nothing written) when the row does not fit the sets
template <bool EMIT>
__device__ bool node_topo4_sets(const TopoArgs &a, int32_t j, int lane, int32_t r0, int32_t len,
                                Topo4Lds &L) {
  const Coords4 X{a.X.x, a.X.y, a.X.z, a.xw};
  const uint64_t below = (1ull << lane) - 1;
  uint32_t *const nk = L.sets, *const fk = L.sets, *const fc = L.sets + H4;
  int32_t *const tl = L.lists, *const ts = L.lists + H4 / 2 + 4;
  uint32_t *const bl = reinterpret_cast<uint32_t *>(L.lists);
  for (int s = lane; s < H4; s += 64) nk[s] = H4_EMPTY;
  if (lane == 0) {
    L.n_nb = 0;
    L.n_face = 0;
    L.over = 0;
  }
  __syncthreads();
  // 1. the distinct neighbours
  for (int32_t i = lane; i < len; i += 64) {
    const int4 q = L.ro[i];
    // (a slot of -1, the set full, is never read: the row falls back)
    L.sl[i] = make_ushort4((uint16_t)h4_insert(nk, (uint32_t)q.x, &L.n_nb, &L.over),
                           (uint16_t)h4_insert(nk, (uint32_t)q.y, &L.n_nb, &L.over),
                           (uint16_t)h4_insert(nk, (uint32_t)q.z, &L.n_nb, &L.over),
                           (uint16_t)h4_insert(nk, (uint32_t)q.w, &L.n_nb, &L.over));
  }
  __syncthreads();
  const int32_t nd = L.n_nb;
  if (L.over || nd > H4 / 2) return false;
  int32_t nlow = 0;
  {
    int32_t base = 0;
    for (int s0 = 0; s0 < H4; s0 += 64) {
      const uint32_t v = nk[s0 + lane];
      const bool has = v != H4_EMPTY;
      const uint64_t m = __builtin_amdgcn_ballot_w64(has);
      const int pos = base + __builtin_popcountll(m & below);
      if (has) {
        tl[pos] = (int32_t)v;
        ts[pos] = s0 + lane;
      }
      base += __builtin_popcountll(m);
      nlow += __builtin_popcountll(__builtin_amdgcn_ballot_w64(has && (int32_t)v < j));
    }
    if (lane < 4) tl[nd + lane] = INT32_MAX;
  }
  __syncthreads();
  const int4 *const tl4 = reinterpret_cast<const int4 *>(tl);
  for (int32_t idx = lane; idx < nd; idx += 64) {
    const int32_t v = tl[idx];
    int32_t r = 0;
    for (int32_t u = 0; u < nd; u += 4) {
      const int4 w = tl4[u >> 2];
      r += (w.x < v ? 1 : 0) + (w.y < v ? 1 : 0) + (w.z < v ? 1 : 0) + (w.w < v ? 1 : 0);
    }
    L.nr[ts[idx]] = r;
    L.sn[r] = v;
  }
  for (int s = lane; s < H4; s += 64) {  // (the neighbour set is read out)
    fk[s] = H4_EMPTY;
    fc[s] = 0;
  }
  __syncthreads();
  // 2. candidate faces with the node as smallest vertex
  for (int32_t i = lane; i < len; i += 64) {
    const int4 q = L.ro[i];
    const ushort4 g = L.sl[i];
    const int32_t o[4] = {q.x, q.y, q.z, q.w};
    const int32_t so[4] = {g.x, g.y, g.z, g.w};
    int32_t ru[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) ru[m] = o[m] > j ? L.nr[so[m]] - nlow : -1;
#pragma unroll
    for (int drop = 0; drop < 4; ++drop) {
      int32_t t[3];
      int n = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (m != drop) t[n++] = ru[m];
      const int32_t x = min(t[0], t[1]), y = max(t[0], t[1]), z = t[2];
      const int32_t lo = min(x, z), hi = max(y, z), mid = max(x, min(y, z));
      if (lo < 0) continue;
      const int s = h4_insert(fk, (uint32_t)(lo << 16 | mid << 8 | hi), &L.n_face, &L.over);
      if (s >= 0) atomicAdd(&fc[s], 0x10000u + (uint32_t)i);
    }
  }
  __syncthreads();
  if (L.over || L.n_face > H4 / 2) return false;

  // the neighbours' outputs
  if constexpr (EMIT) {
    const int32_t e0 = a.eoff[j], in_end = a.in_cur[j];
    const int32_t nlow_known = a.ein_scan[j] - (j > 0 ? a.ein_scan[j - 1] : 0);
    for (int32_t r = lane; r < nd; r += 64) {
      const int32_t v = L.sn[r];
      if (v < j) {
        a.node_in_edge[in_end - nlow_known + r] = v;
      } else {
        a.edge_tail[e0 + r - nlow] = j;
        a.edge_head[e0 + r - nlow] = v;
      }
    }
    if (lane == 0) a.in_cur[j] = in_end - nlow;
  } else if (lane == 0) {
    a.outdeg[j] = nd - nlow;
    a.ein[j] = nlow;
  }

  // the faces held once, and any held more than twice
  int32_t nb = 0;
  bool bad = false;
  for (int s0 = 0; s0 < H4; s0 += 64) {
    const uint32_t k = fk[s0 + lane], c = fc[s0 + lane];
    const bool has = k != H4_EMPTY;
    bad = bad || (has && (c >> 16) > 2);
    const bool once = has && (c >> 16) == 1;
    const uint64_t m = __builtin_amdgcn_ballot_w64(once);
    if (once) bl[nb + __builtin_popcountll(m & below)] = k << 8 | (c & 0xFFu);
    nb += __builtin_popcountll(m);
  }
  if (__builtin_amdgcn_ballot_w64(bad) != 0) {
    if (lane == 0) raise_status(a.st, EB_ENONMANIFOLD, j);
    return true;
  }
  __syncthreads();
  const int32_t f0 = EMIT ? a.foff[j] : 0;
  for (int32_t idx = lane; idx < nb; idx += 64) {
    const uint32_t b = bl[idx], k = b >> 8;
    const int32_t fv[4] = {j, L.sn[nlow + (int32_t)(k >> 16)],
                           L.sn[nlow + (int32_t)((k >> 8) & 0xFFu)],
                           L.sn[nlow + (int32_t)(k & 0xFFu)]};
    if constexpr (!EMIT) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a.bflag[fv[s]] = 1;
        atomicAdd(&a.bfn[fv[s]], 1);
      }
    } else {
      int32_t r = 0;
      for (int32_t u = 0; u < nb; ++u) r += bl[u] < b ? 1 : 0;
      emit_bface4(a, X, fv, a.node_inc[r0 + (int32_t)(b & 0xFFu)], f0 + r);
    }
  }
  if constexpr (!EMIT) {
    if (lane == 0) a.fmin[j] = nb;
  }
  return true;
}

template <bool EMIT>
__global__ __launch_bounds__(64) void k4_node_topo(TopoArgs a) {
  __shared__ Topo4Lds L;
  if (build_failed(a.st)) return;
  const int lane = (int)threadIdx.x;
  for (int64_t jj = blockIdx.x; jj < a.nv; jj += gridDim.x) {
    const int32_t j = (int32_t)jj;
    const int32_t r0 = a.node_inc_off[j], len = a.node_inc_off[j + 1] - r0;
    const bool staged = len <= R4_CAP;
    __syncthreads();  // (the previous node is done with the LDS)
    if (staged)
      for (int32_t i = lane; i < len; i += 64) {
        int32_t o[4];
        others4(a.elem, a.node_inc[r0 + i], o);
        L.ro[i] = make_int4(o[0], o[1], o[2], o[3]);
      }
    __syncthreads();
    if (!staged || !node_topo4_sets<EMIT>(a, j, lane, r0, len, L))
      node_topo4_rounds<EMIT>(a, j, lane, staged ? L.ro : nullptr);
  }
}

// element -> edge map and signs: the ten local pairs in lexicographic order
__global__ void k4_elem_maps(const int32_t *__restrict__ elem, int64_t nelem,
                             const int32_t *__restrict__ node_edge_off,
                             const int32_t *__restrict__ head, int32_t *elem_edge,
                             int8_t *elem_edge_sign, StatusBlock *st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nelem || build_failed(st)) return;
  int32_t v[5], pa[10], pb[10], id[10];
  load_conn4(elem, e, v);
  int k = 0;
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = p + 1; q < 5; ++q) {
      pa[k] = v[p];
      pb[k++] = v[q];
    }
  find_edges<10>(node_edge_off, head, pa, pb, id);
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    if (id[q] < 0) raise_status(st, EB_EINVAL, e);  // cannot happen for a consistent build
    elem_edge[e * 10 + q] = id[q];
    elem_edge_sign[e * 10 + q] = (int8_t)(pa[q] < pb[q] ? 1 : -1);
  }
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
  // the per-node arrays and slice lengths are contiguous lines of the workspace
  EB_TRY(fill_i32(eoff, (int64_t)((L.scan_tmp - L.eoff) / 4), 0, s));
  EB_TRY(fill_i32(node_inc_off, nv + 1, 0, s));

  // node -> element lists
  if (nelem > 0) {
    hipLaunchKernelGGL(k_count_nodes<D>, dim3(grid_for(nelem, AGG_TB * AGG_EPT)), dim3(AGG_TB),
                       0, s, elem, nelem, nv, X, node_inc_off, st);
    EB_LAUNCH_CHECK();
  }
  // the row ends must be the scan total of what was counted: elements
  // rejected above are neither counted nor scattered
  EB_TRY(scan_inclusive(node_inc_off, node_inc_off, nv, node_inc_off + nv, tmp, s));
  if (nelem > 0) {
    // the row ends, fixed for the scatter (the edge-offset array is free until
    // the count pass)
    int32_t *ends = ws_at<int32_t>(ws, L.eoff);
    EB_HIP_CHECK(hipMemcpyAsync(ends, node_inc_off, sizeof(int32_t) * (size_t)nv,
                                hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_scatter_nodes<D>, dim3(grid_for(nelem, AGG_TB * AGG_EPT)),
                       dim3(AGG_TB), 0, s, elem, nelem, nv, node_inc_off, (const int32_t *)ends,
                       ws_at<int4>(ws, L.rows4), ws_at<int32_t>(ws, L.inc_pos), node_inc);
    EB_LAUNCH_CHECK();
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(pass == 0 ? k_row_rank<RK_SHORT> : k_row_rank<RK_CAP>,
                         dim3(grid_for(nv, RK_TB)), dim3(RK_TB), 0, s, nv,
                         (const int32_t *)node_inc_off, (const int4 *)ws_at<int4>(ws, L.rows4),
                         node_inc, ws_at<uint16_t>(ws, L.row_rank), (const StatusBlock *)st);
      EB_LAUNCH_CHECK();
    }
  }

  // per-node counts of edges, boundary faces, boundary nodes
  TopoArgs ta{};
  ta.nv = nv;
  ta.elem = elem;
  ta.X = X;
  ta.node_inc_off = node_inc_off;
  ta.node_inc = node_inc;
  ta.rows4 = ws_at<const int32_t>(ws, L.rows4);
  ta.nset = ws_at<int32_t>(ws, L.nset);
  ta.row_rank = ws_at<const uint16_t>(ws, L.row_rank);
  ta.outdeg = eoff;
  ta.fmin = foff;
  ta.bflag = bidx;
  ta.bfn = bfn;
  ta.ein = ein;
  ta.queue = ws_at<int32_t>(ws, L.queue);
  ta.st = st;
  hipLaunchKernelGGL((k_node_topo<D, false>), dim3(grid_for(nv, TB)), dim3(TB), 0, s, ta);
  EB_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_node_topo_general<D, false>), dim3(1024), dim3(64), 0, s, ta);
  EB_LAUNCH_CHECK();
  // the per-node counts become offsets, all five in one scan pass
  ScanJobs J{};
  const int32_t *sin[5] = {eoff, foff, bidx, bfn, ein};
  int32_t *sout[5] = {eoff, foff, bidx, bfn_scan, ein};
  int32_t *stot[5] = {&st->totals[T_EDGES], &st->totals[T_BFACES], &st->totals[T_BNODES],
                      nullptr, nullptr};
  const int32_t sincl[5] = {0, 0, 0, 1, 1};
  for (int q = 0; q < 5; ++q) {
    J.in[q] = sin[q];
    J.out[q] = sout[q];
    J.total[q] = stot[q];
    J.inclusive[q] = sincl[q];
  }
  EB_TRY(scan_many(J, 5, nv + 1, tmp, s));
  const int64_t nsl = n_slices(nv);
  int32_t *slen = ws_at<int32_t>(ws, L.slen);
  hipLaunchKernelGGL(k_slice_len, dim3(grid_for(nsl, 256)), dim3(256), 0, s,
                     (const int32_t *)node_inc_off, nv, slen, st);
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
  // (the slice lengths sum to at most the (D+1) n_elems < 2^31 incidences,
  // so their scan does not wrap; the slot count is 64 times that)
  const int64_t n_slots = (int64_t)SELL * h.totals[T_SELL_ROWS];
  sizes->plan_param[0] = n_slots;
  // narrow entries while every neighbour offset fits int16; wide ones with
  // step words while the offsets fit the words' 20 bits; else wide alone
  // (more than 31 out-edges need the wide 10-bit slot fields either way)
  sizes->plan_param[1] = h.totals[T_MAXOUT] > 31             ? PLAN_WIDE
                         : h.totals[T_MAXDELTA] <= 32767         ? PLAN_NARROW
                         : h.totals[T_MAXDELTA] <= STEP_MAX_DELTA ? PLAN_WIDE_STEPS
                                                                  : PLAN_WIDE;
  sizes->plan_bytes = (int64_t)plan_bytes_of(sizes);
  if (h.status != EB_OK) {
    set_detail("%s at %s %lld", eb_status_string(h.status),
               h.status == EB_ERANGE || h.status == EB_EDEGENERATE ? "element" : "node",
               (long long)h.detail);
    return h.status;
  }
  if (h.totals[T_MAXROW] > MAX_NODE_ELEMS || h.totals[T_MAXOUT] > MAX_OUT_EDGES) {
    set_detail("a node has %d elements (at most %d) or %d out-edges (at most %d)",
               h.totals[T_MAXROW], MAX_NODE_ELEMS, h.totals[T_MAXOUT], MAX_OUT_EDGES);
    return EB_ECAPACITY;
  }
  if (n_slots >= (int64_t(1) << 31)) {
    set_detail("the kernel plan would have %lld slots (int32 indexing)", (long long)n_slots);
    return EB_EOVERFLOW;
  }
  return EB_OK;
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

  const PlanPtrs pl = plan_ptrs(sz, tp->plan);
  const int64_t nsl = n_slices(nv);
  hipLaunchKernelGGL(k_emit_slices, dim3(grid_for(nsl + 1, 256)), dim3(256), 0, s,
                     (const int32_t *)ws_at<int32_t>(ws, L.slen), nsl, pl.slice_off,
                     (const StatusBlock *)st);
  EB_LAUNCH_CHECK();

  TopoArgs ta{};
  ta.nv = nv;
  ta.elem = elem;
  ta.X = coords_rows(coords, D, nv);
  ta.node_inc_off = tp->node_inc_off;
  ta.node_inc = tp->node_inc;
  ta.rows4 = ws_at<const int32_t>(ws, L.rows4);
  ta.nset = ws_at<int32_t>(ws, L.nset);
  ta.row_rank = ws_at<const uint16_t>(ws, L.row_rank);
  ta.eoff = eoff;
  ta.foff = foff;
  ta.ein_scan = ein;
  ta.edge_tail = tp->edge;
  ta.edge_head = tp->edge + sz->n_edges;
  ta.bface = tp->bface;
  ta.bface_owner = tp->bface_owner;
  ta.in_cur = tp->node_in_off;
  ta.node_in_edge = tp->node_in_edge;
  ta.bf_cur = bfn_scan;
  ta.bnode_face = tp->bnode_face;
  ta.node_sell_off = pl.slice_off;
  ta.node_sell = pl.entry;
  ta.sell_wide = plan_wide(sz);
  ta.queue = ws_at<int32_t>(ws, L.queue);
  ta.st = st;
  hipLaunchKernelGGL((k_node_topo<D, true>), dim3(grid_for(nv, TB)), dim3(TB), 0, s, ta);
  EB_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_node_topo_general<D, true>), dim3(1024), dim3(64), 0, s, ta);
  EB_LAUNCH_CHECK();
  if (sz->n_edges > 0) {
    hipLaunchKernelGGL(k_node_in_ids, dim3(grid_for(nv, 256)), dim3(256), 0, s, nv,
                       (const int32_t *)tp->node_in_off, (const int32_t *)tp->node_edge_off,
                       (const int32_t *)(tp->edge + sz->n_edges), tp->node_in_edge, st);
    EB_LAUNCH_CHECK();
  }
  EB_TRY(rowsort(tp->bnode_face_off, tp->bnode_face, sz->n_bnodes, s));
  if (nelem > 0) {
    if (plan_wide(sz))
      hipLaunchKernelGGL((k_elem_maps<D, true>), dim3(grid_for(nelem, EM_TB)), dim3(EM_TB), 0, s,
                         elem, nelem, (const int32_t *)ws_at<int32_t>(ws, L.inc_pos),
                         (const uint16_t *)ws_at<uint16_t>(ws, L.row_rank),
                         (const int32_t *)pl.slice_off,
                         (const uint64_t *)pl.entry, (const int32_t *)tp->node_edge_off,
                         tp->elem_edge, tp->elem_edge_sign, pl.inc_slot, (const StatusBlock *)st);
    else
      hipLaunchKernelGGL((k_elem_maps<D, false>), dim3(grid_for(nelem, EM_TB)), dim3(EM_TB), 0, s,
                         elem, nelem, (const int32_t *)ws_at<int32_t>(ws, L.inc_pos),
                         (const uint16_t *)ws_at<uint16_t>(ws, L.row_rank),
                         (const int32_t *)pl.slice_off,
                         (const uint64_t *)pl.entry, (const int32_t *)tp->node_edge_off,
                         tp->elem_edge, tp->elem_edge_sign, pl.inc_slot, (const StatusBlock *)st);
    EB_LAUNCH_CHECK();
  }

  if (nelem > 0) {  // rows in strip order (after the element maps read them ascending)
    if (plan_wide(sz))
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(pass == 0 ? (k_strip<D, true, SP_SHORT>) : (k_strip<D, true, STRIP>),
                           dim3(grid_for(nv, SP_TB)), dim3(SP_TB), 0, s, nv,
                           (const int32_t *)tp->node_inc_off, (const int32_t *)pl.slice_off,
                           pl.entry, pl.step, (const StatusBlock *)st);
        EB_LAUNCH_CHECK();
      }
    else
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(pass == 0 ? (k_strip<D, false, SP_SHORT>) : (k_strip<D, false, STRIP>),
                           dim3(grid_for(nv, SP_TB)), dim3(SP_TB), 0, s, nv,
                           (const int32_t *)tp->node_inc_off, (const int32_t *)pl.slice_off,
                           pl.entry, pl.step, (const StatusBlock *)st);
        EB_LAUNCH_CHECK();
      }
  }

  const bool want_inc = tp->edge_inc_off && tp->edge_inc;
  if (want_inc) {
    EB_TRY(fill_i32(tp->edge_inc_off, sz->n_edges + 1, 0, s));
    if (nelem > 0) {
      hipLaunchKernelGGL(k_edge_inc_count<D>, dim3(grid_for(nelem * NE, 256)), dim3(256), 0, s,
                         nelem, (const int32_t *)tp->elem_edge, tp->edge_inc_off, st);
      EB_LAUNCH_CHECK();
    }
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


// ---------------------------------------------------- dim 4 host side

int build4_impl(int64_t nv, int64_t nelem, const int32_t *elem, const double *coords,
                int32_t *node_inc_off, int32_t *node_inc, void *ws, eb_sizes *sizes,
                hipStream_t s) {
  const WsLayout L = ws_layout(4, nv, nelem);
  StatusBlock *st = ws_at<StatusBlock>(ws, 0);
  int32_t *eoff = ws_at<int32_t>(ws, L.eoff), *foff = ws_at<int32_t>(ws, L.foff);
  int32_t *bidx = ws_at<int32_t>(ws, L.bidx), *bfn = ws_at<int32_t>(ws, L.bfn);
  int32_t *bfn_scan = ws_at<int32_t>(ws, L.bfn_scan), *ein = ws_at<int32_t>(ws, L.ein_scan);
  int32_t *tmp = ws_at<int32_t>(ws, L.scan_tmp);
  const Coords4 X = coords4_rows(coords, nv);

  EB_TRY(fill_i32(reinterpret_cast<int32_t *>(st), sizeof(StatusBlock) / 4, 0, s));
  EB_TRY(fill_i32(eoff, (int64_t)((L.scan_tmp - L.eoff) / 4), 0, s));
  EB_TRY(fill_i32(node_inc_off, nv + 1, 0, s));
  if (nelem > 0) {
    hipLaunchKernelGGL(k4_count, dim3(grid_for(nelem, AGG_TB * AGG_EPT)), dim3(AGG_TB), 0, s,
                       elem, nelem, nv, X, node_inc_off, st);
    EB_LAUNCH_CHECK();
  }
  EB_TRY(scan_inclusive(node_inc_off, node_inc_off, nv, node_inc_off + nv, tmp, s));
  if (nelem > 0) {
    hipLaunchKernelGGL(k4_scatter, dim3(grid_for(nelem, AGG_TB * AGG_EPT)), dim3(AGG_TB), 0, s,
                       elem, nelem, nv, node_inc_off, node_inc);
    EB_LAUNCH_CHECK();
    EB_TRY(rowsort(node_inc_off, node_inc, nv, s));
  }
  TopoArgs ta{};
  ta.nv = nv;
  ta.elem = elem;
  ta.X = Coords{X.x, X.y, X.z};
  ta.xw = X.w;
  ta.node_inc_off = node_inc_off;
  ta.node_inc = node_inc;
  ta.outdeg = eoff;
  ta.fmin = foff;
  ta.bflag = bidx;
  ta.bfn = bfn;
  ta.ein = ein;
  ta.st = st;
  hipLaunchKernelGGL((k4_node_topo<false>), dim3((unsigned)std::min<int64_t>(nv, 16384)), dim3(64),
                     0, s, ta);
  EB_LAUNCH_CHECK();
  ScanJobs J{};
  const int32_t *sin[5] = {eoff, foff, bidx, bfn, ein};
  int32_t *sout[5] = {eoff, foff, bidx, bfn_scan, ein};
  int32_t *stot[5] = {&st->totals[T_EDGES], &st->totals[T_BFACES], &st->totals[T_BNODES],
                      nullptr, nullptr};
  const int32_t sincl[5] = {0, 0, 0, 1, 1};
  for (int q = 0; q < 5; ++q) {
    J.in[q] = sin[q];
    J.out[q] = sout[q];
    J.total[q] = stot[q];
    J.inclusive[q] = sincl[q];
  }
  EB_TRY(scan_many(J, 5, nv + 1, tmp, s));
  StatusBlock h;
  EB_HIP_CHECK(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
  EB_HIP_CHECK(hipStreamSynchronize(s));
  sizes->dim = 4;
  sizes->n_nodes = nv;
  sizes->n_elems = nelem;
  sizes->n_edges = h.totals[T_EDGES];
  sizes->n_bfaces = h.totals[T_BFACES];
  sizes->n_bnodes = h.totals[T_BNODES];
  sizes->plan_param[0] = 0;  // no kernel plan in four dimensions
  sizes->plan_param[1] = 0;
  sizes->plan_bytes = (int64_t)plan_bytes_of(sizes);
  if (h.status != EB_OK) {
    set_detail("%s at %s %lld", eb_status_string(h.status),
               h.status == EB_ERANGE || h.status == EB_EDEGENERATE ? "element" : "node",
               (long long)h.detail);
    return h.status;
  }
  return EB_OK;
}

int emit4_impl(const eb_sizes *sz, const int32_t *elem, const double *coords,
               const eb_topology *tp, void *ws, hipStream_t s) {
  const int64_t nv = sz->n_nodes, nelem = sz->n_elems;
  const WsLayout L = ws_layout(4, nv, nelem);
  StatusBlock *st = ws_at<StatusBlock>(ws, 0);
  int32_t *eoff = ws_at<int32_t>(ws, L.eoff), *foff = ws_at<int32_t>(ws, L.foff);
  int32_t *bidx = ws_at<int32_t>(ws, L.bidx), *bfn = ws_at<int32_t>(ws, L.bfn);
  int32_t *bfn_scan = ws_at<int32_t>(ws, L.bfn_scan), *ein = ws_at<int32_t>(ws, L.ein_scan);
  int32_t *tmp = ws_at<int32_t>(ws, L.scan_tmp);
  constexpr int NE = 10;
  const Coords4 X = coords4_rows(coords, nv);

  EmitNodeArgs en{nv, 4, eoff, bidx, bfn, bfn_scan, ein, tp->node_edge_off, tp->node_bnode,
                  tp->bnode, tp->bnode_face_off, tp->node_in_off, st};
  hipLaunchKernelGGL(k_emit_nodes, dim3(grid_for(nv + 1, 256)), dim3(256), 0, s, en);
  EB_LAUNCH_CHECK();
  TopoArgs ta{};
  ta.nv = nv;
  ta.elem = elem;
  ta.X = Coords{X.x, X.y, X.z};
  ta.xw = X.w;
  ta.node_inc_off = tp->node_inc_off;
  ta.node_inc = tp->node_inc;
  ta.eoff = eoff;
  ta.foff = foff;
  ta.ein_scan = ein;
  ta.edge_tail = tp->edge;
  ta.edge_head = tp->edge + sz->n_edges;
  ta.bface = tp->bface;
  ta.bface_owner = tp->bface_owner;
  ta.in_cur = tp->node_in_off;
  ta.node_in_edge = tp->node_in_edge;
  ta.bf_cur = bfn_scan;
  ta.bnode_face = tp->bnode_face;
  ta.st = st;
  hipLaunchKernelGGL((k4_node_topo<true>), dim3((unsigned)std::min<int64_t>(nv, 16384)), dim3(64),
                     0, s, ta);
  EB_LAUNCH_CHECK();
  if (sz->n_edges > 0) {
    hipLaunchKernelGGL(k_node_in_ids, dim3(grid_for(nv, 256)), dim3(256), 0, s, nv,
                       (const int32_t *)tp->node_in_off, (const int32_t *)tp->node_edge_off,
                       (const int32_t *)(tp->edge + sz->n_edges), tp->node_in_edge, st);
    EB_LAUNCH_CHECK();
  }
  EB_TRY(rowsort(tp->bnode_face_off, tp->bnode_face, sz->n_bnodes, s));
  if (nelem > 0) {
    hipLaunchKernelGGL(k4_elem_maps, dim3(grid_for(nelem, 256)), dim3(256), 0, s, elem, nelem,
                       (const int32_t *)tp->node_edge_off,
                       (const int32_t *)(tp->edge + sz->n_edges), tp->elem_edge,
                       tp->elem_edge_sign, st);
    EB_LAUNCH_CHECK();
  }
  const bool want_inc = tp->edge_inc_off && tp->edge_inc;
  if (want_inc) {
    EB_TRY(fill_i32(tp->edge_inc_off, sz->n_edges + 1, 0, s));
    if (nelem > 0) {
      hipLaunchKernelGGL(k_edge_inc_count<4>, dim3(grid_for(nelem * NE, 256)), dim3(256), 0, s,
                         nelem, (const int32_t *)tp->elem_edge, tp->edge_inc_off, st);
      EB_LAUNCH_CHECK();
    }
  }
  if (sz->n_bfaces > 0) {
    hipLaunchKernelGGL(k_bface_edge<4>, dim3(grid_for(sz->n_bfaces, 256)), dim3(256), 0, s,
                       (const int32_t *)tp->bface, sz->n_bfaces,
                       (const int32_t *)tp->node_edge_off,
                       (const int32_t *)(tp->edge + sz->n_edges), tp->bface_edge, st);
    EB_LAUNCH_CHECK();
  }
  if (want_inc) {
    EB_TRY(scan_inclusive(tp->edge_inc_off, tp->edge_inc_off, sz->n_edges, nullptr, tmp, s));
    EB_TRY(fill_i32(tp->edge_inc_off + sz->n_edges, 1, (int32_t)(NE * nelem), s));
    if (nelem > 0) {
      hipLaunchKernelGGL(k_scatter_edge_inc<4>, dim3(grid_for(nelem * NE, 256)), dim3(256), 0,
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
  if (dim < 2 || dim > 4) {
    set_detail("dim must be 2, 3 or 4, got %d", dim);
    return EB_EINVAL;
  }
  if (n_nodes <= 0 || n_elems < 0 || !sizes_host || !coords || !node_inc_off ||
      (n_elems > 0 && (!elem || !node_inc))) {
    set_detail("null pointer or negative size");
    return EB_EINVAL;
  }
  const int64_t ne = (int64_t)dim * (dim + 1) / 2;
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
  if (dim == 4)
    return build4_impl(n_nodes, n_elems, elem, coords, node_inc_off, node_inc, ws, sizes_host,
                       stream);
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
      (has_el && (!t.elem_edge || !t.elem_edge_sign || !t.node_inc)) || !t.plan ||
      (has_f && (!t.bface || !t.bface_owner || !t.bface_edge)) ||
      (has_bn && (!t.bnode || !t.bnode_face))) {
    set_detail("a required topology array is null");
    return EB_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(t.plan) & 255u) != 0) {
    set_detail("the plan must be 256-byte aligned");
    return EB_EINVAL;
  }
  if ((t.edge_inc_off == nullptr) != (t.edge_inc == nullptr)) {
    set_detail("edge_inc_off and edge_inc must both be set or both be null");
    return EB_EINVAL;
  }
  EB_TRY(check_ws(sizes->dim, sizes->n_nodes, sizes->n_elems, ws, ws_bytes));
  if (sizes->dim == 4) return emit4_impl(sizes, elem, coords, topo, ws, stream);
  return sizes->dim == 2 ? emit_impl<2>(sizes, elem, coords, topo, ws, stream)
                         : emit_impl<3>(sizes, elem, coords, topo, ws, stream);
}

}  // extern "C"
