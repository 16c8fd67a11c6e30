// Internal declarations shared by the HIP sources of libeb (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>

#include "eb.h"

namespace eb {

// ----------------------------------------------------------- status block
// The first 256 bytes of every workspace.  Kernels record the first error
// they meet (sticky); eb_build_edges and eb_check_errors read it back.
struct StatusBlock {
  int32_t status;
  int32_t pad;
  int64_t detail;       // e.g. the offending element or node id
  int32_t totals[8];    // device-side totals of the last scans
  uint32_t fq[4];       // fused kernel: blocks that have finished each phase
  int32_t _reserved[48];
};
static_assert(sizeof(StatusBlock) == 256, "status block is 256 bytes");

enum TotalSlot {
  T_EDGES = 0, T_BFACES = 1, T_BNODES = 2, T_SELL_ROWS = 3, T_MAXDELTA = 4, T_MAXOUT = 5,
  T_QUEUE = 6, T_MAXROW = 7
};

constexpr int SELL = 64;  // nodes per slice of the kernel plan (one wave)
__host__ __device__ inline int64_t n_slices(int64_t n_nodes) { return (n_nodes + SELL - 1) / SELL; }

__device__ inline void raise_status(StatusBlock *st, int code, int64_t detail) {
  if (atomicCAS(&st->status, 0, code) == 0) st->detail = detail;
}

// ------------------------------------------------------ workspace layout
// [status 256 B][eoff][foff][bidx][bfn][bfn_scan][ein_scan][slen][queue][scan scratch]
// [incidence rows (build) | gradient pieces (gather adjoint)]
// Each per-node array holds n_nodes+1 int32 and starts on a 256-byte line.
// neighbours per node the build's fast node passes keep (the count pass
// stores each node's sorted set for the emit pass)
constexpr int NSET = 24;

struct WsLayout {
  size_t eoff, foff, bidx, bfn, bfn_scan, ein_scan, slen, queue, scan_tmp, nset, rows4, inc_pos,
      row_rank, total;
  int64_t scan_tmp_count;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int MAX_SCAN_JOBS = 5;  // arrays one scan pass serves at most
constexpr int64_t SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;  // items per scan block

inline WsLayout ws_layout(int dim, int64_t n_nodes, int64_t n_elems) {
  WsLayout L{};
  const size_t per = align256(sizeof(int32_t) * (size_t)(n_nodes + 1));
  size_t off = sizeof(StatusBlock);
  L.eoff = off; off += per;
  L.foff = off; off += per;
  L.bidx = off; off += per;
  L.bfn = off; off += per;
  L.bfn_scan = off; off += per;
  L.ein_scan = off; off += per;
  L.slen = off; off += align256(sizeof(int32_t) * (size_t)(n_slices(n_nodes) + 1));
  L.queue = off; off += per;
  // the longest array any call scans: ne*n_elems incidences
  const int64_t ne = (int64_t)dim * (dim + 1) / 2;
  int64_t longest = std::max<int64_t>(n_nodes + 1, ne * n_elems + 1);
  // (or the node arrays' block sums, MAX_SCAN_JOBS arrays at once)
  L.scan_tmp_count = std::max<int64_t>((longest + SCAN_TILE - 1) / SCAN_TILE,
                                       MAX_SCAN_JOBS * ((n_nodes + SCAN_TILE) / SCAN_TILE)) +
                     64;
  L.scan_tmp = off; off += align256(sizeof(int32_t) * (size_t)L.scan_tmp_count);
  // each node's neighbour set, slice-major (slot s of node j at
  // slice(j) * NSET * 64 + 64 s + lane(j))
  L.nset = off; off += align256(sizeof(int32_t) * (size_t)NSET * 64 * (size_t)n_slices(n_nodes));
  // build only (the adjoint reuses the space): per incidence a 16-byte row
  // entry, its position in the unsorted rows, and its rank within its row
  const size_t ninc = (size_t)(dim + 1) * (size_t)n_elems;
  L.rows4 = off; off += align256(16 * ninc);
  L.inc_pos = off; off += align256(4 * ninc);
  L.row_rank = off; off += align256(2 * ninc);
  L.total = off;
  return L;
}

// The gather adjoint's per-incidence gradient pieces follow the layout above:
// D rows of n_slots doubles (one per slot of the kernel plan).
// The build's incidence rows are dead once the emit pass is done, so the
// pieces take their place.
inline size_t gpiece_offset(int dim, int64_t n_nodes, int64_t n_elems) {
  return ws_layout(dim, n_nodes, n_elems).rows4;
}
inline size_t backward_ws_total(int dim, int64_t n_nodes, int64_t n_elems, int64_t n_slots) {
  const WsLayout L = ws_layout(dim, n_nodes, n_elems);
  return std::max(L.total,
                  L.rows4 + align256(sizeof(double) * (size_t)dim * (size_t)n_slots));
}

template <class T> inline T *ws_at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// ------------------------------------------------------------ host errors
void set_detail(const char *fmt, ...);
void clear_detail();

#define EB_HIP_CHECK(expr)                                                    \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess) {                                                   \
      ::eb::set_detail("%s: %s (%s:%d)", #expr, hipGetErrorString(_e),        \
                       __FILE__, __LINE__);                                   \
      return EB_EHIP;                                                         \
    }                                                                         \
  } while (0)

#define EB_LAUNCH_CHECK()                                                     \
  do {                                                                        \
    hipError_t _e = hipGetLastError();                                        \
    if (_e != hipSuccess) {                                                   \
      ::eb::set_detail("kernel launch: %s (%s:%d)", hipGetErrorString(_e),    \
                       __FILE__, __LINE__);                                   \
      return EB_EHIP;                                                         \
    }                                                                         \
  } while (0)

#define EB_TRY(expr)                                                          \
  do {                                                                        \
    int _rc = (expr);                                                         \
    if (_rc != EB_OK) return _rc;                                             \
  } while (0)

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

int check_ws(int dim, int64_t n_nodes, int64_t n_elems, const void *ws, size_t ws_bytes);
// A grid without elements has no edges, boundary faces or boundary nodes (the
// build finds none): every per-node sum a call returns is empty (zero), and
// the per-edge and per-boundary-node outputs have no entries (their pointers
// may be null).
inline bool no_elements(const eb_sizes *s) {
  return s->n_elems == 0 && s->n_edges == 0 && s->n_bfaces == 0 && s->n_bnodes == 0;
}
int check_sizes(const eb_sizes *s);
// EB_EINVAL (with detail) for dim 4, which only the build, the forward and
// the volume calls support
int only_dims23(const eb_sizes *s);

// ---------------------------------------------------------------- scans
// Device scans of int32 arrays (n < 2^31, partial sums must fit int32).
// `out` may alias `in`.  The total is written to *total_dev (device) when
// total_dev is not null.
int scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev,
                   int32_t *tmp, hipStream_t s);
int scan_inclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev,
                   int32_t *tmp, hipStream_t s);
// Up to MAX_SCAN_JOBS scans of arrays of the same length n in one pass (three
// launches); tmp holds count * ceil(n / SCAN_TILE) block sums.
struct ScanJobs {
  const int32_t *in[MAX_SCAN_JOBS];
  int32_t *out[MAX_SCAN_JOBS];
  int32_t *total[MAX_SCAN_JOBS];  // device, or null
  int32_t inclusive[MAX_SCAN_JOBS];
};
int scan_many(const ScanJobs &J, int count, int64_t n, int32_t *tmp, hipStream_t s);
// Sort every CSR row of `val` ascending.
int rowsort(const int32_t *off, int32_t *val, int64_t nrows, hipStream_t s);
// Fill an int32 array with a value (graph-capturable; no memset nodes).
int fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
int fill_f64(double *p, int64_t n, double v, hipStream_t s);

// ------------------------------------------------------ launch helpers
inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

// Coordinates as three SoA rows (z row unused in 2D).
struct Coords {
  const double *x, *y, *z;
};
inline Coords coords_rows(const double *c, int dim, int64_t nv) {
  return Coords{c, c + nv, dim == 3 ? c + 2 * nv : c};
}

}  // namespace eb
