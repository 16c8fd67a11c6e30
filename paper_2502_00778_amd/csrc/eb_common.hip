// Status handling, workspace checks and the device primitives the topology
// build is made of: exclusive/inclusive scans, per-row sorts, fills.
#include <cstdarg>
#include <cstring>

#include "eb_plan.h"

namespace eb {

namespace {
thread_local char g_detail[512] = "";
}

void set_detail(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_detail, sizeof(g_detail), fmt, ap);
  va_end(ap);
}
void clear_detail() { g_detail[0] = 0; }

int check_ws(int dim, int64_t n_nodes, int64_t n_elems, const void *ws, size_t ws_bytes) {
  if (!ws) {
    set_detail("workspace pointer is null");
    return EB_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) {
    set_detail("workspace must be 256-byte aligned");
    return EB_EINVAL;
  }
  size_t need = ws_layout(dim, n_nodes, n_elems).total;
  if (ws_bytes < need) {
    set_detail("workspace has %zu bytes, needs %zu", ws_bytes, need);
    return EB_EWORKSPACE;
  }
  return EB_OK;
}

int only_dims23(const eb_sizes *s) {
  if (s && s->dim == 4) {
    set_detail("this call supports dim 2 and 3 (dim 4: eb_build_edges, eb_directed_areas and "
               "eb_dual_volumes)");
    return EB_EINVAL;
  }
  return EB_OK;
}

int check_sizes(const eb_sizes *s) {
  if (!s) {
    set_detail("sizes pointer is null");
    return EB_EINVAL;
  }
  if (s->dim < 2 || s->dim > 4) {
    set_detail("dim must be 2, 3 or 4, got %d", s->dim);
    return EB_EINVAL;
  }
  if (s->n_nodes <= 0 || s->n_elems < 0 || s->n_edges < 0 || s->n_bfaces < 0 ||
      s->n_bnodes < 0) {
    set_detail("negative or empty sizes");
    return EB_EINVAL;
  }
  const int64_t ne = (int64_t)s->dim * (s->dim + 1) / 2;
  if (ne * s->n_elems >= (int64_t(1) << 31) || s->n_nodes >= (int64_t(1) << 31) - 1) {
    set_detail("grid too large for int32 indexing");
    return EB_EOVERFLOW;
  }
  if (!plan_params_valid(s)) {
    set_detail("eb_sizes does not come from eb_build_edges (plan fields)");
    return EB_EINVAL;
  }
  return EB_OK;
}

// ------------------------------------------------------------------ scans

__device__ inline int32_t wave_incl_scan(int32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ inline int32_t wave_sum(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// exclusive scan of one value per thread across the block; returns the
// block total through *total
__device__ inline int32_t block_excl_scan(int32_t v, int32_t *total) {
  __shared__ int32_t wsum[SCAN_BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
    int32_t s = wsum[w];
    if (w < wid) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// Every scan kernel serves up to MAX_SCAN_JOBS arrays of one length at once:
// blockIdx.y (blockIdx.x in the partials pass) picks the array, and array
// j's block sums live at tmp + j * nb.
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(ScanJobs J, int64_t n,
                                                            int32_t *tmp) {
  __shared__ int32_t wsum[SCAN_BLOCK / 64];
  const int32_t *in = J.in[blockIdx.y];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) t += wsum[w];
    tmp[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// exclusive scan of one array's nb block sums, in place, by one block
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_partials(ScanJobs J, int32_t *tmp,
                                                              int64_t nb) {
  int32_t *t = tmp + (int64_t)blockIdx.x * nb;
  int32_t carry = 0;
  for (int64_t b = 0; b < nb; b += SCAN_BLOCK) {
    int64_t i = b + threadIdx.x;
    int32_t v = i < nb ? t[i] : 0;
    int32_t tot;
    int32_t ex = block_excl_scan(v, &tot);
    if (i < nb) t[i] = carry + ex;
    carry += tot;
  }
  int32_t *total = J.total[blockIdx.x];
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(ScanJobs J, int64_t n,
                                                           const int32_t *tmp) {
  const int32_t *in = J.in[blockIdx.y];
  int32_t *out = J.out[blockIdx.y];
  const int32_t incl = J.inclusive[blockIdx.y] ? -1 : 0;  // mask: add the item itself
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  // a thread's items are contiguous: whole, 16-byte aligned runs move as
  // int4 (4 loads or stores per thread instead of 16)
  static_assert(SCAN_ITEMS % 4 == 0, "items per thread move in int4 pieces");
  const bool vec = base + SCAN_ITEMS <= n &&
                   ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  int32_t v[SCAN_ITEMS];
  if (vec) {
    const int4 *src = reinterpret_cast<const int4 *>(in + base);
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS / 4; ++q) {
      const int4 x = src[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) v[i] = base + i < n ? in[base + i] : 0;
  }
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) s += v[i];
  int32_t tot;
  int32_t run = block_excl_scan(s, &tot) + tmp[(int64_t)blockIdx.y * gridDim.x + blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const int32_t x = v[i];
    v[i] = run + (x & incl);
    run += x;
  }
  if (vec) {
    int4 *dst = reinterpret_cast<int4 *>(out + base);
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS / 4; ++q)
      dst[q] = int4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
      if (base + i < n) out[base + i] = v[i];
  }
}

int scan_many(const ScanJobs &J, int count, int64_t n, int32_t *tmp, hipStream_t s) {
  if (count < 1 || count > MAX_SCAN_JOBS) return EB_EINVAL;
  if (n <= 0) {
    for (int j = 0; j < count; ++j)
      if (J.total[j]) EB_TRY(fill_i32(J.total[j], 1, 0, s));
    return EB_OK;
  }
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb, (unsigned)count), dim3(SCAN_BLOCK), 0, s,
                     J, n, tmp);
  EB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)count), dim3(SCAN_BLOCK), 0, s, J, tmp, nb);
  EB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb, (unsigned)count), dim3(SCAN_BLOCK), 0, s,
                     J, n, (const int32_t *)tmp);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

static int scan_one(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev,
                    int32_t *tmp, bool inclusive, hipStream_t s) {
  ScanJobs J{};
  J.in[0] = in;
  J.out[0] = out;
  J.total[0] = total_dev;
  J.inclusive[0] = inclusive;
  return scan_many(J, 1, n, tmp, s);
}

int scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev,
                   int32_t *tmp, hipStream_t s) {
  return scan_one(in, out, n, total_dev, tmp, false, s);
}
int scan_inclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev,
                   int32_t *tmp, hipStream_t s) {
  return scan_one(in, out, n, total_dev, tmp, true, s);
}

// -------------------------------------------------------------- row sort
// One wavefront per 64 consecutive rows.  Rows up to RS_CAP long are sorted
// by their own lane, by insertion in LDS (a column per lane, conflict-free);
// longer rows then by the whole wave in turn, with a bitonic network over the
// row padded to a power of two in LDS, and rows beyond RS_LONG by insertion
// in global memory (lane 0).
constexpr int RS_CAP = 32;
constexpr int RS_LONG = RS_CAP * 64;

__global__ __launch_bounds__(64) void k_rowsort(const int32_t *off, int32_t *val,
                                                int64_t nrows) {
  __shared__ int32_t buf[RS_LONG];  // [RS_CAP][64] for the short rows
  const int t = threadIdx.x;
  const int64_t row = (int64_t)blockIdx.x * 64 + t;
  int32_t b = 0, len = 0;
  if (row < nrows) {
    b = off[row];
    len = off[row + 1] - b;
  }
  if (len > 1 && len <= RS_CAP) {
    for (int i = 0; i < len; ++i) buf[i * 64 + t] = val[b + i];
    for (int i = 1; i < len; ++i) {
      const int32_t x = buf[i * 64 + t];
      int k = i - 1;
      while (k >= 0 && buf[k * 64 + t] > x) {
        buf[(k + 1) * 64 + t] = buf[k * 64 + t];
        --k;
      }
      buf[(k + 1) * 64 + t] = x;
    }
    for (int i = 0; i < len; ++i) val[b + i] = buf[i * 64 + t];
  }
  uint64_t todo = __builtin_amdgcn_ballot_w64(len > RS_CAP);
  while (todo) {
    const int r = __builtin_ctzll(todo);
    todo &= todo - 1;
    const int32_t rb = __shfl(b, r, 64), rl = __shfl(len, r, 64);
    __syncthreads();  // (the stage is free)
    if (rl > RS_LONG) {
      if (t == 0)
        for (int32_t i = rb + 1; i < rb + rl; ++i) {
          const int32_t x = val[i];
          int32_t k = i - 1;
          while (k >= rb && val[k] > x) {
            val[k + 1] = val[k];
            --k;
          }
          val[k + 1] = x;
        }
      continue;
    }
    int P = 64;
    while (P < rl) P <<= 1;
    for (int i = t; i < P; i += 64) buf[i] = i < rl ? val[rb + i] : INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = t; i < P / 2; i += 64) {
          const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1)), hi = lo + j;
          const int32_t x = buf[lo], y = buf[hi];
          if ((x > y) == ((lo & k) == 0)) {
            buf[lo] = y;
            buf[hi] = x;
          }
        }
        __syncthreads();
      }
    for (int i = t; i < rl; i += 64) val[rb + i] = buf[i];
  }
}

int rowsort(const int32_t *off, int32_t *val, int64_t nrows, hipStream_t s) {
  if (nrows <= 0) return EB_OK;
  hipLaunchKernelGGL(k_rowsort, dim3(grid_for(nrows, 64)), dim3(64), 0, s, off, val, nrows);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

// ------------------------------------------------------------------ fills

template <class T> __global__ void k_fill(T *p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <class T> static int fill_impl(T *p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return EB_OK;
  int64_t g = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)g), dim3(256), 0, s, p, n, v);
  EB_LAUNCH_CHECK();
  return EB_OK;
}
int fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) { return fill_impl(p, n, v, s); }
int fill_f64(double *p, int64_t n, double v, hipStream_t s) { return fill_impl(p, n, v, s); }

}  // namespace eb

// =================================================================== C ABI

extern "C" {

size_t eb_workspace_bytes(int dim, int64_t n_nodes, int64_t n_elems) {
  if (dim < 2 || dim > 4 || n_nodes <= 0 || n_elems < 0) return 0;
  return eb::ws_layout(dim, n_nodes, n_elems).total;
}

size_t eb_backward_workspace_bytes(const eb_sizes *sizes) {
  if (eb::check_sizes(sizes) != EB_OK) return 0;
  return eb::backward_ws_total(sizes->dim, sizes->n_nodes, sizes->n_elems,
                               eb::plan_slots(sizes));
}

int eb_plan_describe(const eb_sizes *sizes, const void *plan, eb_plan_view *view) {
  eb::clear_detail();
  EB_TRY(eb::check_sizes(sizes));
  if (!plan || !view) {
    eb::set_detail("null pointer");
    return EB_EINVAL;
  }
  const eb::PlanPtrs p = eb::plan_ptrs(sizes, const_cast<void *>(plan));
  view->slice_off = p.slice_off;
  view->entry = p.entry;
  view->step = p.step;
  view->inc_slot = p.inc_slot;
  view->n_slots = eb::plan_slots(sizes);
  view->words = eb::plan_wide(sizes) ? 2 : 1;
  return EB_OK;
}

int eb_check_errors(void *ws, hipStream_t stream) {
  eb::clear_detail();
  if (!ws) {
    eb::set_detail("workspace pointer is null");
    return EB_EINVAL;
  }
  eb::StatusBlock hst;
  EB_HIP_CHECK(hipMemcpyAsync(&hst, ws, sizeof(hst), hipMemcpyDeviceToHost, stream));
  EB_HIP_CHECK(hipStreamSynchronize(stream));
  EB_TRY(eb::fill_i32(static_cast<int32_t *>(ws), 4, 0, stream));
  if (hst.status != EB_OK)
    eb::set_detail("device reported %s (detail %lld)", eb_status_string(hst.status),
                   (long long)hst.detail);
  return hst.status;
}

const char *eb_status_string(int status) {
  switch (status) {
    case EB_OK: return "ok";
    case EB_EINVAL: return "invalid argument";
    case EB_ERANGE: return "node id out of range";
    case EB_EDEGENERATE: return "element of zero measure";
    case EB_ENONMANIFOLD: return "face shared by more than two elements";
    case EB_EWORKSPACE: return "workspace too small";
    case EB_EOVERFLOW: return "sizes overflow int32 indexing";
    case EB_EHIP: return "HIP runtime error";
    case EB_ECAPACITY: return "node beyond the kernel plan's per-node limits";
    case EB_ETIMEOUT: return "a persistent kernel's bounded wait ran out";
    default: return "unknown status";
  }
}

const char *eb_last_error_detail(void) { return eb::g_detail; }

const char *eb_version(void) { return "eb 0.1 (gfx950)"; }

}  // extern "C"
