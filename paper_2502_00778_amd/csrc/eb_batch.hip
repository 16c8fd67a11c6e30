// Fused forward + adjoint in one persistent launch, per-grid offsets of a
// batch of grids, graph capture of the fused enqueue, and launch-shape tuning.
//
// A batch of grids is one grid whose node ids are concatenated: the meshes
// are disconnected, so the edge extraction, the sliced incidence layout and
// every gather kernel treat the whole batch at once, and each mesh's edges,
// boundary nodes and boundary faces come out as one contiguous range (edges
// are ordered by tail id, boundary lists by smallest vertex id).
//
// The fused kernel runs the deterministic forward (n, b, V) and the gather
// adjoint (dL/dx for a loss linear in n, b, V, whose weights do not depend on
// the forward outputs) as phases of one persistent launch:
//   phase 0: forward node tiles, interleaved with adjoint element-piece tiles
//   phase 1: forward boundary tiles, interleaved with adjoint node tiles
//   phase 2: adjoint boundary tiles
// With the adjoint's FP64 atomics instead (EB_FUSED_PERSISTENT_ATOMIC) the
// adjoint needs no second pass and nothing of the forward:
//   phase 0: forward node tiles, interleaved with adjoint element blocks
//            (per-node sums in LDS, then atomics) and boundary-face blocks
//   phase 1: forward boundary tiles
// Block b of a grid of G takes items b, b + G, b + 2G, ... of each phase
// (a fixed assignment: a shared work counter costs one same-address device
// atomic per item, which serializes at about 10 ns each).  At the end of a
// phase every block publishes (one counted release per block), and a block
// with work in a later phase waits, bounded, until all G blocks have
// published.  The grid never exceeds what is resident at once (occupancy x
// compute units), so every block it waits for is running and the waits end.
#include <hip/hip_runtime.h>

#include "eb_adjoint.h"
#include "eb_gather.h"

namespace eb {
namespace {

constexpr int EPT = 4;                       // elements per thread in a piece item
constexpr int64_t kDefaultSpinLimit = 1 << 22;  // ~ seconds of s_sleep polling
int64_t g_spin_limit = kDefaultSpinLimit;

struct FusedPlan {
  int64_t nF, nP, nB, nG, nH;  // item counts of each kind
  int64_t spin_limit;
  int64_t nQ;                  // (atomic adjoint) boundary-face blocks
};

__global__ void k_fused_reset(StatusBlock *st) {
  if (threadIdx.x < 4) st->fq[threadIdx.x] = 0u;
}

// Item k of a merged run of nX items of one kind and nXY - nX of another,
// spread evenly: the first kind iff the running count k*nX/nXY steps at k.
__device__ __forceinline__ bool first_kind(int64_t k, int64_t nX, int64_t nXY, int64_t &idx) {
  const int64_t c0 = k * nX / nXY, c1 = (k + 1) * nX / nXY;
  if (c1 > c0) {
    idx = c0;
    return true;
  }
  idx = k - c0;
  return false;
}

// End of a phase for the calling block: publish its writes of the phase
// (every wave's stores visible on all XCDs, then one counted release by
// thread 0) and, when the block has work in a later phase, wait until all
// blocks of the grid have published.  False (in every thread) when the wait
// ran out of polls: EB_ETIMEOUT is recorded and the block must exit.
__device__ __forceinline__ bool phase_end(StatusBlock *st, uint32_t *ctr, bool wait,
                                          int64_t spin_limit) {
  __shared__ int s_stop;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int stop = 0;
    if (wait) {
      int64_t spins = 0;
      while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
        __builtin_amdgcn_s_sleep(8);
        if (++spins > spin_limit) {
          raise_status(st, EB_ETIMEOUT, blockIdx.x);
          stop = 1;
          break;
        }
      }
    }
    s_stop = stop;
  }
  __syncthreads();
  if (s_stop) return false;
  // see every write of the completed phase, made on any XCD
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

template <int D, int TN, int CAP, int U, bool WIDE, bool STEP>
__global__ __launch_bounds__(TN) void k_fused(FwdArgs a, FusedPlan p) {
  __shared__ double acc[D][CAP];
  uint32_t *const q = a.st->fq;  // q[ph]: blocks that have finished phase ph
  const int t = threadIdx.x;
  const int64_t G = gridDim.x, b = blockIdx.x;
  const int64_t nA = p.nF + p.nP, nB = p.nB + p.nG, nC = p.nH;
  for (int64_t k = b; k < nA; k += G) {
    int64_t idx;
    if (first_kind(k, p.nF, nA, idx)) {
      fwd_node_tile<D, TN, CAP, U, WIDE, VAR_NODE, STEP>(a, idx, acc);
    } else {
      const int64_t e0 = idx * (int64_t)TN * EPT;
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        const int64_t e = e0 + (int64_t)m * TN + t;
        if (e < a.nelem) bwd_elem_piece<D>(a, e);
      }
    }
    __syncthreads();  // the LDS accumulator is free again
  }
  if (!phase_end(a.st, &q[0], b < nB || b < nC, p.spin_limit)) return;
  for (int64_t k = b; k < nB; k += G) {
    int64_t idx;
    if (first_kind(k, p.nB, nB, idx)) {
      const int64_t bj = idx * TN + t;
      if (bj < a.nbnode) fwd_boundary_node<D>(a, bj);
    } else {
      const int64_t j = idx * TN + t;
      if (j < a.nv) bwd_node_sum<D>(a, j);
    }
  }
  if (!phase_end(a.st, &q[1], b < nC, p.spin_limit)) return;
  for (int64_t k = b; k < nC; k += G) {
    const int64_t bj = k * TN + t;
    if (bj < a.nbnode) bwd_boundary_node<D>(a, bj);
  }
}

// Elements per thread of an adjoint element item of the atomic form, and its
// LDS node slots (two per element, as in the separate atomic kernel).
constexpr int EPA = 2;

template <int D, int TN, int CAP, int U, bool WIDE, bool STEP>
__global__ __launch_bounds__(TN) void k_fused_atomic(FwdArgs a, FusedPlan p) {
  constexpr int HA = 2 * TN * EPA;
  __shared__ union {
    double acc[D][CAP];    // forward node tile
    LdsAcc<HA, D> tg;      // adjoint element block
  } sm;
  uint32_t *const q = a.st->fq;  // q[0]: blocks that have finished phase 0
  const int t = threadIdx.x;
  const int64_t G = gridDim.x, b = blockIdx.x;
  const int64_t nR = p.nP + p.nQ, nA = p.nF + nR;
  for (int64_t k = b; k < nA; k += G) {
    int64_t idx;
    if (first_kind(k, p.nF, nA, idx)) {
      fwd_node_tile<D, TN, CAP, U, WIDE, VAR_NODE, STEP>(a, idx, sm.acc);
    } else if (first_kind(idx, p.nP, nR, idx)) {
      bwd_atomic_elem_block<D, TN, EPA>(a, idx, sm.tg);
    } else {
      const int64_t f = idx * TN + t;
      if (f < a.nbface) bwd_atomic_bface_one<D>(a, f);
    }
    __syncthreads();  // the LDS is free again
  }
  if (!phase_end(a.st, &q[0], b < p.nB, p.spin_limit)) return;
  for (int64_t k = b; k < p.nB; k += G) {
    const int64_t bj = k * TN + t;
    if (bj < a.nbnode) fwd_boundary_node<D>(a, bj);
  }
}

int g_num_cus = 0;

int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&g_num_cus, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess ||
        g_num_cus <= 0)
      g_num_cus = 256;
  }
  return g_num_cus;
}

template <class K>
int launch_fused_kernel(K kernel, int tn, const FwdArgs &a, const FusedPlan &p, int blocks_per_cu,
                        hipStream_t s) {
  int occ = 0;
  EB_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, tn, 0));
  if (occ <= 0) occ = 1;
  const int per_cu = blocks_per_cu > 0 ? std::min(blocks_per_cu, occ) : occ;
  const int64_t total = p.nF + p.nP + p.nB + p.nG + p.nH + p.nQ;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(total, (int64_t)per_cu * num_cus()));
  launch_principal(kernel, dim3((unsigned)grid), dim3(tn), 0, s, a, p);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

template <int D>
int fused_atomic_impl(const FwdArgs &a, const FusedCfg &cfg, hipStream_t s) {
  const int64_t tn = cfg.tile;
  FusedPlan p{};
  p.nF = (a.nv + tn - 1) / tn;
  p.nP = (a.w_x || a.c) ? (a.nelem + tn * EPA - 1) / (tn * EPA) : 0;
  p.nQ = (a.w_x || a.be_x) ? (a.nbface + tn - 1) / tn : 0;
  p.nB = (a.nbnode + tn - 1) / tn;
  p.spin_limit = g_spin_limit;
  if (p.nF + p.nP + p.nQ + p.nB >= (int64_t)1 << 31) {
    set_detail("too many work items for the fused kernel");
    return EB_EOVERFLOW;
  }
  // the gradient is summed with atomics: zeroed first (a fill kernel, no
  // memset node), and the phase counters cleared
  EB_TRY(fill_f64(a.g_x, D * a.nv, 0.0, s));
  hipLaunchKernelGGL(k_fused_reset, dim3(1), dim3(64), 0, s, a.st);
  EB_LAUNCH_CHECK();
#define EB_FUSED_CASE(TN_, CAP_, U_)                                                        \
  if (cfg.tile == TN_ && cfg.unroll == U_) {                                                \
    if (!a.sell_wide)                                                                       \
      return launch_fused_kernel(k_fused_atomic<D, TN_, CAP_, U_, false, true>, TN_, a, p,   \
                                 cfg.blocks_per_cu, s);                                     \
    if (a.node_step)                                                                        \
      return launch_fused_kernel(k_fused_atomic<D, TN_, CAP_, U_, true, true>, TN_, a, p,    \
                                 cfg.blocks_per_cu, s);                                     \
    return launch_fused_kernel(k_fused_atomic<D, TN_, CAP_, U_, true, false>, TN_, a, p,     \
                               cfg.blocks_per_cu, s);                                       \
  }
  EB_FUSED_CASE(64, 512, 1)
  EB_FUSED_CASE(64, 512, 2)
  EB_FUSED_CASE(64, 512, 4)
  EB_FUSED_CASE(128, 1024, 1)
  EB_FUSED_CASE(128, 1024, 2)
  EB_FUSED_CASE(128, 1024, 4)
  EB_FUSED_CASE(256, 2048, 1)
  EB_FUSED_CASE(256, 2048, 2)
  EB_FUSED_CASE(256, 2048, 4)
#undef EB_FUSED_CASE
  set_detail("unsupported fused tile %d / unroll %d", cfg.tile, cfg.unroll);
  return EB_EINVAL;
}

template <int D>
int fused_impl(const FwdArgs &a0, const FusedCfg &cfg, hipStream_t s) {
  if (cfg.separate) {  // the same work as the separate calls, one after the other
    const LaunchCfg g = default_cfg();
    FwdArgs a = a0;
    a.xcd_remap = g.xcd_remap;
    EB_TRY(forward_impl<D>(a, EB_REDUCE_GATHER, g, s));
    return backward_impl<D>(a, cfg.atomic ? EB_REDUCE_ATOMIC : EB_REDUCE_GATHER, g, s);
  }
  const FwdArgs &a = a0;
  const int64_t tn = cfg.tile;
  if (cfg.atomic) return fused_atomic_impl<D>(a, cfg, s);
  FusedPlan p{};
  p.nF = (a.nv + tn - 1) / tn;
  p.nP = (a.nelem + tn * EPT - 1) / (tn * EPT);
  p.nB = (a.nbnode + tn - 1) / tn;
  p.nG = p.nF;
  p.nH = (a.w_x || a.be_x) ? p.nB : 0;
  p.spin_limit = g_spin_limit;
  if (p.nF + p.nP + p.nB + p.nG + p.nH >= (int64_t)1 << 31) {
    set_detail("too many work items for the fused kernel");
    return EB_EOVERFLOW;
  }
  hipLaunchKernelGGL(k_fused_reset, dim3(1), dim3(64), 0, s, a.st);
  EB_LAUNCH_CHECK();
#define EB_FUSED_CASE(TN_, CAP_, U_)                                                        \
  if (cfg.tile == TN_ && cfg.unroll == U_) {                                                \
    if (!a.sell_wide)                                                                       \
      return launch_fused_kernel(k_fused<D, TN_, CAP_, U_, false, true>, TN_, a, p,          \
                                 cfg.blocks_per_cu, s);                                     \
    if (a.node_step)                                                                        \
      return launch_fused_kernel(k_fused<D, TN_, CAP_, U_, true, true>, TN_, a, p,           \
                                 cfg.blocks_per_cu, s);                                     \
    return launch_fused_kernel(k_fused<D, TN_, CAP_, U_, true, false>, TN_, a, p,            \
                               cfg.blocks_per_cu, s);                                       \
  }
  EB_FUSED_CASE(64, 512, 1)
  EB_FUSED_CASE(64, 512, 2)
  EB_FUSED_CASE(64, 512, 4)
  EB_FUSED_CASE(128, 1024, 1)
  EB_FUSED_CASE(128, 1024, 2)
  EB_FUSED_CASE(128, 1024, 4)
  EB_FUSED_CASE(256, 2048, 1)
  EB_FUSED_CASE(256, 2048, 2)
  EB_FUSED_CASE(256, 2048, 4)
#undef EB_FUSED_CASE
  set_detail("unsupported fused tile %d / unroll %d", cfg.tile, cfg.unroll);
  return EB_EINVAL;
}

// -------------------------------------------------------- batch offsets

// lower bound of v in the non-decreasing sequence key(0..n-1)
template <class Key>
__device__ __forceinline__ int64_t lower_bound_by(int64_t n, int64_t v, Key key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key(mid) < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// out = [edge_off | bnode_off | bface_off], n_mesh+1 each
__global__ void k_batch_offsets(int n_mesh, const int64_t *__restrict__ node_off,
                                const int32_t *__restrict__ node_edge_off,
                                const int32_t *__restrict__ bnode, int64_t nbn,
                                const int32_t *__restrict__ bface, int dim, int64_t nbf,
                                int64_t *out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m > n_mesh) return;
  const int64_t v = node_off[m];
  out[m] = node_edge_off[v];
  out[n_mesh + 1 + m] = lower_bound_by(nbn, v, [&](int64_t i) { return (int64_t)bnode[i]; });
  out[2 * (n_mesh + 1) + m] = lower_bound_by(nbf, v, [&](int64_t f) {
    int64_t k = bface[f * dim];
    for (int s = 1; s < dim; ++s) k = min(k, (int64_t)bface[f * dim + s]);
    return k;
  });
}

// every element of mesh m references only mesh m's nodes
template <int D>
__global__ void k_batch_check(int n_mesh, const int64_t *__restrict__ node_off,
                              const int64_t *__restrict__ elem_off,
                              const int32_t *__restrict__ elem, int64_t nelem, StatusBlock *st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nelem) return;
  // the mesh m with elem_off[m] <= e < elem_off[m+1]
  int64_t lo = 0, hi = n_mesh;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (elem_off[mid] <= e) lo = mid;
    else hi = mid;
  }
  int32_t v[D + 1];
  load_conn<D>(elem, e, v);
#pragma unroll
  for (int i = 0; i <= D; ++i)
    if (v[i] < node_off[lo] || v[i] >= node_off[lo + 1]) raise_status(st, EB_EINVAL, e);
}

int pack_fused(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
               const double *coords, const double *grad_n, const double *grad_b,
               const double *grad_vol, double *n_edge, double *b_node, double *vol,
               double *grad_coords, void *ws, size_t ws_bytes, FwdArgs &a) {
  EB_TRY(pack(sizes, topo, elem, coords, ws, ws_bytes, a));
  if (!n_edge || !grad_coords) {
    set_detail("n_edge and grad_coords are required");
    return EB_EINVAL;
  }
  const int D = sizes->dim;
  rows(n_edge, D, sizes->n_edges, a.n_x, a.n_y, a.n_z);
  rows(sizes->n_bnodes > 0 ? b_node : nullptr, D, sizes->n_bnodes, a.b_x, a.b_y, a.b_z);
  a.vol = vol;
  crows(grad_n, D, sizes->n_edges, a.w_x, a.w_y, a.w_z);
  crows(sizes->n_bnodes > 0 ? grad_b : nullptr, D, sizes->n_bnodes, a.be_x, a.be_y, a.be_z);
  a.c = grad_vol;
  rows(grad_coords, D, sizes->n_nodes, a.g_x, a.g_y, a.g_z);
  EB_TRY(check_fwd_gather(sizes, a));
  EB_TRY(check_bwd_gather(sizes, a, ws, ws_bytes));
  return EB_OK;
}

}  // namespace
}  // namespace eb

using namespace eb;

struct eb_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

int eb_batch_forward_backward(const eb_sizes *sizes, const eb_topology *topo,
                              const int32_t *elem, const double *coords, const double *grad_n,
                              const double *grad_b, const double *grad_vol, double *n_edge,
                              double *b_node, double *vol, double *grad_coords, void *ws,
                              size_t ws_bytes, hipStream_t stream) {
  PrincipalScope scope;
  clear_detail();
  EB_TRY(only_dims23(sizes));
  FwdArgs a;
  EB_TRY(pack_fused(sizes, topo, elem, coords, grad_n, grad_b, grad_vol, n_edge, b_node, vol,
                    grad_coords, ws, ws_bytes, a));
  const FusedCfg cfg = fused_cfg();
  return sizes->dim == 2 ? fused_impl<2>(a, cfg, stream) : fused_impl<3>(a, cfg, stream);
}

int eb_batch_offsets(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                     int n_mesh, const int64_t *node_off_host, const int64_t *elem_off_host,
                     int64_t *edge_off_host, int64_t *bnode_off_host, int64_t *bface_off_host,
                     void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_detail();
  EB_TRY(check_sizes(sizes));
  EB_TRY(only_dims23(sizes));
  if (!topo || !node_off_host || !elem_off_host || !edge_off_host || !bnode_off_host ||
      !bface_off_host || n_mesh <= 0 || (sizes->n_elems > 0 && !elem)) {
    set_detail("null pointer or n_mesh <= 0");
    return EB_EINVAL;
  }
  if (!topo->node_edge_off || (sizes->n_bnodes > 0 && !topo->bnode) ||
      (sizes->n_bfaces > 0 && !topo->bface)) {
    set_detail("node_edge_off, bnode and bface are required");
    return EB_EINVAL;
  }
  if (node_off_host[0] != 0 || elem_off_host[0] != 0 ||
      node_off_host[n_mesh] != sizes->n_nodes || elem_off_host[n_mesh] != sizes->n_elems) {
    set_detail("offsets must start at 0 and end at n_nodes / n_elems");
    return EB_EINVAL;
  }
  for (int m = 0; m < n_mesh; ++m)
    if (node_off_host[m + 1] <= node_off_host[m] || elem_off_host[m + 1] < elem_off_host[m]) {
      set_detail("mesh %d: node offsets must increase, element offsets must not decrease", m);
      return EB_EINVAL;
    }
  EB_TRY(check_ws(sizes->dim, sizes->n_nodes, sizes->n_elems, ws, ws_bytes));
  const size_t off = gpiece_offset(sizes->dim, sizes->n_nodes, sizes->n_elems);
  const size_t need_b = off + sizeof(int64_t) * 5 * (size_t)(n_mesh + 1);
  if (ws_bytes < need_b) {
    set_detail("eb_batch_offsets needs %zu workspace bytes, got %zu", need_b, ws_bytes);
    return EB_EWORKSPACE;
  }
  int64_t *d_node = ws_at<int64_t>(ws, off);
  int64_t *d_elem = d_node + (n_mesh + 1);
  int64_t *d_out = d_elem + (n_mesh + 1);
  StatusBlock *st = ws_at<StatusBlock>(ws, 0);
  const size_t nb = sizeof(int64_t) * (size_t)(n_mesh + 1);
  EB_HIP_CHECK(hipMemcpyAsync(d_node, node_off_host, nb, hipMemcpyHostToDevice, stream));
  EB_HIP_CHECK(hipMemcpyAsync(d_elem, elem_off_host, nb, hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_batch_offsets, dim3(grid_for(n_mesh + 1, 256)), dim3(256), 0, stream,
                     n_mesh, (const int64_t *)d_node, (const int32_t *)topo->node_edge_off,
                     (const int32_t *)topo->bnode, sizes->n_bnodes, (const int32_t *)topo->bface,
                     (int)sizes->dim, sizes->n_bfaces, d_out);
  EB_LAUNCH_CHECK();
  if (sizes->n_elems > 0) {
    if (sizes->dim == 2)
      hipLaunchKernelGGL(k_batch_check<2>, dim3(grid_for(sizes->n_elems, 256)), dim3(256), 0,
                         stream, n_mesh, (const int64_t *)d_node, (const int64_t *)d_elem, elem,
                         sizes->n_elems, st);
    else
      hipLaunchKernelGGL(k_batch_check<3>, dim3(grid_for(sizes->n_elems, 256)), dim3(256), 0,
                         stream, n_mesh, (const int64_t *)d_node, (const int64_t *)d_elem, elem,
                         sizes->n_elems, st);
    EB_LAUNCH_CHECK();
  }
  EB_HIP_CHECK(hipMemcpyAsync(edge_off_host, d_out, nb, hipMemcpyDeviceToHost, stream));
  EB_HIP_CHECK(
      hipMemcpyAsync(bnode_off_host, d_out + (n_mesh + 1), nb, hipMemcpyDeviceToHost, stream));
  EB_HIP_CHECK(hipMemcpyAsync(bface_off_host, d_out + 2 * (n_mesh + 1), nb,
                              hipMemcpyDeviceToHost, stream));
  StatusBlock h;
  EB_HIP_CHECK(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, stream));
  EB_HIP_CHECK(hipStreamSynchronize(stream));
  if (h.status != EB_OK) {  // reported here, so cleared like eb_check_errors does
    set_detail("%s (element %lld)", eb_status_string(h.status), (long long)h.detail);
    EB_HIP_CHECK(hipMemsetAsync(st, 0, 16, stream));
    EB_HIP_CHECK(hipStreamSynchronize(stream));
    return h.status;
  }
  return EB_OK;
}

int eb_batch_graph_create(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                          const double *coords, const double *grad_n, const double *grad_b,
                          const double *grad_vol, double *n_edge, double *b_node, double *vol,
                          double *grad_coords, void *ws, size_t ws_bytes, eb_graph *out) {
  clear_detail();
  if (!out) {
    set_detail("out is null");
    return EB_EINVAL;
  }
  *out = nullptr;
  EB_TRY(only_dims23(sizes));
  clear_armed_events();  // a captured launch records no timing events
  hipStream_t cs = nullptr;
  EB_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    set_detail("hipStreamBeginCapture: %s", hipGetErrorString(e));
    return EB_EHIP;
  }
  const int rc = eb_batch_forward_backward(sizes, topo, elem, coords, grad_n, grad_b, grad_vol,
                                           n_edge, b_node, vol, grad_coords, ws, ws_bytes, cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (rc != EB_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (rc != EB_OK) return rc;
    set_detail("hipStreamEndCapture: %s", hipGetErrorString(e));
    return EB_EHIP;
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    set_detail("hipGraphInstantiate: %s", hipGetErrorString(e));
    return EB_EHIP;
  }
  *out = new eb_graph_s{g, x};
  return EB_OK;
}

int eb_graph_launch(eb_graph graph, hipStream_t stream) {
  clear_detail();
  if (!graph) {
    set_detail("graph is null");
    return EB_EINVAL;
  }
  EB_HIP_CHECK(hipGraphLaunch(graph->exec, stream));
  return EB_OK;
}

int eb_graph_destroy(eb_graph graph) {
  clear_detail();
  if (!graph) return EB_OK;
  hipError_t e1 = hipGraphExecDestroy(graph->exec);
  hipError_t e2 = hipGraphDestroy(graph->graph);
  delete graph;
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_detail("graph destroy: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return EB_EHIP;
  }
  return EB_OK;
}

int eb_set_fused_shape(int tile, int unroll, int blocks_per_cu) {
  clear_detail();
  if ((tile != 64 && tile != 128 && tile != 256) || (unroll != 1 && unroll != 2 && unroll != 4) ||
      blocks_per_cu < 0 || blocks_per_cu > 32) {
    set_detail("tile must be 64/128/256, unroll 1/2/4, blocks_per_cu 0..32");
    return EB_EINVAL;
  }
  FusedCfg c = fused_cfg();
  c.tile = tile;
  c.unroll = unroll;
  c.blocks_per_cu = blocks_per_cu;
  set_fused_cfg(c);
  return EB_OK;
}

void eb_get_fused_shape(int *tile, int *unroll, int *blocks_per_cu) {
  const FusedCfg c = fused_cfg();
  if (tile) *tile = c.tile;
  if (unroll) *unroll = c.unroll;
  if (blocks_per_cu) *blocks_per_cu = c.blocks_per_cu;
}

int eb_set_fused_mode(int mode) {
  clear_detail();
  if (mode != EB_FUSED_PERSISTENT && mode != EB_FUSED_SEPARATE &&
      mode != EB_FUSED_PERSISTENT_ATOMIC && mode != EB_FUSED_SEPARATE_ATOMIC) {
    set_detail("mode must be EB_FUSED_PERSISTENT, EB_FUSED_SEPARATE, "
               "EB_FUSED_PERSISTENT_ATOMIC or EB_FUSED_SEPARATE_ATOMIC");
    return EB_EINVAL;
  }
  FusedCfg c = fused_cfg();
  c.separate = mode == EB_FUSED_SEPARATE || mode == EB_FUSED_SEPARATE_ATOMIC;
  c.atomic = mode == EB_FUSED_PERSISTENT_ATOMIC || mode == EB_FUSED_SEPARATE_ATOMIC;
  set_fused_cfg(c);
  return EB_OK;
}

int eb_get_fused_mode(void) {
  const FusedCfg c = fused_cfg();
  if (c.separate) return c.atomic ? EB_FUSED_SEPARATE_ATOMIC : EB_FUSED_SEPARATE;
  return c.atomic ? EB_FUSED_PERSISTENT_ATOMIC : EB_FUSED_PERSISTENT;
}

int eb_set_fused_wait_limit(int64_t spins) {
  clear_detail();
  if (spins < 0) {
    set_detail("spins must be >= 0 (0 restores the default)");
    return EB_EINVAL;
  }
  g_spin_limit = spins == 0 ? kDefaultSpinLimit : spins;
  return EB_OK;
}

int eb_autotune(const eb_sizes *sizes, const eb_topology *topo, const int32_t *elem,
                const double *coords, const double *grad_n, const double *grad_b,
                const double *grad_vol, double *n_edge, double *b_node, double *vol,
                double *grad_coords, void *ws, size_t ws_bytes, int reps, hipStream_t stream,
                eb_tuning *out) {
  clear_detail();
  EB_TRY(only_dims23(sizes));
  if (!out || reps < 1 || reps > 100) {
    set_detail("out is null or reps outside 1..100");
    return EB_EINVAL;
  }
  {  // validate everything once, before any timing
    FwdArgs a;
    EB_TRY(pack_fused(sizes, topo, elem, coords, grad_n, grad_b, grad_vol, n_edge, b_node, vol,
                      grad_coords, ws, ws_bytes, a));
  }
  clear_armed_events();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EB_HIP_CHECK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_detail("hipEventCreate failed");
    return EB_EHIP;
  }
  const LaunchCfg g0 = default_cfg();
  const FusedCfg f0 = fused_cfg();
  auto time_it = [&](auto &&run, float &ms) -> int {
    EB_TRY(run());  // warm-up
    EB_HIP_CHECK(hipEventRecord(e0, stream));
    for (int r = 0; r < reps; ++r) EB_TRY(run());
    EB_HIP_CHECK(hipEventRecord(e1, stream));
    EB_HIP_CHECK(hipEventSynchronize(e1));
    EB_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    return EB_OK;
  };
  const int tiles[3] = {64, 128, 256}, unrolls[3] = {1, 2, 4}, per_cu[5] = {1, 2, 4, 8, 0};
  eb_tuning best{};
  best.gather_ms = best.fused_ms = 1e30f;
  int rc = EB_OK, tried = 0;
  for (int ti = 0; ti < 3 && rc == EB_OK; ++ti)
    for (int ui = 0; ui < 3 && rc == EB_OK; ++ui)
      for (int x = 0; x < 2 && rc == EB_OK; ++x) {
        LaunchCfg c;
        c.tile = tiles[ti];
        c.unroll = unrolls[ui];
        c.xcd_remap = x;
        set_gather_cfg(c);
        float ms = 0.f;
        rc = time_it(
            [&]() {
              return eb_directed_areas(sizes, topo, elem, coords, EB_REDUCE_GATHER, n_edge,
                                       b_node, vol, ws, ws_bytes, stream);
            },
            ms);
        ++tried;
        if (rc == EB_OK && ms < best.gather_ms) {
          best.gather_ms = ms;
          best.gather_tile = c.tile;
          best.gather_unroll = c.unroll;
          best.gather_xcd_remap = c.xcd_remap;
        }
      }
  for (int ti = 0; ti < 3 && rc == EB_OK; ++ti)
    for (int ui = 0; ui < 3 && rc == EB_OK; ++ui)
      for (int pi = 0; pi < 5 && rc == EB_OK; ++pi) {
        FusedCfg c;
        c.separate = 0;
        c.atomic = f0.atomic;
        c.tile = tiles[ti];
        c.unroll = unrolls[ui];
        c.blocks_per_cu = per_cu[pi];
        set_fused_cfg(c);
        float ms = 0.f;
        rc = time_it(
            [&]() {
              return eb_batch_forward_backward(sizes, topo, elem, coords, grad_n, grad_b,
                                               grad_vol, n_edge, b_node, vol, grad_coords, ws,
                                               ws_bytes, stream);
            },
            ms);
        ++tried;
        if (rc == EB_OK && ms < best.fused_ms) {
          best.fused_ms = ms;
          best.fused_tile = c.tile;
          best.fused_unroll = c.unroll;
          best.fused_blocks_per_cu = c.blocks_per_cu;
        }
      }
  // the separate kernels in sequence (with the best gather shape, and the
  // adjoint of the reduction in force) as one more candidate for the whole
  // enqueue
  if (rc == EB_OK) {
    LaunchCfg g;
    g.tile = best.gather_tile;
    g.unroll = best.gather_unroll;
    g.xcd_remap = best.gather_xcd_remap;
    set_gather_cfg(g);
    FusedCfg c;
    c.separate = 1;
    c.atomic = f0.atomic;
    set_fused_cfg(c);
    float ms = 0.f;
    rc = time_it(
        [&]() {
          return eb_batch_forward_backward(sizes, topo, elem, coords, grad_n, grad_b, grad_vol,
                                           n_edge, b_node, vol, grad_coords, ws, ws_bytes,
                                           stream);
        },
        ms);
    ++tried;
    best.separate_ms = ms;
    best.fused_separate = ms < best.fused_ms ? 1 : 0;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != EB_OK) {
    set_gather_cfg(g0);
    set_fused_cfg(f0);
    return rc;
  }
  LaunchCfg g;
  g.tile = best.gather_tile;
  g.unroll = best.gather_unroll;
  g.xcd_remap = best.gather_xcd_remap;
  set_gather_cfg(g);
  FusedCfg f;
  f.tile = best.fused_tile;
  f.unroll = best.fused_unroll;
  f.blocks_per_cu = best.fused_blocks_per_cu;
  f.separate = best.fused_separate;
  f.atomic = f0.atomic;
  set_fused_cfg(f);
  best.n_tried = tried;
  *out = best;
  // leave the outputs as the chosen shape computes them (identical bits, but
  // for grad_coords of the atomic mode)
  return eb_batch_forward_backward(sizes, topo, elem, coords, grad_n, grad_b, grad_vol, n_edge,
                                   b_node, vol, grad_coords, ws, ws_bytes, stream);
}

}  // extern "C"
