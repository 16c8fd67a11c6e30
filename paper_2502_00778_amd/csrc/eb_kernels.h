// Kernel argument packs and launchers shared by the C-ABI entry points.
#pragma once

#include <hip/hip_ext.h>

#include "eb_plan.h"

namespace eb {

// Everything the metric and adjoint kernels may read or write.  Pointers not
// needed by a given kernel may be null.
struct FwdArgs {
  int64_t nv, nelem, nedge, nbface, nbnode;
  const int32_t *elem;
  Coords X;
  const int32_t *elem_edge;
  const int32_t *node_inc_off, *node_inc;
  // the kernel plan (layout in eb_plan.h)
  const int32_t *node_sell_off;  // slice offsets
  const uint64_t *node_sell;     // per-slot entries
  const int32_t *inc_sell;       // incidence -> slot
  const uint32_t *node_step;     // per slot: the step from the previous entry (narrow)
  int sell_wide;
  const int32_t *node_edge_off, *edge_tail, *edge_head;
  const int32_t *node_in_off, *node_in_edge;
  const int32_t *bface, *bface_edge, *node_bnode, *bnode, *bnode_face_off, *bnode_face;
  double *n_x, *n_y, *n_z;  // [D][Ne] rows
  double *b_x, *b_y, *b_z;  // [D][Nbn] rows
  double *vol;              // [Nv]
  // adjoint inputs / output
  const double *w_x, *w_y, *w_z;     // dL/dn rows
  const double *be_x, *be_y, *be_z;  // dL/db rows
  const double *c;                   // dL/dV
  double *g_x, *g_y, *g_z;           // dL/dx rows
  double *gpiece;  // workspace: per-incidence gradient pieces, D rows of gstride
  int64_t gstride;  // (the plan's slots: node_sell_off[n_slices])
  double *vterm;   // workspace: per-edge terms of the edge loop
  StatusBlock *st;
  int xcd_remap;
};

// The tile (of nodes or elements) a block handles.  Blocks are dealt round-robin to the 8
// XCDs (block b runs on XCD b % 8); with remapping, XCD x takes one
// contiguous run of tiles in order, so neighbouring tiles (which share
// elements and coordinates) meet in the same L2.  A bijection for any count.
__device__ __forceinline__ int64_t tile_of_block(int64_t nblocks, int xcd_remap) {
  const int64_t b = blockIdx.x;
  if (!xcd_remap || nblocks < 16) return b;
  const int64_t per = nblocks >> 3, rem = nblocks & 7;
  const int64_t x = b & 7, k = b >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

// Launch shape of the node-centred (gather) kernels: nodes per block
// (64/128/256), loads in flight per thread (1/2/4), XCD-aware tile order.
struct LaunchCfg {
  int tile = 64;
  int unroll = 2;
  int xcd_remap = 1;
};

// Launch shape of the fused persistent forward + adjoint kernel: threads per
// block (= nodes per node tile), loads in flight per thread, and resident
// blocks per compute unit (0: as many as occupancy allows).
struct FusedCfg {
  int tile = 128;
  int unroll = 2;
  int blocks_per_cu = 0;
  int separate = 0;  // 1: the gather forward and adjoint kernels in sequence instead
  int atomic = 0;    // 1: one persistent kernel with the adjoint's FP64 atomics
};
FusedCfg fused_cfg();
void set_fused_cfg(const FusedCfg &c);
void set_gather_cfg(const LaunchCfg &c);

LaunchCfg default_cfg();

// Events armed by eb_time_next_launch for the principal kernel of the current
// call (consumed by its first launch_principal; cleared when the call ends).
struct TimedLaunch {
  hipEvent_t start = nullptr, stop = nullptr;
};
TimedLaunch take_principal_events();
void principal_begin();      // the armed events become the current call's
void principal_end();        // the current call's unused events are dropped
void clear_armed_events();   // disarm (graph capture, tuning)
struct PrincipalScope {
  PrincipalScope() { principal_begin(); }
  ~PrincipalScope() { principal_end(); }
  PrincipalScope(const PrincipalScope &) = delete;
  PrincipalScope &operator=(const PrincipalScope &) = delete;
};

TimedLaunch take_span_events();  // eb_time_next_call's events for this launch

// A launch that takes part in the call's span timing (eb_time_next_call).
template <class K, class... A>
void launch_span(K kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, A... args) {
  const TimedLaunch t = take_span_events();
  if (t.stop)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t.start, t.stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

// The call's principal kernel (eb_time_next_launch); a call timed by span
// (eb_time_next_call) takes part in that instead.
template <class K, class... A>
void launch_principal(K kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, A... args) {
  const TimedLaunch sp = take_span_events();
  if (sp.stop) {
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, sp.start, sp.stop, 0u, args...);
    return;
  }
  const TimedLaunch t = take_principal_events();
  if (t.start)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t.start, t.stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

// Host-side argument packing and validation shared by the entry points.
int pack(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem, const double *coords,
         void *ws, size_t ws_bytes, FwdArgs &a);
// the array pointers alone (no workspace, a.st left null); sizes checked by
// the caller; elem may be null unless need_elem
int pack_arrays(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem,
                const double *coords, bool need_elem, FwdArgs &a);
int need(bool ok, const char *what);
void rows(double *p, int dim, int64_t n, double *&x, double *&y, double *&z);
void crows(const double *p, int dim, int64_t n, const double *&x, const double *&y,
           const double *&z);
int check_fwd_gather(const eb_sizes *sizes, const FwdArgs &a);
// also points a.gpiece into the workspace
int check_bwd_gather(const eb_sizes *sizes, FwdArgs &a, void *ws, size_t ws_bytes);
int check_elem_edge_aligned(const eb_sizes *sizes, const FwdArgs &a);

template <int D> int launch_fwd_nodes(const FwdArgs &a, const LaunchCfg &cfg, hipStream_t s);
template <int D> int forward_impl(const FwdArgs &a, int reduce, const LaunchCfg &cfg, hipStream_t s);
template <int D>
int volumes_impl(const FwdArgs &a, int mode, int reduce, const double *n_edge, hipStream_t s);
template <int D>
int forward_variant_impl(const FwdArgs &a, int variant, const LaunchCfg &cfg, hipStream_t s);
template <int D>
int residual_impl(const FwdArgs &a, const double *n_edge, const double *F, int linear,
                  double *res, hipStream_t s);
template <int D> int backward_impl(const FwdArgs &a, int reduce, const LaunchCfg &cfg, hipStream_t s);

// dim 4 (pentatopes): eb_directed_areas and eb_dual_volumes in full
int forward4(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem,
             const double *coords, int reduce, double *n_edge, double *b_node, double *vol,
             void *ws, size_t ws_bytes, hipStream_t s);
int volumes4(const eb_sizes *sz, const eb_topology *tp, const int32_t *elem,
             const double *coords, int mode, const double *n_edge, int reduce, double *vol,
             void *ws, size_t ws_bytes, hipStream_t s);

// ------------------------------------------------ ordered sums of terms
// s + term[e] (or s - term[e]) over edges e = b .. e1-1, or over e = idx[b ..
// e1-1], in that order; eight loads are issued before any is added, so a
// node's terms arrive together instead of one round trip each
template <bool SUB>
__device__ __forceinline__ double sum_terms(double s, const double *__restrict__ term, int32_t b,
                                            int32_t e1) {
  for (int32_t i = b; i < e1; i += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = term[min(i + u, e1 - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i + u < e1) s = SUB ? s - v[u] : s + v[u];
  }
  return s;
}
template <bool SUB>
__device__ __forceinline__ double sum_terms_at(double s, const double *__restrict__ term,
                                               const int32_t *__restrict__ idx, int32_t b,
                                               int32_t e1) {
  for (int32_t i = b; i < e1; i += 8) {
    int32_t k[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) k[u] = idx[min(i + u, e1 - 1)];
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = term[k[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i + u < e1) s = SUB ? s - v[u] : s + v[u];
  }
  return s;
}

}  // namespace eb
