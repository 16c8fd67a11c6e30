// Kernel argument packs and launchers shared by the C-ABI entry points.
#pragma once

#include "eb_internal.h"

namespace eb {

// Everything the metric and adjoint kernels may read or write.  Pointers not
// needed by a given kernel may be null.
struct FwdArgs {
  int64_t nv, nelem, nedge, nbface, nbnode;
  const int32_t *elem;
  Coords X;
  const int32_t *elem_edge;
  const int32_t *node_inc_off, *node_inc;
  const int32_t *node_sell_off;
  const uint64_t *node_sell;
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
  StatusBlock *st;
  int xcd_remap;
};

// Launch shape of the node-centred (gather) kernels: nodes per block
// (64/128/256), loads in flight per thread (1/2/4), XCD-aware tile order.
struct LaunchCfg {
  int tile = 128;
  int unroll = 2;
  int xcd_remap = 1;
};

LaunchCfg default_cfg();

template <int D> int forward_impl(const FwdArgs &a, int reduce, const LaunchCfg &cfg, hipStream_t s);
template <int D>
int volumes_impl(const FwdArgs &a, int mode, int reduce, const double *n_edge, hipStream_t s);
template <int D> int backward_impl(const FwdArgs &a, int reduce, const LaunchCfg &cfg, hipStream_t s);

}  // namespace eb
