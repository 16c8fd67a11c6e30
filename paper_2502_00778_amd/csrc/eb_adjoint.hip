// Adjoint kernels and launcher (the derivation is in eb_adjoint.h).
#include "eb_adjoint.h"

namespace eb {

// ------------------------------------------------------------- atomic path

// One thread per element: dL_E/dx_i for each vertex, summed per node in the
// block's LDS table and added to the zeroed gradient with one FP64 atomic
// per distinct node and component (eb_adjoint.h).
template <int D>
__global__ __launch_bounds__(ATOMIC_TB) void k_bwd_atomic_elem(FwdArgs a) {
  __shared__ LdsAcc<ATOMIC_HV, D> tg;
  bwd_atomic_elem_block<D, ATOMIC_TB, ATOMIC_EPT>(a, blockIdx.x, tg);
}

// One thread per boundary face; a block's 256 faces (in bface order,
// consecutive ones sharing most vertices) sum their terms per node in an LDS
// table first, then add each sum with one FP64 atomic per component.
constexpr int BF_TB = 256, BF_H = 512;

template <int D>
__global__ __launch_bounds__(BF_TB) void k_bwd_atomic_bface(FwdArgs a) {
  __shared__ LdsAcc<BF_H, D> T;
  const int t = threadIdx.x;
  double *const gout[3] = {a.g_x, a.g_y, a.g_z};
  lds_acc_init<BF_TB>(T, t);
  __syncthreads();
  const int64_t f = (int64_t)blockIdx.x * BF_TB + t;
  if (f < a.nbface) {
    int32_t fv[D];
    V3 G[D];
    bwd_bface_terms<D>(a, f, fv, G);
#pragma unroll
    for (int p = 0; p < D; ++p) {
      double c[D];
      c[0] = G[p].x;
      c[1] = G[p].y;
      if constexpr (D == 3) c[D - 1] = G[p].z;
      lds_acc_add(T, gout, fv[p], c);
    }
  }
  __syncthreads();
  lds_acc_flush<BF_TB>(T, gout, t);
}

// ------------------------------------------------------------- gather path

template <int D>
__global__ __launch_bounds__(256) void k_bwd_elem_pieces(FwdArgs a) {
  // XCD-aware order: neighbouring element ranges share vertices and edges,
  // so each XCD takes one contiguous run of them (one L2)
  const int64_t e = tile_of_block(gridDim.x, 1) * blockDim.x + threadIdx.x;
  if (e < a.nelem) bwd_elem_piece<D>(a, e);
}

template <int D>
__global__ __launch_bounds__(256) void k_bwd_node_gather(FwdArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < a.nv) bwd_node_sum<D>(a, j);
}

template <int D>
__global__ __launch_bounds__(256) void k_bwd_boundary_gather(FwdArgs a) {
  const int64_t bj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bj < a.nbnode) bwd_boundary_node<D>(a, bj);
}

template <int D>
int backward_impl(const FwdArgs &a, int reduce, const LaunchCfg &cfg, hipStream_t s) {
  (void)cfg;
  if (reduce == EB_REDUCE_ATOMIC) {
    EB_TRY(fill_f64(a.g_x, a.nv, 0.0, s));
    EB_TRY(fill_f64(a.g_y, a.nv, 0.0, s));
    if (D == 3) EB_TRY(fill_f64(a.g_z, a.nv, 0.0, s));
    if (a.nelem > 0 && (a.w_x || a.c)) {
      launch_principal(k_bwd_atomic_elem<D>, dim3(grid_for(a.nelem, ATOMIC_TB * ATOMIC_EPT)),
                       dim3(ATOMIC_TB), 0, s, a);
      EB_LAUNCH_CHECK();
    }
    if (a.nbface > 0 && (a.w_x || a.be_x)) {
      hipLaunchKernelGGL(k_bwd_atomic_bface<D>, dim3(grid_for(a.nbface, BF_TB)), dim3(BF_TB), 0,
                         s, a);
      EB_LAUNCH_CHECK();
    }
    return EB_OK;
  }
  if (a.nelem > 0) {
    launch_principal(k_bwd_elem_pieces<D>, dim3(grid_for(a.nelem, 256)), dim3(256), 0, s, a);
    EB_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_bwd_node_gather<D>, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a);
  EB_LAUNCH_CHECK();
  if (a.nbnode > 0 && (a.w_x || a.be_x)) {
    hipLaunchKernelGGL(k_bwd_boundary_gather<D>, dim3(grid_for(a.nbnode, 256)), dim3(256), 0, s,
                       a);
    EB_LAUNCH_CHECK();
  }
  return EB_OK;
}

template int backward_impl<2>(const FwdArgs &, int, const LaunchCfg &, hipStream_t);
template int backward_impl<3>(const FwdArgs &, int, const LaunchCfg &, hipStream_t);

}  // namespace eb
