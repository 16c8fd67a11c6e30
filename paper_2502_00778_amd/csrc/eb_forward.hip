// The node pass of the deterministic forward (the kernel the HBM roofline is
// quoted for): one block per tile of TN consecutive nodes, the body in
// eb_gather.h; launched for the shape chosen at run time.
#include "eb_gather.h"

namespace eb {

template <int D, int TN, int CAP, int U, bool WIDE, bool STEP = false>
__global__ __launch_bounds__(TN) void k_fwd_gather(FwdArgs a) {
  __shared__ double acc[D][CAP];
  fwd_node_tile<D, TN, CAP, U, WIDE, VAR_NODE, STEP>(a, tile_of_block(gridDim.x, a.xcd_remap), acc);
}

template <int D>
int launch_fwd_nodes(const FwdArgs &a, const LaunchCfg &cfg, hipStream_t s) {
  const int64_t ntiles = (a.nv + cfg.tile - 1) / cfg.tile;
  const dim3 grid((unsigned)ntiles);
#define EB_GATHER_CASE(TN_, CAP_, U_)                                                   \
  if (cfg.tile == TN_ && cfg.unroll == U_) {                                            \
    if (!a.sell_wide) /* narrow entries always come with step words */                  \
      launch_principal((k_fwd_gather<D, TN_, CAP_, U_, false, true>), grid, dim3(TN_), 0, s, \
                       a);                                                              \
    else if (a.node_step)                                                               \
      launch_principal((k_fwd_gather<D, TN_, CAP_, U_, true, true>), grid, dim3(TN_), 0, s, \
                       a);                                                              \
    else                                                                                \
      launch_principal((k_fwd_gather<D, TN_, CAP_, U_, true>), grid, dim3(TN_), 0, s, a); \
    EB_LAUNCH_CHECK();                                                                  \
    return EB_OK;                                                                       \
  }
  EB_GATHER_CASE(64, 512, 1)
  EB_GATHER_CASE(64, 512, 2)
  EB_GATHER_CASE(64, 512, 4)
  EB_GATHER_CASE(128, 1024, 1)
  EB_GATHER_CASE(128, 1024, 2)
  EB_GATHER_CASE(128, 1024, 4)
  EB_GATHER_CASE(256, 2048, 1)
  EB_GATHER_CASE(256, 2048, 2)
  EB_GATHER_CASE(256, 2048, 4)
#undef EB_GATHER_CASE
  set_detail("unsupported gather tile %d / unroll %d", cfg.tile, cfg.unroll);
  return EB_EINVAL;
}

template int launch_fwd_nodes<2>(const FwdArgs &, const LaunchCfg &, hipStream_t);
template int launch_fwd_nodes<3>(const FwdArgs &, const LaunchCfg &, hipStream_t);

}  // namespace eb
