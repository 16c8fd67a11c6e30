// The edge loop of eb_dual_volumes for callers that cannot allocate: its
// per-edge terms live in a fixed device array of the library instead of the
// caller's workspace.
#include <mutex>

#include "eb_kernels.h"

namespace eb {
namespace {

constexpr size_t kScratchBytes = EB_NOALLOC_SCRATCH_BYTES;

// One copy per GPU, at its own address; host code uses the address
// hipGetSymbolAddress returns for the current device, never this name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// The current device's address of `scratch`, looked up once per device.
int scratch_address(void **out) {
  int dev = -1;
  EB_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_detail("device %d beyond the %d devices the library tracks", dev, kMaxDevices);
    return EB_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    EB_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return EB_OK;
}

}  // namespace
}  // namespace eb

using namespace eb;

extern "C" int eb_dual_volumes_noalloc(const eb_sizes *sizes, const eb_topology *topo,
                                       const double *coords, const double *n_edge, int reduce,
                                       double *vol, hipStream_t stream) {
  PrincipalScope scope;
  clear_detail();
  EB_TRY(check_sizes(sizes));
  EB_TRY(only_dims23(sizes));
  FwdArgs a;
  EB_TRY(pack_arrays(sizes, topo, nullptr, coords, false, a));
  if ((reduce != EB_REDUCE_ATOMIC && reduce != EB_REDUCE_GATHER) || !vol) {
    set_detail("bad reduce, or vol / n_edge is null");
    return EB_EINVAL;
  }
  if (no_elements(sizes)) return fill_f64(vol, sizes->n_nodes, 0.0, stream);
  if (!n_edge) {
    set_detail("bad reduce, or vol / n_edge is null");
    return EB_EINVAL;
  }
  EB_TRY(need(a.edge_tail && a.edge_head, "edge"));
  if (reduce == EB_REDUCE_GATHER) {
    EB_TRY(need(a.node_edge_off && a.node_in_off && a.node_in_edge, "node_edge_off, node_in"));
    if ((size_t)sizes->n_edges > kScratchBytes / sizeof(double)) {
      set_detail("%lld edges: the library's fixed scratch holds the terms of at most %zu",
                 (long long)sizes->n_edges, kScratchBytes / sizeof(double));
      return EB_EWORKSPACE;
    }
    void *p = nullptr;
    EB_TRY(scratch_address(&p));
    a.vterm = static_cast<double *>(p);  // every term is written before it is read
  }
  a.vol = vol;
  return sizes->dim == 2 ? volumes_impl<2>(a, EB_VOL_EDGE, reduce, n_edge, stream)
                         : volumes_impl<3>(a, EB_VOL_EDGE, reduce, n_edge, stream);
}
