"""Edge-based grid metrics on MI355X (gfx950): HIP kernels behind a C ABI.

Lumped directed-area vectors of edges, boundary dual-face normals and
median-dual volumes computed straight from element geometry (Nishikawa,
"An Efficient Implementation of Edge-Based Discretization without Forming
Dual Control Volumes"), with GPU edge extraction and a hand-written adjoint.
The shared library ``libeb.so`` is loaded on first use; importing this
package does not touch the GPU.
"""
from .api import (REDUCE, VOL_MODE, Topology, build_edges, check_errors,  # noqa: F401
                  directed_areas, directed_areas_backward, dual_volumes,
                  dual_volumes_noalloc, directed_areas_variant, edge_residual, get_gather_shape,
                  set_gather_shape, time_next_call,
                  time_next_launch, workspace_bytes)
from ._lib import EbError  # noqa: F401
from .autograd import EdgeMetrics, edge_metrics  # noqa: F401
from .batch import (Batch, ForwardBackwardGraph, autotune, batch_offsets,  # noqa: F401
                    concat_host, forward_backward, get_fused_mode, get_fused_shape,
                    set_fused_mode, set_fused_shape, set_fused_wait_limit)

__version__ = "0.1.0"
