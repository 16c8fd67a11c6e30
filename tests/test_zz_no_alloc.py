"""eb_dual_volumes_noalloc (the edge loop without a workspace, for callers
that cannot allocate) against eb_dual_volumes EB_VOL_EDGE on the same
inputs, through the C ABI: two calls in a row on the library's one fixed
array, the second on a smaller grid, and the size limit."""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest
import torch

import meshgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _grid(mesh):
    import paper_2502_00778_amd as eb
    X = torch.from_numpy(np.ascontiguousarray(mesh.coords)).cuda()
    E = torch.from_numpy(np.ascontiguousarray(mesh.elems)).cuda()
    topo = eb.build_edges(E, X, edge_inc=False, adjoint=False)
    n, _, _ = eb.directed_areas(X, topo, E, "gather", volumes=False, boundary=False)
    return X, E, topo, n


def test_noalloc_matches_workspace_call_twice():
    import paper_2502_00778_amd as eb
    assert torch.cuda.is_available()
    for name, mesh in (("3d-41", meshgen.cube_kuhn(41, 0)), ("3d-17", meshgen.cube_kuhn(17, 3)),
                       ("2d-33", meshgen.square_tri(33, 1))):
        say(f"[noalloc] {name}: {mesh.n_elems} elements")
        X, E, topo, n = _grid(mesh)
        for reduce in ("gather", "atomic"):
            ref = eb.dual_volumes(X, topo, E, mode="edge", n=n, reduce=reduce)
            got = eb.dual_volumes_noalloc(X, topo, n, reduce=reduce)
            torch.cuda.synchronize()
            if reduce == "gather":  # same kernels, same order: the same bits
                assert torch.equal(got, ref), name
            else:
                used = ref > 0
                rel = ((got - ref).abs()[used] / ref[used]).max().item()
                assert rel <= 1e-12, (name, rel)
                assert (got[~used] == 0).all()
        eb.check_errors(topo)


def test_noalloc_rejects_grids_beyond_its_array():
    """More edges than the fixed array holds terms for: EB_EWORKSPACE before
    any device work (the size is checked on the host)."""
    import paper_2502_00778_amd as eb
    from paper_2502_00778_amd import _lib
    mesh = meshgen.cube_kuhn(9, 0)
    X, E, topo, n = _grid(mesh)
    sz = _lib.EbSizes()
    ctypes.memmove(ctypes.byref(sz), ctypes.byref(topo.sizes), ctypes.sizeof(sz))
    cap = (64 << 20) // 8
    sz.n_edges = cap + 1
    V = torch.empty(topo.n_nodes, dtype=torch.float64, device="cuda")
    rc = _lib.lib().eb_dual_volumes_noalloc(ctypes.byref(sz), ctypes.byref(topo.struct),
                                            ctypes.c_void_p(X.data_ptr()),
                                            ctypes.c_void_p(n.data_ptr()), 1,
                                            ctypes.c_void_p(V.data_ptr()), None)
    assert rc == -5
    assert b"fixed scratch" in _lib.lib().eb_last_error_detail()
