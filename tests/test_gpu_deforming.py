"""Deforming-grid loop: the topology is built once, the node coordinates move
in place every step, and a captured HIP graph replays the metric calls
(forward n, b, V; edge-based V; adjoint; residual).  Every replay must equal
the eager calls on the same coordinates bit for bit, with eager work and
synchronizations between replays, and the replayed metrics must still match
the oracle on the moved grid."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import meshgen
import oracle
from tests.test_gpu_parity import assert_vec_close, assert_vol_close, piece_scales, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2502_00778_amd as eb
    eb._lib.lib()
    yield


def eb():
    import paper_2502_00778_amd as m
    return m


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def frames(mesh, k, seed):
    """k moved copies of the grid: interior nodes displaced by up to 0.05 h."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (mesh.meta["n"] - 1)
    inside = ((mesh.coords > 0) & (mesh.coords < 1)).all(axis=0)
    out = []
    for _ in range(k):
        d = rng.uniform(-0.05 * h, 0.05 * h, size=mesh.coords.shape) * inside
        out.append(np.ascontiguousarray(mesh.coords + d))
    return out


@pytest.mark.parametrize("dim", [3, 2])
def test_graph_replay_on_moving_grid(dim):
    mesh = meshgen.cube_kuhn(17, 5) if dim == 3 else meshgen.square_tri(33, 5)
    X, E = T(mesh.coords), T(mesh.elems)
    t = eb().build_edges(E, X)
    w, c, beta = meshgen.loss_weights(5, dim, t.n_edges, t.n_nodes, t.n_bnodes)
    W, C, B = T(w), T(c), T(beta)
    F = T(np.random.default_rng(3).normal(size=(dim, t.n_nodes)))
    f64 = dict(dtype=torch.float64, device="cuda")
    n, b, V = torch.empty(dim, t.n_edges, **f64), torch.empty(dim, t.n_bnodes, **f64), \
        torch.empty(t.n_nodes, **f64)
    Ve, g, r = torch.empty(t.n_nodes, **f64), torch.empty(dim, t.n_nodes, **f64), \
        torch.empty(t.n_nodes, **f64)

    def step(outs):
        n_, b_, V_, Ve_, g_, r_ = outs
        eb().directed_areas(X, t, E, "gather", n_out=n_, b_out=b_, v_out=V_)
        eb().dual_volumes(X, t, E, "edge", n=n_, reduce="gather", out=Ve_)
        eb().directed_areas_backward(X, t, E, W, B, C, reduce="gather", out=g_)
        eb().edge_residual(X, t, E, n_, F, b_, bflux="linear", out=r_)

    outs = (n, b, V, Ve, g, r)
    step(outs)  # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step(outs)
    ref_outs = tuple(torch.empty_like(x) for x in outs)
    fr = frames(mesh, 4, 6)
    for k, Xk in enumerate(fr):
        X.copy_(T(Xk))
        graph.replay()
        torch.cuda.synchronize()
        got = [x.clone() for x in outs]
        step(ref_outs)  # eager on the same coordinates, other buffers
        torch.cuda.synchronize()
        for name, a_, b_ in zip(("n", "b", "V", "Ve", "g", "res"), got, ref_outs):
            assert torch.equal(a_, b_), f"frame {k}: {name}"
    eb().check_errors(t)
    # the last replay against the oracle on the moved grid
    Xl = fr[-1]
    ot = oracle.topology(dim, Xl, mesh.elems)
    n0, b0, V0 = oracle.metrics(ot, Xl, mesh.elems)
    S_e, S_b = piece_scales(ot, Xl, mesh.elems)
    assert_vec_close(got[0].cpu().numpy(), n0, S_e, "n")
    assert_vec_close(got[1].cpu().numpy(), b0, S_b, "b")
    assert_vol_close(got[2].cpu().numpy(), V0, "V")
    assert_vol_close(got[3].cpu().numpy(), V0, "edge V")
    say(f"[deforming] dim {dim}: 4 frames replayed, equal to eager, oracle-close")
