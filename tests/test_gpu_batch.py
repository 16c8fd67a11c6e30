"""Batched grids, the fused forward + adjoint kernel, graph replay and the
launch-shape tuner, through the C ABI.

Each mesh of a batch must give what it gives on its own (the gather path
sums in the same order, so the bits are the same), and what the oracle gives
for it (n, b, V relative 1e-12; dL/dx relative 1e-7).  The fused kernel must
be bitwise reproducible for every launch shape, and every graph replay must
equal the eager call bit for bit.
"""
from __future__ import annotations

import json

import numpy as np
import pytest
import torch

import meshgen
import oracle
from tests.test_gpu_parity import (GTOL, assert_vec_close, assert_vol_close, piece_scales,
                                   say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2502_00778_amd as eb
    eb._lib.lib()
    yield
    eb.set_fused_wait_limit(0)
    eb.set_fused_shape(128, 2, 0)


def eb():
    import paper_2502_00778_amd as m
    return m


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class BatchCase:
    """A batch built from per-mesh host arrays, its device topology, offsets
    and seeded loss weights."""

    def __init__(self, meshes, seed=0):
        self.meshes = meshes
        X, E, self.node_off, self.elem_off = eb().concat_host(
            [(m.coords, m.elems) for m in meshes])
        self.dim = meshes[0].dim
        self.Xh, self.Eh = X, E
        self.X, self.E = T(X), T(E)
        self.topo = eb().build_edges(self.E, self.X)
        self.batch = eb().batch_offsets(self.topo, self.E, self.node_off, self.elem_off)
        t = self.topo
        w, c, beta = meshgen.loss_weights(seed, self.dim, t.n_edges, t.n_nodes, t.n_bnodes)
        self.w, self.c, self.beta = w, c, beta
        self.W, self.C, self.B = T(w), T(c), T(beta)

    def fused(self):
        n, b, V, g = eb().forward_backward(self.X, self.topo, self.E, self.W, self.B, self.C)
        return [x.clone() for x in (n, b, V, g)]

    def separate(self):
        n, b, V = eb().directed_areas(self.X, self.topo, self.E, "gather")
        g = eb().directed_areas_backward(self.X, self.topo, self.E, self.W, self.B, self.C,
                                         reduce="gather")
        return [n, b, V, g]

    def mesh_weights(self, m):
        bt = self.batch
        e0, e1 = int(bt.edge_off[m]), int(bt.edge_off[m + 1])
        v0, v1 = int(bt.node_off[m]), int(bt.node_off[m + 1])
        b0, b1 = int(bt.bnode_off[m]), int(bt.bnode_off[m + 1])
        return self.w[:, e0:e1], self.c[v0:v1], self.beta[:, b0:b1]


def kuhn_batch(sizes, seed=0, dim=3):
    if dim == 3:
        return [meshgen.cube_kuhn(int(n), seed + i) for i, n in enumerate(sizes)]
    return [meshgen.square_tri(int(n), seed + i) for i, n in enumerate(sizes)]


@pytest.fixture(scope="module")
def small3():
    return BatchCase(kuhn_batch([5, 9, 3, 12, 7], seed=2), seed=3)


@pytest.fixture(scope="module")
def small2():
    return BatchCase(kuhn_batch([6, 17, 3, 9], seed=4, dim=2), seed=5)


@pytest.mark.parametrize("which", ["small3", "small2"])
def test_offsets_match_oracle_per_mesh(which, request):
    bc = request.getfixturevalue(which)
    say(f"[batch offsets] {which}: {len(bc.meshes)} meshes")
    bt = bc.batch
    g = bc.topo.to_numpy()
    for m, mesh in enumerate(bc.meshes):
        ot = oracle.topology(bc.dim, mesh.coords, mesh.elems)
        assert bt.edge_off[m + 1] - bt.edge_off[m] == ot.n_edges
        assert bt.bnode_off[m + 1] - bt.bnode_off[m] == ot.n_bnodes
        assert bt.bface_off[m + 1] - bt.bface_off[m] == ot.n_bfaces
        e0, e1 = bt.edge_off[m], bt.edge_off[m + 1]
        np.testing.assert_array_equal(g["edge"][:, e0:e1] - bt.node_off[m], ot["edge"])
        f0, f1 = bt.bface_off[m], bt.bface_off[m + 1]
        np.testing.assert_array_equal(g["bface"][f0:f1] - bt.node_off[m], ot["bface"])
        b0, b1 = bt.bnode_off[m], bt.bnode_off[m + 1]
        np.testing.assert_array_equal(g["bnode"][b0:b1] - bt.node_off[m], ot["bnode"])


@pytest.mark.parametrize("which", ["small3", "small2"])
def test_fused_matches_oracle_per_mesh(which, request):
    bc = request.getfixturevalue(which)
    n, b, V, g = (x.cpu().numpy() for x in bc.fused())
    eb().check_errors(bc.topo)
    bt = bc.batch
    for m, mesh in enumerate(bc.meshes):
        ot = oracle.topology(bc.dim, mesh.coords, mesh.elems)
        n0, b0, V0 = oracle.metrics(ot, mesh.coords, mesh.elems)
        S_e, S_b = piece_scales(ot, mesh.coords, mesh.elems)
        nm, bm, Vm, gm = (bt.split(torch.from_numpy(x), k)[m].numpy()
                          for x, k in ((n, "edge"), (b, "bnode"), (V, "node"), (g, "node")))
        assert_vec_close(nm, n0, S_e, f"n mesh {m}")
        assert_vec_close(bm, b0, S_b, f"b mesh {m}")
        assert_vol_close(Vm, V0, f"V mesh {m}")
        w, c, beta = bc.mesh_weights(m)
        _, gref = oracle.node_grad(ot, mesh.coords, mesh.elems, w, c, beta)
        rel = np.linalg.norm(gm.T - gref, axis=1) / np.linalg.norm(gref, axis=1)
        assert (rel <= GTOL).all(), f"mesh {m}: grad rel {rel.max():.2e}"
    say(f"[fused vs oracle] {which}: {len(bc.meshes)} meshes ok")


@pytest.mark.parametrize("which", ["small3", "small2"])
def test_fused_matches_separate_calls(which, request):
    """The fused kernel against the separate gather forward and adjoint calls
    on the same batch (same arithmetic; allowed to differ only by rounding
    from contraction choices, and reported if the bits differ)."""
    bc = request.getfixturevalue(which)
    fu = [x.cpu().numpy() for x in bc.fused()]
    se = [x.cpu().numpy() for x in bc.separate()]
    for name, a, r in zip("nbVg", fu, se):
        scale = np.abs(r).max()
        diff = np.abs(a - r).max()
        same = int((a == r).sum())
        say(f"    {name}: {same}/{a.size} identical bits, max diff {diff:.2e} (scale {scale:.2e})")
        assert diff <= 1e-14 * scale


def test_batch_equals_each_mesh_alone(small3):
    """Each mesh's slice of the batch equals the mesh run on its own, bit for
    bit (gather path: same elements, same order)."""
    bc = small3
    n, b, V, g = (x.cpu() for x in bc.separate())
    bt = bc.batch
    for m, mesh in enumerate(bc.meshes):
        X, E = T(mesh.coords), T(mesh.elems)
        tm = eb().build_edges(E, X)
        w, c, beta = bc.mesh_weights(m)
        n1, b1, V1 = eb().directed_areas(X, tm, E, "gather")
        g1 = eb().directed_areas_backward(X, tm, E, T(w), T(beta), T(c), reduce="gather")
        assert torch.equal(bt.split(n, "edge")[m], n1.cpu())
        assert torch.equal(bt.split(b, "bnode")[m], b1.cpu())
        assert torch.equal(bt.split(V, "node")[m], V1.cpu())
        assert torch.equal(bt.split(g, "node")[m], g1.cpu())


def test_fused_bitwise_across_shapes(small3):
    bc = small3
    eb().set_fused_shape(128, 2, 0)
    ref = bc.fused()
    for tile in (64, 128, 256):
        for unroll in (1, 2, 4):
            for per_cu in (1, 0):
                eb().set_fused_shape(tile, unroll, per_cu)
                got = bc.fused()
                for a, r in zip(got, ref):
                    assert torch.equal(a, r), (tile, unroll, per_cu)
    eb().set_fused_shape(128, 2, 0)
    eb().set_fused_mode("separate")
    got = bc.fused()
    eb().set_fused_mode("persistent")
    for a, r in zip(got, ref):
        assert torch.equal(a, r), "separate mode"
    eb().check_errors(bc.topo)


def test_separate_atomic_mode(small3):
    """The gather forward and the atomic adjoint in sequence: n, b, V equal
    the deterministic enqueue's bits, dL/dx matches it to rounding, eager and
    from a graph."""
    bc = small3
    ref = bc.fused()
    eb().set_fused_mode("separate_atomic")
    try:
        assert eb().get_fused_mode() == "separate_atomic"
        gr = eb().ForwardBackwardGraph(bc.X, bc.topo, bc.E, bc.W, bc.B, bc.C)
        for run in range(3):
            outs = bc.fused() if run == 0 else gr.launch()
            torch.cuda.synchronize()
            for k, (a, b) in enumerate(zip(outs, ref)):
                if k < 3:
                    assert torch.equal(a, b), f"run {run} output {k}"
                else:
                    scale = b.abs().max().item()
                    assert (a - b).abs().max().item() <= 1e-12 * scale, f"run {run} grad"
        gr.close()
        eb().check_errors(bc.topo)
    finally:
        eb().set_fused_mode("persistent")


@pytest.mark.parametrize("mode", ["persistent", "separate"])
def test_graph_modes_equal_eager(small2, mode):
    """Both forms of the enqueue capture into a graph that replays the eager
    result."""
    bc = small2
    eb().set_fused_mode(mode)
    try:
        ref = bc.fused()
        gr = eb().ForwardBackwardGraph(bc.X, bc.topo, bc.E, bc.W, bc.B, bc.C)
        for _ in range(2):
            outs = gr.launch()
            torch.cuda.synchronize()
            for a, b in zip(outs, ref):
                assert torch.equal(a, b)
        gr.close()
    finally:
        eb().set_fused_mode("persistent")


@pytest.mark.parametrize("which", ["small3", "small2"])
def test_atomic_mode_matches_gather_and_oracle(which, request):
    """The persistent kernel with the FP64-atomic adjoint: n, b, V equal the
    gather forward call's bits (the same node and boundary routines), and
    dL/dx matches the gather adjoint to rounding and the oracle per mesh,
    for every launch shape."""
    bc = request.getfixturevalue(which)
    se = [x.cpu().numpy() for x in bc.separate()]
    eb().set_fused_mode("persistent_atomic")
    try:
        assert eb().get_fused_mode() == "persistent_atomic"
        for tile, unroll, per_cu in ((128, 2, 0), (64, 1, 1), (256, 4, 2)):
            eb().set_fused_shape(tile, unroll, per_cu)
            n, b, V, g = (x.cpu().numpy() for x in bc.fused())
            for name, a, r in zip("nbV", (n, b, V), se[:3]):
                diff = np.abs(a - r).max()
                say(f"    {name} ({tile},{unroll},{per_cu}): max diff {diff:.2e}")
                assert diff <= 1e-14 * np.abs(r).max(), name
            scale = np.abs(se[3]).max()
            assert np.abs(g - se[3]).max() <= 1e-12 * scale, "grad vs gather"
            eb().check_errors(bc.topo)
        bt = bc.batch
        for m, mesh in enumerate(bc.meshes):
            ot = oracle.topology(bc.dim, mesh.coords, mesh.elems)
            w, c, beta = bc.mesh_weights(m)
            _, gref = oracle.node_grad(ot, mesh.coords, mesh.elems, w, c, beta)
            gm = bt.split(torch.from_numpy(g), "node")[m].numpy()
            rel = np.linalg.norm(gm.T - gref, axis=1) / np.linalg.norm(gref, axis=1)
            assert (rel <= GTOL).all(), f"mesh {m}: grad rel {rel.max():.2e}"
    finally:
        eb().set_fused_shape(128, 2, 0)
        eb().set_fused_mode("persistent")


def test_atomic_mode_graph_and_tuner(small3, tmp_path):
    """The atomic persistent kernel captures into a graph whose replays (the
    gradient zeroed by a fill kernel each time) match the eager call, and the
    tuner keeps the mode while tuning its shape."""
    bc = small3
    eb().set_fused_mode("persistent_atomic")
    try:
        ref = bc.fused()
        gr = eb().ForwardBackwardGraph(bc.X, bc.topo, bc.E, bc.W, bc.B, bc.C)
        for r in range(3):
            eb().directed_areas(bc.X, bc.topo, bc.E, "gather")
            torch.cuda.synchronize()
            outs = gr.launch()
            torch.cuda.synchronize()
            for k, (a, b) in enumerate(zip(outs, ref)):
                if k < 3:
                    assert torch.equal(a, b), f"replay {r} output {k}"
                else:
                    scale = b.abs().max().item()
                    assert (a - b).abs().max().item() <= 1e-12 * scale, f"replay {r} grad"
        gr.close()
        cache = str(tmp_path / "tune_atomic.json")
        r = eb().autotune(bc.X, bc.topo, bc.E, bc.W, bc.B, bc.C, reps=1, cache=cache)
        say(f"[autotune atomic] {r}")
        assert not r["cached"] and r["n_tried"] == 18 + 45 + 1
        mode = "separate_atomic" if r["fused_separate"] else "persistent_atomic"
        assert eb().get_fused_mode() == mode
        assert eb().get_fused_shape() == (r["fused_tile"], r["fused_unroll"],
                                          r["fused_blocks_per_cu"])
        assert next(iter(json.load(open(cache)))).endswith("|atomic")
        # a cached entry restores the same choice within the atomic modes
        eb().set_fused_mode("persistent_atomic")
        rc = eb().autotune(bc.X, bc.topo, bc.E, bc.W, bc.B, bc.C, reps=1, cache=cache)
        assert rc["cached"] and eb().get_fused_mode() == mode
        eb().check_errors(bc.topo)
    finally:
        eb().set_fused_shape(128, 2, 0)
        eb().set_fused_mode("persistent")
        eb().set_gather_shape(64, 2, 1)


def test_graph_replays_equal_eager(small3):
    """Replays of the captured enqueue, with eager work between them, equal
    the eager call; after coordinates move in place, a replay equals the
    eager call on the new coordinates."""
    bc = small3
    X0 = bc.X.clone()
    ref = bc.fused()
    gr = eb().ForwardBackwardGraph(bc.X, bc.topo, bc.E, bc.W, bc.B, bc.C)
    for r in range(3):
        # unrelated eager work on the same stream and workspace in between
        eb().directed_areas(bc.X, bc.topo, bc.E, "gather")
        torch.cuda.synchronize()
        outs = gr.launch()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), f"replay {r}"
    # a deforming grid: move interior nodes of every mesh a little
    rng = np.random.default_rng(11)
    dx = rng.uniform(-1e-3, 1e-3, size=bc.Xh.shape) * (bc.Xh > 0) * (bc.Xh < 1)
    bc.X.copy_(T(bc.Xh + dx))
    outs = [x.clone() for x in gr.launch()]
    torch.cuda.synchronize()
    ref2 = bc.fused()
    for a, b in zip(outs, ref2):
        assert torch.equal(a, b)
    assert not torch.equal(ref2[0], ref[0])
    gr.close()
    bc.X.copy_(X0)
    eb().check_errors(bc.topo)


def test_autotune_and_cache(small3, tmp_path):
    bc = small3
    ref = bc.fused()
    cache = str(tmp_path / "tune.json")
    r = eb().autotune(bc.X, bc.topo, bc.E, bc.W, bc.B, bc.C, reps=2, cache=cache)
    say(f"[autotune] {r}")
    assert not r["cached"] and r["n_tried"] == 18 + 45 + 1
    assert r["gather_tile"] in (64, 128, 256) and r["fused_tile"] in (64, 128, 256)
    assert eb().get_fused_shape() == (r["fused_tile"], r["fused_unroll"],
                                      r["fused_blocks_per_cu"])
    got = bc.fused()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    r2 = eb().autotune(bc.X, bc.topo, bc.E, bc.W, bc.B, bc.C, cache=cache)
    assert r2["cached"] and json.load(open(cache))
    eb().set_fused_shape(128, 2, 0)
    eb().set_fused_mode("persistent")
    eb().set_gather_shape(64, 2, 1)  # the defaults


def test_offsets_reject_cross_mesh_element(small3):
    bc = small3
    bad = bc.node_off.copy()
    bad[1] -= 1  # the last node of mesh 0 now belongs to mesh 1
    with pytest.raises(eb().EbError) as e:
        eb().batch_offsets(bc.topo, bc.E, bad, bc.elem_off)
    assert e.value.code == -1
    eb().check_errors(bc.topo)  # reported and cleared by the call itself
    with pytest.raises(eb().EbError):
        eb().batch_offsets(bc.topo, bc.E, bc.node_off[:-1], bc.elem_off[:-1])


@pytest.mark.parametrize("mode", ["persistent", "persistent_atomic"])
def test_fused_wait_limit_reports_timeout(mode):
    """A bound of one poll on the fused kernel's phase waits, set from the
    host: the first block to finish phase 0 finds most others still in it
    (about 0.5 us of polling against tiles of several microseconds), gives
    up, records EB_ETIMEOUT and exits, and so, in turn, does every block that
    waits on it (every wave ends); the default bound restores normal runs."""
    mesh = meshgen.cube_kuhn(41, 0)
    X, E = T(mesh.coords), T(mesh.elems)
    t = eb().build_edges(E, X)
    eb().set_fused_mode(mode)
    eb().set_fused_wait_limit(1)
    try:
        eb().forward_backward(X, t, E)
        torch.cuda.synchronize()
        rc = eb()._lib.lib().eb_check_errors(eb().api._ptr(t.ws), None)
        say(f"[wait limit 1, {mode}] status {rc}")
        assert rc == -9
    finally:
        eb().set_fused_wait_limit(0)
        eb().set_fused_mode("persistent")
    n, b, V, g = eb().forward_backward(X, t, E)
    eb().check_errors(t)
    n1, b1, V1 = eb().directed_areas(X, t, E, "gather")
    assert (n - n1).abs().max() <= 1e-14 * n1.abs().max()


@pytest.mark.timeout(900)
def test_full_batch_64():
    """The 64-mesh batch (about 21.8M tets): fused forward + adjoint, every
    mesh's n, b and V against the oracle and its gradient at 200 sampled
    nodes, and the whole batch against the separate gather calls (about half
    a minute of oracle work on the host)."""
    bm = meshgen.batched_kuhn(64, 0)
    meshes = []
    for m in range(64):
        v0, v1 = bm.node_off[m], bm.node_off[m + 1]
        e0, e1 = bm.elem_off[m], bm.elem_off[m + 1]
        meshes.append(meshgen.Mesh(3, bm.coords[:, v0:v1], bm.elems[e0:e1] - v0, f"m{m}"))
    bc = BatchCase(meshes, seed=0)
    say(f"[batch 64] {bc.topo.n_elems} tets, {bc.topo.n_edges} edges")
    fu = bc.fused()
    eb().check_errors(bc.topo)
    se = bc.separate()
    for name, a, r in zip("nbVg", fu, se):
        assert (a - r).abs().max() <= 1e-14 * r.abs().max(), name
    bt = bc.batch
    for m in range(64):
        mesh = meshes[m]
        ot = oracle.topology(3, mesh.coords, mesh.elems)
        n0, b0, V0 = oracle.metrics(ot, mesh.coords, mesh.elems)
        S_e, S_b = piece_scales(ot, mesh.coords, mesh.elems)
        assert_vec_close(bt.split(fu[0], "edge")[m].cpu().numpy(), n0, S_e, f"n mesh {m}")
        assert_vec_close(bt.split(fu[1], "bnode")[m].cpu().numpy(), b0, S_b, f"b mesh {m}")
        assert_vol_close(bt.split(fu[2], "node")[m].cpu().numpy(), V0, f"V mesh {m}")
        w, c, beta = bc.mesh_weights(m)
        nodes = np.random.default_rng(m).choice(ot.n_nodes, 200, replace=False).astype(np.int32)
        _, gref = oracle.node_grad(ot, mesh.coords, mesh.elems, w, c, beta, nodes)
        gm = bt.split(fu[3], "node")[m].cpu().numpy()[:, nodes].T
        rel = np.linalg.norm(gm - gref, axis=1) / np.linalg.norm(gref, axis=1)
        assert (rel <= GTOL).all(), f"mesh {m}: grad rel {rel.max():.2e}"
        if m % 8 == 7:
            say(f"    meshes {m - 7}..{m}: ok")
