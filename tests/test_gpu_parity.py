"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Topology: bit-exact.  n, b, V: per entry, norm-wise, relative 1e-12 of the
oracle value; where an edge (or boundary node) sum cancels below 1e-3 of the
sum of its pieces' magnitudes S, the bound is 1e-12 * S instead.  Gradients:
relative 1e-7 per node against the oracle's forward-mode reference and
against patch-local central differences.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle
from tests._plan import check_plan

pytestmark = pytest.mark.gpu

TOL = 1e-12
GTOL = 1e-7


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2502_00778_amd as eb
    eb._lib.lib()
    yield


def eb():
    import paper_2502_00778_amd as m
    return m


def dev(mesh):
    return (torch.from_numpy(np.ascontiguousarray(mesh.coords)).cuda(),
            torch.from_numpy(np.ascontiguousarray(mesh.elems)).cuda())


TOPO_NAMES = ("edge", "node_edge_off", "elem_edge", "elem_edge_sign", "edge_inc_off",
              "edge_inc", "node_inc_off", "node_inc", "node_in_off", "node_in_edge",
              "bface", "bface_owner", "bface_edge", "bnode", "node_bnode",
              "bnode_face_off", "bnode_face")


def assert_topo_equal(gt, ot, elems):
    """Every topology array bit-exact against the oracle, and the kernel
    plan a faithful view of that topology (tests/_plan.py)."""
    assert (gt.n_edges, gt.n_bfaces, gt.n_bnodes) == (ot.n_edges, ot.n_bfaces, ot.n_bnodes)
    g = gt.to_numpy()
    for name in TOPO_NAMES:
        b = ot[name].reshape(-1)
        a = g[name].reshape(-1)
        assert a.shape == b.shape, (name, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{name}: {bad.size} entries differ, first at {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
    return check_plan(gt, ot, np.asarray(elems))


def bface_normals(ot, coords):
    """|n_B| of every boundary face (numpy, from the oracle's boundary list)."""
    D = ot.dim
    P = coords[:, ot["bface"]]  # [D, NB, D]
    if D == 2:
        d = P[:, :, 1] - P[:, :, 0]
        return np.hypot(d[0], d[1])
    u = (P[:, :, 1] - P[:, :, 0]).T
    v = (P[:, :, 2] - P[:, :, 0]).T
    return 0.5 * np.linalg.norm(np.cross(u, v), axis=1)


def piece_scales(ot, coords, elems):
    """S_e and S_j: sums of the magnitudes of the pieces each sum adds up
    (the oracle's per-element dual-face pieces; the boundary pieces of a node
    are n_B/D of each boundary face, Section 3.2.3)."""
    D = ot.dim
    npc, _ = oracle.element_pieces(D, coords, elems)
    S_e = np.bincount(ot["elem_edge"].reshape(-1), weights=np.linalg.norm(npc, axis=2).reshape(-1),
                      minlength=ot.n_edges)
    del npc
    S_b = np.zeros(ot.n_bnodes)
    nb = bface_normals(ot, coords) / D
    for s in range(D):
        S_b += np.bincount(ot["node_bnode"][ot["bface"][:, s]], weights=nb, minlength=ot.n_bnodes)
    return S_e, S_b


def assert_vec_close(got, ref, S, what, tol=TOL):
    err = np.linalg.norm(got - ref, axis=0)
    mag = np.linalg.norm(ref, axis=0)
    cancel = mag < 1e-3 * S
    bound = np.where(cancel, tol * S, tol * mag)
    bad = err > bound
    if bad.any():
        i = np.nonzero(bad)[0]
        raise AssertionError(f"{what}: {i.size} entries off, worst rel "
                             f"{(err / np.maximum(mag, 1e-300)).max():.3e} at {i[:5]}")
    return int(cancel.sum()), float((err / np.where(cancel, S, mag)).max(initial=0.0))


def assert_vol_close(got, ref, what, tol=TOL):
    rel = np.abs(got - ref) / np.abs(ref)
    assert (rel <= tol).all(), f"{what}: worst rel {rel.max():.3e}"
    return float(rel.max(initial=0.0))


# -------------------------------------------------------------- meshes

def shuffled(mesh, seed):
    rng = np.random.default_rng(seed)
    E = mesh.elems.copy()
    for i in range(E.shape[0]):
        E[i] = E[i, rng.permutation(E.shape[1])]
    return meshgen.Mesh(mesh.dim, mesh.coords, np.ascontiguousarray(E), mesh.name + "-shuf")


def with_isolated_nodes(mesh, extra=5, seed=0):
    # append nodes no element references (ragged: no edges, zero volume)
    rng = np.random.default_rng(seed)
    X = np.concatenate([mesh.coords, rng.uniform(2, 3, size=(mesh.dim, extra))], 1)
    return meshgen.Mesh(mesh.dim, np.ascontiguousarray(X), mesh.elems, mesh.name + "-iso")


def relabelled(mesh, seed):
    # random node numbering: neighbours far apart in id (wide sliced-ELL
    # entries once the grid has more than 32768 nodes)
    lab = np.random.default_rng(seed).permutation(mesh.n_nodes).astype(np.int32)
    X = np.empty_like(mesh.coords)
    X[:, lab] = mesh.coords
    return meshgen.Mesh(mesh.dim, X, np.ascontiguousarray(lab[mesh.elems]), mesh.name + "-relab")


def cone(k, centre=None):
    """2k tetrahedra around one node: a ring of k nodes in a plane, an apex
    above and below, every tet (centre, ring i, ring i+1, apex).  The centre's
    row has 2k entries (a strip longer than 24 when k > 12) and k + 2
    neighbours; it is numbered `centre` (default: in the middle)."""
    ang = np.linspace(0, 2 * np.pi, k, endpoint=False)
    P = np.zeros((3, k + 3))
    P[0, :k], P[1, :k] = np.cos(ang), np.sin(ang)
    P[2, k], P[2, k + 1] = 1.0, -1.0
    c = k + 2
    E = [[c, i, (i + 1) % k, k] for i in range(k)] + [[c, i, (i + 1) % k, k + 1] for i in range(k)]
    E = np.array(E, np.int32)
    # the centre numbered in the middle by default, so it has lower and
    # higher neighbours
    lab = np.roll(np.arange(k + 3), c - ((k + 3) // 2 if centre is None else centre)).astype(np.int32)
    X = np.empty_like(P)
    X[:, lab] = P
    return meshgen.Mesh(3, np.ascontiguousarray(X), np.ascontiguousarray(lab[E]), f"cone{k}")


def fan_mesh(k):
    Xf, Ef = fan(k)
    return meshgen.Mesh(2, np.ascontiguousarray(Xf), Ef, f"fan{k}")


def single(dim):
    if dim == 2:
        return meshgen.Mesh(2, np.array([[0., 1, 0], [0, 0, 1]]), np.array([[0, 2, 1]], np.int32))
    return meshgen.Mesh(3, np.array([[0., 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]]),
                        np.array([[0, 2, 1, 3]], np.int32))


CASES = {
    "2d-33": lambda: meshgen.square_tri(33, 0),
    "2d-33-s1": lambda: meshgen.square_tri(33, 1),
    "2d-65-shuf": lambda: shuffled(meshgen.square_tri(65, 2), 3),
    "3d-41": lambda: meshgen.cube_kuhn(41, 0),
    "3d-41-s2": lambda: meshgen.cube_kuhn(41, 2),
    "3d-17-shuf": lambda: shuffled(meshgen.cube_kuhn(17, 1), 4),
    "3d-scale-33": lambda: meshgen.scale_cube(33, 0, first=5e-3),
    "3d-7-iso": lambda: with_isolated_nodes(meshgen.cube_kuhn(7, 5)),
    "2d-single": lambda: single(2),
    "3d-single": lambda: single(3),
    "3d-batched-4": lambda: meshgen.batched_kuhn(4, 0, lo=3, hi=9),
    "3d-33-relabel": lambda: relabelled(meshgen.cube_kuhn(33, 1), 7),
    "3d-cone-14": lambda: cone(14),
    # 22 neighbours (past two groups of eight set slots), 7 of them higher;
    # a row of 40 entries (longer than a strip)
    "3d-cone-20": lambda: cone(20, centre=15),
    "2d-fan-28": lambda: fan_mesh(28),
    # nodes of high degree (the general per-node kernel): 140 and 400
    # neighbours above the centre (wide entries), a centre with 152
    # neighbours and 300 tetrahedra numbered in the middle and first
    "2d-fan-140": lambda: fan_mesh(140),
    "2d-fan-400": lambda: fan_mesh(400),
    "3d-cone-150": lambda: cone(150),
    "3d-cone-150-low": lambda: cone(150, centre=0),
    # the centre numbered last: 4200 tetrahedra at one node, 2100 around each
    # axis edge and 2100 boundary faces at each apex (CSR rows sorted by one
    # lane beyond 2048 entries)
    "3d-cone-2100-high": lambda: cone(2100, centre=2102),
}

_cache = {}


def case(name):
    if name not in _cache:
        mesh = CASES[name]()
        ot = oracle.topology(mesh.dim, mesh.coords, mesh.elems)
        n, b, V = oracle.metrics(ot, mesh.coords, mesh.elems)
        _cache[name] = (mesh, ot, n, b, V)
    return _cache[name]


# ----------------------------------------------------------------- tests

@pytest.mark.parametrize("name", list(CASES))
def test_topology_bit_exact(name):
    mesh, ot, *_ = case(name)
    say(f"[topology] {name} nv={mesh.n_nodes} ne={mesh.n_elems}")
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    info = assert_topo_equal(gt, ot, mesh.elems)
    say(f"    plan: {info}")
    if name.endswith("relabel") or name in ("2d-fan-140", "2d-fan-400", "3d-cone-150-low"):
        assert info["wide"]


@pytest.mark.parametrize("reduce", ["gather", "atomic"])
@pytest.mark.parametrize("name", list(CASES))
def test_metrics_parity(name, reduce):
    mesh, ot, n0, b0, V0 = case(name)
    say(f"[metrics] {name} reduce={reduce}")
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    n, b, V = eb().directed_areas(X, gt, E, reduce=reduce)
    eb().check_errors(gt)
    S_e, S_b = piece_scales(ot, mesh.coords, mesh.elems)
    ncan, nrel = assert_vec_close(n.cpu().numpy(), n0, S_e, "n")
    bcan, brel = assert_vec_close(b.cpu().numpy(), b0, S_b, "b")
    used = V0 > 0
    vrel = assert_vol_close(V.cpu().numpy()[used], V0[used], "V")
    assert (V.cpu().numpy()[~used] == 0).all()
    say(f"    max rel n {nrel:.2e} (cancelling edges {ncan}), b {brel:.2e}, V {vrel:.2e}")


@pytest.mark.parametrize("name,fmt", [("3d-41", 0), ("3d-33-relabel", 2),
                                      ("3d-cone-150-low", 1), ("2d-fan-400", 1),
                                      ("3d-81-relabel", 1)])
def test_plan_formats(name, fmt):
    """The three plan formats: narrow entries with step words, wide entries
    with step words (offsets within 20 bits, at most 31 out-edges: a random
    numbering of 35,937 nodes), wide entries alone (more than 31 out-edges,
    or offsets beyond 20 bits: a random numbering of 531,441 nodes); each
    valid against the oracle's topology, and the gather forward's n, b, V
    in parity, bitwise equal for every launch shape."""
    if name == "3d-81-relabel":
        mesh = relabelled(meshgen.cube_kuhn(81, 3), 9)
        ot = oracle.topology(3, mesh.coords, mesh.elems)
        n0, b0, V0 = oracle.metrics(ot, mesh.coords, mesh.elems)
    else:
        mesh, ot, n0, b0, V0 = case(name)
    say(f"[plan format] {name}: expect {fmt}")
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    assert int(gt.sizes.plan_param[1]) == fmt
    info = assert_topo_equal(gt, ot, mesh.elems)
    assert info["steps"] == (fmt != 1)
    n, b, V = eb().directed_areas(X, gt, E, reduce="gather")
    eb().check_errors(gt)
    S_e, S_b = piece_scales(ot, mesh.coords, mesh.elems)
    assert_vec_close(n.cpu().numpy(), n0, S_e, "n")
    assert_vec_close(b.cpu().numpy(), b0, S_b, "b")
    used = V0 > 0
    assert_vol_close(V.cpu().numpy()[used], V0[used], "V")
    ref = [x.clone() for x in (n, b, V)]
    try:
        for tile in (64, 128, 256):
            for unroll in (1, 2, 4):
                eb().set_gather_shape(tile, unroll, 1)
                got = eb().directed_areas(X, gt, E, reduce="gather")
                for x, r in zip(got, ref):
                    assert torch.equal(x, r), (tile, unroll)
    finally:
        eb().set_gather_shape(64, 2, 1)


@pytest.mark.parametrize("name", ["3d-41", "2d-33", "3d-7-iso"])
def test_volumes_both_modes(name):
    mesh, ot, n0, b0, V0 = case(name)
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    used = V0 > 0
    for reduce in ("gather", "atomic"):
        say(f"[volumes] {name} reduce={reduce}")
        n, _, _ = eb().directed_areas(X, gt, E, reduce=reduce, volumes=False, boundary=False)
        Ve = eb().dual_volumes(X, gt, E, mode="edge", n=n, reduce=reduce).cpu().numpy()
        Vm = eb().dual_volumes(X, gt, E, mode="element", reduce=reduce).cpu().numpy()
        assert_vol_close(Ve[used], V0[used], "edge-based V")
        assert_vol_close(Vm[used], V0[used], "element-based V")
        assert np.abs(Ve[~used]).max(initial=0) == 0 and np.abs(Vm[~used]).max(initial=0) == 0


def test_gather_bitwise_reproducible_across_shapes():
    mesh, *_ = case("3d-41")
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    keep = eb().get_gather_shape()
    ref = None
    try:
        for tile in (64, 128, 256):
            for unroll in (1, 2, 4):
                for xcd in (0, 1):
                    say(f"[bitwise] tile={tile} unroll={unroll} xcd={xcd}")
                    eb().set_gather_shape(tile, unroll, xcd)
                    out = [t.cpu().numpy() for t in eb().directed_areas(X, gt, E, "gather")]
                    if ref is None:
                        ref = out
                    for a, r in zip(out, ref):
                        assert np.array_equal(a.view(np.uint64), r.view(np.uint64))
    finally:
        eb().set_gather_shape(*keep)


def test_closure_on_gpu_outputs():
    # sum of n out of every node minus in, plus b, vanishes (Section 3.2.3)
    mesh, ot, *_ = case("3d-scale-33")
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    n, b, V = (t.cpu().numpy() for t in eb().directed_areas(X, gt, E, "gather"))
    a = np.zeros((3, mesh.n_nodes))
    for c in range(3):
        np.add.at(a[c], ot["edge"][0], n[c])
        np.add.at(a[c], ot["edge"][1], -n[c])
        np.add.at(a[c], ot["bnode"], b[c])
    scale = np.abs(n).max()
    assert np.abs(a).max() < 1e-13 * scale
    assert abs(V.sum() - 1.0) < 1e-13


# ------------------------------------------------------------- adjoint

def grad_case(dim, n, seed):
    mesh = meshgen.square_tri(n, seed) if dim == 2 else meshgen.cube_kuhn(n, seed)
    ot = oracle.topology(dim, mesh.coords, mesh.elems)
    w, c, beta = meshgen.loss_weights(seed, dim, ot.n_edges, ot.n_nodes, ot.n_bnodes)
    return mesh, ot, w, c, beta


@pytest.mark.parametrize("reduce", ["atomic", "gather"])
@pytest.mark.parametrize("dim,n", [(2, 17), (3, 9), (3, 21)])
def test_backward_matches_oracle_gradient(dim, n, reduce):
    mesh, ot, w, c, beta = grad_case(dim, n, 1)
    say(f"[backward] dim={dim} n={n} reduce={reduce}")
    _, gref = oracle.node_grad(ot, mesh.coords, mesh.elems, w, c, beta)
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = eb().directed_areas_backward(X, gt, E, T(w), T(beta), T(c), reduce=reduce)
    g = g.cpu().numpy().T
    err = np.linalg.norm(g - gref, axis=1)
    mag = np.linalg.norm(gref, axis=1)
    rel = err / mag
    say(f"    max rel {rel.max():.2e}")
    assert (rel <= GTOL).all()


@pytest.mark.parametrize("reduce", ["atomic", "gather"])
def test_autograd_function(reduce):
    """torch.autograd through EdgeMetrics: the gradient of
    L = sum w.n + sum c V + sum beta.b equals the oracle's reference."""
    mesh, ot, w, c, beta = grad_case(3, 9, 5)
    _, gref = oracle.node_grad(ot, mesh.coords, mesh.elems, w, c, beta)
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    Xg = X.clone().requires_grad_(True)
    n, b, V = eb().EdgeMetrics.apply(Xg, gt, E, reduce)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    L = (T(w) * n).sum() + (T(c) * V).sum() + (T(beta) * b).sum()
    (g,) = torch.autograd.grad(L, Xg)
    g = g.cpu().numpy().T
    rel = np.linalg.norm(g - gref, axis=1) / np.linalg.norm(gref, axis=1)
    assert (rel <= GTOL).all()


def test_backward_volume_only_interior_zero():
    mesh = meshgen.cube_kuhn(9, 3)
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    c = torch.ones(mesh.n_nodes, dtype=torch.float64, device="cuda")
    for reduce in ("atomic", "gather"):
        g = eb().directed_areas_backward(X, gt, E, None, None, c, reduce=reduce).cpu().numpy()
        inner = meshgen._interior_mask_3d(9)
        assert np.abs(g[:, inner]).max() < 1e-14
        assert np.abs(g[:, ~inner]).max() > 1e-4


def test_backward_gather_bitwise_reproducible():
    mesh, ot, w, c, beta = grad_case(3, 21, 4)
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g1 = eb().directed_areas_backward(X, gt, E, T(w), T(beta), T(c), reduce="gather")
    g2 = eb().directed_areas_backward(X, gt, E, T(w), T(beta), T(c), reduce="gather")
    assert torch.equal(g1, g2)


@pytest.fixture(scope="module")
def adjoint81():
    mesh = meshgen.cube_kuhn(81, 0)
    say("[backward-fd] 81^3 oracle topology")
    ot = oracle.topology(3, mesh.coords, mesh.elems)
    return mesh, ot


@pytest.mark.parametrize("reduce", ["atomic", "gather"])
def test_backward_fd_81(adjoint81, reduce):
    """81^3 adjoint config: GPU gradient vs patch-local central differences
    of the oracle's loss on 64 seeded nodes (step 1e-6 h), for both
    reductions (the gather one is what bench.py times and autograd uses)."""
    mesh, ot = adjoint81
    say(f"[backward-fd] 81^3 reduce={reduce}")
    w, c, _ = meshgen.loss_weights(0, 3, ot.n_edges, ot.n_nodes)
    nodes = meshgen.fd_nodes(0, ot.n_nodes, 64)
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = eb().directed_areas_backward(X, gt, E, T(w), None, T(c), reduce=reduce).cpu().numpy()
    _, gref = oracle.node_grad(ot, mesh.coords, mesh.elems, w, c, None, nodes)
    h = 1e-6 / 80
    fd = np.empty((nodes.size, 3))
    for k in range(3):
        for q, j in enumerate(nodes):
            Xp = mesh.coords.copy()
            Xm = mesh.coords.copy()
            Xp[k, j] += h
            Xm[k, j] -= h
            Lp, _ = oracle.node_grad(ot, Xp, mesh.elems, w, c, None, [j])
            Lm, _ = oracle.node_grad(ot, Xm, mesh.elems, w, c, None, [j])
            fd[q, k] = (Lp[0] - Lm[0]) / (2 * h)
    gs = g[:, nodes].T
    rel_fd = np.linalg.norm(gs - fd, axis=1) / np.linalg.norm(fd, axis=1)
    rel_ref = np.linalg.norm(gs - gref, axis=1) / np.linalg.norm(gref, axis=1)
    say(f"    max rel vs FD {rel_fd.max():.2e}, vs dual numbers {rel_ref.max():.2e}")
    assert (rel_fd <= GTOL).all()
    assert (rel_ref <= GTOL).all()


# --------------------------------------------------------------- errors

def test_errors_reported():
    from paper_2502_00778_amd import EbError
    X = torch.tensor([[0., 1, 0, 0, .2, .3], [0, 0, 1, 0, .2, .3], [0, 0, 0, 1, -1, -2]],
                     dtype=torch.float64, device="cuda")
    say("[errors] out of range")
    with pytest.raises(EbError) as e:
        eb().build_edges(torch.tensor([[0, 1, 2, 9]], dtype=torch.int32, device="cuda"), X)
    assert e.value.code == -2
    say("[errors] degenerate")
    Xd = X.clone()
    Xd[:, 3] = torch.tensor([1 / 3, 1 / 3, 0], dtype=torch.float64)
    with pytest.raises(EbError) as e:
        eb().build_edges(torch.tensor([[0, 1, 2, 3]], dtype=torch.int32, device="cuda"), Xd)
    assert e.value.code == -3
    say("[errors] non-manifold")
    with pytest.raises(EbError) as e:
        eb().build_edges(torch.tensor([[0, 1, 2, 3], [0, 1, 2, 4], [0, 2, 1, 5]],
                                      dtype=torch.int32, device="cuda"), X)
    assert e.value.code == -4
    say("[errors] capacity: a node with 1100 out-edges, beyond the plan's slot fields")
    with pytest.raises(EbError) as e:
        Xf, Ef = fan(1100)
        eb().build_edges(torch.from_numpy(Ef).cuda(), torch.from_numpy(Xf).cuda())
    assert e.value.code == -8


def fan(k):
    # node 0 at the centre of k triangles: k higher-numbered neighbours
    ang = np.linspace(0, 2 * np.pi, k, endpoint=False)
    Xf = np.zeros((2, k + 1))
    Xf[:, 1:] = 1 + np.stack([np.cos(ang), np.sin(ang)])
    Xf[:, 0] = 1
    Ef = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)
    return Xf, Ef


@pytest.mark.parametrize("dim", [2, 3])
def test_grid_without_elements(dim):
    """Nodes and no elements: no edges, boundary faces or boundary nodes;
    every V_j is an empty sum (0), and so is every gradient entry."""
    say(f"[empty] dim {dim}: 5 nodes, no elements")
    X = torch.rand(dim, 5, dtype=torch.float64, device="cuda")
    E = torch.zeros((0, dim + 1), dtype=torch.int32, device="cuda")
    t = eb().build_edges(E, X)
    assert (t.n_nodes, t.n_elems, t.n_edges, t.n_bfaces, t.n_bnodes) == (5, 0, 0, 0, 0)
    for reduce in ("gather", "atomic"):
        n, b, V = eb().directed_areas(X, t, E, reduce)
        assert tuple(n.shape) == (dim, 0) and tuple(b.shape) == (dim, 0)
        assert torch.equal(V, torch.zeros_like(V))
        Ve = eb().dual_volumes(X, t, E, "edge", n=n, reduce=reduce)
        assert torch.equal(Ve, torch.zeros_like(Ve))
        Vv = eb().dual_volumes(X, t, E, "element", reduce=reduce)
        assert torch.equal(Vv, torch.zeros_like(Vv))
        g = eb().directed_areas_backward(X, t, E, grad_vol=torch.ones(5, dtype=torch.float64,
                                                                       device="cuda"),
                                         reduce=reduce)
        assert torch.equal(g, torch.zeros_like(g))
    for variant in ("edge_normals", "dual_faces"):
        _, _, V = eb().directed_areas_variant(X, t, E, variant)
        assert torch.equal(V, torch.zeros_like(V))
    res = eb().edge_residual(X, t, E, n, torch.rand(dim, 5, dtype=torch.float64, device="cuda"))
    assert torch.equal(res, torch.zeros_like(res))
    Vn = eb().dual_volumes_noalloc(X, t, n)
    assert torch.equal(Vn, torch.zeros_like(Vn))
    eb().check_errors(t)


def test_high_degree_node_queued():
    """A node beyond the fast kernel's per-node capacities (40 out-edges) is
    handled by the general kernel, and its 40 out-edges select the wide plan
    entries; results match the oracle."""
    Xf, Ef = fan(40)
    mesh = meshgen.Mesh(2, Xf, Ef, "fan40")
    ot = oracle.topology(2, Xf, Ef)
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    assert assert_topo_equal(gt, ot, Ef)["wide"]
    n0, b0, V0 = oracle.metrics(ot, Xf, Ef)
    S_e, S_b = piece_scales(ot, Xf, Ef)
    for reduce in ("gather", "atomic"):
        n, b, V = (t.cpu().numpy() for t in eb().directed_areas(X, gt, E, reduce))
        assert_vec_close(n, n0, S_e, "n")
        assert_vec_close(b, b0, S_b, "b")
        assert_vol_close(V, V0, "V")


# ------------------------------------------------------------ full size

@pytest.fixture(scope="module")
def scale161():
    say("[161^3] generating grid and oracle topology + metrics (CPU)")
    mesh = meshgen.scale_cube(161, 0)
    ot = oracle.topology(3, mesh.coords, mesh.elems)
    say("[161^3] oracle metrics")
    n, b, V = oracle.metrics(ot, mesh.coords, mesh.elems)
    return mesh, ot, n, b, V


def test_full_scale_161(scale161):
    """161^3 stretched grid (24.6M tets), in the launch shape bench.py times:
    topology bit-exact, n/b/V of both reductions against the oracle."""
    mesh, ot, n0, b0, V0 = scale161
    X, E = dev(mesh)
    say("[161^3] GPU build")
    gt = eb().build_edges(E, X)
    say("[161^3] topology and plan checks")
    assert_topo_equal(gt, ot, mesh.elems)
    del gt.arrays["edge_inc"]
    say("[161^3] oracle piece scales")
    S_e, S_b = piece_scales(ot, mesh.coords, mesh.elems)
    for reduce in ("gather", "atomic"):
        say(f"[161^3] directed_areas {reduce}")
        n, b, V = eb().directed_areas(X, gt, E, reduce=reduce)
        eb().check_errors(gt)
        ncan, nrel = assert_vec_close(n.cpu().numpy(), n0, S_e, f"n {reduce}")
        assert_vec_close(b.cpu().numpy(), b0, S_b, f"b {reduce}")
        vrel = assert_vol_close(V.cpu().numpy(), V0, f"V {reduce}")
        say(f"    max rel n {nrel:.2e} (cancelling {ncan}), V {vrel:.2e}")
        Ve = eb().dual_volumes(X, gt, E, mode="edge", n=n, reduce=reduce)
        assert_vol_close(Ve.cpu().numpy(), V0, f"edge V {reduce}")
        del n, b, V, Ve


@pytest.mark.parametrize("name", ["3d-41", "2d-33", "3d-33-relabel", "3d-scale-33", "2d-single",
                                  "3d-single"])
@pytest.mark.parametrize("variant", ["edge_normals", "dual_faces"])
def test_forward_variants_match_oracle(name, variant):
    """The comparison variants (a normal per edge; the traditional dual-face
    construction) give the oracle's n, b, V to the same tolerance."""
    mesh, ot, n0, b0, V0 = case(name)
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    S_e, S_b = piece_scales(ot, mesh.coords, mesh.elems)
    n, b, V = (t.cpu().numpy() for t in eb().directed_areas_variant(X, gt, E, variant))
    eb().check_errors(gt)
    c1, w1 = assert_vec_close(n, n0, S_e, f"n {variant}")
    assert_vec_close(b, b0, S_b, f"b {variant}")
    assert_vol_close(V, V0, f"V {variant}")
    say(f"[variant] {name} {variant}: worst rel n {w1:.2e}")


def test_variant_node_normals_is_directed_areas():
    mesh, *_ = case("3d-41")
    X, E = dev(mesh)
    gt = eb().build_edges(E, X)
    a = eb().directed_areas(X, gt, E, "gather")
    v = eb().directed_areas_variant(X, gt, E, "node_normals")
    for x, y in zip(a, v):
        assert torch.equal(x, y)
