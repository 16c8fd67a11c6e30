"""Pins of the CPU oracle to facts the paper and geometry fix (no GPU).

The oracle forms the median dual (midpoints, centroids) — the traditional
algorithm of Sections 3.1 and 4.  Each test below checks it against something
independent of its own arithmetic:

* hand-worked closed forms on one triangle, two triangles, one tetrahedron and
  the 6-tet cube (derived from the face-normal formulas of Section 3.2);
* the paper's efficient formulas (general-D eq. with the boundary correction,
  Section 4.2's V_E/(D+1), Section 3.2.3's n_B/D) evaluated in exact rational
  arithmetic on small random grids (tests/_exact.py);
* the closure check of Section 3.2.3 at every node, boundary included;
* the sum of the dual volumes equals the domain volume (end of Section 4.3);
* the per-element identity n_jk^E = (n_j^E - n_k^E)/(D(D+1)) that follows
  from eq. njk_local_formula_3d (and eq. njk_E1_2d) with sum_i n_i^E = 0;
* invariances (translation, rotation, scaling, reflection, relabelling);
* closed-form sizes and Euler characteristic of the structured grids, brute
  force on tiny grids, and the paper's printed grid sizes (golden fixture).
"""
from __future__ import annotations

import json
import os
from fractions import Fraction as Fr
from itertools import combinations, permutations

import numpy as np
import pytest

import meshgen
import oracle
from tests import _exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- helpers

def run(dim, X, E):
    X = np.asarray(X, dtype=np.float64)
    E = np.asarray(E, dtype=np.int32)
    t = oracle.topology(dim, X, E)
    n, b, V = oracle.metrics(t, X, E)
    return t, n, b, V


def edge_index(t):
    e = t["edge"]
    return {(int(a), int(c)): i for i, (a, c) in enumerate(zip(e[0], e[1]))}


def closure(t, n, b):
    """a_j = sum_{j->k} n_jk - sum_{k->j} n_kj + b_j (Section 3.2.3)."""
    D = t.dim
    a = np.zeros((D, t.n_nodes))
    for c in range(D):
        np.add.at(a[c], t["edge"][0], n[c])
        np.add.at(a[c], t["edge"][1], -n[c])
        np.add.at(a[c], t["bnode"], b[c])
    return a


def dyadic(mesh, bits=12):
    """Round coordinates to multiples of 2^-bits (exact in float and Fraction)."""
    X = np.round(mesh.coords * 2 ** bits) / 2 ** bits
    return X


def shuffle_local(E, seed):
    rng = np.random.default_rng(seed)
    E = E.copy()
    for i in range(E.shape[0]):
        E[i] = E[i, rng.permutation(E.shape[1])]
    return E


def volume_of(dim, X, E):
    P = X[:, E]  # [D, NE, D+1]
    if dim == 2:
        a = P[:, :, 1] - P[:, :, 0]
        c = P[:, :, 2] - P[:, :, 0]
        return np.abs(a[0] * c[1] - a[1] * c[0]) / 2
    a = P[:, :, 1] - P[:, :, 0]
    c = P[:, :, 2] - P[:, :, 0]
    d = P[:, :, 3] - P[:, :, 0]
    return np.abs(np.einsum("ik,ik->k", a, np.cross(c.T, d.T).T)) / 6


def outward_normals(dim, X, E):
    """n_i^E for each element and local vertex i: [NE, D+1, D] (numpy)."""
    P = np.transpose(X[:, E], (1, 2, 0))  # [NE, D+1, D]
    out = np.empty_like(P)
    for i in range(dim + 1):
        o = [k for k in range(dim + 1) if k != i]
        if dim == 2:
            d = P[:, o[1]] - P[:, o[0]]
            nn = np.stack([d[:, 1], -d[:, 0]], 1)
        else:
            nn = 0.5 * np.cross(P[:, o[1]] - P[:, o[0]], P[:, o[2]] - P[:, o[0]])
        s = np.sign(np.einsum("ij,ij->i", nn, P[:, o[0]] - P[:, i]))
        out[:, i] = nn * s[:, None]
    return out


# --------------------------------------------- hand-worked closed forms

def test_single_triangle_closed_form():
    # nodes (0,0),(1,0),(0,1): outward n_0=(1,1), n_1=(-1,0), n_2=(0,-1);
    # every edge is a boundary edge, so n_jk = n_j/3 + n_B/6 (eq.
    # njk_eff_algorithm_tria_02p5_nB): n_01 = (1/3,1/3) + (0,-1/6)
    t, n, b, V = run(2, [[0, 1, 0], [0, 0, 1]], [[0, 1, 2]])
    ix = edge_index(t)
    assert sorted(ix) == [(0, 1), (0, 2), (1, 2)]
    want = {(0, 1): (1 / 3, 1 / 6), (0, 2): (1 / 6, 1 / 3), (1, 2): (-1 / 6, 1 / 6)}
    for e, v in want.items():
        np.testing.assert_allclose(n[:, ix[e]], v, rtol=0, atol=1e-15)
    np.testing.assert_allclose(V, [1 / 6] * 3, rtol=0, atol=1e-15)
    # b_j = n_B/2 over the two boundary edges at j
    np.testing.assert_allclose(b.T, [[-0.5, -0.5], [0.5, 0], [0, 0.5]], atol=1e-15)
    assert t["bface"].tolist() == [[0, 1], [2, 0], [1, 2]]


def test_two_triangle_square():
    X = [[0, 1, 0, 1], [0, 0, 1, 1]]
    t, n, b, V = run(2, X, [[0, 1, 3], [0, 3, 2]])
    ix = edge_index(t)
    want = {(0, 1): (1 / 3, -1 / 6), (0, 2): (-1 / 6, 1 / 3), (0, 3): (1 / 3, 1 / 3),
            (1, 3): (-1 / 6, 1 / 3), (2, 3): (1 / 3, -1 / 6)}
    for e, v in want.items():
        np.testing.assert_allclose(n[:, ix[e]], v, atol=1e-15)
    np.testing.assert_allclose(V, [1 / 3, 1 / 6, 1 / 6, 1 / 3], atol=1e-15)
    np.testing.assert_allclose(b.T, [[-.5, -.5], [.5, -.5], [-.5, .5], [.5, .5]], atol=1e-15)


def test_single_tet_closed_form():
    # unit right tet: outward n_0 = (1,1,1)/2, n_1 = -e_x/2, n_2 = -e_y/2,
    # n_3 = -e_z/2; |E| = 1/6.  Every edge lies on two boundary faces, so
    # n_jk = n_j/6 + (n_B1 + n_B2)/12 (eq. efficient_njk_3d and the boundary
    # correction eq. njk_boundary_correction_3d with the 1/12 scale)
    X = [[0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]]
    t, n, b, V = run(3, X, [[0, 1, 2, 3]])
    ix = edge_index(t)
    want = {(0, 1): (2, 1, 1), (0, 2): (1, 2, 1), (0, 3): (1, 1, 2),
            (1, 2): (-1, 1, 0), (1, 3): (-1, 0, 1), (2, 3): (0, -1, 1)}
    for e, v in want.items():
        np.testing.assert_allclose(n[:, ix[e]] * 24, v, atol=1e-14)
    np.testing.assert_allclose(V * 24, [1, 1, 1, 1], atol=1e-14)
    np.testing.assert_allclose(b.T * 6, [[-1, -1, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]],
                               atol=1e-14)
    # boundary faces: outward, smallest id first
    assert t["bface"].tolist() == [[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]]


def kuhn_cube_unit():
    X = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], float).T
    step = [1, 2, 4]
    E = [[0, step[a], step[a] + step[b], 7] for (a, b, _) in permutations(range(3))]
    return X, np.array(E)


def test_kuhn_cube_closed_form():
    # 6-tet split of the unit cube along the main diagonal; per tet the
    # outward normals are e_a/2, (e_b-e_a)/2, (e_c-e_b)/2, -e_c/2
    X, E = kuhn_cube_unit()
    t, n, b, V = run(3, X, E)
    assert t.n_edges == 19 and t.n_bfaces == 12 and t.n_bnodes == 8
    ix = edge_index(t)
    F = Fr
    want = {
        (0, 7): (F(1, 6),) * 3,
        (0, 1): (F(1, 6), F(-1, 24), F(-1, 24)), (0, 2): (F(-1, 24), F(1, 6), F(-1, 24)),
        (0, 4): (F(-1, 24), F(-1, 24), F(1, 6)),
        (0, 3): (F(1, 12), F(1, 12), F(-1, 12)), (0, 5): (F(1, 12), F(-1, 12), F(1, 12)),
        (0, 6): (F(-1, 12), F(1, 12), F(1, 12)),
        (1, 3): (F(-1, 24), F(1, 12), F(-1, 24)), (1, 5): (F(-1, 24), F(-1, 24), F(1, 12)),
        (2, 3): (F(1, 12), F(-1, 24), F(-1, 24)), (2, 6): (F(-1, 24), F(-1, 24), F(1, 12)),
        (4, 5): (F(1, 12), F(-1, 24), F(-1, 24)), (4, 6): (F(-1, 24), F(1, 12), F(-1, 24)),
        (1, 7): (F(-1, 12), F(1, 12), F(1, 12)), (2, 7): (F(1, 12), F(-1, 12), F(1, 12)),
        (4, 7): (F(1, 12), F(1, 12), F(-1, 12)),
        (3, 7): (F(-1, 24), F(-1, 24), F(1, 6)), (5, 7): (F(-1, 24), F(1, 6), F(-1, 24)),
        (6, 7): (F(1, 6), F(-1, 24), F(-1, 24)),
    }
    assert set(want) == set(ix)
    for e, v in want.items():
        np.testing.assert_allclose(n[:, ix[e]], [float(x) for x in v], atol=1e-15)
    np.testing.assert_allclose(V, [1 / 4, 1 / 12, 1 / 12, 1 / 12, 1 / 12, 1 / 12, 1 / 12, 1 / 4],
                               atol=1e-15)
    third, sixth = 1 / 3, 1 / 6
    wb = {0: (-third,) * 3, 7: (third,) * 3, 1: (third, -sixth, -sixth),
          2: (-sixth, third, -sixth), 4: (-sixth, -sixth, third),
          3: (sixth, sixth, -third), 5: (sixth, -third, sixth), 6: (-third, sixth, sixth)}
    for node, v in wb.items():
        np.testing.assert_allclose(b[:, list(t["bnode"]).index(node)], v, atol=1e-15)


# -------------------------------- efficient formula, exact rationals

@pytest.mark.parametrize("dim,seed", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_efficient_formula_exact(dim, seed):
    mesh = meshgen.square_tri(6, seed) if dim == 2 else meshgen.cube_kuhn(4, seed)
    X = dyadic(mesh)
    E = shuffle_local(mesh.elems, seed + 17)  # any local order (both orientations)
    t, n, b, V = run(dim, X, E)
    Xl = [tuple(Fr(float(c)) for c in X[:, v]) for v in range(X.shape[1])]
    ex = _exact.exact_metrics(dim, Xl, [tuple(int(v) for v in el) for el in E])
    # topology: brute force
    edges, faces = _exact.brute_topology(dim, [tuple(el) for el in E.tolist()])
    assert [tuple(x) for x in t["edge"].T.tolist()] == edges
    assert sorted(tuple(sorted(f)) for f in t["bface"].tolist()) == sorted(ex["bfaces"])
    ix = edge_index(t)
    for e, v in ex["n"].items():
        ref = np.array([float(x) for x in v])
        assert np.linalg.norm(n[:, ix[e]] - ref) <= 1e-14 * max(np.linalg.norm(ref), 1e-3)
    for j, v in ex["V"].items():
        assert abs(V[j] - float(v)) <= 1e-14 * float(v)
    bl = list(t["bnode"])
    assert sorted(ex["b"]) == bl
    for j, v in ex["b"].items():
        ref = np.array([float(x) for x in v])
        assert np.linalg.norm(b[:, bl.index(j)] - ref) <= 1e-14 * np.linalg.norm(ref)
    # outward order of each boundary face matches the exact outward normal
    for f in t["bface"]:
        key = tuple(sorted(int(x) for x in f))
        P = [np.array([float(c) for c in Xl[v]]) for v in f]
        if dim == 2:
            d = P[1] - P[0]
            nb = np.array([d[1], -d[0]])
        else:
            nb = 0.5 * np.cross(P[1] - P[0], P[2] - P[0])
        ref = np.array([float(x) for x in ex["bfaces"][key]])
        np.testing.assert_allclose(nb, ref, atol=1e-15)


def _brute_csrs(dim, nv, elems, X):
    """Every topology array written out from its definition with plain loops
    on a tiny grid: the edge array and element->edge map (Section 2), the
    incidence lists, the in-edge lists, and the boundary elements
    (Section 3.2: faces met by one element) with their outward vertex order,
    owners, edge ids and boundary-node lists."""
    nn, pairs = dim + 1, list(combinations(range(dim + 1), 2))
    edges = sorted({tuple(sorted((el[p], el[q]))) for el in elems for p, q in pairs})
    eid = {e: i for i, e in enumerate(edges)}
    out = {}
    out["edge"] = [[a for a, _ in edges], [b for _, b in edges]]
    out["node_edge_off"] = [sum(1 for a, _ in edges if a < j) for j in range(nv + 1)]
    out["elem_edge"] = [[eid[tuple(sorted((el[p], el[q])))] for p, q in pairs] for el in elems]
    out["elem_edge_sign"] = [[1 if el[p] < el[q] else -1 for p, q in pairs] for el in elems]
    inc = [[i * len(pairs) + le for i, el in enumerate(elems) for le, (p, q) in enumerate(pairs)
            if tuple(sorted((el[p], el[q]))) == e] for e in edges]
    node_inc = [[i * nn + l for i, el in enumerate(elems) for l in range(nn) if el[l] == j]
                for j in range(nv)]
    node_in = [[i for i, (_, b) in enumerate(edges) if b == j] for j in range(nv)]
    for name, rows in (("edge_inc", inc), ("node_inc", node_inc), ("node_in", node_in)):
        off = [0]
        for r in rows:
            off.append(off[-1] + len(r))
        out[name + "_off"] = off
        out[name if name != "node_in" else "node_in_edge"] = [x for r in rows for x in r]
    faces = {}
    for i, el in enumerate(elems):
        for f in range(nn):
            faces.setdefault(tuple(sorted(el[m] for m in range(nn) if m != f)), []).append((i, f))
    bkeys = sorted(k for k, v in faces.items() if len(v) == 1)
    bface, owner = [], []
    for k in bkeys:
        (i, f), = faces[k]
        P = X[:, list(k)].T
        xo = X[:, elems[i][f]]
        if dim == 2:
            d = P[1] - P[0]
            out_ok = d[1] * (P[0][0] - xo[0]) - d[0] * (P[0][1] - xo[1]) > 0
            v = list(k) if out_ok else [k[1], k[0]]
        elif dim == 3:
            c = np.cross(P[1] - P[0], P[2] - P[0])
            v = list(k) if c @ (P[0] - xo) > 0 else [k[0], k[2], k[1]]
        else:  # the sign of det[a - xo; b - a; c - a; d - a]
            s4 = np.linalg.det(np.stack([P[0] - xo, P[1] - P[0], P[2] - P[0], P[3] - P[0]]))
            v = list(k) if s4 > 0 else [k[0], k[1], k[3], k[2]]
        bface.append(v)
        owner.append(i * nn + f)
    out["bface"], out["bface_owner"] = bface, owner
    fp = [(0, 1)] if dim == 2 else list(combinations(range(dim), 2))
    out["bface_edge"] = [[eid[tuple(sorted((f[p], f[q])))] for p, q in fp] for f in bface]
    bnode = sorted({v for f in bface for v in f})
    out["bnode"] = bnode
    out["node_bnode"] = [bnode.index(j) if j in bnode else -1 for j in range(nv)]
    bf = [[fi for fi, f in enumerate(bface) if j in f] for j in bnode]
    out["bnode_face_off"] = [0] + list(np.cumsum([len(r) for r in bf]))
    out["bnode_face"] = [x for r in bf for x in r]
    return out


def _fan(k):
    ang = np.linspace(0, 2 * np.pi, k, endpoint=False)
    X = np.zeros((2, k + 1))
    X[:, 1:] = np.stack([np.cos(ang), np.sin(ang)])
    return X, np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)


@pytest.mark.parametrize("case", ["3d-kuhn-shuf", "2d-tri-shuf", "2d-fan", "3d-relabel",
                                  "4d-kuhn-shuf"])
def test_topology_arrays_brute(case):
    """Every array the oracle's sort-based topology produces, bface_edge and
    the in-edge lists included, equals the plain-loop statement of its
    definition on tiny grids (shuffled local orders, relabelled ids, a node
    of high degree)."""
    if case == "3d-kuhn-shuf":
        m = meshgen.cube_kuhn(3, 1)
        dim, X, E = 3, m.coords, shuffle_local(m.elems, 3)
    elif case == "2d-tri-shuf":
        m = meshgen.square_tri(4, 2)
        dim, X, E = 2, m.coords, shuffle_local(m.elems, 5)
    elif case == "2d-fan":
        dim, (X, E) = 2, _fan(9)
    elif case == "4d-kuhn-shuf":
        m = meshgen.hypercube_kuhn(3, 1)
        dim, X, E = 4, m.coords, shuffle_local(m.elems, 6)
    else:
        m = meshgen.cube_kuhn(3, 0)
        lab = np.random.default_rng(4).permutation(m.n_nodes)
        X = np.empty_like(m.coords)
        X[:, lab] = m.coords
        dim, E = 3, lab[m.elems].astype(np.int32)
    t = oracle.topology(dim, X, E)
    want = _brute_csrs(dim, X.shape[1], E.tolist(), X)
    for name, ref in want.items():
        got = np.asarray(t[name]).reshape(-1)
        assert got.tolist() == np.asarray(ref, dtype=np.int64).reshape(-1).tolist(), name


def test_local_identity_fe_form():
    # per element: traditional piece of edge (j,k) == (n_j - n_k)/(D(D+1))
    for dim, mesh in [(2, meshgen.square_tri(9, 3)), (3, meshgen.cube_kuhn(6, 3))]:
        E = shuffle_local(mesh.elems, 5)
        npc, vpc = oracle.element_pieces(dim, mesh.coords, E)
        nrm = outward_normals(dim, mesh.coords, E)
        pairs = [(0, 1), (0, 2), (1, 2)] if dim == 2 else \
            [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
        for le, (p, q) in enumerate(pairs):
            tail_is_p = E[:, p] < E[:, q]
            j = np.where(tail_is_p, p, q)
            k = np.where(tail_is_p, q, p)
            r = np.arange(E.shape[0])
            ref = (nrm[r, j] - nrm[r, k]) / (dim * (dim + 1))
            err = np.abs(npc[:, le] - ref).max()
            assert err < 1e-15 * 10, err
        vol = volume_of(dim, mesh.coords, E)
        np.testing.assert_allclose(vpc, np.repeat(vol[:, None] / (dim + 1), dim + 1, 1),
                                   rtol=1e-13)


# ------------------------------------------------ closure and volume sum

@pytest.mark.parametrize("cfg", ["2d", "3d", "small-scale"])
def test_closure_and_volume_sum(cfg):
    if cfg == "small-scale":
        # the stretched-wall recipe at n=21 (first spacing 1e-2: a 1e-5 first
        # spacing cannot reach a uniform spacing within 20 cells)
        mesh = meshgen.scale_cube(21, 0, first=1e-2)
    else:
        mesh = meshgen.make(cfg, 0)
    t, n, b, V = run(mesh.dim, mesh.coords, mesh.elems)
    a = closure(t, n, b)
    # scale: the largest edge normal magnitude touching each node
    mag = np.zeros(t.n_nodes)
    nn = np.linalg.norm(n, axis=0)
    np.maximum.at(mag, t["edge"][0], nn)
    np.maximum.at(mag, t["edge"][1], nn)
    assert (np.linalg.norm(a, axis=0) <= 1e-13 * mag).all()
    assert abs(V.sum() - 1.0) < 1e-13
    assert (V > 0).all()
    # closed boundary: the boundary normals sum to zero; unit box faces give
    # +-1 per axis (only the face x_a = 1 has +e_a, only x_a = 0 has -e_a)
    np.testing.assert_allclose(b.sum(1), 0, atol=1e-13)
    for c in range(mesh.dim):
        assert abs(np.clip(b[c], 0, None).sum() - 1) < 1e-13
        assert abs(np.clip(b[c], None, 0).sum() + 1) < 1e-13


def test_unjittered_interior_volumes():
    n3 = 6
    m = meshgen.cube_kuhn(n3, jitter=0)
    t, n, b, V = run(3, m.coords, m.elems)
    h = 1 / (n3 - 1)
    inner = meshgen._interior_mask_3d(n3)
    # 24 tets of volume h^3/6 meet at an interior Kuhn node, each gives 1/4
    np.testing.assert_allclose(V[inner], h ** 3, rtol=1e-13)
    m2 = meshgen.square_tri(7, jitter=0)
    t2, n2, b2, V2 = run(2, m2.coords, m2.elems)
    h2 = 1 / 6
    cnt = np.bincount(m2.elems.reshape(-1), minlength=m2.n_nodes)
    np.testing.assert_allclose(V2, cnt * h2 * h2 / 6, rtol=1e-13)


# ------------------------------------------------------------ invariances

@pytest.mark.parametrize("dim", [2, 3])
def test_invariances(dim):
    mesh = meshgen.square_tri(8, 4) if dim == 2 else meshgen.cube_kuhn(5, 4)
    X, E = mesh.coords, mesh.elems
    t, n, b, V = run(dim, X, E)
    rng = np.random.default_rng(11)
    # translation
    _, n1, b1, V1 = run(dim, X + rng.normal(size=(dim, 1)), E)
    np.testing.assert_allclose(n1, n, atol=1e-13 * np.abs(n).max())
    np.testing.assert_allclose(V1, V, rtol=1e-11)
    # rotation: n, b rotate, V invariant
    Q, _ = np.linalg.qr(rng.normal(size=(dim, dim)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    _, n2, b2, V2 = run(dim, Q @ X, E)
    np.testing.assert_allclose(n2, Q @ n, atol=1e-13 * np.abs(n).max())
    np.testing.assert_allclose(b2, Q @ b, atol=1e-13 * np.abs(b).max())
    np.testing.assert_allclose(V2, V, rtol=1e-12)
    # scaling: n ~ s^(D-1), V ~ s^D
    s = 2.5
    _, n3, b3, V3 = run(dim, s * X, E)
    np.testing.assert_allclose(n3, s ** (dim - 1) * n, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(V3, s ** dim * V, rtol=1e-12)
    # reflection x -> -x flips every element's orientation; outputs mirror
    R = np.eye(dim)
    R[0, 0] = -1
    _, n4, b4, V4 = run(dim, R @ X, E)
    np.testing.assert_allclose(n4, R @ n, atol=1e-13 * np.abs(n).max())
    np.testing.assert_allclose(V4, V, rtol=1e-12)
    # element order and local vertex order do not matter
    perm = rng.permutation(E.shape[0])
    E5 = shuffle_local(E[perm], 3)
    _, n5, b5, V5 = run(dim, X, E5)
    np.testing.assert_allclose(n5, n, atol=1e-13 * np.abs(n).max())
    np.testing.assert_allclose(V5, V, rtol=1e-12)
    np.testing.assert_allclose(b5, b, atol=1e-13 * np.abs(b).max())
    # node relabelling: n flips exactly on edges whose orientation flips
    lab = rng.permutation(X.shape[1]).astype(np.int32)
    inv = np.argsort(lab)
    X6 = X[:, inv]  # node lab[v] sits where v was
    E6 = lab[E]
    t6, n6, b6, V6 = run(dim, X6, E6)
    ix6 = edge_index(t6)
    for i, (a, c) in enumerate(zip(t["edge"][0], t["edge"][1])):
        la, lc = int(lab[a]), int(lab[c])
        sgn = 1 if la < lc else -1
        k = ix6[(min(la, lc), max(la, lc))]
        np.testing.assert_allclose(n6[:, k], sgn * n[:, i], atol=1e-13 * np.abs(n).max())
    np.testing.assert_allclose(V6[lab], V, rtol=1e-12)


# --------------------------------------------------------------- topology

@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_kuhn_counts_and_euler(n):
    m = meshgen.cube_kuhn(n, 0)
    t = oracle.topology(3, m.coords, m.elems)
    cnt = meshgen.kuhn_counts(n)
    assert (t.n_nodes, t.n_elems, t.n_edges, t.n_bfaces, t.n_bnodes) == (
        cnt["n_nodes"], cnt["n_elems"], cnt["n_edges"], cnt["n_bfaces"], cnt["n_bnodes"])
    n_faces = (4 * t.n_elems + t.n_bfaces) // 2
    assert t.n_nodes - t.n_edges + n_faces - t.n_elems == 1
    assert t["edge_inc_off"][-1] == 6 * t.n_elems
    assert t["node_inc_off"][-1] == 4 * t.n_elems
    assert t["node_edge_off"][-1] == t.n_edges
    assert t["bnode_face_off"][-1] == 3 * t.n_bfaces
    assert (np.diff(t["edge_inc_off"]) > 0).all()
    # element -> edge map is consistent with the edge list
    E = m.elems
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for le, (p, q) in enumerate(pairs):
        ee = t["elem_edge"][:, le]
        assert (t["edge"][0][ee] == np.minimum(E[:, p], E[:, q])).all()
        assert (t["edge"][1][ee] == np.maximum(E[:, p], E[:, q])).all()
        assert (t["elem_edge_sign"][:, le] == np.where(E[:, p] < E[:, q], 1, -1)).all()


@pytest.mark.parametrize("n", [2, 5, 33])
def test_tri_counts_and_euler(n):
    m = meshgen.square_tri(n, 1)
    t = oracle.topology(2, m.coords, m.elems)
    cnt = meshgen.tri_counts(n)
    assert (t.n_nodes, t.n_elems, t.n_edges, t.n_bfaces, t.n_bnodes) == (
        cnt["n_nodes"], cnt["n_elems"], cnt["n_edges"], cnt["n_bfaces"], cnt["n_bnodes"])
    assert t.n_nodes - t.n_edges + t.n_elems == 1


def test_paper_grid_sizes():
    """The paper's triangular grid: 65,536 nodes and 130,050 triangles."""
    g = json.load(open(os.path.join(GOLDEN, "paper_grid_sizes.json")))
    tri = g["triangular_unit_square"]
    m = meshgen.square_tri(256, 0)
    assert (m.n_nodes, m.n_elems) == (tri["n_nodes"], tri["n_elems"])
    t = oracle.topology(2, m.coords, m.elems)
    assert t.n_nodes - t.n_edges + t.n_elems == 1
    tet = g["tetrahedral_unit_cube"]
    cnt = meshgen.kuhn_counts(257)
    assert (cnt["n_nodes"], cnt["n_elems"]) == (tet["n_nodes"], tet["n_elems"])


def test_brute_topology_tiny():
    for dim, mesh in [(2, meshgen.square_tri(4, 2)), (3, meshgen.cube_kuhn(3, 2))]:
        E = shuffle_local(mesh.elems, 9)
        t = oracle.topology(dim, mesh.coords, E)
        edges, faces = _exact.brute_topology(dim, [tuple(el) for el in E.tolist()])
        assert [tuple(x) for x in t["edge"].T.tolist()] == edges
        bkeys = sorted(k for k, v in faces.items() if len(v) == 1)
        assert [tuple(sorted(f)) for f in t["bface"].tolist()] == bkeys
        owners = [faces[k][0] for k in bkeys]
        assert t["bface_owner"].tolist() == [e * (dim + 1) + f for e, f in owners]
        if dim == 3:
            assert all(f[0] == min(f) for f in t["bface"].tolist())


# ----------------------------------------------------------------- errors

def test_errors():
    X = np.array([[0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]], float)
    with pytest.raises(oracle.OracleError) as e:
        oracle.topology(3, X, np.array([[0, 1, 2, 4]]))
    assert e.value.code == -2
    Xd = X.copy()
    Xd[:, 3] = [1 / 3, 1 / 3, 0]  # flat
    with pytest.raises(oracle.OracleError) as e:
        oracle.topology(3, Xd, np.array([[0, 1, 2, 3]]))
    assert e.value.code == -3
    X5 = np.concatenate([X, [[0.2], [0.2], [-1.0]], [[0.3], [0.3], [-2.0]]], 1)
    E = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 2, 1, 5]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.topology(3, X5, E)
    assert e.value.code == -4
    with pytest.raises(oracle.OracleError) as e:
        oracle.topology(5, X, np.array([[0, 1, 2, 3, 0, 1]]))
    assert e.value.code == -1


# --------------------------------------------------- reference gradient

def _loss_setup(dim, n, seed):
    mesh = meshgen.square_tri(n, seed) if dim == 2 else meshgen.cube_kuhn(n, seed)
    t = oracle.topology(dim, mesh.coords, mesh.elems)
    w, c, beta = meshgen.loss_weights(seed, dim, t.n_edges, t.n_nodes, t.n_bnodes)
    return mesh, t, w, c, beta


@pytest.mark.parametrize("dim", [2, 3])
def test_grad_matches_patch_fd(dim):
    mesh, t, w, c, beta = _loss_setup(dim, 7 if dim == 2 else 5, 2)
    nodes = meshgen.fd_nodes(2, t.n_nodes, 12)
    L0, g = oracle.node_grad(t, mesh.coords, mesh.elems, w, c, beta, nodes)
    h = 1e-6 / 4
    for q, j in enumerate(nodes):
        fd = np.empty(dim)
        for k in range(dim):
            Xp = mesh.coords.copy()
            Xm = mesh.coords.copy()
            Xp[k, j] += h
            Xm[k, j] -= h
            Lp, _ = oracle.node_grad(t, Xp, mesh.elems, w, c, beta, [j])
            Lm, _ = oracle.node_grad(t, Xm, mesh.elems, w, c, beta, [j])
            fd[k] = (Lp[0] - Lm[0]) / (2 * h)
        assert np.linalg.norm(fd - g[q]) <= 1e-7 * np.linalg.norm(g[q]) + 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_grad_identities(dim):
    """Exact consequences of invariance for L = w.n + c.V + beta.b:
    translation: sum_j g_j = 0; rotation: sum_j x_j x g_j = sum_e n_e x w_e +
    sum_i b_i x beta_i; homogeneity (n, b of degree D-1, V of degree D):
    sum_j x_j.g_j = (D-1)(w.n + beta.b) + D c.V."""
    mesh, t, w, c, beta = _loss_setup(dim, 8 if dim == 2 else 5, 3)
    X = mesh.coords
    _, g = oracle.node_grad(t, X, mesh.elems, w, c, beta)
    n, b, V = oracle.metrics(t, X, mesh.elems)
    scale = np.abs(g).sum()
    np.testing.assert_allclose(g.sum(0), 0, atol=1e-13 * scale)
    if dim == 3:
        lhs = np.cross(X.T, g).sum(0)
        rhs = np.cross(n.T, w.T).sum(0) + np.cross(b.T, beta.T).sum(0)
    else:
        lhs = (X[0] * g[:, 1] - X[1] * g[:, 0]).sum()
        rhs = (n[0] * w[1] - n[1] * w[0]).sum() + (b[0] * beta[1] - b[1] * beta[0]).sum()
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * scale)
    lhs = (X.T * g).sum()
    rhs = (dim - 1) * ((w * n).sum() + (beta * b).sum()) + dim * (c * V).sum()
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_grad_volume_interior_zero():
    # total volume depends on the boundary only: with w = 0 and c = 1 the
    # gradient vanishes at every interior node
    mesh = meshgen.cube_kuhn(5, 6)
    t = oracle.topology(3, mesh.coords, mesh.elems)
    _, g = oracle.node_grad(t, mesh.coords, mesh.elems, None, np.ones(t.n_nodes), None)
    inner = meshgen._interior_mask_3d(5)
    assert np.abs(g[inner]).max() < 1e-15
    assert np.abs(g[~inner]).max() > 1e-3


# ------------------------------------------------ four dimensions (D = 4)
#
# The paper derives the efficient formula for general D (Section 3.2.3) and
# leaves D = 4 to future work; it gives no 4D value to compare with.  The
# oracle's 4D construction (barycentric subdivision of each pentatope) is
# pinned here by what the geometry fixes: a hand-worked single pentatope,
# the finite-element identity per element, closure at every node, the total
# volume and boundary area of the unit 4-cube, unjittered interior volumes,
# closed-form counts, Euler's relation and brute-force topology.

def _face_normals_4d(P):
    """Outward area vectors n_i of the faces of pentatopes P [NE, 5, 4]
    (numpy, independent of the oracle): (1/6) N(b-a, c-a, d-a) of the face
    opposite i, with N(u,v,w).x = det[x; u; v; w], oriented away from
    vertex i."""
    NE = P.shape[0]
    n = np.empty((NE, 5, 4))
    eye = np.eye(4)
    for i in range(5):
        o = [r for r in range(5) if r != i]
        u, v, w = (P[:, o[k]] - P[:, o[0]] for k in (1, 2, 3))
        N = np.stack([np.linalg.det(np.stack([np.broadcast_to(eye[c], u.shape), u, v, w], axis=1))
                      for c in range(4)], axis=1) / 6.0
        sgn = np.sign(np.einsum("ec,ec->e", N, P[:, o[0]] - P[:, i]))
        n[:, i] = N * sgn[:, None]
    return n


def test_4d_single_pentatope_closed_form():
    """Unit pentatope {0, e1, e2, e3, e4}: outward face vectors n_0 =
    (1,1,1,1)/6, n_i = -e_i/6; every face is a boundary face, so the edge
    (j,k), j < k, gets n_j/10 from the element and -(n_j + n_k)/20 from the
    three boundary faces holding it: (n_j - n_k)/20; V_i = (1/24)/5; b_j =
    (1/4) sum of the four faces at j = -n_j/4.  Any local order."""
    X = np.concatenate([np.zeros((4, 1)), np.eye(4)], axis=1)
    nf = np.concatenate([np.full((4, 1), 1 / 6), -np.eye(4) / 6], axis=1)  # [4, 5]
    for perm in ([0, 1, 2, 3, 4], [3, 0, 4, 2, 1], [1, 0, 2, 3, 4]):
        E = np.array([perm], np.int32)
        t, n, b, V = run(4, X, E)
        assert t.n_edges == 10 and t.n_bfaces == 5 and t.n_bnodes == 5
        for e in range(10):
            j, k = t["edge"][:, e]
            np.testing.assert_allclose(n[:, e], (nf[:, j] - nf[:, k]) / 20, atol=1e-16)
        np.testing.assert_allclose(V, np.full(5, 1 / 120), rtol=1e-14)
        np.testing.assert_allclose(b[:, t["node_bnode"]], -nf / 4, atol=1e-16)


def test_4d_fe_identity_per_element():
    """Each element's dual-face pieces equal (n_j^E - n_k^E)/20 (tail j) and
    each vertex's sub-cell |E|/5, with n^E and |E| from numpy determinants."""
    m = meshgen.hypercube_kuhn(4, 2)
    E = shuffle_local(m.elems, 11)
    npc, vpc = oracle.element_pieces(4, m.coords, E)
    P = m.coords.T[E]  # [NE, 5, 4]
    nf = _face_normals_4d(P)
    vol = np.abs(np.linalg.det(P[:, 1:] - P[:, :1])) / 24.0
    pairs = list(combinations(range(5), 2))
    for le, (p, q) in enumerate(pairs):
        tail_p = E[:, p] < E[:, q]
        ref = np.where(tail_p[:, None], nf[:, p] - nf[:, q], nf[:, q] - nf[:, p]) / 20.0
        np.testing.assert_allclose(npc[:, le], ref, atol=1e-15 * np.abs(ref).max())
    np.testing.assert_allclose(vpc, np.repeat(vol[:, None] / 5, 5, axis=1), rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_4d_closure_volume_boundary(seed):
    """Jittered 4-cube: closure at every node (Section 3.2.3), total volume
    1, and per axis the boundary normals' positive parts sum to the area 1
    of the facet x_a = 1 and their negative parts to -1."""
    m = meshgen.hypercube_kuhn(5, seed)
    t, n, b, V = run(4, m.coords, m.elems)
    a = closure(t, n, b)
    assert np.abs(a).max() < 1e-15
    assert abs(V.sum() - 1.0) < 1e-14
    for ax in range(4):
        assert abs(np.clip(b[ax], 0, None).sum() - 1.0) < 1e-14
        assert abs(np.clip(b[ax], None, 0).sum() + 1.0) < 1e-14


def test_4d_unjittered_interior_volume():
    """Unjittered grid: every interior node's dual cell is one cell, h^4."""
    n = 5
    m = meshgen.hypercube_kuhn(n, 0, jitter=0.0)
    t, _, _, V = run(4, m.coords, m.elems)
    a = np.arange(n)
    l, k, j, i = np.meshgrid(a, a, a, a, indexing="ij")
    inner = ((i > 0) & (i < n - 1) & (j > 0) & (j < n - 1) & (k > 0) & (k < n - 1)
             & (l > 0) & (l < n - 1)).reshape(-1)
    np.testing.assert_allclose(V[inner], (1 / (n - 1)) ** 4, rtol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_4d_counts_and_euler(n):
    """Closed-form counts of the split, and V - E + F - T + P = 1 for the
    4-ball (triangles and tetrahedra counted by brute force)."""
    m = meshgen.hypercube_kuhn(n, 0)
    t = oracle.topology(4, m.coords, m.elems)
    cnt = meshgen.kuhn4_counts(n)
    assert (t.n_nodes, t.n_elems, t.n_edges, t.n_bfaces, t.n_bnodes) == (
        cnt["n_nodes"], cnt["n_elems"], cnt["n_edges"], cnt["n_bfaces"], cnt["n_bnodes"])
    tris = {tuple(sorted(c)) for el in m.elems.tolist() for c in combinations(el, 3)}
    tets = {tuple(sorted(c)) for el in m.elems.tolist() for c in combinations(el, 4)}
    assert t.n_nodes - t.n_edges + len(tris) - len(tets) + t.n_elems == 1
    assert len(tets) == (5 * t.n_elems + t.n_bfaces) // 2


@pytest.mark.parametrize("dim", [3, 4])
def test_star_union_gives_the_grids_values(dim):
    """Locality of the formulas (Section 3.2.3): the oracle on the union of
    some nodes' stars gives the whole grid's n at every edge with such a
    node as an end, and its V and b at those nodes; at other edges of the
    union the values differ (their elements are not all there)."""
    from tests._stars import edge_index, stars
    m = meshgen.hypercube_kuhn(7, 3) if dim == 4 else meshgen.cube_kuhn(9, 3)
    t = oracle.topology(dim, m.coords, m.elems)
    n0, b0, V0 = oracle.metrics(t, m.coords, m.elems)
    rng = np.random.default_rng(11)
    nodes = np.unique(np.concatenate([[0, m.n_nodes - 1],
                                      rng.choice(m.n_nodes, 30, replace=False)]))
    ids, sm = stars(m, nodes)
    st = oracle.topology(dim, sm.coords, sm.elems)
    n1, b1, V1 = oracle.metrics(st, sm.coords, sm.elems)
    ge = ids[st["edge"]]
    idx = edge_index(t["edge"], m.n_nodes, ge[0], ge[1])
    mine = np.isin(ge, nodes).any(axis=0)
    scale = np.abs(n0).max()
    np.testing.assert_allclose(n1[:, mine], n0[:, idx[mine]], rtol=1e-13, atol=1e-15 * scale)
    assert np.abs(n1[:, ~mine] - n0[:, idx[~mine]]).max() > 1e-6 * scale
    np.testing.assert_allclose(V1[np.searchsorted(ids, nodes)], V0[nodes], rtol=1e-13)
    gb = ids[st["bnode"]]
    kb = np.isin(gb, nodes)
    assert kb.sum() >= 2  # the grid's first and last nodes are corners
    np.testing.assert_allclose(b1[:, kb], b0[:, t["node_bnode"][gb[kb]]], rtol=1e-13,
                               atol=1e-15 * np.abs(b0).max())
