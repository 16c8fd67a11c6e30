"""Exact-rational evaluation of the paper's efficient formulas (test helper).

This is NOT the oracle: it evaluates the formulas the paper derives for the
lumped directed-area vectors and dual volumes *without* forming the dual, in
``fractions.Fraction`` arithmetic, with a brute-force topology.  The oracle
forms the dual (midpoints and centroids); the paper proves the two agree, so
agreement pins the oracle's construction.

  n_jk = 2/(D(D+1)) * sum_{E containing jk} n_j^E            (general-D eq.)
       + 1/(D(D+1)) * sum_{boundary elements B containing jk} n_B
  V_j  = sum_{E containing j} |E| / (D+1)                    (Section 4.2)
  b_j  = 1/D * sum_{B containing j} n_B                       (Section 3.2.3)

n_j^E is the outward area vector of the face of E opposite j and j is the
smaller node number of the edge (the tail, Section 2).
"""
from __future__ import annotations

from fractions import Fraction as Fr
from itertools import combinations


def _sub(a, b):
    return tuple(x - y for x, y in zip(a, b))


def _dot(a, b):
    return sum(x * y for x, y in zip(a, b))


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0])


def face_normal(dim, pts, inner):
    """Outward area vector of the face through ``pts`` seen from ``inner``."""
    if dim == 2:
        d = _sub(pts[1], pts[0])
        n = (d[1], -d[0])
    else:
        c = _cross(_sub(pts[1], pts[0]), _sub(pts[2], pts[0]))
        n = tuple(Fr(1, 2) * x for x in c)
    s = _dot(n, _sub(pts[0], inner))
    assert s != 0
    return n if s > 0 else tuple(-x for x in n)


def measure(dim, pts):
    if dim == 2:
        a, b = _sub(pts[1], pts[0]), _sub(pts[2], pts[0])
        return abs(a[0] * b[1] - a[1] * b[0]) / 2
    a, b, c = (_sub(p, pts[0]) for p in pts[1:])
    return abs(_dot(a, _cross(b, c))) / 6


def exact_metrics(dim, X, elems):
    """X: list of coordinate tuples (Fractions/ints); elems: list of tuples.

    Returns dict edge -> n (tuple), node -> V, boundary node -> b, plus the
    brute-force edge list, boundary-face dict and face counts.
    """
    D = dim
    kn = Fr(2, D * (D + 1))
    kb = Fr(1, D * (D + 1))
    zero = tuple(Fr(0) for _ in range(D))
    n, V, b = {}, {}, {}
    faces = {}
    for ei, el in enumerate(elems):
        pts = [tuple(Fr(c) for c in X[v]) for v in el]
        vol = measure(D, pts)
        for li, v in enumerate(el):
            V[v] = V.get(v, Fr(0)) + vol / (D + 1)
        for (p, q) in combinations(range(D + 1), 2):
            j, k = sorted((el[p], el[q]))
            lj = el.index(j)
            others = [pts[i] for i in range(D + 1) if i != lj]
            nj = face_normal(D, others, pts[lj])
            cur = n.get((j, k), zero)
            n[(j, k)] = tuple(c + kn * x for c, x in zip(cur, nj))
        for f in range(D + 1):
            key = tuple(sorted(el[i] for i in range(D + 1) if i != f))
            faces.setdefault(key, []).append((ei, f))
    bfaces = {}
    for key, owners in faces.items():
        assert len(owners) <= 2, "non-manifold"
        if len(owners) == 1:
            ei, f = owners[0]
            el = elems[ei]
            pts = [tuple(Fr(c) for c in X[v]) for v in key]
            inner = tuple(Fr(c) for c in X[el[f]])
            nB = face_normal(D, pts, inner)
            bfaces[key] = nB
            for (a, c) in combinations(key, 2):
                cur = n[(a, c)]
                n[(a, c)] = tuple(x + kb * y for x, y in zip(cur, nB))
            for v in key:
                cur = b.get(v, zero)
                b[v] = tuple(x + Fr(1, D) * y for x, y in zip(cur, nB))
    return dict(n=n, V=V, b=b, bfaces=bfaces, faces=faces)


def brute_topology(dim, elems):
    edges = sorted({tuple(sorted((el[p], el[q])))
                    for el in elems for p, q in combinations(range(dim + 1), 2)})
    faces = {}
    for ei, el in enumerate(elems):
        for f in range(dim + 1):
            key = tuple(sorted(el[i] for i in range(dim + 1) if i != f))
            faces.setdefault(key, []).append((ei, f))
    return edges, faces
