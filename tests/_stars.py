"""Sub-grids for checking sampled outputs of a large grid (test helper).

An edge's lumped vector and a node's volume and boundary normal are sums
over the elements and boundary faces that hold that edge or node (the
general-D formula of Section 3.2.3, the volumes of Section 4.2).  The union
of the stars of some nodes (every element holding one of them) holds all
of those elements, and a face holding a sampled node keeps all of its
holders there, so it is a boundary face of the union exactly when it is
one of the grid.  Renumbering the union's nodes in increasing order keeps
each edge's tail (its smaller node number, Section 2), so the oracle on the
union gives the whole grid's values at the sampled nodes and at every edge
that has one of them as an end.
"""
from __future__ import annotations

import numpy as np

import meshgen


def stars(mesh, nodes):
    """(ids, sub-grid): the elements of ``mesh`` holding any of ``nodes``,
    in their order, over the nodes they use; ``ids[i]`` is the grid's id of
    the sub-grid's node i (ascending)."""
    hold = np.isin(mesh.elems, nodes).any(axis=1)
    ids = np.unique(mesh.elems[hold])
    loc = np.searchsorted(ids, mesh.elems[hold]).astype(np.int32)
    return ids, meshgen.Mesh(mesh.dim, np.ascontiguousarray(mesh.coords[:, ids]),
                             np.ascontiguousarray(loc), mesh.name + "-stars")


def edge_index(edge, n_nodes, tails, heads):
    """Positions of the edges (tails[i], heads[i]) in a lexicographic
    [2, n_edges] edge array (asserted present)."""
    key = edge[0].astype(np.int64) * n_nodes + edge[1]
    want = np.asarray(tails, np.int64) * n_nodes + np.asarray(heads)
    idx = np.searchsorted(key, want)
    assert (idx < key.size).all() and np.array_equal(key[idx], want)
    return idx
