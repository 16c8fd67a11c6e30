"""Checks of the GPU library's kernel plan against the oracle's topology.

The plan (eb_topology.plan) is the library's private per-node view of the
incidences; its encoding is stated in the library source (csrc/eb_plan.h)
and nothing the paper defines.  These checks decode it (via
eb_plan_describe) and verify, for every node j, properties that make it a
faithful view of the topology the oracle computes from the paper's
definitions, without re-deriving the library's choices:

* each 64-node slice is as long as its longest node_inc row; slots past a
  node's row hold zeros;
* node j's entries are a permutation of its incidences: the sets of other
  vertices agree as multisets (compared by two independent 64-bit hashes);
* each entry's out-edge slot of vertex o is the position of edge (j, o)
  among j's out-edges, or the all-ones field when o < j;
* rows of at most 32 entries: the first entry is the row's smallest
  incidence with its vertices in local order; a vertex shared with the
  previous entry keeps its place; an entry shares fewer than D-1 vertices
  with the previous one only if no later entry of the row shares D-1;
* longer rows: the entries are the incidences in ascending order, local
  vertex order;
* step words (narrow entries always; wide ones exactly when every offset
  fits 20 bits and no node has more than 31 out-edges): reproduce entry c
  from entry c-1 (one changed place: its new vertex, place and slot; else
  the flag word);
* each incidence's slot is its rank in node j's node_inc row.
"""
from __future__ import annotations

import numpy as np


def _local_others(elems, inc, D):
    e, l = inc // (D + 1), inc % (D + 1)
    o = elems[e][:, :D].astype(np.int64).copy()
    last = elems[e, D].astype(np.int64)
    for m in range(D):
        sel = l == m
        o[sel, m] = last[sel]
    return o


def _hash_rows(a, salt):
    s = np.sort(a, axis=1).astype(np.uint64)
    rng = np.random.default_rng(salt)
    mult = rng.integers(1, 2 ** 63, size=s.shape[1], dtype=np.uint64) | np.uint64(1)
    h = np.zeros(s.shape[0], np.uint64)
    with np.errstate(over="ignore"):
        for m in range(s.shape[1]):
            x = (s[:, m] + np.uint64(0x9E3779B97F4A7C15)) * mult[m]
            h ^= x
            h = h * np.uint64(0xBF58476D1CE4E5B9) + np.uint64(m + 1)
    return h


def check_plan(gt, ot, elems):
    """Raises AssertionError on the first property that fails."""
    D = ot.dim
    pv = gt.plan_view()
    nv = ot.n_nodes
    off = ot["node_inc_off"].astype(np.int64)
    rowlen = np.diff(off)
    ninc = int(off[-1])
    nsl = (nv + 63) // 64
    so = pv["slice_off"].astype(np.int64)
    # slices
    pad = np.zeros(nsl * 64, np.int64)
    pad[:nv] = rowlen
    assert so[0] == 0 and (np.diff(so) == 64 * pad.reshape(nsl, 64).max(axis=1)).all(), "slices"
    assert pv["n_slots"] == so[-1]
    wide = pv["words"] == 2
    B = 10 if wide else 5
    none = (1 << B) - 1
    jj = np.repeat(np.arange(nv, dtype=np.int64), rowlen)
    rr = np.arange(ninc, dtype=np.int64) - np.repeat(off[:-1], rowlen)
    P = so[jj // 64] + 64 * rr + jj % 64
    # the incidences' slots: rank in the row
    inc = ot["node_inc"].astype(np.int64)
    assert (pv["inc_slot"][inc] == P).all(), "incidence slots"
    # decode the entries
    w = pv["entry"]
    if wide:
        w0, w1 = w[2 * P], w[2 * P + 1]
        o = np.stack([(w0 & 0xFFFFFFFF).astype(np.int64), (w0 >> 32).astype(np.int64),
                      (w1 & 0xFFFFFFFF).astype(np.int64)], 1)[:, :D]
        code = (w1 >> 32).astype(np.int64)
    else:
        w0 = w[P]
        o = np.stack([jj + ((w0 >> np.uint64(16 * m)) & 0xFFFF).astype(np.int16).astype(np.int64)
                      for m in range(D)], 1)
        code = ((w0 >> 48) & 0x7FFF).astype(np.int64)
    slot = np.stack([(code >> (B * m)) & none for m in range(D)], 1)
    # zeros past the rows
    covered = np.zeros(pv["n_slots"], bool)
    covered[P] = True
    ww = w.reshape(-1, 2) if wide else w.reshape(-1, 1)
    assert (ww[~covered] == 0).all(), "slots past a row are not zero"
    # permutation of the incidences (multiset of other-vertex sets per node)
    ref = _local_others(elems, inc, D)
    starts = off[:-1][rowlen > 0]
    for salt in (1, 2):
        ha, hb = _hash_rows(o, salt), _hash_rows(ref, salt)
        with np.errstate(over="ignore"):
            sa, sb = np.add.reduceat(ha, starts), np.add.reduceat(hb, starts)
        assert (sa == sb).all(), "entries are not a permutation of the incidences"
    # slots
    edge = ot["edge"].astype(np.int64)
    keys = edge[0] * nv + edge[1]
    eoff = ot["node_edge_off"].astype(np.int64)
    for m in range(D):
        up = o[:, m] > jj
        want = np.full(ninc, none, np.int64)
        k = jj[up] * nv + o[up, m]
        eid = np.searchsorted(keys, k)
        assert (keys[eid] == k).all(), "entry vertex is not a neighbour"
        want[up] = eid - eoff[jj[up]]
        assert (slot[:, m] == want).all(), f"out-edge slots (place {m})"
    # long rows: ascending incidences, local order
    longrow = np.repeat(rowlen > 32, rowlen)
    assert (o[longrow] == ref[longrow]).all(), "rows beyond 32 entries"
    # strips: first entry, places, face sharing
    first = rr == 0
    assert (o[first & ~longrow] == ref[first & ~longrow]).all(), "a strip's first entry"
    nxt = (rr[1:] > 0) & ~longrow[1:]  # pairs (q-1, q) inside one strip
    a, b = o[:-1][nxt], o[1:][nxt]
    inb = np.zeros(a.shape, bool)  # a's place k holds a vertex b also holds
    for k in range(D):
        inb[:, k] = (a[:, [k]] == b).any(axis=1)
    assert ((~inb) | (a == b)).all(), "a shared vertex left its place"
    shared = inb.sum(axis=1)
    brk = np.nonzero(shared < D - 1)[0]
    if brk.size:
        q = np.nonzero(nxt)[0][brk] + 1  # position of the entry after the break
        end = off[jj[q] + 1]
        prev = o[q - 1]
        span = np.arange(32)
        idx = q[:, None] + span[None, :]
        valid = idx < end[:, None]
        cand = o[np.minimum(idx, ninc - 1)]
        sh = np.zeros(valid.shape, np.int64)
        for m in range(D):
            sh += (cand[:, :, m][:, :, None] == prev[:, None, :]).any(axis=2)
        assert not ((sh >= D - 1) & valid).any(), "a strip broke although a face-sharing entry was left"
    # step words: present in the narrow format always, in the wide one when
    # every offset fits 20 bits and no node has more than 31 out-edges
    fits = bool(ninc == 0 or (np.abs(o - jj[:, None]).max() <= (1 << 19) - 1
                              and np.diff(eoff).max(initial=0) <= 31))
    if not wide:
        assert pv["step"] is not None and fits, "narrow plan without step words"
    else:
        assert (pv["step"] is not None) == fits, "wide plan: step words iff they fit"
    if pv["step"] is not None:
        st = pv["step"]
        assert (st[~covered] == 0).all(), "step words past a row"
        sw = st[P].astype(np.int64)
        assert (sw[rr == 0] == 1 << 27).all(), "a row's first step word"
        q = np.nonzero(rr > 0)[0]
        a, b = o[q - 1], o[q]
        ch = a != b
        one = ch.sum(axis=1) == 1
        k = np.argmax(ch, axis=1)
        bk = b[np.arange(q.size), k]
        sk = np.minimum(slot[q, k], 31)  # (wide "none" is 31 in a word)
        want = np.where(one, ((bk - jj[q]) & 0xFFFFF) | (k << 20) | (sk << 22), 1 << 27)
        assert (sw[q] == want).all(), "step words"
    return dict(n_slots=int(pv["n_slots"]), wide=bool(wide), steps=pv["step"] is not None,
                breaks=int(brk.size))
