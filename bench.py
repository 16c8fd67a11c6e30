#!/usr/bin/env python3
"""Benchmark of the edge-based metric path on one MI355X.

One step = the whole hot path over the 161^3 stretched Kuhn grid
(24,576,000 tets): edge extraction and boundary elements (eb_build_edges +
eb_build_edges_emit), the fused forward pass n, b, V (eb_directed_areas,
deterministic gather), the edge-loop dual volumes (eb_dual_volumes EDGE) and
the adjoint dL/dx (eb_directed_areas_backward; FP64 atomics after per-block
sums in LDS by default, the faster of the two reductions here, or the
deterministic gather with --bwd-reduce gather; both are timed as phases).
Inputs are resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Melements/s & HBM GB/s (% peak) for directed-area+dual-volume build; "
          "batched+adjoint vs plain")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes_forward(dim, nv, nel, ne_, nb, nbn):
    """Algorithmic bytes of one fused forward pass (n, b, V): every input read
    once, every output written once, plus one element->edge addressing array.
      coords 8D Nv + elems 4(D+1) NE + addressing 4 ne NE + n 8D Ne + V 8 Nv
      + b 8D Nbn + boundary elements 4(D + ne_B) NB"""
    ne = dim * (dim + 1) // 2       # local edges of an element
    neb = dim * (dim - 1) // 2      # edges of a boundary element
    return (8 * dim * nv + 4 * (dim + 1) * nel + 4 * ne * nel + 8 * dim * ne_ + 8 * nv
            + 8 * dim * nbn + 4 * (dim + neb) * nb)


def alg_bytes_backward(dim, nv, nel, ne_, nb, nbn):
    """coords + elems + elem_edge + boundary elements + dL/dn + dL/db + dL/dV
    + dL/dx (each once)."""
    ne = 3 if dim == 2 else 6
    neb = 1 if dim == 2 else 3
    return (8 * dim * nv + 4 * (dim + 1) * nel + 4 * ne * nel + 4 * (dim + neb) * nb
            + 8 * dim * ne_ + 8 * dim * nbn + 8 * nv + 8 * dim * nv)


def alg_bytes_edge_volume(dim, nv, ne_):
    """edges 8 Ne + n 8D Ne + coords 8D Nv + V 8 Nv."""
    return 8 * ne_ + 8 * dim * ne_ + 8 * dim * nv + 8 * nv


def alg_bytes_build(dim, nv, nel, ne_, nb, nbn, plan_bytes):
    """Edge extraction and boundary elements: connectivity and coordinates
    read once, every topology array and the kernel plan written once (the
    optional edge->element CSR excluded, as in the timed build)."""
    ne = 3 if dim == 2 else 6
    neb = 1 if dim == 2 else 3
    reads = 4 * (dim + 1) * nel + 8 * dim * nv
    writes = (8 * ne_ + 4 * (nv + 1)                 # edge, node_edge_off
              + 4 * ne * nel + ne * nel               # elem_edge, signs
              + 4 * (dim + 1) * nel + 4 * (nv + 1)    # node_inc (+off)
              + 4 * ne_ + 4 * (nv + 1)                # node_in (+off)
              + 4 * dim * nb + 4 * nb + 4 * neb * nb  # bface, owner, bface_edge
              + 4 * nbn + 4 * nv                      # bnode, node_bnode
              + 4 * dim * nb + 4 * (nbn + 1)          # bnode_face (+off)
              + plan_bytes)
    return reads + writes


def source_digest(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2502_00778_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_key, digest):
    """HBM bytes per dispatch measured with rocprofv3 counters, if the kernel
    source is unchanged since (profiles/hbm_traffic_*.md)."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{kernel_key}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source digest:\s*`?([0-9a-f]+)`?", txt)
    b = re.search(r"traffic bytes per dispatch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != digest:
        return None
    return float(b.group(1))


class Timer:
    def __init__(self, torch):
        self.torch = torch

    def time(self, fn, reps):
        t = self.torch
        s = t.cuda.current_stream()
        ev = [(t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(s)
            fn()
            b.record(s)
        t.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        return float(np.mean(ms)), float(np.median(ms)), float(np.min(ms))

    def time_call(self, eb, fn, reps):
        """Kernel time of a forward call: the library records the armed
        events before its first kernel and after its last
        (eb_time_next_call)."""
        t = self.torch
        ev = [(t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record()
            b.record()
        t.cuda.synchronize()
        for a, b in ev:
            eb.time_next_call(a, b)
            fn()
        t.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        return float(np.mean(ms)), float(np.median(ms)), float(np.min(ms))

    def time_principal(self, eb, fn, reps):
        """Duration of the call's principal kernel alone: the library records
        the armed events around that one launch (eb_time_next_launch)."""
        t = self.torch
        ev = [(t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:  # create the events on the device
            a.record()
            b.record()
        t.cuda.synchronize()
        for a, b in ev:
            eb.time_next_launch(a, b)
            fn()
        t.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        return float(np.mean(ms)), float(np.median(ms)), float(np.min(ms))


def cpu_model():
    """The host CPU's model name (lscpu), for the record."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    for ln in out.splitlines():
        if ln.startswith("Model name:"):
            return ln.split(":", 1)[1].strip()
    return None


def cpu_baseline(mesh_full, n_layers=24, target_s=12.0, single_layers=6):
    """The oracle on a slab of the same grid: the first node layers in z (all
    tets between them), grown from n_layers until one run takes about
    target_s, on all host threads; then single-threaded (the paper's serial
    setting) on a thinner slab.  Same rows as a GPU step: topology, n, b, V,
    and the gradient of the same loss (all nodes)."""
    import oracle
    n = mesh_full.meta["n"]
    r = _cpu_slab(mesh_full, n_layers)
    if r["seconds"] < target_s / 1.5 and n_layers < n:
        grow = int(np.ceil(n_layers * target_s / max(r["seconds"], 1e-3)))
        r = _cpu_slab(mesh_full, min(n, max(grow, n_layers + 1)))
    r.pop("seconds")
    threads = oracle.num_threads()
    oracle.set_threads(1)
    try:
        r1 = _cpu_slab(mesh_full, single_layers)
    finally:
        oracle.set_threads(threads)
    r1.pop("seconds")
    r["single_thread"] = {k: r1[k] for k in ("value", "unit", "cores", "sample")}
    r["cpu_model"] = cpu_model()
    r["os_cpu_count"] = os.cpu_count()
    return r


def _cpu_slab(mesh_full, n_layers):
    import meshgen
    import oracle
    n = mesh_full.meta["n"]
    nv_slab = n * n * n_layers
    ne_slab = 6 * (n - 1) ** 2 * (n_layers - 1)
    X = np.ascontiguousarray(mesh_full.coords[:, :nv_slab])
    E = np.ascontiguousarray(mesh_full.elems[:ne_slab])
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    ot = oracle.topology(3, X, E)
    t1 = time.perf_counter()
    oracle.metrics(ot, X, E)
    t2 = time.perf_counter()
    w, c, beta = meshgen.loss_weights(0, 3, ot.n_edges, ot.n_nodes, ot.n_bnodes)
    oracle.node_grad(ot, X, E, w, c, beta)
    t3 = time.perf_counter()
    total = t3 - t0
    return {
        "value": round(ne_slab / total / 1e6, 3),
        "unit": "Melements/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"first {n_layers} of {n} z node layers of the same grid: {ne_slab} tets; "
                   f"topology {t1 - t0:.2f} s, n/b/V {t2 - t1:.2f} s, gradient {t3 - t2:.2f} s"),
        "seconds": total,
    }


def alg_bytes_fused(dim, nv, nel, ne_, nb, nbn):
    """Forward + adjoint with the shared inputs (coords, elems, element->edge
    addressing, boundary elements) counted once."""
    ne = 3 if dim == 2 else 6
    neb = 1 if dim == 2 else 3
    shared = 8 * dim * nv + 4 * (dim + 1) * nel + 4 * ne * nel + 4 * (dim + neb) * nb
    return (alg_bytes_forward(dim, nv, nel, ne_, nb, nbn)
            + alg_bytes_backward(dim, nv, nel, ne_, nb, nbn) - shared)


def bench_batched(torch, eb, meshgen, seed, reps, tm):
    """The 64-mesh batch: forward + adjoint as one enqueue in each fused mode
    (the tuned deterministic one also replayed from a captured graph, and the
    two forms with the atomic adjoint, eager and from a graph)
    against 64 x (plain gather forward + plain adjoint) on the meshes one by
    one, with the gather adjoint for the deterministic modes and the atomic
    one for the atomic mode."""
    t0 = time.perf_counter()
    bm = meshgen.batched_kuhn(64, seed)
    log(f"[bench] batch of 64 meshes: {bm.n_elems} tets ({time.perf_counter() - t0:.1f} s)")
    X = torch.from_numpy(bm.coords).cuda()
    E = torch.from_numpy(bm.elems).cuda()
    topo = eb.build_edges(E, X, edge_inc=False)
    batch = eb.batch_offsets(topo, E, bm.node_off, bm.elem_off)
    nv, nel, ne_, nb, nbn = (topo.n_nodes, topo.n_elems, topo.n_edges, topo.n_bfaces,
                             topo.n_bnodes)
    w, c, beta = meshgen.loss_weights(seed, 3, ne_, nv, nbn)
    W, C, B = (torch.from_numpy(a).cuda() for a in (w, c, beta))
    outs = dict(n=torch.empty(3, ne_, dtype=torch.float64, device="cuda"),
                b=torch.empty(3, nbn, dtype=torch.float64, device="cuda"),
                V=torch.empty(nv, dtype=torch.float64, device="cuda"),
                g=torch.empty(3, nv, dtype=torch.float64, device="cuda"))
    tune = eb.autotune(X, topo, E, W, B, C, reps=3, out=outs)
    log(f"[bench] autotune (batch): {tune}")

    def fused():
        eb.forward_backward(X, topo, E, W, B, C, out=outs)

    tuned_mode = eb.get_fused_mode()
    eb.set_fused_mode("persistent")  # the one persistent launch, best shape
    fused()
    t_fused = tm.time(fused, reps)
    k_fused = tm.time_principal(eb, fused, reps)
    eb.set_fused_mode("separate")    # the gather kernels one after another
    fused()
    t_sep = tm.time(fused, reps)
    atomic = {}
    for mode in ("persistent_atomic", "separate_atomic"):  # the FP64-atomic adjoint
        eb.set_fused_mode(mode)
        fused()
        t_eager = tm.time(fused, reps)
        gr = eb.ForwardBackwardGraph(X, topo, E, W, B, C)
        gr.launch()
        atomic[mode] = (t_eager, tm.time(gr.launch, reps))
        gr.close()
    t_atomic, t_graph_atomic = atomic["persistent_atomic"]
    t_sep_atomic, t_graph_sep_atomic = atomic["separate_atomic"]
    eb.set_fused_mode(tuned_mode)
    gr = eb.ForwardBackwardGraph(X, topo, E, W, B, C)
    gr.launch()
    t_graph = tm.time(gr.launch, reps)
    eb.check_errors(topo)
    gr.close()

    # the same meshes one at a time, each with its own topology
    per = []
    for m in range(64):
        v0, v1 = int(bm.node_off[m]), int(bm.node_off[m + 1])
        e0, e1 = int(bm.elem_off[m]), int(bm.elem_off[m + 1])
        Xm = X[:, v0:v1].contiguous()
        Em = (E[e0:e1] - v0).contiguous()
        tmm = eb.build_edges(Em, Xm, edge_inc=False)
        sl = lambda t, k: batch.split(t, k)[m].contiguous()
        per.append((Xm, Em, tmm, sl(W, "edge"), sl(B, "bnode"), sl(C, "node"),
                    torch.empty(3, tmm.n_edges, dtype=torch.float64, device="cuda"),
                    torch.empty(3, tmm.n_bnodes, dtype=torch.float64, device="cuda"),
                    torch.empty(tmm.n_nodes, dtype=torch.float64, device="cuda"),
                    torch.empty(3, tmm.n_nodes, dtype=torch.float64, device="cuda")))

    def plain():
        for Xm, Em, tmm, Wm, Bm, Cm, n_, b_, V_, g_ in per:
            eb.directed_areas(Xm, tmm, Em, "gather", n_out=n_, b_out=b_, v_out=V_)
            eb.directed_areas_backward(Xm, tmm, Em, Wm, Bm, Cm, reduce="gather", out=g_)

    def plain_atomic():  # (the baseline of the persistent kernel with the atomic adjoint)
        for Xm, Em, tmm, Wm, Bm, Cm, n_, b_, V_, g_ in per:
            eb.directed_areas(Xm, tmm, Em, "gather", n_out=n_, b_out=b_, v_out=V_)
            eb.directed_areas_backward(Xm, tmm, Em, Wm, Bm, Cm, reduce="atomic", out=g_)

    plain()
    t_plain = tm.time(plain, reps)
    plain_atomic()
    t_plain_atomic = tm.time(plain_atomic, reps)
    bytes_ = alg_bytes_fused(3, nv, nel, ne_, nb, nbn)
    res = {
        "workload": (f"64 Kuhn cubes, n log-uniform in [9, 65] (seed {seed}): {nel} tets, "
                     f"{nv} nodes, {ne_} edges; forward n/b/V + adjoint dL/dx"),
        "persistent_ms": round(t_fused[0], 4),
        "persistent_kernel_ms": round(k_fused[0], 4),
        "separate_kernels_ms": round(t_sep[0], 4),
        "persistent_atomic_ms": round(t_atomic[0], 4),
        "separate_atomic_kernels_ms": round(t_sep_atomic[0], 4),
        "graph_separate_atomic_ms": round(t_graph_sep_atomic[0], 4),
        "graph_persistent_atomic_ms": round(t_graph_atomic[0], 4),
        "tuned_mode": tuned_mode,
        "graph_ms": round(t_graph[0], 4),
        "per_mesh_plain_ms": round(t_plain[0], 4),
        "per_mesh_plain_atomic_ms": round(t_plain_atomic[0], 4),
        "speedup_graph_vs_per_mesh": round(t_plain[0] / t_graph[0], 2),
        "speedup_graph_persistent_atomic_vs_per_mesh_atomic":
            round(t_plain_atomic[0] / t_graph_atomic[0], 2),
        "speedup_graph_separate_atomic_vs_per_mesh_atomic":
            round(t_plain_atomic[0] / t_graph_sep_atomic[0], 2),
        "Melements_per_s_graph": round(nel / (t_graph[0] * 1e-3) / 1e6, 1),
        "Melements_per_s_per_mesh": round(nel / (t_plain[0] * 1e-3) / 1e6, 1),
        "alg_GBps_graph": round(bytes_ / (t_graph[0] * 1e-3) / 1e9, 1),
        "frac_hbm_peak_graph": round(bytes_ / (t_graph[0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "alg_bytes": bytes_,
        "tuned_shape": {k: tune[k] for k in ("fused_tile", "fused_unroll",
                                             "fused_blocks_per_cu", "gather_tile",
                                             "gather_unroll", "gather_xcd_remap")},
    }
    log(f"[bench] batched: {res}")
    return res


# context only (another machine, serial CPU): the paper's time for one n_jk
# evaluation on its 257^3 tet grid (Table 3)
PAPER_NJK_PROPOSED_TET_S = 13.5


def bench_deforming(torch, eb, meshgen, seed, steps, tm):
    """Deforming-grid loop at the size of the paper's tet grid (257^3 nodes,
    100,663,296 tets): topology built once, coordinates moved in place each
    step, one captured graph replays the forward (n, b, V) and the edge-based
    V.  Only the replay is timed; the paper's serial time for n_jk alone on a
    grid of this size is quoted beside it for scale."""
    t0 = time.perf_counter()
    m = meshgen.cube_kuhn(257, seed)
    frames_h = [m.coords, meshgen.cube_kuhn(257, seed + 1).coords]
    log(f"[bench] deforming: 257^3 grid, {m.n_elems} tets ({time.perf_counter() - t0:.1f} s)")
    X = torch.from_numpy(m.coords).cuda()
    E = torch.from_numpy(m.elems).cuda()
    frames = [torch.from_numpy(f).cuda() for f in frames_h]
    topo = eb.build_edges(E, X, edge_inc=False, adjoint=False)
    f64 = dict(dtype=torch.float64, device="cuda")
    n = torch.empty(3, topo.n_edges, **f64)
    b = torch.empty(3, topo.n_bnodes, **f64)
    V = torch.empty(topo.n_nodes, **f64)
    Ve = torch.empty(topo.n_nodes, **f64)

    def step():
        eb.directed_areas(X, topo, E, "gather", n_out=n, b_out=b, v_out=V)
        eb.dual_volumes(X, topo, E, "edge", n=n, reduce="gather", out=Ve)

    step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    ms = []
    for k in range(steps):
        X.copy_(frames[k % 2])
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record()
        g.replay()
        ev[1].record()
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    last = (n.clone(), V.clone())
    step()  # eager on the same coordinates: the replay must give the same bits
    torch.cuda.synchronize()
    same = bool(torch.equal(last[0], n) and torch.equal(last[1], V))
    eb.check_errors(topo)
    t_ms = float(np.mean(ms))
    res = {
        "workload": (f"257^3 Kuhn grid (seed {seed}), {m.n_elems} tets, {topo.n_edges} edges; "
                     "per step: coordinates moved in place, graph replay of n, b, V "
                     "(gather) + edge-based V"),
        "ms_per_step": round(t_ms, 4),
        "Melements_per_s": round(m.n_elems / (t_ms * 1e-3) / 1e6, 1),
        "steps": steps,
        "replay_equals_eager": same,
        "paper_serial_njk_s_per_step_context": PAPER_NJK_PROPOSED_TET_S,
    }
    log(f"[bench] deforming: {res}")
    return res


def bench_relabelled(torch, eb, meshgen, mesh, seed, reps, tm):
    """The 161^3 grid with its node ids randomly permuted (seeded; elements
    keep their order and local vertex order): a numbering with no locality,
    for which the kernel plan takes its wide format (neighbour ids beyond
    int16 offsets).  Build, forward (gather), edge-based V and adjoint
    (atomic), each timed with events around the call."""
    nv = mesh.coords.shape[1]
    perm = np.random.default_rng(np.random.SeedSequence([seed, 161])).permutation(nv)
    coords = np.empty_like(mesh.coords)
    coords[:, perm] = mesh.coords
    elems = perm[mesh.elems].astype(np.int32)
    X = torch.from_numpy(coords).cuda()
    E = torch.from_numpy(elems).cuda()
    t_build = tm.time(lambda: eb.build_edges(E, X, edge_inc=False), max(2, reps // 2))
    topo = eb.build_edges(E, X, edge_inc=False)
    nel, ne_ = topo.n_elems, topo.n_edges
    w, c, beta = meshgen.loss_weights(seed, 3, ne_, topo.n_nodes, topo.n_bnodes)
    W, C, B = (torch.from_numpy(a).cuda() for a in (w, c, beta))
    f64 = dict(dtype=torch.float64, device="cuda")
    n = torch.empty(3, ne_, **f64)
    b = torch.empty(3, topo.n_bnodes, **f64)
    V = torch.empty(topo.n_nodes, **f64)
    g = torch.empty(3, topo.n_nodes, **f64)
    fwd = lambda: eb.directed_areas(X, topo, E, "gather", n_out=n, b_out=b, v_out=V)
    vol = lambda: eb.dual_volumes(X, topo, E, "edge", n=n, reduce="gather", out=V)
    bwd = lambda: eb.directed_areas_backward(X, topo, E, W, B, C, reduce="atomic", out=g)
    res = {"workload": (f"161^3 Kuhn grid as timed above with node ids permuted at random "
                        f"(seed {seed}): {nel} tets, {ne_} edges"),
           "wide_plan": bool(topo.sizes.plan_param[1])}
    for name, fn in (("forward_gather", fwd), ("edge_volume_gather", vol), ("adjoint_atomic", bwd)):
        fn()
        res[name + "_ms"] = round(tm.time(fn, reps)[0], 4)
    res["build_ms"] = round(t_build[0], 4)
    eb.check_errors(topo)
    log(f"[bench] relabelled: {res}")
    return res


def bench_2d(torch, eb, meshgen, seed, reps, tm):
    """The triangle grids: the 33 x 33 config and a 256 x 256 grid of the
    paper's size (130,050 triangles): build, forward (gather), edge-based V
    and adjoint (gather), each timed on the stream (these grids are
    launch-bound, far below the HBM roofline)."""
    out = {}
    for name, mesh in (("2d-33", meshgen.square_tri(33, seed)),
                       ("2d-256", meshgen.square_tri(256, seed))):
        X = torch.from_numpy(mesh.coords).cuda()
        E = torch.from_numpy(mesh.elems).cuda()
        topo = eb.build_edges(E, X, edge_inc=False)
        w, c, beta = meshgen.loss_weights(seed, 2, topo.n_edges, topo.n_nodes, topo.n_bnodes)
        W, C, B = (torch.from_numpy(a).cuda() for a in (w, c, beta))
        n, b, V = eb.directed_areas(X, topo, E, "gather")
        fns = {
            "build": lambda: eb.build_edges(E, X, edge_inc=False),
            "forward_gather": lambda: eb.directed_areas(X, topo, E, "gather", n_out=n, b_out=b,
                                                        v_out=V),
            "edge_volume_gather": lambda: eb.dual_volumes(X, topo, E, "edge", n=n,
                                                          reduce="gather"),
            "adjoint_gather": lambda: eb.directed_areas_backward(X, topo, E, W, B, C,
                                                                 reduce="gather"),
        }
        r = {"elements": mesh.n_elems, "nodes": mesh.n_nodes, "edges": topo.n_edges}
        for k, fn in fns.items():
            fn()
            ms = tm.time(fn, reps)[0]
            r[k] = {"ms": round(ms, 4), "Melements_per_s": round(mesh.n_elems / (ms * 1e-3) / 1e6, 1)}
        eb.check_errors(topo)
        out[name] = r
    log(f"[bench] 2d: {out}")
    return out


def bench_4d(torch, eb, meshgen, seed, reps, tm, n=33):
    """Pentatopes: the n^4 Kuhn grid (33^4: 1,185,921 nodes, 25,165,824
    pentatopes, about the 161^3 tet grid's element count): build, forward
    (gather and atomic), edge-based V, each timed on the stream; with the
    checks that hold at any size (the volumes sum to the unit 4-cube's 1,
    the edge-based V equals the element-based V)."""
    t0 = time.perf_counter()
    mesh = meshgen.hypercube_kuhn(n, seed)
    log(f"[bench] 4d: {n}^4 grid, {mesh.n_elems} pentatopes ({time.perf_counter() - t0:.1f} s)")
    X = torch.from_numpy(mesh.coords).cuda()
    E = torch.from_numpy(mesh.elems).cuda()
    topo = eb.build_edges(E, X, edge_inc=False, adjoint=False)
    nv, nel, ne_, nb, nbn = (topo.n_nodes, topo.n_elems, topo.n_edges, topo.n_bfaces,
                             topo.n_bnodes)
    n_, b, V = eb.directed_areas(X, topo, E, "gather")
    Ve = eb.dual_volumes(X, topo, E, "edge", n=n_, reduce="gather")
    vol_sum = float(V.sum())
    rel = float(((Ve - V).abs() / V.abs()).max())
    fns = {
        "build": lambda: eb.build_edges(E, X, edge_inc=False, adjoint=False),
        "forward_gather": lambda: eb.directed_areas(X, topo, E, "gather", n_out=n_, b_out=b,
                                                    v_out=V),
        "forward_atomic": lambda: eb.directed_areas(X, topo, E, "atomic", n_out=n_, b_out=b,
                                                    v_out=V),
        "edge_volume_gather": lambda: eb.dual_volumes(X, topo, E, "edge", n=n_, reduce="gather",
                                                      out=Ve),
    }
    bf = alg_bytes_forward(4, nv, nel, ne_, nb, nbn)
    r = {"workload": f"{n}^4 Kuhn grid (seed {seed}): {nel} pentatopes, {nv} nodes, {ne_} edges",
         "volume_sum": vol_sum, "edge_vs_element_V_max_rel": rel}
    for k, fn in fns.items():
        fn()
        ms = tm.time(fn, max(2, reps // 2) if k == "build" else reps)[0]
        r[k] = {"ms": round(ms, 4), "Melements_per_s": round(nel / (ms * 1e-3) / 1e6, 1)}
        if k.startswith("forward"):
            r[k]["alg_GBps"] = round(bf / (ms * 1e-3) / 1e9, 1)
            r[k]["frac_hbm_peak"] = round(bf / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    eb.check_errors(topo)
    log(f"[bench] 4d: {r}")
    return r


def calibrate(nbytes=1 << 30, reps=5):
    """Kernels of known traffic for scaling the HBM counters: a read-only
    reduction (torch.sum over nbytes of float64: reads nbytes), an
    elementwise product into another array (reads and writes nbytes), and
    a fill and a copy (runtime kernels or DMA), reps times each."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        a.fill_(1.0)
    for _ in range(reps):
        b.copy_(a)
    s = None
    for _ in range(reps):
        s = a.sum()
    for _ in range(reps):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"bytes": nbytes, "reps": reps, "sum": float(s),
                      "fill": "write", "copy": "read+write", "sum_kernel": "read",
                      "mul_kernel": "read+write"}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="3d-scale")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phase-reps", type=int, default=20)
    ap.add_argument("--only", default="", help="profiling: run only this phase "
                    "(topo|fwd|fwd_atomic|vol_edge|bwd|bwd_atomic|fused|fwd_edge_normals|"
                    "fwd_dual_faces) --steps times, or the pentatope section (4d)")
    ap.add_argument("--calibrate", action="store_true",
                    help="run only kernels of known traffic (HBM counter scaling)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-deforming", action="store_true")
    ap.add_argument("--no-relabelled", action="store_true")
    ap.add_argument("--no-4d", action="store_true")
    ap.add_argument("--no-2d", action="store_true")
    ap.add_argument("--bwd-reduce", default="atomic", choices=("atomic", "gather"),
                    help="the adjoint's reduction in the timed step (both are timed as phases)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding "
                          "is a design note, not an implementation", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.calibrate:
        calibrate()
        return

    import torch

    import meshgen
    import paper_2502_00778_amd as eb

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.only == "4d":  # the pentatope section alone, each call --steps times
        bench_4d(torch, eb, meshgen, args.seed, args.steps, Timer(torch))
        return
    t0 = time.perf_counter()
    mesh = meshgen.make(args.config, args.seed)
    log(f"[bench] grid {mesh.name}: {mesh.n_nodes} nodes, {mesh.n_elems} elements "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    dim = mesh.dim
    X = torch.from_numpy(mesh.coords).cuda()
    E = torch.from_numpy(mesh.elems).cuda()
    topo = eb.build_edges(E, X, edge_inc=False)
    nv, nel, ne_, nb, nbn = (topo.n_nodes, topo.n_elems, topo.n_edges, topo.n_bfaces,
                             topo.n_bnodes)
    w, c, beta = meshgen.loss_weights(args.seed, dim, ne_, nv, nbn)
    W = torch.from_numpy(w).cuda()
    C = torch.from_numpy(c).cuda()
    B = torch.from_numpy(beta).cuda()
    n = torch.empty(dim, ne_, dtype=torch.float64, device="cuda")
    b = torch.empty(dim, nbn, dtype=torch.float64, device="cuda")
    V = torch.empty(nv, dtype=torch.float64, device="cuda")
    Ve = torch.empty(nv, dtype=torch.float64, device="cuda")
    g = torch.empty(dim, nv, dtype=torch.float64, device="cuda")
    bwd_reduce = args.bwd_reduce

    def ph_topo():
        eb.build_edges(E, X, edge_inc=False)

    def ph_fwd():
        eb.directed_areas(X, topo, E, "gather", n_out=n, b_out=b, v_out=V)

    def ph_fwd_atomic():
        eb.directed_areas(X, topo, E, "atomic", n_out=n, b_out=b, v_out=V)

    def ph_vol_edge():
        eb.dual_volumes(X, topo, E, "edge", n=n, reduce="gather", out=Ve)

    def ph_bwd():
        eb.directed_areas_backward(X, topo, E, W, B, C, reduce="gather", out=g)

    def ph_bwd_atomic():
        eb.directed_areas_backward(X, topo, E, W, B, C, reduce="atomic", out=g)

    fouts = dict(n=n, b=b, V=V, g=g)

    def ph_fused():
        eb.forward_backward(X, topo, E, W, B, C, out=fouts)

    def ph_fused_atomic():
        eb.set_fused_mode("persistent_atomic")
        try:
            eb.forward_backward(X, topo, E, W, B, C, out=fouts)
        finally:
            eb.set_fused_mode("persistent")

    def ph_fwd_edge_normals():
        eb.directed_areas_variant(X, topo, E, "edge_normals", n_out=n, b_out=b, v_out=V)

    def ph_fwd_dual_faces():
        eb.directed_areas_variant(X, topo, E, "dual_faces", n_out=n, b_out=b, v_out=V)

    phases = {"topo": ph_topo, "fwd": ph_fwd, "fwd_atomic": ph_fwd_atomic,
              "vol_edge": ph_vol_edge, "bwd": ph_bwd, "bwd_atomic": ph_bwd_atomic,
              "fused": ph_fused, "fused_atomic": ph_fused_atomic,
              "fwd_edge_normals": ph_fwd_edge_normals,
              "fwd_dual_faces": ph_fwd_dual_faces}

    if args.only:
        fn = phases[args.only]
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        log(f"[bench] ran {args.only} x{args.steps}")
        if args.only == "fwd":
            # the forward call's kernel time by events in this same process
            # (under a profiler: the profiler's own view beside it)
            t = Timer(torch).time_call(eb, fn, args.steps)
            log(f"[bench] forward call kernels by events: mean {t[0]:.4f} ms, "
                f"median {t[1]:.4f}, min {t[2]:.4f}")
        return

    def step():
        t = eb.build_edges(E, X, edge_inc=False)
        nn_, bb, vv = eb.directed_areas(X, t, E, "gather")
        eb.dual_volumes(X, t, E, "edge", n=nn_, reduce="gather")
        eb.directed_areas_backward(X, t, E, W, B, C, reduce=bwd_reduce)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done; timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    eb.check_errors(topo)
    log(f"[bench] {dt * 1e3:.3f} ms/step")

    # per-phase event timings on the stream the kernels run on
    tm = Timer(torch)
    res = {}
    for name, fn in phases.items():
        for _ in range(3):  # warm-up calls
            fn()
        res[name] = tm.time(fn, args.phase_reps)
        log(f"[bench] phase {name}: mean {res[name][0]:.3f} ms, median {res[name][1]:.3f}, "
            f"min {res[name][2]:.3f}")
    kern = {}
    for name in ("fwd", "fwd_atomic", "vol_edge", "bwd", "bwd_atomic", "fused", "fused_atomic",
                 "fwd_edge_normals", "fwd_dual_faces"):
        kern[name] = tm.time_principal(eb, phases[name], args.phase_reps)
        log(f"[bench] principal kernel of {name}: mean {kern[name][0]:.4f} ms, "
            f"median {kern[name][1]:.4f}, min {kern[name][2]:.4f}")
    fwd_call = tm.time_call(eb, phases["fwd"], args.phase_reps)
    log(f"[bench] forward call kernels (node + boundary pass): mean {fwd_call[0]:.4f} ms, "
        f"median {fwd_call[1]:.4f}, min {fwd_call[2]:.4f}")
    eb.check_errors(topo)
    # a plain device copy on the same box, in the same run: the bandwidth an
    # HBM-bound kernel can reach in practice (read + write bytes / time)
    cp_n = 1 << 30
    cp_a = torch.empty(cp_n // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    cp_b = torch.empty_like(cp_a)
    cp_ms = tm.time(lambda: cp_b.copy_(cp_a), args.phase_reps)[1]
    copy_gbs = 2 * cp_n / (cp_ms * 1e-3) / 1e9
    del cp_a, cp_b
    log(f"[bench] device copy of 1 GiB: {cp_ms:.3f} ms = {copy_gbs:.0f} GB/s")

    bf = alg_bytes_forward(dim, nv, nel, ne_, nb, nbn)
    bb_ = alg_bytes_backward(dim, nv, nel, ne_, nb, nbn)
    bv = alg_bytes_edge_volume(dim, nv, ne_)
    bbuild = alg_bytes_build(dim, nv, nel, ne_, nb, nbn, int(topo.sizes.plan_bytes))
    # roofline of the forward call (eb_directed_areas, gather): its two
    # kernels, the node pass and the boundary pass, from the start of the
    # first to the end of the second (eb_time_next_call); algorithmic bytes
    # B_fwd
    t_call = fwd_call[0] * 1e-3
    achieved = bf / t_call / 1e9
    digest = source_digest("eb_forward.hip", "eb_gather.h", "eb_geom.h", "eb_kernels.h",
                           "eb_internal.h", "eb_metrics.hip", "eb_plan.h")
    traffic = read_traffic("fwd_call_161", digest)

    def ph(name, bytes_):
        ms = res[name][0]
        out = {"ms": round(ms, 4), "Melements_per_s": round(nel / (ms * 1e-3) / 1e6, 1)}
        if bytes_:
            out["alg_GBps"] = round(bytes_ / (ms * 1e-3) / 1e9, 1)
            out["frac_hbm_peak"] = round(bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        if name in kern:
            out["principal_kernel_ms"] = round(kern[name][0], 4)
        return out

    line = {
        "metric": METRIC,
        "value": round(nel / dt / 1e6, 3),
        "unit": "Melements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.config}: {mesh.name} grid, {nel} elements, {nv} nodes, "
                         f"{ne_} edges; step = edge extraction + fused n/b/V forward (gather) "
                         f"+ edge-loop V + adjoint ({bwd_reduce})"),
            "elements": nel, "nodes": nv, "edges": ne_, "seed": args.seed,
        },
        "gather_shape": list(eb.get_gather_shape()),
        "roofline": {
            "kernel": ("eb_directed_areas gather forward call: k_fwd_gather (node pass, n and V) "
                       "+ k_fwd_boundary_gather (boundary pass, n_B terms and b)"),
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes": bf,
            "kernels_ms": round(fwd_call[0], 4),
            "node_pass_ms": round(kern["fwd"][0], 4),
            "call_ms_events_around": round(res["fwd"][0], 4),
            "measured_GBps": (round(traffic / t_call / 1e9, 1) if traffic else None),
            "copy_GBps": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
        },
        "phases": {
            "edge_extraction": dict(
                ph("topo", None),
                keys=(3 if dim == 2 else 6) * nel,
                Mkeys_per_s=round((3 if dim == 2 else 6) * nel / (res["topo"][0] * 1e-3) / 1e6, 1),
                alg_bytes=bbuild,
                alg_GBps=round(bbuild / (res["topo"][0] * 1e-3) / 1e9, 1),
                frac_hbm_peak=round(bbuild / (res["topo"][0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)),
            "forward_gather": ph("fwd", bf),
            "forward_atomic": ph("fwd_atomic", bf),
            "edge_volume_gather": ph("vol_edge", bv),
            "adjoint_gather": ph("bwd", bb_),
            "adjoint_atomic": ph("bwd_atomic", bb_),
            "fused_forward_adjoint": ph("fused", alg_bytes_fused(dim, nv, nel, ne_, nb, nbn)),
            "fused_forward_adjoint_atomic": ph("fused_atomic",
                                               alg_bytes_fused(dim, nv, nel, ne_, nb, nbn)),
            "forward_edge_normals": ph("fwd_edge_normals", bf),
            "forward_dual_faces": ph("fwd_dual_faces", bf),
        },
    }
    # the paper's Table 3 asks how much the dual-face construction costs over
    # the proposed formula (2.16x for n_jk on its serial tet run); on this GPU:
    line["traditional_vs_proposed"] = {
        "dual_faces_over_node_normals": round(kern["fwd_dual_faces"][0] / kern["fwd"][0], 3),
        "edge_normals_over_node_normals": round(kern["fwd_edge_normals"][0] / kern["fwd"][0], 3),
        "paper_serial_tet_njk_ratio": 2.16,
    }
    if not args.no_batched:
        line["batched"] = bench_batched(torch, eb, meshgen, args.seed, args.phase_reps, tm)
    if not args.no_2d:
        line["triangles"] = bench_2d(torch, eb, meshgen, args.seed, args.phase_reps, tm)
    if not args.no_4d:
        line["pentatopes"] = bench_4d(torch, eb, meshgen, args.seed, args.phase_reps, tm)
    if not args.no_relabelled:
        line["relabelled"] = bench_relabelled(torch, eb, meshgen, mesh, args.seed, args.phase_reps,
                                              tm)
    if not args.no_deforming:
        # free the 161^3 working set first
        del topo, X, E, W, C, B, n, b, V, Ve, g, fouts
        torch.cuda.empty_cache()
        line["deforming"] = bench_deforming(torch, eb, meshgen, args.seed, args.phase_reps, tm)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a slab of the same grid")
        line["cpu_baseline"] = cpu_baseline(mesh)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
