"""C-ABI checks that need no GPU: the library loads, exports every function
include/eb.h declares, and host-side validation rejects bad arguments with
the documented status codes before any device work is enqueued."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "eb.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(eb_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_2502_00778_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    from paper_2502_00778_amd import _lib
    names = declared_functions()
    assert "eb_directed_areas" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_status_strings(L):
    for code in range(0, -10, -1):
        s = L.eb_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.eb_status_string(-99).decode() == "unknown status"


def test_workspace_bytes(L):
    assert L.eb_workspace_bytes(5, 10, 10) == 0
    assert L.eb_workspace_bytes(4, 10, 10) > 0  # pentatope grids
    assert L.eb_workspace_bytes(3, 0, 10) == 0
    small = L.eb_workspace_bytes(3, 100, 300)
    big = L.eb_workspace_bytes(3, 161 ** 3, 6 * 160 ** 3)
    assert 256 < small < big
    # per-node arrays plus scan scratch (well under 64 B per node), the kept
    # neighbour sets (96 B per node, rounded up to whole 64-node slices) and
    # 22 bytes per incidence
    assert big < 161 ** 3 * (64 + 97) + 22 * 4 * 6 * 160 ** 3


def _up(x):
    return -(-x // 256) * 256


def sizes(dim, nv, ne, n_edges, n_bfaces, n_bnodes, n_slots=0, wide=0):
    """eb_sizes as eb_build_edges fills them: the plan's slot count and format
    (0 narrow entries, 1 wide entries, 2 wide entries with step words), and
    its byte size (four sections on 256-byte lines: slice offsets, entries,
    step words unless format 1, incidence slots)."""
    from paper_2502_00778_amd._lib import EbSizes
    nb = (_up(4 * ((nv + 63) // 64 + 1)) + _up(8 * n_slots * (1 + (wide != 0)))
          + (0 if wide == 1 else _up(4 * n_slots)) + _up(4 * (dim + 1) * ne))
    sz = EbSizes(dim=dim, n_nodes=nv, n_elems=ne, n_edges=n_edges, n_bfaces=n_bfaces,
                 n_bnodes=n_bnodes, plan_bytes=nb)
    sz.plan_param[0], sz.plan_param[1] = n_slots, wide
    return sz


def test_backward_workspace_bytes(L):
    from paper_2502_00778_amd._lib import EbSizes
    for dim, per in ((3, 24), (2, 16)):
        sz = sizes(dim, 1000, 5000, 6000, 10, 10, n_slots=64 * 400)
        base = L.eb_workspace_bytes(dim, 1000, 5000)
        got = L.eb_backward_workspace_bytes(ctypes.byref(sz))
        # the build keeps 22 bytes per incidence (row entry, position, rank) at
        # the end of its layout; the adjoint's gradient pieces (D doubles per
        # sliced entry) take that place
        up = _up
        ninc = (dim + 1) * 5000
        rows = up(16 * ninc) + up(4 * ninc) + up(2 * ninc)
        pieces = -(-per * 64 * 400 // 256) * 256
        assert got == max(base, base - rows + pieces)
    bad = EbSizes(dim=5, n_nodes=10, n_elems=10)
    assert L.eb_backward_workspace_bytes(ctypes.byref(bad)) == 0
    # plan fields that no build produces are rejected
    bad = sizes(3, 1000, 5000, 6000, 10, 10, n_slots=64 * 400)
    bad.plan_bytes += 256
    assert L.eb_backward_workspace_bytes(ctypes.byref(bad)) == 0
    bad = sizes(3, 1000, 5000, 6000, 10, 10, n_slots=65)
    assert L.eb_backward_workspace_bytes(ctypes.byref(bad)) == 0
    bad = sizes(3, 1000, 5000, 6000, 10, 10, n_slots=64 * 400, wide=2)
    assert L.eb_backward_workspace_bytes(ctypes.byref(bad)) > 0
    bad.plan_param[1] = 3  # no such format
    assert L.eb_backward_workspace_bytes(ctypes.byref(bad)) == 0


def test_plan_describe(L):
    """eb_plan_describe points into the plan at the section offsets and
    reads no device memory; it rejects sizes not made by a build."""
    from paper_2502_00778_amd._lib import EbPlanView
    for wide in (0, 1, 2):
        sz = sizes(3, 1000, 5000, 6000, 10, 10, n_slots=64 * 400, wide=wide)
        v = EbPlanView()
        base = 1 << 20
        assert L.eb_plan_describe(ctypes.byref(sz), ctypes.c_void_p(base), ctypes.byref(v)) == 0
        assert (v.n_slots, v.words) == (64 * 400, 1 + (wide != 0))
        assert v.slice_off == base
        assert v.entry == base + _up(4 * (16 + 1))
        assert (v.step is None) == (wide == 1)
        if wide != 1:
            assert v.step == base + _up(4 * (16 + 1)) + _up(8 * 64 * 400 * v.words)
        assert v.inc_slot == base + sz.plan_bytes - _up(4 * 4 * 5000)
    sz.plan_bytes = 7
    assert L.eb_plan_describe(ctypes.byref(sz), ctypes.c_void_p(1 << 20), ctypes.byref(v)) == -1


def test_host_validation(L):
    from paper_2502_00778_amd._lib import EbSizes, EbTopology
    sz = EbSizes()
    P = ctypes.c_void_p
    fake = P(256)  # never dereferenced: validation fails first
    rc = L.eb_build_edges(5, 10, 10, fake, fake, fake, fake, fake, 10 ** 6,
                          ctypes.byref(sz), None)
    assert rc == -1
    rc = L.eb_build_edges(3, 10, 2 ** 30, fake, fake, fake, fake, fake, 10 ** 6,
                          ctypes.byref(sz), None)
    assert rc == -6  # 6 * 2^30 local edges overflow int32 indexing
    rc = L.eb_build_edges(3, 10, 10, P(258), fake, fake, fake, fake, 10 ** 6,
                          ctypes.byref(sz), None)
    assert rc == -1  # misaligned
    rc = L.eb_build_edges(3, 10, 10, fake, fake, fake, fake, fake, 16,
                          ctypes.byref(sz), None)
    assert rc == -5  # workspace too small
    assert b"workspace" in L.eb_last_error_detail()
    sz = sizes(3, 8, 6, 19, 12, 8)
    tp = EbTopology()
    rc = L.eb_directed_areas(ctypes.byref(sz), ctypes.byref(tp), fake, fake, 7, fake,
                             None, None, fake, 10 ** 6, None)
    assert rc == -1  # bad reduce
    rc = L.eb_directed_areas(ctypes.byref(sz), ctypes.byref(tp), fake, fake, 1, fake,
                             None, None, fake, 10 ** 6, None)
    assert rc == -1  # gather needs node_inc etc.
    assert b"missing topology" in L.eb_last_error_detail()
    rc = L.eb_dual_volumes(ctypes.byref(sz), ctypes.byref(tp), fake, fake, 1, None, 0,
                           fake, fake, 10 ** 6, None)
    assert rc == -1  # edge mode needs n
    rc = L.eb_set_gather_shape(100, 2, 1)
    assert rc == -1
    sz.dim = 5
    rc = L.eb_directed_areas_backward(ctypes.byref(sz), ctypes.byref(tp), fake, fake,
                                      None, None, None, 0, fake, fake, 10 ** 6, None)
    assert rc == -1


def test_package_import_does_not_touch_gpu():
    import paper_2502_00778_amd as eb
    assert callable(eb.directed_areas)
    assert eb.get_gather_shape()[0] in (64, 128, 256)
