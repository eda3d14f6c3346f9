"""The C ABI: libmpcd.so loads and exports every function include/mpcd.h
declares; host-side size queries and argument validation work without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2604_14307_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:int|size_t|void)\s+\**\s*(\w+)\s*\(", src, flags=re.M))
    return names


def test_every_declared_symbol_is_exported():
    L = lib.load()
    names = declared_functions()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(lib.EXPORTS) == names


def sys_desc(**kw):
    d = dict(nsys=1, prec=lib.MPCD_F64, a=1.0, m_solvent=1.0, n_solvent=5000, n_sites=100,
             n_bodies=1, n_cells=1000)
    d.update(kw)
    return lib.MpcdSys(**d)


def test_workspace_size_and_offsets():
    L = lib.load()
    s = sys_desc()
    nb = L.mpcd_workspace_bytes(C.byref(s))
    offs = (C.c_int64 * 8)()
    assert L.mpcd_workspace_offsets(C.byref(s), offs) == 0
    o = list(offs)
    assert all(x % 256 == 0 for x in o) and len(set(o)) == 8 and max(o) < nb
    # cell_start holds C+1 int32, perm holds N+S int32
    assert nb >= 4 * (1001 + 1000 + 3 * 5100) + 2 * 3 * 8 * 100
    big = sys_desc(n_solvent=80_000_000, n_sites=4_244_200, n_bodies=21221, n_cells=8_000_000)
    assert L.mpcd_workspace_bytes(C.byref(big)) > L.mpcd_workspace_bytes(C.byref(s))


@pytest.mark.parametrize("bad", [dict(nsys=0), dict(a=0.0), dict(m_solvent=-1.0), dict(n_cells=0),
                                 dict(n_solvent=2 ** 31), dict(prec=7)])
def test_invalid_sizes_are_rejected(bad):
    L = lib.load()
    assert L.mpcd_workspace_bytes(C.byref(sys_desc(**bad))) == 0


def test_invalid_pointers_rejected_before_any_launch():
    L = lib.load()
    s = sys_desc()  # device arrays left NULL
    assert L.mpcd_stream(None, C.byref(s), None, None, 0.1, None, None, 0) == -1
    assert L.mpcd_advance_step(None, None) == -1
    assert L.mpcd_graph_destroy(None) == -1
    f = C.c_uint32(0)
    assert L.mpcd_status(None, None, 0, C.byref(f)) == -1


def brick_enumeration(ncells, b=(8, 8, 4)):
    """Storage position of every cell (canonical order), by enumerating the
    bricks x-fastest and each brick's cells x-fastest."""
    out, off = [], 0
    for nx, ny, nz in ncells:
        pos = np.empty(nx * ny * nz, dtype=np.int64)
        q = off
        for z0 in range(0, nz, b[2]):
            for y0 in range(0, ny, b[1]):
                for x0 in range(0, nx, b[0]):
                    for jz in range(z0, min(z0 + b[2], nz)):
                        for jy in range(y0, min(y0 + b[1], ny)):
                            for jx in range(x0, min(x0 + b[0], nx)):
                                pos[(jz * ny + jy) * nx + jx] = q
                                q += 1
        out.append(pos)
        off += nx * ny * nz
    return np.concatenate(out)


@pytest.mark.parametrize("ncells", [[(10, 10, 10)], [(7, 9, 11)], [(60, 60, 60)], [(1, 1, 1)],
                                    [(12, 17, 24), (13, 13, 13), (3, 20, 5)]])
def test_cell_order_is_the_brick_enumeration(ncells):
    L = lib.load()
    nc = np.ascontiguousarray(np.array(ncells, dtype=np.int32).reshape(-1))
    C_tot = int(sum(a * b * c for a, b, c in ncells))
    pos = np.empty(C_tot, dtype=np.int64)
    rc = L.mpcd_cell_order(len(ncells), nc.ctypes.data_as(C.POINTER(C.c_int32)),
                             pos.ctypes.data_as(C.POINTER(C.c_int64)))
    assert rc == 0
    assert np.array_equal(pos, brick_enumeration(ncells))


def test_cell_order_rejects_bad_boxes():
    L = lib.load()
    pos = np.empty(8, dtype=np.int64)
    for bad in ([2, 2, 0], [2, -1, 2]):
        nc = np.array(bad, dtype=np.int32)
        assert L.mpcd_cell_order(1, nc.ctypes.data_as(C.POINTER(C.c_int32)),
                                   pos.ctypes.data_as(C.POINTER(C.c_int64))) == -1


def test_tile_shape_follows_the_tuning():
    L = lib.load()
    s = sys_desc(prec=lib.MPCD_F32, n_solvent=1_080_000, n_sites=38_200, n_bodies=191, n_cells=216_000)
    out = (C.c_int32 * 4)()
    assert L.mpcd_tile_shape(C.byref(s), None, out) == 0
    items, cpb, cap, ntiles = list(out)
    # default: 4 items per thread, cells per tile the largest power of two whose
    # average membership (5.18 per cell) stays within 70% of 1024
    assert (items, cap) == (4, 1024) and cpb == 128 and ntiles == 216_000 // 128 + 1
    t = lib.MpcdTune(8, 85, 2)
    assert L.mpcd_tile_shape(C.byref(s), C.byref(t), out) == 0
    assert list(out)[:3] == [8, 256, 2048]
    for bad in ((3, 0, 0), (0, 5, 0), (0, 101, 0), (0, 0, 17), (1, 0, 0), (0, 0, 0, 2), (0, 0, 0, 0, 4)):
        assert L.mpcd_tile_shape(C.byref(s), C.byref(lib.MpcdTune(*bad)), out) == -1
    s64 = sys_desc(prec=lib.MPCD_F64)
    assert L.mpcd_tile_shape(C.byref(s64), C.byref(lib.MpcdTune(1, 0, 0)), out) == 0 and out[0] == 1
    assert L.mpcd_tile_shape(C.byref(s64), C.byref(lib.MpcdTune(8, 0, 0)), out) == -1


def binned_layout(systems, prec=None):
    """mpcd_binned_layout of workload dicts (host only)."""
    L = lib.load()
    prec = lib.MPCD_F32 if prec is None else prec
    nc = np.array([s["ncell"] for s in systems], dtype=np.int32).reshape(-1)
    Ns = [s["x"].shape[1] for s in systems]
    Ss = [len(s["sm"]) for s in systems]
    so = np.concatenate([[0], np.cumsum(Ns)]).astype(np.int64)
    ss = np.concatenate([[0], np.cumsum(Ss)]).astype(np.int64)
    C_ = int(sum(int(np.prod(s["ncell"])) for s in systems))
    s = sys_desc(nsys=len(systems), prec=prec, n_solvent=int(so[-1]), n_sites=int(ss[-1]),
                 n_bodies=sum(len(x["M"]) for x in systems), n_cells=C_)
    b = lib.MpcdBinned()
    rc = L.mpcd_binned_layout(C.byref(s), nc.ctypes.data_as(C.POINTER(C.c_int32)),
                              so.ctypes.data_as(C.POINTER(C.c_int64)), ss.ctypes.data_as(C.POINTER(C.c_int64)),
                              C.byref(b))
    return rc, b, int(so[-1])


def test_binned_layout_plan():
    from paper_2604_14307_amd import workloads as W
    systems = W.batched_replicas(nrep=8, seed=4)[0]
    rc, b, N = binned_layout(systems)
    assert rc == 0
    # bricks of 8 x 8 x 4 cells at 5 per cell; each region holds the brick's
    # own sub-region (1280 + 6 sigma + 16 for a full brick) and one per
    # neighbouring writer (a layer of 1.25 cells): about 4.5 N slots in all
    ncells = [int(np.prod(s["ncell"])) for s in systems]
    assert b.nbricks >= sum(c // 256 for c in ncells)
    assert 3.0 * N < b.capacity < 6.0 * N
    assert b.items == (7 if b.nbricks >= 4096 else 4) and b.ws_bytes > 0 and b.site_slots > 0
    # a denser system gets smaller bricks, not more members per block
    wl = W.make_system((16, 16, 16), 10, [], np.zeros((0, 3)), np.zeros((0, 4)), np.random.default_rng(1))
    rc, b10, N10 = binned_layout([wl])
    assert rc == 0 and b10.nbricks == 32  # 128-cell bricks
    # inconsistent offsets are rejected
    s = sys_desc(prec=lib.MPCD_F32)
    nc = np.array([10, 10, 10], dtype=np.int32)
    so = np.array([0, 4999], dtype=np.int64)
    ss = np.array([0, 100], dtype=np.int64)
    bb = lib.MpcdBinned()
    assert lib.load().mpcd_binned_layout(C.byref(s), nc.ctypes.data_as(C.POINTER(C.c_int32)),
                                         so.ctypes.data_as(C.POINTER(C.c_int64)),
                                         ss.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(bb)) == -1  # MPCD_EINVAL
