"""The C ABI: libmpcd.so loads and exports every function include/mpcd.h
declares; host-side size queries and argument validation work without a GPU."""
import ctypes as C
import os
import re

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
