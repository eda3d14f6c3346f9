"""The reverse nonequilibrium exchange without allocation
(mpcd_rnemd_exchange_noalloc, a static device array per GPU) against the
workspace form (mpcd_rnemd_exchange), both through the C ABI: the same
velocities bit for bit, the same moved momentum, the same flags.  Two calls in
a row, the second on a smaller system, so the second finds the first call's
lists in the array; FP64 and FP32.  The workspace form itself is held to the
oracle bit for bit by the parity tests."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2604_14307_amd import lib as L
from paper_2604_14307_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ptr(t):
    return C.c_void_p(t.data_ptr())


def system(shape, seed, prec):
    from paper_2604_14307_amd.sim import GPUSystem
    wl = W.make_system(shape, 5, [], [], np.zeros((0, 4)), np.random.default_rng(seed))
    par = W.srd_params(seed, kT_cell=1.0)
    g = GPUSystem(wl, par, prec=prec)
    g.step(3)  # velocities after a few collisions
    torch.cuda.synchronize()
    return g


def both_forms(g, r):
    """One exchange by each entry point from the same velocities."""
    lib = L.load()
    st = g.stream
    v_ws, v_na = g.v.clone(), g.v.clone()
    dp_ws = torch.zeros(1, dtype=torch.float64, device=g.device)
    dp_na = torch.zeros(1, dtype=torch.float64, device=g.device)
    status = torch.zeros(1, dtype=torch.int32, device=g.device)
    torch.cuda.synchronize()
    rc = lib.mpcd_rnemd_exchange(st, C.byref(g.csys), ptr(g.x), ptr(v_ws), ptr(g.tag), C.byref(r), ptr(dp_ws),
                                 ptr(g.ws), g.ws_bytes)
    L.check(rc, "mpcd_rnemd_exchange")
    rc = lib.mpcd_rnemd_exchange_noalloc(st, C.byref(g.csys), ptr(g.x), ptr(v_na), ptr(g.tag), C.byref(r),
                                         ptr(dp_na), ptr(status))
    L.check(rc, "mpcd_rnemd_exchange_noalloc")
    torch.cuda.synchronize()
    return v_ws, v_na, float(dp_ws.cpu()[0]), float(dp_na.cpu()[0]), int(status.cpu()[0]), g.status()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_exchange_equals_workspace_exchange(prec):
    big = system((16, 24, 16), 301, prec)
    small = system((8, 12, 8), 302, prec)
    cases = [(big, L.MpcdRnemd(y0=0.0, y1=12.0, dy=1.0, target=0.5, npairs=100)),
             (small, L.MpcdRnemd(y0=1.0, y1=7.0, dy=1.0, target=0.5, npairs=37))]
    for n, (g, r) in enumerate(cases):
        say("no-alloc exchange %s, call %d, N %d, npairs %d" % (prec, n, g.N, r.npairs))
        v_ws, v_na, dp_ws, dp_na, flags_na, flags_ws = both_forms(g, r)
        assert torch.equal(v_ws, v_na)
        assert not torch.equal(v_ws, g.v)  # the exchange moved something
        assert dp_na == dp_ws != 0.0
        assert flags_na == 0 and flags_ws == 0
    # the first system again, after the smaller call left its lists behind
    g, r = cases[0]
    v_ws, v_na, dp_ws, dp_na, flags_na, _ = both_forms(g, r)
    assert torch.equal(v_ws, v_na) and dp_na == dp_ws and flags_na == 0


def test_noalloc_exchange_rejects_bad_arguments():
    """Host-side checks: too many pairs for the array, no status word, more
    than one system (nothing is launched)."""
    lib = L.load()
    g = system((8, 12, 8), 303, "f64")
    dp = torch.zeros(1, dtype=torch.float64, device=g.device)
    status = torch.zeros(1, dtype=torch.int32, device=g.device)
    args = (g.stream, C.byref(g.csys), ptr(g.x), ptr(g.v), ptr(g.tag))
    too_many = L.MpcdRnemd(y0=0.0, y1=6.0, dy=1.0, target=0.5, npairs=1025)
    assert lib.mpcd_rnemd_exchange_noalloc(*args, C.byref(too_many), ptr(dp), ptr(status)) == -1
    ok = L.MpcdRnemd(y0=0.0, y1=6.0, dy=1.0, target=0.5, npairs=10)
    assert lib.mpcd_rnemd_exchange_noalloc(*args, C.byref(ok), ptr(dp), C.c_void_p(0)) == -1
    two = L.MpcdSys.from_buffer_copy(g.csys)
    two.nsys = 2
    assert lib.mpcd_rnemd_exchange_noalloc(g.stream, C.byref(two), ptr(g.x), ptr(g.v), ptr(g.tag), C.byref(ok),
                                           ptr(dp), ptr(status)) == -4
    torch.cuda.synchronize()
    assert float(dp.cpu()[0]) == 0.0 and int(status.cpu()[0]) == 0
