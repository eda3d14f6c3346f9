"""CPU FP64 oracle for the MPCD + rigid-body step (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports it, and it imports nothing from the product.

The arithmetic lives in ``mpcd_oracle.c`` (plain C, FP64, built with
``-ffp-contract=off``).  This module only builds/loads that shared library and
marshals numpy arrays into it.  Section and equation citations refer to
Bush, Palmer, Howard, arXiv 2604.14307.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpcd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NONFINITE, ESCAPE, FIXOVF, RNGLOOP = 1, 2, 4, 8

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, contraction off, no -march, no fast-math."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcSys(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("a", C.c_double),
                ("N", C.c_int64), ("m", C.c_double),
                ("x", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)),
                ("B", C.c_int64),
                ("R", C.POINTER(C.c_double)), ("img", C.POINTER(C.c_int32)),
                ("q", C.POINTER(C.c_double)), ("P", C.POINTER(C.c_double)),
                ("p", C.POINTER(C.c_double)), ("F", C.POINTER(C.c_double)),
                ("T", C.POINTER(C.c_double)),
                ("M", C.POINTER(C.c_double)), ("I", C.POINTER(C.c_double)),
                ("S", C.c_int64), ("site_off", C.POINTER(C.c_int64)),
                ("dhat", C.POINTER(C.c_double)), ("sm", C.POINTER(C.c_double)),
                ("xs", C.POINTER(C.c_double)), ("vs", C.POINTER(C.c_double)),
                ("vpre", C.POINTER(C.c_double)), ("d", C.POINTER(C.c_double))]


class OrcPar(C.Structure):
    _fields_ = [("dt", C.c_double), ("cos_a", C.c_double), ("sin_a", C.c_double),
                ("kT", C.c_double), ("kT_cell", C.c_double),
                ("seed", C.c_uint64), ("replica", C.c_uint64),
                ("thermalize", C.c_int32), ("wca_mode", C.c_int32),
                ("eps", C.c_double), ("sigma", C.c_double), ("delta", C.c_double),
                ("g", C.c_double * 3), ("f_ext", C.c_double * 3)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        u64, i64, dp = C.c_uint64, C.c_int64, C.POINTER(C.c_double)
        sysp, parp = C.POINTER(OrcSys), C.POINTER(OrcPar)
        L.orc_philox.argtypes = [C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]
        L.orc_dlog.restype = C.c_double
        L.orc_dlog.argtypes = [C.c_double]
        L.orc_dsincos.argtypes = [C.c_double, dp, dp]
        L.orc_dlog_n.argtypes = [dp, dp, i64]
        L.orc_dsincos_n.argtypes = [dp, dp, dp, i64]
        L.orc_shift.argtypes = [u64, u64, u64, C.c_double, dp]
        L.orc_site_normals.restype = C.c_uint32
        L.orc_site_normals.argtypes = [u64, u64, u64, u64, dp]
        L.orc_site_normals_n.restype = C.c_uint32
        L.orc_site_normals_n.argtypes = [u64, u64, u64, i64, dp]
        L.orc_cell_axis.restype = C.c_uint32
        L.orc_cell_axis.argtypes = [u64, u64, u64, u64, dp]
        L.orc_cell_axis_n.restype = C.c_uint32
        L.orc_cell_axis_n.argtypes = [u64, u64, u64, i64, dp]
        L.orc_gamma.restype = C.c_uint32
        L.orc_gamma.argtypes = [u64, u64, u64, u64, C.c_double, dp]
        L.orc_gamma_n.restype = C.c_uint32
        L.orc_gamma_n.argtypes = [u64, u64, u64, C.c_double, i64, dp]
        L.orc_cell_draws_n.restype = C.c_uint32
        L.orc_cell_draws_n.argtypes = [u64, u64, u64, C.c_double, i64, dp, dp]
        L.orc_sites_thermalize.restype = C.c_uint32
        L.orc_sites_thermalize.argtypes = [sysp, parp, u64, dp]
        L.orc_bin.restype = C.c_uint32
        L.orc_bin.argtypes = [sysp, dp, C.POINTER(C.c_int32), C.POINTER(i64), C.POINTER(i64)]
        L.orc_collide.restype = C.c_uint32
        L.orc_collide.argtypes = [sysp, parp, u64, C.POINTER(i64), C.POINTER(i64), dp]
        L.orc_sites_to_body.restype = C.c_uint32
        L.orc_sites_to_body.argtypes = [sysp, dp, dp]
        L.orc_body_forces.restype = C.c_uint32
        L.orc_body_forces.argtypes = [sysp, parp]
        L.orc_site_wca_bodies.restype = C.c_uint32
        L.orc_site_wca_bodies.argtypes = [sysp, parp, C.POINTER(i64), i64, dp, dp]
        L.orc_wca_energy.restype = C.c_double
        L.orc_wca_energy.argtypes = [sysp, parp]
        L.orc_body_integrate.restype = C.c_uint32
        L.orc_body_integrate.argtypes = [sysp, parp, dp, dp]
        L.orc_stream_forced.restype = C.c_uint32
        L.orc_stream_forced.argtypes = [sysp, C.c_double, dp]
        L.orc_stream.restype = C.c_uint32
        L.orc_stream.argtypes = [sysp, C.c_double]
        L.orc_step.restype = C.c_uint32
        L.orc_step.argtypes = [sysp, parp, u64]
        L.orc_run.restype = C.c_uint32
        L.orc_run.argtypes = [sysp, parp, u64, i64]
        _lib = L
    return _lib


def _p(a, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct))


# ---------------------------------------------------------------------------
# Primitives (for the pins)

def philox(ctr, key):
    c = (C.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) for x in key])
    o = (C.c_uint64 * 4)()
    lib().orc_philox(c, k, o)
    return [int(x) for x in o]


def dlog(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().orc_dlog_n(_p(x), _p(y), x.size)
    return y


def dsincos(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    s, c = np.empty_like(x), np.empty_like(x)
    lib().orc_dsincos_n(_p(x), _p(s), _p(c), x.size)
    return s, c


def shift(seed, step, replica, a=1.0):
    s = np.zeros(3)
    lib().orc_shift(seed, step, replica, a, _p(s))
    return s


def site_normals(seed, step, replica, n):
    z = np.zeros((n, 3))
    flags = lib().orc_site_normals_n(seed, step, replica, n, _p(z))
    return z, flags


def cell_axes(seed, step, replica, n):
    ax = np.zeros((n, 3))
    flags = lib().orc_cell_axis_n(seed, step, replica, n, _p(ax))
    return ax, flags


def gammas(seed, step, replica, k, n):
    g = np.zeros(n)
    flags = lib().orc_gamma_n(seed, step, replica, k, n, _p(g))
    return g, flags


def cell_draws(seed, step, replica, k, n):
    """Axis and Gamma(k) variate of cells 0..n-1 from their one stream each."""
    ax = np.zeros((n, 3))
    g = np.zeros(n)
    flags = lib().orc_cell_draws_n(seed, step, replica, k, n, _p(ax), _p(g))
    return ax, g, flags


# ---------------------------------------------------------------------------
# Whole-system oracle

def make_par(p: dict, replica: int = 0) -> OrcPar:
    wca = p.get("wca", {"mode": 0})
    return OrcPar(dt=p["dt"], cos_a=p["cos_a"], sin_a=p["sin_a"], kT=p["kT"],
                  kT_cell=p["kT_cell"], seed=p["seed"], replica=replica,
                  thermalize=int(p.get("thermalize", 1)), wca_mode=int(wca.get("mode", 0)),
                  eps=float(wca.get("eps", 0.0)), sigma=float(wca.get("sigma", 0.0)),
                  delta=float(wca.get("delta", 0.0)),
                  g=(C.c_double * 3)(*[float(a) for a in p.get("g", (0.0, 0.0, 0.0))]),
                  f_ext=(C.c_double * 3)(*[float(a) for a in p.get("f_ext", (0.0, 0.0, 0.0))]))


class OracleSystem:
    """One periodic system held in numpy arrays, advanced by the C oracle.

    ``wl`` is a single-system workload dict (see the workload generators):
    component-major arrays ``x, v`` [3,N]; bodies ``R, img, q, P, p, F, T, M, I``;
    sites ``site_off, dhat, sm``.  Arrays are copied.
    """

    KEYS_F = ("x", "v", "R", "q", "P", "p", "F", "T", "M", "I", "dhat", "sm")

    def __init__(self, wl: dict, params: dict, replica: int = 0):
        self.ncell = tuple(int(n) for n in wl["ncell"])
        self.a = float(wl["a"])
        self.m = float(wl["m"])
        for k in self.KEYS_F:
            setattr(self, k, np.ascontiguousarray(np.array(wl[k], dtype=np.float64, copy=True)))
        self.img = np.ascontiguousarray(np.array(wl["img"], dtype=np.int32, copy=True))
        self.site_off = np.ascontiguousarray(np.array(wl["site_off"], dtype=np.int64, copy=True))
        self.N = self.x.shape[1]
        self.B = self.M.shape[0]
        self.S = self.sm.shape[0]
        self.xs = np.zeros((3, self.S))
        self.vs = np.zeros((3, self.S))
        self.vpre = np.zeros((3, self.S))
        self.d = np.zeros((3, self.S))
        self.params = dict(params)
        self.par = make_par(params, replica)
        self.replica = replica
        self._sys = OrcSys(n=(C.c_int32 * 3)(*self.ncell), a=self.a, N=self.N, m=self.m,
                           x=_p(self.x), v=_p(self.v), B=self.B, R=_p(self.R),
                           img=_p(self.img, C.c_int32), q=_p(self.q), P=_p(self.P), p=_p(self.p),
                           F=_p(self.F), T=_p(self.T), M=_p(self.M), I=_p(self.I), S=self.S,
                           site_off=_p(self.site_off, C.c_int64), dhat=_p(self.dhat),
                           sm=_p(self.sm), xs=_p(self.xs), vs=_p(self.vs), vpre=_p(self.vpre),
                           d=_p(self.d))

    @property
    def C(self):
        return self.ncell[0] * self.ncell[1] * self.ncell[2]

    # --- stages -----------------------------------------------------------
    def sites_thermalize(self, step, vt=None):
        vt_p = None
        if vt is not None:
            self._vt = np.ascontiguousarray(vt, dtype=np.float64)
            vt_p = _p(self._vt)
        return lib().orc_sites_thermalize(C.byref(self._sys), C.byref(self.par), step, vt_p)

    def shift(self, step):
        return shift(self.par.seed, step, self.replica, self.a)

    def bin(self, sh):
        sh = np.ascontiguousarray(sh, dtype=np.float64)
        NT = self.N + self.S
        cell = np.zeros(max(NT, 1), dtype=np.int32)
        cs = np.zeros(self.C + 1, dtype=np.int64)
        mem = np.zeros(max(NT, 1), dtype=np.int64)
        flags = lib().orc_bin(C.byref(self._sys), _p(sh), _p(cell, C.c_int32), _p(cs, C.c_int64),
                              _p(mem, C.c_int64))
        return cell[:NT], cs, mem[:NT], flags

    def collide(self, step, cell_start, members, axis=None):
        ax_p = None
        if axis is not None:
            self._ax = np.ascontiguousarray(axis, dtype=np.float64)
            ax_p = _p(self._ax)
        cs = np.ascontiguousarray(cell_start, dtype=np.int64)
        mem = np.ascontiguousarray(members, dtype=np.int64)
        if mem.size == 0:
            mem = np.zeros(1, dtype=np.int64)
        return lib().orc_collide(C.byref(self._sys), C.byref(self.par), step, _p(cs, C.c_int64),
                                 _p(mem, C.c_int64), ax_p)

    def sites_to_body(self):
        J = np.zeros((3, max(self.B, 1)))
        K = np.zeros((3, max(self.B, 1)))
        lib().orc_sites_to_body(C.byref(self._sys), _p(J), _p(K))
        return J[:, :self.B].copy(), K[:, :self.B].copy()

    def body_forces(self):
        return lib().orc_body_forces(C.byref(self._sys), C.byref(self.par))

    def site_wca_bodies(self, idx):
        """Mode 2 force and torque ([3][n] each) of the listed bodies only."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        F = np.zeros((3, max(len(idx), 1)))
        T = np.zeros((3, max(len(idx), 1)))
        flags = lib().orc_site_wca_bodies(C.byref(self._sys), C.byref(self.par), _p(idx, C.c_int64), len(idx),
                                          _p(F), _p(T))
        return F[:, :len(idx)].copy(), T[:, :len(idx)].copy(), flags

    def rnemd(self, y0, y1, dy, target, npairs, dp=0.0, tag=None):
        """One reverse nonequilibrium exchange (Sec. III.B); returns the updated
        momentum accumulator and the number of pairs swapped."""
        L = lib()
        if not hasattr(L, "_rnemd_ready"):
            L.orc_rnemd.restype = C.c_uint32
            L.orc_rnemd.argtypes = [C.POINTER(OrcSys), C.POINTER(C.c_int32), C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
            L._rnemd_ready = True
        acc = C.c_double(dp)
        ns = C.c_int64(0)
        tg = None
        if tag is not None:
            self._tag = np.ascontiguousarray(tag, dtype=np.int32)
            tg = _p(self._tag, C.c_int32)
        L.orc_rnemd(C.byref(self._sys), tg, y0, y1, dy, target, npairs, C.byref(acc), C.byref(ns))
        return acc.value, ns.value

    def wca_energy(self):
        """Total WCA potential energy of the current body poses, Eq. (1)."""
        return lib().orc_wca_energy(C.byref(self._sys), C.byref(self.par))

    def body_integrate(self, J, K):
        J = np.ascontiguousarray(J, dtype=np.float64)
        K = np.ascontiguousarray(K, dtype=np.float64)
        if J.size == 0:
            J = np.zeros((3, 1)); K = np.zeros((3, 1))
        return lib().orc_body_integrate(C.byref(self._sys), C.byref(self.par), _p(J), _p(K))

    def stream(self, dt=None, g=None):
        dt = self.par.dt if dt is None else dt
        if g is None:
            return lib().orc_stream(C.byref(self._sys), dt)
        gg = np.ascontiguousarray(g, dtype=np.float64)
        return lib().orc_stream_forced(C.byref(self._sys), dt, _p(gg))

    def step(self, step):
        return lib().orc_step(C.byref(self._sys), C.byref(self.par), step)

    def run(self, step0, nsteps):
        return lib().orc_run(C.byref(self._sys), C.byref(self.par), step0, nsteps)

    # --- observables ------------------------------------------------------
    def body_velocity(self):
        return self.P / self.M[None, :]

    def body_angmom_bodyframe(self):
        """Lhat_k = 1/2 p . P_k q (Miller et al.)."""
        q, p = self.q, self.p
        P1 = np.stack([-q[1], q[0], q[3], -q[2]])
        P2 = np.stack([-q[2], -q[3], q[0], q[1]])
        P3 = np.stack([-q[3], q[2], -q[1], q[0]])
        return 0.5 * np.stack([(p * P1).sum(0), (p * P2).sum(0), (p * P3).sum(0)])

    def state(self):
        return {k: getattr(self, k).copy() for k in
                ("x", "v", "R", "img", "q", "P", "p", "F", "T", "xs", "vs", "vpre", "d")}


# ---------------------------------------------------------------------------
# Harmonic-bond comparator (Sec. II.B.1)

class OrcHarm(C.Structure):
    _fields_ = [("B", C.c_int64), ("xc", C.POINTER(C.c_double)), ("vc", C.POINTER(C.c_double)),
                ("imgc", C.POINTER(C.c_int32)), ("imgs", C.POINTER(C.c_int32)),
                ("mc", C.c_double), ("kb", C.c_double),
                ("site_off", C.POINTER(C.c_int64)), ("site_body", C.POINTER(C.c_int32)),
                ("adj_off", C.POINTER(C.c_int64)), ("adj", C.POINTER(C.c_int32)),
                ("adj_r0", C.POINTER(C.c_double)), ("rc0", C.POINTER(C.c_double)),
                ("fs", C.POINTER(C.c_double)), ("fc", C.POINTER(C.c_double))]


def _harm_lib():
    L = lib()
    if not hasattr(L, "_harm_ready"):
        sysp, parp, hp = C.POINTER(OrcSys), C.POINTER(OrcPar), C.POINTER(OrcHarm)
        L.orc_harm_forces.restype = C.c_uint32
        L.orc_harm_forces.argtypes = [sysp, hp, parp]
        L.orc_harm_md.restype = C.c_uint32
        L.orc_harm_md.argtypes = [sysp, hp, parp, C.c_double, C.c_int64]
        L.orc_harm_step.restype = C.c_uint32
        L.orc_harm_step.argtypes = [sysp, hp, parp, C.c_uint64, C.c_double, C.c_int64]
        L.orc_harm_energy.restype = C.c_double
        L.orc_harm_energy.argtypes = [sysp, hp, parp]
        L._harm_ready = True
    return L


class HarmonicOracle:
    """The harmonic-bond model of one system (see workloads.harmonic_from_rigid),
    advanced by the C oracle: solvent x, v; surface sites xs, vs (they collide);
    centre sites xc, vc; forces fs, fc."""

    def __init__(self, hw: dict, params: dict, replica: int = 0):
        f64 = lambda a: np.ascontiguousarray(np.array(a, dtype=np.float64, copy=True))
        self.ncell = tuple(int(n) for n in hw["ncell"])
        self.a, self.m = float(hw["a"]), float(hw["m"])
        self.x, self.v = f64(hw["x"]), f64(hw["v"])
        self.xs, self.vs, self.sm = f64(hw["xs"]), f64(hw["vs"]), f64(hw["sm"])
        self.xc, self.vc = f64(hw["xc"]), f64(hw["vc"])
        self.imgs = np.ascontiguousarray(np.array(hw["imgs"], dtype=np.int32, copy=True))
        self.imgc = np.ascontiguousarray(np.array(hw["imgc"], dtype=np.int32, copy=True))
        self.site_off = np.ascontiguousarray(np.array(hw["site_off"], dtype=np.int64))
        self.site_body = np.ascontiguousarray(np.array(hw["site_body"], dtype=np.int32))
        self.adj_off = np.ascontiguousarray(np.array(hw["adj_off"], dtype=np.int64))
        self.adj = np.ascontiguousarray(np.array(hw["adj"], dtype=np.int32))
        self.adj_r0, self.rc0 = f64(hw["adj_r0"]), f64(hw["rc0"])
        self.N, self.S, self.B = self.x.shape[1], self.xs.shape[1], self.xc.shape[1]
        self.fs, self.fc = np.zeros((3, self.S)), np.zeros((3, self.B))
        self._dummy = np.zeros(8)
        self._zero_off = np.zeros(1, dtype=np.int64)
        self._zero_i = np.zeros(3, dtype=np.int32)
        self._vpre, self._d = np.zeros((3, self.S)), np.zeros((3, self.S))
        self.par = make_par(params, replica)
        d = self._dummy
        self._sys = OrcSys(n=(C.c_int32 * 3)(*self.ncell), a=self.a, N=self.N, m=self.m,
                           x=_p(self.x), v=_p(self.v), B=0, R=_p(d), img=_p(self._zero_i, C.c_int32),
                           q=_p(d), P=_p(d), p=_p(d), F=_p(d), T=_p(d), M=_p(d), I=_p(d), S=self.S,
                           site_off=_p(self._zero_off, C.c_int64), dhat=_p(self._d), sm=_p(self.sm),
                           xs=_p(self.xs), vs=_p(self.vs), vpre=_p(self._vpre), d=_p(self._d))
        self._h = OrcHarm(B=self.B, xc=_p(self.xc), vc=_p(self.vc), imgc=_p(self.imgc, C.c_int32),
                          imgs=_p(self.imgs, C.c_int32), mc=float(hw["mc"]), kb=float(hw["kb"]),
                          site_off=_p(self.site_off, C.c_int64), site_body=_p(self.site_body, C.c_int32),
                          adj_off=_p(self.adj_off, C.c_int64), adj=_p(self.adj, C.c_int32),
                          adj_r0=_p(self.adj_r0), rc0=_p(self.rc0), fs=_p(self.fs), fc=_p(self.fc))
        self.mc = float(hw["mc"])

    def forces(self):
        return _harm_lib().orc_harm_forces(C.byref(self._sys), C.byref(self._h), C.byref(self.par))

    def md(self, dt, nsub):
        return _harm_lib().orc_harm_md(C.byref(self._sys), C.byref(self._h), C.byref(self.par), dt, nsub)

    def step(self, step, dt_md, nsub):
        return _harm_lib().orc_harm_step(C.byref(self._sys), C.byref(self._h), C.byref(self.par), step, dt_md,
                                         nsub)

    def energy(self):
        return _harm_lib().orc_harm_energy(C.byref(self._sys), C.byref(self._h), C.byref(self.par))
