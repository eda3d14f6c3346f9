"""Device-resident system state and calls into libmpcd.so.

``GPUSystem`` packs one or more independent periodic systems (workload dicts
from :mod:`paper_2604_14307_amd.workloads`) into torch device tensors, owns the
workspace and the device step counter, and exposes each C-ABI entry point as a
method.  PyTorch provides device memory and the stream; all arithmetic of the
step runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import lib as L


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


class GPUSystem:
    def __init__(self, systems, params: dict, prec: str = "f64", replica0: int = 0,
                 device: str = "cuda:0", fuse_stream: bool = True, out_of_place: bool = True,
                 layout: str = "dense"):
        self.lib = L.load()
        if isinstance(systems, dict):
            systems = [systems]
        self.nsys = len(systems)
        self.device = torch.device(device)
        self.prec = L.MPCD_F64 if prec == "f64" else L.MPCD_F32
        self.real = torch.float64 if self.prec == L.MPCD_F64 else torch.float32
        self.params = dict(params)
        a = float(systems[0]["a"])
        m = float(systems[0]["m"])
        for s in systems:
            if float(s["a"]) != a or float(s["m"]) != m:
                raise ValueError("all systems must share the cell edge and solvent mass")
        dev = self.device
        ncell = np.array([s["ncell"] for s in systems], dtype=np.int32).reshape(-1)
        Ns = [s["x"].shape[1] for s in systems]
        Cs = [int(np.prod(s["ncell"])) for s in systems]
        Bs = [s["M"].shape[0] for s in systems]
        Ss = [s["sm"].shape[0] for s in systems]
        self.N, self.C, self.B, self.S = sum(Ns), sum(Cs), sum(Bs), sum(Ss)
        self.solv_off_h = np.concatenate([[0], np.cumsum(Ns)]).astype(np.int64)
        self.cell_off_h = np.concatenate([[0], np.cumsum(Cs)]).astype(np.int64)
        self.body_off_h = np.concatenate([[0], np.cumsum(Bs)]).astype(np.int64)
        self.site_sys_off_h = np.concatenate([[0], np.cumsum(Ss)]).astype(np.int64)
        self.ncell_h = ncell.reshape(-1, 3)

        def cat(key, dtype, rows):
            if sum(s[key].shape[-1] for s in systems) == 0:
                return torch.zeros((rows, 0), dtype=dtype, device=dev)
            arr = np.concatenate([np.asarray(s[key]).reshape(rows, -1) for s in systems], axis=1)
            return torch.tensor(arr, dtype=dtype, device=dev).contiguous()

        def cat1(key, dtype):
            arr = np.concatenate([np.asarray(s[key]).reshape(-1) for s in systems])
            return torch.tensor(arr, dtype=dtype, device=dev).contiguous()

        self.ncell = torch.tensor(ncell, dtype=torch.int32, device=dev)
        self.solv_off = torch.tensor(self.solv_off_h, device=dev)
        self.cell_off = torch.tensor(self.cell_off_h, device=dev)
        self.body_off = torch.tensor(self.body_off_h, device=dev)
        self.x = cat("x", self.real, 3)
        self.v = cat("v", self.real, 3)
        # solvent identities (global index in packing order); the storage
        # order changes (out-of-place steps, reorder) carry them along
        self.tag = torch.arange(self.N, dtype=torch.int32, device=dev)
        # out-of-place steps write the solvent in cell order into a second set
        # of arrays; the two sets swap roles after every step
        self.out_of_place = bool(out_of_place) and bool(fuse_stream)
        if self.out_of_place:
            self.x2 = torch.empty_like(self.x)
            self.v2 = torch.empty_like(self.v)
            self.tag2 = torch.empty_like(self.tag)
        self.pos = cat("R", torch.float64, 3)
        self.image = cat("img", torch.int32, 3)
        self.quat = cat("q", torch.float64, 4)
        self.mom = cat("P", torch.float64, 3)
        self.angmom = cat("p", torch.float64, 4)
        self.force = cat("F", torch.float64, 3)
        self.torque = cat("T", torch.float64, 3)
        self.mass = cat1("M", torch.float64)
        self.inertia = cat("I", torch.float64, 3)
        site_off, site_body, base, bbase = [0], [], 0, 0
        for s in systems:
            so = np.asarray(s["site_off"], dtype=np.int64)
            site_off.extend((so[1:] + base).tolist())
            for b in range(len(so) - 1):
                site_body.extend([bbase + b] * int(so[b + 1] - so[b]))
            base += int(so[-1])
            bbase += len(so) - 1
        self.site_off = torch.tensor(np.array(site_off, dtype=np.int64), device=dev)
        self.site_body = torch.tensor(np.array(site_body, dtype=np.int32), device=dev)
        self.site_d = cat("dhat", torch.float64, 3)
        self.site_m = cat1("sm", torch.float64)
        self.xs = torch.zeros((3, self.S), dtype=self.real, device=dev)
        self.vs = torch.zeros((3, self.S), dtype=self.real, device=dev)
        self.J = torch.zeros((3, self.B), dtype=torch.float64, device=dev)
        self.K = torch.zeros((3, self.B), dtype=torch.float64, device=dev)
        self.d_step = torch.zeros(1, dtype=torch.int64, device=dev)

        self.csys = L.MpcdSys(nsys=self.nsys, prec=self.prec, a=a, m_solvent=m, n_solvent=self.N,
                              n_sites=self.S, n_bodies=self.B, n_cells=self.C, replica0=replica0,
                              ncell=_ptr(self.ncell), solv_off=_ptr(self.solv_off),
                              cell_off=_ptr(self.cell_off), body_off=_ptr(self.body_off))
        self.ws_bytes = int(self.lib.mpcd_workspace_bytes(C.byref(self.csys)))
        if self.ws_bytes == 0:
            raise L.MpcdError("invalid system description")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        offs = (C.c_int64 * 8)()
        L.check(self.lib.mpcd_workspace_offsets(C.byref(self.csys), offs), "mpcd_workspace_offsets")
        self.ws_off = dict(zip(("status", "shift", "cell_start", "perm", "cellid", "slot", "site_d", "vpre"),
                               [int(o) for o in offs]))
        self.cbodies = L.MpcdBodies(
            pos=_ptr(self.pos), image=_ptr(self.image), quat=_ptr(self.quat), mom=_ptr(self.mom),
            angmom=_ptr(self.angmom), force=_ptr(self.force), torque=_ptr(self.torque),
            mass=_ptr(self.mass), inertia=_ptr(self.inertia), site_off=_ptr(self.site_off),
            site_body=_ptr(self.site_body), site_d=_ptr(self.site_d), site_m=_ptr(self.site_m))
        w = self.params.get("wca", {"mode": 0})
        # site-site WCA: bound on a site's distance from its body centre
        dh = [np.asarray(s["dhat"]) for s in systems if np.asarray(s["dhat"]).size]
        reach = max(float(np.sqrt((d ** 2).sum(0)).max()) for d in dh) * (1.0 + 1e-9) if dh else 0.0
        self.cwca = L.MpcdWca(mode=int(w.get("mode", 0)), eps=float(w.get("eps", 0.0)),
                              sigma=float(w.get("sigma", 0.0)), delta=float(w.get("delta", 0.0)),
                              reach=float(w.get("reach", reach)))
        self.fuse_stream = bool(fuse_stream)
        # optional reverse nonequilibrium exchange after every step
        self.rnemd = None
        self.rnemd_dp = torch.zeros(1, dtype=torch.float64, device=dev)
        # launch shapes (zero: the library's defaults); results do not depend on them
        self.tuning = L.MpcdTune(0, 0, 0, 0, 0)
        self.ws_init()
        self._graph = None
        self._state = self._STATE
        self.layout = layout
        self.binned = None
        if layout == "binned":
            self._setup_binned()
        elif layout != "dense":
            raise ValueError("layout must be 'dense' or 'binned'")
        # the uploads, initialisation and packing ran on the current stream:
        # wait for them, so that the system can be stepped on any stream
        torch.cuda.synchronize(self.device)

    def _host_offsets(self):
        nc = np.ascontiguousarray(self.ncell_h.reshape(-1), dtype=np.int32)
        so = np.ascontiguousarray(self.solv_off_h, dtype=np.int64)
        ss = np.ascontiguousarray(self.site_sys_off_h, dtype=np.int64)
        return nc, so, ss, (nc.ctypes.data_as(C.POINTER(C.c_int32)), so.ctypes.data_as(C.POINTER(C.c_int64)),
                            ss.ctypes.data_as(C.POINTER(C.c_int64)))

    def _setup_binned(self):
        """The binned solvent layout (see mpcd_binned_layout): solvent in
        per-brick regions of the step's grid, double-buffered."""
        if not self.out_of_place:
            raise ValueError("the binned layout steps out of place")
        nc, so, ss, hp = self._host_offsets()
        b = L.MpcdBinned()
        L.check(self.lib.mpcd_binned_layout(C.byref(self.csys), *hp, C.byref(b)), "mpcd_binned_layout")
        self.bws = torch.empty(int(b.ws_bytes), dtype=torch.uint8, device=self.device)
        b.ws = _ptr(self.bws)
        self.binned = b
        L.check(self.lib.mpcd_binned_init(self.stream, C.byref(self.csys), *hp, C.byref(b)), "mpcd_binned_init")
        cap = int(b.capacity)
        xd, vd, td = self.x, self.v, self.tag
        # x, x2: the solvent records of the current and the next step (FP32: 7
        # values each, position, identity bits, velocity; FP64: 8, with one
        # unused); no v, tag
        rec = 8 if self.prec == L.MPCD_F64 else 7
        self.x = torch.zeros((cap, rec), dtype=self.real, device=self.device)
        self.x2 = torch.zeros_like(self.x)
        self.v = self.v2 = self.tag = self.tag2 = None
        self._pack(xd, vd, td)
        self._state = tuple(k for k in self._STATE if k not in ("v", "tag")) + ("bws",)

    def _pack(self, xd, vd, td):
        L.check(self.lib.mpcd_binned_pack(self.stream, C.byref(self.csys), _ptr(xd), _ptr(vd), _ptr(td), _ptr(self.x),
                                          self.params["seed"], _ptr(self.d_step), _ptr(self.ws), self.ws_bytes,
                                          C.byref(self.binned)), "mpcd_binned_pack")

    def dense_solvent(self):
        """(x [3,N], v [3,N], tag [N]) of the current solvent as device tensors:
        the arrays themselves (dense layout) or, for the binned layout, a copy
        in identity order."""
        if self.binned is None:
            return self.x, self.v, self.tag
        # a particle missing from the binned arrays would stay NaN (tag -1)
        xd = torch.full((3, self.N), float("nan"), dtype=self.real, device=self.device)
        vd = torch.full((3, self.N), float("nan"), dtype=self.real, device=self.device)
        td = torch.full((self.N,), -1, dtype=torch.int32, device=self.device)
        L.check(self.lib.mpcd_binned_unpack(self.stream, C.byref(self.csys), _ptr(self.x), _ptr(xd), _ptr(vd),
                                            _ptr(td), _ptr(self.d_step), _ptr(self.ws), self.ws_bytes,
                                            C.byref(self.binned)), "mpcd_binned_unpack")
        return xd, vd, td

    # ------------------------------------------------------------------
    @property
    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def ws_init(self):
        L.check(self.lib.mpcd_ws_init(self.stream, C.byref(self.csys), _ptr(self.ws), self.ws_bytes),
                "mpcd_ws_init")

    def set_step(self, n: int):
        if self.binned is None:
            self.d_step.fill_(int(n))
            return
        # the binned solvent lies in the bricks of its step's grid: repack
        xd, vd, td = self.dense_solvent()
        self.d_step.fill_(int(n))
        self._pack(xd, vd, td)

    def step_args(self, reorder_every: int = 0) -> L.MpcdStepArgs:
        p = self.params
        par = L.MpcdParams(dt=p["dt"], cos_a=p["cos_a"], sin_a=p["sin_a"], kT=p["kT"], kT_cell=p["kT_cell"],
                           seed=p["seed"], thermalize=int(p.get("thermalize", 1)),
                           fuse_stream=int(self.fuse_stream), wca=self.cwca, g=self._vec("g"),
                           f_ext=self._vec("f_ext"), tune=self.tuning)
        out = self.out_of_place
        self._args = L.MpcdStepArgs(sys=C.pointer(self.csys), bodies=self.cbodies, x=_ptr(self.x), v=_ptr(self.v),
                                    tag=_ptr(self.tag), xs=_ptr(self.xs), vs=_ptr(self.vs), J=_ptr(self.J),
                                    K=_ptr(self.K), d_step=_ptr(self.d_step), ws=_ptr(self.ws),
                                    ws_bytes=self.ws_bytes, par=par, reorder_every=int(reorder_every),
                                    x_out=_ptr(self.x2) if out else C.c_void_p(0),
                                    v_out=_ptr(self.v2) if out else C.c_void_p(0),
                                    tag_out=_ptr(self.tag2) if out else C.c_void_p(0),
                                    rnemd=C.pointer(self.rnemd) if self.rnemd is not None else None,
                                    rnemd_dp=_ptr(self.rnemd_dp),
                                    binned=C.pointer(self.binned) if self.binned is not None else None)
        return self._args

    def set_tuning(self, tile_items: int = 0, tile_fill: int = 0, draw_cells: int = 0, draws_inline: int = 0,
                   overlap: int = 0):
        """Launch shapes of the step (see mpcd_tune); 0 keeps a default."""
        self.tuning = L.MpcdTune(int(tile_items), int(tile_fill), int(draw_cells), int(draws_inline), int(overlap))
        self.tile_shape()  # validates

    def tile_shape(self, tune=None):
        """(items per thread, cells per tile, member capacity, tiles) of a tuning."""
        out = (C.c_int32 * 4)()
        t = self.tuning if tune is None else L.MpcdTune(*[int(a) for a in tune])
        L.check(self.lib.mpcd_tile_shape(C.byref(self.csys), C.byref(t), out), "mpcd_tile_shape")
        return tuple(out)

    _STATE = ("x", "v", "tag", "xs", "vs", "pos", "image", "quat", "mom", "angmom", "force", "torque", "J", "K",
              "d_step", "rnemd_dp")

    def snapshot(self):
        """Device copies of the whole simulation state (for timing runs).  Waits
        for all work on the device first: steps may still run on another stream."""
        torch.cuda.synchronize(self.device)
        snap = {k: getattr(self, k).clone() for k in self._state}
        torch.cuda.synchronize(self.device)
        return snap

    def restore(self, snap):
        torch.cuda.synchronize(self.device)
        for k in self._state:
            getattr(self, k).copy_(snap[k])
        torch.cuda.synchronize(self.device)

    def set_rnemd(self, y0, y1, dy=1.0, target=0.5, npairs=100):
        """Exchange after every step (Sec. III.B); None-like npairs=0 turns it off."""
        self.rnemd = L.MpcdRnemd(y0=float(y0), y1=float(y1), dy=float(dy), target=float(target),
                                 npairs=int(npairs)) if npairs else None

    def rnemd_exchange(self, y0, y1, dy=1.0, target=0.5, npairs=100):
        r = L.MpcdRnemd(y0=float(y0), y1=float(y1), dy=float(dy), target=float(target), npairs=int(npairs))
        L.check(self.lib.mpcd_rnemd_exchange(self.stream, C.byref(self.csys), _ptr(self.x), _ptr(self.v),
                                             _ptr(self.tag), C.byref(r), _ptr(self.rnemd_dp), _ptr(self.ws),
                                             self.ws_bytes), "mpcd_rnemd_exchange")

    def _vec(self, key):
        return (C.c_double * 3)(*[float(a) for a in self.params.get(key, (0.0, 0.0, 0.0))])

    def _vec_ptr(self, key):
        v = self.params.get(key)
        if v is None or not any(float(a) != 0.0 for a in v):
            return None
        return self._vec(key)

    def _swap(self):
        self.x, self.x2 = self.x2, self.x
        self.v, self.v2 = self.v2, self.v
        self.tag, self.tag2 = self.tag2, self.tag

    # --- entry points -------------------------------------------------
    def sites_thermalize(self):
        p = self.params
        L.check(self.lib.sites_thermalize(self.stream, C.byref(self.csys), C.byref(self.cbodies), p["kT"],
                                          int(p.get("thermalize", 1)), p["seed"], _ptr(self.d_step),
                                          _ptr(self.xs), _ptr(self.vs), _ptr(self.ws), self.ws_bytes),
                "sites_thermalize")

    def bin(self):
        L.check(self.lib.mpcd_bin(self.stream, C.byref(self.csys), _ptr(self.x), _ptr(self.xs),
                                  C.byref(self.cbodies), self.params["seed"], _ptr(self.d_step),
                                  _ptr(self.ws), self.ws_bytes), "mpcd_bin")

    def collide(self, stream_x: bool = False):
        p = self.params
        L.check(self.lib.mpcd_collide(self.stream, C.byref(self.csys), _ptr(self.v), _ptr(self.tag),
                                      _ptr(self.vs), C.byref(self.cbodies), p["cos_a"], p["sin_a"],
                                      p["kT_cell"], p["seed"], _ptr(self.d_step), _ptr(self.ws),
                                      self.ws_bytes, _ptr(self.x) if stream_x else C.c_void_p(0), p["dt"]),
                "mpcd_collide")

    def cell_draws(self):
        p = self.params
        L.check(self.lib.mpcd_cell_draws(self.stream, C.byref(self.csys), p["kT_cell"], p["seed"],
                                         _ptr(self.d_step), _ptr(self.ws), self.ws_bytes), "mpcd_cell_draws")

    def collide_drawn(self, stream_x: bool = False):
        p = self.params
        L.check(self.lib.mpcd_collide_drawn(self.stream, C.byref(self.csys), _ptr(self.v), _ptr(self.tag),
                                            _ptr(self.vs), C.byref(self.cbodies), p["cos_a"], p["sin_a"],
                                            p["kT_cell"], _ptr(self.d_step), _ptr(self.ws), self.ws_bytes,
                                            _ptr(self.x) if stream_x else C.c_void_p(0), p["dt"],
                                            C.c_void_p(0), C.c_void_p(0), C.c_void_p(0), p["seed"],
                                            C.byref(self.tuning)),
                "mpcd_collide_drawn")

    def sites_to_body(self):
        L.check(self.lib.sites_to_body(self.stream, C.byref(self.csys), C.byref(self.cbodies), _ptr(self.vs),
                                       _ptr(self.ws), self.ws_bytes, _ptr(self.J), _ptr(self.K)),
                "sites_to_body")

    def body_forces(self):
        L.check(self.lib.body_forces(self.stream, C.byref(self.csys), C.byref(self.cbodies),
                                     C.byref(self.cwca), self._vec_ptr("f_ext"), _ptr(self.ws), self.ws_bytes),
                "body_forces")

    def body_integrate(self, impulse: bool = True):
        L.check(self.lib.body_integrate(self.stream, C.byref(self.csys), C.byref(self.cbodies),
                                        _ptr(self.J) if impulse else C.c_void_p(0),
                                        _ptr(self.K) if impulse else C.c_void_p(0), C.byref(self.cwca),
                                        self._vec_ptr("f_ext"), self.params["dt"], _ptr(self.ws), self.ws_bytes),
                "body_integrate")

    def stream_solvent(self):
        L.check(self.lib.mpcd_stream(self.stream, C.byref(self.csys), _ptr(self.x), _ptr(self.v),
                                     self.params["dt"], self._vec_ptr("g"), _ptr(self.ws), self.ws_bytes),
                "mpcd_stream")

    def advance(self):
        L.check(self.lib.mpcd_advance_step(self.stream, _ptr(self.d_step)), "mpcd_advance_step")

    def step(self, nsteps: int = 1):
        for _ in range(nsteps):
            args = self.step_args()
            L.check(self.lib.mpcd_step(self.stream, C.byref(args)), "mpcd_step")
            if self.out_of_place:
                self._swap()

    def forces_prep(self, step_next):
        """mpcd_forces_prep on the current state: body forces, kick and counter
        advance, then the next step's site thermalization and binning of the
        current solvent, for the step index held in step_next (device int64)."""
        a = self.step_args()  # a.x: the solvent the last step wrote
        L.check(self.lib.mpcd_forces_prep(self.stream, C.byref(a), _ptr(step_next)), "mpcd_forces_prep")

    def binned_sites(self):
        """mpcd_binned_sites: the current step's sites thermalized and listed."""
        L.check(self.lib.mpcd_binned_sites(self.stream, C.byref(self.step_args())), "mpcd_binned_sites")

    def binned_collide(self):
        """mpcd_binned_collide: the current step's brick collision into the
        other set of arrays (repeatable; the state is not advanced)."""
        L.check(self.lib.mpcd_binned_collide(self.stream, C.byref(self.step_args())), "mpcd_binned_collide")

    def recollide_last(self, restore_sites: bool = True):
        """Repeat the last out-of-place step's collide + stream pass from its
        inputs into the current arrays.  The sites collide in place, so their
        velocities entering that collision are restored first (then the result
        is bit-identical); without the restore, cells with sites see the sites'
        post-collision velocities (same work, for timing the kernel)."""
        if not self.out_of_place:
            raise ValueError("recollide_last needs the out-of-place form")
        if restore_sites and self.S > 0:
            self.vs.copy_(self.ws_view("vpre", torch.float64, 3 * self.S).view(3, self.S))
        p = self.params
        L.check(self.lib.mpcd_collide_drawn(self.stream, C.byref(self.csys), _ptr(self.v2), _ptr(self.tag2),
                                            _ptr(self.vs), C.byref(self.cbodies), p["cos_a"], p["sin_a"],
                                            p["kT_cell"], _ptr(self.d_step), _ptr(self.ws), self.ws_bytes,
                                            _ptr(self.x2), p["dt"], _ptr(self.x), _ptr(self.v), _ptr(self.tag),
                                            p["seed"], C.byref(self.tuning)),
                "mpcd_collide_drawn")

    def reorder(self):
        L.check(self.lib.mpcd_reorder(self.stream, C.byref(self.csys), _ptr(self.x), _ptr(self.v), _ptr(self.tag),
                                      _ptr(self.ws), self.ws_bytes), "mpcd_reorder")

    def graph(self, nsteps: int, reorder_every: int = 0):
        """Capture nsteps steps into a HIP graph (the current stream must not be
        the null stream).  Out of place, nsteps must be even (a replay leaves the
        state in the current arrays); in place, a storage reorder follows every
        reorder_every steps."""
        if self.out_of_place and nsteps % 2:
            raise ValueError("out-of-place graphs capture an even number of steps")
        self.release_graph()
        args = self.step_args(reorder_every)
        h = C.c_void_p(0)
        L.check(self.lib.mpcd_graph_create(self.stream, C.byref(args), int(nsteps), C.byref(h)),
                "mpcd_graph_create")
        self._graph = h
        self._graph_args = args
        return h

    def graph_launch(self):
        L.check(self.lib.mpcd_graph_launch(self.stream, self._graph), "mpcd_graph_launch")

    def release_graph(self):
        if self._graph is not None:
            self.lib.mpcd_graph_destroy(self._graph)
            self._graph = None

    def status(self) -> int:
        f = C.c_uint32(0)
        L.check(self.lib.mpcd_status(self.stream, _ptr(self.ws), self.ws_bytes, C.byref(f)), "mpcd_status")
        return int(f.value)

    # --- inspection -----------------------------------------------------
    def ws_view(self, key, dtype, count):
        off = self.ws_off[key]
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype)

    def cell_order(self):
        """Storage position of every cell, in canonical cell order (host)."""
        if getattr(self, "_cell_order", None) is None:
            nc = np.ascontiguousarray(self.ncell_h.reshape(-1), dtype=np.int32)
            pos = np.empty(self.C, dtype=np.int64)
            L.check(self.lib.mpcd_cell_order(self.nsys, nc.ctypes.data_as(C.POINTER(C.c_int32)),
                                             pos.ctypes.data_as(C.POINTER(C.c_int64))), "mpcd_cell_order")
            self._cell_order = pos
        return self._cell_order

    def bins(self, storage: bool = False):
        """The last binning's cell lists: (cell_start [C+1], members [N+S], shifts).
        Cells in canonical order (system, then (j_z n_y + j_y) n_x + j_x), or as
        stored (storage=True)."""
        cs = self.ws_view("cell_start", torch.int32, self.C + 1).cpu().numpy().astype(np.int64)
        perm = self.ws_view("perm", torch.int32, self.N + self.S).cpu().numpy().astype(np.int64)
        shift = self.ws_view("shift", torch.float64, 3 * self.nsys).cpu().numpy().reshape(-1, 3)
        if storage:
            return cs, perm, shift
        pos = self.cell_order()
        cnt = cs[pos + 1] - cs[pos]
        cc = np.concatenate([[0], np.cumsum(cnt)])
        idx = np.repeat(cs[pos] - cc[:-1], cnt) + np.arange(cc[-1])
        return cc, perm[idx], shift

    def site_state(self):
        d = self.ws_view("site_d", torch.float64, 3 * self.S).cpu().numpy().reshape(3, -1)
        vpre = self.ws_view("vpre", torch.float64, 3 * self.S).cpu().numpy().reshape(3, -1)
        return d, vpre

    def download(self):
        """Per-system dicts of numpy float64 arrays in the oracle's layout."""
        torch.cuda.synchronize(self.device)
        g = {k: getattr(self, k).detach().cpu().numpy() for k in
             ("pos", "image", "quat", "mom", "angmom", "force", "torque", "xs", "vs", "J", "K")}
        xd, vd, td = self.dense_solvent()
        torch.cuda.synchronize(self.device)
        g["x"], g["v"] = xd.cpu().numpy(), vd.cpu().numpy()
        # solvent back into identity order
        tag = td.cpu().numpy().astype(np.int64)
        for k in ("x", "v"):
            a = np.empty_like(g[k])
            a[:, tag] = g[k]
            g[k] = a
        out = []
        for r in range(self.nsys):
            n0, n1 = self.solv_off_h[r], self.solv_off_h[r + 1]
            b0, b1 = self.body_off_h[r], self.body_off_h[r + 1]
            s0, s1 = self.site_sys_off_h[r], self.site_sys_off_h[r + 1]
            out.append(dict(x=g["x"][:, n0:n1].astype(np.float64), v=g["v"][:, n0:n1].astype(np.float64),
                            R=g["pos"][:, b0:b1], img=g["image"][:, b0:b1], q=g["quat"][:, b0:b1],
                            P=g["mom"][:, b0:b1], p=g["angmom"][:, b0:b1], F=g["force"][:, b0:b1],
                            T=g["torque"][:, b0:b1], xs=g["xs"][:, s0:s1].astype(np.float64),
                            vs=g["vs"][:, s0:s1].astype(np.float64), J=g["J"][:, b0:b1], K=g["K"][:, b0:b1]))
        return out


class HarmonicGPU:
    """Device state of the harmonic-bond comparator (one system; see
    workloads.harmonic_from_rigid), FP64, out-of-place solvent."""

    def __init__(self, hw: dict, params: dict, device: str = "cuda:0"):
        self.lib = L.load()
        dev = self.device = torch.device(device)
        self.params = dict(params)
        f64 = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
        i32 = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.int32), device=dev)
        i64 = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.int64), device=dev)
        ncell = np.array(hw["ncell"], dtype=np.int32)
        self.N, self.S, self.B = hw["x"].shape[1], hw["xs"].shape[1], hw["xc"].shape[1]
        self.C = int(np.prod(ncell))
        self.ncell = i32(ncell)
        self.solv_off = i64([0, self.N])
        self.cell_off = i64([0, self.C])
        self.body_off = i64([0, self.B])
        self.x, self.v = f64(hw["x"]), f64(hw["v"])
        self.x2, self.v2 = torch.empty_like(self.x), torch.empty_like(self.v)
        self.tag = torch.arange(self.N, dtype=torch.int32, device=dev)
        self.tag2 = torch.empty_like(self.tag)
        self.xs, self.vs = f64(hw["xs"]), f64(hw["vs"])
        self.xs_alt = torch.empty_like(self.xs)
        self.xc, self.vc = f64(hw["xc"]), f64(hw["vc"])
        self.xc_alt = torch.empty_like(self.xc)
        self.fs, self.fc = torch.zeros_like(self.xs), torch.zeros_like(self.xc)
        self.imgs, self.imgc = i32(hw["imgs"]), i32(hw["imgc"])
        self.site_off, self.site_body = i64(hw["site_off"]), i32(hw["site_body"])
        self.adj_off, self.adj, self.adj_r0 = i64(hw["adj_off"]), i32(hw["adj"]), f64(hw["adj_r0"])
        self.rc0, self.site_m = f64(hw["rc0"]), f64(hw["sm"])
        self.d_step = torch.zeros(1, dtype=torch.int64, device=dev)
        self.csys = L.MpcdSys(nsys=1, prec=L.MPCD_F64, a=float(hw["a"]), m_solvent=float(hw["m"]), n_solvent=self.N,
                              n_sites=self.S, n_bodies=self.B, n_cells=self.C, replica0=0,
                              ncell=_ptr(self.ncell), solv_off=_ptr(self.solv_off), cell_off=_ptr(self.cell_off),
                              body_off=_ptr(self.body_off))
        self.ws_bytes = int(self.lib.mpcd_workspace_bytes(C.byref(self.csys)))
        if self.ws_bytes == 0:
            raise L.MpcdError("invalid system description")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.ch = L.MpcdHarm(xs_alt=_ptr(self.xs_alt), xc=_ptr(self.xc), xc_alt=_ptr(self.xc_alt), vc=_ptr(self.vc),
                             fs=_ptr(self.fs), fc=_ptr(self.fc), imgs=_ptr(self.imgs), imgc=_ptr(self.imgc),
                             mc=float(hw["mc"]), kb=float(hw["kb"]), site_off=_ptr(self.site_off),
                             site_body=_ptr(self.site_body), adj_off=_ptr(self.adj_off), adj=_ptr(self.adj),
                             adj_r0=_ptr(self.adj_r0), rc0=_ptr(self.rc0), site_m=_ptr(self.site_m))
        self.cbodies = L.MpcdBodies(site_off=_ptr(self.site_off), site_body=_ptr(self.site_body),
                                    site_m=_ptr(self.site_m))
        w = self.params.get("wca", {"mode": 0})
        self.cwca = L.MpcdWca(mode=int(w.get("mode", 0)), eps=float(w.get("eps", 0.0)),
                              sigma=float(w.get("sigma", 0.0)), delta=float(w.get("delta", 0.0)), reach=0.0)
        L.check(self.lib.mpcd_ws_init(self.stream, C.byref(self.csys), _ptr(self.ws), self.ws_bytes), "mpcd_ws_init")
        self._graph = None

    @property
    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def forces(self):
        L.check(self.lib.harm_forces(self.stream, C.byref(self.csys), C.byref(self.ch), _ptr(self.xs),
                                     C.byref(self.cwca), _ptr(self.ws), self.ws_bytes), "harm_forces")

    def args(self) -> L.MpcdStepArgs:
        p = self.params
        par = L.MpcdParams(dt=p["dt"], cos_a=p["cos_a"], sin_a=p["sin_a"], kT=p["kT"], kT_cell=p["kT_cell"],
                           seed=p["seed"], thermalize=0, fuse_stream=1, wca=self.cwca)
        self._args = L.MpcdStepArgs(sys=C.pointer(self.csys), bodies=self.cbodies, x=_ptr(self.x), v=_ptr(self.v),
                                    tag=_ptr(self.tag), xs=_ptr(self.xs), vs=_ptr(self.vs), d_step=_ptr(self.d_step),
                                    ws=_ptr(self.ws), ws_bytes=self.ws_bytes, par=par, x_out=_ptr(self.x2),
                                    v_out=_ptr(self.v2), tag_out=_ptr(self.tag2))
        return self._args

    def step(self, dt_md: float, nsub: int, n: int = 1):
        for _ in range(n):
            a = self.args()
            L.check(self.lib.harm_step(self.stream, C.byref(a), C.byref(self.ch), float(dt_md), int(nsub)),
                    "harm_step")
            self.x, self.x2 = self.x2, self.x
            self.v, self.v2 = self.v2, self.v
            self.tag, self.tag2 = self.tag2, self.tag

    def graph(self, dt_md: float, nsub: int, nperiods: int):
        if nperiods % 2:
            raise ValueError("out-of-place graphs capture an even number of periods")
        self.release_graph()
        a = self.args()
        h = C.c_void_p(0)
        L.check(self.lib.harm_graph_create(self.stream, C.byref(a), C.byref(self.ch), float(dt_md), int(nsub),
                                           int(nperiods), C.byref(h)), "harm_graph_create")
        self._graph = h
        self._graph_args = a
        return h

    def graph_launch(self):
        L.check(self.lib.mpcd_graph_launch(self.stream, self._graph), "mpcd_graph_launch")

    def release_graph(self):
        if self._graph is not None:
            self.lib.mpcd_graph_destroy(self._graph)
            self._graph = None

    def status(self) -> int:
        f = C.c_uint32(0)
        L.check(self.lib.mpcd_status(self.stream, _ptr(self.ws), self.ws_bytes, C.byref(f)), "mpcd_status")
        return int(f.value)

    def download(self):
        torch.cuda.synchronize(self.device)
        tag = self.tag.cpu().numpy().astype(np.int64)
        out = {}
        for k in ("x", "v"):
            a = getattr(self, k).cpu().numpy()
            b = np.empty_like(a)
            b[:, tag] = a
            out[k] = b
        for k in ("xs", "vs", "xc", "vc", "fs", "fc", "imgs", "imgc"):
            out[k] = getattr(self, k).cpu().numpy()
        return out
