"""ctypes binding of libmpcd.so (argument marshalling only).

Every step of the MPCD path runs in the HIP kernels of libmpcd.so; this module
loads the library, packs torch device tensors into the C-ABI structs and calls
the entry points declared in include/mpcd.h with the same names.  There is no
CPU fallback: loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpcd.so")

MPCD_F64, MPCD_F32 = 0, 1
FLAG_NONFINITE, FLAG_ESCAPE, FLAG_FIXOVF, FLAG_RNGLOOP, FLAG_BINERR, FLAG_REACH, FLAG_CROWD = 1, 2, 4, 8, 16, 32, 64

EXPORTS = ("mpcd_workspace_bytes", "mpcd_workspace_offsets", "mpcd_ws_init", "mpcd_stream", "mpcd_bin", "mpcd_collide",
           "mpcd_cell_draws", "mpcd_collide_drawn",
           "sites_thermalize", "sites_to_body", "body_integrate", "body_forces",
           "mpcd_advance_step", "mpcd_step", "mpcd_forces_prep", "mpcd_reorder", "mpcd_graph_create", "mpcd_graph_launch",
           "mpcd_graph_destroy", "mpcd_status", "mpcd_last_hip_error",
           "harm_forces", "harm_md", "harm_step", "harm_graph_create", "mpcd_rnemd_exchange", "mpcd_cell_order",
           "mpcd_tile_shape", "mpcd_binned_layout", "mpcd_binned_init", "mpcd_binned_pack", "mpcd_binned_unpack",
           "mpcd_binned_collide", "mpcd_binned_sites", "mpcd_rnemd_exchange_noalloc")

vp = C.c_void_p


class MpcdSys(C.Structure):
    _fields_ = [("nsys", C.c_int32), ("prec", C.c_int32), ("a", C.c_double), ("m_solvent", C.c_double),
                ("n_solvent", C.c_int64), ("n_sites", C.c_int64), ("n_bodies", C.c_int64),
                ("n_cells", C.c_int64), ("replica0", C.c_uint64),
                ("ncell", vp), ("solv_off", vp), ("cell_off", vp), ("body_off", vp)]


class MpcdBodies(C.Structure):
    _fields_ = [("pos", vp), ("image", vp), ("quat", vp), ("mom", vp), ("angmom", vp),
                ("force", vp), ("torque", vp), ("mass", vp), ("inertia", vp),
                ("site_off", vp), ("site_body", vp), ("site_d", vp), ("site_m", vp)]


class MpcdWca(C.Structure):
    _fields_ = [("mode", C.c_int32), ("eps", C.c_double), ("sigma", C.c_double), ("delta", C.c_double),
                ("reach", C.c_double)]


class MpcdTune(C.Structure):
    _fields_ = [("tile_items", C.c_int32), ("tile_fill", C.c_int32), ("draw_cells", C.c_int32),
                ("draws_inline", C.c_int32), ("overlap", C.c_int32)]


class MpcdParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("cos_a", C.c_double), ("sin_a", C.c_double), ("kT", C.c_double),
                ("kT_cell", C.c_double), ("seed", C.c_uint64), ("thermalize", C.c_int32),
                ("fuse_stream", C.c_int32), ("wca", MpcdWca), ("g", C.c_double * 3), ("f_ext", C.c_double * 3),
                ("tune", MpcdTune)]


class MpcdRnemd(C.Structure):
    _fields_ = [("y0", C.c_double), ("y1", C.c_double), ("dy", C.c_double), ("target", C.c_double),
                ("npairs", C.c_int32)]


class MpcdBinned(C.Structure):
    _fields_ = [("ws", vp), ("ws_bytes", C.c_size_t), ("nbricks", C.c_int64), ("capacity", C.c_int64),
                ("site_slots", C.c_int64), ("items", C.c_int32)]


class MpcdStepArgs(C.Structure):
    _fields_ = [("sys", C.POINTER(MpcdSys)), ("bodies", MpcdBodies), ("x", vp), ("v", vp), ("tag", vp),
                ("xs", vp), ("vs", vp), ("J", vp), ("K", vp), ("d_step", vp), ("ws", vp),
                ("ws_bytes", C.c_size_t), ("par", MpcdParams), ("reorder_every", C.c_int32),
                ("x_out", vp), ("v_out", vp), ("tag_out", vp), ("rnemd", C.POINTER(MpcdRnemd)),
                ("rnemd_dp", vp), ("binned", C.POINTER(MpcdBinned))]


class MpcdHarm(C.Structure):
    _fields_ = [("xs_alt", vp), ("xc", vp), ("xc_alt", vp), ("vc", vp), ("fs", vp), ("fc", vp),
                ("imgs", vp), ("imgc", vp), ("mc", C.c_double), ("kb", C.c_double),
                ("site_off", vp), ("site_body", vp), ("adj_off", vp), ("adj", vp), ("adj_r0", vp),
                ("rc0", vp), ("site_m", vp)]


_lib = None


class MpcdError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load libmpcd.so.  Raises if it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MpcdError("libmpcd.so not built (%s); run __graft_entry__.build()" % path)
    L = C.CDLL(path)
    sp, bp, wp = C.POINTER(MpcdSys), C.POINTER(MpcdBodies), C.POINTER(MpcdWca)
    sz, dbl, u64, i32 = C.c_size_t, C.c_double, C.c_uint64, C.c_int32
    sig = {
        "mpcd_workspace_bytes": (sz, [sp]),
        "mpcd_workspace_offsets": (C.c_int, [sp, C.POINTER(C.c_int64)]),
        "mpcd_cell_order": (C.c_int, [i32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
        "mpcd_tile_shape": (C.c_int, [sp, C.POINTER(MpcdTune), C.POINTER(C.c_int32)]),
        "mpcd_ws_init": (C.c_int, [vp, sp, vp, sz]),
        "mpcd_stream": (C.c_int, [vp, sp, vp, vp, dbl, C.POINTER(dbl), vp, sz]),
        "mpcd_bin": (C.c_int, [vp, sp, vp, vp, bp, u64, vp, vp, sz]),
        "mpcd_collide": (C.c_int, [vp, sp, vp, vp, vp, bp, dbl, dbl, dbl, u64, vp, vp, sz, vp, dbl]),
        "mpcd_cell_draws": (C.c_int, [vp, sp, dbl, u64, vp, vp, sz]),
        "mpcd_collide_drawn": (C.c_int, [vp, sp, vp, vp, vp, bp, dbl, dbl, dbl, vp, vp, sz, vp, dbl, vp, vp, vp,
                                         u64, C.POINTER(MpcdTune)]),
        "sites_thermalize": (C.c_int, [vp, sp, bp, dbl, i32, u64, vp, vp, vp, vp, sz]),
        "sites_to_body": (C.c_int, [vp, sp, bp, vp, vp, sz, vp, vp]),
        "body_integrate": (C.c_int, [vp, sp, bp, vp, vp, wp, C.POINTER(dbl), dbl, vp, sz]),
        "body_forces": (C.c_int, [vp, sp, bp, wp, C.POINTER(dbl), vp, sz]),
        "mpcd_advance_step": (C.c_int, [vp, vp]),
        "mpcd_step": (C.c_int, [vp, C.POINTER(MpcdStepArgs)]),
        "mpcd_forces_prep": (C.c_int, [vp, C.POINTER(MpcdStepArgs), vp]),
        "mpcd_reorder": (C.c_int, [vp, sp, vp, vp, vp, vp, sz]),
        "mpcd_graph_create": (C.c_int, [vp, C.POINTER(MpcdStepArgs), i32, C.POINTER(vp)]),
        "mpcd_graph_launch": (C.c_int, [vp, vp]),
        "mpcd_graph_destroy": (C.c_int, [vp]),
        "mpcd_status": (C.c_int, [vp, vp, sz, C.POINTER(C.c_uint32)]),
        "mpcd_last_hip_error": (C.c_int, []),
        "mpcd_rnemd_exchange": (C.c_int, [vp, sp, vp, vp, vp, C.POINTER(MpcdRnemd), vp, vp, sz]),
        "mpcd_rnemd_exchange_noalloc": (C.c_int, [vp, sp, vp, vp, vp, C.POINTER(MpcdRnemd), vp, vp]),
        "harm_forces": (C.c_int, [vp, sp, C.POINTER(MpcdHarm), vp, wp, vp, sz]),
        "harm_md": (C.c_int, [vp, sp, C.POINTER(MpcdHarm), vp, vp, wp, dbl, i32, vp, sz]),
        "harm_step": (C.c_int, [vp, C.POINTER(MpcdStepArgs), C.POINTER(MpcdHarm), dbl, i32]),
        "harm_graph_create": (C.c_int, [vp, C.POINTER(MpcdStepArgs), C.POINTER(MpcdHarm), dbl, i32, i32,
                                        C.POINTER(vp)]),
        "mpcd_binned_layout": (C.c_int, [sp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                         C.POINTER(MpcdBinned)]),
        "mpcd_binned_init": (C.c_int, [vp, sp, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                       C.POINTER(MpcdBinned)]),
        "mpcd_binned_pack": (C.c_int, [vp, sp, vp, vp, vp, vp, u64, vp, vp, sz, C.POINTER(MpcdBinned)]),
        "mpcd_binned_unpack": (C.c_int, [vp, sp, vp, vp, vp, vp, vp, vp, sz, C.POINTER(MpcdBinned)]),
        "mpcd_binned_collide": (C.c_int, [vp, C.POINTER(MpcdStepArgs)]),
        "mpcd_binned_sites": (C.c_int, [vp, C.POINTER(MpcdStepArgs)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc: int, what: str = "mpcd call"):
    if rc != 0:
        hip = load().mpcd_last_hip_error()
        raise MpcdError("%s failed: rc=%d (hip error %d)" % (what, rc, hip))
