"""ctypes binding of libfcsdnn.so (argument marshalling only).

Every compute function here forwards device pointers of torch tensors to the
C ABI declared in include/fcsdnn.h; all arithmetic runs in the library's HIP
kernels.  The library must be built (``python -m paper_2506_16076_amd.build``
or ``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcsdnn.so")

STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EHIP", 5: "EUNSUPPORTED", 6: "ENONFINITE"}
WS_RHS, WS_AV, WS_STEP, WS_RHS_ADJ, WS_STEP_ADJ, WS_FILTER_ADJ, WS_SMEAR, WS_STAGE_ADJ = 0, 1, 2, 3, 4, 5, 6, 7
LAYOUT_ROWS, LAYOUT_B8X4 = 0, 1
SCHED_SPLIT, SCHED_FUSED, SCHED_PERSISTENT, SCHED_FUSED_WIDE = 0, 1, 2, 3


def blocked_layout(n1, n2, base_off=None):
    """Offsets and plane size of the 8x4-blocked storage of patches n1 x n2
    (patches back to back, each padded to whole blocks)."""
    off, o = [], 0
    for a, b in zip(n1, n2):
        off.append(o)
        o += ((int(a) + 7) // 8 * 8) * ((int(b) + 3) // 4 * 4)
    return np.asarray(off, np.int64), (o + 63) // 64 * 64


def layout_index(n1, n2, off_rows, off_blk):
    """Plane indices (rows, blocked) of every patch point, for converting
    planes between the two storages."""
    rows, blk = [], []
    for a, b, orow, oblk in zip(n1, n2, off_rows, off_blk):
        a, b = int(a), int(b)
        j, i = np.meshgrid(np.arange(b), np.arange(a), indexing="ij")
        rows.append(int(orow) + j * a + i)
        nb1 = (a + 7) // 8
        blk.append(int(oblk) + ((j // 4) * nb1 + i // 8) * 32 + (j % 4) * 8 + i % 8)
    return np.concatenate([r.ravel() for r in rows]), np.concatenate([q.ravel() for q in blk])


class FcsdError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"fcsdnn {STATUS.get(code, code)}: {msg}")
        self.code = code


class PatchDesc(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("C1", ctypes.c_int32),
                ("C2", ctypes.c_int32), ("off", ctypes.c_int64), ("hhat", ctypes.c_double),
                ("htilde", ctypes.c_double), ("internal", ctypes.c_uint8 * 4),
                ("reserved", ctypes.c_int32)]


class Mlp(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]


class PatchMap(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a0", ctypes.c_double), ("da", ctypes.c_double),
                ("b0", ctypes.c_double), ("db", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("ux", ctypes.c_double), ("uy", ctypes.c_double),
                ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("side", ctypes.c_double),
                ("nmodes", ctypes.c_int32), ("cx", ctypes.c_double * 8), ("sx", ctypes.c_double * 8),
                ("cy", ctypes.c_double * 8), ("sy", ctypes.c_double * 8)]

    @classmethod
    def from_row(cls, r):
        """A patch-map row (kind, a0, da, b0, db, x0, y0, ux, uy, vx, vy, side,
        nmodes, cx[8], sx[8], cy[8], sy[8]); rows of 5 numbers are the
        Cartesian and polar maps."""
        r = np.zeros(45) if r is None else np.concatenate([np.asarray(r, np.float64), np.zeros(45)])[:45]
        m = cls()
        m.kind = int(r[0])
        m.a0, m.da, m.b0, m.db = (float(v) for v in r[1:5])
        m.x0, m.y0, m.ux, m.uy, m.vx, m.vy = (float(v) for v in r[5:11])
        m.side = float(r[11])
        m.nmodes = int(r[12])
        for name, o in (("cx", 13), ("sx", 21), ("cy", 29), ("sy", 37)):
            arr = getattr(m, name)
            for k in range(8):
                arr[k] = float(r[o + k])
        return m


class StepArgs(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("metric", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("tau", ctypes.c_void_p), ("argmax", ctypes.c_void_p), ("dt_dev", ctypes.c_void_p),
                ("dirichlet_mask", ctypes.c_void_p), ("dirichlet_state", ctypes.c_float * 4),
                ("ref", ctypes.c_float * 4), ("gamma", ctypes.c_float), ("cfl", ctypes.c_float),
                ("fixed_dt", ctypes.c_int), ("w", ctypes.c_void_p), ("fixed_tau", ctypes.c_int),
                ("filter", ctypes.c_int), ("record", ctypes.c_void_p)]


RECORD_PLANES = 66  # planes of a step record (stage inputs, mu, maximisers, pre-filter state, derivatives)


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, f32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "fcsd_ctx_create": [i32, vp, P(vp)],
            "fcsd_ctx_destroy": [vp],
            "fcsd_ctx_set_stream": [vp, vp],
            "fcsd_ctx_sync": [vp],
            "fcsd_set_create": [vp, i32, P(PatchDesc), i32, i64, i32, i32, i32, P(vp)],
            "fcsd_set_destroy": [vp],
            "fcsd_set_tune": [vp, P(i32), P(i32), i32],
            "fcsd_set_schedule": [vp, i32],
            "fcsd_stage_errors": [vp, P(ctypes.c_int32)],
            "fcsd_set_filter": [vp, ctypes.c_double, i32],
            "fcsd_filter": [vp, vp, vp, vp, i64, f32],
            "fcsd_set_interp": [vp, vp, i32, P(i64)],
            "fcsd_set_walls": [vp, vp, f32],
            "fcsd_smear": [vp, vp, vp, vp, vp, i64, f32, ctypes.c_double, i32, ctypes.c_double, ctypes.c_double,
                           vp, sz],
            "fcsd_filter_adj": [vp, vp, vp, vp, vp, i64, f32, vp, sz],
            "fcsd_workspace_size": [vp, i32, P(sz)],
            "fcsd_ext_size": [vp, i32, P(i64)],
            "fc_continue": [vp, vp, i32, i32, vp, i64, vp, i64],
            "fc_continue_adj": [vp, vp, i32, i32, vp, i64, vp, i64],
            "fc_diff": [vp, vp, i32, i32, vp, vp, i64],
            "fc_diff_adj": [vp, vp, i32, i32, vp, vp, i64],
            "euler_rhs": [vp, vp, vp, vp, P(f32), f32, vp, i64, vp, sz],
            "av_apply": [vp, vp, vp, vp, vp, P(f32), vp, i64, vp, sz],
            "fcsd_rhs": [vp, vp, vp, vp, vp, P(f32), f32, vp, i64, vp, sz],
            "fcsd_rhs_adj": [vp, vp, vp, vp, vp, P(f32), f32, vp, vp, vp, i64, vp, sz],
            "euler_rhs_adj": [vp, vp, vp, vp, P(f32), f32, vp, vp, i64, vp, sz],
            "av_apply_adj": [vp, vp, vp, vp, vp, P(f32), vp, vp, vp, i64, vp, sz],
            "sdnn_infer_adj": [vp, vp, vp, f32, P(Mlp), vp, vp, i64, vp, sz],
            "fcsd_stage_adj": [vp, vp, i32, vp, vp, vp, P(f32), f32, vp, vp, vp, vp, vp, vp, i64, vp, sz],
            "rk_stage": [vp, vp, i32, vp, vp, vp, vp, vp, vp, i64],
            "rk_stage_adj": [vp, vp, i32, vp, vp, vp, vp, vp, vp, i64],
            "fcsd_cfl_dt": [vp, vp, vp, vp, f32, f32, vp, i64, vp, sz],
            "fcsd_cfl_dt_noalloc": [vp, vp, vp, vp, f32, f32, vp, i64],
            "fcsd_check": [vp, vp, vp, f32, vp, i64],
            "sdnn_infer": [vp, vp, vp, f32, P(Mlp), vp, vp, i64, vp, sz],
            "av_viscosity": [vp, vp, vp, vp, f32, vp, vp, i64, vp, sz],
            "av_viscosity_adj": [vp, vp, vp, vp, vp, f32, vp, vp, i64, vp, sz],
            "fcsd_glue": [vp, vp, vp, i64, vp, P(f32)],
            "fcsd_glue_adj": [vp, vp, vp, i64, vp, P(f32), vp, vp],
            "fcsd_step_adj": [vp, vp, P(StepArgs), vp, vp, P(f32), vp, i64, vp, sz],
            "fcsd_stage": [vp, vp, i32, vp, vp, vp, vp, vp, vp, P(f32), f32, vp, i64, vp, sz],
            "fcsd_stage_per_patch": [vp, vp, i32, vp, vp, vp, vp, vp, vp, P(f32), f32, vp, i64, vp, sz],
            "fcsd_stage_pass": [vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, P(f32), f32, vp, i64, vp, sz],
            "fcsd_step": [vp, vp, P(StepArgs), i64, vp, sz, i32],
            "fcsd_fc_matrix": [i32, i32, P(ctypes.c_double)],
            "fcsd_fft_plan": [i32, P(i32), P(i32)],
            "fcsd_validate_patches": [i32, P(PatchDesc), i32, i64, i32, i32, i32, ctypes.c_char_p, i32],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.fcsd_last_error.argtypes = [vp]
        L.fcsd_last_error.restype = ctypes.c_char_p
        L.fcsd_ctx_stream.argtypes = [vp]
        L.fcsd_ctx_stream.restype = vp
        L.fcsd_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


# the names every header declaration exports (checked by the CPU tests)
EXPORTS = ["fcsd_ctx_create", "fcsd_ctx_destroy", "fcsd_ctx_set_stream", "fcsd_last_error",
           "fcsd_ctx_stream", "fcsd_ctx_sync", "fcsd_set_create", "fcsd_set_destroy", "fcsd_set_tune",
           "fcsd_set_schedule", "fcsd_stage_errors",
           "fcsd_set_filter", "fcsd_filter", "fcsd_filter_adj", "fcsd_smear", "fcsd_set_interp", "fcsd_set_walls",
           "fcsd_workspace_size", "fcsd_ext_size", "fc_continue", "fc_continue_adj", "fc_diff",
           "fc_diff_adj", "euler_rhs", "av_apply", "fcsd_rhs", "fcsd_rhs_adj", "euler_rhs_adj", "av_apply_adj",
           "sdnn_infer_adj", "fcsd_stage_adj", "rk_stage",
           "rk_stage_adj", "fcsd_cfl_dt", "fcsd_cfl_dt_noalloc", "fcsd_check", "sdnn_infer", "av_viscosity", "av_viscosity_adj",
           "fcsd_glue", "fcsd_glue_adj", "fcsd_step_adj", "fcsd_stage", "fcsd_stage_per_patch", "fcsd_stage_pass", "fcsd_step", "fcsd_fc_matrix",
           "fcsd_validate_patches", "fcsd_fft_plan", "fcsd_version"]


def patch_descs(n1, n2, C1, C2, off, hhat, htilde, internal):
    n = len(n1)
    arr = (PatchDesc * n)()
    for p in range(n):
        d = arr[p]
        d.n1, d.n2, d.C1, d.C2 = int(n1[p]), int(n2[p]), int(C1[p]), int(C2[p])
        d.off = int(off[p])
        d.hhat, d.htilde = float(hhat[p]), float(htilde[p])
        for s in range(4):
            d.internal[s] = int(internal[p][s])
    return arr


# ------------------------------------------------------------------ host-only helpers

def fc_matrix(d: int, C: int) -> np.ndarray:
    """The library's A_r Q^T (C x d, FP64), computed on the host."""
    out = np.zeros((C, d))
    rc = lib().fcsd_fc_matrix(d, C, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise FcsdError(rc, "fc_matrix")
    return out


def fft_plan(L: int):
    n = ctypes.c_int(0)
    r = (ctypes.c_int * 8)()
    rc = lib().fcsd_fft_plan(L, ctypes.byref(n), r)
    if rc:
        raise FcsdError(rc, f"no radix plan for L={L}")
    return [r[i] for i in range(n.value)]


def validate_patches(descs, d, plane, ring_sectors=0, ring_shells=0, layout=0):
    buf = ctypes.create_string_buffer(256)
    rc = lib().fcsd_validate_patches(len(descs), descs, d, plane, ring_sectors, ring_shells, layout, buf, 256)
    return rc, buf.value.decode()
