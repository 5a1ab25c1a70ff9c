"""Torch-facing wrappers of the C ABI (same names as include/fcsdnn.h).

Torch supplies device memory and streams only.  A ``Context`` owns the
library context and its HIP stream (wrapped as a torch ExternalStream);
every call orders itself after torch's current stream and makes torch's
current stream wait for it, so tensors can be used freely on either side.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from ._lib import (LAYOUT_B8X4, LAYOUT_ROWS, RECORD_PLANES, FcsdError, Mlp, StepArgs, WS_AV, WS_RHS, WS_RHS_ADJ, WS_STEP,
                   WS_STEP_ADJ, WS_FILTER_ADJ, WS_SMEAR, WS_STAGE_ADJ, blocked_layout, layout_index, lib,
                   patch_descs)


def _p(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _f4(vals):
    return (ctypes.c_float * 4)(*[float(v) for v in vals])


class Context:
    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise FcsdError(3, "no HIP device")
        torch.cuda.set_device(device)
        self.device = device
        h = ctypes.c_void_p()
        rc = lib().fcsd_ctx_create(device, None, ctypes.byref(h))
        if rc:
            raise FcsdError(rc, "fcsd_ctx_create")
        self.h = h
        self.stream = torch.cuda.ExternalStream(lib().fcsd_ctx_stream(h), device=torch.device("cuda", device))

    def check(self, rc, what):
        if rc:
            raise FcsdError(rc, f"{what}: {lib().fcsd_last_error(self.h).decode()}")

    def enter(self):
        self.stream.wait_stream(torch.cuda.current_stream())

    def leave(self):
        torch.cuda.current_stream().wait_stream(self.stream)

    def sync(self):
        self.check(lib().fcsd_ctx_sync(self.h), "sync")

    def close(self):
        if self.h:
            lib().fcsd_ctx_destroy(self.h)
            self.h = None


class PatchSet:
    """Device-side patch set built from plain arrays (n1, n2, C1, C2, off,
    hhat, htilde, internal), the plane size and the storage layout."""

    def __init__(self, ctx: Context, n1, n2, C1, C2, off, hhat, htilde, internal, d: int, plane: int,
                 ring_sectors: int = 0, ring_shells: int = 0, layout: int = LAYOUT_ROWS):
        self.ctx = ctx
        self.plane = int(plane)
        self.layout = int(layout)
        self.npatch = len(n1)
        self.npoints = int(np.sum(np.asarray(n1, np.int64) * np.asarray(n2, np.int64)))
        self.descs = patch_descs(n1, n2, C1, C2, off, hhat, htilde, internal)
        h = ctypes.c_void_p()
        ctx.check(lib().fcsd_set_create(ctx.h, self.npatch, self.descs, d, self.plane, ring_sectors,
                                        ring_shells, self.layout, ctypes.byref(h)), "fcsd_set_create")
        self.h = h
        self._ws = {}
        self._map = None
        self.schedule = 1    # the library's default: SCHED_FUSED

    @classmethod
    def from_layout(cls, ctx, ps, layout: int = LAYOUT_ROWS):
        """From any object with the attributes of synth.PatchSet (row-major
        planes).  With LAYOUT_B8X4 the device planes are blocked; to_device /
        to_host convert the row-major host planes."""
        if layout == LAYOUT_ROWS:
            s = cls(ctx, ps.n1, ps.n2, ps.C1, ps.C2, ps.off, ps.hhat, ps.htilde, ps.internal, ps.d,
                    ps.plane, ps.nsec, ps.nshell)
            s.host_plane = ps.plane
            return s
        off, plane = blocked_layout(ps.n1, ps.n2)
        s = cls(ctx, ps.n1, ps.n2, ps.C1, ps.C2, off, ps.hhat, ps.htilde, ps.internal, ps.d, plane, ps.nsec,
                ps.nshell, layout)
        rows, blk = layout_index(ps.n1, ps.n2, ps.off, off)
        dev = f"cuda:{ctx.device}"
        s._map = (torch.from_numpy(rows).to(dev), torch.from_numpy(blk).to(dev))
        s.host_plane = ps.plane
        return s

    def to_device(self, arr, dtype=None) -> torch.Tensor:
        """Row-major host planes [..., host_plane] -> flat device planes in
        the set's storage (padding zero)."""
        a = np.ascontiguousarray(arr)
        lead = a.shape[:-1]
        t = torch.from_numpy(a.reshape(-1, a.shape[-1]))
        if dtype is not None:
            t = t.to(dtype)
        dev = f"cuda:{self.ctx.device}"
        if self._map is None:
            return t.reshape(-1).to(dev).contiguous()
        rows, blk = self._map
        src = t.to(dev)
        out = torch.zeros((src.shape[0], self.plane), dtype=src.dtype, device=dev)
        out[:, blk] = src[:, rows]
        return out.reshape(-1).contiguous()

    def to_host(self, t: torch.Tensor, nf: int = None) -> np.ndarray:
        """Flat device planes in the set's storage -> row-major host planes
        [nf, host_plane]."""
        nf = nf or t.numel() // self.plane
        src = t.reshape(nf, -1)[:, :self.plane]
        if self._map is None:
            return src.cpu().numpy()
        rows, blk = self._map
        out = torch.zeros((nf, self.host_plane), dtype=src.dtype, device=src.device)
        out[:, rows] = src[:, blk]
        return out.cpu().numpy()

    def workspace_size(self, op: int) -> int:
        b = ctypes.c_size_t()
        self.ctx.check(lib().fcsd_workspace_size(self.h, op, ctypes.byref(b)), "workspace_size")
        return b.value

    def workspace(self, op: int) -> torch.Tensor:
        if op not in self._ws:
            n = (self.workspace_size(op) + 3) // 4
            self._ws[op] = torch.empty(n, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        return self._ws[op]

    ORDER_LPT, ORDER_XCD = 0, 1

    def tune(self, budgets, threads=(256, 256, 256), order: int = 1):
        """Tile split and workgroup size of the three tile sets (q1 lines:
        passes A, C; q2 lines: pass B2; q2 lines with two complex lines per
        grid line: pass B1) and the launch order (ORDER_LPT or ORDER_XCD).
        budgets / threads: one int (all sets) or three."""
        if isinstance(budgets, int):
            budgets = (budgets,) * 3
        if isinstance(threads, int):
            threads = (threads,) * 3
        b = (ctypes.c_int * 3)(*[int(x) for x in budgets])
        t = (ctypes.c_int * 3)(*[int(x) for x in threads])
        self.ctx.check(lib().fcsd_set_tune(self.h, b, t, int(order)), "fcsd_set_tune")
        self.tuning = (tuple(int(x) for x in budgets), tuple(int(x) for x in threads), int(order))

    SCHED_SPLIT, SCHED_FUSED, SCHED_PERSISTENT, SCHED_FUSED_WIDE = 0, 1, 2, 3

    def set_schedule(self, schedule: int):
        """Launch schedule of a stage's line passes: SCHED_SPLIT (four
        launches), SCHED_FUSED (three: passes B1 and B2 on one q2 tile),
        SCHED_PERSISTENT (one launch per stage taking tiles from a queue) or
        SCHED_FUSED_WIDE (three, the q2 tile holding all eight H fields)."""
        self.ctx.check(lib().fcsd_set_schedule(self.h, int(schedule)), "fcsd_set_schedule")
        self.schedule = int(schedule)

    def stage_errors(self) -> int:
        """Read and clear the set's device error word (bit 0: a persistent
        stage's dependency wait gave up; bit 1: network weights that can take
        the operands of its fp16 products out of the fp16 range)."""
        v = ctypes.c_int32(0)
        self.ctx.check(lib().fcsd_stage_errors(self.h, ctypes.byref(v)), "fcsd_stage_errors")
        return int(v.value)

    def set_filter(self, alpha: float = 10.0, p: int = 14):
        """Parameters of the spectral filter (paper Sec. 4.3.1): factors
        exp(-alpha (2k/L)^p) on the coefficients of every line extension."""
        self.ctx.check(lib().fcsd_set_filter(self.h, float(alpha), int(p)), "fcsd_set_filter")
        self.filter_params = (float(alpha), int(p))

    def set_walls(self, sides, gamma: float = 1.4):
        """No-slip adiabatic wall sides: [npatch, 4] flags (q1-, q1+, q2-,
        q2+), or None to clear."""
        if sides is None:
            self.ctx.check(lib().fcsd_set_walls(self.h, None, float(gamma)), "fcsd_set_walls")
            return
        arr = np.ascontiguousarray(np.asarray(sides, np.uint8).reshape(-1, 4))
        self._walls = arr
        self.ctx.check(lib().fcsd_set_walls(self.h, arr.ctypes.data_as(ctypes.c_void_p), float(gamma)),
                       "fcsd_set_walls")

    def set_interp(self, maps, nf: int = 5) -> int:
        """Inter-patch interpolation of the fringe (paper Sec. 3.4.1) from
        patch maps, one row per patch: (kind, a0, da, b0, db, x0, y0, ux, uy,
        vx, vy, side, nmodes, cx[8], sx[8], cy[8], sy[8]) (fcsd_patch_map;
        kind 0 Cartesian, 1 polar, 2 affine, 3 S-type; rows of 5 numbers
        for the first two).  Returns the number of fringe points."""
        from ._lib import PatchMap
        rows = [np.asarray(r, np.float64) for r in maps]
        arr = (PatchMap * len(rows))(*[PatchMap.from_row(r) for r in rows])
        n = ctypes.c_int64()
        self.ctx.check(lib().fcsd_set_interp(self.h, arr, int(nf), ctypes.byref(n)), "fcsd_set_interp")
        return n.value

    def ext_size(self, direction: int) -> int:
        v = ctypes.c_int64()
        self.ctx.check(lib().fcsd_ext_size(self.h, direction, ctypes.byref(v)), "ext_size")
        return v.value

    def close(self):
        if self.h:
            lib().fcsd_set_destroy(self.h)
            self.h = None


def _call(s: PatchSet, name, *args):
    ctx = s.ctx
    ctx.enter()
    rc = getattr(lib(), name)(ctx.h, s.h, *args)
    ctx.leave()
    ctx.check(rc, name)


def _chk(t, dtype=torch.float32, numel=None, name="tensor"):
    if t is None:
        return
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise FcsdError(1, f"{name}: needs a contiguous {dtype} device tensor")
    if numel is not None and t.numel() < numel:
        raise FcsdError(1, f"{name}: has {t.numel()} elements, needs {numel}")


# ------------------------------------------------------------------ line operators

def fc_diff(s, direction, inp, out, nf=None):
    nf = nf or inp.numel() // s.plane
    _chk(inp, numel=nf * s.plane, name="in"), _chk(out, numel=nf * s.plane, name="out")
    _call(s, "fc_diff", direction, nf, _p(inp), _p(out), s.plane)


def fc_diff_adj(s, direction, out_bar, in_bar, nf=None):
    nf = nf or out_bar.numel() // s.plane
    _chk(out_bar, numel=nf * s.plane), _chk(in_bar, numel=nf * s.plane)
    _call(s, "fc_diff_adj", direction, nf, _p(out_bar), _p(in_bar), s.plane)


def fc_continue(s, direction, inp, ext, nf=None):
    nf = nf or inp.numel() // s.plane
    ep = s.ext_size(direction)
    _chk(inp, numel=nf * s.plane), _chk(ext, numel=nf * ep)
    _call(s, "fc_continue", direction, nf, _p(inp), s.plane, _p(ext), ep)


def fc_continue_adj(s, direction, ext_bar, in_bar, nf=None):
    ep = s.ext_size(direction)
    nf = nf or ext_bar.numel() // ep
    _chk(ext_bar, numel=nf * ep), _chk(in_bar, numel=nf * s.plane)
    _call(s, "fc_continue_adj", direction, nf, _p(ext_bar), ep, _p(in_bar), s.plane)


# ------------------------------------------------------------------ right-hand side

def euler_rhs(s, u, metric, ref, gamma, rhs):
    _chk(u, numel=4 * s.plane), _chk(metric, numel=4 * s.plane), _chk(rhs, numel=4 * s.plane)
    ws = s.workspace(WS_RHS)
    _call(s, "euler_rhs", _p(u), _p(metric), _f4(ref), float(gamma), _p(rhs), s.plane, _p(ws), ws.numel() * 4)


def av_apply(s, u, metric, mu, ref, rhs):
    _chk(u, numel=4 * s.plane), _chk(mu, numel=s.plane), _chk(rhs, numel=4 * s.plane)
    ws = s.workspace(WS_RHS)
    _call(s, "av_apply", _p(u), _p(metric), _p(mu), _f4(ref), _p(rhs), s.plane, _p(ws), ws.numel() * 4)


def fcsd_rhs(s, u, metric, mu, ref, gamma, rhs):
    _chk(u, numel=4 * s.plane), _chk(metric, numel=4 * s.plane), _chk(mu, numel=s.plane)
    _chk(rhs, numel=4 * s.plane)
    ws = s.workspace(WS_RHS)
    _call(s, "fcsd_rhs", _p(u), _p(metric), _p(mu), _f4(ref), float(gamma), _p(rhs), s.plane, _p(ws),
          ws.numel() * 4)


def fcsd_rhs_adj(s, u, metric, mu, ref, gamma, rhs_bar, u_bar, mu_bar=None):
    _chk(u, numel=4 * s.plane), _chk(rhs_bar, numel=4 * s.plane), _chk(u_bar, numel=4 * s.plane)
    _chk(mu, numel=s.plane), _chk(mu_bar, numel=s.plane)
    ws = s.workspace(WS_RHS_ADJ)
    _call(s, "fcsd_rhs_adj", _p(u), _p(metric), _p(mu), _f4(ref), float(gamma), _p(rhs_bar), _p(u_bar),
          _p(mu_bar), s.plane, _p(ws), ws.numel() * 4)


def euler_rhs_adj(s, u, metric, ref, gamma, rhs_bar, u_bar):
    """u_bar += transpose of euler_rhs at u applied to rhs_bar."""
    _chk(u, numel=4 * s.plane), _chk(rhs_bar, numel=4 * s.plane), _chk(u_bar, numel=4 * s.plane)
    ws = s.workspace(WS_RHS_ADJ)
    _call(s, "euler_rhs_adj", _p(u), _p(metric), _f4(ref), float(gamma), _p(rhs_bar), _p(u_bar), s.plane, _p(ws),
          ws.numel() * 4)


def av_apply_adj(s, u, metric, mu, ref, rhs_bar, u_bar, mu_bar=None):
    """u_bar (and mu_bar) += transpose of av_apply at (u, mu) applied to rhs_bar."""
    _chk(u, numel=4 * s.plane), _chk(rhs_bar, numel=4 * s.plane), _chk(u_bar, numel=4 * s.plane)
    _chk(mu, numel=s.plane), _chk(mu_bar, numel=s.plane)
    ws = s.workspace(WS_RHS_ADJ)
    _call(s, "av_apply_adj", _p(u), _p(metric), _p(mu), _f4(ref), _p(rhs_bar), _p(u_bar), _p(mu_bar), s.plane,
          _p(ws), ws.numel() * 4)


# ------------------------------------------------------------------ stepping

def rk_stage(s, stage, dt_dev, rhs, u0, ui, acc, uout):
    for t in (rhs, u0, ui, uout):
        _chk(t, numel=4 * s.plane)
    _chk(acc, numel=4 * s.plane), _chk(dt_dev, numel=1)
    _call(s, "rk_stage", int(stage), _p(dt_dev), _p(rhs), _p(u0), _p(ui), _p(acc), _p(uout), s.plane)


def rk_stage_adj(s, stage, dt_dev, uout_bar, u0_bar, ui_bar, acc_bar, rhs_bar):
    _call(s, "rk_stage_adj", int(stage), _p(dt_dev), _p(uout_bar), _p(u0_bar), _p(ui_bar), _p(acc_bar),
          _p(rhs_bar), s.plane)


def fcsd_cfl_dt(s, u, mu, cfl, gamma, dt_dev):
    _chk(u, numel=4 * s.plane), _chk(mu, numel=s.plane), _chk(dt_dev, numel=1)
    ws = s.workspace(WS_AV)
    _call(s, "fcsd_cfl_dt", _p(u), _p(mu), float(cfl), float(gamma), _p(dt_dev), s.plane, _p(ws),
          ws.numel() * 4)


def sdnn_infer_adj(s, u, gamma, W, logits_bar, feat_bar):
    """feat_bar [2][plane][16] = transpose of the network at the state's
    window features applied to logits_bar [2][plane][4] (subgrid points)."""
    _chk(u, numel=4 * s.plane), _chk(logits_bar, numel=8 * s.plane), _chk(feat_bar, numel=32 * s.plane)
    ws = s.workspace(WS_AV)
    m = mlp_struct(W)
    _call(s, "sdnn_infer_adj", _p(u), float(gamma), ctypes.byref(m), _p(logits_bar), _p(feat_bar), s.plane,
          _p(ws), ws.numel() * 4)


def fcsd_cfl_dt_noalloc(s, u, mu, cfl, gamma, dt_dev):
    """fcsd_cfl_dt without a workspace: the library's static per-device
    scratch (at most 16384 patches; overlapping calls on one device race)."""
    _chk(u, numel=4 * s.plane), _chk(mu, numel=s.plane), _chk(dt_dev, numel=1)
    _call(s, "fcsd_cfl_dt_noalloc", _p(u), _p(mu), float(cfl), float(gamma), _p(dt_dev), s.plane)


def fcsd_check(s, u, gamma, flags_dev):
    """State monitor: flags_dev (one int32 on the device) becomes the OR of
    1 (non-finite value), 2 (rho <= 0), 4 (p <= 0) over the grid points."""
    _chk(u, numel=4 * s.plane), _chk(flags_dev, dtype=torch.int32, numel=1)
    _call(s, "fcsd_check", _p(u), float(gamma), _p(flags_dev), s.plane)


# ------------------------------------------------------------------ viscosity

def mlp_struct(W: dict):
    m = Mlp()
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        _chk(W[k], name=k)
        setattr(m, k, W[k].data_ptr())
    return m


def sdnn_infer(s, u, gamma, W, tau, logits=None):
    _chk(u, numel=4 * s.plane), _chk(tau, torch.int8, s.plane), _chk(logits, numel=8 * s.plane)
    m = mlp_struct(W)
    ws = s.workspace(WS_AV)
    _call(s, "sdnn_infer", _p(u), float(gamma), ctypes.byref(m), _p(tau), _p(logits), s.plane, _p(ws),
          ws.numel() * 4)


def av_viscosity(s, u, tau, gamma, mu, argmax=None):
    _chk(u, numel=4 * s.plane), _chk(tau, torch.int8, s.plane), _chk(mu, numel=s.plane)
    _chk(argmax, torch.int32, s.plane)
    ws = s.workspace(WS_AV)
    _call(s, "av_viscosity", _p(u), _p(tau), float(gamma), _p(mu), _p(argmax), s.plane, _p(ws), ws.numel() * 4)


def av_viscosity_adj(s, u, tau, argmax, gamma, mu_bar, u_bar):
    _chk(u, numel=4 * s.plane), _chk(tau, torch.int8, s.plane), _chk(argmax, torch.int32, s.plane)
    _chk(mu_bar, numel=s.plane), _chk(u_bar, numel=4 * s.plane)
    ws = s.workspace(WS_AV)
    _call(s, "av_viscosity_adj", _p(u), _p(tau), _p(argmax), float(gamma), _p(mu_bar), _p(u_bar), s.plane,
          _p(ws), ws.numel() * 4)


def fcsd_glue(s, u, mask=None, state=(0, 0, 0, 0)):
    _chk(u, numel=4 * s.plane), _chk(mask, torch.uint8, s.plane)
    _call(s, "fcsd_glue", _p(u), s.plane, _p(mask), _f4(state))


def fcsd_glue_adj(s, u_bar, mask=None, dstate=(0, 0, 0, 0), dparam=None, glued=None):
    """Transpose of fcsd_glue in place; dparam (float64 device, 1 element)
    is incremented by the Dirichlet points' cotangent dotted with dstate;
    glued: the glue's output state (needed on sets with walls)."""
    _chk(u_bar, numel=4 * s.plane), _chk(mask, torch.uint8, s.plane), _chk(dparam, torch.float64, 1)
    _chk(glued, numel=4 * s.plane)
    _call(s, "fcsd_glue_adj", _p(u_bar), s.plane, _p(mask), _f4(dstate), _p(dparam), _p(glued))


def fcsd_filter(s, u, out, gamma=1.4):
    """Per-step state filter (rho, rho u, rho v, theta; E rebuilt); out may
    be u."""
    _chk(u, numel=4 * s.plane), _chk(out, numel=4 * s.plane)
    _call(s, "fcsd_filter", _p(u), _p(out), s.plane, float(gamma))


def fcsd_smear(s, u, region, out, gamma=1.4, alpha=10.0, p=2, c=18.0, r=9.0):
    """Localized smearing of discontinuous initial data (once, before the
    first step): `region` is a uint8 label plane (discontinuities between
    line neighbours with different labels); out may be u."""
    _chk(u, numel=4 * s.plane), _chk(out, numel=4 * s.plane)
    _chk(region, torch.uint8, s.plane, name="region")
    ws = s.workspace(WS_SMEAR)
    _call(s, "fcsd_smear", _p(u), _p(region), _p(out), s.plane, float(gamma), float(alpha), int(p), float(c),
          float(r), _p(ws), ws.numel() * 4)


def fcsd_filter_adj(s, u, out_bar, u_bar, gamma=1.4):
    """Reverse mode of fcsd_filter at u: u_bar = cotangent of u given the
    filtered state's cotangent out_bar (u_bar may be out_bar)."""
    for t in (u, out_bar, u_bar):
        _chk(t, numel=4 * s.plane)
    ws = s.workspace(WS_FILTER_ADJ)
    _call(s, "fcsd_filter_adj", _p(u), _p(out_bar), _p(u_bar), s.plane, float(gamma), _p(ws), ws.numel() * 4)


# ------------------------------------------------------------------ fused

def fcsd_stage(s, stage, u0, ui, acc, uout, metric, mu, ref, gamma, dt_dev, per_patch=False):
    for t in (u0, ui, acc, uout, metric):
        _chk(t, numel=4 * s.plane)
    _chk(mu, numel=s.plane), _chk(dt_dev, numel=1)
    ws = s.workspace(WS_RHS)
    name = "fcsd_stage_per_patch" if per_patch else "fcsd_stage"
    _call(s, name, int(stage), _p(u0), _p(ui), _p(acc), _p(uout), _p(metric), _p(mu), _f4(ref),
          float(gamma), _p(dt_dev), s.plane, _p(ws), ws.numel() * 4)


def fcsd_stage_adj(s, stage, ui, metric, mu, ref, gamma, dt_dev, uout_bar, u0_bar, ui_bar, acc_bar=None,
                   mu_bar=None):
    """Reverse mode of fcsd_stage at ui (see the header): u0_bar, ui_bar,
    acc_bar, mu_bar accumulated / updated in place."""
    for t in (ui, uout_bar, u0_bar, ui_bar):
        _chk(t, numel=4 * s.plane)
    _chk(acc_bar, numel=4 * s.plane), _chk(mu, numel=s.plane), _chk(mu_bar, numel=s.plane), _chk(dt_dev, numel=1)
    ws = s.workspace(WS_STAGE_ADJ)
    _call(s, "fcsd_stage_adj", int(stage), _p(ui), _p(metric), _p(mu), _f4(ref), float(gamma), _p(dt_dev),
          _p(uout_bar), _p(u0_bar), _p(ui_bar), _p(acc_bar), _p(mu_bar), s.plane, _p(ws), ws.numel() * 4)


def fcsd_stage_pass(s, pass_id, stage, u0, ui, acc, uout, metric, mu, ref, gamma, dt_dev):
    ws = s.workspace(WS_RHS)
    _call(s, "fcsd_stage_pass", int(pass_id), int(stage), _p(u0), _p(ui), _p(acc), _p(uout), _p(metric), _p(mu),
          _f4(ref), float(gamma), _p(dt_dev), s.plane, _p(ws), ws.numel() * 4)


class Stepper:
    """Holds the buffers of fcsd_step (state advanced in place)."""

    def __init__(self, s: PatchSet, u, metric, ref, gamma=1.4, cfl=0.5, W=None, mu=None,
                 dirichlet_mask=None, dirichlet_state=(0, 0, 0, 0), fixed_dt=None, filt=False):
        dev = u.device
        self.s = s
        self.u, self.metric = u, metric
        self.W = W
        self.mu = mu if mu is not None else torch.zeros(s.plane, device=dev)
        self.tau = torch.zeros(s.plane, dtype=torch.int8, device=dev)
        self.argmax = torch.zeros(s.plane, dtype=torch.int32, device=dev)
        self.dt = torch.zeros(1, device=dev)
        self.mask = dirichlet_mask
        a = StepArgs()
        a.u, a.metric, a.mu = u.data_ptr(), metric.data_ptr(), self.mu.data_ptr()
        a.tau, a.argmax, a.dt_dev = self.tau.data_ptr(), self.argmax.data_ptr(), self.dt.data_ptr()
        a.dirichlet_mask = dirichlet_mask.data_ptr() if dirichlet_mask is not None else None
        a.dirichlet_state = _f4(dirichlet_state)
        a.ref = _f4(ref)
        a.gamma, a.cfl = float(gamma), float(cfl)
        a.fixed_dt = 0
        a.fixed_tau = 0
        a.filter = 1 if filt else 0   # spectral filter after the viscosity (PatchSet.set_filter first)
        if fixed_dt is not None:
            self.dt.fill_(float(fixed_dt))
            a.fixed_dt = 1
        self.mlp = mlp_struct(W) if W is not None else None
        a.w = ctypes.cast(ctypes.pointer(self.mlp), ctypes.c_void_p) if W is not None else None
        self.args = a
        self.ws = s.workspace(WS_STEP)

    def new_record(self):
        """A buffer for one step record (RECORD_PLANES float planes)."""
        return torch.empty(RECORD_PLANES * self.s.plane, device=self.u.device)

    def step(self, use_graph=False, record=None):
        """One step; with `record` (from new_record) the step also stores
        what step_adj needs to skip the forward recomputation."""
        _chk(record, torch.float32, RECORD_PLANES * self.s.plane)
        a = self.args
        a.record = record.data_ptr() if record is not None else None
        try:
            _call(self.s, "fcsd_step", ctypes.byref(a), self.s.plane, _p(self.ws), self.ws.numel() * 4,
                  1 if use_graph else 0)
        finally:
            a.record = None

    def replay(self, tau, dt, use_graph=False, record=None):
        """One step with recorded decisions: classes `tau` (int8 plane) and
        step size `dt` (1-element tensor) instead of the network and CFL."""
        a = self.args
        self.tau.copy_(tau)
        self.dt.copy_(dt)
        fd, ft = a.fixed_dt, a.fixed_tau
        a.fixed_dt, a.fixed_tau = 1, 1 if self.W is not None else 0
        try:
            self.step(use_graph=use_graph, record=record)
        finally:
            a.fixed_dt, a.fixed_tau = fd, ft

    def step_adj(self, u_in, u_bar, tau, dt, dstate=(0, 0, 0, 0), dparam=None, record=None):
        """Reverse mode of a step from state u_in with recorded decisions:
        u_bar (cotangent of the step output) becomes the cotangent of u_in;
        dparam (float64, 1 element) gathers the boundary-state derivative.
        With `record` (written by step/replay of this same step) the forward
        step is not recomputed and u_in may be None."""
        if record is None:
            _chk(u_in, numel=4 * self.s.plane)
        _chk(u_bar, numel=4 * self.s.plane)
        _chk(dparam, torch.float64, 1)
        _chk(record, torch.float32, RECORD_PLANES * self.s.plane)
        a = self.args
        self.tau.copy_(tau)
        self.dt.copy_(dt)
        fd, ft = a.fixed_dt, a.fixed_tau
        a.fixed_dt, a.fixed_tau = 1, 1 if self.W is not None else 0
        a.record = record.data_ptr() if record is not None else None
        ws = self.s.workspace(WS_STEP_ADJ)
        try:
            _call(self.s, "fcsd_step_adj", ctypes.byref(a), _p(u_in), _p(u_bar), _f4(dstate), _p(dparam),
                  self.s.plane, _p(ws), ws.numel() * 4)
        finally:
            a.fixed_dt, a.fixed_tau = fd, ft
            a.record = None
