"""Autotuner of the batched line-tile schedule.

The tile split of a patch set decides how many lines share a workgroup,
the workgroup size how many threads work on each line, and the launch order
which die (L2) runs which tiles.  Results do not depend on any of them:
every line is transformed by the same arithmetic whatever its tile.  There
are three tile sets -- q1 lines (passes A, C), q2 lines (pass B2), q2 lines
with two complex lines per grid line (pass B1) -- each with its own LDS
budget and workgroup size.  The tuner times the four passes of one stage
through fcsd_stage_pass with HIP events on the library's stream for every
(budget, workgroup size) candidate under each launch order, picks the best
candidate per tile set and keeps the order with the smallest stage time.
"""
from __future__ import annotations

import torch

from . import api

SET_PASSES = ((0, 3), (2,), (1,))   # tile set -> passes timed (A+C, B2, B1)
DEFAULT_BUDGETS = (24576, 32768, 49152, 65536, 81920, 98304, 131072, 163840)
DEFAULT_THREADS = (256, 512, 1024)


def time_passes(s, bufs, passes, reps=3):
    """Mean milliseconds of each pass in `passes` (stage 1 of SSPRK)."""
    u0, ui, acc, uout, metric, mu, ref, gamma, dt = bufs
    ctx = s.ctx
    out = {}
    # every pass reads what the passes before it wrote
    for q in range(4):
        api.fcsd_stage_pass(s, q, 1, u0, ui, acc, uout, metric, mu, ref, gamma, dt)
    for p in passes:
        api.fcsd_stage_pass(s, p, 1, u0, ui, acc, uout, metric, mu, ref, gamma, dt)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            api.fcsd_stage_pass(s, p, 1, u0, ui, acc, uout, metric, mu, ref, gamma, dt)
        e1.record(ctx.stream)
        e1.synchronize()
        out[p] = e0.elapsed_time(e1) / reps
    return out


def autotune(s, u, metric, mu, ref, gamma=1.4, dt=None, budgets=DEFAULT_BUDGETS, threads=DEFAULT_THREADS,
             orders=(api.PatchSet.ORDER_LPT, api.PatchSet.ORDER_XCD), reps=3):
    """Choose the schedule of patch set `s` on state `u`; applies the choice
    and returns it with the timing table."""
    dev = u.device
    ui = torch.empty_like(u).copy_(u)
    acc = torch.zeros_like(u)
    uout = torch.zeros_like(u)
    if dt is None:
        dt = torch.full((1,), 1e-6, device=dev)
    bufs = (u, ui, acc, uout, metric, mu, ref, gamma, dt)
    cands = []
    for t in threads:
        for b in budgets:
            try:
                s.tune(b, t, orders[0])
                cands.append((b, t))
            except api.FcsdError:      # above the device's LDS per workgroup
                pass
    table = {}
    for order in orders:
        for (b, t) in cands:
            s.tune(b, t, order)
            table[(order, b, t)] = time_passes(s, bufs, (0, 1, 2, 3), reps)
    best = None
    for order in orders:
        pick, ms = [], 0.0
        for passes in SET_PASSES:
            c = min(cands, key=lambda bt: sum(table[(order,) + bt][p] for p in passes))
            pick.append(c)
            ms += sum(table[(order,) + c][p] for p in passes)
        if best is None or ms < best[2]:
            best = (pick, order, ms)
    pick, order, ms = best
    s.tune([c[0] for c in pick], [c[1] for c in pick], order)
    return {"budgets": [c[0] for c in pick], "threads": [c[1] for c in pick],
            "order": "xcd" if order else "lpt", "stage_passes_ms": ms,
            "table": {f"{'xcd' if o else 'lpt'}-{b // 1024}K-{t}": {["A", "B1", "B2", "C"][p]: round(v, 4)
                                                                   for p, v in tm.items()}
                      for (o, b, t), tm in table.items()}}
