"""Autotuner of the batched line-tile schedule.

The tile split of a patch set decides how many lines share a workgroup (and
so how many threads work on each line: 256 / lines) and how long the
contiguous row segments of the q2-line passes are; the launch order decides
which die (L2) runs which tiles.  Results do not depend on either: every
line is transformed by the same arithmetic whatever its tile.  The tuner
times the four passes of one stage through fcsd_stage_pass with HIP events
on the library's stream, picks the fastest LDS budget for the q1-line passes
(A, C) and for the q2-line passes (B1, B2) under each launch order, and
keeps the order with the smallest stage time.
"""
from __future__ import annotations

import torch

from . import api

Q1_PASSES = (0, 3)   # A, C
Q2_PASSES = (1, 2)   # B1, B2
DEFAULT_BUDGETS = (16384, 24576, 32768, 49152, 65536, 98304, 131072, 163840)


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


def autotune(s, u, metric, mu, ref, gamma=1.4, dt=None, budgets=DEFAULT_BUDGETS,
             orders=(api.PatchSet.ORDER_LPT, api.PatchSet.ORDER_XCD), reps=3):
    """Choose (q1 budget, q2 budget, order) for patch set `s` on state `u`;
    applies the choice and returns it with the timing table."""
    dev = u.device
    ui = torch.empty_like(u).copy_(u)
    acc = torch.zeros_like(u)
    uout = torch.zeros_like(u)
    if dt is None:
        dt = torch.full((1,), 1e-6, device=dev)
    bufs = (u, ui, acc, uout, metric, mu, ref, gamma, dt)
    table = {}
    usable = []
    for b in budgets:
        try:
            s.tune(b, b, orders[0])
            usable.append(b)
        except api.FcsdError:      # above the device's LDS per workgroup
            pass
    budgets = tuple(usable)
    for order in orders:
        for b in budgets:
            s.tune(b, b, order)
            t = time_passes(s, bufs, Q1_PASSES + Q2_PASSES, reps)
            table[(order, b)] = t
    best = None
    for order in orders:
        b1 = min(budgets, key=lambda b: sum(table[(order, b)][p] for p in Q1_PASSES))
        b2 = min(budgets, key=lambda b: sum(table[(order, b)][p] for p in Q2_PASSES))
        ms = sum(table[(order, b1)][p] for p in Q1_PASSES) + sum(table[(order, b2)][p] for p in Q2_PASSES)
        if best is None or ms < best[3]:
            best = (b1, b2, order, ms)
    s.tune(best[0], best[1], best[2])
    return {"q1_budget": best[0], "q2_budget": best[1], "order": "xcd" if best[2] else "lpt",
            "stage_passes_ms": best[3],
            "table": {f"{'xcd' if o else 'lpt'}-{b // 1024}K": {["A", "B1", "B2", "C"][p]: round(v, 4)
                                                              for p, v in t.items()}
                      for (o, b), t in table.items()}}
