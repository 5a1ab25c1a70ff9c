"""Autotuner of the batched line-tile schedule.

The tile split of a patch set decides how many lines share a workgroup,
the workgroup size how many threads work on each line, the launch order
which die (L2) runs which tiles, and the stage schedule how the passes are
launched (four launches, three with passes B1 and B2 fused on one q2 tile,
or one persistent launch per stage).  Results do not depend on any of them:
every line is transformed by the same arithmetic whatever its tile and
launch.  There are three tile sets -- q1 lines (passes A, C), q2 lines
(pass B2), q2 lines with two complex lines per grid line (passes B1 and the
fused B) -- each with its own LDS budget and workgroup size.  The tuner
times the passes of one stage through fcsd_stage_pass with HIP events on
the library's stream for every (budget, workgroup size) candidate under each
launch order, picks the best candidate per tile set for the split and the
fused schedules, times whole stages of both and of persistent candidates
(one workgroup size and budgets that leave room for the queue slot), and
keeps the fastest.
"""
from __future__ import annotations

import torch

from . import api

SET_PASSES = ((0, 3), (2,), (1,))   # tile set -> passes timed (A+C, B2, B1)
FUSED_PASSES = ((0, 3), (2,), (4,))  # the same with the fused B pass on the third set
WIDE_PASSES = ((0, 3), (2,), (5,))   # the fused B pass with all H fields in LDS
PERSISTENT_BUDGET = 163840 - 256    # leaves room for the persistent kernel's queue slot
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


def time_stage(s, bufs, reps=3):
    """Mean milliseconds of one whole stage (stage 1) under the set's
    current schedule."""
    u0, ui, acc, uout, metric, mu, ref, gamma, dt = bufs
    ctx = s.ctx
    api.fcsd_stage(s, 1, u0, ui, acc, uout, metric, mu, ref, gamma, dt)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    for _ in range(reps):
        api.fcsd_stage(s, 1, u0, ui, acc, uout, metric, mu, ref, gamma, dt)
    e1.record(ctx.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(s, u, metric, mu, ref, gamma=1.4, dt=None, budgets=DEFAULT_BUDGETS, threads=DEFAULT_THREADS,
             orders=(api.PatchSet.ORDER_LPT, api.PatchSet.ORDER_XCD), reps=3, schedules=(0, 1, 2, 3)):
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
            tm = time_passes(s, bufs, (0, 1, 2, 3, 4), reps)
            try:
                tm.update(time_passes(s, bufs, (5,), reps))
            except api.FcsdError:     # wide q2 tiles do not fit the LDS at this budget
                tm[5] = float("inf")
            table[(order, b, t)] = tm
    # per-set picks of the split and fused schedules under each order, then
    # whole stages of each pick and of the persistent candidates
    stage = []   # (ms, schedule, budgets, threads, order)
    for order in orders:
        for sched, set_passes in ((0, SET_PASSES), (1, FUSED_PASSES), (3, WIDE_PASSES)):
            if sched not in schedules:
                continue
            pick = [min(cands, key=lambda bt: sum(table[(order,) + bt][p] for p in passes))
                    for passes in set_passes]
            bud, thr = [c[0] for c in pick], [c[1] for c in pick]
            s.tune(bud, thr, order)
            try:
                s.set_schedule(sched)
            except api.FcsdError:
                continue
            stage.append((time_stage(s, bufs, reps), sched, bud, thr, order))
        if 2 in schedules:
            # one workgroup size for every task of the launch; budgets of the
            # fused pick, capped for the queue slot, and uniform ones
            fused = [r for r in stage if r[1] == 1 and r[4] == order]
            fb = fused[-1][2] if fused else [max(budgets)] * 3
            pers = {tuple(min(b, PERSISTENT_BUDGET) for b in fb)} | \
                {(b, b, b) for b in budgets if 65536 <= b <= PERSISTENT_BUDGET}
            pthreads = [t for t in threads if t >= 512] or [max(threads)]
            for bud in sorted(pers):
                for t in pthreads:
                    try:
                        s.tune(list(bud), [t] * 3, order)
                        s.set_schedule(2)
                    except api.FcsdError:
                        continue
                    stage.append((time_stage(s, bufs, reps), 2, list(bud), [t] * 3, order))
    ms, sched, bud, thr, order = min(stage, key=lambda r: r[0])
    s.tune(bud, thr, order)
    s.set_schedule(sched)
    names = ["split", "fused", "persistent", "fused_wide"]
    return {"budgets": bud, "threads": thr, "order": "xcd" if order else "lpt", "schedule": names[sched],
            "stage_ms": ms,
            "stages": [{"ms": round(r[0], 4), "schedule": names[r[1]], "budgets": r[2], "threads": r[3],
                        "order": "xcd" if r[4] else "lpt"} for r in stage],
            "table": {f"{'xcd' if o else 'lpt'}-{b // 1024}K-{t}": {["A", "B1", "B2", "C", "Bf", "Bw"][p]: round(v, 4)
                                                                   for p, v in tm.items()}
                      for (o, b, t), tm in table.items()}}
