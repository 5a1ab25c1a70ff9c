"""Throughput of the FC-SDNN hot path on one MI355X.

Workload: 200 independent annulus-sector patches with side lengths drawn
uniformly from 48..512 (seed 2), Mach-3 flow with a seeded 1% density
perturbation, FP32 state, network classifier and smooth artificial
viscosity every step, SSPRK(5,4) (five stages per step).  A timed "step" is
one full time step of the hot path: glue, network classes, preliminary
viscosity and smoothing-blending operator, CFL step size and five fused
stages, replayed as one captured hipGraph.

Metric: grid-point RK stages per second = points x 5 x steps / time.  Also
reported: the per-patch plain variant of the stages, the dominant kernel's
achieved algorithmic bandwidth against the HBM peak (HIP events around
repeated launches of that pass on the library's stream) and the FP64 oracle
timed on a bounded sample of the same workload on the host CPU.

HBM traffic of the dominant kernel comes from rocprofv3 FETCH_SIZE and
WRITE_SIZE counter runs of this script (recorded in profiles/traffic.txt
together with a digest of the kernel sources; reported as null when the
sources have changed since).  --copy-calib adds a plain device copy of known
size to the run, whose counter readings give the scale factor.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--no-per-patch] [--copy-calib] [--layout rows|blocked]
                       [--schedule auto|B0,B1,B2,T0,T1,T2,ORDER]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["engine.h", "kernels.h", "kernels2.h", "radix.h", "radix_gen.h", "fcsdnn.hip"]
COPY_MIB = 1024


def source_digest():
    """sha256 over the device sources, to tie counter readings to a build."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2506_16076_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, npts):
    """HBM bytes per launch of `kernel` from profiles/traffic.txt (lines
    key=value), scaled by the copy-kernel factor; None if absent or stale."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#") or "=" not in line:
                continue
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    if rec.get("source_digest") != source_digest() or rec.get("kernel") != kernel or \
            int(rec.get("points", -1)) != npts:
        return None
    fetch = float(rec["fetch_kib"]) * 1024 / float(rec["copy_fetch_factor"])
    write = float(rec["write_kib"]) * 1024 / float(rec["copy_write_factor"])
    return fetch + write


# per-step filter: q1 pass reads and writes the 4 state fields, the q2 pass
# again (FP32)
FILTER_BYTES = 64

PASS_KERNEL = {"A": "k_dev_diff2<1>", "B1": "k_passB1", "B2": "k_passB2", "C": "k_passC", "Bf": "k_passB",
               "Bw": "k_passB4", "stage": "k_stage"}
# passes of a stage under each schedule (Bf: passes B1 and B2 in one launch)
SCHED_PASSES = {"split": ["A", "B1", "B2", "C"], "fused": ["A", "Bf", "C"], "persistent": ["A", "Bf", "C"],
                "fused_wide": ["A", "Bw", "C"]}
SCHED_ID = {"split": 0, "fused": 1, "persistent": 2, "fused_wide": 3}


def pass_bytes(stage):
    """Algorithmic HBM bytes per grid point of each pass of one stage (FP32).
    A: read e (16), write d1e (16).  B1: read e, d1e, metric, mu (52), write H
    (32).  B2: read H (32), metric q2 row (8), write r2 (16).  C: read H (32),
    r2 (16), metric q1 row (8), register reads/writes of the stage."""
    rk_read = {0: 16, 1: 32, 2: 32, 3: 48, 4: 32}[stage]
    rk_write = {0: 16, 1: 16, 2: 32, 3: 32, 4: 16}[stage]
    # Bf: read e, d1e, metric, mu (52), write H (32) and r2 (16)
    return {"A": 32, "B1": 84, "B2": 56, "C": 32 + 16 + 8 + rk_read + rk_write, "Bf": 100, "Bw": 100}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_patch_step(args):
    """One full oracle step (network, viscosity, dt, five stages) of one
    patch of the workload, in a single-threaded pool worker; returns
    (points, seconds)."""
    p, n1, n2, d, mach, pert, ref, mlp = args
    import synth
    from oracle import fcgram, solver
    fcgram.FFT_WORKERS = 1
    sub = synth._polar_patches([(0.3 * p, ((2 * np.pi / 16) * 255 / 237) / (n1 - 1), 0.5, 1.5 / (n2 - 1))],
                               [n1], [n2], d, 27)
    e = synth.mach_state(sub, mach, pert)
    c = synth.Config("sample", sub, synth._f32(e, sub), ref, mach=mach, pert=pert, mlp=mlp)
    run = solver.Run(c)
    t0 = time.perf_counter()
    run.step()
    return n1 * n2, time.perf_counter() - t0


_THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def _single_thread_env():
    """Pool worker initializer: one BLAS thread (the environment the worker
    was spawned with already says so; threadpoolctl covers a BLAS that was
    loaded before)."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:  # pragma: no cover
        pass


def cpu_baseline(cfg, budget_s=20.0, workers=None):
    """The oracle (FP64 numpy) over the host's cores: a process pool of
    single-threaded workers, one patch of the workload each (the bench
    workload's patches are independent), one full step per patch; patches
    are handed out in the workload's order as workers free up until ~budget_s
    of wall time has passed.  Throughput = the points stepped x 5 / the wall
    time until the last of them finished."""
    import multiprocessing as mp

    ps = cfg.ps
    workers = workers or min(os.cpu_count() or 1, 16)
    ctx = mp.get_context("spawn")
    pts, wall, used = 0, 0.0, 0
    saved = {k: os.environ.get(k) for k in _THREAD_VARS}
    for k in _THREAD_VARS:
        os.environ[k] = "1"            # inherited by the spawned workers
    try:
        pool = ctx.Pool(workers, initializer=_single_thread_env)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    with pool:
        # warm the workers (imports) outside the timed region
        pool.map(_single_thread_env_probe, range(workers))
        todo = [(q, int(ps.n1[q]), int(ps.n2[q]), ps.d, cfg.mach, cfg.pert, cfg.ref, cfg.mlp)
                for q in range(ps.npatch)]
        t0 = time.perf_counter()
        flight = [pool.apply_async(_oracle_patch_step, (todo[q],)) for q in range(min(workers, len(todo)))]
        nxt = len(flight)
        while flight:
            done = [f for f in flight if f.ready()]
            if not done:
                time.sleep(0.005)
                continue
            for f in done:
                flight.remove(f)
                n, _ = f.get()
                pts += n
                used += 1
                if nxt < len(todo) and time.perf_counter() - t0 < budget_s:
                    flight.append(pool.apply_async(_oracle_patch_step, (todo[nxt],)))
                    nxt += 1
        wall = time.perf_counter() - t0
    return {"value": pts * 5 / wall, "unit": "grid-pt RK-stages/s", "cores": workers, "kind": "oracle",
            "cpu": _cpu_model(),
            "sample": f"{used} of {ps.npatch} patches ({pts} points), one full step each, FP64 numpy, "
                      f"pool of {workers} single-threaded processes, {wall:.1f} s wall"}


def _single_thread_env_probe(_):
    import synth  # noqa: F401
    from oracle import solver  # noqa: F401
    return 0


def oracle_configs():
    """The FP64 oracle (one process, library FFT and BLAS threads on the
    host) on the 64 x 64 square for its 10 steps and on the 64-patch annulus
    of 512 x 512 patches for one step (network, viscosity, glue and inflow
    at every stage), in grid-pt RK-stages/s."""
    import synth
    from oracle import solver
    out = {"cpu": _cpu_model(), "threads": os.cpu_count()}
    for name, idx, steps in (("square_64x64_10_steps", 0, 10), ("annulus_64x512x512_1_step", 4, 1)):
        cfg = synth.config(idx)
        run = solver.Run(cfg)
        t0 = time.perf_counter()
        for k in range(steps):
            run.step(progress=lambda st, k=k: print(f"  {name}: step {k} stage {st} done, "
                                                     f"{time.perf_counter() - t0:.1f} s", file=sys.stderr,
                                                     flush=True))
        secs = time.perf_counter() - t0
        out[name] = {"points": cfg.ps.npoints, "steps": steps, "seconds": secs,
                     "value": cfg.ps.npoints * 5 * steps / secs, "finite": bool(np.isfinite(run.u).all())}
        print(name, out[name], file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--npatch", type=int, default=200)
    ap.add_argument("--no-per-patch", action="store_true")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--no-paper", action="store_true", help="skip the 101 x 101, d = 2 subpatch workload")
    ap.add_argument("--layout", default="blocked", choices=["rows", "blocked"],
                    help="plane storage: row-major or 8x4 blocks (default)")
    ap.add_argument("--adj-steps", type=int, default=8, help="steps of the timed reverse sweep (0: skip)")
    ap.add_argument("--adj-every", type=int, default=4, help="checkpoint spacing of the reverse sweep")
    ap.add_argument("--schedule", default="auto",
                    help="auto (autotuner) or B_q1,B_q2,B_q2wide,T_q1,T_q2,T_q2wide,lpt|xcd[,split|fused|"
                         "persistent] (LDS budgets in bytes, workgroup sizes, launch order, stage schedule)")
    ap.add_argument("--oracle-configs", action="store_true",
                    help="only time the FP64 oracle on the host: the 64 x 64 square for its 10 steps and the "
                         "64-patch annulus (16.8 M points) for one step, one process; prints one JSON line")
    args = ap.parse_args()
    if args.oracle_configs:
        print(json.dumps(oracle_configs()), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus must be 1 "
              "(multi-GPU sharding by whole patches is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2506_16076_amd import api

    cfg = synth.config(2, npatch=args.npatch)
    ps = cfg.ps
    ctx = api.Context(0)
    layout = {"rows": 0, "blocked": 1}[args.layout]
    s = api.PatchSet.from_layout(ctx, ps, layout)
    dev = "cuda:0"

    def t(a, dtype=None):
        x = torch.from_numpy(np.ascontiguousarray(a).reshape(-1))
        return (x.to(dtype) if dtype else x).to(dev).contiguous()

    u = s.to_device(cfg.u0)
    metric = s.to_device(ps.metric)
    W = {k: t(v) for k, v in cfg.mlp.items()}
    npts = ps.npoints
    # schedule: autotuned tile split and launch order (outside the timed region)
    if args.schedule == "auto":
        from paper_2506_16076_amd import autotune
        mu0 = torch.full((s.plane,), 1e-3, device=dev)
        tuning = autotune.autotune(s, u, metric, mu0, cfg.ref, 1.4)
        print("autotune:", json.dumps(tuning), file=sys.stderr, flush=True)
    else:
        # B0,B1,B2,T0,T1,T2,ORDER: LDS budgets and workgroup sizes of the three tile sets
        f = args.schedule.split(",")
        bud, thr, order = [int(x) for x in f[0:3]], [int(x) for x in f[3:6]], f[6]
        sched = f[7] if len(f) > 7 else "fused"
        s.tune(bud, thr, {"lpt": 0, "xcd": 1}[order])
        s.set_schedule(SCHED_ID[sched])
        tuning = {"budgets": bud, "threads": thr, "order": order, "schedule": sched, "given": True}

    aux_tuning = {}

    def apply_tuning(ss, uu=None, mm=None, ref=None, name=None):
        order = {"lpt": 0, "xcd": 1}[tuning["order"]]
        if tuning.get("given") or uu is None:
            ss.tune(tuning["budgets"], tuning["threads"], order)
            ss.set_schedule(SCHED_ID[tuning["schedule"]])
            return
        # the other workloads are tuned for themselves too (a patch set's
        # best tiles depend on its line lengths), quickly: among the main
        # workload's budgets and workgroup sizes and the largest ones
        from paper_2506_16076_amd import autotune
        mu0 = torch.full((ss.plane,), 1e-3, device=dev)
        r = autotune.autotune(ss, uu, mm, mu0, ref, 1.4, budgets=tuple(sorted(set(tuning["budgets"]) | {163840})),
                              threads=tuple(sorted(set(tuning["threads"]) | {1024})), orders=(order,),
                              schedules=(0, 1, 3))
        aux_tuning[name] = {k: r[k] for k in ("budgets", "threads", "order", "schedule", "stage_ms")}
    st = api.Stepper(s, u, metric, cfg.ref, W=W)

    # ---------------- full step, graph replay
    for _ in range(args.warmup):
        st.step(use_graph=True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(ctx.stream):
        ev0.record(ctx.stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st.step(use_graph=True)
    with torch.cuda.stream(ctx.stream):
        ev1.record(ctx.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / args.steps
    value = npts * 5 * args.steps / (ms / 1e3)
    finite = bool(torch.isfinite(u).all().item())

    # ---------------- stages only: batched vs per-patch (same state, frozen mu, dt)
    mu = st.mu
    dtd = st.dt
    acc = torch.zeros_like(u)
    ua = torch.zeros_like(u)
    ub = torch.zeros_like(u)

    uc = torch.zeros_like(u)

    def stages(per_patch):
        ins, outs = [u, ua, ub, ua, ub], [ua, ub, ua, ub, uc]
        for k in range(5):
            api.fcsd_stage(s, k, u, ins[k], acc, outs[k], metric, mu, cfg.ref, 1.4, dtd, per_patch=per_patch)

    def time_stages(per_patch, reps):
        stages(per_patch)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            stages(per_patch)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_batched = time_stages(False, 3)
    # the same stages under each schedule at the chosen tiling
    sched_ms = {}
    for name, sid in SCHED_ID.items():
        try:
            s.set_schedule(sid)
        except api.FcsdError:
            sched_ms[name] = None
            continue
        sched_ms[name] = time_stages(False, 3) / 5
    s.set_schedule(SCHED_ID[tuning["schedule"]])
    stage_errors = s.stage_errors()
    ms_pp = None if args.no_per_patch else time_stages(True, 2)

    # ---------------- per-pass timing (dominant kernel), every pass at each
    # of the five stages (pass C's register traffic depends on the stage)
    names = ["A", "B1", "B2", "C", "Bf", "Bw"]
    passes, pass_gb = {}, {}
    for pid, name in enumerate(names):
        tot_ms, tot_bytes = 0.0, 0.0
        if name == "Bw":
            try:   # the wide q2 tiles may not fit the LDS at the tuned budget
                api.fcsd_stage_pass(s, pid, 0, u, ua, acc, ub, metric, mu, cfg.ref, 1.4, dtd)
            except api.FcsdError:
                passes[name] = pass_gb[name] = None
                continue
        for stage in range(5):
            # prerequisites so every pass reads defined data
            for q in range(min(pid + 1, 4)):
                api.fcsd_stage_pass(s, q, stage, u, ua, acc, ub, metric, mu, cfg.ref, 1.4, dtd)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 4
            e0.record(ctx.stream)
            for _ in range(reps):
                api.fcsd_stage_pass(s, pid, stage, u, ua, acc, ub, metric, mu, cfg.ref, 1.4, dtd)
            e1.record(ctx.stream)
            torch.cuda.synchronize()
            tot_ms += e0.elapsed_time(e1) / reps
            tot_bytes += pass_bytes(stage)[name] * npts
        passes[name] = tot_ms / 5
        pass_gb[name] = tot_bytes / 5 / 1e9
    used = SCHED_PASSES[tuning["schedule"]]
    if tuning["schedule"] == "persistent":
        # one kernel per stage: its bytes are those of its passes, its time the stage's
        passes["stage"] = ms_batched / 5
        pass_gb["stage"] = sum(pass_gb[n] for n in used)
        dom = "stage"
    else:
        dom = max(used, key=passes.get)
    achieved = pass_gb[dom] / (passes[dom] / 1e3)
    stage_bytes = sum(pass_gb[n] for n in used) * 1e9 / npts
    traffic = recorded_traffic(PASS_KERNEL[dom], npts)

    # ---------------- per-step spectral filter (paper Sec. 4.3.1, alpha 10,
    # p 14), timed on its own: two line passes over the state in place
    s.set_filter(10.0, 14)
    uf = u.clone()
    api.fcsd_filter(s, uf, uf, 1.4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    for _ in range(4):
        api.fcsd_filter(s, uf, uf, 1.4)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    ms_filter = e0.elapsed_time(e1) / 4
    filt = {"ms": ms_filter, "bytes_per_point": FILTER_BYTES,
            "achieved_GBs": FILTER_BYTES * npts / (ms_filter / 1e3) / 1e9,
            "finite": bool(torch.isfinite(uf).all().item())}
    del uf

    # ---------------- reverse mode: checkpointed adjoint of K steps
    adjoint = None
    if args.adj_steps > 0:
        from paper_2506_16076_amd import autodiff
        K, every = args.adj_steps, args.adj_every
        u_start = u.clone()
        par = torch.zeros((), device=dev, requires_grad=True)
        # one untimed forward and backward first: the reverse sweep's buffers
        # (step records, workspace) are allocated there, as in any repeated
        # gradient evaluation
        for warm in (True, False):
            u.copy_(u_start)
            u0 = u_start.clone().requires_grad_(True)
            uT = autodiff.rollout(st, u0, par, K, every)
            gseed = torch.ones_like(uT)
            if warm:
                uT.backward(gseed)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        uT.backward(gseed)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms_adj = e0.elapsed_time(e1)
        adjoint = {"value": npts * 5 * K / (ms_adj / 1e3), "unit": "grid-pt RK-stages/s (reverse, incl. "
                   "checkpoint recomputation)", "steps": K, "checkpoint_every": every, "ms_per_step": ms_adj / K,
                   "finite": bool(torch.isfinite(u0.grad).all().item())}
        u.copy_(u_start)

    # ---------------- the paper's discretisation at the same point count:
    # 48 x 32 annulus subpatches of 101 x 101 (d = 2, C = 27, L = 128) with
    # fringe glue, the Dirichlet inflow and the cylinder wall, network every
    # step
    paper = None
    if not args.no_paper:
        pc = synth.with_cylinder_wall(synth.paper_subpatches(48, 32))
        pps = pc.ps
        s2 = api.PatchSet.from_layout(ctx, pps, layout)
        s2.set_walls(pps.wall, 1.4)
        u2 = s2.to_device(pc.u0)
        m2 = s2.to_device(pps.metric)
        apply_tuning(s2, u2, m2, pc.ref, "paper_subpatches")
        st2 = api.Stepper(s2, u2, m2, pc.ref, W={k: t(v) for k, v in pc.mlp.items()},
                          dirichlet_mask=s2.to_device(pps.dirichlet), dirichlet_state=synth.freestream(pc.mach))
        for _ in range(args.warmup):
            st2.step(use_graph=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(args.steps):
            st2.step(use_graph=True)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms2 = e0.elapsed_time(e1) / args.steps
        paper = {"workload": f"annulus, {pps.npatch} subpatches of 101 x 101 (48 sectors x 32 shells), d 2, "
                             f"C 27 (L 128), fringe glue, Dirichlet inflow, no-slip adiabatic cylinder wall, "
                             f"network every step",
                 "points": int(pps.npoints), "value": pps.npoints * 5 / (ms2 / 1e3), "unit": "grid-pt RK-stages/s",
                 "ms_per_step": ms2, "finite": bool(torch.isfinite(u2).all().item())}
        s2.close()
        del st2, u2

    # ---------------- the strict continuation length: the bench workload with
    # C = 27 on every line; most extension lengths N + 27 have a prime factor
    # above 13 and their circulants run embedded in a 13-smooth transform of
    # length >= N + L (about twice the transform work)
    strict = None
    if not args.no_paper:
        sps = synth.with_continuation(ps, 27)
        nemb = sum(1 for n in list(sps.n1) + list(sps.n2) if not synth.smooth13(int(n) + 27))
        s5 = api.PatchSet.from_layout(ctx, sps, layout)
        u5 = s5.to_device(cfg.u0)
        m5 = s5.to_device(sps.metric)
        apply_tuning(s5, u5, m5, cfg.ref, "strict_continuation")
        st5 = api.Stepper(s5, u5, m5, cfg.ref, W=W)
        for _ in range(args.warmup):
            st5.step(use_graph=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(args.steps):
            st5.step(use_graph=True)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms5 = e0.elapsed_time(e1) / args.steps
        strict = {"workload": "the bench workload with C = 27 on every line (no 13-smooth rule)",
                  "embedded_line_families": nemb, "line_families": 2 * sps.npatch,
                  "value": npts * 5 / (ms5 / 1e3), "unit": "grid-pt RK-stages/s", "ms_per_step": ms5,
                  "finite": bool(torch.isfinite(u5).all().item())}
        s5.close()
        del st5, u5

    # ---------------- inter-patch interpolation (Sec. 3.4.1) on a Cartesian /
    # polar pair of 1024 x 1024 patches that overlap without shared grid
    # lines: step rate with the network viscosity
    interp_rec = None
    if not args.no_paper:
        oc = synth.overlap_config(1024, network=True)
        ops = oc.ps
        s3 = api.PatchSet.from_layout(ctx, ops, layout)
        nrecv = s3.set_interp(ops.geom)
        u3 = s3.to_device(oc.u0)
        apply_tuning(s3, u3, s3.to_device(ops.metric), oc.ref, "interpolated_pair")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st3 = api.Stepper(s3, u3, s3.to_device(ops.metric), oc.ref, W={k: t(v) for k, v in oc.mlp.items()})
        for _ in range(args.warmup):
            st3.step(use_graph=True)
        torch.cuda.synchronize()
        e0.record(ctx.stream)
        for _ in range(args.steps):
            st3.step(use_graph=True)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms3 = e0.elapsed_time(e1) / args.steps
        interp_rec = {"workload": "Cartesian / polar patch pair, 1024 x 1024 each, fringe interpolated at every stage "
                                  "(3 x 3 Neville stencils), network viscosity smoothed across the pair",
                      "points": int(ops.npoints), "receivers": int(nrecv),
                      "value": ops.npoints * 5 / (ms3 / 1e3), "unit": "grid-pt RK-stages/s", "ms_per_step": ms3,
                      "finite": bool(torch.isfinite(u3).all().item())}
        s3.close()
        del st3, u3

    # ---------------- the 64-patch annulus (16 sectors x 4 shells of 512 x 512,
    # Mach 5, glue and inflow every stage, network every step): forward step
    # rate, a 20-step checkpointed reverse sweep (checkpoints every 5) and the
    # device memory both need
    shells = None
    if not args.no_paper:
        from paper_2506_16076_amd import autodiff
        c4 = synth.config(4)
        ps4 = c4.ps
        torch.cuda.synchronize()
        mem0 = torch.cuda.memory_allocated()      # buffers of the other workloads still held
        s4 = api.PatchSet.from_layout(ctx, ps4, layout)
        u4 = s4.to_device(c4.u0)
        m4 = s4.to_device(ps4.metric)
        apply_tuning(s4, u4, m4, c4.ref, "annulus_shells")
        st4 = api.Stepper(s4, u4, m4, c4.ref, W={k: t(v) for k, v in c4.mlp.items()},
                          dirichlet_mask=s4.to_device(ps4.dirichlet), dirichlet_state=synth.freestream(c4.mach))
        for _ in range(args.warmup):
            st4.step(use_graph=True)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base4 = torch.cuda.memory_allocated()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        C4_STEPS = 100          # the configuration's forward run
        e0.record(ctx.stream)
        for _ in range(C4_STEPS):
            st4.step(use_graph=True)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms4 = e0.elapsed_time(e1) / C4_STEPS
        fwd_peak = torch.cuda.max_memory_allocated()
        K4, every4 = 20, 5
        ustart = u4.clone()
        for warm in (True, False):
            u4.copy_(ustart)
            v0 = ustart.clone().requires_grad_(True)
            par4 = torch.zeros((), device=dev, requires_grad=True)
            uT4 = autodiff.rollout(st4, v0, par4, K4, every4, autodiff.freestream_dmach(c4.mach))
            seed = torch.ones_like(uT4)
            if warm:
                uT4.backward(seed)
                torch.cuda.synchronize()
                torch.cuda.reset_peak_memory_stats()
        e0.record(ctx.stream)
        uT4.backward(seed)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms4a = e0.elapsed_time(e1)
        adj_peak = torch.cuda.max_memory_allocated()
        fin4 = bool(torch.isfinite(v0.grad).all().item())
        del uT4, seed, v0
        # the same sweep without step records: each step is recomputed from
        # its input inside the reverse mode (less memory, one more forward)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        u4.copy_(ustart)
        v0 = ustart.clone().requires_grad_(True)
        par4 = torch.zeros((), device=dev, requires_grad=True)
        uT4 = autodiff.rollout(st4, v0, par4, K4, every4, autodiff.freestream_dmach(c4.mach), record=False)
        seed = torch.ones_like(uT4)
        e0.record(ctx.stream)
        uT4.backward(seed)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms4n = e0.elapsed_time(e1)
        nrec_peak = torch.cuda.max_memory_allocated()
        shells = {"workload": "annulus of 16 sectors x 4 shells of 512 x 512, Mach 5 +-1% density, fringe glue "
                              "and Dirichlet inflow every stage, network every step",
                  "points": int(ps4.npoints), "value": ps4.npoints * 5 / (ms4 / 1e3), "unit": "grid-pt RK-stages/s",
                  "ms_per_step": ms4, "steps": C4_STEPS,
                  "adjoint": {"value": ps4.npoints * 5 * K4 / (ms4a / 1e3), "steps": K4, "checkpoint_every": every4,
                              "ms_per_step": ms4a / K4, "finite": fin4},
                  "adjoint_without_records": {"value": ps4.npoints * 5 * K4 / (ms4n / 1e3), "steps": K4,
                                              "checkpoint_every": every4, "ms_per_step": ms4n / K4,
                                              "reverse_peak_GB": (nrec_peak - mem0) / 1e9,
                                              "finite": bool(torch.isfinite(v0.grad).all().item())},
                  "footprint_GB": {"note": "torch-allocated device memory of this workload (state, metric, "
                                           "workspaces, checkpoints, step records); the library's tables are "
                                           "not included",
                                   "buffers": (base4 - mem0) / 1e9, "forward_peak": (fwd_peak - mem0) / 1e9,
                                   "reverse_peak": (adj_peak - mem0) / 1e9}}
        s4.close()
        del st4, u4, v0, uT4, seed, ustart
        torch.cuda.empty_cache()

    if args.copy_calib:
        # plain copy of known size for the counter scale factors: reads and
        # writes COPY_MIB MiB once per launch, after a fill of another buffer
        # of that size has evicted the source from the caches
        x = torch.ones(COPY_MIB * 2 ** 18, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.fill_(0.0)
            torch.cuda.synchronize()
            y.copy_(x)
            torch.cuda.synchronize()
        del x, y

    out = {
        "metric": "grid-pt RK-stages/s fwd & adjoint, batched vs per-patch, % HBM peak",
        "value": value,
        "unit": "grid-pt RK-stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"uneven-{ps.npatch}-patches-48to512 (seed 2), Mach 3 +-1% density, "
                               "network classifier + smooth AV every step, SSPRK(5,4), batched hipGraph step",
                   "layout": args.layout,
                   "points": npts, "patches": ps.npatch},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": PASS_KERNEL[dom],
                     "bytes_per_point": pass_gb[dom] * 1e9 / npts, "ms": passes[dom],
                     "note": "achieved = algorithmic bytes of the kernel averaged over the five stages / "
                             "its mean launch time (HIP events on the library stream)"},
        "stage_ms": {"batched": ms_batched / 5, "per_patch": None if ms_pp is None else ms_pp / 5,
                     "batched_over_per_patch": None if ms_pp is None else ms_pp / ms_batched,
                     "by_schedule": sched_ms, "persistent_wait_errors": stage_errors},
        "pass_ms": passes,
        "adjoint": adjoint,
        "filter": filt,
        "paper_subpatches": paper,
        "strict_continuation": strict,
        "interpolated_pair": interp_rec,
        "annulus_shells": shells,
        "schedule": {k: v for k, v in tuning.items() if k != "table"},
        "other_workloads_schedules": aux_tuning,
        "stage_bytes_per_point": stage_bytes,
        "stage_effective_GBs": stage_bytes * npts / (ms_batched / 5 / 1e3) / 1e9,
        "wall_s": wall,
        "finite": finite,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
