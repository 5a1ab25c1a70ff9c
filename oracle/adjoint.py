"""Discrete adjoint (reverse mode) of the FP64 FC-SDNN time stepping.

Test infrastructure only (see oracle/__init__.py).

Differentiates the discrete map the oracle's solver.Run applies, with the
non-differentiable decisions of a recorded forward run frozen: the network
classes tau, the 7x7 maximiser positions, the step sizes dt and the boundary
masks (reading: the derivative of the fixed branch; the classifier
contributes nothing through tau).  Building blocks:

  * the right-hand side VJP (euler.full_rhs_vjp) at every glued stage input;
  * the viscosity VJP (av.viscosity_vjp) at the glued step input;
  * the spectral filter's VJP (filter.filter_state_vjp) and the glue after
    it, when the step filters;
  * the transpose of the glue: Dirichlet overwrite (cotangent zeroed, the
    free-stream's Mach derivative collected), then the shell and sector
    fringe copies in reverse order (receiver cotangent moved to its donor);
  * the reverse of the Shu-Osher stages of rk.ssprk_step.
"""
from __future__ import annotations

import numpy as np

from oracle import av, euler, interp, rk, solver, wall
from oracle import filter as spectral_filter


def glue_vjp(eb, ps, mach, gamma=1.4, e_glued=None):
    """In-place transpose of solver.glue on a cotangent [4, plane]; returns
    the derivative with respect to the free-stream Mach number.  e_glued:
    the glued state (needed with walls, whose condition is not linear)."""
    dM = 0.0
    if getattr(ps, "wall", None) is not None and ps.wall.any():
        if e_glued is None:
            raise ValueError("the wall condition's reverse mode needs the glued state")
        wall.apply_vjp(eb, e_glued, ps, gamma)
    if ps.nsec == 0:
        if ps.geom is not None:
            if getattr(ps, "_interp_table", None) is None:
                ps._interp_table = interp.build(ps)
            interp.interpolate_adj(eb, ps, ps._interp_table)
        return dM
    if ps.dirichlet is not None:
        m = ps.dirichlet.astype(bool)
        dfs = np.array([0.0, 1.4, 0.0, 1.4 * mach])
        dM += float(np.sum(eb[:, m] * dfs[:, None]))
        eb[:, m] = 0.0
    NF, OVL = solver.NF, solver.OVL
    S, K = ps.nsec, ps.nshell
    for k in range(K):
        for s in range(S):
            p = ps.patch_of_shell(s, k)
            b = int(ps.n2[p])
            dst = ps.view(eb, p)
            if k > 0:
                src = ps.view(eb, ps.patch_of_shell(s, k - 1))
                src[:, b - OVL:b - OVL + NF, :] += dst[:, :NF, :]
                dst[:, :NF, :] = 0.0
            if k < K - 1:
                src = ps.view(eb, ps.patch_of_shell(s, k + 1))
                src[:, OVL - NF:OVL, :] += dst[:, b - NF:, :]
                dst[:, b - NF:, :] = 0.0
    if S > 1:
        for k in range(K):
            for s in range(S):
                p = ps.patch_of_shell(s, k)
                a = int(ps.n1[p])
                dst = ps.view(eb, p)
                left = ps.view(eb, ps.patch_of_shell((s - 1) % S, k))
                right = ps.view(eb, ps.patch_of_shell((s + 1) % S, k))
                left[:, :, a - OVL:a - OVL + NF] += dst[:, :, :NF]
                dst[:, :, :NF] = 0.0
                right[:, :, OVL - NF:OVL] += dst[:, :, a - NF:]
                dst[:, :, a - NF:] = 0.0
    return dM


def step_vjp(run, entry, ub_next):
    """Cotangent of the step input given the cotangent of its output.
    entry: a record written by solver.Run.step(record=True).  Returns
    (ub_in, dMach)."""
    ps, g, mach = run.ps, run.gamma, run.mach
    st = entry["stages"]            # glued stage inputs u^(0..4)
    mu, dt = entry["mu"], entry["dt"]
    visc = run.cfg.mu_const is None
    n = rk.NSTAGE
    ub = [np.zeros_like(st[0]) for _ in range(n)]
    rb = [np.zeros_like(st[0]) for _ in range(n)]
    mub = np.zeros(ps.plane)
    dM = 0.0

    def distribute(i, ubar):
        # u^(i) = sum_k alpha[i-1][k] u^(k) + beta[i-1][k] dt L(u^(k))
        for k in range(i):
            a, b = rk.ALPHA[i - 1][k], rk.BETA[i - 1][k]
            if a:
                ub[k] += a * ubar
            if b:
                rb[k] += b * dt * ubar

    distribute(n, np.array(ub_next, np.float64))
    for i in range(n - 1, -1, -1):
        eb, mb = euler.full_rhs_vjp(st[i], ps.metric, mu, ps, g, rb[i])
        ub[i] += eb
        mub += mb
        if i >= 1:
            dM += glue_vjp(ub[i], ps, mach, g, st[i])
            distribute(i, ub[i])
    u_visc = st[0]
    if entry.get("filt") is not None:
        alpha, p = entry["filt"]
        dM += glue_vjp(ub[0], ps, mach, g, st[0])
        ub[0] = spectral_filter.filter_state_vjp(entry["pre"], ub[0], ps, alpha, p, g)
        u_visc = entry["pre"]
    if visc:
        ub[0] += av.viscosity_vjp(u_visc, entry["tau"], entry["arg"], ps, g, mub)
    dM += glue_vjp(ub[0], ps, mach, g, u_visc)
    return ub[0], dM


def forward(cfg, steps, u0=None, mach=None, replay=None, record=True, filt=None):
    """Run `steps` steps in FP64 from u0 (default cfg.u0); replay: list of
    recorded entries whose dt, tau, arg are reused; filt = (alpha, p): the
    spectral filter in every step."""
    run = solver.Run(cfg)
    if u0 is not None:
        run.u = np.array(u0, np.float64)
    if mach is not None:
        run.mach = mach
    for k in range(steps):
        if replay is not None:
            e = replay[k]
            run.step(dt=e["dt"], tau=e["tau"], arg=e["arg"], record=record, filt=filt)
        else:
            run.step(record=record, filt=filt)
    return run


def outer_density_loss(ps, u):
    """L = (sum over patches of rho^2 on the outermost grid row)^(1/2) and dL/du."""
    tot = 0.0
    for p in range(ps.npatch):
        tot += float(np.sum(ps.view(u[0], p)[-1, :] ** 2))
    L = np.sqrt(tot)
    gb = np.zeros_like(u)
    for p in range(ps.npatch):
        ps.view(gb[0], p)[-1, :] = ps.view(u[0], p)[-1, :] / L
    return L, gb


def initial_state(ps, mach, amp, pert, gamma=1.4):
    """IC of the annulus workloads as a function of (M, a_k) and its
    Jacobian columns: rho = 1.4 (1 + sum a_k phi_k), m = rho M, n = 0,
    E = 1/(gamma-1) + rho M^2 / 2."""
    phi = pert.modes(ps.xy)                   # [K, plane]
    rho = 1.4 * (1 + amp @ phi)
    e = np.stack([rho, rho * mach, 0 * rho, 1 / (gamma - 1) + 0.5 * rho * mach * mach])
    de_dM = np.stack([0 * rho, rho, 0 * rho, rho * mach])
    drho = 1.4 * phi                          # [K, plane]
    de_da = np.stack([drho, drho * mach, 0 * drho, 0.5 * drho * mach * mach], axis=1)   # [K, 4, plane]
    return e, de_dM, de_da


def gradient(cfg, steps, replay=None, filt=None):
    """Loss and its gradient with respect to (M, a_1..a_K) through `steps`
    steps, decisions frozen at the base run (or at `replay`, recorded dt /
    tau / arg per step).  Returns (L, g, base_run)."""
    ps = cfg.ps
    e0, de_dM, de_da = initial_state(ps, cfg.mach, cfg.pert.amp, cfg.pert)
    run = forward(cfg, steps, u0=e0, mach=cfg.mach, replay=replay, filt=filt)
    L, ub = outer_density_loss(ps, run.u)
    dM_bc = 0.0
    for k in range(steps - 1, -1, -1):
        ub, dM = step_vjp(run, run.log[k], ub)
        dM_bc += dM
    gM = float(np.sum(ub * de_dM)) + dM_bc
    ga = np.einsum("kfp,fp->k", de_da, ub)
    return L, np.concatenate([[gM], ga]), run


def loss_at(cfg, steps, mach, amp, replay, filt=None):
    e0, _, _ = initial_state(cfg.ps, mach, amp, cfg.pert)
    run = forward(cfg, steps, u0=e0, mach=mach, replay=replay, record=False, filt=filt)
    return outer_density_loss(cfg.ps, run.u)[0]
