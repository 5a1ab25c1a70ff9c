"""Multi-patch FC-SDNN time stepping, FP64 (paper Algorithm 1, Secs. 3.4, 4).

Test infrastructure only (see oracle/__init__.py).

Per time step (Algorithm 1): evaluate the viscosity mu (network classifier,
preliminary viscosity, smoothing-blending; or a given constant), optionally
apply the spectral filter of Sec. 4.3.1 to the state (then glue again),
evaluate the step size dt (eq. CFL), then advance the five SSPRK stages,
enforcing boundary conditions and patch communication on every stage input
(Sec. 4.2).

Readings for the index-aligned annulus used by the synthetic workloads:
  * communication = copy of the n_f = 5 fringe lines from the neighbour's
    point with the same global index (Sec. 3.4.1 degenerates to a copy when
    grids coincide); first across sectors (all rows), then across shells (all
    columns, after the sector copy);
  * Dirichlet overwrite with the free stream (1.4, M, 0, 1) on the outer
    circle where x < 0, after the communication; the inner circle is left
    free (no wall model on this path);
  * the state is glued once at the start of each step (before mu and dt) and
    on every later stage input.

Patch sets that carry patch maps (``geom``) and are not index-aligned take
their communication from the inter-patch interpolation of Sec. 3.4.1
(oracle.interp) instead.  Sides flagged as walls get the no-slip adiabatic
condition of oracle.wall after the rest of the glue.
"""
from __future__ import annotations

import numpy as np

from oracle import av, euler, filter as spectral_filter, interp, rk, wall

NF = 5
OVL = 19


def glue(e, ps, mach, gamma=1.4):
    """In-place fringe copy (or interpolation) and Dirichlet overwrite on a
    [4, plane] state."""
    if ps.nsec == 0:
        if ps.geom is not None:
            if getattr(ps, "_interp_table", None) is None:
                ps._interp_table = interp.build(ps)
            interp.interpolate(e, ps, ps._interp_table)
        return wall.apply(e, ps, gamma)
    S, K = ps.nsec, ps.nshell
    for k in range(K):
        for s in range(S):
            p = ps.patch_of_shell(s, k)
            a = int(ps.n1[p])
            if S > 1:
                left = ps.patch_of_shell((s - 1) % S, k)
                right = ps.patch_of_shell((s + 1) % S, k)
                dst = ps.view(e, p)
                # receivers i < NF take the left neighbour's column i + (a - OVL)
                dst[:, :, :NF] = ps.view(e, left)[:, :, a - OVL:a - OVL + NF]
                dst[:, :, a - NF:] = ps.view(e, right)[:, :, OVL - NF:OVL]
    # the sector pass reads only donor columns, which are never receivers
    for k in range(K):
        for s in range(S):
            p = ps.patch_of_shell(s, k)
            b = int(ps.n2[p])
            dst = ps.view(e, p)
            if k > 0:
                dst[:, :NF, :] = ps.view(e, ps.patch_of_shell(s, k - 1))[:, b - OVL:b - OVL + NF, :]
            if k < K - 1:
                dst[:, b - NF:, :] = ps.view(e, ps.patch_of_shell(s, k + 1))[:, OVL - NF:OVL, :]
    if ps.dirichlet is not None:
        fs = np.array([1.4, 1.4 * mach, 0.0, 1.0 / (gamma - 1) + 0.5 * 1.4 * mach * mach])
        m = ps.dirichlet.astype(bool)
        e[:, m] = fs[:, None]
    wall.apply(e, ps, gamma)        # no-slip adiabatic walls (oracle.wall), last
    return e


class Run:
    """A configuration advanced in FP64.  ``replay`` fixes the per-step
    decisions (tau, 7x7 argmax, dt) to recorded values."""

    def __init__(self, cfg, gamma=1.4):
        self.cfg = cfg
        self.ps = cfg.ps
        self.gamma = gamma
        self.u = np.array(cfg.u0, np.float64)
        self.mach = cfg.mach
        self.log = []

    def viscosity(self, e):
        ps = self.ps
        if self.cfg.mu_const is not None:
            mu = np.zeros(ps.plane)
            for p in range(ps.npatch):
                ps.view(mu, p)[...] = self.cfg.mu_const
            return mu, None, None
        return av.viscosity(e, ps, self.cfg.mlp, self.gamma)

    def step(self, dt=None, tau=None, arg=None, record=False, filt=None, progress=None):
        """One step; dt, tau, arg replay recorded decisions.  record keeps
        the glued stage inputs for the discrete adjoint.  filt = (alpha, p)
        applies the spectral filter after the viscosity.  progress(stage),
        if given, is called as each stage's right-hand side is done."""
        ps, g = self.ps, self.gamma
        e = self.u
        glue(e, ps, self.mach, g)
        if self.cfg.mu_const is None and (tau is not None or arg is not None):
            mu, tau_used, arg = av.viscosity(e, ps, self.cfg.mlp, g, tau=tau, arg=arg)
        else:
            mu, tau_used, arg = self.viscosity(e)
        pre = None
        if filt is not None:
            pre = np.array(e)
            e = spectral_filter.filter_state(e, ps, filt[0], filt[1], g)
            glue(e, ps, self.mach, g)
        if dt is None:
            dt = rk.cfl_dt(e, mu, ps, self.cfg.cfl, g)
        def L(u, s):
            r = euler.full_rhs(u, ps.metric, mu, ps, g)
            if progress is not None:
                progress(s)
            return r
        new, stages, rhs = rk.ssprk_step(e, dt, L, glue=lambda u, s: glue(u, ps, self.mach, g))
        entry = dict(dt=dt, tau=tau_used, arg=arg, mu=mu, filt=filt, pre=pre)
        if record:
            entry["stages"] = [np.array(x) for x in stages[:-1]]
        self.log.append(entry)
        self.u = new
        return new
