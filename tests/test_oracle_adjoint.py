"""Pins of the oracle's discrete adjoint: transpose identities of the glue
and a step, and central finite differences of the outer-density loss with
respect to the Mach number and the perturbation amplitudes (decisions
frozen at the base run, FP64, h = 1e-4 as in the differentiation
workload)."""
import numpy as np
import pytest

import synth
from oracle import adjoint, solver


def small_annulus_cfg(n=40, nshell=1):
    cfg = synth.config(3, n=n)
    if nshell > 1:
        ps = synth.annulus(16, nshell, n, n)
        e = synth.mach_state(ps, cfg.mach, cfg.pert)
        cfg = synth.Config(cfg.name, ps, synth._f32(e, ps), cfg.ref, mach=cfg.mach, pert=cfg.pert,
                           mlp=cfg.mlp, steps=cfg.steps)
    return cfg


def test_glue_transpose():
    ps = synth.annulus(4, 3, 40, 32)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4, ps.plane))
    y = rng.standard_normal((4, ps.plane))
    gx = x.copy()
    solver.glue(gx, ps, 0.0)          # Mach 0: the Dirichlet value has no Mach part in rho u
    fs = synth.freestream(0.0)
    m = ps.dirichlet.astype(bool)
    lin = gx.copy()
    lin[:, m] -= fs[:, None]          # glue minus its constant part is linear
    yt = y.copy()
    adjoint.glue_vjp(yt, ps, 0.0)
    assert np.isclose(np.sum(lin * y), np.sum(x * yt), rtol=1e-13)


@pytest.mark.slow
def test_adjoint_matches_central_differences():
    cfg = small_annulus_cfg(40)
    steps = 2
    L, g, run = adjoint.gradient(cfg, steps)
    replay = run.log
    h = 1e-4
    # Mach
    lp = adjoint.loss_at(cfg, steps, cfg.mach + h, cfg.pert.amp, replay)
    lm = adjoint.loss_at(cfg, steps, cfg.mach - h, cfg.pert.amp, replay)
    fdM = (lp - lm) / (2 * h)
    # rounding floor of a central difference of an O(L) loss
    floor = 20 * np.finfo(float).eps * L / h
    assert abs(fdM - g[0]) <= 1e-6 * abs(fdM) + floor
    # three perturbation amplitudes
    for k in (0, 5, 11):
        a = cfg.pert.amp.copy()
        a[k] += h
        lp = adjoint.loss_at(cfg, steps, cfg.mach, a, replay)
        a[k] -= 2 * h
        lm = adjoint.loss_at(cfg, steps, cfg.mach, a, replay)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[1 + k]) <= 1e-6 * abs(fd) + floor, (k, fd, g[1 + k])


@pytest.mark.slow
def test_adjoint_with_filter_matches_central_differences():
    """The step with the spectral filter (alpha 10, p 14) after the
    viscosity: the discrete adjoint against central differences."""
    cfg = small_annulus_cfg(40)
    steps = 2
    filt = (10.0, 14)
    L, g, run = adjoint.gradient(cfg, steps, filt=filt)
    replay = run.log
    h = 1e-4
    floor = 20 * np.finfo(float).eps * L / h
    lp = adjoint.loss_at(cfg, steps, cfg.mach + h, cfg.pert.amp, replay, filt=filt)
    lm = adjoint.loss_at(cfg, steps, cfg.mach - h, cfg.pert.amp, replay, filt=filt)
    fdM = (lp - lm) / (2 * h)
    assert abs(fdM - g[0]) <= 1e-6 * abs(fdM) + floor
    for k in (2, 9):
        a = cfg.pert.amp.copy()
        a[k] += h
        lp = adjoint.loss_at(cfg, steps, cfg.mach, a, replay, filt=filt)
        a[k] -= 2 * h
        lm = adjoint.loss_at(cfg, steps, cfg.mach, a, replay, filt=filt)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[1 + k]) <= 1e-6 * abs(fd) + floor, (k, fd, g[1 + k])
    # the filter changes the gradient (it is in the differentiated map)
    L0, g0, _ = adjoint.gradient(cfg, steps, replay=replay)
    assert np.abs(g - g0).max() > 1e-6 * np.abs(g0).max()


@pytest.mark.slow
def test_frozen_decisions_against_the_free_rollout():
    """How far the derivative of the frozen branch (decisions -- step sizes,
    classes, maximisers -- fixed at the base run, what the hand-written
    adjoint computes) is from a central difference of the free rollout,
    whose step sizes and decisions follow the parameter, on the annulus at
    40 x 40 over two steps.  The perturbation amplitudes change the rollout
    mostly through the state: within 3 % (a class or maximiser that flips
    inside +-h makes the free difference depend on h).  The inflow Mach
    number also sets the step size through the wave speeds of the CFL
    condition, which the frozen branch leaves out: there the free
    derivative is about a third of the frozen one, and smooth (the same at
    h = 1e-4 and 1e-5)."""
    cfg = small_annulus_cfg(40)
    steps = 2
    L, g, run = adjoint.gradient(cfg, steps)
    free = {}
    for h in (1e-4, 1e-5):
        lp = adjoint.loss_at(cfg, steps, cfg.mach + h, cfg.pert.amp, None)
        lm = adjoint.loss_at(cfg, steps, cfg.mach - h, cfg.pert.amp, None)
        free[h] = (lp - lm) / (2 * h)
    print("d/dM frozen", g[0], "free", free)
    assert abs(free[1e-4] - free[1e-5]) <= 1e-6 * abs(free[1e-4])
    assert 0.2 < free[1e-4] / g[0] < 0.5
    for k in (0, 5):
        h = 1e-4
        a = cfg.pert.amp.copy()
        a[k] += h
        lp = adjoint.loss_at(cfg, steps, cfg.mach, a, None)
        a[k] -= 2 * h
        lm = adjoint.loss_at(cfg, steps, cfg.mach, a, None)
        fd = (lp - lm) / (2 * h)
        print("d/da", k, "frozen", g[1 + k], "free", fd)
        assert abs(fd - g[1 + k]) <= 3e-2 * abs(g[1 + k])
