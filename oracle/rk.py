"""SSPRK(5,4) time stepping and the adaptive step size, FP64 (paper Sec. 4.1).

Test infrastructure only (see oracle/__init__.py).

The paper advances the semi-discrete system de/dt = L[e] with the
fourth-order strong-stability-preserving Runge-Kutta scheme of its ref.
(Gottlieb 2005) with five stages nu = 1..5 (Sec. 4.2), but prints no
coefficients.  Reading: the five-stage, fourth-order SSP scheme of Spiteri
and Ruuth in Shu-Osher form, with the published 15-digit coefficients

    u^(i) = sum_{k<i} ( alpha[i][k] u^(k) + dt beta[i][k] L(u^(k)) ),  i = 1..5.

The coefficients are pinned by the classical order conditions (tests).

Step size, eq. "CFL":
    dt = (1/pi) min_patches CFL / ( max S/h~ + max mu/h~^2 ),
S = |u| + |v| + a the maximum-wave-speed bound (Sec. 5.1) and h~ the
patch's minimum grid spacing.
"""
from __future__ import annotations

import numpy as np

from oracle import euler

ALPHA = [
    [1.0],
    [0.444370493651235, 0.555629506348765],
    [0.620101851488403, 0.0, 0.379898148511597],
    [0.178079954393132, 0.0, 0.0, 0.821920045606868],
    [0.0, 0.0, 0.517231671970585, 0.096059710526147, 0.386708617503269],
]
BETA = [
    [0.391752226571890],
    [0.0, 0.368410593050371],
    [0.0, 0.0, 0.251891774271694],
    [0.0, 0.0, 0.0, 0.544974750228521],
    [0.0, 0.0, 0.0, 0.063692468666290, 0.226007483236906],
]
NSTAGE = 5


def butcher():
    """Butcher tableau (A, b, c) equivalent to the Shu-Osher form: writing
    u^(i) = u0 + dt sum_j A'[i][j] L(u^(j)) recursively."""
    s = NSTAGE
    # coefficient of L(u^(j)) in u^(i), i = 0..s (u^(0) = u0)
    K = np.zeros((s + 1, s))
    for i in range(1, s + 1):
        for k in range(i):
            K[i] += ALPHA[i - 1][k] * K[k]
            K[i, k] += BETA[i - 1][k]
    return K[:s], K[s], K[:s].sum(axis=1)


def ssprk_step(u0, dt, L, glue=None):
    """One step; L(u, stage) returns the right-hand side.  glue(u, stage),
    if given, is applied in place to every stage input before L is evaluated
    (boundary overwrite and communication, Sec. 4.2)."""
    stages = [np.array(u0, np.result_type(u0, np.float64), copy=True)]
    rhs = []
    for i in range(1, NSTAGE + 1):
        ui = stages[i - 1]
        if glue is not None and i > 1:
            glue(ui, i - 1)
        rhs.append(L(ui, i - 1))
        new = np.zeros_like(ui)
        for k in range(i):
            a, b = ALPHA[i - 1][k], BETA[i - 1][k]
            if a:
                new += a * stages[k]
            if b:
                new += b * dt * rhs[k]
        stages.append(new)
    return stages[-1], stages, rhs


def wave_speed(e, gamma):
    """S = |u| + |v| + a (Sec. 5.1, MWSB)."""
    rho, u, v, p = euler.primitives(np.asarray(e, np.float64), gamma)
    return np.abs(u) + np.abs(v) + np.sqrt(gamma * p / rho)


def cfl_dt(e, mu, ps, cfl, gamma):
    """eq. CFL, minimum over patches."""
    best = np.inf
    for p in range(ps.npatch):
        h = ps.htilde[p]
        s = wave_speed(ps.view(np.asarray(e, np.float64), p), gamma).max() / h
        m = ps.view(np.asarray(mu, np.float64), p).max() / h ** 2 if mu is not None else 0.0
        best = min(best, cfl / (s + m))
    return best / np.pi
