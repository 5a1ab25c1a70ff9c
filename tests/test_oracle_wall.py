"""Pins of the oracle's wall condition (paper Sec. 2.2 on Neumann data,
Remarks adiabatic_th, adiabatic): the Neumann boundary value is exact for
polynomials of degree < d given their derivative at the wall, matches the
closed forms for d = 2 (F_1 - g) and d = 3 ((4 F_1 - F_2 - 2 g) / 3); the
wall condition zeroes the momenta, leaves rho, keeps p / rho at the wall
equal to its Neumann value (an interior temperature that is a polynomial of
degree < d in the normal index with zero slope at the wall is continued
exactly), and touches nothing off the wall line."""
import numpy as np
import pytest

import synth
from oracle import wall


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_neumann_value_exact_on_polynomials(d):
    rng = np.random.default_rng(d)
    c = wall.neumann_weights(d)
    for _ in range(5):
        a = rng.standard_normal(d)
        p = lambda t: sum(a[m] * t ** m for m in range(d))
        g = a[1] if d > 1 else 0.0
        val = c[0] * g + sum(c[k] * p(float(k)) for k in range(1, d))
        assert abs(val - a[0]) <= 1e-12 * np.abs(a).sum()


def test_neumann_closed_forms():
    c2 = wall.neumann_weights(2)
    assert np.allclose(c2, [-1.0, 1.0], atol=1e-15)
    c3 = wall.neumann_weights(3)
    assert np.allclose(c3, [-2.0 / 3, 4.0 / 3, -1.0 / 3], atol=1e-15)


def test_wall_condition_on_the_inner_circle():
    gamma = 1.4
    ps = synth.annulus(16, 1, 48, 40)
    ps.wall = np.zeros((ps.npatch, 4), np.uint8)
    ps.wall[:, 2] = 1                       # r = 0.5, the q2- side of every sector
    rng = np.random.default_rng(0)
    e = np.zeros((4, ps.plane))
    for p in range(ps.npatch):
        v = ps.view(e, p)
        n2, n1 = v.shape[1:]
        j = np.arange(n2)[:, None] * np.ones((1, n1))
        rho = 1.2 + 0.1 * rng.standard_normal((n2, n1)) ** 2
        theta = 0.9 + 0.01 * j ** 2 - 0.001 * j ** 3     # zero slope at j = 0, degree < 5
        u, vv = rng.standard_normal((2, n2, n1)) * 0.1
        v[0] = rho
        v[1] = rho * u
        v[2] = rho * vv
        v[3] = rho * theta / (gamma - 1) + 0.5 * rho * (u * u + vv * vv)
    before = e.copy()
    wall.apply(e, ps, gamma)
    for p in range(ps.npatch):
        a, b = ps.view(e, p), ps.view(before, p)
        assert np.array_equal(a[:, 1:], b[:, 1:])            # off the wall line
        assert np.array_equal(a[0, 0], b[0, 0])              # rho evolves freely
        assert np.all(a[1, 0] == 0) and np.all(a[2, 0] == 0)  # no slip
        th_w = a[3, 0] * (gamma - 1) / a[0, 0]
        assert np.abs(th_w - 0.9).max() <= 1e-12          # the exact zero-slope value


def test_wall_transpose_and_step_reverse_mode():
    """The wall condition's VJP against central differences of the glue,
    and one network step with the cylinder wall against central differences
    of the step map (decisions frozen)."""
    from oracle import adjoint, solver
    gamma = 1.4
    cfg = synth.with_cylinder_wall(synth.config(1, n=40))
    ps = cfg.ps
    rng = np.random.default_rng(1)
    e = cfg.u0.astype(np.float64) * (1 + 0.01 * rng.standard_normal((4, ps.plane)))
    w = rng.standard_normal((4, ps.plane))

    def glued(x):
        y = x.copy()
        solver.glue(y, ps, cfg.mach, gamma)
        return y

    g = glued(e)
    wb = w.copy()
    adjoint.glue_vjp(wb, ps, cfg.mach, gamma, g)
    h = 1e-6
    for _ in range(2):
        v = rng.standard_normal(e.shape) * np.abs(e).max(axis=1, keepdims=True)
        fd = np.sum((glued(e + h * v) - glued(e - h * v)) * w) / (2 * h)
        assert abs(fd - np.sum(wb * v)) <= 1e-6 * abs(fd)
    run = solver.Run(cfg)
    u0 = run.u.copy()
    run.step(record=True)
    entry = run.log[-1]

    def F(u):
        r = solver.Run(cfg)
        r.u = u.copy()
        r.step(dt=entry["dt"], tau=entry["tau"], arg=entry["arg"])
        return r.u

    ub, _ = adjoint.step_vjp(run, entry, w)
    for _ in range(2):
        v = rng.standard_normal(u0.shape) * np.abs(u0).max(axis=1, keepdims=True)
        fd = np.sum((F(u0 + h * v) - F(u0 - h * v)) * w) / (2 * h)
        an = np.sum(ub * v)
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
