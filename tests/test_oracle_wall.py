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


def _square_with_walls(n, flags, d=5):
    import dataclasses
    ps = synth.unit_square(n, d=d)
    return dataclasses.replace(ps, wall=np.array([flags], np.uint8))


@pytest.mark.parametrize("flags", [(1, 0, 1, 0), (0, 1, 0, 1), (1, 1, 1, 1), (0, 1, 1, 0)])
def test_corner_walls_continue_polynomial_temperatures_exactly(flags):
    """Walls meeting at corners: with theta a polynomial of degree < d in
    each index with zero slope at every wall, the wall condition reproduces
    theta exactly at every wall point, corners included (the corner takes
    the tensor product of the two one-sided Neumann values), zeroes the
    momenta there and leaves the interior alone."""
    gamma = 1.4
    n = 24
    ps = _square_with_walls(n, flags)
    j, i = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    # zero slope at i = 0 (and at i = n-1), likewise in j, through (i - a)^2 (i - b)^2 terms of degree 4 < d
    s1 = (i * (n - 1 - i)) ** 2 / (n - 1) ** 4
    s2 = (j * (n - 1 - j)) ** 2 / (n - 1) ** 4
    th = 2.0 + 0.7 * s1 + 0.4 * s2 + 0.3 * s1 * s2
    rho = 1.0 + 0.1 * np.cos(0.3 * i + 0.2 * j)
    u, v = 0.3 + 0.01 * i, -0.2 + 0.01 * j
    e = np.zeros((4, ps.plane))
    view = ps.view(e, 0)
    view[0], view[1], view[2] = rho, rho * u, rho * v
    view[3] = rho * th / (gamma - 1) + 0.5 * rho * (u * u + v * v)
    before = e.copy()
    wall.apply(e, ps, gamma)
    after = ps.view(e, 0)
    on = np.zeros((n, n), bool)
    if flags[0]:
        on[:, 0] = True
    if flags[1]:
        on[:, -1] = True
    if flags[2]:
        on[0, :] = True
    if flags[3]:
        on[-1, :] = True
    assert np.all(after[1][on] == 0) and np.all(after[2][on] == 0)
    assert np.array_equal(after[0], ps.view(before, 0)[0])
    th_after = wall.theta_of(after, gamma)
    assert np.abs(th_after[on] - th[on]).max() <= 1e-11
    assert np.array_equal(after[:, ~on], ps.view(before, 0)[:, ~on])


def test_corner_wall_transpose_matches_central_differences():
    """apply_vjp with two walls meeting at a corner: <e_bar, de> against the
    central difference of <apply(e), y> along de (the condition is smooth
    in the state away from rho = 0)."""
    gamma = 1.4
    n = 20
    ps = _square_with_walls(n, (1, 0, 1, 1))
    rng = np.random.default_rng(3)
    e = np.zeros((4, ps.plane))
    v = ps.view(e, 0)
    v[0] = 1 + 0.2 * rng.random((n, n))
    v[1] = 0.3 * rng.standard_normal((n, n))
    v[2] = 0.3 * rng.standard_normal((n, n))
    v[3] = 3 + rng.random((n, n))
    y = rng.standard_normal((4, ps.plane))
    de = rng.standard_normal((4, ps.plane))
    glued = wall.apply(e.copy(), ps, gamma)
    eb = y.copy()
    wall.apply_vjp(eb, glued, ps, gamma)
    h = 1e-6
    fd = (np.sum(wall.apply(e + h * de, ps, gamma) * y) - np.sum(wall.apply(e - h * de, ps, gamma) * y)) / (2 * h)
    assert abs(fd - np.sum(eb * de)) <= 1e-7 * abs(fd)


def test_energy_derivatives_by_the_product_rule_on_wall_patches():
    """On a patch with a wall side the energy's derivatives are formed by
    the sum and product rules (Remark adiabatic, eqs. p_T, perfect_gas_T)
    from the FC derivatives of rho, rho u, rho v and theta: with those four
    polynomials of degree < d along every line, each derivative is exact to
    FC precision and so is the energy's, while the FC derivative of E itself
    (rho theta of degree 6) is not; a patch without walls keeps E's own."""
    from oracle import euler
    gamma = 1.4
    n = 40
    ps = _square_with_walls(n, (0, 0, 1, 0))
    x, y = ps.xy
    rho = 1.0 + 0.2 * x + 0.1 * y * y - 0.05 * x ** 3
    th = 2.0 + 0.3 * y ** 3 - 0.2 * x * y + 0.1 * x ** 2
    m = 0.3 + 0.1 * x - 0.2 * y
    nn = -0.1 + 0.2 * x * y
    E = rho * th / (gamma - 1) + 0.5 * (m * m + nn * nn) / rho
    e = np.stack([rho, m, nn, E])
    drho = (0.2 - 0.15 * x ** 2, 0.2 * y)
    dth = (-0.2 * y + 0.2 * x, 0.9 * y ** 2 - 0.2 * x)
    dm = (0.1 * np.ones_like(x), -0.2 * np.ones_like(x))
    dn = (0.2 * y, 0.2 * x)
    d1, d2 = euler.derivatives(e, ps, gamma)
    for k, dd in enumerate((d1, d2)):
        want = (drho[k] * th + rho * dth[k]) / (gamma - 1) + (m * dm[k] + nn * dn[k]) / rho \
            - 0.5 * (m * m + nn * nn) * drho[k] / rho ** 2
        got = ps.view(dd, 0)[3]
        w = ps.view(want, 0)
        assert np.abs(got - w).max() <= 1e-8 * np.abs(w).max(), k
        plain = ps.view(euler.fcgram.diff_plane(e, ps, k + 1), 0)[3]
        assert np.abs(plain - w).max() >= 1e-7 * np.abs(w).max()
    import dataclasses
    free = dataclasses.replace(ps, wall=np.zeros((1, 4), np.uint8))
    f1, _ = euler.derivatives(e, free, gamma)
    assert np.array_equal(f1, euler.fcgram.diff_plane(e, free, 1))


def test_product_rule_derivatives_vjp_matches_central_differences():
    from oracle import euler
    gamma = 1.4
    ps = synth.annulus(4, 1, 40, 36)
    ps.wall = np.zeros((ps.npatch, 4), np.uint8)
    ps.wall[:, 2] = 1
    rng = np.random.default_rng(5)
    e = np.zeros((4, ps.plane))
    for p in range(ps.npatch):
        v = ps.view(e, p)
        v[0] = 1 + 0.1 * rng.random(v[0].shape)
        v[1] = 0.3 * rng.standard_normal(v[1].shape)
        v[2] = 0.3 * rng.standard_normal(v[2].shape)
        v[3] = 3 + rng.random(v[3].shape)
    g1, g2 = rng.standard_normal((4, ps.plane)), rng.standard_normal((4, ps.plane))
    de = rng.standard_normal((4, ps.plane))
    keep = np.zeros(ps.plane, bool)
    keep[euler.points(ps)] = True
    de[:, ~keep] = 0
    eb = euler.derivatives_vjp(e, ps, gamma, g1, g2)
    # the map is rational in the state: central differences at h = 1e-4 have
    # a truncation error ~h^2 and little FP64 cancellation on these noisy fields
    h = 1e-4
    f = lambda ee: sum(np.sum(d * g) for d, g in zip(euler.derivatives(ee, ps, gamma), (g1, g2)))
    fd = (f(e + h * de) - f(e - h * de)) / (2 * h)
    assert abs(fd - np.sum(eb * de)) <= 1e-6 * abs(fd)
