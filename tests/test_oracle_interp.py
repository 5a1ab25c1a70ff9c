"""Pins of the oracle's inter-patch interpolation (paper Sec. 3.4.1, Remark
overlap_cond) against facts that do not restate its code:

* Neville's three-point recurrence reproduces every quadratic exactly
  (a + b s + c s^2 at the nodes -1, 0, 1) and is the Lagrange interpolant;
* the iterated interpolation reproduces, at every fringe point, a field that
  is a product of quadratics in the donor's own parameters (x, y on the
  Cartesian patch; theta, r on the sector) to rounding;
* for a smooth field the fringe error falls like h^3 (third order of
  quadratic interpolation): about 8x per halving of h;
* the table: every fringe point of both patches gets a donor of the other
  patch whose 3 x 3 stencil holds the point's preimage, no stencil point is
  a fringe point, and a decomposition whose overlap is too thin for that is
  refused.
"""
import numpy as np
import pytest

import synth
from oracle import interp


def test_neville_is_exact_on_quadratics():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, b, c = rng.standard_normal(3)
        f = lambda s: a + b * s + c * s * s
        s = rng.uniform(-1.5, 1.5, 7)
        got = interp.neville3(f(-1.0), f(0.0), f(1.0), s)
        assert np.abs(got - f(s)).max() <= 1e-14 * (abs(a) + abs(b) + abs(c)) * 3
    # Lagrange weights at s = 1/2: (-1/8, 3/4, 3/8)
    assert abs(interp.neville3(1.0, 0.0, 0.0, 0.5) + 0.125) < 1e-16
    assert abs(interp.neville3(0.0, 1.0, 0.0, 0.5) - 0.75) < 1e-16
    assert abs(interp.neville3(0.0, 0.0, 1.0, 0.5) - 0.375) < 1e-16


def _fill(ps, f_cart, f_polar):
    e = np.zeros((1, ps.plane))
    for p in range(ps.npatch):
        x, y = ps.view(ps.xy, p)
        ps.view(e, p)[0] = f_cart(x, y) if int(ps.geom[p, 0]) == 0 else f_polar(np.arctan2(y, x), np.hypot(x, y))
    return e


def test_quadratics_in_donor_parameters_are_reproduced():
    ps = synth.overlap_pair(48)
    table = interp.build(ps)
    fc = lambda x, y: (1 + 0.3 * x - 0.7 * x * x) * (0.5 - y + 0.2 * y * y)
    fp = lambda th, r: (0.2 + th - 0.4 * th * th) * (1.1 + 0.5 * r - 0.3 * r * r)
    # each patch holds the field its receivers' donors interpolate: a
    # receiver of the Cartesian patch reads the sector (fp), and back
    e = _fill(ps, fc, fp)
    want = e.copy()
    for (p, i, j, q, ic, jc, s, t) in table:
        x, y = ps.view(ps.xy, p)[:, j, i]
        want_val = fc(x, y) if int(ps.geom[q, 0]) == 0 else fp(np.arctan2(y, x), np.hypot(x, y))
        ps.view(want, p)[0, j, i] = want_val
    got = interp.interpolate(e.copy(), ps, table)
    assert np.abs(got - want).max() <= 1e-13


def test_smooth_field_third_order():
    f = lambda x, y: np.sin(2.1 * x + 0.7) * np.cos(1.3 * y - 0.2)
    errs = []
    for n in (48, 95, 189):
        ps = synth.overlap_pair(n)
        table = interp.build(ps)
        e = np.zeros((1, ps.plane))
        for p in range(ps.npatch):
            x, y = ps.view(ps.xy, p)
            ps.view(e, p)[0] = f(x, y)
        exact = e.copy()
        # perturb the fringe so only interpolated values can restore it
        for (p, i, j, *_r) in table:
            ps.view(e, p)[0, j, i] = 0.0
        got = interp.interpolate(e, ps, table)
        errs.append(np.abs(got - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.6), (errs, rates)


def test_table_is_a_valid_decomposition():
    ps = synth.overlap_pair(48)
    table = interp.build(ps)
    masks = [interp.receivers(ps, p) for p in range(ps.npatch)]
    assert len(table) == sum(int(m.sum()) for m in masks)
    for (p, i, j, q, ic, jc, s, t) in table:
        assert q != p and masks[p][j, i]
        assert not masks[q][jc - 1:jc + 2, ic - 1:ic + 2].any()
        assert abs(s) <= 1.0 and abs(t) <= 1.0
        x, y = ps.view(ps.xy, p)[:, j, i]
        xi, eta = interp.preimage(ps.geom[q], x, y)
        assert abs(ic + s - xi) < 1e-12 and abs(jc + t - eta) < 1e-12


# ------------------------------------------------------------ the paper's patch kinds (Sec. 3.1)

def test_stype_map_of_a_circle_is_the_polar_map():
    """An S-type band (eq. param_S) along the circle l(t) = R (cos t, sin t)
    with the normal pointing outwards is the polar patch (theta, r) =
    (t, R + s): the same points, and the Newton preimage equals the closed
    form (the textbook inverse of polar coordinates)."""
    R, a0, da, b0, db = 0.7, 0.3, 0.02, 0.05, 0.01
    gS = synth.geom_row(3, a0, da, b0, db, side=1.0, cx=(0.0, R), sy=(0.0, R))
    gP = synth.geom_row(1, a0, da, R + b0, db)
    rng = np.random.default_rng(1)
    i, j = rng.uniform(-0.5, 40.5, 40), rng.uniform(-0.5, 30.5, 40)
    xP, yP = interp.image(gP, i, j)
    xS, yS = interp.image(gS, i, j)
    assert np.abs(xS - xP).max() < 1e-14 and np.abs(yS - yP).max() < 1e-14
    xi, eta = interp.preimage(gS, xP, yP, 41, 31)
    assert np.abs(xi - i).max() < 1e-10 and np.abs(eta - j).max() < 1e-10
    xq, eq = interp.preimage(gP, xP, yP)
    assert np.abs(xi - xq).max() < 1e-10 and np.abs(eta - eq).max() < 1e-10
    # side = -1 turns the normal inwards: the band of radius R - s
    gI = synth.geom_row(3, a0, da, b0, db, side=-1.0, cx=(0.0, R), sy=(0.0, R))
    xI, yI = interp.image(gI, i, j)
    r = R - (b0 + j * db)
    assert np.abs(xI - r * np.cos(a0 + i * da)).max() < 1e-14


def test_affine_map_preimage():
    """An affine map with axis-aligned steps is the Cartesian map; a
    rotated, sheared one inverts exactly."""
    gA = synth.geom_row(2, affine=(-0.3, 0.2, 0.01, 0.0, 0.0, 0.02))
    gC = synth.geom_row(0, -0.3, 0.01, 0.2, 0.02)
    rng = np.random.default_rng(2)
    x, y = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50)
    a, b = interp.preimage(gA, x, y)
    c, d = interp.preimage(gC, x, y)
    assert np.abs(a - c).max() < 1e-12 and np.abs(b - d).max() < 1e-12
    gR = synth.geom_row(2, affine=(0.1, -0.4, 0.013, 0.004, -0.003, 0.017))
    i, j = rng.uniform(0, 60, 50), rng.uniform(0, 60, 50)
    a, b = interp.preimage(gR, *interp.image(gR, i, j))
    assert np.abs(a - i).max() < 1e-10 and np.abs(b - j).max() < 1e-10


def test_stype_trio_geometry():
    """The S-type / affine trio: the Newton preimage inverts the band's map
    on and around its grid (fractional indices), and the recipe's metric
    terms are the inverse Jacobians of the maps (central differences of the
    images, second order)."""
    ps = synth.stype_trio(48)
    rng = np.random.default_rng(3)
    g = ps.geom[0]
    i, j = rng.uniform(-0.5, 47.5, 60), rng.uniform(-0.5, 47.5, 60)
    xi, eta = interp.preimage(g, *interp.image(g, i, j), 48, 48)
    assert np.abs(xi - i).max() < 1e-9 and np.abs(eta - j).max() < 1e-9
    for p in range(3):
        gp = ps.geom[p]
        I, J = np.meshgrid(np.arange(48.0), np.arange(48.0))
        e = 1e-4
        xq1 = (np.array(interp.image(gp, I + e, J)) - np.array(interp.image(gp, I - e, J))) / (2 * e) * 47
        xq2 = (np.array(interp.image(gp, I, J + e)) - np.array(interp.image(gp, I, J - e))) / (2 * e) * 47
        det = xq1[0] * xq2[1] - xq2[0] * xq1[1]
        inv = np.array([xq2[1] / det, -xq2[0] / det, -xq1[1] / det, xq1[0] / det])
        got = ps.view(ps.metric, p)
        assert np.abs(got - inv).max() <= 1e-5 * np.abs(inv).max()
        x, y = ps.view(ps.xy, p)
        X, Y = interp.image(gp, I, J)
        assert np.abs(x - X).max() < 1e-13 and np.abs(y - Y).max() < 1e-13


def test_stype_trio_table_and_quadratics():
    """On the trio every fringe point gets a donor (S-type donors through
    the Newton preimage) whose stencil holds no fringe point, and the
    iterated interpolation reproduces, at every fringe point, a field that
    is a product of quadratics in its donor's own grid indices."""
    ps = synth.stype_trio(48)
    table = interp.build(ps)
    masks = [interp.receivers(ps, p) for p in range(ps.npatch)]
    assert len(table) == sum(int(m.sum()) for m in masks)
    kinds = set()
    for (p, i, j, q, ic, jc, s, t) in table:
        assert q != p and masks[p][j, i] and not masks[q][jc - 1:jc + 2, ic - 1:ic + 2].any()
        kinds.add(int(ps.geom[q, 0]))
    assert kinds == {2, 3}
    Q = [lambda i, j: (1 + 0.03 * i - 0.001 * i * i) * (0.5 - 0.02 * j + 0.0007 * j * j),
         lambda i, j: (0.2 + 0.05 * i - 0.0008 * i * i) * (1.1 + 0.01 * j - 0.0004 * j * j),
         lambda i, j: (0.7 - 0.04 * i + 0.0006 * i * i) * (0.3 + 0.03 * j + 0.0005 * j * j)]
    e = np.zeros((1, ps.plane))
    for p in range(3):
        J, I = np.mgrid[0:48, 0:48]
        ps.view(e, p)[0] = Q[p](I.astype(float), J.astype(float))
    want = e.copy()
    for (p, i, j, q, ic, jc, s, t) in table:
        ps.view(want, p)[0, j, i] = Q[q](ic + s, jc + t)
    got = interp.interpolate(e.copy(), ps, table)
    assert np.abs(got - want).max() <= 1e-12


def test_thin_overlap_is_refused():
    ps = synth.overlap_pair(48)
    # shrink the Cartesian patch's reach: its fringe now lies where the
    # sector's stencils would touch the sector's own fringe
    ps.geom = ps.geom.copy()
    ps.internal[0] = (0, 1, 0, 0)
    ps.internal[1] = (0, 0, 1, 0)
    x0 = ps.view(ps.xy, 0)[0]
    ps.xy[0, :x0.size] -= 0.3          # fringe of patch 0 near x = 0.3, close to r = 0.3
    with pytest.raises(ValueError):
        interp.build(ps)


# ------------------------------------------------------------ smoothing across non-aligned patches

def test_multipatch_smoothing_partition_of_unity_and_locality():
    from oracle import av
    ps = synth.overlap_pair(48)
    muh = np.zeros(ps.plane)
    for p in range(ps.npatch):
        ps.view(muh, p)[...] = 0.013
    mu = av.smooth_blend(muh, ps)
    for p in range(ps.npatch):
        assert np.abs(ps.view(mu, p) - 0.013).max() <= 1e-15
    # far from the overlap the result is the patch's own smoothing
    rng = np.random.default_rng(3)
    for p in range(ps.npatch):
        ps.view(muh, p)[...] = rng.uniform(0, 1, ps.view(muh, p).shape)
    mu = av.smooth_blend(muh, ps)
    single = synth.overlap_pair(48)
    single.geom = None
    with np.errstate(invalid="ignore"):     # strips without D~ points nearby: 0 / 0
        mu1 = av.smooth_blend(muh, single)
    far = ps.view(ps.xy, 0)[0] < -0.2          # Cartesian points left of the sector
    assert np.array_equal(ps.view(mu, 0)[far], ps.view(mu1, 0)[far])
    assert not np.allclose(ps.view(mu, 0)[~far], ps.view(mu1, 0)[~far])


def test_multipatch_smoothing_brute_force_at_overlap_points():
    """eqs. W, multipatch_W, zeta, multipatch_W_norm written out as explicit
    sums over every D~ point of both patches, at a few overlap points."""
    from oracle import av
    ps = synth.overlap_pair(48)
    rng = np.random.default_rng(4)
    muh = rng.uniform(0, 1, ps.plane)
    mu = av.smooth_blend(muh, ps)
    wk = lambda k: np.cos(np.pi * k / 18) ** 2 if abs(k) <= 8 else 0.0

    def rnd(t):
        return int(np.floor(t + 0.5))

    for (p, i, j) in [(0, 45, 20), (0, 40, 30), (1, 10, 2), (1, 30, 7)]:
        x, y = ps.view(ps.xy, p)[:, j, i]
        num = den = 0.0
        for R in range(ps.npatch):
            xi, eta = interp.preimage(ps.geom[R], x, y)
            if not (0 <= xi <= ps.n1[R] - 1 and 0 <= eta <= ps.n2[R] - 1):
                continue
            I, J = rnd(xi), rnd(eta)
            m = av.dtilde_mask(ps, R)
            vals = ps.view(muh, R)
            for jj in range(ps.n2[R]):
                for ii in range(ps.n1[R]):
                    if m[jj, ii]:
                        wgt = wk(I - ii) * wk(J - jj)
                        num += wgt * vals[jj, ii]
                        den += wgt
        assert abs(ps.view(mu, p)[j, i] - num / den) <= 1e-14


# ------------------------------------------------------------ reverse mode

def test_interpolation_transpose():
    ps = synth.overlap_pair(48)
    table = interp.build(ps)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, ps.plane))
    y = rng.standard_normal((4, ps.plane))
    gx = interp.interpolate(x.copy(), ps, table)
    yt = interp.interpolate_adj(y.copy(), ps, table)
    assert abs(np.sum(gx * y) - np.sum(x * yt)) <= 1e-12 * np.sum(np.abs(gx * y))


def test_multipatch_smoothing_transpose():
    from oracle import av
    ps = synth.overlap_pair(48)
    rng = np.random.default_rng(6)
    muh = rng.standard_normal(ps.plane)
    yb = rng.standard_normal(ps.plane)
    lhs = np.sum(av.smooth_blend(muh, ps) * yb)
    rhs = np.sum(muh * av.smooth_blend_adj(yb, ps))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_step_reverse_mode_on_the_pair_matches_central_differences():
    """One network step on the interpolated pair with its decisions frozen:
    the FP64 step VJP against a central difference along random directions."""
    from oracle import adjoint, solver
    cfg = synth.overlap_config(48, network=True)
    run = solver.Run(cfg)
    u0 = run.u.copy()
    run.step(record=True)
    entry = run.log[-1]

    def F(u):
        r = solver.Run(cfg)
        r.u = u.copy()
        r.step(dt=entry["dt"], tau=entry["tau"], arg=entry["arg"])
        return r.u

    rng = np.random.default_rng(7)
    w = rng.standard_normal(u0.shape)
    ub, _ = adjoint.step_vjp(run, entry, w)
    h = 1e-6
    for _ in range(2):
        v = rng.standard_normal(u0.shape) * np.abs(u0).max(axis=1, keepdims=True)
        fd = np.sum((F(u0 + h * v) - F(u0 - h * v)) * w) / (2 * h)
        an = np.sum(ub * v)
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
