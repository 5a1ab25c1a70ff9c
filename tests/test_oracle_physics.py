"""Pins of the oracle's Euler right-hand side, viscous term, SSPRK(5,4)
stepping, step size, classifier and viscosity operator against closed forms,
invariants, order conditions and brute force."""
import numpy as np
import pytest

import synth
from oracle import av, euler, fcgram, rk, solver

G = 1.4


def periodic_square(n):
    """Cartesian periodic patch: C = 0 marks plain Fourier mode along both
    directions; spacing 1/n on [0,1)."""
    ps = synth.unit_square(n)
    ps.C1[:] = 0
    ps.C2[:] = 0
    g = np.arange(n) / n
    X, Y = np.meshgrid(g, g)
    ps.xy[0, :n * n] = X.ravel()
    ps.xy[1, :n * n] = Y.ravel()
    return ps


def smooth_state(ps, rng, amp=0.1):
    x, y = ps.xy
    rho = 1 + amp * np.sin(2 * np.pi * (x + 2 * y) + rng.uniform(0, 6))
    u = 0.3 + amp * np.cos(2 * np.pi * (2 * x - y) + rng.uniform(0, 6))
    v = -0.2 + amp * np.sin(2 * np.pi * (x - y) + rng.uniform(0, 6))
    p = 1 + amp * np.cos(2 * np.pi * (x + y) + rng.uniform(0, 6))
    return synth.prim_to_cons(rho, u, v, p)


def test_fluxes_closed_form():
    e = synth.prim_to_cons(np.array(2.0), np.array(3.0), np.array(-1.0), np.array(5.0))
    assert np.allclose(e, [2, 6, -2, 5 / 0.4 + 0.5 * 2 * 10])
    F, Gf = euler.fluxes(e, G)
    E = e[3]
    assert np.allclose(F, [6, 2 * 9 + 5, 2 * 3 * -1, 3 * (E + 5)])
    assert np.allclose(Gf, [-2, 2 * 3 * -1, 2 * 1 + 5, -1 * (E + 5)])
    assert np.isclose(euler.sound_speed(e, G), np.sqrt(1.4 * 5 / 2))


def test_conservation_in_periodic_mode():
    rng = np.random.default_rng(0)
    ps = periodic_square(32)
    e = smooth_state(ps, rng)
    mu = 0.01 * (1 + 0.5 * np.sin(2 * np.pi * ps.xy[0]))
    r = euler.full_rhs(e, ps.metric, mu, ps, G)
    F, Gf = euler.fluxes(e, G)
    scale = np.abs(F).max() * 32 * 32 * 2 * np.pi
    # 1^T S = 0 for the periodic spectral derivative
    assert np.abs(r.sum(axis=1)).max() <= 1e-12 * scale


def test_single_mode_viscous_term():
    ps = periodic_square(24)
    x, y = ps.xy
    k = 3
    e = np.stack([np.sin(2 * np.pi * k * x), np.cos(2 * np.pi * k * y), np.sin(2 * np.pi * (x + y)), 0 * x + 1])
    mu = 0.02 * np.ones(ps.plane)
    t = euler.av_term(e, ps.metric, mu, ps)
    lap = np.stack([-(2 * np.pi * k) ** 2 * e[0], -(2 * np.pi * k) ** 2 * e[1],
                    -2 * (2 * np.pi) ** 2 * e[2], 0 * x])
    assert np.abs(t - 0.02 * lap).max() <= 1e-9 * 0.02 * (2 * np.pi * k) ** 2


def test_free_stream_preservation_on_curvilinear_annulus():
    ps = synth.annulus(4, 1, 64, 48)
    fs = synth.freestream(3.0)
    e = np.repeat(fs[:, None], ps.plane, axis=1)
    r = euler.full_rhs(e, ps.metric, 0.01 * np.ones(ps.plane), ps, G)
    F, Gf = euler.fluxes(fs, G)
    scale = np.abs(F).max() * np.abs(ps.metric).max()
    assert np.abs(r).max() <= 1e-8 * scale


def test_rotation_symmetry_on_square():
    rng = np.random.default_rng(5)
    ps = synth.unit_square(40)
    n = 40
    e = smooth_state(ps, rng)
    mu = 0.01 + 0.005 * ps.xy[0] * ps.xy[1]
    r = euler.full_rhs(e, ps.metric, mu, ps, G)
    # swap x <-> y (transpose the grid) and u <-> v
    def tr(a):
        return a[..., :n * n].reshape(a.shape[:-1] + (n, n)).swapaxes(-1, -2).reshape(a.shape[:-1] + (n * n,))
    e2 = tr(e)[[0, 2, 1, 3]]
    r2 = euler.full_rhs(np.pad(e2, ((0, 0), (0, ps.plane - n * n))), ps.metric,
                        np.pad(tr(mu), (0, ps.plane - n * n)), ps, G)
    want = tr(r)[[0, 2, 1, 3]]
    assert np.abs(r2[:, :n * n] - want).max() <= 1e-10 * np.abs(r).max()


def test_flux_vjp_matches_finite_differences():
    rng = np.random.default_rng(6)
    e = synth.prim_to_cons(1 + 0.2 * rng.random(7), rng.standard_normal(7), rng.standard_normal(7), 1 + rng.random(7))
    Fb, Gb = rng.standard_normal((4, 7)), rng.standard_normal((4, 7))
    eb = euler.fluxes_vjp(e, G, Fb, Gb)
    de = rng.standard_normal((4, 7))
    h = 1e-6
    Fp, Gp = euler.fluxes(e + h * de, G)
    Fm, Gm = euler.fluxes(e - h * de, G)
    fd = np.sum((Fp - Fm) * Fb + (Gp - Gm) * Gb) / (2 * h)
    assert abs(fd - np.sum(eb * de)) <= 1e-7 * abs(fd)


def test_rhs_vjp_matches_finite_differences():
    rng = np.random.default_rng(7)
    ps = synth.annulus(3, 1, 40, 28)
    e = synth.mach_state(ps, 2.0, synth.draw_perturbation(rng, level=0.05))
    mu = 0.002 * (1 + 0.3 * np.sin(ps.xy[0]))
    rb = rng.standard_normal((4, ps.plane))
    eb, mub = euler.full_rhs_vjp(e, ps.metric, mu, ps, G, rb)
    de = rng.standard_normal((4, ps.plane)) * 1e-2
    dm = rng.standard_normal(ps.plane) * 1e-4
    h = 1e-4
    fp = np.sum(euler.full_rhs(e + h * de, ps.metric, mu + h * dm, ps, G) * rb)
    fm = np.sum(euler.full_rhs(e - h * de, ps.metric, mu - h * dm, ps, G) * rb)
    fd = (fp - fm) / (2 * h)
    an = np.sum(eb * de) + np.sum(mub * dm)
    assert abs(fd - an) <= 1e-6 * abs(fd)


# ------------------------------------------------------------------ SSPRK(5,4)

def test_ssprk_order_conditions():
    A, b, c = rk.butcher()
    conds = [
        (b.sum(), 1.0),
        (b @ c, 1 / 2),
        (b @ c ** 2, 1 / 3),
        (b @ A @ c, 1 / 6),
        (b @ c ** 3, 1 / 4),
        (b @ (c * (A @ c)), 1 / 8),
        (b @ A @ c ** 2, 1 / 12),
        (b @ A @ A @ c, 1 / 24),
    ]
    for got, want in conds:
        assert abs(got - want) <= 1e-14
    for i, row in enumerate(rk.ALPHA):
        assert abs(sum(row) - 1) <= 1e-14
        assert all(a >= 0 for a in row) and all(x >= 0 for x in rk.BETA[i])
    # explicit: A strictly lower triangular
    assert np.allclose(np.triu(A), 0)


def test_ssprk_observed_order_four():
    lam = -1.3 + 0.7j
    errs = []
    for n in (20, 40, 80):
        dt = 1.0 / n
        y = np.array([1.0 + 0j])
        for _ in range(n):
            y, _, _ = rk.ssprk_step(y, dt, lambda u, s: lam * u)
        errs.append(abs(y[0] - np.exp(lam)))
    assert np.log2(errs[0] / errs[1]) > 3.8 and np.log2(errs[1] / errs[2]) > 3.8
    # nonlinear: y' = -y^2, y(0) = 1 -> y = 1/(1+t)
    errs = []
    for n in (10, 20, 40):
        y = np.array([1.0])
        for _ in range(n):
            y, _, _ = rk.ssprk_step(y, 1.0 / n, lambda u, s: -u * u)
        errs.append(abs(y[0] - 0.5))
    assert np.log2(errs[1] / errs[2]) > 3.7


def test_cfl_closed_form_for_uniform_state():
    cfg = synth.config(0)
    ps = cfg.ps
    e = np.repeat(synth.prim_to_cons(np.float64(1), np.float64(0), np.float64(0), np.float64(1))[:, None], ps.plane, 1)
    mu = 1e-3 * np.ones(ps.plane)
    dt = rk.cfl_dt(e, mu, ps, 0.5, G)
    assert np.isclose(dt, (0.5 / np.pi) / (63 * np.sqrt(1.4) + 1e-3 * 63 ** 2), rtol=1e-14)


# ------------------------------------------------------------------ AV

def test_window_weights():
    w = av.window_weights()
    assert len(w) == 17 and np.isclose(w.sum(), 9.0, atol=1e-14)
    assert np.isclose(w[8], 1.0) and np.isclose(np.cos(np.pi * 9 / 18) ** 2, 0, atol=1e-30)
    assert np.all(np.diff(w[8:]) < 0)


def test_partition_of_unity():
    for ps in (synth.uneven_sectors(3, 30, 60, 0), synth.annulus(3, 2, 44, 40)):
        mu = av.smooth_blend(np.full(ps.plane, 2.5), ps)
        for p in range(ps.npatch):
            assert np.allclose(ps.view(mu, p), 2.5, rtol=1e-14)


def test_lambda_matches_bruteforce_definition():
    """Explicit normalised sum over every patch's D~ points of the product
    window, patch by patch and point by point (eqs. W, multipatch_W_norm,
    Lambda), on a tiny 3x2 annulus."""
    ps = synth.annulus(3, 2, 30, 26)
    rng = np.random.default_rng(8)
    muh = rng.random(ps.plane)
    for p in range(ps.npatch):
        ps.view(muh, p)[~av.dtilde_mask(ps, p)] = 0
    fast = av.smooth_blend(muh, ps)
    wt = lambda k: np.cos(np.pi * k / 18) ** 2 if abs(k) <= 8 else 0.0
    ring = 3 * (30 - 19)

    def gidx(p, i, j):
        s, k = p % 3, p // 3
        return ((s * 11 + i) % ring, k * 7 + j)

    # map global index -> list of (patch, i, j)
    where = {}
    for p in range(ps.npatch):
        for j in range(26):
            for i in range(30):
                where.setdefault(gidx(p, i, j), []).append((p, i, j))
    for (p0, i0, j0) in [(0, 0, 0), (1, 15, 20), (4, 29, 3), (5, 3, 25), (2, 10, 12)]:
        gx = gidx(p0, i0, j0)
        num = den = 0.0
        for (p, i1, j1) in where[gx]:           # patches containing x, x = (i1, j1) in patch p
            m = av.dtilde_mask(ps, p)
            for j in range(26):
                for i in range(30):
                    if m[j, i]:
                        w = wt(i1 - i) * wt(j1 - j)
                        num += w * ps.view(muh, p)[j, i]
                        den += w
        assert np.isclose(ps.view(fast, p0)[j0, i0], num / den, rtol=1e-12)


def test_stencil_max_bruteforce():
    rng = np.random.default_rng(9)
    S = rng.random((9, 11))
    mx, arg = av.stencil_max(S)
    for j in range(9):
        for i in range(11):
            blk = S[max(0, j - 3):j + 4, max(0, i - 3):i + 4]
            assert mx[j, i] == blk.max()
            assert S.ravel()[arg[j, i]] == blk.max()


def test_mlp_matches_naive_loops():
    W = synth.mlp_weights(3)
    rng = np.random.default_rng(10)
    x = rng.uniform(-1, 1, (5, 16))
    out = av.mlp_logits(x, W)
    for r in range(5):
        h1 = [max(0.0, sum(x[r, i] * float(W["W1"][i, j]) for i in range(16)) + float(W["b1"][j])) for j in range(64)]
        h2 = [max(0.0, sum(h1[i] * float(W["W2"][i, j]) for i in range(64)) + float(W["b2"][j])) for j in range(64)]
        o = [sum(h2[i] * float(W["W3"][i, j]) for i in range(64)) + float(W["b3"][j]) for j in range(4)]
        assert np.allclose(out[r], o, rtol=1e-12, atol=1e-12)


def test_wave_speed_and_proxy_at_known_states():
    """S = |u| + |v| + a and Phi = |u| sqrt(rho / (gamma p)) (Sec. 5.1) at
    (rho, u, v, p) = (2, 3, -1, 5): S = 4 + sqrt(3.5), Phi = sqrt(20/7); at
    (0.5, -2, 4, 0.7): S = 6 + 1.4, Phi = sqrt(20 * 0.5 / 0.98).  The
    conserved states are written out: E = p/(gamma-1) + rho |u|^2/2."""
    e = np.array([[2.0, 0.5], [6.0, -1.0], [-2.0, 2.0], [22.5, 6.75]])
    S = rk.wave_speed(e, G)
    phi = av.proxy(e, G)
    assert np.allclose(S, [4 + np.sqrt(3.5), 7.4], rtol=1e-14, atol=0)
    assert np.allclose(phi, [np.sqrt(20 / 7), np.sqrt(10 / 0.98)], rtol=1e-14, atol=0)


def test_two_direction_class_rule():
    """The class of a point is 1 + the smaller of the two directions'
    argmax indices, a direction's ties going to the lowest index."""
    l1 = np.array([[0.1, 0.5, 0.5, 0.2], [0.9, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 1.0], [0.3, 0.3, 0.3, 0.3]])
    l2 = np.array([[0.3, 0.1, 0.2, 0.6], [0.0, 0.0, 0.7, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.1, 0.1, 0.0]])
    assert av.classes_from_logits(l1, l2).tolist() == [2, 1, 3, 1]


def _probe_network():
    """A 16-64-64-4 network with known logits: unit 0 carries the window's
    first feature x0 (offset -8), unit 1 carries -x0, so the logits are
    (relu(x0), relu(-x0), 1/4, 1/4)."""
    W = {"W1": np.zeros((16, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((64, 4)), "b3": np.array([0.0, 0.0, 0.25, 0.25])}
    W["W1"][0, 0], W["W1"][0, 1] = 1.0, -1.0
    W["W2"][0, 0] = W["W2"][1, 1] = 1.0
    W["W3"][0, 0] = W["W3"][1, 1] = 1.0
    return W


def test_classify_combines_directions_by_the_smaller_class():
    """On a 40 x 40 square with rho = 1, p = 1/gamma, v = 0 the proxy is
    Phi = |u|.  With u = 1 + 0.1 x - 0.1 y every q1 window rises (x0 = -1:
    logits (0, 1, 1/4, 1/4), class 2) and every q2 window falls (x0 = 1:
    logits (1, 0, 1/4, 1/4), class 1): the point's class is 1.  With u
    constant every window is flat (x = 0): logits (0, 0, 1/4, 1/4), tied,
    class 3 in both directions.  Points outside D~ (here the 9 columns next
    to the internal q1- side and the 9 rows next to the internal q2+ side)
    are 0."""
    import dataclasses
    ps = synth.unit_square(40)
    ps = dataclasses.replace(ps, internal=np.array([[1, 0, 0, 1]], np.uint8))
    x, y = ps.xy
    W = _probe_network()
    for u, want_in in [(1.0 + 0.1 * x - 0.1 * y, 1), (np.full(ps.plane, 1.3), 3)]:
        e = np.stack([np.ones(ps.plane), u, np.zeros(ps.plane), 1 / (G * (G - 1)) + 0.5 * u * u])
        tau, lg = av.classify(e, ps, W, G, return_logits=True)
        t = ps.view(tau, 0)
        assert np.all(t[:, :9] == 0) and np.all(t[-9:, :] == 0)
        assert np.all(t[:-9, 9:] == want_in)
    l1, l2 = lg[0]
    assert np.allclose(l1[20, 20], [0, 0, 0.25, 0.25]) and np.allclose(l2[20, 20], [0, 0, 0.25, 0.25])


def test_viscosity_generation_subgrid_width():
    """D~ leaves out exactly n_v = 9 grid lines next to each internal side
    (eq. fringe_region with the equation's strict inequality), for every
    combination of internal sides of a 30 x 26 patch."""
    import dataclasses
    import itertools
    ps = synth.uneven_sectors(1, 30, 30, 0)
    ps = dataclasses.replace(ps, n1=np.array([30], np.int32), n2=np.array([26], np.int32))
    for flags in itertools.product([0, 1], repeat=4):
        q = dataclasses.replace(ps, internal=np.array([flags], np.uint8))
        m = av.dtilde_mask(q, 0)
        assert m.shape == (26, 30)
        for j in range(26):
            for i in range(30):
                out = (flags[0] and i <= 8) or (flags[1] and i >= 21) or (flags[2] and j <= 8) or (flags[3] and j >= 17)
                assert m[j, i] == (not out), (flags, j, i)
        assert m.sum() == (30 - 9 * (flags[0] + flags[1])) * (26 - 9 * (flags[2] + flags[3]))


def test_features():
    lines = np.array([np.arange(40, dtype=float), np.full(40, 3.0)])
    f = av.features_lines(lines)
    assert np.allclose(f[0, 20], np.linspace(-1, 1, 16))
    assert np.all(f[1] == 0)
    # clamped at the left end: window of point 0 repeats sample 0 eight times
    assert np.all(f[0, 0, :9] == -1) and f[0, 0, -1] == 1


def test_preliminary_viscosity_values():
    cfg = synth.config(1, n=40)
    ps = cfg.ps
    tau = np.zeros(ps.plane, np.int8)
    for p in range(ps.npatch):
        m = av.dtilde_mask(ps, p)
        ps.view(tau, p)[m] = 1 + (np.arange(m.sum()) % 4)
    muh, arg = av.preliminary(cfg.u0, tau, ps, G)
    p = 3
    S = rk.wave_speed(ps.view(cfg.u0.astype(np.float64), p), G)
    m = av.dtilde_mask(ps, p)
    j, i = np.argwhere(m)[17]
    blk = S[max(0, j - 3):j + 4, max(0, i - 3):i + 4].max()
    t = ps.view(tau, p)[j, i]
    assert np.isclose(ps.view(muh, p)[j, i], [1.5, 1, 0.5, 0][t - 1] * blk * ps.hhat[p], rtol=1e-14)
    assert np.all(ps.view(muh, p)[~m] == 0)


def test_viscosity_vjp_matches_finite_differences():
    cfg = synth.config(1, n=36)
    ps = cfg.ps
    e = np.array(cfg.u0, np.float64)
    mu, tau, arg = av.viscosity(e, ps, cfg.mlp, G)
    rng = np.random.default_rng(11)
    mb = rng.standard_normal(ps.plane)
    eb = av.viscosity_vjp(e, tau, arg, ps, G, mb)
    de = rng.standard_normal((4, ps.plane)) * 1e-3
    h = 1e-5
    # frozen decisions: recompute mu^ with the recorded tau and argmax
    def mu_frozen(ee):
        muh = np.zeros(ps.plane)
        for p in range(ps.npatch):
            S = rk.wave_speed(ps.view(ee, p), G)
            t = ps.view(tau, p).astype(int)
            r = np.where(t > 0, av.R_TABLE[np.clip(t - 1, 0, 3)], 0.0)
            muh_p = r * S.ravel()[ps.view(arg, p)] * ps.hhat[p]
            ps.view(muh, p)[...] = np.where(av.dtilde_mask(ps, p), muh_p, 0)
        return av.smooth_blend(muh, ps)
    assert np.allclose(mu_frozen(e), mu, rtol=1e-13)
    fd = np.sum((mu_frozen(e + h * de) - mu_frozen(e - h * de)) * mb) / (2 * h)
    assert abs(fd - np.sum(eb * de)) <= 1e-6 * abs(fd)
    # Lambda transpose: dot-product identity
    x, y = rng.random(ps.plane), rng.random(ps.plane)
    for p in range(ps.npatch):
        ps.view(x, p)[~av.dtilde_mask(ps, p)] = 0
    assert np.isclose(np.sum(av.smooth_blend(x, ps) * y), np.sum(x * av.smooth_blend_adj(y, ps)), rtol=1e-12)


# ------------------------------------------------------------------ glue

def test_glue_copies_same_physical_point():
    ps = synth.annulus(4, 3, 40, 30)
    f = lambda xy: np.sin(1.3 * xy[0] + 0.2) * np.cos(0.7 * xy[1])
    e = np.zeros((4, ps.plane))
    e[0] = f(ps.xy)
    e[1:] = 7.0
    ref = e.copy()
    # scramble fringes, then glue must restore the values of f at those points
    for p in range(ps.npatch):
        v = ps.view(e, p)
        v[:, :, :5] = -1
        v[:, :, -5:] = -1
        v[:, :5, :] = -1 if p >= 4 else v[:, :5, :]
        if p < 8:
            v[:, -5:, :] = -1
    solver.glue(e, ps, 3.0)
    d = ps.dirichlet.astype(bool)
    assert np.allclose(e[0, ~d], ref[0, ~d], atol=1e-12)
    assert np.allclose(e[:, d], synth.freestream(3.0)[:, None])


def test_mlp_vjp_matches_central_differences_and_loops():
    """The network's reverse mode (Sec. 5.1 network, transposed): <x_bar, dx>
    equals the central difference of <logits, l_bar> along dx (FP64, away
    from ReLU kinks), and a naive loop over units gives the same x_bar."""
    W = synth.mlp_weights(4)
    rng = np.random.default_rng(12)
    x = rng.uniform(-1, 1, (7, 16))
    lb = rng.standard_normal((7, 4))
    xb = av.mlp_vjp(x, W, lb)
    for r in range(7):
        dx = rng.standard_normal(16)
        h = 1e-6
        fd = np.sum((av.mlp_logits(x[r] + h * dx, W) - av.mlp_logits(x[r] - h * dx, W)) * lb[r]) / (2 * h)
        assert abs(fd - xb[r] @ dx) <= 1e-7 * max(1.0, abs(fd))
    Wd = {k: np.asarray(v, np.float64) for k, v in W.items()}
    for r in range(2):
        z1 = [sum(x[r, i] * Wd["W1"][i, j] for i in range(16)) + Wd["b1"][j] for j in range(64)]
        h1 = [max(0.0, v) for v in z1]
        z2 = [sum(h1[i] * Wd["W2"][i, k] for i in range(64)) + Wd["b2"][k] for k in range(64)]
        g2 = [sum(Wd["W3"][k, l] * lb[r, l] for l in range(4)) if z2[k] > 0 else 0.0 for k in range(64)]
        g1 = [sum(Wd["W2"][j, k] * g2[k] for k in range(64)) if z1[j] > 0 else 0.0 for j in range(64)]
        want = [sum(Wd["W1"][i, j] * g1[j] for j in range(64)) for i in range(16)]
        assert np.allclose(xb[r], want, rtol=1e-12, atol=1e-12)


def test_viscous_term_vjp_matches_central_differences():
    """av_term_vjp: e_bar and mu_bar against central differences of the
    viscous term div_x (mu grad_x e) on the 3 x 2 annulus (linear in each of
    e and mu, so the difference is exact up to rounding)."""
    ps = synth.annulus(3, 2, 40, 36)
    rng = np.random.default_rng(13)
    e = rng.standard_normal((4, ps.plane))
    mu = 1e-3 * (1 + rng.random(ps.plane))
    rb = rng.standard_normal((4, ps.plane))
    eb, mub = euler.av_term_vjp(e, ps.metric, mu, ps, rb)
    de = rng.standard_normal((4, ps.plane))
    dm = 1e-3 * rng.standard_normal(ps.plane)
    keep = np.zeros(ps.plane, bool)
    keep[euler.points(ps)] = True
    de[:, ~keep] = 0
    dm[~keep] = 0
    h = 1e-3
    fe = np.sum((euler.av_term(e + h * de, ps.metric, mu, ps) - euler.av_term(e - h * de, ps.metric, mu, ps)) * rb) / (2 * h)
    fm = np.sum((euler.av_term(e, ps.metric, mu + h * dm, ps) - euler.av_term(e, ps.metric, mu - h * dm, ps)) * rb) / (2 * h)
    assert abs(fe - np.sum(eb * de)) <= 1e-9 * abs(fe)
    assert abs(fm - np.sum(mub * dm)) <= 1e-9 * abs(fm)
