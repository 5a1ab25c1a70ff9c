"""GPU parity of every hot-path operator against the FP64 oracle on the same
seeded FP32 inputs (upcast for the oracle).  Calls go through the C ABI.

Floating-point bar: relative L2 error per field <= 1e-5 (per right-hand
side evaluation) and <= 1e-4 after multi-step runs; integer outputs (classes,
maximiser indices) bit-exact, with network classes compared only where the
oracle's top-two logit gap exceeds the FP32 rounding bound."""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import av, euler, fcgram, rk, solver

pytestmark = pytest.mark.gpu
G = 1.4
RHS_TOL = 1e-5
STEP_TOL = 1e-4
# single reverse-mode evaluations: the transposed FC operators fold their
# tail onto the end samples in FP64 from the cotangent itself (the fold's
# entries reach ~1e4), so they keep the forward's accuracy up to the
# longer chains of FP32 products in the reverse passes
ADJ_TOL = 2e-5
# pointwise bar: the largest error of a component, relative to the
# component's largest value, within 10x the component's relative-L2 bar
# (errors gathered at line ends or patch edges cannot hide in the norm)
PT = 10.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_16076_amd import api
    ctx = api.Context(0)
    yield api, ctx, torch
    ctx.sync()


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a).reshape(-1))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0").contiguous()


def host(t, shape=None):
    a = t.detach().cpu().numpy()
    return a.reshape(shape) if shape is not None else a


def mkset(api, ctx, ps, layout):
    """Patch set in a storage layout with converters: D(host planes) ->
    device planes, H(device planes) -> flat row-major host planes."""
    s = api.PatchSet.from_layout(ctx, ps, layout)

    def D(a, dtype=None):
        a = np.asarray(a)
        return s.to_device(a.reshape(-1, ps.plane), dtype)

    def H(t):
        return s.to_host(t).reshape(-1)

    return s, D, H


LAYOUTS = [0, 1]


def relerr(ps, got, want):
    """relative L2 per leading field over valid patch points"""
    got = np.asarray(got, np.float64).reshape(-1, ps.plane)
    want = np.asarray(want, np.float64).reshape(-1, ps.plane)
    out = []
    for f in range(want.shape[0]):
        g = np.concatenate([ps.view(got[f], p).ravel() for p in range(ps.npatch)])
        w = np.concatenate([ps.view(want[f], p).ravel() for p in range(ps.npatch)])
        out.append(np.linalg.norm(g - w) / max(np.linalg.norm(w), 1e-300))
    return np.array(out)


def relerr_phys(ps, got, want):
    """relative L2 per conserved component, the two momentum components
    measured against their common scale sqrt(|m_x|^2 + |m_y|^2) (a flow
    along x has a y-momentum and y-momentum right-hand side that are zero up
    to rounding, so their own norm is no scale)"""
    got = np.asarray(got, np.float64).reshape(4, ps.plane)
    want = np.asarray(want, np.float64).reshape(4, ps.plane)
    def flat(a, f):
        return np.concatenate([ps.view(a[f], p).ravel() for p in range(ps.npatch)])
    nrm = [np.linalg.norm(flat(want, f)) for f in range(4)]
    mom = np.hypot(nrm[1], nrm[2])
    den = [nrm[0], mom, mom, nrm[3]]
    return np.array([np.linalg.norm(flat(got, f) - flat(want, f)) / den[f] for f in range(4)])


def maxrel_phys(ps, got, want):
    """max |got - want| per conserved component over valid patch points,
    relative to the component's largest |want| (the momentum components to
    their common scale, as in relerr_phys); any number of fields when not 4
    (then each to its own scale)"""
    got = np.asarray(got, np.float64).reshape(-1, ps.plane)
    want = np.asarray(want, np.float64).reshape(-1, ps.plane)
    nf = want.shape[0]
    def flat(a, f):
        return np.concatenate([ps.view(a[f], p).ravel() for p in range(ps.npatch)])
    sc = [np.abs(flat(want, f)).max() for f in range(nf)]
    if nf == 4:
        sc[1] = sc[2] = max(sc[1], sc[2])
    return np.array([np.abs(flat(got, f) - flat(want, f)).max() / max(sc[f], 1e-300) for f in range(nf)])


# ------------------------------------------------------------------ decisions
# The network classes and the 7 x 7 maximisers are integers decided by
# floating point.  The oracle decides in FP64 (the definition); the kernels
# decide on FP32 values.  Bounds on the FP32 values' errors:
#   * Phi and S from an FP32 state: relative error <= (4 kappa + 8) u,
#     u = 2^-24, kappa = E / (E - |m|^2/(2 rho)) the cancellation factor of
#     the pressure (a chain of about eight roundings, the subtraction's
#     operands' errors amplified by kappa);
#   * features x = 2 (w - lo)/(hi - lo) - 1 of a window whose samples carry
#     absolute errors <= eps: |dx| <= 8 eps / (rng - 2 eps) + 8 u
#     (rng = hi - lo; unbounded when 2 eps >= rng or when rng is within
#     2 eps of the flatness threshold; a window of identical samples is flat
#     on both sides);
#   * logits, to first order: |dl_k| <= sum_i |J_ik| max |dx|, J the
#     network's Jacobian at the window (W1 D1 W2 D2 W3, D the ReLU masks),
#     plus the network's own rounding (fp16 splits with FP32 sums: <= 100 u
#     times the magnitude of every layer's products, carried on by the
#     later layers' largest column sums of |W|).
# A decision whose FP64 margin (top-two logit gap, or best minus second
# 7 x 7 value) exceeds twice the bound is compared exactly; at every other
# point the GPU's choice must be one of the FP64 candidates within twice
# the bound of the best.  The features are ill-conditioned (the window's
# range of Phi is ~1e-3 of Phi on a +-1 % flow, less on small subpatches),
# so on these workloads 10-50 % of the classes, and as many of the
# maximisers (S varies along plane waves, so stencils hold near-equal
# values), are such near ties; their count is printed.
U32 = 2.0 ** -24


def fp32_value_bound(e):
    """Relative FP32 error bound of Phi and S at every point of e [4, ...]."""
    rho, m, n, E = np.asarray(e, np.float64)
    ke = 0.5 * (m * m + n * n) / rho
    return (4.0 * np.abs(E) / np.abs(E - ke) + 8.0) * U32


def _window_dx_bound(phi, eps):
    """[nl, n] lines of Phi and of its absolute error bound -> [nl, n] bound
    on max |dx| over each point's window (inf where undecidable)."""
    nl, n = phi.shape
    idx = np.clip(np.arange(n)[:, None] + np.arange(-8, 8)[None, :], 0, n - 1)
    w, ew = phi[:, idx], eps[:, idx]
    lo, hi = w.min(-1), w.max(-1)
    rng = hi - lo
    em = ew.max(-1)
    thr = 1e-6 * np.maximum(1.0, np.abs(hi))
    with np.errstate(divide="ignore", invalid="ignore"):
        dx = np.where(2 * em < rng, 8 * em / (rng - 2 * em) + 8 * U32, np.inf)
    dx = np.where(np.abs(rng - thr) <= 2 * em, np.inf, dx)          # flatness undecidable
    dx = np.where(rng + 2 * em < thr, 8 * U32, dx)                   # flat on both sides
    dx = np.where(rng == 0, 0.0, dx)                                 # identical samples
    return dx


def _logit_bound(x, dx, W):
    """First-order bound of |FP32 logits - FP64 logits| for feature rows x
    [..., 16] with feature errors <= dx [...]."""
    W = {k: np.asarray(v, np.float64) for k, v in W.items()}
    A = {k: np.abs(v) for k, v in W.items()}
    z1 = x @ W["W1"] + W["b1"]
    z2 = np.maximum(z1, 0) @ W["W2"] + W["b2"]
    Tm = np.matmul(W["W2"], (z2 > 0)[..., :, None] * W["W3"])            # [..., 64, 4]
    J = np.matmul(W["W1"], (z1 > 0)[..., :, None] * Tm)                  # [..., 16, 4]
    first = np.abs(J).sum(-2) * dx[..., None]
    n = [A[k].sum(0).max() for k in ("W1", "W2", "W3")]
    m1 = np.abs(x) @ A["W1"] + A["b1"]
    m2 = m1 @ A["W2"] + A["b2"]
    m3 = m2 @ A["W3"] + A["b3"]
    own = 100 * U32 * (m3 + n[2] * m2.max(-1, keepdims=True) + n[2] * n[1] * m1.max(-1, keepdims=True))
    with np.errstate(invalid="ignore"):
        return first + own


def decision_check(ps, e, mlp, tau_gpu, arg_gpu=None, logits_gpu=None, label=""):
    """Compare the GPU's classes (and maximisers, logits) at the FP32 state
    e with the oracle's FP64 decisions: exactly where the FP64 margin is
    above twice the FP32 bound, and as a choice among the near-tied FP64
    candidates everywhere else; logits within the bound."""
    from oracle import rk
    e = np.asarray(e, np.float64).reshape(4, ps.plane)
    want, lg = av.classify(e, ps, mlp, G, return_logits=True)
    comp = excl = acomp = aexcl = 0
    for p in range(ps.npatch):
        ep = ps.view(e, p)
        rel = fp32_value_bound(ep)
        phi = av.proxy(ep, G)
        eps = rel * np.abs(phi)
        m = av.dtilde_mask(ps, p)
        l1, l2 = lg[p]
        x1 = av.features_lines(phi)
        x2 = np.swapaxes(av.features_lines(phi.T), 0, 1)
        b1 = _logit_bound(x1, _window_dx_bound(phi, eps), mlp)
        b2 = _logit_bound(x2, np.swapaxes(_window_dx_bound(phi.T, eps.T), 0, 1), mlp)
        B1, B2 = b1.max(-1), b2.max(-1)

        def gap(l):
            srt = np.sort(l, axis=-1)
            return srt[..., -1] - srt[..., -2]
        sure = (gap(l1) > 2 * B1) & (gap(l2) > 2 * B2) & m
        g = ps.view(tau_gpu, p)
        assert np.array_equal(g[sure], ps.view(want, p)[sure]), (label, p)
        assert np.all(g[~m] == 0) and np.all((g[m] >= 1) & (g[m] <= 4))
        # near ties: the GPU's class is 1 + min(i, j) over candidates i of
        # direction 1 and j of direction 2 within 2B of their best logit
        c1 = l1 >= l1.max(-1, keepdims=True) - 2 * B1[..., None]
        c2 = l2 >= l2.max(-1, keepdims=True) - 2 * B2[..., None]
        ok = np.zeros(g.shape, bool)
        for i in range(4):
            for j in range(4):
                ok |= c1[..., i] & c2[..., j] & (g == 1 + min(i, j))
        assert np.all(ok[m & ~sure]), (label, p)
        comp += int(sure.sum())
        excl += int((m & ~sure).sum())
        if logits_gpu is not None:
            o, a_, b_ = int(ps.off[p]), int(ps.n1[p]), int(ps.n2[p])
            gls = []
            for k, (lw, bd) in enumerate(((l1, b1), (l2, b2))):
                gl = logits_gpu[k][o:o + a_ * b_].reshape(b_, a_, 4)
                fin = m[..., None] & np.isfinite(bd)
                assert np.all(np.abs(gl - lw)[fin] <= bd[fin]), (label, p, k)
                assert np.all(gl[~m] == 0)
                gls.append(gl)
            # the GPU's classes are its own logits' classes (same rule)
            assert np.array_equal(g[m], av.classes_from_logits(gls[0], gls[1])[m]), (label, p)
        if arg_gpu is not None:
            a, x = maximiser_check(ep, ps.view(arg_gpu, p), (label, p))
            acomp += a
            aexcl += x
    say("  decisions", label, "classes compared", comp, "near ties", excl,
        "| maximisers compared", acomp, "near ties", aexcl)
    assert comp > 0 and (arg_gpu is None or acomp > 0)
    return comp, excl


def maximiser_check(ep, ga, label=""):
    """The GPU's 7 x 7 maximisers ga [n2, n1] (patch-local flat indices) at
    the FP32 patch state ep [4, n2, n1]: the FP64 maximiser wherever the
    margin best - second exceeds twice the FP32 bound of S, elsewhere a
    position of the clamped stencil whose FP64 value is within that bound
    of the best.  Returns (compared, near ties)."""
    from oracle import rk
    S = rk.wave_speed(ep, G)
    best, arg, second = av.stencil_max(S, second=True)
    dS, _ = av.stencil_max(fp32_value_bound(ep) * S)
    sure = best - second > 2 * dS
    assert np.array_equal(ga[sure], arg[sure]), label
    b_, a_ = S.shape
    J_, I_ = np.meshgrid(np.arange(b_), np.arange(a_), indexing="ij")
    inside = (ga >= 0) & (ga < a_ * b_) & (np.abs(ga // a_ - J_) <= 3) & (np.abs(ga % a_ - I_) <= 3)
    assert np.all(inside), label
    assert np.all(S.ravel()[np.clip(ga, 0, a_ * b_ - 1)] >= best - 2 * dS), label
    return int(sure.sum()), int((~sure).sum())


def first_step_input(api, s, D, ps, u, cfg):
    """The glued FP32 state a step's network sees: a copy of the device
    state through fcsd_glue (fringe copies, Dirichlet inflow, walls)."""
    x = u.clone()
    if ps.dirichlet is not None:
        api.fcsd_glue(s, x, D(ps.dirichlet), synth.freestream(cfg.mach))
    else:
        api.fcsd_glue(s, x)
    return s.to_host(x).reshape(4, -1)


def smooth_fields(ps, nf, seed):
    rng = np.random.default_rng(seed)
    x, y = ps.xy
    out = np.zeros((nf, ps.plane), np.float32)
    for f in range(nf):
        v = np.zeros(ps.plane)
        for _ in range(3):
            k = rng.uniform(-2, 2, 2)
            v += rng.uniform(-1, 1) * np.sin(2 * np.pi * (k[0] * x + k[1] * y) + rng.uniform(0, 6))
        v += rng.uniform(-1, 1)
        for p in range(ps.npatch):
            ps.view(out[f], p)[...] = ps.view(v, p)
    return out


def uneven(seed=11, npatch=6, nmax=160):
    return synth.uneven_sectors(npatch, 48, nmax, seed)


# ------------------------------------------------------------------ FC line operators

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("direction", [1, 2])
def test_fc_diff_uneven_patches(env, direction, layout):
    api, ctx, torch = env
    ps = uneven()
    say("fc_diff uneven", direction, "layout", layout, list(zip(ps.n1, ps.n2)))
    s, D, H = mkset(api, ctx, ps, layout)
    F = smooth_fields(ps, 3, 1)
    out = torch.zeros(3 * s.plane, device="cuda:0")
    api.fc_diff(s, direction, D(F), out, nf=3)
    want = fcgram.diff_plane(F.astype(np.float64), ps, direction)
    err = relerr(ps, H(out), want)
    mx = maxrel_phys(ps, H(out), want)
    say("  rel L2", err, "max", mx)
    assert np.all(err < RHS_TOL) and np.all(mx < PT * RHS_TOL)
    s.close()


@pytest.mark.parametrize("direction", [1, 2])
def test_periodic_fc_diff(env, direction):
    """C = 0 is the periodic Fourier derivative (Sec. 2.2 without
    continuation; h = 1/N, period 1): on a 60 x 60 patch of samples of
    trigonometric polynomials with wavenumbers below N/2 it is the textbook
    derivative, and its transpose is its negative."""
    api, ctx, torch = env
    ps = synth.unit_square(60, C=0)
    s = api.PatchSet.from_layout(ctx, ps)
    q = np.arange(60) / 60.0
    Q1, Q2 = np.meshgrid(q, q)                      # [j, i]: Q1 along q1 (i), Q2 along q2 (j)
    F = np.zeros((2, ps.plane))
    dF = np.zeros((2, ps.plane))
    f0 = np.sin(2 * np.pi * 3 * Q1) * np.cos(2 * np.pi * 2 * Q2) + 0.5 * np.cos(2 * np.pi * 7 * Q1 + 0.3)
    f1 = np.cos(2 * np.pi * 11 * Q2 - 0.2) * (1 + 0.3 * np.sin(2 * np.pi * Q1)) + 0.2 * np.sin(2 * np.pi * 5 * (Q1 + Q2))
    if direction == 1:
        d0 = 6 * np.pi * np.cos(2 * np.pi * 3 * Q1) * np.cos(2 * np.pi * 2 * Q2) - 7 * np.pi * np.sin(2 * np.pi * 7 * Q1 + 0.3)
        d1 = np.cos(2 * np.pi * 11 * Q2 - 0.2) * 0.6 * np.pi * np.cos(2 * np.pi * Q1) + 2 * np.pi * np.cos(2 * np.pi * 5 * (Q1 + Q2))
    else:
        d0 = -4 * np.pi * np.sin(2 * np.pi * 3 * Q1) * np.sin(2 * np.pi * 2 * Q2)
        d1 = -22 * np.pi * np.sin(2 * np.pi * 11 * Q2 - 0.2) * (1 + 0.3 * np.sin(2 * np.pi * Q1)) + 2 * np.pi * np.cos(2 * np.pi * 5 * (Q1 + Q2))
    for f, (a, b) in enumerate(((f0, d0), (f1, d1))):
        ps.view(F[f], 0)[...] = a
        ps.view(dF[f], 0)[...] = b
    F32 = F.astype(np.float32)
    out = torch.zeros(2 * ps.plane, device="cuda:0")
    api.fc_diff(s, direction, dev(torch, F32), out, nf=2)
    got = host(out).reshape(2, -1)
    err_t = relerr(ps, got, dF)
    err_o = relerr(ps, got, fcgram.diff_plane(F32.astype(np.float64), ps, direction))
    acc = torch.zeros(2 * ps.plane, device="cuda:0")
    api.fc_diff_adj(s, direction, dev(torch, F32), acc, nf=2)
    err_a = relerr(ps, host(acc).reshape(2, -1), -fcgram.diff_plane(F32.astype(np.float64), ps, direction))
    say("periodic fc_diff", direction, "vs textbook", err_t, "vs oracle", err_o, "transpose", err_a)
    assert np.all(err_t < RHS_TOL) and np.all(err_o < RHS_TOL) and np.all(err_a < RHS_TOL)
    s.close()


@pytest.mark.parametrize("direction", [1, 2])
def test_fc_diff_adjoint(env, direction):
    api, ctx, torch = env
    ps = uneven(seed=12, npatch=4)
    s = api.PatchSet.from_layout(ctx, ps)
    Y = smooth_fields(ps, 2, 2)
    acc = dev(torch, smooth_fields(ps, 2, 3))
    base = host(acc).copy()
    api.fc_diff_adj(s, direction, dev(torch, Y), acc, nf=2)
    want = base.reshape(2, -1) + fcgram.diff_plane_adj(Y.astype(np.float64), ps, direction)
    err = relerr(ps, host(acc), want)
    # the transposed part alone (the accumulator's base is exact)
    d_err = relerr(ps, host(acc) - base, want - base.reshape(2, -1))
    mx = maxrel_phys(ps, host(acc) - base, want - base.reshape(2, -1))
    say("fc_diff_adj", direction, err, "transposed part", d_err, "max", mx)
    assert np.all(d_err < ADJ_TOL) and np.all(mx < PT * ADJ_TOL)
    s.close()


@pytest.mark.parametrize("direction", [1, 2])
def test_fc_continue_and_transpose(env, direction):
    api, ctx, torch = env
    ps = uneven(seed=13, npatch=3, nmax=120)
    s = api.PatchSet.from_layout(ctx, ps)
    F = smooth_fields(ps, 2, 4)
    ep = s.ext_size(direction)
    ext = torch.zeros(2 * ep, device="cuda:0")
    api.fc_continue(s, direction, dev(torch, F), ext, nf=2)
    got = host(ext).reshape(2, ep)
    want = fcgram.continue_plane(F.astype(np.float64), ps, direction)
    o = 0
    for p in range(ps.npatch):
        w = want[p]                       # [2, nlines, L]
        n = w.shape[1] * w.shape[2]
        g = got[:, o:o + n].reshape(w.shape)
        assert np.abs(g - w).max() <= 1e-5 * np.abs(w).max()
        o += n
    # transpose
    rng = np.random.default_rng(5)
    eb = rng.standard_normal((2, ep)).astype(np.float32)
    inb = torch.zeros(2 * ps.plane, device="cuda:0")
    api.fc_continue_adj(s, direction, dev(torch, eb), inb, nf=2)
    bars, o = [], 0
    for p in range(ps.npatch):
        shp = want[p].shape
        n = shp[1] * shp[2]
        bars.append(eb[:, o:o + n].reshape(shp).astype(np.float64))
        o += n
    wb = fcgram.continue_plane_adj(bars, ps, direction, (2, ps.plane))
    err = relerr(ps, host(inb), wb)
    say("fc_continue_adj", direction, err)
    assert np.all(err < RHS_TOL)
    s.close()


# ------------------------------------------------------------------ strict continuation length
# C = 27 on every line: most extension lengths N + 27 then have a prime
# factor above 13 and their circulants run embedded in a 13-smooth transform
# of length M >= N + L (zero padding, wrapped first column).

def strict_uneven(seed=21, npatch=6, nmax=400):
    ps = synth.with_continuation(synth.uneven_sectors(npatch, 48, nmax, seed), 27)
    emb = [(n, n + 27) for n in list(ps.n1) + list(ps.n2) if not synth.smooth13(int(n) + 27)]
    say("strict C = 27:", len(emb), "of", 2 * ps.npatch, "line families embedded", emb)
    assert len(emb) >= ps.npatch
    return ps


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("direction", [1, 2])
def test_strict_continuation_fc_diff(env, direction, layout):
    """fc_diff and fc_diff_adj on lines whose N + 27 has a prime factor
    above 13, against the oracle (which transforms length N + 27 directly)."""
    api, ctx, torch = env
    ps = strict_uneven()
    s, D, H = mkset(api, ctx, ps, layout)
    F = smooth_fields(ps, 3, 1)
    out = torch.zeros(3 * s.plane, device="cuda:0")
    api.fc_diff(s, direction, D(F), out, nf=3)
    want = fcgram.diff_plane(F.astype(np.float64), ps, direction)
    err, mx = relerr(ps, H(out), want), maxrel_phys(ps, H(out), want)
    Y = smooth_fields(ps, 2, 2)
    acc = torch.zeros(2 * s.plane, device="cuda:0")
    api.fc_diff_adj(s, direction, D(Y), acc, nf=2)
    wa = fcgram.diff_plane_adj(Y.astype(np.float64), ps, direction)
    ea, ma = relerr(ps, H(acc), wa), maxrel_phys(ps, H(acc), wa)
    say("strict fc_diff", direction, layout, "rel L2", err, "max", mx, "transpose", ea, "max", ma)
    assert np.all(err < RHS_TOL) and np.all(mx < PT * RHS_TOL)
    assert np.all(ea < ADJ_TOL) and np.all(ma < PT * ADJ_TOL)
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_strict_continuation_rhs_and_filter(env, layout):
    """The full right-hand side and the spectral filter of the strict set
    against the oracle."""
    from oracle import filter as flt
    api, ctx, torch = env
    ps = strict_uneven(seed=22, npatch=5, nmax=300)
    cfg = synth.config(2, npatch=5, nmax=300)
    u = np.zeros((4, ps.plane), np.float32)
    e = synth.mach_state(ps, 3.0, cfg.pert)
    for p in range(ps.npatch):
        ps.view(u, p)[...] = ps.view(e, p)
    mu = (0.002 * (1.5 + np.sin(4 * ps.xy[1]))).astype(np.float32)
    s, D, H = mkset(api, ctx, ps, layout)
    rhs = torch.zeros(4 * s.plane, device="cuda:0")
    api.fcsd_rhs(s, D(u), D(ps.metric), D(mu), cfg.ref, G, rhs)
    want = euler.full_rhs(u.astype(np.float64), ps.metric, mu.astype(np.float64), ps, G)
    err, mx = relerr_phys(ps, H(rhs), want), maxrel_phys(ps, H(rhs), want)
    un = noisy_state(ps, u, 3)
    s.set_filter(ALPHA_F, P_F)
    out = torch.zeros(4 * s.plane, device="cuda:0")
    api.fcsd_filter(s, D(un), out, G)
    wf = flt.filter_state(un.astype(np.float64), ps, ALPHA_F, P_F, G)
    got = H(out).reshape(4, -1)
    ef = relerr_phys(ps, got, wf)
    ec = relerr_phys(ps, got - un, wf - un)
    say("strict rhs", layout, "rel L2", err, "max", mx, "filter", ef, "filter change", ec)
    assert np.all(err < RHS_TOL) and np.all(mx < PT * RHS_TOL)
    assert np.all(ef < FILTER_TOL) and np.all(ec < 2e-2)
    s.close()


def test_strict_continuation_steps_with_network(env):
    """Three network steps of the 16-sector annulus at 52 x 52 with C = 27
    (L = 79, prime: every line runs embedded), the oracle replaying the
    GPU's decisions."""
    api, ctx, torch = env
    cfg = synth.config(1, n=52)
    import dataclasses
    cfg = dataclasses.replace(cfg, ps=synth.with_continuation(cfg.ps, 27))
    ps = cfg.ps
    assert not synth.smooth13(52 + 27)
    s, D, H = mkset(api, ctx, ps, 1)
    u = D(cfg.u0)
    st = api.Stepper(s, u, D(ps.metric), cfg.ref, W={k: dev(torch, v) for k, v in cfg.mlp.items()},
                     dirichlet_mask=D(ps.dirichlet), dirichlet_state=synth.freestream(cfg.mach))
    run = solver.Run(cfg)
    for k in range(3):
        st.step(use_graph=(k > 0))
        run.step(dt=float(host(st.dt)[0]), tau=H(st.tau), arg=H(st.argmax))
    got = H(u).reshape(4, -1)
    err, mx = relerr_phys(ps, got, run.u), maxrel_phys(ps, got, run.u)
    say("strict annulus 3 steps", err, "max", mx)
    assert np.all(err < STEP_TOL) and np.all(mx < PT * STEP_TOL)
    s.close()


# ------------------------------------------------------------------ right-hand side

def rhs_case(name):
    if name == "square64":
        cfg = synth.config(0)
        mu = np.full(cfg.ps.plane, 1e-3, np.float32)
        return cfg.ps, cfg.u0, mu, cfg.ref
    if name == "annulus":
        cfg = synth.config(1, n=48)
        ps = cfg.ps
        mu = (0.004 * (1.2 + np.sin(3 * ps.xy[0]) * np.cos(2 * ps.xy[1]))).astype(np.float32)
        return ps, cfg.u0, mu, cfg.ref
    if name == "shells":
        ps = synth.annulus(16, 2, 48, 40)
        rng = np.random.default_rng(9)
        e = synth.mach_state(ps, 3.0, synth.draw_perturbation(rng))
        u = np.zeros((4, ps.plane), np.float32)
        for p in range(ps.npatch):
            ps.view(u, p)[...] = ps.view(e, p)
        mu = (0.003 * (1.1 + np.cos(2 * ps.xy[0] + ps.xy[1]))).astype(np.float32)
        return ps, u, mu, np.array([1.4, 3.0, 0.0, 1.0])
    if name == "paper_d2":
        # the paper's subpatches: 101 x 101 points, d = 2, C = 27 (L = 128)
        cfg = synth.paper_subpatches(8, 2)
        ps = cfg.ps
        mu = (0.003 * (1.3 + np.sin(2 * ps.xy[0] - ps.xy[1]))).astype(np.float32)
        return ps, cfg.u0, mu, cfg.ref
    if name == "overlap":
        cfg = synth.overlap_config(48)
        ps = cfg.ps
        mu = (0.002 * (1.2 + np.sin(2 * ps.xy[0] + ps.xy[1]))).astype(np.float32)
        return ps, cfg.u0, mu, cfg.ref
    if name == "uneven":
        cfg = synth.config(2, npatch=5, nmax=200)
        ps = cfg.ps
        mu = (0.002 * (1.5 + np.sin(4 * ps.xy[1]))).astype(np.float32)
        return ps, cfg.u0, mu, cfg.ref
    raise KeyError(name)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", ["square64", "annulus", "shells", "uneven", "paper_d2"])
def test_full_rhs(env, case, layout):
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case(case)
    say("fcsd_rhs", case, "layout", layout, ps.npatch, "patches", ps.npoints, "points")
    s, D, H = mkset(api, ctx, ps, layout)
    metric = D(ps.metric)
    ud, mud = D(u), D(mu)
    rhs = torch.zeros(4 * s.plane, device="cuda:0")
    api.fcsd_rhs(s, ud, metric, mud, ref, G, rhs)
    want = euler.full_rhs(u.astype(np.float64), ps.metric, mu.astype(np.float64), ps, G)
    err = relerr_phys(ps, H(rhs), want)
    # inviscid and viscous parts through their own entry points
    r1 = torch.zeros(4 * s.plane, device="cuda:0")
    api.euler_rhs(s, ud, metric, ref, G, r1)
    w1 = euler.euler_rhs(u.astype(np.float64), ps.metric, ps, G)
    e1 = relerr_phys(ps, H(r1), w1)
    api.av_apply(s, ud, metric, mud, ref, r1)
    e2 = relerr_phys(ps, H(r1), want)
    mx = maxrel_phys(ps, H(rhs), want)
    say("  full rhs rel L2", err, "max", mx, "euler_rhs", e1, "euler_rhs + av_apply", e2)
    assert np.all(err < RHS_TOL) and np.all(mx < PT * RHS_TOL)
    assert np.all(e1 < RHS_TOL) and np.all(e2 < RHS_TOL)
    s.close()


# ------------------------------------------------------------------ time stepping

def test_rk_stages_match_shu_osher(env):
    api, ctx, torch = env
    ps = uneven(seed=14, npatch=2, nmax=64)
    s = api.PatchSet.from_layout(ctx, ps)
    rng = np.random.default_rng(6)
    u0 = rng.standard_normal((4, ps.plane)).astype(np.float32)
    R = [rng.standard_normal((4, ps.plane)).astype(np.float32) for _ in range(5)]
    dt = np.float32(0.013)
    dtd = dev(torch, np.array([dt], np.float32))
    U0 = dev(torch, u0)
    bufs = [torch.zeros(4 * ps.plane, device="cuda:0") for _ in range(2)]
    acc = torch.zeros(4 * ps.plane, device="cuda:0")
    ins = [U0, bufs[0], bufs[1], bufs[0], bufs[1]]
    outs = [bufs[0], bufs[1], bufs[0], bufs[1], U0]
    for k in range(5):
        api.rk_stage(s, k, dtd, dev(torch, R[k]), U0, ins[k], acc, outs[k])
    new, _, _ = rk.ssprk_step(u0.astype(np.float64), float(dt), lambda u, k: R[k].astype(np.float64))
    err = np.abs(host(U0).reshape(4, -1) - new).max() / np.abs(new).max()
    say("rk_stage x5 max rel", err)
    assert err < 1e-6
    s.close()


def test_cfl_step_size(env):
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case("shells")
    s = api.PatchSet.from_layout(ctx, ps)
    dtd = torch.zeros(1, device="cuda:0")
    api.fcsd_cfl_dt(s, dev(torch, u), dev(torch, mu), 0.5, G, dtd)
    want = rk.cfl_dt(u.astype(np.float64), mu.astype(np.float64), ps, 0.5, G)
    got = float(host(dtd)[0])
    say("cfl dt", got, want)
    assert abs(got - want) <= 2e-6 * want
    s.close()


def test_state_monitor(env):
    """fcsd_check: 0 on an admissible state; each planted defect at a grid
    point sets its bit (1 non-finite, 2 rho <= 0, 4 p <= 0); a defect in
    the padding between patches is not looked at."""
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case("uneven")
    s = api.PatchSet.from_layout(ctx, ps)
    flags = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")

    def run(v):
        api.fcsd_check(s, dev(torch, v), G, flags)
        return int(host(flags)[0])

    assert run(u) == 0
    p = ps.npatch // 2
    n1, n2 = int(ps.n1[p]), int(ps.n2[p])
    for field, val, want in [(2, np.nan, 1 | 4), (0, -1.0, 2), (3, 0.0, 4), (1, np.inf, 1 | 4)]:
        v = u.copy()
        ps.view(v, p)[field, n2 - 1, n1 - 1] = val
        got = run(v)
        say("planted", field, val, got)
        assert got == want
    two = u.copy()
    ps.view(two, 0)[0, 0, 0] = -1.0
    ps.view(two, ps.npatch - 1)[2, 3, 5] = np.nan
    assert run(two) == (1 | 2 | 4)
    used = np.zeros(ps.plane, bool)
    for q in range(ps.npatch):
        used[int(ps.off[q]):int(ps.off[q]) + int(ps.n1[q]) * int(ps.n2[q])] = True
    if not used.all():
        v = u.copy()
        v[:, np.nonzero(~used)[0][0]] = np.nan
        assert run(v) == 0
    s.close()


# ------------------------------------------------------------------ viscosity

@pytest.mark.parametrize("layout", LAYOUTS)
def test_network_classes(env, layout):
    """sdnn_infer against the oracle's FP64 classifier: logits of both
    directions within the FP32 bound of every window, classes equal wherever
    the FP64 top-two gap exceeds twice it (near ties counted); both storage
    layouts (their window gathers differ)."""
    api, ctx, torch = env
    cfg = synth.config(1, n=48)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    tau = torch.zeros(s.plane, dtype=torch.int8, device="cuda:0")
    logits = torch.zeros(8 * s.plane, device="cuda:0")
    api.sdnn_infer(s, D(cfg.u0), G, W, tau, logits)
    # [2][plane][4] -> per (direction, class) planes -> host [2][plane][4]
    lg = logits.view(2, s.plane, 4).permute(0, 2, 1).contiguous().view(8, s.plane)
    gl = H(lg).reshape(2, 4, ps.plane).transpose(0, 2, 1)
    decision_check(ps, cfg.u0, cfg.mlp, H(tau), logits_gpu=gl, label=f"network layout {layout}")
    assert s.stage_errors() == 0
    s.close()


def test_network_range_flag(env):
    """Weights that let a hidden activation reach the fp16 range set bit 1
    of the set's error word (the split products would overflow); ordinary
    weights leave it clear, and reading the word clears it."""
    api, ctx, torch = env
    cfg = synth.config(1, n=48)
    ps = cfg.ps
    s = api.PatchSet.from_layout(ctx, ps)
    u = dev(torch, cfg.u0)
    tau = torch.zeros(ps.plane, dtype=torch.int8, device="cuda:0")
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    api.sdnn_infer(s, u, G, W, tau)
    assert s.stage_errors() == 0
    big = dict(cfg.mlp)
    big["W1"] = cfg.mlp["W1"] * 3e4
    api.sdnn_infer(s, u, G, {k: dev(torch, v) for k, v in big.items()}, tau)
    assert s.stage_errors() == 2
    assert s.stage_errors() == 0
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", ["annulus", "shells", "uneven", "overlap"])
def test_viscosity_operator(env, case, layout):
    api, ctx, torch = env
    ps, u, _, ref = rhs_case(case)
    s, D, H = mkset(api, ctx, ps, layout)
    if ps.geom is not None:
        s.set_interp(ps.geom)        # smoothing across the non-aligned pair
    rng = np.random.default_rng(15)
    tau = np.zeros(ps.plane, np.int8)
    for p in range(ps.npatch):
        m = av.dtilde_mask(ps, p)
        ps.view(tau, p)[m] = rng.integers(1, 5, m.sum())
    mu = torch.zeros(s.plane, device="cuda:0")
    amax = torch.zeros(s.plane, dtype=torch.int32, device="cuda:0")
    api.av_viscosity(s, D(u), D(tau), G, mu, amax)
    muh, arg = av.preliminary(u.astype(np.float64), tau, ps, G)
    want = av.smooth_blend(muh, ps)
    err = relerr(ps, H(mu), want)
    mx = maxrel_phys(ps, H(mu), want)
    # maximisers: the FP64 one where the margin exceeds the FP32 bound of S,
    # elsewhere a near-tied stencil position
    ga = H(amax)
    comp = excl = 0
    for p in range(ps.npatch):
        a, x = maximiser_check(ps.view(np.asarray(u, np.float64), p), ps.view(ga, p), (case, p))
        comp += a
        excl += x
    say("av_viscosity", case, err, "max", mx, "maximisers compared", comp, "near ties", excl)
    assert err[0] < 2e-6 and mx[0] < 2e-5 and comp > 0
    s.close()


def test_glue(env):
    api, ctx, torch = env
    ps = synth.annulus(4, 3, 44, 40)
    rng = np.random.default_rng(16)
    u = rng.standard_normal((4, ps.plane)).astype(np.float32)
    mask = ps.dirichlet
    st = synth.freestream(3.0).astype(np.float32)
    s = api.PatchSet.from_layout(ctx, ps)
    ud = dev(torch, u)
    api.fcsd_glue(s, ud, dev(torch, mask), st)
    want = u.astype(np.float64).copy()
    solver.glue(want, ps, 3.0)
    got = host(ud).reshape(4, -1)
    for p in range(ps.npatch):
        assert np.array_equal(ps.view(got, p), ps.view(want.astype(np.float32), p))
    s.close()


# ------------------------------------------------------------------ fused stage, step

@pytest.mark.parametrize("layout", LAYOUTS)
def test_fused_stage_and_per_patch_equal(env, layout):
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case("uneven")
    s, D, H = mkset(api, ctx, ps, layout)
    dt = 2e-2
    dtd = dev(torch, np.array([dt], np.float32))
    metric, mud = D(ps.metric), D(mu)
    u0 = D(u)
    ui = D(u * np.float32(1.0001))
    outs = []
    for per in (False, True):
        acc = torch.zeros(4 * s.plane, device="cuda:0")
        uo = torch.zeros(4 * s.plane, device="cuda:0")
        api.fcsd_stage(s, 1, u0, ui, acc, uo, metric, mud, ref, G, dtd, per_patch=per)
        outs.append(H(uo))
    assert np.array_equal(outs[0], outs[1])
    ui64 = (u * np.float32(1.0001)).astype(np.float64)
    r = euler.full_rhs(ui64, ps.metric, mu.astype(np.float64), ps, G)
    want = rk.ALPHA[1][0] * u.astype(np.float64) + rk.ALPHA[1][1] * ui64 + rk.BETA[1][1] * dt * r
    err = relerr_phys(ps, outs[0], want)
    say("fused stage state", err)
    assert np.all(err < 1e-6)
    s.close()


SCHEDULES = (0, 1, 2, 3)   # split (four launches), fused (three), persistent (one per stage), fused wide


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", ["uneven", "annulus", "square64", "overlap", "uneven_inviscid"])
def test_schedules_give_identical_stages(env, case, layout):
    """The launch schedules of a stage's line passes run the same FP32
    operations on every line: all five stages, viscous and inviscid, are
    bit-identical across them and across the two tilings (and the
    persistent queue's waits never give up).  Small tiles make the
    persistent queue long (many tasks per patch and per workgroup), and
    there pass A's two-line tiles would need more LDS than its one-line
    ones, so it runs on the latter (the large tiling uses the former)."""
    api, ctx, torch = env
    name = case.replace("_inviscid", "")
    ps, u, mu, ref = rhs_case(name)
    s, D, H = mkset(api, ctx, ps, layout)
    metric = D(ps.metric)
    mud = None if case.endswith("_inviscid") else D(mu)
    dtd = dev(torch, np.array([1e-3], np.float32))
    u0 = D(u)
    first = None
    for tiles in [((65536,) * 3, (512,) * 3), ((16384, 16384, 24576), (256,) * 3)]:
        s.tune(*tiles, 1)
        outs = {}
        for sched in SCHEDULES:
            s.set_schedule(sched)
            acc = torch.zeros(4 * s.plane, device="cuda:0")
            ua = torch.zeros(4 * s.plane, device="cuda:0")
            ub = torch.zeros(4 * s.plane, device="cuda:0")
            uc = torch.zeros(4 * s.plane, device="cuda:0")
            ins, outs_ = [u0, ua, ub, ua, ub], [ua, ub, ua, ub, uc]
            for k in range(5):
                api.fcsd_stage(s, k, u0, ins[k], acc, outs_[k], metric, mud, ref, G, dtd)
            outs[sched] = (H(uc), H(acc))
        assert s.stage_errors() == 0
        say(case, layout, tiles, "max |split - fused|", float(np.abs(outs[0][0] - outs[1][0]).max()),
            "max |split - persistent|", float(np.abs(outs[0][0] - outs[2][0]).max()))
        for sched in SCHEDULES[1:]:
            assert np.array_equal(outs[sched][0], outs[0][0])
            assert np.array_equal(outs[sched][1], outs[0][1])
        if first is None:
            first = outs[0]
        else:
            assert np.array_equal(outs[0][0], first[0]) and np.array_equal(outs[0][1], first[1])
    assert np.all(np.isfinite(outs[0][0]))
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_reverse_q2_pass_schedules_agree(env, layout):
    """The viscous right-hand side's reverse mode with its q2 pass fused with
    the q2 transpose (on tiles of all four components) agrees with the split
    one (the pass, then fc_diff_adj) to FP32 rounding -- the transposes'
    tail folds sum over a tile-dependent number of lanes, so the two are not
    bit-identical: u_bar and mu_bar within 1e-6 of their largest value, on
    the uneven patches and the annulus."""
    api, ctx, torch = env
    for case in ("uneven", "annulus"):
        ps, u, mu, ref = rhs_case(case)
        s, D, H = mkset(api, ctx, ps, layout)
        rng = np.random.default_rng(31)
        rb = D(rng.standard_normal((4, ps.plane)).astype(np.float32))
        outs = []
        for sched in (0, 1):
            s.set_schedule(sched)
            ub = torch.zeros(4 * s.plane, device="cuda:0")
            mub = torch.zeros(s.plane, device="cuda:0")
            api.fcsd_rhs_adj(s, D(u), D(ps.metric), D(mu), ref, G, rb, ub, mub)
            outs.append((H(ub), H(mub)))
        du = np.abs(outs[0][0] - outs[1][0]).max() / np.abs(outs[0][0]).max()
        dm = np.abs(outs[0][1] - outs[1][1]).max() / np.abs(outs[0][1]).max()
        say("reverse q2 split vs fused", case, layout, "u_bar", du, "mu_bar", dm)
        assert du <= 1e-6 and dm <= 1e-6
        s.close()


def test_persistent_schedule_steps_with_network(env):
    """Five full steps of the 16-sector annulus (network, viscosity, step
    size, glue and inflow every stage, graph replay) give bit-identical
    states with the split, persistent and wide fused schedules."""
    api, ctx, torch = env
    cfg = synth.config(1, n=48)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, 1)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    res = []
    for sched in (0, 2, 3):
        s.set_schedule(sched)
        u = D(cfg.u0)
        st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W, dirichlet_mask=D(ps.dirichlet),
                         dirichlet_state=synth.freestream(cfg.mach))
        for k in range(5):
            st.step(use_graph=(k > 0))
        res.append(H(u))
    assert s.stage_errors() == 0
    assert np.all(np.isfinite(res[0])) and all(np.array_equal(res[0], r) for r in res[1:])
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_schedules_give_identical_steps_and_records(env, layout):
    """Uneven independent patches: five steps with the network (graph
    replay), the last one recorded, give states and step records
    bit-identical under the split, fused, persistent and wide fused
    schedules."""
    api, ctx, torch = env
    cfg = synth.config(2, npatch=8, nmax=136, seed=31)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    res, recs = [], []
    for sched in (0, 1, 2, 3):
        s.set_schedule(sched)
        u = D(cfg.u0)
        st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W)
        for k in range(4):
            st.step(use_graph=(k > 0))
        rec = st.new_record().zero_()
        st.step(record=rec)
        res.append(H(u))
        recs.append(rec.cpu().numpy())
    assert s.stage_errors() == 0
    say("schedules, uneven set, layout", layout, "change", float(np.abs(res[0] - H(D(cfg.u0))).max()))
    assert np.all(np.isfinite(res[0]))
    assert all(np.array_equal(res[0], r) for r in res[1:])
    assert all(np.array_equal(recs[0], r) for r in recs[1:])
    s.close()


def test_ten_steps_square(env):
    api, ctx, torch = env
    cfg = synth.config(0)
    ps = cfg.ps
    s = api.PatchSet.from_layout(ctx, ps)
    u = dev(torch, cfg.u0)
    mu = dev(torch, np.full(ps.plane, 1e-3, np.float32))
    st = api.Stepper(s, u, dev(torch, ps.metric), cfg.ref, mu=mu)
    run = solver.Run(cfg)
    for k in range(cfg.steps):
        st.step(use_graph=(k > 0))
        run.step()
    got = host(u).reshape(4, -1)
    err = relerr_phys(ps, got, run.u)
    dev_ = relerr_phys(ps, got - cfg.u0, run.u - cfg.u0)
    say("10 steps square64: state", err, "change", dev_)
    assert np.all(err < STEP_TOL) and np.all(dev_ < 10 * STEP_TOL)
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_steps_annulus_with_network(env, layout):
    api, ctx, torch = env
    cfg = synth.config(1, n=48)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    u = D(cfg.u0)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W, dirichlet_mask=D(ps.dirichlet),
                     dirichlet_state=synth.freestream(cfg.mach))
    run = solver.Run(cfg)
    for k in range(3):
        u_in = first_step_input(api, s, D, ps, u, cfg) if k == 0 else None
        st.step()
        if k == 0:
            decision_check(ps, u_in, cfg.mlp, H(st.tau), H(st.argmax), label="annulus first step")
        run.step(tau=H(st.tau), arg=H(st.argmax))
        say("step", k, "layout", layout, "dt", float(host(st.dt)[0]), run.log[-1]["dt"])
    got = H(u).reshape(4, -1)
    err = relerr_phys(ps, got, run.u)
    chg = relerr_phys(ps, got - cfg.u0, run.u - cfg.u0)
    say("3 steps annulus: state rel L2", err, "change", chg)
    assert np.all(err < STEP_TOL)
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_steps_paper_subpatches(env, layout):
    """Three steps with the network on the paper's discretisation (16
    subpatches of 101 x 101, d = 2, C = 27, fringe glue between them)."""
    api, ctx, torch = env
    cfg = synth.paper_subpatches(16, 1)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    u = D(cfg.u0)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W, dirichlet_mask=D(ps.dirichlet),
                     dirichlet_state=synth.freestream(cfg.mach))
    run = solver.Run(cfg)
    for k in range(3):
        u_in = first_step_input(api, s, D, ps, u, cfg) if k == 0 else None
        st.step()
        if k == 0:
            decision_check(ps, u_in, cfg.mlp, H(st.tau), H(st.argmax), label="paper subpatches first step")
        run.step(tau=H(st.tau), arg=H(st.argmax))
        say("paper subpatches step", k, "layout", layout, "dt", float(host(st.dt)[0]), run.log[-1]["dt"])
    err = relerr_phys(ps, H(u).reshape(4, -1), run.u)
    say("3 steps paper subpatches: state rel L2", err)
    assert np.all(err < STEP_TOL)
    s.close()


# ------------------------------------------------------------------ inter-patch interpolation

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("geometry", ["pair", "stype"])
def test_interpolated_fringe(env, layout, geometry):
    """fcsd_set_interp + fcsd_glue against the oracle's interpolation on the
    Cartesian / polar pair and on the S-type / affine trio of the paper's
    patch kinds (Sec. 3.4.1; S-type donors through Newton preimages): the
    same receivers, and fringe values within FP32 rounding of the weights
    (relative 1e-6 of the field scale); every other point untouched."""
    from oracle import interp
    api, ctx, torch = env
    cfg = synth.overlap_config(48, stype=geometry == "stype")
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    n = s.set_interp(ps.geom)
    table = interp.build(ps)
    say("interpolated fringe layout", layout, "receivers", n, "oracle", len(table))
    assert n == len(table)
    x = cfg.u0.astype(np.float32)
    xd = D(x)
    api.fcsd_glue(s, xd)
    got = H(xd).reshape(4, -1)
    want = interp.interpolate(x.astype(np.float64).copy(), ps, table)
    # per component; rho v is zero in this flow, so its scale is the momentum's
    scale = np.abs(want).max(axis=1)
    scale[2] = max(scale[1], scale[2])
    err = np.abs(got - want).max(axis=1) / scale
    say("  fringe max rel error", err)
    assert np.all(err <= 1e-6)
    mask = np.zeros(ps.plane, bool)
    for (p, i, j, *_r) in table:
        ps.view(mask, p)[j, i] = True
    for p in range(ps.npatch):
        a, b, m = ps.view(got, p), ps.view(x, p), ps.view(mask, p)
        assert np.array_equal(a[:, ~m], b[:, ~m])
    s.close()


@pytest.mark.parametrize("geometry", ["pair", "stype"])
@pytest.mark.parametrize("network", [False, True])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_steps_interpolated_patches(env, layout, network, geometry):
    """Five steps on the non-aligned pair (and on the S-type / affine trio)
    with the fringe interpolated at every stage, constant viscosity or the
    network's (smoothed across the patches), against the oracle (state <=
    1e-4).  With the network the oracle replays the GPU's decisions
    (classes, maximisers, step sizes), whose first step must agree with the
    oracle's FP64 decisions wherever their margin exceeds the FP32 bound."""
    api, ctx, torch = env
    cfg = synth.overlap_config(48, network=network, stype=geometry == "stype")
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    s.set_interp(ps.geom)
    u = D(cfg.u0)
    if network:
        W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
        st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W)
    else:
        st = api.Stepper(s, u, D(ps.metric), cfg.ref, mu=D(np.full(ps.plane, cfg.mu_const, np.float32)))
    run = solver.Run(cfg)
    for k in range(5):
        u_in = first_step_input(api, s, D, ps, u, cfg) if (network and k == 0) else None
        st.step(use_graph=(k > 0))
        if not network:
            run.step()
            continue
        if k == 0:
            decision_check(ps, u_in, cfg.mlp, H(st.tau), H(st.argmax), label="interpolated pair first step")
        run.step(dt=float(host(st.dt)[0]), tau=H(st.tau), arg=H(st.argmax))
    got = H(u).reshape(4, -1)
    err = relerr_phys(ps, got, run.u)
    chg = relerr_phys(ps, got - cfg.u0, run.u - cfg.u0)
    floor = change_floor(ps, run.u, cfg.u0, 5)
    say("5 steps interpolated", geometry, "layout", layout, "state rel L2", err, "change", chg, "floor", floor)
    # the change over five steps is ~1e-5 of the state: its FP32 floor (the
    # stored state's rounding) is a few per cent of it
    assert np.all(err < STEP_TOL) and np.all(chg[[0, 1, 3]] < np.maximum(1e-2, 8 * floor[[0, 1, 3]]))
    s.close()


def test_interpolation_refuses_bad_decompositions(env):
    api, ctx, torch = env
    ps = synth.overlap_pair(48)
    s = api.PatchSet.from_layout(ctx, ps)
    geom = ps.geom.copy()
    geom[0, 1] -= 0.3                 # the Cartesian patch moved left: its fringe now meets the sector's
    with pytest.raises(api.FcsdError):
        s.set_interp(geom)
    with pytest.raises(api.FcsdError):
        s.set_interp(ps.geom, nf=40)   # fringe wider than the patches allow
    s.close()


@pytest.mark.parametrize("geometry", ["pair", "stype"])
def test_interpolated_glue_and_step_reverse_mode(env, geometry):
    """Transposes on the interpolated pair (and the S-type / affine trio):
    fcsd_glue_adj against the oracle's (dot-product exact up to FP32
    accumulation), and one network step's reverse mode against the oracle's
    step VJP at the GPU's decisions (relative L2 per component <= 1e-4)."""
    from oracle import adjoint, interp
    api, ctx, torch = env
    cfg = synth.overlap_config(48, network=True, stype=geometry == "stype")
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, 1)
    s.set_interp(ps.geom)
    rng = np.random.default_rng(21)
    y = rng.standard_normal((4, ps.plane)).astype(np.float32)
    yd = D(y)
    api.fcsd_glue_adj(s, yd)
    want = y.astype(np.float64).copy()
    adjoint.glue_vjp(want, ps, cfg.mach)
    gerr = relerr_phys(ps, H(yd).reshape(4, -1), want)
    say("interpolated glue transpose rel L2", gerr)
    assert np.all(gerr < 1e-6)
    # one step and its reverse mode
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    u = D(cfg.u0)
    st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W)
    u_in = u.clone()
    st.step()
    tau, dt, arg = st.tau.clone(), st.dt.clone(), H(st.argmax)
    w = rng.standard_normal((4, ps.plane)).astype(np.float32)
    ub = D(w)
    st.step_adj(u_in, ub, tau, dt)
    run = solver.Run(cfg)
    run.u = H(u_in).reshape(4, -1).astype(np.float64)
    run.step(dt=float(host(dt)[0]), tau=H(tau), arg=arg, record=True)
    want, _ = adjoint.step_vjp(run, run.log[-1], w.astype(np.float64))
    err = relerr_phys(ps, H(ub).reshape(4, -1), want)
    say("interpolated pair step reverse mode rel L2", err)
    assert np.all(err < 1e-4)
    s.close()


# ------------------------------------------------------------------ walls

def test_wall_condition(env):
    """fcsd_set_walls + fcsd_glue (with the fringe copies and the Dirichlet
    inflow) against the oracle's glue on the annulus with its inner circle
    a wall: momenta zero there, E from the Neumann temperature (relative
    1e-6)."""
    from oracle import wall
    api, ctx, torch = env
    cfg = synth.with_cylinder_wall(synth.config(1, n=48))
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, 1)
    s.set_walls(ps.wall, G)
    x = noisy_state(ps, cfg.u0, 8, amp=1e-2)
    xd = D(x)
    api.fcsd_glue(s, xd, D(ps.dirichlet), synth.freestream(cfg.mach))
    got = H(xd).reshape(4, -1)
    want = x.astype(np.float64).copy()
    solver.glue(want, ps, cfg.mach, G)
    # rho v is zero in this flow: its error is taken against the momentum's scale
    scale = np.abs(want).max(axis=1)
    scale[2] = scale[1]
    err = np.abs(got - want).max(axis=1) / scale
    say("wall glue max rel error", err)
    assert np.all(err <= 1e-6)
    for p in range(ps.npatch):
        if ps.wall[p, 2]:
            assert np.all(ps.view(got, p)[1:3, 0] == 0)
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_steps_with_cylinder_wall(env, layout):
    """Three network steps on the annulus with the no-slip adiabatic
    cylinder wall, fringe copies and the Dirichlet inflow, against the
    oracle replaying the GPU's decisions (state <= 1e-4)."""
    api, ctx, torch = env
    cfg = synth.with_cylinder_wall(synth.config(1, n=48))
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    s.set_walls(ps.wall, G)
    u = D(cfg.u0)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W, dirichlet_mask=D(ps.dirichlet),
                     dirichlet_state=synth.freestream(cfg.mach))
    run = solver.Run(cfg)
    for k in range(3):
        st.step(use_graph=(k > 0))
        run.step(dt=float(host(st.dt)[0]), tau=H(st.tau), arg=H(st.argmax))
    err = relerr_phys(ps, H(u).reshape(4, -1), run.u)
    say("3 steps with the cylinder wall layout", layout, "state rel L2", err)
    assert np.all(err < STEP_TOL)
    with pytest.raises(api.FcsdError):
        api.fcsd_glue_adj(s, torch.zeros_like(u))      # no state: refused with walls
    s.close()


@pytest.mark.parametrize("flags", [(1, 1, 1, 1), (1, 0, 1, 0), (0, 1, 1, 1)])
def test_corner_walls_glue_and_transpose(env, flags):
    """Walls that meet at patch corners (the corner's theta from the tensor
    product of the two one-sided Neumann values): fcsd_glue against the
    oracle's wall condition, and fcsd_glue_adj at the glued state against
    the oracle's transpose."""
    import dataclasses
    from oracle import adjoint
    api, ctx, torch = env
    ps = dataclasses.replace(synth.unit_square(37), wall=np.array([flags], np.uint8))   # L = 64
    s, D, H = mkset(api, ctx, ps, 1)
    s.set_walls(ps.wall, G)
    rng = np.random.default_rng(41)
    x = noisy_state(ps, smooth_state(ps), 42, amp=1e-2)
    xd = D(x)
    api.fcsd_glue(s, xd)
    got = H(xd).reshape(4, -1)
    want = x.astype(np.float64).copy()
    solver.glue(want, ps, 3.0, G)
    err = np.abs(got - want).max(axis=1) / np.abs(want).max(axis=1)
    y = rng.standard_normal((4, ps.plane)).astype(np.float32)
    yd = D(y)
    api.fcsd_glue_adj(s, yd, glued=xd)
    wb = y.astype(np.float64).copy()
    adjoint.glue_vjp(wb, ps, 3.0, G, e_glued=got.astype(np.float64))
    eb = relerr_phys(ps, H(yd).reshape(4, -1), wb)
    say("corner walls", flags, "glue max rel", err, "transpose rel L2", eb)
    # a corner's theta sums (d-1)^2 FP32 temperatures with weights of total
    # size sum |c_k c_l| = 17 (d = 5): a few 1e-6 of the field there
    assert np.all(err <= 1e-5) and np.all(eb <= 1e-6)
    with pytest.raises(api.FcsdError):
        api.fcsd_glue_adj(s, yd)                        # walls need the glued state
    s.close()


def smooth_state(ps):
    """A smooth admissible state on any patch set (rho ~ 1, p ~ 1, |u| ~ 0.3)."""
    x, y = ps.xy
    rho = 1.0 + 0.1 * np.sin(2 * x + 1) * np.cos(3 * y)
    u = 0.3 + 0.1 * np.cos(x - 2 * y)
    v = -0.2 + 0.1 * np.sin(3 * x + y)
    p = 1.0 + 0.1 * np.cos(2 * x) * np.sin(y + 0.5)
    e = np.stack([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])
    out = np.zeros((4, ps.plane), np.float32)
    for q in range(ps.npatch):
        ps.view(out, q)[...] = ps.view(e, q)
    return out


def wall_layer_state(ps, r0, dr):
    """smooth_state with a velocity layer two cells thick at the circle r = r0
    (the velocity falls to zero there): under-resolved enough that the
    energy's product rule differs from the plain FC derivative far beyond
    FP32 rounding, at a low Mach number where the energy lane is well
    conditioned."""
    x, y = ps.xy
    layer = 1.0 - np.exp(-(np.hypot(x, y) - r0) / (2.0 * dr))
    rho = 1.0 + 0.1 * np.sin(2 * x + 1) * np.cos(3 * y)
    u = (0.3 + 0.1 * np.cos(x - 2 * y)) * layer
    v = (-0.2 + 0.1 * np.sin(3 * x + y)) * layer
    p = 1.0 + 0.1 * np.cos(2 * x) * np.sin(y + 0.5)
    e = np.stack([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])
    out = np.zeros((4, ps.plane), np.float32)
    for q in range(ps.npatch):
        ps.view(out, q)[...] = ps.view(e, q)
    return out


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rhs_with_wall_patches(env, layout):
    """The full right-hand side and its reverse mode on the annulus whose
    inner circle is a wall: on the wall patches the energy's derivatives
    come from the product rule over theta's FC derivatives (Remark
    adiabatic).  Against the oracle at the RHS / reverse bars, on a state
    with a thin velocity layer at the wall, where the rule changes the
    result by far more than the error."""
    api, ctx, torch = env
    cfg = synth.with_cylinder_wall(synth.config(1, n=48))
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    s.set_walls(ps.wall, G)
    wall_r = min(np.hypot(*[ps.view(c, q) for c in ps.xy]).min() for q in range(ps.npatch) if ps.wall[q].any())
    x32 = wall_layer_state(ps, wall_r, 1.5 / 47)          # the annulus' radial spacing: 1.5 over 47 cells
    ref = (1.0, 0.3, -0.2, 1.0)
    mu = (0.004 * (1.2 + np.sin(3 * ps.xy[0]) * np.cos(2 * ps.xy[1]))).astype(np.float32)
    rhs = torch.zeros(4 * s.plane, device="cuda:0")
    api.fcsd_rhs(s, D(x32), D(ps.metric), D(mu), ref, G, rhs)
    want = euler.full_rhs(x32.astype(np.float64), ps.metric, mu.astype(np.float64), ps, G)
    err = relerr_phys(ps, H(rhs), want)
    mx = maxrel_phys(ps, H(rhs), want)
    import dataclasses
    plain = euler.full_rhs(x32.astype(np.float64), ps.metric, mu.astype(np.float64),
                           dataclasses.replace(ps, wall=None), G)
    effect = relerr_phys(ps, plain, want)
    # the layer makes the lanes ill conditioned: the bar per lane is the
    # larger of the RHS bar and the exact result's response to FP32 rounding
    # of the input (a relative 2^-24 perturbation, seeded)
    rng = np.random.default_rng(45)
    xp = x32.astype(np.float64) * (1 + 2.0 ** -24 * rng.choice((-1.0, 1.0), x32.shape))
    sens = relerr_phys(ps, euler.full_rhs(xp, ps.metric, mu.astype(np.float64), ps, G), want)
    bar = np.maximum(RHS_TOL, sens)
    rb = smooth_fields(ps, 4, 44)
    ub = torch.zeros(4 * s.plane, device="cuda:0")
    mb = torch.zeros(s.plane, device="cuda:0")
    api.fcsd_rhs_adj(s, D(x32), D(ps.metric), D(mu), ref, G, D(rb), ub, mb)
    we, wm = euler.full_rhs_vjp(x32.astype(np.float64), ps.metric, mu.astype(np.float64), ps, G,
                                rb.astype(np.float64))
    e1, e2 = relerr_phys(ps, H(ub), we), relerr(ps, H(mb), wm)
    say("rhs with wall patches layout", layout, "rel L2", err, "max", mx, "bar", bar, "rule's effect", effect,
        "| reverse", e1, e2)
    assert np.all(err < bar) and np.all(mx < PT * bar)
    assert effect[3] > 20 * err[3]
    assert np.all(e1 < ADJ_TOL) and e2[0] < ADJ_TOL
    s.close()


def test_step_reverse_mode_with_cylinder_wall(env):
    """One network step's reverse mode with the cylinder wall against the
    oracle's step VJP at the GPU's decisions (relative L2 <= 1e-4)."""
    from oracle import adjoint
    api, ctx, torch = env
    cfg = synth.with_cylinder_wall(synth.config(1, n=48))
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, 1)
    s.set_walls(ps.wall, G)
    u = D(cfg.u0)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W, dirichlet_mask=D(ps.dirichlet),
                     dirichlet_state=synth.freestream(cfg.mach))
    st.step()                       # a state that has met the wall once
    u_in = u.clone()
    st.step()
    tau, dt, arg = st.tau.clone(), st.dt.clone(), H(st.argmax)
    rng = np.random.default_rng(23)
    w = rng.standard_normal((4, ps.plane)).astype(np.float32)
    ub = D(w)
    dpar = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    st.step_adj(u_in, ub, tau, dt, (0.0, 1.4, 0.0, 1.4 * cfg.mach), dpar)
    run = solver.Run(cfg)
    run.u = H(u_in).reshape(4, -1).astype(np.float64)
    run.step(dt=float(host(dt)[0]), tau=H(tau), arg=arg, record=True)
    want, dM = adjoint.step_vjp(run, run.log[-1], w.astype(np.float64))
    err = relerr_phys(ps, H(ub).reshape(4, -1), want)
    say("step reverse mode with the cylinder wall rel L2", err, "dM gpu", float(dpar), "oracle", dM)
    assert np.all(err < 1e-4)
    assert abs(float(dpar) - dM) <= 1e-4 * abs(dM)
    s.close()


# ------------------------------------------------------------------ adjoints

@pytest.mark.parametrize("case", ["square64", "shells"])
def test_rhs_reverse_mode(env, case):
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case(case)
    s = api.PatchSet.from_layout(ctx, ps)
    rng = np.random.default_rng(17)
    rb = smooth_fields(ps, 4, 18)
    ub = torch.zeros(4 * ps.plane, device="cuda:0")
    mb = torch.zeros(ps.plane, device="cuda:0")
    api.fcsd_rhs_adj(s, dev(torch, u), dev(torch, ps.metric), dev(torch, mu), ref, G, dev(torch, rb), ub, mb)
    we, wm = euler.full_rhs_vjp(u.astype(np.float64), ps.metric, mu.astype(np.float64), ps, G,
                                rb.astype(np.float64))
    e1 = relerr_phys(ps, host(ub), we)
    e2 = relerr(ps, host(mb), wm)
    m1 = maxrel_phys(ps, host(ub), we)
    m2 = maxrel_phys(ps, host(mb), wm)
    say("rhs adjoint", case, e1, e2, "max", m1, m2)
    assert np.all(e1 < ADJ_TOL) and e2[0] < ADJ_TOL
    assert np.all(m1 < PT * ADJ_TOL) and m2[0] < PT * ADJ_TOL
    s.close()


@pytest.mark.parametrize("case", ["square64", "shells"])
def test_euler_rhs_and_av_apply_reverse_modes(env, case):
    """euler_rhs_adj (inviscid right-hand side transposed) and av_apply_adj
    (the viscous term alone, with its viscosity cotangent) against the
    oracle's vector-Jacobian products, accumulating into nonzero buffers."""
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case(case)
    s = api.PatchSet.from_layout(ctx, ps)
    rb = smooth_fields(ps, 4, 31)
    base = smooth_fields(ps, 4, 32)
    ub = dev(torch, base)
    api.euler_rhs_adj(s, dev(torch, u), dev(torch, ps.metric), ref, G, dev(torch, rb), ub)
    we, _ = euler.full_rhs_vjp(u.astype(np.float64), ps.metric, None, ps, G, rb.astype(np.float64))
    got = host(ub).reshape(4, -1) - base
    e1, m1 = relerr_phys(ps, got, we), maxrel_phys(ps, got, we)
    ub = dev(torch, base)
    mb0 = smooth_fields(ps, 1, 33)[0]
    mb = dev(torch, mb0)
    api.av_apply_adj(s, dev(torch, u), dev(torch, ps.metric), dev(torch, mu), ref, dev(torch, rb), ub, mb)
    wa, wm = euler.av_term_vjp(u.astype(np.float64), ps.metric, mu.astype(np.float64), ps, rb.astype(np.float64))
    ga = host(ub).reshape(4, -1) - base
    gm = host(mb) - mb0
    e2, m2 = relerr(ps, ga, wa), maxrel_phys(ps, ga, wa)
    e3, m3 = relerr(ps, gm, wm), maxrel_phys(ps, gm, wm)
    say("euler_rhs_adj", case, e1, "max", m1, "| av_apply_adj", e2, "max", m2, "mu_bar", e3, m3)
    assert np.all(e1 < ADJ_TOL) and np.all(m1 < PT * ADJ_TOL)
    assert np.all(e2 < ADJ_TOL) and np.all(m2 < PT * ADJ_TOL)
    assert e3[0] < ADJ_TOL and m3[0] < PT * ADJ_TOL
    s.close()


@pytest.mark.parametrize("stage", [1, 4])
def test_stage_reverse_mode(env, stage):
    """fcsd_stage_adj against the oracle: stage 1 maps (u0, u1) to
    u2 = a10 u0 + a11 u1 + b11 dt L(u1), stage 4 maps (acc, u4) to
    acc + a44 u4 + b44 dt L(u4) (Shu-Osher coefficients of the oracle's
    scheme; acc holds the earlier terms of the last stage), so the
    cotangents are u0_bar += a10 y, acc_bar += y, ui_bar += a y +
    L'(ui)^T (b dt y), mu_bar += the viscosity part."""
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case("uneven")
    s = api.PatchSet.from_layout(ctx, ps)
    ui = (u * (1 + 1e-3 * smooth_fields(ps, 4, 34))).astype(np.float32)     # a smooth stage input
    y = smooth_fields(ps, 4, 35)
    dt = 2e-3
    dtd = dev(torch, np.array([dt], np.float32))
    b0 = smooth_fields(ps, 4, 36)
    u0b, uib, accb = dev(torch, b0), dev(torch, b0 * 0.5), dev(torch, b0 * 0.25)
    mb = torch.zeros(ps.plane, device="cuda:0")
    api.fcsd_stage_adj(s, stage, dev(torch, ui), dev(torch, ps.metric), dev(torch, mu), ref, G, dtd, dev(torch, y),
                       u0b, uib, accb, mb)
    a, b = rk.ALPHA[stage][stage], rk.BETA[stage][stage]
    re, rm = euler.full_rhs_vjp(ui.astype(np.float64), ps.metric, mu.astype(np.float64), ps, G,
                                b * float(np.float32(dt)) * y.astype(np.float64))
    want_ui = 0.5 * b0 + a * y + re
    err_ui = relerr_phys(ps, host(uib).reshape(4, -1), want_ui)
    mx_ui = maxrel_phys(ps, host(uib).reshape(4, -1), want_ui)
    err_mu = relerr(ps, host(mb), rm)
    if stage == 1:
        want_0 = b0 + rk.ALPHA[1][0] * y
        other = relerr_phys(ps, host(u0b).reshape(4, -1), want_0)
        assert np.array_equal(host(accb), (b0 * 0.25).reshape(-1))
    else:
        want_acc = 0.25 * b0 + y
        other = relerr_phys(ps, host(accb).reshape(4, -1), want_acc)
        assert np.array_equal(host(u0b), b0.reshape(-1))
    say("stage", stage, "reverse: ui_bar", err_ui, "max", mx_ui, "mu_bar", err_mu, "u0/acc", other)
    assert np.all(err_ui < ADJ_TOL) and np.all(mx_ui < PT * ADJ_TOL) and err_mu[0] < ADJ_TOL
    assert np.all(other < 1e-6)
    s.close()


def test_network_reverse_mode(env):
    """sdnn_infer_adj (the network's transpose at the state's window
    features) against the oracle's mlp_vjp on the 64 x 64 square, whose
    features are well conditioned.  Compared at the windows whose ReLU masks
    are the same in FP32 and FP64 for certain (every unit's input beyond
    twice its FP32 error bound); the count of the others is printed."""
    api, ctx, torch = env
    cfg = synth.config(0)
    ps = cfg.ps
    W = synth.mlp_weights(5)
    s = api.PatchSet.from_layout(ctx, ps)
    Wd = {k: dev(torch, v) for k, v in W.items()}
    rng = np.random.default_rng(37)
    lb = rng.standard_normal((2, ps.plane, 4)).astype(np.float32)
    fb = torch.full((32 * ps.plane,), 7.0, device="cuda:0")
    api.sdnn_infer_adj(s, dev(torch, cfg.u0), G, Wd, dev(torch, lb), fb)
    got = host(fb).reshape(2, ps.plane, 16)
    A = {k: np.abs(np.asarray(v, np.float64)) for k, v in W.items()}
    Wf = {k: np.asarray(v, np.float64) for k, v in W.items()}
    e = np.asarray(cfg.u0, np.float64)
    comp = excl = 0
    errs, wants, scale = [], [], 0.0
    for p in range(ps.npatch):
        ep = ps.view(e, p)
        phi = av.proxy(ep, G)
        eps = fp32_value_bound(ep) * np.abs(phi)
        o, a_, b_ = int(ps.off[p]), int(ps.n1[p]), int(ps.n2[p])
        for d in range(2):
            if d == 0:
                x = av.features_lines(phi)
                dx = _window_dx_bound(phi, eps)
            else:
                x = np.swapaxes(av.features_lines(phi.T), 0, 1)
                dx = np.swapaxes(_window_dx_bound(phi.T, eps.T), 0, 1)
            want = av.mlp_vjp(x, W, lb[d, o:o + a_ * b_].reshape(b_, a_, 4).astype(np.float64))
            z1 = x @ Wf["W1"] + Wf["b1"]
            d1 = dx[..., None] * A["W1"].sum(0) + 32 * U32 * (np.abs(x) @ A["W1"] + A["b1"])
            h1 = np.maximum(z1, 0)
            z2 = h1 @ Wf["W2"] + Wf["b2"]
            d2 = np.where(z1 > -d1, d1, 0) @ A["W2"] + 128 * U32 * (h1 @ A["W2"] + A["b2"])
            sure = np.all(np.abs(z1) > 2 * d1, -1) & np.all(np.abs(z2) > 2 * d2, -1)
            sure &= np.isfinite(dx)
            g = got[d, o:o + a_ * b_].reshape(b_, a_, 16)
            errs.append((g - want)[sure])
            wants.append(want[sure])
            scale = max(scale, np.abs(want).max())
            comp += int(sure.sum())
            excl += int((~sure).sum())
    err = np.concatenate(errs)
    rel = np.linalg.norm(err) / np.linalg.norm(np.concatenate(wants))
    say("network reverse mode: compared", comp, "uncertain masks", excl, "rel L2", rel,
        "max", np.abs(err).max() / scale)
    assert comp > 0.9 * (comp + excl)
    assert rel < 1e-5 and np.abs(err).max() <= 1e-4 * scale
    s.close()


@pytest.mark.parametrize("case", ["annulus", "overlap"])
def test_viscosity_reverse_mode(env, case):
    api, ctx, torch = env
    cfg = synth.config(1, n=40) if case == "annulus" else synth.overlap_config(48, network=True)
    ps = cfg.ps
    e = cfg.u0.astype(np.float64)
    mu, tau, arg = av.viscosity(e, ps, cfg.mlp, G)
    rng = np.random.default_rng(19)
    mb = rng.standard_normal(ps.plane).astype(np.float32)
    s = api.PatchSet.from_layout(ctx, ps)
    if ps.geom is not None:
        s.set_interp(ps.geom)
    ub = torch.zeros(4 * ps.plane, device="cuda:0")
    api.av_viscosity_adj(s, dev(torch, cfg.u0), dev(torch, tau.astype(np.int8)), dev(torch, arg.astype(np.int32)),
                         G, dev(torch, mb), ub)
    want = av.viscosity_vjp(e, tau, arg, ps, G, mb.astype(np.float64))
    err = relerr(ps, host(ub), want)
    say("viscosity adjoint", err)
    assert np.all(err < 1e-5)
    s.close()


# ------------------------------------------------------------------ schedules

@pytest.mark.parametrize("case", ["uneven", "overlap", "square64"])
def test_tiling_and_order_do_not_change_results(env, case):
    """Every line is transformed by the same arithmetic whatever its tile and
    launch slot: the right-hand side is bit-identical across LDS budgets and
    launch orders (with one or two patches the XCD order cuts each patch
    into runs of tiles on several dies)."""
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case(case)
    s = api.PatchSet.from_layout(ctx, ps)
    metric = dev(torch, ps.metric)
    ud, mud = dev(torch, u), dev(torch, mu)
    outs = []
    for budgets, threads, order in [((65536,) * 3, (256,) * 3, 1), ((16384, 131072, 98304), (256, 1024, 512), 0),
                                    ((32768, 24576, 163840), (512, 256, 1024), 1),
                                    ((98304, 16384, 49152), (1024, 128, 256), 0)]:
        say("tiling", budgets, threads, order)
        s.tune(budgets, threads, order)
        rhs = torch.zeros(4 * ps.plane, device="cuda:0")
        api.fcsd_rhs(s, ud, metric, mud, ref, G, rhs)
        outs.append(host(rhs))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    s.close()


def test_autotuner_picks_a_schedule(env):
    from paper_2506_16076_amd import autotune
    api, ctx, torch = env
    ps, u, mu, ref = rhs_case("uneven")
    s = api.PatchSet.from_layout(ctx, ps)
    metric = dev(torch, ps.metric)
    ud, mud = dev(torch, u), dev(torch, mu)
    res = autotune.autotune(s, ud, metric, mud, ref, G, budgets=(16384, 32768, 65536), threads=(256, 512), reps=1)
    say("autotune", {k: v for k, v in res.items() if k != "table"})
    assert all(b in (16384, 32768, 65536) for b in res["budgets"]) and all(t in (256, 512) for t in res["threads"])
    assert s.tuning == (tuple(res["budgets"]), tuple(res["threads"]), 1 if res["order"] == "xcd" else 0)
    rhs = torch.zeros(4 * ps.plane, device="cuda:0")
    api.fcsd_rhs(s, ud, metric, mud, ref, G, rhs)
    want = euler.full_rhs(u.astype(np.float64), ps.metric, mu.astype(np.float64), ps, G)
    assert np.all(relerr_phys(ps, host(rhs), want) < RHS_TOL)
    s.close()


# ------------------------------------------------------------------ time-stepping reverse mode

def _annulus_ic(torch, ps, pert, M, amp, s):
    """rho = 1.4 (1 + sum a_k phi_k), m = rho M, n = 0, E = 1/(gamma-1) + rho M^2/2 (FP64 on the
    device, differentiable in M and amp), returned as the FP32 state in the set's storage."""
    phi = s.to_device(pert.modes(ps.xy)).reshape(len(pert.amp), -1)
    rho = 1.4 * (1 + amp @ phi)
    e = torch.stack([rho, rho * M, 0 * rho, 1 / (G - 1) + 0.5 * rho * M * M])
    return e.to(torch.float32).reshape(-1)


def _rollout_gradient_check(env, n, steps, every, layout=0, filt=None):
    """Gradient of the outer-row density norm after `steps` steps
    (checkpoints every `every`) on the 16-sector annulus with n x n patches,
    with respect to the inflow Mach number and the 16 perturbation
    amplitudes, through torch.autograd and the hand-written step reverse
    mode, against the FP64 oracle's discrete adjoint with the same recorded
    decisions (classes, maximisers, step sizes).  Bar: relative L2 over the
    gradient vector <= 1e-4 and 1e-2 on the small Mach component plus the
    gradient's FP32 noise floor (FP32 forward and reverse sweeps over
    5 x steps stages)."""
    from paper_2506_16076_amd import autodiff
    from oracle import adjoint
    api, ctx, torch = env
    cfg = synth.config(3, n=n)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    if filt is not None:
        s.set_filter(*filt)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    metric = D(ps.metric)
    mask = D(ps.dirichlet)
    M = torch.tensor(cfg.mach, dtype=torch.float64, device="cuda:0", requires_grad=True)
    amp = torch.tensor(cfg.pert.amp, dtype=torch.float64, device="cuda:0", requires_grad=True)
    ubuf = torch.zeros(4 * s.plane, device="cuda:0")
    st = api.Stepper(s, ubuf, metric, cfg.ref, W=W, dirichlet_mask=mask,
                     dirichlet_state=synth.freestream(cfg.mach), filt=filt is not None)
    # recorded decisions of the forward run, for the oracle
    u0 = _annulus_ic(torch, ps, cfg.pert, M, amp, s)
    ubuf.copy_(u0.detach())
    rec = []
    for _ in range(steps):
        st.step()
        rec.append(dict(dt=float(host(st.dt)[0]), tau=H(st.tau).copy(), arg=H(st.argmax).copy()))
    say("rollout", steps, "steps, checkpoints every", every)
    uT = autodiff.rollout(st, u0, M.to(torch.float32), steps, every, autodiff.freestream_dmach(cfg.mach))
    rows = np.zeros(ps.plane, np.float32)
    for p in range(ps.npatch):
        ps.view(rows, p)[-1, :] = 1
    idx = torch.nonzero(D(rows) > 0).reshape(-1)
    loss = torch.sqrt(torch.sum(uT[idx].double() ** 2))
    loss.backward()
    g_gpu = np.concatenate([[float(M.grad)], host(amp.grad)])
    L, g_or, _ = adjoint.gradient(cfg, steps, replay=rec, filt=filt)
    err = np.linalg.norm(g_gpu - g_or) / np.linalg.norm(g_or)
    say("  loss gpu", float(loss), "oracle", L, "grad rel L2", err)
    say("  dL/dM gpu", g_gpu[0], "oracle", g_or[0])
    assert abs(float(loss) - L) <= 1e-5 * abs(L)
    assert err <= 1e-4
    # the Mach entry to 1 %, above the FP32 noise of the whole gradient (the
    # relative-L2 bar): with the filter dL/dM is ~2e-3 of the gradient norm
    assert abs(g_gpu[0] - g_or[0]) <= 1e-2 * abs(g_or[0]) + 1e-4 * np.linalg.norm(g_or)
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rollout_gradient_matches_oracle_adjoint(env, layout):
    # 10 steps with checkpoints every 4: a ragged last segment
    _rollout_gradient_check(env, 48, 10, 4, layout)


def test_rollout_gradient_with_filter(env):
    """The same with the per-step spectral filter (alpha 10, p 14) in every
    step, transposed by fcsd_step_adj."""
    _rollout_gradient_check(env, 48, 6, 4, 1, filt=(10.0, 14))


@pytest.mark.parametrize("filt", [None, (10.0, 14)])
def test_step_record_equals_recompute(env, filt):
    """A step that writes its record advances the state exactly as one that
    does not, and the reverse mode read from the record equals, bit for bit,
    the one that recomputes the step (network classes, Dirichlet glue, with
    and without the filter); the boundary-parameter derivative to FP64
    rounding."""
    api, ctx, torch = env
    cfg = synth.config(3, n=48)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, 1)
    if filt is not None:
        s.set_filter(*filt)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    ubuf = D(cfg.u0)
    st = api.Stepper(s, ubuf, D(ps.metric), cfg.ref, W=W, dirichlet_mask=D(ps.dirichlet),
                     dirichlet_state=synth.freestream(cfg.mach), filt=filt is not None)
    st.step()                      # a state with shocks forming
    u_in = ubuf.clone()
    st.step()
    plain = ubuf.clone()
    tau, dt = st.tau.clone(), st.dt.clone()
    ubuf.copy_(u_in)
    rec = st.new_record()
    st.replay(tau, dt, record=rec)
    assert torch.equal(ubuf, plain)
    g = torch.randn(4 * s.plane, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(11))
    dstate = autodiff_dmach(cfg)
    b1, b2 = g.clone(), g.clone()
    p1 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    p2 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    st.step_adj(u_in, b1, tau, dt, dstate, p1)
    st.step_adj(None, b2, tau, dt, dstate, p2, record=rec)
    say("record vs recompute: max |diff|", float((b1 - b2).abs().max()), "dparam", float(p1), float(p2))
    assert torch.equal(b1, b2)
    # dparam is a sum of FP64 atomic adds: its rounding depends on their order
    assert abs(float(p1) - float(p2)) <= 1e-12 * abs(float(p1))
    assert float(b1.abs().max()) > 0 and float(p1.abs()) > 0
    s.close()


def autodiff_dmach(cfg):
    from paper_2506_16076_amd import autodiff
    return autodiff.freestream_dmach(cfg.mach)


@pytest.mark.timeout(900)
def test_rollout_gradient_full_size(env):
    """The differentiation workload at its stated size: 16 patches of
    128 x 128, 40 steps, checkpoints every 8 (a few minutes of FP64 oracle
    work on the host)."""
    _rollout_gradient_check(env, 128, 40, 8, 1)


# ------------------------------------------------------------------ full sizes, sampled patches

def _subset(ps, plist):
    """The oracle's view of a few patches of a layout (same planes)."""
    import dataclasses
    idx = np.asarray(plist)
    return dataclasses.replace(ps, n1=ps.n1[idx], n2=ps.n2[idx], C1=ps.C1[idx], C2=ps.C2[idx], off=ps.off[idx],
                               htilde=ps.htilde[idx], hhat=ps.hhat[idx], internal=ps.internal[idx],
                               nsec=0, nshell=0, dirichlet=None)


@pytest.mark.parametrize("idx", [1, 2, 4, "2-strict"])
def test_full_size_rhs_sampled_patches(env, idx):
    """The full right-hand side (convective + viscous) of the workloads at
    their stated sizes (c1 16 x 256^2, c2 200 uneven patches 48..512, c4
    64 x 512^2, and c2 with C = 27 on every line as the bench's strict-C
    field runs it), computed on the GPU for every patch in the configuration
    the bench uses (blocked storage, autotuned tiles and schedule), against
    the oracle on five sampled patches (first, last, largest, two seeded);
    bar 1e-5 per component."""
    from paper_2506_16076_amd import autotune
    api, ctx, torch = env
    strict = idx == "2-strict"
    idx = 2 if strict else idx
    cfg = synth.config(idx)
    if strict:
        import dataclasses
        cfg = dataclasses.replace(cfg, ps=synth.with_continuation(cfg.ps, 27))
    ps = cfg.ps
    say("full-size rhs", cfg.name, ps.npatch, "patches", ps.npoints, "points")
    s, D, H = mkset(api, ctx, ps, 1)
    metric = D(ps.metric)
    ud = D(cfg.u0)
    mu = (0.002 * (1.5 + np.sin(3 * ps.xy[0]) * np.cos(2 * ps.xy[1]))).astype(np.float32)
    mud = D(mu)
    res = autotune.autotune(s, ud, metric, mud, cfg.ref, G, reps=1)
    say("  schedule", {k: v for k, v in res.items() if k != "table"})
    rhs = torch.zeros(4 * s.plane, device="cuda:0")
    api.fcsd_rhs(s, ud, metric, mud, cfg.ref, G, rhs)
    got = H(rhs).reshape(4, -1)
    sizes = ps.n1.astype(np.int64) * ps.n2
    rng = np.random.default_rng(idx)
    plist = sorted({0, ps.npatch - 1, int(np.argmax(sizes)), *rng.choice(ps.npatch, 2, replace=False).tolist()})
    sub = _subset(ps, plist)
    want = euler.full_rhs(cfg.u0.astype(np.float64), ps.metric, mu.astype(np.float64), sub, G)
    err = relerr_phys(sub, got, want)
    mx = maxrel_phys(sub, got, want)
    say("  patches", plist, "rel L2", err, "max", mx)
    assert np.all(err < RHS_TOL) and np.all(mx < PT * RHS_TOL)
    s.close()


def test_interpolated_pair_at_bench_size(env):
    """The bench's interpolated pair (a Cartesian and a polar patch of
    1024 x 1024, blocked storage): the fringe table and interpolated values
    against the oracle's, and the full right-hand side of the glued state
    (viscous term with a smooth viscosity) against the oracle's (1e-5 per
    component)."""
    from oracle import interp
    api, ctx, torch = env
    cfg = synth.overlap_config(1024, network=True)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, 1)
    n = s.set_interp(ps.geom)
    table = interp.build(ps)
    say("interpolated pair 1024^2: receivers", n, "oracle", len(table))
    assert n == len(table)
    x = cfg.u0.astype(np.float32)
    xd = D(x)
    api.fcsd_glue(s, xd)
    got = H(xd).reshape(4, -1)
    want = interp.interpolate(x.astype(np.float64).copy(), ps, table)
    scale = np.abs(want).max(axis=1)
    scale[2] = max(scale[1], scale[2])
    ferr = np.abs(got - want).max(axis=1) / scale
    mu = (0.002 * (1.5 + np.sin(3 * ps.xy[0]) * np.cos(2 * ps.xy[1]))).astype(np.float32)
    rhs = torch.zeros(4 * s.plane, device="cuda:0")
    api.fcsd_rhs(s, xd, D(ps.metric), D(mu), cfg.ref, G, rhs)
    wr = euler.full_rhs(got.astype(np.float64), ps.metric, mu.astype(np.float64), ps, G)
    err, mx = relerr_phys(ps, H(rhs), wr), maxrel_phys(ps, H(rhs), wr)
    say("  fringe max rel", ferr, "rhs rel L2", err, "max", mx)
    assert np.all(ferr <= 1e-6)
    assert np.all(err < RHS_TOL) and np.all(mx < PT * RHS_TOL)
    s.close()


def change_floor(ps, u_end, u0, steps):
    """FP32 floor of the change of a state over `steps` SSPRK(5,4) steps,
    relative to that change, per conserved component: every stage stores
    the state in FP32 (rounding <= u32 |u| per point), so over 5 steps
    stages the stored state carries ~sqrt(5 steps) u32 ||u|| of rounding
    however exact the arithmetic, against a change ||u_end - u0|| (the
    momentum components on their common scale, as in relerr_phys)."""
    u_end = np.asarray(u_end, np.float64).reshape(4, -1)
    u0 = np.asarray(u0, np.float64).reshape(4, -1)

    def flat(a, f):
        return np.concatenate([ps.view(a[f], p).ravel() for p in range(ps.npatch)])
    nu = [np.linalg.norm(flat(u_end, f)) for f in range(4)]
    nd = [np.linalg.norm(flat(u_end - u0, f)) for f in range(4)]
    mu_, md_ = np.hypot(nu[1], nu[2]), np.hypot(nd[1], nd[2])
    nu = np.array([nu[0], mu_, mu_, nu[3]])
    nd = np.array([nd[0], md_, md_, nd[3]])
    return np.sqrt(5.0 * steps) * U32 * nu / np.maximum(nd, 1e-300)


def _replayed_steps(env, cfg, steps, label):
    """`steps` GPU steps of an annulus configuration, its first step's
    decisions checked against the oracle's FP64 ones, then every step
    replayed in the oracle with the GPU's decisions (classes, maximisers,
    step sizes).  Returns (state error, change error, change floor, max
    error)."""
    api, ctx, torch = env
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, 1)
    u = D(cfg.u0)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W, dirichlet_mask=D(ps.dirichlet),
                     dirichlet_state=synth.freestream(cfg.mach))
    run = solver.Run(cfg)
    for k in range(steps):
        u_in = first_step_input(api, s, D, ps, u, cfg) if k == 0 else None
        st.step(use_graph=(k > 0))
        if k == 0:
            decision_check(ps, u_in, cfg.mlp, H(st.tau), H(st.argmax), label=label + " first step")
        run.step(dt=float(host(st.dt)[0]), tau=H(st.tau), arg=H(st.argmax))
        if k % 10 == 9:
            say("  step", k + 1)
    got = H(u).reshape(4, -1)
    assert np.all(np.isfinite(got))
    err = relerr_phys(ps, got, run.u)
    chg = relerr_phys(ps, got - cfg.u0, run.u - cfg.u0)
    floor = change_floor(ps, run.u, cfg.u0, steps)
    mx = maxrel_phys(ps, got, run.u)
    say(label, steps, "steps: state rel L2", err, "max", mx, "change", chg, "change floor", floor)
    s.close()
    return err, chg, floor, mx


def test_hundred_steps_annulus_replayed(env):
    """100 full steps (network, viscosity, step size, five stages, glue and
    inflow boundary) of the 16-sector annulus at 48 x 48 per patch; the
    oracle replays the GPU's decisions (classes, maximisers, step sizes) so
    the comparison measures arithmetic only.  Bars: 1e-4 relative L2 per
    component of the state (pointwise 10x that), and the change of the
    state over the run within 8x its FP32 floor (change_floor: the +-1 %
    flow moves by ~3e-4 of its norm in 100 steps, so the stored FP32 state's
    own rounding is ~0.5 % of that change)."""
    err, chg, floor, mx = _replayed_steps(env, synth.config(1, n=48), 100, "annulus 48^2")
    assert np.all(err < STEP_TOL) and np.all(mx < PT * STEP_TOL)
    assert np.all(chg[[0, 1, 3]] < 8 * floor[[0, 1, 3]])


@pytest.mark.timeout(900)
def test_twenty_steps_full_size_annulus_replayed(env):
    """20 full steps of the annulus at its stated size (16 sectors of
    256 x 256, about 1.05 M points), the oracle replaying the GPU's
    decisions; the same bars as the 100-step run."""
    err, chg, floor, mx = _replayed_steps(env, synth.config(1), 20, "annulus 256^2")
    assert np.all(err < STEP_TOL) and np.all(mx < PT * STEP_TOL)
    assert np.all(chg[[0, 1, 3]] < 8 * floor[[0, 1, 3]])


# ------------------------------------------------------------------ spectral filter
# Bar: the filter returns the state up to FP32 rounding of the transform pair
# on the extension (~ eps32 log2 L relative) and of the temperature round
# trip (E - |rho u|^2 / (2 rho) cancels up to ~2 bits at Mach 3): relative
# L2 per component <= 2e-6.  A seeded 1e-3 perturbation makes the filter
# change the state by ~100 times that, and the change itself must match the
# oracle's to 2 %.
FILTER_TOL = 2e-6
ALPHA_F, P_F = 10.0, 14


def noisy_state(ps, u, seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    out = np.array(u, np.float32, copy=True).reshape(4, ps.plane)
    for p in range(ps.npatch):
        v = ps.view(out, p)
        v *= (1.0 + amp * rng.standard_normal(v.shape)).astype(np.float32)
    return out


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", ["square64", "annulus", "shells", "uneven"])
def test_spectral_filter(env, case, layout):
    from oracle import filter as flt
    api, ctx, torch = env
    ps, u, _, _ = rhs_case(case)
    s, D, H = mkset(api, ctx, ps, layout)
    s.set_filter(ALPHA_F, P_F)
    x = noisy_state(ps, u, 5)
    xd = D(x)
    out = torch.zeros_like(xd)
    api.fcsd_filter(s, xd, out, G)
    got = H(out).reshape(4, -1)
    want = flt.filter_state(x.astype(np.float64), ps, ALPHA_F, P_F, G)
    err = relerr_phys(ps, got, want)
    chg = relerr_phys(ps, got - x, want - x)
    size = relerr_phys(ps, want, x)          # |want - x| / |x|: what the filter changes
    say("filter", case, "layout", layout, "state rel L2", err, "change rel L2", chg, "change size", size)
    assert np.all(err < FILTER_TOL)
    # rho and E always change; a momentum component that is zero (flow along
    # x) stays zero, so only the larger of the two is required to change
    assert size[0] > 100 * FILTER_TOL and size[3] > 100 * FILTER_TOL and max(size[1], size[2]) > 100 * FILTER_TOL
    assert np.all(chg < 2e-2)
    # in place gives the same bits
    api.fcsd_filter(s, xd, xd, G)
    assert torch.equal(xd, out)
    s.close()


def discontinuous_case(case):
    """A discontinuous initial state on a test geometry: region 1 (a disc
    on the square, x < -0.3 on the annulus sets, the left half of each
    uneven patch) has 1.5 times the density and twice the pressure of the
    smooth base state, at the same velocity."""
    ps, u, _, _ = rhs_case(case)
    x, y = ps.xy
    if case == "square64":
        lab = ((x - 0.45) ** 2 + (y - 0.55) ** 2 < 0.2 ** 2)
    elif case == "uneven":
        lab = np.zeros(ps.plane, bool)
        for p in range(ps.npatch):
            v = ps.view(lab, p)
            v[:, : v.shape[1] // 2] = True
    else:
        lab = x < -0.3
    lab = lab.astype(np.uint8)
    e = np.array(u, np.float64).reshape(4, ps.plane)
    rho, m, n, E = e
    ke = 0.5 * (m * m + n * n) / np.where(rho > 0, rho, 1)
    pr = (G - 1) * (E - ke)
    f = np.where(lab > 0, 1.5, 1.0)
    out = np.stack([rho * f, m * f, n * f, np.where(lab > 0, 2.0, 1.0) * pr / (G - 1) + ke * f])
    return ps, out.astype(np.float32), lab


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", ["square64", "shells", "uneven", "paper_d2"])
def test_initial_smearing(env, case, layout):
    """fcsd_smear against the oracle (Sec. 4.3.2; alpha 10, p 2, c 18, r 9).
    Bar: FP32 rounding of the filtered lines and the window, relative L2 per
    component <= 2e-6 of the state, or 3 times the FP32-emulation floor (the
    oracle with the extension and transform pair in FP32) where that is
    larger: with d = 5 a discontinuity within d points of a line end gives
    continuation tails up to sum |A_r Q^T| ~ 1e4 times the jump, which no
    FP32 transform resolves better; the change (the smearing itself, a few
    per cent of the state) to 1e-3."""
    from oracle import smear
    api, ctx, torch = env
    ps, x, lab = discontinuous_case(case)
    s, D, H = mkset(api, ctx, ps, layout)
    xd = D(x)
    out = torch.zeros_like(xd)
    labd = D(lab)
    api.fcsd_smear(s, xd, labd, out, G)
    got = H(out).reshape(4, -1)
    want = smear.smear_state(x.astype(np.float64), lab, ps, G)
    err = relerr_phys(ps, got, want)
    chg = relerr_phys(ps, got - x, want - x)
    size = relerr_phys(ps, want, x)
    floor = relerr_phys(ps, smear.smear_state(x.astype(np.float64), lab, ps, G, fp32=True), want)
    say("smear", case, "layout", layout, "state rel L2", err, "FP32 floor", floor, "change rel L2", chg,
        "change size", size)
    assert np.all(err < np.maximum(FILTER_TOL, 3 * floor))
    assert size[0] > 1e-3 and size[3] > 1e-3
    assert chg[0] < 1e-3 and chg[3] < 1e-3
    api.fcsd_smear(s, xd, labd, xd, G)
    assert torch.equal(xd, out)
    s.close()


def test_filter_needs_configuration(env):
    api, ctx, torch = env
    ps, u, _, _ = rhs_case("square64")
    s = api.PatchSet.from_layout(ctx, ps)
    xd = dev(torch, u)
    with pytest.raises(api.FcsdError):
        api.fcsd_filter(s, xd, xd, G)
    with pytest.raises(api.FcsdError):
        s.set_filter(10.0, 13)
    s.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_steps_with_filter(env, layout):
    """Three steps of the annulus with the network and the per-step filter
    (Algorithm 1 order: viscosity, filter, glue, step size, stages)."""
    api, ctx, torch = env
    cfg = synth.config(1, n=48)
    ps = cfg.ps
    s, D, H = mkset(api, ctx, ps, layout)
    s.set_filter(ALPHA_F, P_F)
    u0 = noisy_state(ps, cfg.u0, 8)
    u = D(u0)
    W = {k: dev(torch, v) for k, v in cfg.mlp.items()}
    st = api.Stepper(s, u, D(ps.metric), cfg.ref, W=W, dirichlet_mask=D(ps.dirichlet),
                     dirichlet_state=synth.freestream(cfg.mach), filt=True)
    run = solver.Run(cfg)
    run.u = u0.astype(np.float64)
    ref_run = solver.Run(cfg)
    ref_run.u = u0.astype(np.float64)
    for k in range(3):
        u_in = first_step_input(api, s, D, ps, u, cfg) if k == 0 else None
        st.step()
        if k == 0:
            decision_check(ps, u_in, cfg.mlp, H(st.tau), H(st.argmax), label="filtered first step")
        run.step(tau=H(st.tau), arg=H(st.argmax), filt=(ALPHA_F, P_F))
        ref_run.step(dt=run.log[-1]["dt"], tau=run.log[-1]["tau"], arg=run.log[-1]["arg"])
    got = H(u).reshape(4, -1)
    err = relerr_phys(ps, got, run.u)
    eff = relerr_phys(ps, run.u, ref_run.u)     # what the filter changed over three steps
    say("3 filtered steps: state rel L2", err, "filter effect", eff)
    assert np.all(err < STEP_TOL)
    assert np.all(eff[[0, 3]] > 10 * err[[0, 3]])
    s.close()


@pytest.mark.parametrize("case", ["square64", "annulus", "uneven"])
def test_filter_reverse_mode(env, case):
    """fcsd_filter_adj against the oracle's vector-Jacobian product of the
    state filter at the same state.  The transposed line filter folds its
    tail onto the d end samples of each line in FP64 from the cotangent
    (the fold's entries reach ~1e4), so the bar holds over the whole field:
    relative L2 <= 1e-5 and pointwise <= 1e-4 per component, and <= 1e-5
    away from the patch edges."""
    from oracle import filter as flt
    api, ctx, torch = env
    ps, u, _, _ = rhs_case(case)
    s, D, H = mkset(api, ctx, ps, 1)
    s.set_filter(ALPHA_F, P_F)
    x = noisy_state(ps, u, 21)
    yb = smooth_fields(ps, 4, 23) + noisy_state(ps, np.ones((4, ps.plane), np.float32), 24, amp=0.1) - 1.0
    ub = torch.zeros(4 * s.plane, device="cuda:0")      # the layout's plane (blocked storage pads)
    api.fcsd_filter_adj(s, D(x), D(yb), ub, G)
    want = flt.filter_state_vjp(x.astype(np.float64), yb.astype(np.float64), ps, ALPHA_F, P_F, G)
    got = H(ub).reshape(4, -1)
    err = relerr(ps, got, want)
    inner = np.zeros((4, ps.plane))
    for p in range(ps.npatch):
        ps.view(inner[0], p)[10:-10, 10:-10] = 1
    inner[1:] = inner[0]
    err_in = relerr(ps, got * inner, want * inner)
    mx = maxrel_phys(ps, got, want)
    say("filter reverse mode", case, "rel L2", err, "interior", err_in, "max", mx)
    assert np.all(err < 1e-5) and np.all(err_in < 1e-5) and np.all(mx < PT * 1e-5)
    # in place (u_bar = out_bar)
    yd = D(yb)
    api.fcsd_filter_adj(s, D(x), yd, yd, G)
    assert torch.equal(yd, ub)
    s.close()
