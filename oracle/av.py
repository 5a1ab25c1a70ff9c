"""Network-driven smooth artificial viscosity, FP64 (paper Secs. 5.1, 5.2).

Test infrastructure only (see oracle/__init__.py).

  * Proxy variable: the Mach number Phi = |u| sqrt(rho / (gamma p)) (Sec. 5.1).
  * Viscosity-generation subgrid D~ (eqs. "viscosity_generation",
    "index_viscosity_generation"): patch points outside the n_v-point fringe of
    the internal sides (n_v = 9; fringe = max-index distance < n_v, eq.
    "fringe_region").
  * Smoothness classifier tau~ (Sec. 5.1).  The trained network and its
    stencils live in a reference the paper does not reproduce; reading: for
    every D~ point and each parameter direction a 16-sample window of Phi
    along the grid line (offsets -8..+7, indices clamped to the line) is
    rescaled to [-1, 1] (x = 2 (w - min w)/(max w - min w) - 1; x = 0 when the
    range is <= 1e-6 max(1, |max w|)) and fed to a 16-64-64-4 ReLU network;
    tau = 1 + argmax of the four outputs (ties to the lowest index) and the
    2D class is the smaller (more viscous) of the two directions.
  * Preliminary viscosity (eq. "V2D_unscaled"):
    mu^_ij = R(tau_ij) max_{7x7 stencil} S  h^,  R = (1.5, 1, 0.5, 0),
    S = |u| + |v| + a, the 7x7 stencil clamped to the patch grid, h^ the
    patch's maximum spacing.
  * Smoothing-blending operator (eqs. "W", "multipatch_W",
    "multipatch_W_norm", "Lambda", "viscosity"): mu = sum W~ mu^ with the
    separable cos^2 window of eq. "qf" at c = 0, r = 9.  Reading of the garbled
    window: w(k h) = cos^2(pi |k| / (2 r)) for |k| < r, 0 beyond, i.e.
    cos^2(pi k / 18) for |k| <= 8.  Normalisation sums over all patches; on
    the index-aligned annulus the nearest-point map zeta is an index shift, so
    Lambda is a separable window sum over a global index lattice followed by
    division by the window sum of the D~ indicator.  On patches that overlap
    without shared grid lines (sets with patch maps), zeta_R(x) is the grid
    point of R nearest to x's preimage (eq. zeta, rnd(n + 1/2) = n + 1), x
    in R's domain meaning its preimage lies in R's closed parameter
    rectangle; the numerator and denominator at x sum R's window sums at
    zeta_R(x) over every patch R holding x.
"""
from __future__ import annotations

import numpy as np

from oracle import euler, interp

NV = 9
R_TABLE = np.array([1.5, 1.0, 0.5, 0.0])
WIN_HALF = 8
STENCIL = 3          # 7x7 stencil half-width
FEAT = 16


def window_weights():
    k = np.arange(-WIN_HALF, WIN_HALF + 1)
    return np.cos(np.pi * k / 18.0) ** 2


def proxy(e, gamma):
    rho, u, v, p = euler.primitives(np.asarray(e, np.float64), gamma)
    return np.sqrt(u * u + v * v) * np.sqrt(rho / (gamma * p))


def dtilde_mask(ps, p):
    """Boolean [n2, n1] mask of D~ for patch p."""
    a, b = int(ps.n1[p]), int(ps.n2[p])
    m = np.ones((b, a), bool)
    q1m, q1p, q2m, q2p = ps.internal[p]
    if q1m:
        m[:, :NV] = False
    if q1p:
        m[:, a - NV:] = False
    if q2m:
        m[:NV, :] = False
    if q2p:
        m[b - NV:, :] = False
    return m


def features_lines(phi_lines):
    """[nl, n] lines -> [nl, n, 16] rescaled windows centred at every point."""
    nl, n = phi_lines.shape
    idx = np.clip(np.arange(n)[:, None] + np.arange(-8, 8)[None, :], 0, n - 1)
    w = phi_lines[:, idx]                       # [nl, n, 16]
    lo = w.min(axis=-1, keepdims=True)
    hi = w.max(axis=-1, keepdims=True)
    rng = hi - lo
    flat = rng <= 1e-6 * np.maximum(1.0, np.abs(hi))
    x = 2.0 * (w - lo) / np.where(flat, 1.0, rng) - 1.0
    return np.where(flat, 0.0, x)


def mlp_logits(x, W):
    """Plain forward pass: ReLU(x W1 + b1) -> ReLU(. W2 + b2) -> . W3 + b3."""
    h = np.maximum(x @ W["W1"].astype(np.float64) + W["b1"].astype(np.float64), 0.0)
    h = np.maximum(h @ W["W2"].astype(np.float64) + W["b2"].astype(np.float64), 0.0)
    return h @ W["W3"].astype(np.float64) + W["b3"].astype(np.float64)


def mlp_vjp(x, W, lb):
    """Cotangent of the features x [..., 16] given that of the logits lb
    [..., 4]: the reverse of mlp_logits, through the ReLU masks at x
    (derivative 0 at a unit whose input is exactly 0)."""
    Wd = {k: np.asarray(v, np.float64) for k, v in W.items()}
    z1 = x @ Wd["W1"] + Wd["b1"]
    z2 = np.maximum(z1, 0.0) @ Wd["W2"] + Wd["b2"]
    g2 = (lb @ Wd["W3"].T) * (z2 > 0)
    g1 = (g2 @ Wd["W2"].T) * (z1 > 0)
    return g1 @ Wd["W1"].T


def classes_from_logits(l1, l2):
    """2D smoothness class from the logits of the two directions (reading
    of Sec. 5.1): a direction's class is 1 + the index of its largest logit
    (the lowest index among equal largest logits), and the point takes the
    smaller of the two directions' classes (the more viscous one)."""
    return np.minimum(np.argmax(l1, -1), np.argmax(l2, -1)) + 1


def classify(e, ps, W, gamma, return_logits=False):
    """tau plane (int8, 0 outside D~) and optionally the per-direction logits
    {patch: (l1, l2)}, each [n2, n1, 4]; proxy, features and network in
    FP64."""
    e = np.asarray(e, np.float64)
    tau = np.zeros(ps.plane, np.int8)
    logits = {}
    for p in range(ps.npatch):
        ph = proxy(ps.view(e, p), gamma)                                      # [n2, n1]
        l1 = mlp_logits(features_lines(ph), W)                                # lines along q1
        l2 = np.swapaxes(mlp_logits(features_lines(ph.T), W), 0, 1)           # lines along q2 -> [n2, n1, 4]
        t = classes_from_logits(l1, l2)
        ps.view(tau, p)[...] = np.where(dtilde_mask(ps, p), t, 0)
        logits[p] = (l1, l2)
    return (tau, logits) if return_logits else tau


def stencil_max(S2d, second=False):
    """7x7 maximum clamped to the grid, with the flat index of the maximiser
    (first in row-major stencil order on ties); second=True also returns
    the largest value at any other stencil position (the decision's
    margin is best - second)."""
    b, a = S2d.shape
    best = np.full((b, a), -np.inf)
    nxt = np.full((b, a), -np.inf)
    arg = np.zeros((b, a), np.int64)
    J, I = np.meshgrid(np.arange(b), np.arange(a), indexing="ij")
    for dj in range(-STENCIL, STENCIL + 1):
        for di in range(-STENCIL, STENCIL + 1):
            jj, ii = J + dj, I + di
            ok = (jj >= 0) & (jj < b) & (ii >= 0) & (ii < a)
            val = np.where(ok, S2d[np.clip(jj, 0, b - 1), np.clip(ii, 0, a - 1)], -np.inf)
            better = val > best
            nxt = np.where(better, best, np.maximum(nxt, val))
            best = np.where(better, val, best)
            arg = np.where(better, np.clip(jj, 0, b - 1) * a + np.clip(ii, 0, a - 1), arg)
    return (best, arg, nxt) if second else (best, arg)


def preliminary(e, tau, ps, gamma, arg=None):
    """mu^ plane (0 outside D~) and the argmax plane (patch-local flat
    index), FP64.  arg: replay recorded maximiser positions (frozen
    decision) and take S there."""
    from oracle.rk import wave_speed
    e = np.asarray(e, np.float64)
    if arg is not None:
        muh = np.zeros(ps.plane)
        for p in range(ps.npatch):
            mx = wave_speed(ps.view(e, p), gamma).ravel()[ps.view(arg, p)]
            t = ps.view(tau, p).astype(np.int64)
            r = np.where(t > 0, R_TABLE[np.clip(t - 1, 0, 3)], 0.0)
            ps.view(muh, p)[...] = np.where(dtilde_mask(ps, p), r * mx * ps.hhat[p], 0.0)
        return muh, arg
    muh = np.zeros(ps.plane)
    arg = np.zeros(ps.plane, np.int64)
    for p in range(ps.npatch):
        mx, am = stencil_max(wave_speed(ps.view(e, p), gamma))
        t = ps.view(tau, p).astype(np.int64)
        r = np.where(t > 0, R_TABLE[np.clip(t - 1, 0, 3)], 0.0)
        ps.view(muh, p)[...] = np.where(dtilde_mask(ps, p), r * mx * ps.hhat[p], 0.0)
        ps.view(arg, p)[...] = am
    return muh, arg


def _global_index(ps, p):
    """Global lattice coordinates (G, J) of patch p's points (annulus) or None."""
    if ps.nsec == 0:
        return None
    a, b = int(ps.n1[p]), int(ps.n2[p])
    s, k = p % ps.nsec, p // ps.nsec
    ring = ps.nsec * (a - 2 * NV - 1)
    g = (s * (a - 2 * NV - 1) + np.arange(a)) % ring
    jj = k * (b - 2 * NV - 1) + np.arange(b)
    return g, jj, ring, ps.nshell * (b - 2 * NV - 1) + 2 * NV + 1


def smooth_blend(muh, ps):
    """mu = Lambda[mu^] (eqs. Lambda, viscosity)."""
    w = window_weights()
    mu = np.zeros(ps.plane)
    if ps.nsec == 0:
        nums, dens = [], []
        for p in range(ps.npatch):
            m = dtilde_mask(ps, p).astype(np.float64)
            nums.append(_sep_conv(ps.view(muh, p) * m, w))
            dens.append(_sep_conv(m, w))
        if ps.geom is None:
            for p in range(ps.npatch):
                ps.view(mu, p)[...] = nums[p] / dens[p]
            return mu
        # patches that overlap without shared grid lines (eqs. multipatch_W,
        # zeta): a point x of patch p also collects, from every other patch
        # R whose domain holds it, R's window sums at zeta_R(x), the grid
        # point of R nearest to x's preimage (rnd(n + 1/2) = n + 1)
        for p in range(ps.npatch):
            num, den = nums[p].copy(), dens[p].copy()
            x, y = ps.view(ps.xy, p)
            for q in range(ps.npatch):
                if q == p:
                    continue
                n1, n2 = int(ps.n1[q]), int(ps.n2[q])
                xi, eta = interp.preimage(ps.geom[q], x, y, n1, n2)
                inside = (xi >= 0) & (xi <= n1 - 1) & (eta >= 0) & (eta <= n2 - 1)
                I = np.floor(np.where(inside, xi, 0) + 0.5).astype(int)
                J = np.floor(np.where(inside, eta, 0) + 0.5).astype(int)
                num += np.where(inside, nums[q][J, I], 0.0)
                den += np.where(inside, dens[q][J, I], 0.0)
            ps.view(mu, p)[...] = num / den
        return mu
    g0, j0, ring, nJ = _global_index(ps, 0)
    num = np.zeros((nJ, ring))
    den = np.zeros((nJ, ring))
    for p in range(ps.npatch):
        g, jj, _, _ = _global_index(ps, p)
        m = dtilde_mask(ps, p)
        G, JJ = np.meshgrid(g, jj)
        np.add.at(num, (JJ[m], G[m]), ps.view(muh, p)[m])
        np.add.at(den, (JJ[m], G[m]), 1.0)
    num = _sep_conv(num, w, periodic_cols=True)
    den = _sep_conv(den, w, periodic_cols=True)
    for p in range(ps.npatch):
        g, jj, _, _ = _global_index(ps, p)
        G, JJ = np.meshgrid(g, jj)
        ps.view(mu, p)[...] = num[JJ, G] / den[JJ, G]
    return mu


def _sep_conv(a, w, periodic_cols=False):
    """sum_{k,l} w[k] w[l] a[j+k, i+l] with zero padding (rows) and zero or
    periodic padding (columns)."""
    h = len(w) // 2
    b, n = a.shape
    out = np.zeros_like(a)
    for l in range(-h, h + 1):
        if periodic_cols:
            out += w[l + h] * np.roll(a, -l, axis=1)
        else:
            sh = np.zeros_like(a)
            if l >= 0:
                sh[:, :n - l] = a[:, l:]
            else:
                sh[:, -l:] = a[:, :n + l]
            out += w[l + h] * sh
    res = np.zeros_like(out)
    for k in range(-h, h + 1):
        sh = np.zeros_like(out)
        if k >= 0:
            sh[:b - k] = out[k:]
        else:
            sh[-k:] = out[:b + k]
        res += w[k + h] * sh
    return res


def viscosity(e, ps, W, gamma, tau=None, arg=None):
    """Full per-step viscosity: classifier, preliminary, Lambda.  Returns
    (mu, tau, argmax).  tau / arg given: replayed decisions."""
    if tau is None:
        tau = classify(e, ps, W, gamma)
    muh, arg = preliminary(e, tau, ps, gamma, arg=arg)
    return smooth_blend(muh, ps), tau, arg


# ------------------------------------------------------------------ adjoints

def smooth_blend_adj(mub, ps):
    """Transpose of smooth_blend (a linear map of mu^)."""
    w = window_weights()
    out = np.zeros(ps.plane)
    if ps.nsec == 0 and ps.geom is not None:
        # mu(x) = sum_R num_R(zeta_R(x)) / D(x): t = mu_bar / D goes back to
        # every cell it was read from, then through the (symmetric) window
        # sums and the D~ indicator
        ms = [dtilde_mask(ps, p).astype(np.float64) for p in range(ps.npatch)]
        dens = [_sep_conv(m, w) for m in ms]
        cells = []          # per patch: list of (other patch, inside, I, J)
        D = []
        for p in range(ps.npatch):
            x, y = ps.view(ps.xy, p)
            d = dens[p].copy()
            lst = []
            for q in range(ps.npatch):
                if q == p:
                    continue
                n1, n2 = int(ps.n1[q]), int(ps.n2[q])
                xi, eta = interp.preimage(ps.geom[q], x, y, n1, n2)
                inside = (xi >= 0) & (xi <= n1 - 1) & (eta >= 0) & (eta <= n2 - 1)
                I = np.floor(np.where(inside, xi, 0) + 0.5).astype(int)
                J = np.floor(np.where(inside, eta, 0) + 0.5).astype(int)
                d += np.where(inside, dens[q][J, I], 0.0)
                lst.append((q, inside, I, J))
            cells.append(lst)
            D.append(d)
        acc = [np.zeros_like(d) for d in dens]
        for p in range(ps.npatch):
            t = ps.view(mub, p) / D[p]
            acc[p] += t
            for (q, inside, I, J) in cells[p]:
                np.add.at(acc[q], (J[inside], I[inside]), t[inside])
        for p in range(ps.npatch):
            ps.view(out, p)[...] = ms[p] * _sep_conv(acc[p], w)
        return out
    if ps.nsec == 0:
        for p in range(ps.npatch):
            m = dtilde_mask(ps, p).astype(np.float64)
            den = _sep_conv(m, w)
            ps.view(out, p)[...] = m * _sep_conv(ps.view(mub, p) / den, w)
        return out
    g0, j0, ring, nJ = _global_index(ps, 0)
    den = np.zeros((nJ, ring))
    for p in range(ps.npatch):
        g, jj, _, _ = _global_index(ps, p)
        m = dtilde_mask(ps, p)
        G, JJ = np.meshgrid(g, jj)
        np.add.at(den, (JJ[m], G[m]), 1.0)
    den = _sep_conv(den, w, periodic_cols=True)
    acc = np.zeros((nJ, ring))
    for p in range(ps.npatch):
        g, jj, _, _ = _global_index(ps, p)
        G, JJ = np.meshgrid(g, jj)
        np.add.at(acc, (JJ, G), ps.view(mub, p) / den[JJ, G])
    acc = _sep_conv(acc, w, periodic_cols=True)   # window is symmetric
    for p in range(ps.npatch):
        g, jj, _, _ = _global_index(ps, p)
        G, JJ = np.meshgrid(g, jj)
        ps.view(out, p)[...] = dtilde_mask(ps, p) * acc[JJ, G]
    return out


def wave_speed_vjp(e, gamma, Sb):
    """e_bar for S = |u| + |v| + a (sign(0) = 0)."""
    rho, m, n, E = np.asarray(e, np.float64)
    u, v = m / rho, n / rho
    g1 = gamma - 1
    p = g1 * (E - 0.5 * rho * (u * u + v * v))
    a = np.sqrt(gamma * p / rho)
    # a = sqrt(gamma p / rho): da = gamma/(2 a rho) dp - a/(2 rho) drho
    out = np.zeros((4,) + np.shape(rho))
    su, sv = np.sign(u), np.sign(v)
    # u = m / rho
    out[0] += Sb * (su * (-u / rho) + sv * (-v / rho))
    out[1] += Sb * su / rho
    out[2] += Sb * sv / rho
    ap = gamma / (2 * a * rho)
    p_rho, p_m, p_n, p_E = g1 * 0.5 * (u * u + v * v), -g1 * u, -g1 * v, g1
    out[0] += Sb * (ap * p_rho - a / (2 * rho))
    out[1] += Sb * ap * p_m
    out[2] += Sb * ap * p_n
    out[3] += Sb * ap * p_E
    return out


def viscosity_vjp(e, tau, arg, ps, gamma, mub):
    """e_bar through mu = Lambda[R(tau) S(argmax) h^] with tau and the argmax
    frozen."""
    muhb = smooth_blend_adj(mub, ps)
    Sb = np.zeros(ps.plane)
    for p in range(ps.npatch):
        t = ps.view(tau, p).astype(np.int64)
        r = np.where(t > 0, R_TABLE[np.clip(t - 1, 0, 3)], 0.0) * dtilde_mask(ps, p)
        contrib = (r * ps.hhat[p] * ps.view(muhb, p)).ravel()
        sb = np.zeros(contrib.size)
        np.add.at(sb, ps.view(arg, p).ravel(), contrib)
        ps.view(Sb, p)[...] = sb.reshape(ps.view(Sb, p).shape)
    out = np.zeros((4, ps.plane))
    for p in range(ps.npatch):
        ps.view(out, p)[...] = wave_speed_vjp(ps.view(np.asarray(e, np.float64), p), gamma, ps.view(Sb, p))
    return out
