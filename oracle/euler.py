"""Euler fluxes and the curvilinear FC right-hand side, FP64.

Test infrastructure only (see oracle/__init__.py).

  * Conserved state e = (rho, rho u, rho v, E), closure E = p/(gamma-1) +
    rho |u|^2 / 2 (Sec. 2.1, eqs. "euler 2d equation", "perfect_gas").
  * Fluxes F (x) and G (y) of eq. "euler 2d equation".
  * Curvilinear form (Sec. 3.3, eq. "general_curvilinear"): with the metric
    terms m[m,a] = dq^m/dx_a, the x-divergence of a flux pair (f_x, f_y) is
    sum_{m,a} m[m,a] d/dq^m f_a (chain rule, non-conservative reading).
  * Artificial viscosity (Sec. 2.3, eqs. "f_visc", "convection diffusion
    eqn"): f_visc = mu grad_x e applied to all four components; the
    right-hand side gains div_x f_visc.  Evaluated as the chain-rule
    divergence of mu times the chain-rule gradient (two FC differentiations).

Metric plane order: m1x = dq1/dx, m1y = dq1/dy, m2x = dq2/dx, m2y = dq2/dy.
"""
from __future__ import annotations

import numpy as np

from oracle import fcgram, wall


def points(ps):
    """Flat plane indices of every patch's grid points (the padding between
    patches, which holds no state, is left out of pointwise work)."""
    idx = getattr(ps, "_points", None)
    if idx is None:
        idx = np.concatenate([np.arange(int(o), int(o) + int(a) * int(b))
                              for o, a, b in zip(ps.off, ps.n1, ps.n2)])
        ps._points = idx
    return idx


def primitives(e, gamma):
    rho = e[0]
    u = e[1] / rho
    v = e[2] / rho
    p = (gamma - 1) * (e[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def fluxes(e, gamma):
    """(F, G), each [4, ...]: F = (rho u, rho u^2 + p, rho u v, u (E + p)),
    G = (rho v, rho u v, rho v^2 + p, v (E + p))."""
    rho, u, v, p = primitives(e, gamma)
    E = e[3]
    F = np.stack([rho * u, rho * u * u + p, rho * u * v, u * (E + p)])
    G = np.stack([rho * v, rho * u * v, rho * v * v + p, v * (E + p)])
    return F, G


def sound_speed(e, gamma):
    """a = sqrt(gamma p / rho) (eq. snd_sp)."""
    rho, u, v, p = primitives(e, gamma)
    return np.sqrt(gamma * p / rho)


def _metric(metric):
    m = np.asarray(metric, np.float64)
    return m[0], m[1], m[2], m[3]


def divergence(fx, fy, metric, ps):
    """sum_{m,a} m[m,a] d/dq^m f_a for stacks fx, fy of shape [k, plane]."""
    m1x, m1y, m2x, m2y = _metric(metric)
    d1x = fcgram.diff_plane(fx, ps, 1)
    d2x = fcgram.diff_plane(fx, ps, 2)
    d1y = fcgram.diff_plane(fy, ps, 1)
    d2y = fcgram.diff_plane(fy, ps, 2)
    return m1x * d1x + m2x * d2x + m1y * d1y + m2y * d2y


def _wall_patches(ps):
    w = getattr(ps, "wall", None)
    return [] if w is None else [p for p in range(ps.npatch) if np.asarray(w[p]).any()]


def _patch_diff(x, ps, p, direction):
    """FC derivative of one patch array [n2, n1] along q^direction."""
    C = int(ps.C1[p] if direction == 1 else ps.C2[p])
    if direction == 1:
        return fcgram.diff_lines(x, ps.d, C)
    return fcgram.diff_lines(x.T, ps.d, C).T


def _patch_diff_adj(y, ps, p, direction):
    C = int(ps.C1[p] if direction == 1 else ps.C2[p])
    if direction == 1:
        return fcgram.diff_lines_adj(y, ps.d, C)
    return fcgram.diff_lines_adj(y.T, ps.d, C).T


def _energy_rule(v, gamma):
    """Coefficients of the energy derivative by the sum and product rules
    (Remark adiabatic, eqs. p_T, perfect_gas_T): with E = rho theta /
    (gamma - 1) + |m|^2 / (2 rho), dE = A d rho + B d theta + Cx d m_x +
    Cy d m_y, A = E / rho - |m|^2 / rho^2, B = rho / (gamma - 1),
    C = m / rho; and their partial derivatives in (rho, m_x, m_y, E)."""
    rho, m, n, E = v
    g1 = gamma - 1.0
    q = m * m + n * n
    A, B, Cx, Cy = E / rho - q / rho ** 2, rho / g1, m / rho, n / rho
    z = np.zeros_like(rho)
    dA = (-E / rho ** 2 + 2 * q / rho ** 3, -2 * m / rho ** 2, -2 * n / rho ** 2, 1 / rho)
    dB = (np.full_like(rho, 1 / g1), z, z, z)
    dCx = (-m / rho ** 2, 1 / rho, z, z)
    dCy = (-n / rho ** 2, z, 1 / rho, z)
    return (A, B, Cx, Cy), (dA, dB, dCx, dCy)


def derivatives(e, ps, gamma=1.4):
    """(d e/dq^1, d e/dq^2) of the four state components by FC (Sec. 2.2).
    On patches with a wall side the energy's derivatives are formed by the
    sum and product rules from those of rho, rho u, rho v and theta = p /
    rho (Remark adiabatic; eqs. p_T, perfect_gas_T), theta's expansion
    being the one through the wall values the glue sets (Neumann-consistent,
    oracle.wall)."""
    e = np.asarray(e, np.float64)
    d = [fcgram.diff_plane(e, ps, 1), fcgram.diff_plane(e, ps, 2)]
    for p in _wall_patches(ps):
        v = ps.view(e, p)
        th = wall.theta_of(v, gamma)
        (A, B, Cx, Cy), _ = _energy_rule(v, gamma)
        for k, direction in ((0, 1), (1, 2)):
            dv = ps.view(d[k], p)
            dth = _patch_diff(th, ps, p, direction)
            dv[3] = A * dv[0] + B * dth + Cx * dv[1] + Cy * dv[2]
    return d[0], d[1]


def derivatives_vjp(e, ps, gamma, g1, g2):
    """Cotangent of e given those of derivatives(e) (g1, g2: [4, plane])."""
    e = np.asarray(e, np.float64)
    g = [np.array(g1, np.float64, copy=True), np.array(g2, np.float64, copy=True)]
    eb = np.zeros(e.shape)
    for p in _wall_patches(ps):
        v = ps.view(e, p)
        th = wall.theta_of(v, gamma)
        (A, B, Cx, Cy), (dA, dB, dCx, dCy) = _energy_rule(v, gamma)
        ebp = ps.view(eb, p)
        for k, direction in ((0, 1), (1, 2)):
            gv = ps.view(g[k], p)
            gE = gv[3].copy()
            dv = ps.view(fcgram.diff_plane(e, ps, direction), p)
            dth = _patch_diff(th, ps, p, direction)
            # the rule's coefficients depend on the state at the point
            for f in range(4):
                ebp[f] += gE * (dA[f] * dv[0] + dB[f] * dth + dCx[f] * dv[1] + dCy[f] * dv[2])
            # the derivatives it combines: rho, m_x, m_y lanes and theta's
            gv[0] += A * gE
            gv[1] += Cx * gE
            gv[2] += Cy * gE
            gv[3] = 0.0
            ebp += wall.theta_vjp(v, _patch_diff_adj(B * gE, ps, p, direction), gamma)
    return eb + fcgram.diff_plane_adj(g[0], ps, 1) + fcgram.diff_plane_adj(g[1], ps, 2)


def gradient(e, metric, ps, gamma=1.4):
    """(d e/dx, d e/dy) by the chain rule: d/dx_a = sum_m m[m,a] d/dq^m."""
    m1x, m1y, m2x, m2y = _metric(metric)
    d1, d2 = derivatives(e, ps, gamma)
    return m1x * d1 + m2x * d2, m1y * d1 + m2y * d2


def euler_rhs(e, metric, ps, gamma):
    """Inviscid right-hand side r = - div_x f(e)."""
    e = np.asarray(e, np.float64)
    k = points(ps)
    F, G = np.zeros(e.shape), np.zeros(e.shape)
    F[:, k], G[:, k] = fluxes(e[:, k], gamma)
    return -divergence(F, G, metric, ps)


def av_term(e, metric, mu, ps, gamma=1.4):
    """Viscous term div_x (mu grad_x e)."""
    ex, ey = gradient(np.asarray(e, np.float64), metric, ps, gamma)
    mu = np.asarray(mu, np.float64)
    return divergence(mu * ex, mu * ey, metric, ps)


def full_rhs(e, metric, mu, ps, gamma):
    """L[e] = - div_x f(e) + div_x (mu grad_x e)  (eq. semi-discrete)."""
    r = euler_rhs(e, metric, ps, gamma)
    if mu is not None:
        r = r + av_term(e, metric, mu, ps, gamma)
    return r


# ------------------------------------------------------------------ adjoints

def fluxes_vjp(e, gamma, Fb, Gb):
    """e_bar = (dF/de)^T F_bar + (dG/de)^T G_bar, pointwise.

    Written from the primitive chain: with rho, m = rho u, n = rho v, E,
    u = m/rho, v = n/rho, p = (gamma-1)(E - (m^2+n^2)/(2 rho))."""
    rho, m, n, E = e
    u, v = m / rho, n / rho
    g1 = gamma - 1
    q2 = u * u + v * v
    p = g1 * (E - 0.5 * rho * q2)
    # partial derivatives of p
    p_rho = g1 * 0.5 * q2
    p_m = -g1 * u
    p_n = -g1 * v
    p_E = g1
    # partials of u, v w.r.t. (rho, m, n)
    u_rho, u_m = -u / rho, 1 / rho
    v_rho, v_n = -v / rho, 1 / rho
    out = np.zeros_like(e)
    H = E + p
    # F = (m, m u + p, m v, u H)
    out[1] += Fb[0]
    # F1 = m u + p
    out[0] += Fb[1] * (m * u_rho + p_rho)
    out[1] += Fb[1] * (u + m * u_m + p_m)
    out[2] += Fb[1] * p_n
    out[3] += Fb[1] * p_E
    # F2 = m v
    out[0] += Fb[2] * (m * v_rho)
    out[1] += Fb[2] * v
    out[2] += Fb[2] * (m * v_n)
    # F3 = u (E + p)
    out[0] += Fb[3] * (u_rho * H + u * p_rho)
    out[1] += Fb[3] * (u_m * H + u * p_m)
    out[2] += Fb[3] * (u * p_n)
    out[3] += Fb[3] * (u * (1 + p_E))
    # G = (n, n u, n v + p, v H)
    out[2] += Gb[0]
    out[0] += Gb[1] * (n * u_rho)
    out[1] += Gb[1] * (n * u_m)
    out[2] += Gb[1] * u
    out[0] += Gb[2] * (n * v_rho + p_rho)
    out[1] += Gb[2] * p_m
    out[2] += Gb[2] * (v + n * v_n + p_n)
    out[3] += Gb[2] * p_E
    out[0] += Gb[3] * (v_rho * H + v * p_rho)
    out[1] += Gb[3] * (v * p_m)
    out[2] += Gb[3] * (v_n * H + v * p_n)
    out[3] += Gb[3] * (v * (1 + p_E))
    return out


def divergence_adj(rb, metric, ps):
    """Transpose of divergence(): returns (fx_bar, fy_bar)."""
    m1x, m1y, m2x, m2y = _metric(metric)
    fxb = fcgram.diff_plane_adj(m1x * rb, ps, 1) + fcgram.diff_plane_adj(m2x * rb, ps, 2)
    fyb = fcgram.diff_plane_adj(m1y * rb, ps, 1) + fcgram.diff_plane_adj(m2y * rb, ps, 2)
    return fxb, fyb


def gradient_adj(exb, eyb, metric, ps, e=None, gamma=1.4):
    """Transpose of gradient at e (e is needed only on patches with walls,
    where the energy's derivatives depend on the state)."""
    m1x, m1y, m2x, m2y = _metric(metric)
    g1, g2 = m1x * exb + m1y * eyb, m2x * exb + m2y * eyb
    if _wall_patches(ps):
        return derivatives_vjp(e, ps, gamma, g1, g2)
    return fcgram.diff_plane_adj(g1, ps, 1) + fcgram.diff_plane_adj(g2, ps, 2)


def av_term_vjp(e, metric, mu, ps, rb, gamma=1.4):
    """(e_bar, mu_bar) for the map (e, mu) -> av_term(e, metric, mu): the
    term is the divergence of V = mu grad_x e, so with (V_x_bar, V_y_bar) the
    divergence transpose of rb, mu_bar = V_bar . grad_x e and e_bar is the
    gradient transpose of mu V_bar."""
    e = np.asarray(e, np.float64)
    mu = np.asarray(mu, np.float64)
    fxb, fyb = divergence_adj(rb, metric, ps)
    ex, ey = gradient(e, metric, ps, gamma)
    mub = np.sum(fxb * ex + fyb * ey, axis=0)
    return gradient_adj(mu * fxb, mu * fyb, metric, ps, e, gamma), mub


def full_rhs_vjp(e, metric, mu, ps, gamma, rb):
    """(e_bar, mu_bar) for the map (e, mu) -> full_rhs(e, metric, mu)."""
    e = np.asarray(e, np.float64)
    fxb, fyb = divergence_adj(rb, metric, ps)
    k = points(ps)
    eb = np.zeros(e.shape)
    eb[:, k] = fluxes_vjp(e[:, k], gamma, -fxb[:, k], -fyb[:, k])
    mub = None
    if mu is not None:
        mu = np.asarray(mu, np.float64)
        ex, ey = gradient(e, metric, ps, gamma)
        mub = np.sum(fxb * ex + fyb * ey, axis=0)
        eb = eb + gradient_adj(mu * fxb, mu * fyb, metric, ps, e, gamma)
    return eb, mub
