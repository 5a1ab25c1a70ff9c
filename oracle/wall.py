"""No-slip adiabatic walls through a Neumann FC boundary value, FP64 (paper
Sec. 2.2 on Neumann data, Sec. 4.2, Remarks adiabatic_th and adiabatic).

Test infrastructure only (see oracle/__init__.py).

A Neumann continuation is built from the vector (F_0, ..., F_{N-2},
F'_{N-1}): the d matching conditions at a wall end are the values at the
d - 1 grid points next to it and the derivative at the wall point.  The
Gram polynomial of degree < d that the continuation extends is then the one
that meets those conditions, and its value at the wall point is the value
the continuation assigns there.  This module computes that value; with it,
the continuation is the ordinary one of the line whose wall value has been
replaced.

At every stage input (with the rest of the glue) a wall side of a patch
gets: rho u = rho v = 0 (no slip); the temperature theta = p / rho (eq. p_T)
at the wall point from its zero normal derivative along the grid line that
meets the wall (adiabatic), through the Neumann value above; E rebuilt from
rho, the (zero) momenta and that theta (eq. perfect_gas_T); rho itself is
evolved like an interior value.

Readings:
  * the normal derivative is taken along the grid line that meets the wall
    (on the annulus the radial q^2 lines, normal to the cylinder);
  * the derivatives of E and p inside the right-hand side are those of the
    FC expansions of the glued state (the wall value carries the adiabatic
    condition), not rebuilt by the product rule from a Neumann expansion of
    theta as Remark adiabatic describes -- a simplification of this build;
  * wall points are set after the fringe exchange and the Dirichlet
    overwrite (so the reverse mode transposes them first).
"""
from __future__ import annotations

import numpy as np


def neumann_weights(d: int) -> np.ndarray:
    """c with p(0) = c[0] g + sum_{k=1}^{d-1} c[k] F_k for the polynomial p of
    degree < d with p(k) = F_k (k = 1..d-1, grid units from the wall) and
    p'(0) = g."""
    A = np.zeros((d, d))
    for k in range(1, d):
        A[k - 1] = [float(k) ** m for m in range(d)]
    A[d - 1, 1] = 1.0                      # derivative at the wall point
    inv = np.linalg.inv(A)
    # p(0) = a_0 = row 0 of A^-1 applied to (F_1, .., F_{d-1}, g)
    row = inv[0]
    return np.concatenate([[row[d - 1]], row[:d - 1]])


def wall_lines(ps, p, side):
    """Index arrays (wall point, interior points k = 1..d-1 away) of one side
    of patch p as slices of its [n2, n1] view: returns a function of k that
    gives the k-th line parallel to the wall."""
    n1, n2 = int(ps.n1[p]), int(ps.n2[p])
    if side == 0:
        return lambda v, k: v[..., :, k]
    if side == 1:
        return lambda v, k: v[..., :, n1 - 1 - k]
    if side == 2:
        return lambda v, k: v[..., k, :]
    return lambda v, k: v[..., n2 - 1 - k, :]


def apply(e, ps, gamma=1.4):
    """In-place wall condition on a [4, plane] state for every side flagged
    in ps.wall ([P, 4]: q1-, q1+, q2-, q2+)."""
    if getattr(ps, "wall", None) is None:
        return e
    c = neumann_weights(ps.d)
    g1 = gamma - 1.0
    for p in range(ps.npatch):
        for side in range(4):
            if not ps.wall[p, side]:
                continue
            v = ps.view(e, p)
            line = wall_lines(ps, p, side)
            th = np.zeros_like(line(v[0], 0))
            for k in range(1, ps.d):
                rho, m, n, E = (line(v[f], k) for f in range(4))
                th += c[k] * g1 * (E - 0.5 * (m * m + n * n) / rho) / rho
            rho_w = line(v[0], 0)
            line(v[1], 0)[...] = 0.0
            line(v[2], 0)[...] = 0.0
            line(v[3], 0)[...] = rho_w * th / g1
    return e


def apply_vjp(eb, e_glued, ps, gamma=1.4):
    """In-place transpose of apply at the state it produced (e_glued: the
    wall leaves rho and every point off the wall line as it found them, so
    its inputs are read there).  The momenta and E of a wall point are
    overwritten: their cotangents are dropped; rho_w gets theta_w / (gamma
    - 1) times E_w's cotangent, and each interior point k the Neumann weight
    c_k times rho_w / (gamma - 1) times E_w's cotangent times d theta_k / d e_k."""
    if getattr(ps, "wall", None) is None:
        return eb
    c = neumann_weights(ps.d)
    g1 = gamma - 1.0
    for p in range(ps.npatch):
        for side in range(4):
            if not ps.wall[p, side]:
                continue
            v = ps.view(e_glued, p)
            b = ps.view(eb, p)
            line = wall_lines(ps, p, side)
            rho_w = line(v[0], 0)
            Eb = line(b[3], 0).copy()
            th = np.zeros_like(rho_w)
            for k in range(1, ps.d):
                rho, m, n, E = (line(v[f], k) for f in range(4))
                th += c[k] * g1 * (E - 0.5 * (m * m + n * n) / rho) / rho
            line(b[0], 0)[...] += Eb * th / g1
            line(b[1], 0)[...] = 0.0
            line(b[2], 0)[...] = 0.0
            line(b[3], 0)[...] = 0.0
            tb = Eb * rho_w / g1               # cotangent of theta_w
            for k in range(1, ps.d):
                rho, m, n, E = (line(v[f], k) for f in range(4))
                tk = c[k] * tb
                # theta = g1 (E / rho - (m^2 + n^2) / (2 rho^2))
                line(b[0], k)[...] += tk * g1 * (-E / rho ** 2 + (m * m + n * n) / rho ** 3)
                line(b[1], k)[...] += -tk * g1 * m / rho ** 2
                line(b[2], k)[...] += -tk * g1 * n / rho ** 2
                line(b[3], k)[...] += tk * g1 / rho
    return eb
