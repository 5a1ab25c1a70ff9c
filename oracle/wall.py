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
  * where two walls meet at a patch corner, the corner point takes the zero
    normal slope in both directions: theta_c = sum_k sum_l c_k c_l
    theta(k, l) over the interior points k, l = 1..d-1 away from the two
    walls (the tensor product of the one-sided Neumann values); every other
    wall point takes its own normal line, which then holds interior points
    only, so the result does not depend on the order of the sides;
  * inside the right-hand side, on patches with a wall side, the
    derivatives of E are formed by the sum and product rules from those of
    rho, rho u, rho v and theta (Remark adiabatic; euler.derivatives), the
    theta lines through the wall values above being the Neumann-consistent
    expansion; in the flux form used here E's derivatives enter the viscous
    flux mu grad_x E, and p's do not appear apart from the flux values;
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


def theta_of(v, gamma):
    """theta = p / rho (eqs. perfect_gas, p_T) of a state [4, ...]."""
    rho, m, n, E = v
    return (gamma - 1.0) * (E - 0.5 * (m * m + n * n) / rho) / rho


def _corner_index(ps, p, side, end):
    """(i, j) index function of the interior points (k, l) of the corner
    where wall `side` of patch p meets the wall at its tangential `end`
    (0: t = 0, 1: t = last): k along the side's normal, l along the wall."""
    n1, n2 = int(ps.n1[p]), int(ps.n2[p])
    if side < 2:                      # wall along j: t = j, normal along i
        ii = (lambda k: k) if side == 0 else (lambda k: n1 - 1 - k)
        jj = (lambda l: l) if end == 0 else (lambda l: n2 - 1 - l)
        return lambda k, l: (jj(l), ii(k))
    jj = (lambda k: k) if side == 2 else (lambda k: n2 - 1 - k)
    ii = (lambda l: l) if end == 0 else (lambda l: n1 - 1 - l)
    return lambda k, l: (jj(k), ii(l))


def corners(ps, p):
    """Corner points of patch p shared by two wall sides: list of
    (side owning the point, end, index function) -- the q1 side (0 or 1)
    owns a corner it shares with a q2 side."""
    out = []
    w = ps.wall[p]
    for side in (0, 1):
        if not w[side]:
            continue
        for end, other in ((0, 2), (1, 3)):
            if w[other]:
                out.append((side, end, _corner_index(ps, p, side, end)))
    return out


def _wall_points(ps, p, side):
    """Tangential index range of the non-corner points of a wall side."""
    n1, n2 = int(ps.n1[p]), int(ps.n2[p])
    length = n2 if side < 2 else n1
    w = ps.wall[p]
    lo = 1 if (side < 2 and w[2]) or (side >= 2 and w[0]) else 0
    hi = length - 1 if (side < 2 and w[3]) or (side >= 2 and w[1]) else length
    return lo, hi


def rules(ps, p):
    """The wall points of patch p with the interior points their theta is
    formed from: a list of (jj, ii, terms), jj / ii index arrays of wall
    points in the patch's [n2, n1] view and terms a list of (weight, js,
    is) with index arrays aligned with them: theta_w = sum weight
    theta(js, is)."""
    c = neumann_weights(ps.d)
    n1, n2 = int(ps.n1[p]), int(ps.n2[p])
    out = []
    for side in range(4):
        if not ps.wall[p, side]:
            continue
        lo, hi = _wall_points(ps, p, side)
        t = np.arange(lo, hi)
        if side == 0:
            jj, ii, nrm = t, np.zeros_like(t), (lambda k: (t, np.full_like(t, k)))
        elif side == 1:
            jj, ii, nrm = t, np.full_like(t, n1 - 1), (lambda k: (t, np.full_like(t, n1 - 1 - k)))
        elif side == 2:
            jj, ii, nrm = np.zeros_like(t), t, (lambda k: (np.full_like(t, k), t))
        else:
            jj, ii, nrm = np.full_like(t, n2 - 1), t, (lambda k: (np.full_like(t, n2 - 1 - k), t))
        out.append((jj, ii, [(c[k],) + nrm(k) for k in range(1, ps.d)]))
    for side, end, idx in corners(ps, p):
        j0, i0 = idx(0, 0)
        terms = []
        for k in range(1, ps.d):
            for l in range(1, ps.d):
                j, i = idx(k, l)
                terms.append((c[k] * c[l], np.array([j]), np.array([i])))
        out.append((np.array([j0]), np.array([i0]), terms))
    return out


def apply(e, ps, gamma=1.4):
    """In-place wall condition on a [4, plane] state for every side flagged
    in ps.wall ([P, 4]: q1-, q1+, q2-, q2+), corners shared by two walls
    included.  Every theta used is an interior point's, read before any
    wall point is written."""
    if getattr(ps, "wall", None) is None:
        return e
    g1 = gamma - 1.0
    for p in range(ps.npatch):
        if not ps.wall[p].any():
            continue
        v = ps.view(e, p)
        th_all = theta_of(v, gamma)
        writes = [(jj, ii, sum(w * th_all[js, is_] for w, js, is_ in terms)) for jj, ii, terms in rules(ps, p)]
        for jj, ii, th in writes:
            v[1, jj, ii] = 0.0
            v[2, jj, ii] = 0.0
            v[3, jj, ii] = v[0, jj, ii] * th / g1
    return e


def theta_vjp(v, tb, gamma):
    """Cotangent of a state [4, ...] given that of theta = theta_of(v)."""
    rho, m, n, E = v
    g1 = gamma - 1.0
    return np.stack([tb * g1 * (-E / rho ** 2 + (m * m + n * n) / rho ** 3), -tb * g1 * m / rho ** 2,
                     -tb * g1 * n / rho ** 2, tb * g1 / rho])


def apply_vjp(eb, e_glued, ps, gamma=1.4):
    """In-place transpose of apply at the state it produced (e_glued: the
    wall leaves rho and every point off the wall points as it found them, so
    its inputs are read there).  The momenta and E of a wall point are
    overwritten: their cotangents are dropped; rho_w gets theta_w / (gamma
    - 1) times E_w's cotangent, and each interior source point its weight
    times rho_w / (gamma - 1) times E_w's cotangent through d theta / d e."""
    if getattr(ps, "wall", None) is None:
        return eb
    g1 = gamma - 1.0
    for p in range(ps.npatch):
        if not ps.wall[p].any():
            continue
        v = ps.view(e_glued, p)
        b = ps.view(eb, p)
        th_all = theta_of(v, gamma)
        rl = rules(ps, p)
        # every cotangent read before any is written (wall points are never sources)
        reads = [(b[3, jj, ii].copy(), sum(w * th_all[js, is_] for w, js, is_ in terms)) for jj, ii, terms in rl]
        for (jj, ii, terms), (Eb, th) in zip(rl, reads):
            b[0, jj, ii] += Eb * th / g1
            b[1, jj, ii] = 0.0
            b[2, jj, ii] = 0.0
            b[3, jj, ii] = 0.0
            tb = Eb * v[0, jj, ii] / g1          # cotangent of theta_w
            for w, js, is_ in terms:
                np.add.at(b, (slice(None), js, is_), theta_vjp(v[:, js, is_], w * tb, gamma))
    return eb
