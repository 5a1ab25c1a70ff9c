"""Inter-patch interpolation of fringe values, FP64 (paper Sec. 3.4.1,
inter-patch data communication; Remark overlap_cond).

Test infrastructure only (see oracle/__init__.py).

Before every stage, each point of the fringe region of a patch (the n_f
points nearest to a side shared with another patch) is overwritten with a
value interpolated from a donor patch that contains it: among the other
patches whose grid holds a 3 x 3 stencil around the point, the one in which
the point lies farthest from the boundary.  The 3 x 3 stencil of donor grid
points around the point is interpolated by iterated one-dimensional
quadratic interpolation in the donor's parameter space, each evaluated with
Neville's algorithm: along q^1 on the three stencil rows, then along q^2.
The decomposition is checked first: no donor point may itself be a fringe
(receiving) point.

Readings:
  * patch maps are given per patch (synth.PatchSet.geom): Cartesian
    (x, y) = (a0 + i da, b0 + j db) or polar (theta, r) = (a0 + i da,
    b0 + j db); a point's donor coordinates (xi, eta) are the fractional
    grid indices of its preimage;
  * the stencil is centred on the nearest grid point, floor(xi + 1/2),
    moved inwards to stay on the grid; the local coordinates s = xi - ic,
    t = eta - jc lie in [-1/2, 1/2] (up to the inward move);
  * "farthest from the boundary" is min(xi, n1 - 1 - xi, eta, n2 - 1 - eta)
    in grid units, largest wins, the lower patch index on ties; a donor must
    hold the point with that distance >= 1 (a full stencil);
  * the fringe of a side is the n_f grid lines nearest to it (n_f = 5).
"""
from __future__ import annotations

import numpy as np

NF = 5


def preimage(geom_row, x, y):
    """Fractional grid indices (xi, eta) of physical points in one patch."""
    kind, a0, da, b0, db = geom_row
    if int(kind) == 0:
        return (x - a0) / da, (y - b0) / db
    th = np.arctan2(y, x)
    r = np.hypot(x, y)
    return (th - a0) / da, (r - b0) / db


def receivers(ps, p, nf=NF):
    """Boolean [n2, n1] mask of patch p's fringe points."""
    n1, n2 = int(ps.n1[p]), int(ps.n2[p])
    m = np.zeros((n2, n1), bool)
    s = ps.internal[p]
    if s[0]:
        m[:, :nf] = True
    if s[1]:
        m[:, n1 - nf:] = True
    if s[2]:
        m[:nf, :] = True
    if s[3]:
        m[n2 - nf:, :] = True
    return m


def build(ps, nf=NF):
    """The receiver table: list of (p, i, j, q, ic, jc, s, t) -- receiver
    patch and indices, donor patch, stencil centre and local coordinates."""
    masks = [receivers(ps, p, nf) for p in range(ps.npatch)]
    table = []
    for p in range(ps.npatch):
        jj, ii = np.nonzero(masks[p])
        xy = ps.view(ps.xy, p)
        for i, j in zip(ii, jj):
            x, y = xy[0, j, i], xy[1, j, i]
            best = None
            for q in range(ps.npatch):
                if q == p:
                    continue
                xi, eta = preimage(ps.geom[q], x, y)
                n1, n2 = int(ps.n1[q]), int(ps.n2[q])
                dist = min(xi, n1 - 1 - xi, eta, n2 - 1 - eta)
                if dist >= 1 and (best is None or dist > best[0]):
                    best = (dist, q, xi, eta)
            if best is None:
                raise ValueError(f"fringe point ({p}, {i}, {j}) has no donor patch")
            _, q, xi, eta = best
            n1, n2 = int(ps.n1[q]), int(ps.n2[q])
            ic = min(max(int(np.floor(xi + 0.5)), 1), n1 - 2)
            jc = min(max(int(np.floor(eta + 0.5)), 1), n2 - 2)
            if masks[q][jc - 1:jc + 2, ic - 1:ic + 2].any():
                raise ValueError(f"donor stencil of ({p}, {i}, {j}) in patch {q} holds fringe points")
            table.append((p, int(i), int(j), q, ic, jc, xi - ic, eta - jc))
    return table


def neville3(ym, y0, yp, s):
    """Quadratic through (-1, ym), (0, y0), (1, yp) at s, by Neville's
    recurrence: the two linear interpolants, then their combination."""
    p01 = (s + 1) * y0 - s * ym          # through -1 and 0
    p12 = (1 - s) * y0 + s * yp          # through 0 and 1
    return ((s + 1) * p12 - (s - 1) * p01) / 2


def interpolate(e, ps, table):
    """Overwrite the fringe values of a [nf, plane] array in place (values
    are read from donor points, which are never fringe points)."""
    for (p, i, j, q, ic, jc, s, t) in table:
        d = ps.view(e, q)
        rows = [neville3(d[:, jc + k, ic - 1], d[:, jc + k, ic], d[:, jc + k, ic + 1], s) for k in (-1, 0, 1)]
        ps.view(e, p)[:, j, i] = neville3(rows[0], rows[1], rows[2], t)
    return e


def lagrange3(s):
    """Weights of the nodes -1, 0, 1 in the quadratic through them at s (the
    polynomial Neville's recurrence evaluates)."""
    return np.array([0.5 * s * (s - 1), 1 - s * s, 0.5 * s * (s + 1)])


def interpolate_adj(eb, ps, table):
    """In-place transpose of interpolate on a cotangent [nf, plane]: each
    fringe point's cotangent goes to its nine donor points with the
    interpolation weights and is then zeroed (its old value is overwritten
    by the forward map; donors are never fringe points)."""
    for (p, i, j, q, ic, jc, s, t) in table:
        g = ps.view(eb, p)[:, j, i].copy()
        ps.view(eb, p)[:, j, i] = 0.0
        ws, wt = lagrange3(s), lagrange3(t)
        d = ps.view(eb, q)
        for b in range(3):
            for a in range(3):
                d[:, jc - 1 + b, ic - 1 + a] += wt[b] * ws[a] * g
    return eb
