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
  * patch maps are given per patch (synth.PatchSet.geom, one row of GEOM
    numbers each): Cartesian (x, y) = (a0 + i da, b0 + j db); polar
    (theta, r) = (a0 + i da, b0 + j db); affine (x, y) = (x0, y0) +
    i (ux, uy) + j (vx, vy) (the C- and I-type patches of Sec. 3.1); and
    S-type (eq. param_S) M = l(t) + s nu(t) with t = a0 + i da,
    s = b0 + j db, the arc l(t) = sum_k (cx_k cos kt + sx_k sin kt,
    cy_k cos kt + sy_k sin kt) and nu the unit normal, the tangent turned
    by -90 degrees (side = +1) or +90 degrees (side = -1); a point's donor
    coordinates (xi, eta) are the fractional grid indices of its preimage
    (for S-type patches found by Newton's method on (t, s));
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


# layout of a patch-map row (synth.PatchSet.geom)
KIND, A0, DA, B0, DB = 0, 1, 2, 3, 4
X0, Y0, UX, UY, VX, VY = 5, 6, 7, 8, 9, 10
SIDE, NMODES = 11, 12
KMAX = 8
CX, SX, CY, SY = 13, 13 + KMAX, 13 + 2 * KMAX, 13 + 3 * KMAX
GEOM = 13 + 4 * KMAX
CARTESIAN, POLAR, AFFINE, STYPE = 0, 1, 2, 3


def arc(g, t, order=0):
    """The S-type arc l(t) (order 0), l'(t) (1) or l''(t) (2), shape [2, ...]."""
    t = np.asarray(t, np.float64)
    x = np.zeros_like(t)
    y = np.zeros_like(t)
    for k in range(int(g[NMODES])):
        c, s = np.cos(k * t), np.sin(k * t)
        # d^order/dt^order of (a cos kt + b sin kt)
        if order == 0:
            fc, fs = c, s
        elif order == 1:
            fc, fs = -k * s, k * c
        else:
            fc, fs = -k * k * c, -k * k * s
        x = x + g[CX + k] * fc + g[SX + k] * fs
        y = y + g[CY + k] * fc + g[SY + k] * fs
    return np.array([x, y])


def normal(g, t):
    """Unit normal nu(t) of the S-type arc and its derivative d nu / dt."""
    d1, d2 = arc(g, t, 1), arc(g, t, 2)
    sd = float(g[SIDE])
    n = np.hypot(d1[0], d1[1])
    rot = lambda v: sd * np.array([v[1], -v[0]])       # the tangent turned by -90 degrees (side +1)
    nu = rot(d1) / n
    dn = rot(d2) / n - rot(d1) * (d1[0] * d2[0] + d1[1] * d2[1]) / n ** 3
    return nu, dn


def image(g, i, j):
    """Physical point (x, y) of fractional grid indices (i, j) of a patch."""
    kind = int(g[KIND])
    i = np.asarray(i, np.float64)
    j = np.asarray(j, np.float64)
    if kind == CARTESIAN:
        return g[A0] + i * g[DA], g[B0] + j * g[DB]
    if kind == POLAR:
        th, r = g[A0] + i * g[DA], g[B0] + j * g[DB]
        return r * np.cos(th), r * np.sin(th)
    if kind == AFFINE:
        return g[X0] + i * g[UX] + j * g[VX], g[Y0] + i * g[UY] + j * g[VY]
    t, s = g[A0] + i * g[DA], g[B0] + j * g[DB]
    l = arc(g, t)
    nu, _ = normal(g, t)
    return l[0] + s * nu[0], l[1] + s * nu[1]


def _grid_image(g, n1, n2):
    """Grid indices and images of the n1 x n2 grid and one ring beyond it."""
    I, J = np.meshgrid(np.arange(-1, n1 + 1), np.arange(-1, n2 + 1))
    I, J = I.ravel(), J.ravel()
    gx, gy = image(g, I, J)
    return I, J, gx, gy


def _stype_preimage(g, x, y, grid):
    """(t, s) with l(t) + s nu(t) = (x, y) by Newton's method on the 2 x 2
    system, started from the grid point (of the patch grid and one ring of
    points beyond it) nearest to (x, y); NaN where the iteration does not
    settle."""
    I, J, gx, gy = grid
    k = int(np.argmin((gx - x) ** 2 + (gy - y) ** 2))
    t = g[A0] + I[k] * g[DA]
    s = g[B0] + J[k] * g[DB]
    scale = 1.0 + abs(x) + abs(y)
    for _ in range(50):
        l = arc(g, t)
        d1 = arc(g, t, 1)
        nu, dn = normal(g, t)
        f = np.array([l[0] + s * nu[0] - x, l[1] + s * nu[1] - y])
        Jm = np.array([[d1[0] + s * dn[0], nu[0]], [d1[1] + s * dn[1], nu[1]]])
        step = np.linalg.solve(Jm, f)
        t -= step[0]
        s -= step[1]
        if np.hypot(f[0], f[1]) <= 1e-14 * scale and abs(step[0]) <= 1e-13 * (1 + abs(t)):
            return t, s
    l = arc(g, t)
    nu, _ = normal(g, t)
    if np.hypot(l[0] + s * nu[0] - x, l[1] + s * nu[1] - y) <= 1e-12 * scale:
        return t, s
    return np.nan, np.nan


def preimage(geom_row, x, y, n1=None, n2=None):
    """Fractional grid indices (xi, eta) of physical points in one patch
    (n1, n2: the patch grid, needed for S-type patches)."""
    g = geom_row
    kind = int(g[KIND])
    if kind == CARTESIAN:
        return (x - g[A0]) / g[DA], (y - g[B0]) / g[DB]
    if kind == POLAR:
        th = np.arctan2(y, x)
        r = np.hypot(x, y)
        return (th - g[A0]) / g[DA], (r - g[B0]) / g[DB]
    if kind == AFFINE:
        det = g[UX] * g[VY] - g[VX] * g[UY]
        dx, dy = x - g[X0], y - g[Y0]
        return (dx * g[VY] - dy * g[VX]) / det, (g[UX] * dy - g[UY] * dx) / det
    key = (np.asarray(g, np.float64).tobytes(), int(n1), int(n2), np.asarray(x, np.float64).tobytes(),
           np.asarray(y, np.float64).tobytes())
    if key not in _STYPE_CACHE:
        grid = _grid_image(g, int(n1), int(n2))
        out = [_stype_preimage(g, float(a), float(b), grid) for a, b in zip(np.ravel(x), np.ravel(y))]
        t = np.array([o[0] for o in out]).reshape(np.shape(x))
        s = np.array([o[1] for o in out]).reshape(np.shape(x))
        if len(_STYPE_CACHE) > 256:
            _STYPE_CACHE.clear()
        _STYPE_CACHE[key] = ((t - g[A0]) / g[DA], (s - g[B0]) / g[DB])
    xi, eta = _STYPE_CACHE[key]
    return (float(xi), float(eta)) if np.ndim(x) == 0 else (xi.copy(), eta.copy())


# S-type preimages of repeated queries (the same points every step)
_STYPE_CACHE = {}


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
                n1, n2 = int(ps.n1[q]), int(ps.n2[q])
                xi, eta = preimage(ps.geom[q], x, y, n1, n2)
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
