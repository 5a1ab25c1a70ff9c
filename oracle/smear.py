"""Localized discontinuity-smearing of initial data, FP64 (paper Sec. 4.3.2,
eqs. q and qf).

Test infrastructure only (see oracle/__init__.py).

Before time stepping, every line of a subpatch that crosses a discontinuity
of the initial data is blended with a strongly filtered copy of itself near
the discontinuity:

    F_sm = w F~ + (1 - w) F,

F~ the line filtered by eq. filtering with alpha = 10, p = 2 (see
oracle.filter), w a window centred on the discontinuity (eq. qf, c = 18,
r = 9 grid spacings).  It is applied along q^1 for every q^2, then along
q^2 for every q^1 of the result, to rho, rho u, rho v and theta = p / rho;
E is rebuilt from those with eq. perfect_gas_T, as in the per-step filter.

Readings:
  * the initial data is described by a region label per grid point
    (smooth within a region, discontinuous across regions); a line has a
    discontinuity between neighbours j and j + 1 whose labels differ,
    located at z = j + 1/2 (grid units);
  * distances are in grid units of the line's own direction, so the window
    of eq. qf reads, for a distance s from z,
        1                                   s < c/2,
        cos^2(pi (s - c/2) / (2 r))          c/2 <= s <= c/2 + r,
        0                                   s > c/2 + r;
    the printed denominator r h would make the window return to 1 at the
    outer edge of its support, so 2 r h is taken (the same reading as for
    the smoothing window of the viscosity operator);
  * two windows overlap when their open supports intersect, i.e. when their
    centres are less than c + 2 r apart; a group of overlapping windows (the
    transitive closure) is replaced by one window that is 1 from the
    plateau start of its leftmost member to the plateau end of its
    rightmost member and follows those two members' rises outside;
  * a line without a discontinuity has w = 0 and is left as it is; E is
    rebuilt at every point of every patch, so away from discontinuities it
    changes by rounding only.
"""
from __future__ import annotations

import numpy as np

from oracle import filter as flt

ALPHA, P_ORDER, C_WIN, R_WIN = 10.0, 2, 18.0, 9.0


def rise(s, c: float = C_WIN, r: float = R_WIN):
    """Window value at distance s (grid units) from one discontinuity."""
    s = np.asarray(s, np.float64)
    out = np.where(s < c / 2, 1.0, np.cos(np.pi * (s - c / 2) / (2 * r)) ** 2)
    return np.where(s > c / 2 + r, 0.0, out)


def jumps_of(labels) -> np.ndarray:
    """Discontinuity positions z = j + 1/2 of one line of region labels."""
    lab = np.asarray(labels)
    return np.nonzero(lab[1:] != lab[:-1])[0] + 0.5


def window(labels, c: float = C_WIN, r: float = R_WIN) -> np.ndarray:
    """Window of one line (eq. qf with the grouping rule)."""
    n = len(labels)
    z = jumps_of(labels)
    w = np.zeros(n)
    if len(z) == 0:
        return w
    x = np.arange(n, dtype=np.float64)
    # groups: consecutive discontinuities closer than c + 2 r
    groups, start = [], 0
    for k in range(1, len(z) + 1):
        if k == len(z) or z[k] - z[k - 1] >= c + 2 * r:
            groups.append((z[start], z[k - 1]))
            start = k
    for zl, zr in groups:
        wg = np.where(x < zl, rise(zl - x, c, r), np.where(x > zr, rise(x - zr, c, r), 1.0))
        w = np.maximum(w, wg)   # supports of different groups are disjoint
    return w


def smear_lines(F: np.ndarray, labels: np.ndarray, d: int, C: int, alpha: float = ALPHA, p: int = P_ORDER,
                c: float = C_WIN, r: float = R_WIN, fp32: bool = False) -> np.ndarray:
    """Eq. q on every line (last axis) of F [..., nlines, N] with the region
    labels of those lines [nlines, N] (fp32: the filter's FP32 emulation,
    see oracle.filter.filter_lines)."""
    F = np.asarray(F, np.float64)
    Ft = flt.filter_lines(F, d, C, alpha, p, fp32)
    w = np.stack([window(lab, c, r) for lab in np.asarray(labels)])
    return w * Ft + (1.0 - w) * F


def smear_state_patch(e: np.ndarray, labels: np.ndarray, d: int, C1: int, C2: int, gamma: float,
                      alpha: float = ALPHA, p: int = P_ORDER, c: float = C_WIN, r: float = R_WIN,
                      fp32: bool = False) -> np.ndarray:
    """Smearing of one patch's state [4, n2, n1] with labels [n2, n1]: along
    q^1 (rows), then along q^2 (columns) of the result; E rebuilt."""
    e = np.asarray(e, np.float64)
    q = np.stack([e[0], e[1], e[2], flt.theta_of(e, gamma)])
    q = smear_lines(q, labels, d, C1, alpha, p, c, r, fp32)
    qt = smear_lines(np.swapaxes(q, -1, -2), np.asarray(labels).T, d, C2, alpha, p, c, r, fp32)
    q = np.swapaxes(qt, -1, -2)
    return np.stack([q[0], q[1], q[2], flt.energy_of(q[0], q[1], q[2], q[3], gamma)])


def smear_state(e: np.ndarray, labels: np.ndarray, ps, gamma: float, alpha: float = ALPHA, p: int = P_ORDER,
                c: float = C_WIN, r: float = R_WIN, fp32: bool = False) -> np.ndarray:
    """Smearing of a multi-patch state [4, plane] with region labels [plane]
    (every patch on its own grid; padding between patches kept)."""
    out = np.array(e, np.float64, copy=True)
    for k in range(ps.npatch):
        src = ps.view(np.asarray(e, np.float64), k)
        lab = ps.view(np.asarray(labels), k)
        ps.view(out, k)[...] = smear_state_patch(src, lab, ps.d, int(ps.C1[k]), int(ps.C2[k]), gamma,
                                                 alpha, p, c, r, fp32)
    return out
