"""Seeded synthetic inputs for the FC-SDNN hot path (geometry, states, weights).

This module is shared by the FP64 oracle, the tests and the benchmark.  It
holds no arithmetic of the numerical method itself: it only lays out patches,
evaluates patch mappings and their closed-form inverse Jacobians (metric
terms), draws initial states and random network weights.  Every draw comes
from ``numpy.random.default_rng(seed)`` in a fixed order.

Geometry follows the paper's patch description: each patch is the image of
the unit square under a smooth map (Sec. 3.1, eq. for S-type patches
M(q1,q2) = l_A(q1) + q2 H nu(q1)); the grid is uniform in parameter space
(Sec. 3.2.1) with spacing h = 1/(N-1) along each direction; the metric terms
are the entries of the Jacobian of the inverse map used in the curvilinear
form of the equations (Sec. 3.3).  Initial states are the uniform Mach-M flow
(rho, u, v, p) = (1.4, M, 0, 1) of Sec. 7 plus a small seeded perturbation, or
smooth sinusoidal states on the unit square.

Field layout: every field is one "plane" holding all patches back to back;
patch p occupies [off[p], off[p] + n1[p]*n2[p]) with element (i, j) at
off[p] + j*n1[p] + i (i runs along q1 and is contiguous).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

GAMMA = 1.4
NV = 9          # boundary-vicinity / viscosity fringe width (Sec. 3.2.1, Sec. 3.4)
NF = 5          # communication fringe width (Sec. 3.4)
OVERLAP = 2 * NV + 1   # minimum overlap between neighbouring patches (Sec. 3.2.2)
ALIGN = 64      # patch offsets are rounded up to this many elements


def smooth13(n: int) -> bool:
    for p in (2, 3, 5, 7, 11, 13):
        while n % p == 0:
            n //= p
    return n == 1


def cont_points(n: int, c_min: int = 27) -> int:
    """Number C of continuation points for a line of n points.

    Smallest C >= c_min such that the periodic extension length n + C has no
    prime factor above 13 (so an exact mixed-radix FFT exists).  For n = 64
    and n = 512 this keeps C = 27 (L = 91 and 539)."""
    c = c_min
    while not smooth13(n + c):
        c += 1
    return c


@dataclass
class PatchSet:
    n1: np.ndarray            # int32 [P] points along q1
    n2: np.ndarray            # int32 [P] points along q2
    C1: np.ndarray            # int32 [P] continuation points for q1 lines
    C2: np.ndarray            # int32 [P] continuation points for q2 lines
    d: int                    # matching points per line end
    off: np.ndarray           # int64 [P] element offset of each patch in a plane
    plane: int                # elements per plane (padded)
    metric: np.ndarray        # float32 [4, plane]: dq1/dx, dq1/dy, dq2/dx, dq2/dy
    htilde: np.ndarray        # float64 [P] lower bound of the physical grid spacing
    hhat: np.ndarray          # float64 [P] upper bound of the physical grid spacing
    internal: np.ndarray      # uint8 [P, 4] internal sides: q1-, q1+, q2-, q2+
    xy: np.ndarray            # float64 [2, plane] physical coordinates
    # multi-patch annulus coupling (None for independent patches)
    nsec: int = 0
    nshell: int = 0
    dirichlet: Optional[np.ndarray] = None   # uint8 [plane]: freestream-overwrite points
    # patch maps for inter-patch interpolation (None: not described)
    # float64 [P, 5]: kind (0 Cartesian x = a0 + i da, y = b0 + j db;
    # 1 polar theta = a0 + i da, r = b0 + j db), a0, da, b0, db
    geom: Optional[np.ndarray] = None
    # no-slip adiabatic wall sides (None: none), uint8 [P, 4]: q1-, q1+, q2-, q2+
    wall: Optional[np.ndarray] = None

    @property
    def npatch(self) -> int:
        return len(self.n1)

    @property
    def npoints(self) -> int:
        return int(np.sum(self.n1.astype(np.int64) * self.n2))

    def view(self, arr: np.ndarray, p: int) -> np.ndarray:
        """[..., plane] -> [..., n2, n1] view of patch p."""
        o, a, b = int(self.off[p]), int(self.n1[p]), int(self.n2[p])
        return arr[..., o:o + a * b].reshape(arr.shape[:-1] + (b, a))

    def patch_of_shell(self, s: int, k: int) -> int:
        return k * self.nsec + s


def _offsets(n1, n2):
    off = np.zeros(len(n1), np.int64)
    acc = 0
    for p in range(len(n1)):
        off[p] = acc
        acc += int(n1[p]) * int(n2[p])
        acc = (acc + ALIGN - 1) // ALIGN * ALIGN
    return off, acc


def _polar_patches(specs, n1, n2, d, c_min):
    """specs: list of (theta0, htheta, r0, hr) for polar-sector patches.

    Patch map: x = r(q2) (cos t(q1), sin t(q1)), t = theta0 + q1*(n1-1)*htheta,
    r = r0 + q2*(n2-1)*hr.  Inverse Jacobian in closed form."""
    n1 = np.asarray(n1, np.int32)
    n2 = np.asarray(n2, np.int32)
    off, plane = _offsets(n1, n2)
    metric = np.zeros((4, plane), np.float64)
    xy = np.zeros((2, plane), np.float64)
    htl = np.zeros(len(n1))
    hht = np.zeros(len(n1))
    for p, (t0, ht, r0, hr) in enumerate(specs):
        a, b = int(n1[p]), int(n2[p])
        th = t0 + ht * np.arange(a)
        r = r0 + hr * np.arange(b)
        T, R = np.meshgrid(th, r)          # [b, a]
        span_t = (a - 1) * ht
        span_r = (b - 1) * hr
        o = int(off[p])
        sl = slice(o, o + a * b)
        xy[0, sl] = (R * np.cos(T)).ravel()
        xy[1, sl] = (R * np.sin(T)).ravel()
        metric[0, sl] = (-np.sin(T) / (R * span_t)).ravel()
        metric[1, sl] = (np.cos(T) / (R * span_t)).ravel()
        metric[2, sl] = (np.cos(T) / span_r).ravel()
        metric[3, sl] = (np.sin(T) / span_r).ravel()
        htl[p] = min(r0 * ht, hr)
        hht[p] = max((r0 + span_r) * ht, hr)
    C1 = np.array([cont_points(int(x), c_min) for x in n1], np.int32)
    C2 = np.array([cont_points(int(x), c_min) for x in n2], np.int32)
    return PatchSet(n1=n1, n2=n2, C1=C1, C2=C2, d=d, off=off, plane=plane,
                    metric=metric.astype(np.float32), htilde=htl, hhat=hht,
                    internal=np.zeros((len(n1), 4), np.uint8), xy=xy)


def annulus(nsec: int, nshell: int, n1: int, n2: int, d: int = 5, c_min: int = 27,
            r_in: float = 0.5, r_out: float = 2.0) -> PatchSet:
    """Annulus r in [r_in, r_out] covered by nsec sectors x nshell shells of
    n1 x n2 points.  Neighbouring sectors (and shells) overlap by 2*NV+1 grid
    lines and sit on a common global index lattice, so the communication
    between them is an index copy."""
    ht = 2 * np.pi / (nsec * (n1 - OVERLAP))
    hr = (r_out - r_in) / (nshell * (n2 - OVERLAP) + OVERLAP - 1)
    specs = []
    for k in range(nshell):
        for s in range(nsec):
            specs.append((s * (n1 - OVERLAP) * ht, ht, r_in + k * (n2 - OVERLAP) * hr, hr))
    ps = _polar_patches(specs, [n1] * len(specs), [n2] * len(specs), d, c_min)
    ps.nsec, ps.nshell = nsec, nshell
    for k in range(nshell):
        for s in range(nsec):
            p = ps.patch_of_shell(s, k)
            ps.internal[p] = (nsec > 1, nsec > 1, k > 0, k < nshell - 1)
    # Dirichlet freestream on the outer circle where the flow enters (x < 0)
    dm = np.zeros(ps.plane, np.uint8)
    for s in range(nsec):
        p = ps.patch_of_shell(s, nshell - 1)
        v = ps.view(dm, p)
        x = ps.view(ps.xy[0], p)
        v[-1, :] = (x[-1, :] < 0).astype(np.uint8)
    ps.dirichlet = dm
    return ps


def uneven_sectors(npatch: int, nmin: int, nmax: int, seed: int, d: int = 5,
                   c_min: int = 27) -> PatchSet:
    """Independent annulus-sector patches with side lengths drawn uniformly
    from {nmin..nmax}; each spans the angular width of one of 16 overlapping
    256-point sectors and the radial range [0.5, 2]."""
    rng = np.random.default_rng(seed)
    n1 = rng.integers(nmin, nmax + 1, npatch)
    n2 = rng.integers(nmin, nmax + 1, npatch)
    t0 = rng.uniform(0, 2 * np.pi, npatch)
    span = (2 * np.pi / 16) * 255 / 237
    specs = [(t0[p], span / (n1[p] - 1), 0.5, 1.5 / (n2[p] - 1)) for p in range(npatch)]
    return _polar_patches(specs, n1, n2, d, c_min)


def overlap_pair(n: int = 48, d: int = 5, c_min: int = 27) -> PatchSet:
    """Two overlapping patches of different kinds that are not index-aligned:
    a Cartesian patch on [-1, 0.6] x [-0.5, 0.5] whose q1+ side (x = 0.6)
    is an inter-patch side, and a polar sector theta in [-1, 1], r in
    [0.3, 1.5] whose q2- side (r = 0.3) is one; each side's fringe lies
    inside the other patch.  n x n points each."""
    n1 = np.array([n, n], np.int32)
    n2 = n1.copy()
    ps = _polar_patches([(0.0, 1.0, 0.3, 1.2 / (n - 1))] * 2, n1, n2, d, c_min)
    # patch 1: the sector
    ht, hr = 2.0 / (n - 1), 1.2 / (n - 1)
    sec = _polar_patches([(-1.0, ht, 0.3, hr)], n1[:1], n2[:1], d, c_min)
    o = int(ps.off[1])
    ps.xy[:, o:o + n * n] = sec.xy[:, :n * n]
    ps.metric[:, o:o + n * n] = sec.metric[:, :n * n]
    ps.htilde[1], ps.hhat[1] = sec.htilde[0], sec.hhat[0]
    # patch 0: Cartesian
    hx, hy = 1.6 / (n - 1), 1.0 / (n - 1)
    X, Y = np.meshgrid(-1.0 + hx * np.arange(n), -0.5 + hy * np.arange(n))
    ps.xy[0, :n * n] = X.ravel()
    ps.xy[1, :n * n] = Y.ravel()
    ps.metric[:, :n * n] = 0
    ps.metric[0, :n * n] = 1 / 1.6
    ps.metric[3, :n * n] = 1 / 1.0
    ps.htilde[0], ps.hhat[0] = min(hx, hy), max(hx, hy)
    ps.internal[0] = (0, 1, 0, 0)
    ps.internal[1] = (0, 0, 1, 0)
    ps.geom = np.array([geom_row(0, -1.0, hx, -0.5, hy), geom_row(1, -1.0, ht, 0.3, hr)])
    return ps


# patch-map rows (PatchSet.geom): kind, a0, da, b0, db, affine x0, y0, ux, uy,
# vx, vy, S-type side, mode count, then the arc's cos / sin coefficients of x
# and of y (GEOM_KMAX each)
GEOM_KMAX = 8
GEOM_LEN = 13 + 4 * GEOM_KMAX


def geom_row(kind, a0=0.0, da=1.0, b0=0.0, db=1.0, affine=(0, 0, 1, 0, 0, 1), side=1.0, cx=(), sx=(), cy=(),
             sy=()):
    """One patch map: 0 Cartesian (x, y) = (a0 + i da, b0 + j db); 1 polar
    (theta, r) = (a0 + i da, b0 + j db); 2 affine (x, y) = (x0, y0) +
    i (ux, uy) + j (vx, vy); 3 S-type (eq. param_S) l(t) + s nu(t),
    t = a0 + i da, s = b0 + j db, l(t) = sum_k (cx_k cos kt + sx_k sin kt,
    cy_k cos kt + sy_k sin kt), nu the unit normal (tangent turned by
    -90 degrees for side = +1)."""
    g = np.zeros(GEOM_LEN)
    g[:5] = kind, a0, da, b0, db
    g[5:11] = affine
    g[11] = side
    K = max(len(cx), len(sx), len(cy), len(sy))
    g[12] = K
    for o, c in ((13, cx), (13 + GEOM_KMAX, sx), (13 + 2 * GEOM_KMAX, cy), (13 + 3 * GEOM_KMAX, sy)):
        g[o:o + len(c)] = c
    return g


def _arc_derivs(g, t):
    """l, l', l'' of an S-type row's arc at t (arrays [2, ...])."""
    K = int(g[12])
    out = [np.zeros((2,) + np.shape(t)) for _ in range(3)]
    for k in range(K):
        c, s_ = np.cos(k * t), np.sin(k * t)
        for comp, (oc, os_) in enumerate(((13, 13 + GEOM_KMAX), (13 + 2 * GEOM_KMAX, 13 + 3 * GEOM_KMAX))):
            a, b = g[oc + k], g[os_ + k]
            out[0][comp] += a * c + b * s_
            out[1][comp] += k * (-a * s_ + b * c)
            out[2][comp] += -k * k * (a * c + b * s_)
    return out


def _mapped_patch(g, n1, n2):
    """Physical points [2, n2, n1] and inverse-Jacobian metric terms
    [4, n2, n1] (dq1/dx, dq1/dy, dq2/dx, dq2/dy, with q = index / (n - 1))
    of an affine or S-type patch map, in closed form."""
    I, J = np.meshgrid(np.arange(n1, dtype=np.float64), np.arange(n2, dtype=np.float64))
    if int(g[0]) == 2:
        x0, y0, ux, uy, vx, vy = g[5:11]
        X, Y = x0 + I * ux + J * vx, y0 + I * uy + J * vy
        xq1, yq1 = np.full_like(I, ux * (n1 - 1)), np.full_like(I, uy * (n1 - 1))
        xq2, yq2 = np.full_like(I, vx * (n2 - 1)), np.full_like(I, vy * (n2 - 1))
    else:
        t, sv = g[1] + I * g[2], g[3] + J * g[4]
        l, d1, d2 = _arc_derivs(g, t)
        sd = g[11]
        nrm = np.hypot(d1[0], d1[1])
        nu = sd * np.array([d1[1], -d1[0]]) / nrm
        dot = d1[0] * d2[0] + d1[1] * d2[1]
        dnu = sd * (np.array([d2[1], -d2[0]]) / nrm - np.array([d1[1], -d1[0]]) * dot / nrm ** 3)
        X, Y = l[0] + sv * nu[0], l[1] + sv * nu[1]
        xq1, yq1 = (d1[0] + sv * dnu[0]) * g[2] * (n1 - 1), (d1[1] + sv * dnu[1]) * g[2] * (n1 - 1)
        xq2, yq2 = nu[0] * g[4] * (n2 - 1), nu[1] * g[4] * (n2 - 1)
    det = xq1 * yq2 - xq2 * yq1
    metric = np.array([yq2 / det, -xq2 / det, -yq1 / det, xq1 / det])
    return np.array([X, Y]), metric


def stype_trio(n: int = 48, d: int = 5, c_min: int = 27) -> PatchSet:
    """Three patches of the paper's kinds that overlap without shared grid
    lines: patch 0 an S-type band (eq. param_S) of width 0.5 along the arc
    t in [pi/2 - 0.6, pi/2 + 0.6] of the smooth closed curve
    l(t) = (0.6 cos t + 0.04 cos 3t, 0.4 sin t + 0.03 sin 2t), normal
    pointing away from the curve's inside; patch 1 an affine (I-type)
    parallelogram over it (rotated 8 degrees); patch 2 a small affine square
    (rotated -12 degrees) inside the band.  Internal sides: the band's outer
    side (fringe inside patch 1) and every side of patch 2 (fringe inside the
    band); the other sides are free.  n x n points each."""
    n1 = np.array([n] * 3, np.int32)
    n2 = n1.copy()
    off, plane = _offsets(n1, n2)
    span, H = 1.2, 0.5
    g0 = geom_row(3, np.pi / 2 - 0.6, span / (n - 1), 0.0, H / (n - 1), side=1.0,
                  cx=(0.0, 0.6, 0.0, 0.04), sy=(0.0, 0.4, 0.03))
    a1, a2 = np.deg2rad(8.0), np.deg2rad(-12.0)
    w1, h1 = 1.9, 0.9
    u1 = np.array([np.cos(a1), np.sin(a1)]) * w1 / (n - 1)
    v1 = np.array([-np.sin(a1), np.cos(a1)]) * h1 / (n - 1)
    c1 = np.array([0.0, 1.05]) - 0.5 * (n - 1) * (u1 + v1)
    g1 = geom_row(2, affine=(c1[0], c1[1], u1[0], u1[1], v1[0], v1[1]))
    w2 = 0.3
    u2 = np.array([np.cos(a2), np.sin(a2)]) * w2 / (n - 1)
    v2 = np.array([-np.sin(a2), np.cos(a2)]) * w2 / (n - 1)
    c2 = np.array([0.0, 0.65]) - 0.5 * (n - 1) * (u2 + v2)
    g2 = geom_row(2, affine=(c2[0], c2[1], u2[0], u2[1], v2[0], v2[1]))
    xy = np.zeros((2, plane))
    metric = np.zeros((4, plane), np.float32)
    htl = np.zeros(3)
    hht = np.zeros(3)
    for p, g in enumerate((g0, g1, g2)):
        P, M = _mapped_patch(g, n, n)
        o = int(off[p])
        xy[:, o:o + n * n] = P.reshape(2, -1)
        metric[:, o:o + n * n] = M.reshape(4, -1).astype(np.float32)
        hs = np.concatenate([np.hypot(*np.diff(P, axis=2)).ravel(), np.hypot(*np.diff(P, axis=1)).ravel()])
        htl[p], hht[p] = hs.min(), hs.max()
    C1 = np.array([cont_points(n, c_min)] * 3, np.int32)
    ps = PatchSet(n1=n1, n2=n2, C1=C1, C2=C1.copy(), d=d, off=off, plane=plane, metric=metric, htilde=htl,
                  hhat=hht, internal=np.zeros((3, 4), np.uint8), xy=xy)
    ps.internal[0] = (0, 0, 0, 1)
    ps.internal[2] = (1, 1, 1, 1)
    ps.geom = np.array([g0, g1, g2])
    return ps


def with_continuation(ps: PatchSet, C: int = 27) -> PatchSet:
    """The same patches with C continuation points on every line (the
    strict reading of the continuation length, C = 27 whatever N + C
    factors into)."""
    import dataclasses
    n = len(ps.n1)
    return dataclasses.replace(ps, C1=np.full(n, C, np.int32), C2=np.full(n, C, np.int32))


def unit_square(n: int, d: int = 5, C: int = 27) -> PatchSet:
    """One Cartesian patch on [0,1]^2 (identity metric)."""
    n1 = np.array([n], np.int32)
    off, plane = _offsets(n1, n1)
    g = np.linspace(0, 1, n)
    X, Y = np.meshgrid(g, g)
    xy = np.zeros((2, plane))
    xy[0, :n * n] = X.ravel()
    xy[1, :n * n] = Y.ravel()
    metric = np.zeros((4, plane), np.float32)
    metric[0, :n * n] = 1
    metric[3, :n * n] = 1
    h = 1.0 / (n - 1)
    return PatchSet(n1=n1, n2=n1.copy(), C1=np.array([C], np.int32), C2=np.array([C], np.int32),
                    d=d, off=off, plane=plane, metric=metric, htilde=np.array([h]),
                    hhat=np.array([h]), internal=np.zeros((1, 4), np.uint8), xy=xy)


# ---------------------------------------------------------------- states

def prim_to_cons(rho, u, v, p, gamma=GAMMA):
    """Conserved variables (rho, rho u, rho v, E) with E = p/(gamma-1) + rho|u|^2/2
    (ideal-gas closure, Sec. 2.1)."""
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)])


@dataclass
class Perturbation:
    kappa: np.ndarray   # [K, 2] integer wave vectors in physical coordinates
    psi: np.ndarray     # [K] phases
    amp: np.ndarray     # [K] amplitudes a_k

    def modes(self, xy):
        """phi_k(x) = sin(2 pi kappa_k . x + psi_k), shape [K, npts]."""
        return np.sin(2 * np.pi * (self.kappa @ xy) + self.psi[:, None])


def draw_perturbation(rng, nmodes=16, level=0.01) -> Perturbation:
    kap = []
    while len(kap) < nmodes:
        k = rng.integers(-3, 4, 2)
        if k[0] or k[1]:
            kap.append(k)
    psi = rng.uniform(0, 2 * np.pi, nmodes)
    amp = level * rng.uniform(-1, 1, nmodes) / nmodes
    return Perturbation(np.array(kap, np.float64), psi, amp)


def mach_state(ps: PatchSet, mach: float, pert: Perturbation):
    """Uniform Mach flow (1.4, M, 0, 1) with rho <- 1.4 (1 + sum a_k phi_k)."""
    rho = 1.4 * (1 + pert.amp @ pert.modes(ps.xy))
    one = np.ones_like(rho)
    e = prim_to_cons(rho, mach * one, 0 * one, one)
    return e


def freestream(mach: float, gamma=GAMMA):
    return prim_to_cons(np.float64(1.4), np.float64(mach), np.float64(0), np.float64(1), gamma)


def square_state(ps: PatchSet, rng):
    """rho = 1 + 0.1 sum_4 sin(2 pi (a x + b y) + phi), p likewise,
    u, v = sum_4 A sin(...) with A ~ U(-0.2, 0.2)."""
    x, y = ps.xy

    def draw():
        out = []
        for _ in range(4):
            while True:
                a, b = rng.integers(0, 4, 2)
                if a or b:
                    break
            out.append((a, b, rng.uniform(0, 2 * np.pi)))
        return out

    def ev(modes, amps):
        return sum(A * np.sin(2 * np.pi * (a * x + b * y) + ph) for (a, b, ph), A in zip(modes, amps))

    rho = 1 + ev(draw(), [0.1] * 4)
    p = 1 + ev(draw(), [0.1] * 4)
    u = ev(draw(), rng.uniform(-0.2, 0.2, 4))
    v = ev(draw(), rng.uniform(-0.2, 0.2, 4))
    return prim_to_cons(rho, u, v, p)


# ---------------------------------------------------------------- network

def mlp_weights(seed: int, sizes=(16, 64, 64, 4)):
    """Random-init MLP: W ~ U(+-1/sqrt(fan_in)), b likewise.  W_l has shape
    [fan_in, fan_out] (row-vector convention y = x W + b)."""
    rng = np.random.default_rng(seed)
    out = {}
    for l in range(len(sizes) - 1):
        lim = 1.0 / np.sqrt(sizes[l])
        out[f"W{l + 1}"] = rng.uniform(-lim, lim, (sizes[l], sizes[l + 1])).astype(np.float32)
        out[f"b{l + 1}"] = rng.uniform(-lim, lim, sizes[l + 1]).astype(np.float32)
    return out


# ---------------------------------------------------------------- configs

@dataclass
class Config:
    name: str
    ps: PatchSet
    u0: np.ndarray                 # float32 [4, plane]
    ref: np.ndarray                # float64 [4] reference primitive state (rho, u, v, p)
    mach: float = 0.0
    pert: Optional[Perturbation] = None
    mu_const: Optional[float] = None   # constant viscosity (no network)
    mlp: Optional[dict] = None
    steps: int = 0
    cfl: float = 0.5
    extra: dict = field(default_factory=dict)


def _f32(e, ps):
    out = np.zeros((4, ps.plane), np.float32)
    for p in range(ps.npatch):
        o = int(ps.off[p])
        n = int(ps.n1[p]) * int(ps.n2[p])
        out[:, o:o + n] = e[:, o:o + n]
    return out


def config(idx: int, n: Optional[int] = None, npatch: Optional[int] = None,
           nmax: Optional[int] = None, seed: Optional[int] = None) -> Config:
    """The five workloads.  Optional arguments shrink them for tests:
    n = points per patch side, npatch = patch count (uneven set), nmax =
    largest side of the uneven set."""
    seed = idx if seed is None else seed
    rng = np.random.default_rng(seed)
    if idx == 0:
        ps = unit_square(n or 64)
        e = square_state(ps, rng)
        return Config("c0-square-64", ps, _f32(e, ps), np.array([1.0, 0, 0, 1.0]),
                      mu_const=1e-3, steps=10)
    if idx in (1, 3):
        side = n or (256 if idx == 1 else 128)
        ps = annulus(16, 1, side, side)
        pert = draw_perturbation(rng)
        mach = 3.0
        e = mach_state(ps, mach, pert)
        return Config(f"c{idx}-annulus-16x{side}", ps, _f32(e, ps),
                      np.array([1.4, mach, 0, 1.0]), mach=mach, pert=pert,
                      mlp=mlp_weights(1000 + seed), steps=200 if idx == 1 else 40)
    if idx == 2:
        ps = uneven_sectors(npatch or 200, 48, nmax or 512, seed)
        pert = draw_perturbation(rng)
        mach = 3.0
        e = mach_state(ps, mach, pert)
        return Config(f"c2-uneven-{ps.npatch}", ps, _f32(e, ps), np.array([1.4, mach, 0, 1.0]),
                      mach=mach, pert=pert, mlp=mlp_weights(1000 + seed), steps=0)
    if idx == 4:
        side = n or 512
        ps = annulus(16, 4, side, side)
        pert = draw_perturbation(rng)
        mach = 5.0
        e = mach_state(ps, mach, pert)
        return Config(f"c4-annulus-64x{side}", ps, _f32(e, ps), np.array([1.4, mach, 0, 1.0]),
                      mach=mach, pert=pert, mlp=mlp_weights(1000 + seed), steps=100)
    raise ValueError(idx)


def paper_subpatches(nsec: int = 16, nshell: int = 1, seed: int = 5, mach: float = 3.0) -> Config:
    """The paper's production discretisation on the annulus: subpatches of
    101 x 101 points (n0 = 83 plus 2 n_v = 18 overlap points), d = 2
    matching points and C = 27 continuation points, so every line extends
    to L = 128; neighbouring subpatches overlap by 2 n_v + 1 = 19 lines.
    Mach-3 freestream state with the +-1 % density perturbation, seeded
    network weights."""
    rng = np.random.default_rng(seed)
    ps = annulus(nsec, nshell, 101, 101, d=2, c_min=27)
    pert = draw_perturbation(rng)
    e = mach_state(ps, mach, pert)
    return Config(f"paper-d2-{nsec}x{nshell}-101", ps, _f32(e, ps), np.array([1.4, mach, 0, 1.0]),
                  mach=mach, pert=pert, mlp=mlp_weights(1000 + seed), steps=100)


def overlap_config(n: int = 48, seed: int = 6, mach: float = 3.0, network: bool = False,
                   stype: bool = False) -> Config:
    """The Cartesian / polar patch pair of overlap_pair (stype=True: the
    S-type / affine trio of stype_trio) with the Mach-3 freestream state and
    its +-1 % density perturbation, seeded network weights (network=False: a
    constant viscosity instead); no Dirichlet points."""
    rng = np.random.default_rng(seed)
    ps = overlap_pair(n) if not stype else stype_trio(n)
    pert = draw_perturbation(rng)
    e = mach_state(ps, mach, pert)
    if not network:
        return Config(f"overlap-pair-{n}", ps, _f32(e, ps), np.array([1.4, mach, 0, 1.0]), mach=mach, pert=pert,
                      mu_const=2e-3, steps=10)
    return Config(f"overlap-pair-{n}", ps, _f32(e, ps), np.array([1.4, mach, 0, 1.0]), mach=mach, pert=pert,
                  mlp=mlp_weights(1000 + seed), steps=10)


def with_cylinder_wall(cfg: Config) -> Config:
    """An annulus workload whose inner circle (r = 0.5, the q2- side of the
    innermost shell) is a no-slip adiabatic wall."""
    ps = cfg.ps
    ps.wall = np.zeros((ps.npatch, 4), np.uint8)
    for s in range(ps.nsec):
        ps.wall[ps.patch_of_shell(s, 0), 2] = 1
    return cfg


def random_lines(rng, nlines: int, n: int, smooth: bool = True):
    """Seeded test lines: smooth non-periodic functions (sum of a few random
    low-frequency sinusoids plus a random polynomial) or white noise."""
    if not smooth:
        return rng.standard_normal((nlines, n))
    x = np.linspace(0, 1, n)
    out = np.zeros((nlines, n))
    for l in range(nlines):
        for _ in range(3):
            out[l] += rng.uniform(-1, 1) * np.sin(2 * np.pi * rng.uniform(0, 4) * x + rng.uniform(0, 6.3))
        out[l] += np.polyval(rng.uniform(-1, 1, 4), x)
    return out
