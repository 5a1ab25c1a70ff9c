"""FC-Gram Fourier continuation and FC differentiation, FP64 (paper Sec. 2.2).

Test infrastructure only (see oracle/__init__.py).

The paper (eq. "continuation") extends the N samples F_0..F_{N-1} of a line,
h = 1/(N-1), by C values at the points N h, ..., (N+C-1) h:

    F^c = [ F ; A_l Q^T F_l + A_r Q^T F_r ],

F_l / F_r = first / last d samples, Q a d x d orthogonal matrix and A_l, A_r
C x d matrices "computed once and stored".  The derivative (eq. "fc_der") is
obtained by FFT of F^c, multiplication of coefficient k by 2 pi i k / beta
with beta = (N+C) h the period, inverse FFT and restriction to the first N
points.

Readings (the paper defers the construction of Q, A_l, A_r to its refs.):
  * Q: the Gram basis of the d matching points, i.e. Q from the QR
    factorisation V = Q R of the d x d Vandermonde matrix V[j,k] = j^k
    (points t = 0..d-1 in units of h).  Column k of Q holds the values of the
    k-th discrete-orthonormal (Gram) polynomial p_k(t) = sum_m t^m (R^-1)[m,k].
  * A_r column k: the "blend-to-zero" continuation of p_k.  A trigonometric
    polynomial T_k(t) = c_0 + sum_{n=1..K} c_n cos(2 pi n t/P) + s_n sin(2 pi n t/P)
    of period P = 2(d + C) is fitted in the least-squares sense to p_k on the
    matching interval [0, d-1] and to 0 on the zero interval [d+C, 2d+C-1]
    (where the first d samples of the next period sit), both sampled at
    spacing 1/NOS.  A_r[m, k] = T_k(d + m), m = 0..C-1.  K = 18, NOS = 20.
    The fit is computed in 40-digit arithmetic (mpmath) and rounded to FP64.
  * A_l by mirror symmetry: the left blend of F_l is the reversed right blend
    of reversed F_l, i.e. (A_l Q^T)[m, j] = (A_r Q^T)[C-1-m, d-1-j].
  * beta = (N + C) h with h = 1/(N-1); k runs over fftfreq order; for even
    L = N + C the Nyquist coefficient of the derivative is set to zero (so the
    derivative of a real line is real and the periodic operator is exactly
    antisymmetric).
"""
from __future__ import annotations

import functools
import os

import numpy as np

FC_K = 18       # trigonometric modes in the blend-to-zero fit
FC_NOS = 20     # samples per grid interval in the fit
FC_DPS = 40     # working decimal digits of the fit
FFT_WORKERS = -1  # host threads of the library FFT (-1: all; a process pool sets 1 per worker)

_TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "tests", "golden", "fc_tables.npz")


def gram_basis(d: int, dps: int = FC_DPS):
    """Gram basis of the points t = 0..d-1: QR of V[j,k] = j^k (mpmath)."""
    import mpmath as mp
    mp.mp.dps = dps
    V = mp.matrix(d, d)
    for j in range(d):
        for k in range(d):
            V[j, k] = mp.mpf(j) ** k
    Q, R = mp.qr(V)
    return Q, R ** -1


def build_continuation(d: int, C: int, dps: int = FC_DPS) -> np.ndarray:
    """A_r Q^T (C x d, FP64) from the least-squares blend-to-zero fit."""
    import mpmath as mp
    mp.mp.dps = dps
    Q, Rinv = gram_basis(d, dps)
    P = 2 * (d + C)
    match = [mp.mpf(i) / FC_NOS for i in range((d - 1) * FC_NOS + 1)]
    zero = [d + C + mp.mpf(i) / FC_NOS for i in range((d - 1) * FC_NOS + 1)]
    pts = match + zero
    ncol = 2 * FC_K + 1

    def trig_row(s):
        row = [mp.mpf(1)]
        for n in range(1, FC_K + 1):
            a = 2 * mp.pi * n * s / P
            row += [mp.cos(a), mp.sin(a)]
        return row

    A = mp.matrix([trig_row(s) for s in pts])
    Qa, Ra = mp.qr(A)                       # A = Qa Ra, Ra upper-triangular (rows >= ncol zero)
    evalrows = mp.matrix([trig_row(mp.mpf(d + m)) for m in range(C)])
    Ar = mp.matrix(C, d)
    for k in range(d):
        b = mp.matrix(len(pts), 1)
        for r, s in enumerate(match):
            v = mp.mpf(0)
            for m in range(d):
                v += s ** m * Rinv[m, k]
            b[r] = v                           # p_k on the matching interval, 0 on the zero interval
        y = Qa.T * b
        c = [mp.mpf(0)] * ncol
        for i in range(ncol - 1, -1, -1):      # back substitution Ra[:ncol,:ncol] c = y[:ncol]
            acc = y[i]
            for j in range(i + 1, ncol):
                acc -= Ra[i, j] * c[j]
            c[i] = acc / Ra[i, i]
        col = evalrows * mp.matrix(c)
        for m in range(C):
            Ar[m, k] = col[m]
    ArQ = Ar * Q.T
    return np.array([[float(ArQ[m, j]) for j in range(d)] for m in range(C)])


@functools.lru_cache(maxsize=None)
def _table():
    if os.path.exists(_TABLE):
        with np.load(_TABLE, allow_pickle=False) as z:
            return {k: z[k].copy() for k in z.files}
    return {}


@functools.lru_cache(maxsize=None)
def continuation_matrix(d: int, C: int) -> np.ndarray:
    """A_r Q^T for (d, C); read from the committed table written by
    oracle/make_fc_tables.py when present, else computed."""
    key = f"d{d}_C{C}"
    tab = _table()
    if key in tab:
        return tab[key]
    return build_continuation(d, C)


def left_matrix(ArQ: np.ndarray) -> np.ndarray:
    """A_l Q^T from A_r Q^T by the mirror reading."""
    return ArQ[::-1, ::-1]


def extend(F: np.ndarray, ArQ: np.ndarray) -> np.ndarray:
    """F^c = [F; A_l Q^T F_l + A_r Q^T F_r] along the last axis (eq. continuation)."""
    C, d = ArQ.shape
    tail = F[..., -d:] @ ArQ.T + F[..., :d] @ left_matrix(ArQ).T
    return np.concatenate([F, tail], axis=-1)


def dft(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Direct O(L^2) discrete Fourier transform along the last axis
    (X_k = sum_n x_n exp(-2 pi i k n / L); inverse with + sign and 1/L)."""
    L = x.shape[-1]
    n = np.arange(L)
    sgn = 1.0 if inverse else -1.0
    W = np.exp(sgn * 2j * np.pi * np.outer(n, n) / L)
    out = x @ W.T
    return out / L if inverse else out


def wavenumbers(L: int) -> np.ndarray:
    """Signed integer wavenumbers in FFT order; the Nyquist entry of an even
    length is zeroed (derivative reading)."""
    k = np.fft.fftfreq(L) * L
    if L % 2 == 0:
        k[L // 2] = 0.0
    return k


def periodic_derivative(ext: np.ndarray, period: float) -> np.ndarray:
    """Derivative of the trigonometric interpolant of a periodic sample
    vector: FFT, multiply by 2 pi i k / period, inverse FFT, real part
    (eq. fc_der).  The library FFT transforms the batch of lines on every
    host thread."""
    import scipy.fft
    L = ext.shape[-1]
    X = scipy.fft.fft(ext, axis=-1, workers=FFT_WORKERS)
    X = X * (2j * np.pi * wavenumbers(L) / period)
    return np.real(scipy.fft.ifft(X, axis=-1, workers=FFT_WORKERS))


def diff_lines(F: np.ndarray, d: int, C: int) -> np.ndarray:
    """FC derivative d/dq of lines sampled at q_j = j/(N-1), q in [0, 1].
    C = 0 means plain periodic Fourier differentiation with h = 1/N, beta = 1."""
    N = F.shape[-1]
    if C == 0:
        return periodic_derivative(F, 1.0) * 1.0
    ArQ = continuation_matrix(d, C)
    h = 1.0 / (N - 1)
    ext = extend(F, ArQ)
    return periodic_derivative(ext, (N + C) * h)[..., :N]


def extend_adj(G: np.ndarray, ArQ: np.ndarray, N: int) -> np.ndarray:
    """Transpose of the extension E = [I; T]: E^T g = g[:N] + T^T g[N:]."""
    C, d = ArQ.shape
    out = np.array(G[..., :N], copy=True)
    tail = G[..., N:]
    out[..., -d:] += tail @ ArQ
    out[..., :d] += tail @ left_matrix(ArQ)
    return out


def diff_lines_adj(Y: np.ndarray, d: int, C: int) -> np.ndarray:
    """Transpose of diff_lines.  D = R S E with R the restriction to N points,
    S the periodic spectral derivative (antisymmetric) and E the extension,
    so D^T y = E^T (-S) R^T y."""
    N = Y.shape[-1]
    if C == 0:
        return -periodic_derivative(Y, 1.0)
    ArQ = continuation_matrix(d, C)
    h = 1.0 / (N - 1)
    pad = np.concatenate([Y, np.zeros(Y.shape[:-1] + (C,))], axis=-1)
    g = -periodic_derivative(pad, (N + C) * h)
    return extend_adj(g, ArQ, N)


# ------------------------------------------------------------ multi-patch planes

def _lines(ps, x, p, direction):
    """Patch p of plane x as an array of lines along q^direction (last axis)."""
    v = ps.view(x, p)                 # [..., n2, n1]
    return v if direction == 1 else np.swapaxes(v, -1, -2)


def _put(ps, out, p, direction, lines):
    v = ps.view(out, p)
    v[...] = lines if direction == 1 else np.swapaxes(lines, -1, -2)


def diff_plane(x: np.ndarray, ps, direction: int) -> np.ndarray:
    """d/dq^direction of every patch of a field plane (or stack of planes)."""
    out = np.zeros(x.shape, np.float64)
    for p in range(ps.npatch):
        C = int(ps.C1[p] if direction == 1 else ps.C2[p])
        _put(ps, out, p, direction, diff_lines(_lines(ps, np.asarray(x, np.float64), p, direction), ps.d, C))
    return out


def diff_plane_adj(y: np.ndarray, ps, direction: int) -> np.ndarray:
    out = np.zeros(y.shape, np.float64)
    for p in range(ps.npatch):
        C = int(ps.C1[p] if direction == 1 else ps.C2[p])
        _put(ps, out, p, direction, diff_lines_adj(_lines(ps, np.asarray(y, np.float64), p, direction), ps.d, C))
    return out


def continue_plane(x: np.ndarray, ps, direction: int):
    """Extended lines per patch: list of arrays [..., nlines, N + C]."""
    res = []
    for p in range(ps.npatch):
        C = int(ps.C1[p] if direction == 1 else ps.C2[p])
        res.append(extend(_lines(ps, np.asarray(x, np.float64), p, direction), continuation_matrix(ps.d, C)))
    return res


def continue_plane_adj(ext_bars, ps, direction: int, shape) -> np.ndarray:
    out = np.zeros(shape, np.float64)
    for p in range(ps.npatch):
        C = int(ps.C1[p] if direction == 1 else ps.C2[p])
        n = int(ps.n1[p] if direction == 1 else ps.n2[p])
        _put(ps, out, p, direction, extend_adj(ext_bars[p], continuation_matrix(ps.d, C), n))
    return out
