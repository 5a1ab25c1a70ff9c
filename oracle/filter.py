"""Spectral filter of FC expansions, FP64 (paper Sec. 4.3.1, eq. filtering).

Test infrastructure only (see oracle/__init__.py).

A line F_0..F_{N-1} is extended to length L = N + C by the FC continuation
(eq. continuation); each coefficient of the extension, at signed wavenumber
k, is multiplied by

    sigma(2k / (N + C)) = exp(-alpha (2k / (N + C))^p)

and the filtered expansion is evaluated back at the N grid points.  On a
patch the one-dimensional filter runs along q^1 for every q^2, then along q^2
for every q^1 of the result.  Once per time step (Algorithm 1: after the
viscosity, before the step size) it is applied to rho, rho u, rho v and the
temperature theta = p / rho (eq. p_T); E is not filtered but rebuilt from the
filtered fields with eq. perfect_gas_T, E = rho theta / (gamma - 1) +
|rho u|^2 / (2 rho).  The paper's values are alpha = 10, p = 14.

Readings:
  * p is an even integer, so sigma is even in k and a real line stays real;
    for an even L the single coefficient k = -L/2 (not split between +-M as
    in the paper's odd count of terms) gets sigma(-1) = exp(-alpha);
  * C = 0 (a periodic direction) filters the N samples themselves, L = N;
  * the paper filters "at every time step following the initial time": the
    step functions take the filter as an option and the caller decides which
    steps apply it.
"""
from __future__ import annotations

import numpy as np

from oracle import fcgram


def sigma(L: int, alpha: float, p: int) -> np.ndarray:
    """Filter factors of the L coefficients in FFT order (eq. filtering)."""
    if p % 2:
        raise ValueError("the filter order p must be even")
    k = np.fft.fftfreq(L) * L
    return np.exp(-alpha * (2.0 * k / L) ** p)


def filter_lines(F: np.ndarray, d: int, C: int, alpha: float, p: int, fp32: bool = False) -> np.ndarray:
    """Filter every line (last axis) of F: extend, scale the coefficients by
    sigma, evaluate at the first N points.

    fp32=True rounds the extension and the factors to FP32 and runs the
    transform pair in single precision: not the method, but the size of the
    rounding error any FP32 implementation carries (a step within d points
    of a line end gives tails up to sum |A_r Q^T| times the step)."""
    F = np.asarray(F, np.float64)
    N = F.shape[-1]
    ext = F if C == 0 else fcgram.extend(F, fcgram.continuation_matrix(d, C))
    if fp32:
        import scipy.fft
        e32 = ext.astype(np.float32)
        X = scipy.fft.fft(e32, axis=-1) * sigma(ext.shape[-1], alpha, p).astype(np.float32)
        return np.real(scipy.fft.ifft(X.astype(np.complex64), axis=-1))[..., :N].astype(np.float64)
    X = np.fft.fft(ext, axis=-1) * sigma(ext.shape[-1], alpha, p)
    return np.real(np.fft.ifft(X, axis=-1))[..., :N]


def filter_patch(x: np.ndarray, d: int, C1: int, C2: int, alpha: float, p: int) -> np.ndarray:
    """Two-dimensional filter of one patch array [..., n2, n1]: along q^1
    (last axis) first, then along q^2."""
    y = filter_lines(x, d, C1, alpha, p)
    return np.swapaxes(filter_lines(np.swapaxes(y, -1, -2), d, C2, alpha, p), -1, -2)


def theta_of(e: np.ndarray, gamma: float) -> np.ndarray:
    """Temperature theta = p / rho (eq. p_T) with p from eq. perfect_gas."""
    rho, m, n, E = e[0], e[1], e[2], e[3]
    p = (gamma - 1.0) * (E - 0.5 * (m * m + n * n) / rho)
    return p / rho


def energy_of(rho, m, n, theta, gamma: float):
    """E from rho, rho u, rho v and theta (eq. perfect_gas_T)."""
    return rho * theta / (gamma - 1.0) + 0.5 * (m * m + n * n) / rho


def filter_state_patch(e: np.ndarray, d: int, C1: int, C2: int, alpha: float, p: int,
                       gamma: float) -> np.ndarray:
    """The per-step filter of one patch's conserved state [4, n2, n1]."""
    e = np.asarray(e, np.float64)
    q = np.stack([e[0], e[1], e[2], theta_of(e, gamma)])
    f = filter_patch(q, d, C1, C2, alpha, p)
    return np.stack([f[0], f[1], f[2], energy_of(f[0], f[1], f[2], f[3], gamma)])


def filter_state(e: np.ndarray, ps, alpha: float, p: int, gamma: float) -> np.ndarray:
    """The per-step filter of a multi-patch state [4, plane] (every patch
    independently; padding between patches is left as it is)."""
    out = np.array(e, np.float64, copy=True)
    for k in range(ps.npatch):
        src = ps.view(np.asarray(e, np.float64), k)
        ps.view(out, k)[...] = filter_state_patch(src, ps.d, int(ps.C1[k]), int(ps.C2[k]), alpha, p, gamma)
    return out


# ------------------------------------------------------------ reverse mode

def filter_lines_adj(Y: np.ndarray, d: int, C: int, alpha: float, p: int) -> np.ndarray:
    """Transpose of filter_lines.  The line filter is R S E (E the extension,
    S = F^-1 diag(sigma) F the real symmetric circulant, R the restriction to
    N points), so its transpose is E^T S R^T: zero-pad, filter the padded
    line, fold the tail back through the continuation matrix."""
    Y = np.asarray(Y, np.float64)
    if C == 0:
        return filter_lines(Y, d, 0, alpha, p)
    N = Y.shape[-1]
    pad = np.concatenate([Y, np.zeros(Y.shape[:-1] + (C,))], axis=-1)
    X = np.fft.fft(pad, axis=-1) * sigma(N + C, alpha, p)
    g = np.real(np.fft.ifft(X, axis=-1))
    return fcgram.extend_adj(g, fcgram.continuation_matrix(d, C), N)


def filter_patch_adj(y: np.ndarray, d: int, C1: int, C2: int, alpha: float, p: int) -> np.ndarray:
    """Transpose of filter_patch: the q^2 pass transposed, then the q^1 pass."""
    t = np.swapaxes(filter_lines_adj(np.swapaxes(y, -1, -2), d, C2, alpha, p), -1, -2)
    return filter_lines_adj(t, d, C1, alpha, p)


def filter_state_patch_vjp(e: np.ndarray, eb: np.ndarray, d: int, C1: int, C2: int, alpha: float, p: int,
                           gamma: float) -> np.ndarray:
    """Cotangent of the state filter's input e given that of its output."""
    e = np.asarray(e, np.float64)
    eb = np.asarray(eb, np.float64)
    g1 = gamma - 1.0
    rho, m, n, E = e
    q = np.stack([rho, m, n, theta_of(e, gamma)])
    f = filter_patch(q, d, C1, C2, alpha, p)
    rf, mf, nf, tf = f
    # E' = rho' theta' / (gamma - 1) + (m'^2 + n'^2) / (2 rho')
    Eb = eb[3]
    qb = np.stack([eb[0] + Eb * (tf / g1 - 0.5 * (mf * mf + nf * nf) / (rf * rf)),
                   eb[1] + Eb * mf / rf,
                   eb[2] + Eb * nf / rf,
                   Eb * rf / g1])
    b = filter_patch_adj(qb, d, C1, C2, alpha, p)
    # theta = (gamma - 1) (E / rho - (m^2 + n^2) / (2 rho^2))
    tb = b[3]
    return np.stack([b[0] + tb * g1 * (-E / (rho * rho) + (m * m + n * n) / rho ** 3),
                     b[1] - tb * g1 * m / (rho * rho),
                     b[2] - tb * g1 * n / (rho * rho),
                     tb * g1 / rho])


def filter_state_vjp(e: np.ndarray, eb: np.ndarray, ps, alpha: float, p: int, gamma: float) -> np.ndarray:
    """Cotangent of filter_state's input (padding between patches passes
    through unchanged, as the forward map leaves it)."""
    out = np.array(eb, np.float64, copy=True)
    for k in range(ps.npatch):
        ps.view(out, k)[...] = filter_state_patch_vjp(ps.view(np.asarray(e, np.float64), k),
                                                      ps.view(np.asarray(eb, np.float64), k), ps.d,
                                                      int(ps.C1[k]), int(ps.C2[k]), alpha, p, gamma)
    return out
