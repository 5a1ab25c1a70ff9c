"""Pins of the oracle's localized discontinuity-smearing (paper Sec. 4.3.2,
eqs. q and qf) against facts that do not restate its code:

* the window: 1 on the plateau, exactly 1/2 halfway up the rise
  (cos^2(pi/4)), 0 beyond the support, symmetric about the discontinuity,
  and the rise is antisymmetric about its midpoint (w(m + t) + w(m - t) = 1,
  cos^2 + sin^2);
* grouping: two discontinuities closer than c + 2 r = 36 grid spacings give
  one window that is 1 all the way between them, farther apart two windows
  with a zero between them;
* a line without a discontinuity, and points farther than c/2 + r from every
  discontinuity, are left exactly as they are; within c/2 of one the line
  equals the filtered line;
* a unit step is smeared by a Gaussian: the factors exp(-10 (2k/L)^2) are
  a Gaussian of standard deviation L / sqrt(80) in the wavenumber, whose
  kernel has standard deviation s = sqrt(80) / (2 pi) grid points, so the
  largest difference between neighbours drops from 1 to the peak density
  of the smoothed step, 1 / (sqrt(2 pi) s) = 0.2803;
* a contact discontinuity (density jump at constant velocity and pressure):
  rho u and rho v are smeared with the same window and filter as rho, so
  the velocity stays constant to rounding.
"""
import numpy as np
import pytest

import synth
from oracle import smear

C, R = 18.0, 9.0


def test_rise_plateau_midpoint_support_and_complement():
    assert smear.rise(0.0) == 1.0 and smear.rise(8.99) == 1.0 and smear.rise(9.0) == 1.0
    assert abs(smear.rise(13.5) - 0.5) <= 1e-15
    assert smear.rise(18.0) <= 1e-30 and smear.rise(18.5) == 0.0 and smear.rise(40.0) == 0.0
    t = np.linspace(0, 4.5, 10)
    assert np.abs(smear.rise(13.5 + t) + smear.rise(13.5 - t) - 1).max() <= 1e-15
    s = np.linspace(0, 20, 401)
    assert np.all(np.diff(smear.rise(s)) <= 0)


def test_window_of_one_discontinuity():
    lab = np.zeros(60, np.int8)
    lab[21:] = 1                       # discontinuity at z = 20.5
    w = smear.window(lab)
    x = np.arange(60)
    assert np.all(w[np.abs(x - 20.5) < 9] == 1.0)
    assert np.all(w[np.abs(x - 20.5) > 18] == 0.0)
    assert abs(w[7] - 0.5) <= 1e-15 and abs(w[34] - 0.5) <= 1e-15   # 13.5 from z
    # symmetric about z
    for k in range(1, 20):
        assert w[20 - k + 1] == w[20 + k]


def test_grouping_of_nearby_discontinuities():
    x = np.arange(100)
    lab = np.zeros(100, np.int8)
    lab[21:41] = 1                     # z = 20.5 and 40.5: 20 apart (< 36)
    w = smear.window(lab)
    assert np.all(w[(x > 11.5) & (x < 49.5)] == 1.0)
    assert abs(w[7] - 0.5) <= 1e-15 and abs(w[54] - 0.5) <= 1e-15
    lab = np.zeros(100, np.int8)
    lab[21:61] = 1                     # 40 apart: two windows
    w = smear.window(lab)
    assert w[40] == 0.0 and w[41] == 0.0
    assert abs(w[34] - 0.5) <= 1e-15 and abs(w[47] - 0.5) <= 1e-15


def test_lines_untouched_far_from_and_filtered_near_discontinuities():
    from oracle import filter as flt
    rng = np.random.default_rng(8)
    N, Cc = 120, 28
    F = synth.random_lines(rng, 3, N)
    lab = np.zeros((3, N), np.int8)
    lab[1, 60:] = 2                    # line 1: discontinuity at 59.5
    out = smear.smear_lines(F, lab, 5, Cc)
    assert np.array_equal(out[0], F[0]) and np.array_equal(out[2], F[2])
    x = np.arange(N)
    far = np.abs(x - 59.5) > 18
    assert np.array_equal(out[1, far], F[1, far])
    near = np.abs(x - 59.5) < 9
    Ft = flt.filter_lines(F[1], 5, Cc, 10.0, 2)
    assert np.abs(out[1, near] - Ft[near]).max() <= 1e-15 * np.abs(Ft).max()


@pytest.mark.parametrize("N", [101, 256])
def test_unit_step_is_smeared_over_a_few_points(N):
    lab = (np.arange(N) >= N // 2).astype(np.int8)
    f = lab.astype(np.float64)
    g = smear.smear_lines(f[None], lab[None], 2 if N == 101 else 5, 27)[0]
    jumps = np.abs(np.diff(g))
    s = np.sqrt(80.0) / (2 * np.pi)
    assert abs(jumps.max() - 1 / (np.sqrt(2 * np.pi) * s)) < 2e-3
    # the rest of the line is (nearly) flat; both ends are untouched
    assert np.array_equal(g[:N // 2 - 19], f[:N // 2 - 19]) and np.array_equal(g[N // 2 + 19:], f[N // 2 + 19:])


def test_contact_discontinuity_keeps_velocity_constant():
    gamma = 1.4
    ps = synth.unit_square(64)
    n = 64
    xy = ps.xy[:, :n * n].reshape(2, n, n)
    inside = (xy[0] - 0.45) ** 2 + (xy[1] - 0.55) ** 2 < 0.2 ** 2
    lab = inside.astype(np.int8)
    rho = np.where(inside, 2.0, 1.0)
    u, v, p = 0.3, -0.2, 1.0
    e = np.stack([rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)])
    out = smear.smear_state_patch(e, lab, 5, 27, 27, gamma)
    assert np.abs(out[1] / out[0] - u).max() <= 1e-13
    assert np.abs(out[2] / out[0] - v).max() <= 1e-13
    # density was smeared across the circle, and only near it
    assert np.abs(out[0] - rho).max() > 0.1
    far = np.abs(np.hypot(xy[0] - 0.45, xy[1] - 0.55) - 0.2) > 0.4
    assert np.abs(out[0][far] - rho[far]).max() <= 1e-13


def test_state_without_discontinuities_is_unchanged():
    cfg = synth.config(1, n=48)
    ps = cfg.ps
    e = cfg.u0.astype(np.float64)
    out = smear.smear_state(e, np.zeros(ps.plane, np.int8), ps, 1.4)
    for k in range(ps.npatch):
        a, b = ps.view(out, k), ps.view(e, k)
        assert np.array_equal(a[:3], b[:3])
        assert np.abs(a[3] - b[3]).max() <= 1e-14 * np.abs(b[3]).max()
