"""Pins of the oracle's spectral filter (paper Sec. 4.3.1, eq. filtering)
against closed forms and invariants that do not restate its code:

* periodic direction (C = 0): a single Fourier mode cos(2 pi k0 j / N + phi)
  comes back multiplied by exp(-alpha (2 k0 / N)^p), the Nyquist mode of an
  even N by exp(-alpha); on a doubly periodic patch a product mode by the
  product of the two factors (the two one-dimensional passes and their
  directions);
* FC direction (C > 0): a smooth, well-resolved non-periodic line is left
  unchanged to 1e-9, and the change of a less resolved one decays fast with
  N (the extension is smooth, so its coefficients near the filtered band
  are negligible: a wrong or missing continuation would put a jump into the
  periodic extension and change the line at the 1e-3 level), while a line
  with a jump loses its high frequencies;
* alpha = 0 is the identity;
* reverse mode: <F x, y> = <x, F^T y> for the two-dimensional filter
  (periodic and FC directions), and the state filter's vector-Jacobian
  product against central differences;
* the state filter on a doubly periodic patch with constant velocity and
  single-mode rho and theta = p / rho: rho and theta are filtered as single
  modes, rho u = u rho stays u times the filtered rho, and E is
  rho theta / (gamma - 1) + rho |u|^2 / 2 of the filtered fields (eqs. p_T,
  perfect_gas_T) -- pins the temperature and the rebuilt energy.
"""
import numpy as np
import pytest

from oracle import filter as flt

ALPHA, P = 10.0, 14


@pytest.mark.parametrize("N", [16, 17, 64, 101])
def test_periodic_single_modes(N):
    j = np.arange(N)
    for k0 in range(0, N // 2 + 1):
        f = np.cos(2 * np.pi * k0 * j / N + 0.3)
        if 2 * k0 == N:   # the Nyquist mode of an even N is a pure cosine
            f = np.cos(np.pi * j)
        want = np.exp(-ALPHA * (2.0 * k0 / N) ** P) * f
        got = flt.filter_lines(f, 5, 0, ALPHA, P)
        assert np.abs(got - want).max() <= 1e-13


def test_nyquist_factor_and_monotone_sigma():
    s = flt.sigma(64, ALPHA, P)
    assert s[0] == 1.0 and abs(s[32] - np.exp(-ALPHA)) <= 1e-16
    half = s[:33]
    assert np.all(np.diff(half) <= 0)
    with pytest.raises(ValueError):
        flt.sigma(64, ALPHA, 3)


def test_doubly_periodic_product_mode():
    n1, n2 = 24, 30
    j2, j1 = np.meshgrid(np.arange(n2), np.arange(n1), indexing="ij")
    for k1, k2 in [(1, 2), (7, 11), (12, 3), (5, 15)]:
        x = np.cos(2 * np.pi * (k1 * j1 / n1 + k2 * j2 / n2))
        want = np.exp(-ALPHA * (2.0 * k1 / n1) ** P) * np.exp(-ALPHA * (2.0 * k2 / n2) ** P) * x
        got = flt.filter_patch(x, 5, 0, 0, ALPHA, P)
        assert np.abs(got - want).max() <= 1e-13


@pytest.mark.parametrize("N,C", [(128, 28), (256, 30), (512, 27)])
def test_fc_filter_leaves_smooth_lines(N, C):
    x = np.linspace(0.0, 1.0, N)
    for f in (np.sin(3.3 * x + 0.4), 1.0 + x ** 3):
        got = flt.filter_lines(f, 5, C, ALPHA, P)
        assert np.abs(got - f).max() <= 1e-9 * np.abs(f).max()


def test_fc_filter_change_vanishes_with_resolution():
    """exp(sin(5.4 pi x - 2.7 pi) - cos 2 pi x) has coefficients that reach
    the filtered band at coarse grids: the change decays fast with N."""
    errs = []
    for N, C in [(128, 28), (256, 30), (512, 27)]:
        x = np.linspace(0.0, 1.0, N)
        f = np.exp(np.sin(5.4 * np.pi * x - 2.7 * np.pi) - np.cos(2 * np.pi * x))
        errs.append(np.abs(flt.filter_lines(f, 5, C, ALPHA, P) - f).max() / np.abs(f).max())
    assert errs[0] < 1e-6 and errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10 and errs[2] < 1e-9


def test_fc_filter_damps_a_jump():
    N, C = 200, 30
    f = np.where(np.arange(N) < 90, 1.0, 0.0)
    g = flt.filter_lines(f, 5, C, ALPHA, P)
    # high-frequency content of the line is removed: its differences shrink
    assert np.abs(np.diff(g)).max() < 0.9 * np.abs(np.diff(f)).max()
    assert np.abs(g[:70] - 1).max() < 0.05 and np.abs(g[110:]).max() < 0.05


def test_alpha_zero_is_identity():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((3, 77))
    # rounding of the FFT pair relative to the extension (random data has a
    # tail up to |A_r Q^T| ~ 1e4 times its size)
    assert np.abs(flt.filter_lines(f, 5, 31, 0.0, P) - f).max() <= 1e-10
    assert np.abs(flt.filter_lines(f, 5, 0, 0.0, P) - f).max() <= 1e-13


def test_state_filter_constant_velocity_closed_form():
    gamma = 1.4
    n1, n2 = 32, 20
    j2, j1 = np.meshgrid(np.arange(n2), np.arange(n1), indexing="ij")
    u, v = 0.7, -0.2
    ka, kb = (3, 2), (9, 5)
    ma = np.cos(2 * np.pi * (ka[0] * j1 / n1 + ka[1] * j2 / n2))
    mb = np.sin(2 * np.pi * (kb[0] * j1 / n1 + kb[1] * j2 / n2))
    rho = 1.2 + 0.1 * ma
    theta = 0.9 + 0.05 * mb
    p = rho * theta
    e = np.stack([rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)])
    sa = np.exp(-ALPHA * (2.0 * ka[0] / n1) ** P) * np.exp(-ALPHA * (2.0 * ka[1] / n2) ** P)
    sb = np.exp(-ALPHA * (2.0 * kb[0] / n1) ** P) * np.exp(-ALPHA * (2.0 * kb[1] / n2) ** P)
    rho_f = 1.2 + 0.1 * sa * ma
    theta_f = 0.9 + 0.05 * sb * mb
    want = np.stack([rho_f, u * rho_f, v * rho_f,
                     rho_f * theta_f / (gamma - 1) + 0.5 * rho_f * (u * u + v * v)])
    got = flt.filter_state_patch(e, 5, 0, 0, ALPHA, P, gamma)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


# ------------------------------------------------------------ reverse mode

@pytest.mark.parametrize("C1,C2", [(0, 0), (27, 30), (31, 0)])
def test_patch_filter_transpose_dot_product(C1, C2):
    rng = np.random.default_rng(C1 + 7 * C2)
    n1, n2 = 40, 33
    x = rng.standard_normal((n2, n1))
    y = rng.standard_normal((n2, n1))
    lhs = np.sum(flt.filter_patch(x, 5, C1, C2, ALPHA, P) * y)
    rhs = np.sum(x * flt.filter_patch_adj(y, 5, C1, C2, ALPHA, P))
    # random lines have extension tails up to |A_r Q^T| ~ 1e4 times their
    # size, so FP64 rounding of the FFT pair reaches ~1e-11 here
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_state_filter_vjp_central_differences():
    gamma = 1.4
    rng = np.random.default_rng(5)
    n1, n2 = 36, 30
    j2, j1 = np.meshgrid(np.arange(n2) / (n2 - 1), np.arange(n1) / (n1 - 1), indexing="ij")
    rho = 1.0 + 0.2 * np.sin(2.1 * j1 + 1.3 * j2) + 0.01 * rng.standard_normal((n2, n1))
    u = 0.5 + 0.1 * np.cos(1.7 * j2)
    v = -0.2 + 0.1 * np.sin(2.3 * j1)
    pr = 1.0 + 0.1 * np.cos(3.0 * j1 * j2)
    e = np.stack([rho, rho * u, rho * v, pr / (gamma - 1) + 0.5 * rho * (u * u + v * v)])
    eb = rng.standard_normal(e.shape)
    g = flt.filter_state_patch_vjp(e, eb, 5, 27, 28, ALPHA, P, gamma)
    for _ in range(3):
        de = rng.standard_normal(e.shape)
        h = 1e-6
        fp = flt.filter_state_patch(e + h * de, 5, 27, 28, ALPHA, P, gamma)
        fm = flt.filter_state_patch(e - h * de, 5, 27, 28, ALPHA, P, gamma)
        fd = np.sum((fp - fm) * eb) / (2 * h)
        an = np.sum(g * de)
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_fp32_emulation_is_rounding_only():
    """The FP32 emulation (used for parity bars, not a method) differs from
    the FP64 filter by single-precision rounding on smooth lines, and by
    ~eps32 times the continuation tail for a step that sits at a line end
    (the tail is then thousands of times the step)."""
    rng = np.random.default_rng(6)
    from oracle import fcgram
    import synth
    F = synth.random_lines(rng, 4, 150)
    a = flt.filter_lines(F, 5, 27, ALPHA, 2)
    b = flt.filter_lines(F, 5, 27, ALPHA, 2, fp32=True)
    assert 0 < np.abs(a - b).max() <= 1e-6 * np.abs(a).max()
    step = np.zeros(150)
    step[-3:] = 1.0
    big = np.abs(flt.filter_lines(step, 5, 27, ALPHA, 2) - flt.filter_lines(step, 5, 27, ALPHA, 2, fp32=True)).max()
    amp = np.abs(fcgram.extend(step, fcgram.continuation_matrix(5, 27))).max()   # the tail, ~2.5e3
    assert amp > 1e3 and 1e-8 * amp < big < 1e-6 * amp
