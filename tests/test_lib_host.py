"""CPU checks of libfcsdnn.so: it loads, exports every symbol the header
declares, and its host-side precomputation (continuation matrices, radix
plans, digit-reversed multiplier tables, patch validation) agrees with the
oracle and with a plain numpy DFT.  No device is needed."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import fcgram

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcsdnn.h")


@pytest.fixture(scope="module")
def L():
    from paper_2506_16076_amd import _lib
    return _lib


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:fcsd_status|const char\*|void\*)\s+(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function(L):
    lib = L.lib()
    declared = header_functions()
    assert len(declared) >= 30
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(L.EXPORTS)
    assert lib.fcsd_version().startswith(b"fcsdnn")


def test_context_without_device_reports_edevice(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    assert L.lib().fcsd_ctx_create(0, None, ctypes.byref(h)) == 3


@pytest.mark.parametrize("C", list(range(27, 46)))
def test_continuation_matrix_matches_oracle(L, C):
    lib_m = L.fc_matrix(5, C)
    ora = fcgram.continuation_matrix(5, C)
    assert np.abs(lib_m - ora).max() <= 1e-12 * np.abs(ora).max()


def test_fft_plans(L):
    for Lx in range(8, 600):
        if not synth.smooth13(Lx):
            with pytest.raises(L.FcsdError):
                L.fft_plan(Lx)
            continue
        r = L.fft_plan(Lx)
        assert int(np.prod(r)) == Lx and set(r) <= set(range(2, 17)) and 1 <= len(r) <= 8
        # composite radices: never more stages than the prime factorisation
        n, primes = Lx, 0
        for p in (2, 3, 5, 7, 11, 13):
            while n % p == 0:
                n //= p
                primes += 1
        assert len(r) <= primes


def _twiddles(lib, n):
    out = np.zeros(2 * n, np.float32)
    lib.fcsd_host_twiddles(ctypes.c_int(n), out.ctypes.data_as(ctypes.c_void_p))
    return out[0::2].astype(np.float64) + 1j * out[1::2]


def _kmul(lib, N, n, rad, periodic=0):
    out = np.zeros(2 * n, np.float32)
    r = (ctypes.c_int * 8)(*rad)
    lib.fcsd_host_kmul(ctypes.c_int(N), ctypes.c_int(n), ctypes.c_int(len(rad)), r,
                       out.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(periodic))
    return out[0::2].astype(np.float64) + 1j * out[1::2]


def _dmatrix(lib, d, C):
    out = np.zeros((C + 1) * 2 * d)
    assert lib.fcsd_host_fc_dmatrix(ctypes.c_int(d), ctypes.c_int(C), out.ctypes.data_as(ctypes.c_void_p)) == 0
    return out.reshape(C + 1, 2 * d)


@pytest.mark.parametrize("C", [27, 31, 45])
def test_differenced_continuation_rows(L, C):
    """Row r of the differenced table applied to the 2d end samples equals
    ext[N+r] - ext[N-1+r] of the oracle's extension (ext[L] = ext[0])."""
    lib = L.lib()
    Dq = _dmatrix(lib, 5, C)
    rng = np.random.default_rng(C)
    F = synth.random_lines(rng, 3, 40)
    ArQ = L.fc_matrix(5, C)
    for f in F:
        ext = fcgram.extend(f, ArQ)
        N = len(f)
        per = np.concatenate([ext, ext[:1]])
        want = per[N:] - per[N - 1:-1]
        got = Dq @ np.concatenate([f[N - 5:], f[:5]])
        assert np.abs(got - want).max() <= 1e-12 * np.abs(ext).max() * np.abs(ArQ).max()


def emulate_engine(x, rad, tw, inverse):
    """numpy replay of the device stage loop: in-place decimation in
    frequency (forward) / in time (inverse) with the library's twiddles."""
    z = np.array(x, np.complex128)
    n = len(z)
    order = range(len(rad)) if not inverse else range(len(rad) - 1, -1, -1)
    Ms = []
    M = n
    for r in rad:
        Ms.append(M)
        M //= r
    for s in order:
        R, M = rad[s], Ms[s]
        m, stride = M // R, n // M
        W = np.exp((1j if inverse else -1j) * 2 * np.pi * np.outer(np.arange(R), np.arange(R)) / R)
        for b in range(n // R):
            blk, j = divmod(b, m)
            idx = blk * M + j + m * np.arange(R)
            v = z[idx]
            tws = tw[(stride * j * np.arange(R)) % n]
            if inverse:
                v = W @ (v * np.conj(tws))
            else:
                v = (W @ v) * tws
            z[idx] = v
    return z


@pytest.mark.parametrize("Lx,N", [(91, 64), (156, 128), (286, 256), (539, 512), (64, 64), (120, 93)])
def test_digit_reversed_engine_and_multiplier_table(L, Lx, N):
    lib = L.lib()
    rad = L.fft_plan(Lx)
    tw = _twiddles(lib, Lx)
    assert np.abs(tw - np.exp(-2j * np.pi * np.arange(Lx) / Lx)).max() < 1e-7
    rng = np.random.default_rng(Lx)
    x = rng.standard_normal(Lx) + 1j * rng.standard_normal(Lx)
    X = np.fft.fft(x)
    Y = emulate_engine(x, rad, np.exp(-2j * np.pi * np.arange(Lx) / Lx), False)
    km = _kmul(lib, N, Lx, rad)
    # the multiplier is i w_k / (exp(2 pi i k / L) - 1), w_k = 2 pi k (N-1) / L^2:
    # recover the wavenumber of every position from it
    scale = 2 * np.pi * (N - 1) / Lx ** 2
    kk = np.zeros(Lx, int)
    for p in range(Lx):
        if km[p] == 0:
            continue
        cand = np.arange(1, Lx)
        ks = np.where(cand <= Lx // 2, cand, cand - Lx)
        sym = 1j * scale * ks / (np.exp(2j * np.pi * cand / Lx) - 1)
        i = int(np.argmin(np.abs(sym - km[p])))
        assert abs(sym[i] - km[p]) <= 1e-6 * abs(sym[i])
        kk[p] = cand[i]
    zero = km == 0
    if Lx % 2 == 0:
        assert zero.sum() == 2          # k = 0 and the zeroed Nyquist
    else:
        assert zero.sum() == 1 and sorted(kk[~zero]) == list(range(1, Lx))
    ok = ~zero
    assert np.abs(Y[ok] - X[kk[ok]]).max() <= 1e-10 * np.abs(X).max()
    # the inverse pass returns L x in natural order
    back = emulate_engine(Y, rad, np.exp(-2j * np.pi * np.arange(Lx) / Lx), True)
    assert np.abs(back / Lx - x).max() <= 1e-12 * np.abs(x).max()
    # derivative through the emulated engine (differenced extension, complex
    # multipliers) equals the oracle's FC derivative, and the transposed
    # sequence (Delta^T, conjugate multipliers, fold) its transpose
    if Lx > N:
        C = Lx - N
        F = synth.random_lines(rng, 2, N)
        ArQ = L.fc_matrix(5, C)
        Dq = _dmatrix(lib, 5, C)
        f = F[0] + 1j * F[1]
        dz = np.concatenate([f[1:] - f[:-1], Dq @ np.concatenate([f[N - 5:], f[:5]])])
        Z = emulate_engine(dz, rad, tw, False)
        d = emulate_engine(km * Z, rad, tw, True)[:N]
        want = fcgram.diff_lines(F, 5, C)
        assert np.abs(d.real - want[0]).max() <= 1e-5 * np.abs(want[0]).max()
        assert np.abs(d.imag - want[1]).max() <= 1e-5 * np.abs(want[1]).max()
        # the transpose amplifies table rounding by |A_r Q^T| ~ 1e4 at the
        # folded samples: check the sequence with exact tables
        ks = np.where(kk <= Lx // 2, kk, kk - Lx)
        with np.errstate(all="ignore"):
            km_ex = np.where(zero, 0, 1j * scale * ks / (np.exp(2j * np.pi * kk / Lx) - 1))
        tw_ex = np.exp(-2j * np.pi * np.arange(Lx) / Lx)
        y = synth.random_lines(rng, 2, N)
        yz = np.concatenate([y[0] + 1j * y[1], np.zeros(C)])
        dty = np.roll(yz, 1) - yz
        t = emulate_engine(np.conj(km_ex) * emulate_engine(dty, rad, tw_ex, False), rad, tw_ex, True)
        want_adj = fcgram.diff_lines_adj(y, 5, C)
        got = t[:N].copy()
        tail = t[N:]
        got[N - 5:] += ArQ.T @ tail
        got[:5] += fcgram.left_matrix(ArQ).T @ tail
        assert np.abs(got.real - want_adj[0]).max() <= 1e-9 * np.abs(want_adj[0]).max()
        assert np.abs(got.imag - want_adj[1]).max() <= 1e-9 * np.abs(want_adj[1]).max()


def test_patch_validation(L):
    ps = synth.uneven_sectors(5, 48, 120, 3)
    descs = L.patch_descs(ps.n1, ps.n2, ps.C1, ps.C2, ps.off, ps.hhat, ps.htilde, ps.internal)
    assert L.validate_patches(descs, 5, ps.plane)[0] == 0
    end = int(ps.off[-1] + ps.n1[-1] * ps.n2[-1])
    assert L.validate_patches(descs, 5, end)[0] == 0
    assert L.validate_patches(descs, 5, end - 1)[0] == 1                  # outside the plane
    # extension lengths with a prime factor above 13 run embedded in a longer
    # 13-smooth transform: accepted, unless that transform exceeds 8192
    emb = L.patch_descs(ps.n1, ps.n2, 17 * 7 - ps.n1, ps.C2, ps.off, ps.hhat, ps.htilde, ps.internal)
    assert L.validate_patches(emb, 5, ps.plane)[0] == 0
    big = L.patch_descs([4096], [50], [27], [27], [0], [0.1], [0.1], [[0, 0, 0, 0]])
    rc, msg = L.validate_patches(big, 5, 4096 * 50)
    assert rc == 5 and "prime factor above 13" in msg
    over = L.patch_descs(ps.n1, ps.n2, ps.C1, ps.C2, np.zeros(5, np.int64), ps.hhat, ps.htilde, ps.internal)
    assert L.validate_patches(over, 5, ps.plane)[0] == 1                  # overlapping patches
    tiny = L.patch_descs([9], [40], [27], [27], [0], [0.1], [0.1], [[0, 0, 0, 0]])
    assert L.validate_patches(tiny, 5, 10000)[0] == 1                     # n < 2d + 1
    ann = synth.annulus(4, 2, 48, 40)
    descs = L.patch_descs(ann.n1, ann.n2, ann.C1, ann.C2, ann.off, ann.hhat, ann.htilde, ann.internal)
    assert L.validate_patches(descs, 5, ann.plane, 4, 2)[0] == 0
    assert L.validate_patches(descs, 5, ann.plane, 3, 2)[0] == 1


def test_blocked_layout_tables(L):
    """8x4-blocked storage: offsets and plane of blocked_layout pass the
    library's validation, misaligned offsets do not, and the row <-> block
    index maps are bijections onto distinct in-range positions that follow
    the documented address (32 (j/4 nb1 + i/8) + 8 (j%4) + i%8)."""
    ps = synth.uneven_sectors(6, 48, 130, 5)
    off, plane = L.blocked_layout(ps.n1, ps.n2)
    descs = L.patch_descs(ps.n1, ps.n2, ps.C1, ps.C2, off, ps.hhat, ps.htilde, ps.internal)
    assert L.validate_patches(descs, 5, plane, layout=1)[0] == 0
    assert L.validate_patches(descs, 5, plane, layout=7)[0] == 1
    bad = L.patch_descs(ps.n1, ps.n2, ps.C1, ps.C2, off + 8, ps.hhat, ps.htilde, ps.internal)
    assert L.validate_patches(bad, 5, plane + 64, layout=1)[0] == 1          # not a multiple of 32
    tight = int(off[-1]) + int(ps.n1[-1]) * int(ps.n2[-1])
    assert L.validate_patches(descs, 5, tight, layout=1)[0] == 1              # padded patch does not fit
    rows, blk = L.layout_index(ps.n1, ps.n2, ps.off, off)
    assert len(np.unique(rows)) == len(rows) == ps.npoints
    assert len(np.unique(blk)) == len(blk) and blk.max() < plane
    p = 3
    n1, n2 = int(ps.n1[p]), int(ps.n2[p])
    nb1 = (n1 + 7) // 8
    i, j = n1 - 1, n2 - 2
    want = int(off[p]) + 32 * ((j // 4) * nb1 + i // 8) + 8 * (j % 4) + i % 8
    k = int(np.sum(ps.n1[:p].astype(np.int64) * ps.n2[:p])) + j * n1 + i
    assert rows[k] == int(ps.off[p]) + j * n1 + i and blk[k] == want


def _fold(lib, N, C, d, kind, alpha=0.0, p=0):
    arq = np.ascontiguousarray(fcgram.continuation_matrix(d, C), np.float64)
    out = np.zeros(N * 2 * d, np.float64)
    rc = lib.fcsd_host_fold_matrix(ctypes.c_int(N), ctypes.c_int(C), ctypes.c_int(d),
                                   arq.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(kind),
                                   ctypes.c_double(alpha), ctypes.c_int(p), out.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    return out.reshape(N, 2 * d)


@pytest.mark.parametrize("N,C,d", [(48, 30, 5), (64, 27, 5), (101, 27, 2), (120, 36, 5), (57, 33, 5)])
def test_fold_matrix_is_the_transposed_operators_tail_fold(L, N, C, d):
    """The library's fold matrix G (host, binary128 / long double) applied
    to a cotangent equals what the oracle's transposed operator adds to the
    2d end samples beyond its circulant part: D^T y - (-S pad(y))[:N] for the
    derivative, F^T y - (F pad(y))[:N] for the filter (F symmetric)."""
    from oracle import filter as flt
    lib = L.lib()
    rng = np.random.default_rng(N + C)
    Y = rng.standard_normal((6, N))
    h = 1.0 / (N - 1)
    pad = np.concatenate([Y, np.zeros((6, C))], axis=-1)
    for kind in (0, 1):
        if kind == 0:
            G = _fold(lib, N, C, d, 0)
            full = fcgram.diff_lines_adj(Y, d, C)
            circ = -fcgram.periodic_derivative(pad, (N + C) * h)[:, :N]
        else:
            G = _fold(lib, N, C, d, 1, 10.0, 14)
            full = flt.filter_lines_adj(Y, d, C, 10.0, 14)
            circ = np.real(np.fft.ifft(np.fft.fft(pad, axis=-1) * flt.sigma(N + C, 10.0, 14), axis=-1))[:, :N]
        fold = full - circ
        want = np.concatenate([fold[:, N - d:], fold[:, :d]], axis=-1)     # e < d right, e >= d left
        got = Y @ G
        # the oracle folds an FP64 FFT tail: its own rounding, eps64 times
        # sum |A_r Q^T| (~1.4e4 for d = 5) times the transform's size
        bound = 16 * np.finfo(float).eps * np.abs(fcgram.continuation_matrix(d, C)).sum() * np.abs(full).max()
        assert np.abs(got - want).max() <= bound, kind
        # nothing is folded onto the interior samples
        assert np.abs(fold[:, d:N - d]).max() <= 1e-12 * np.abs(full).max()


def _position_wavenumbers(M, rad):
    """Wavenumber held by every position of the engine's digit-reversed
    order (the forward transform of a unit impulse at n = 1 puts
    exp(-2 pi i k / M) at the position of k)."""
    e = np.zeros(M, complex)
    e[1] = 1.0
    Y = emulate_engine(e, rad, np.exp(-2j * np.pi * np.arange(M) / M), False)
    return np.rint(-np.angle(Y) * M / (2 * np.pi)).astype(int) % M


@pytest.mark.parametrize("N,C", [(128, 27), (256, 27), (100, 27), (61, 28), (97, 0)])
def test_embedded_circulant_tables(L, N, C):
    """Lines whose extension length L = N + C has a prime factor above 13:
    the library wraps the circulant's first column onto a 13-smooth length
    M >= N + L.  Through the emulated engine (differenced extension padded
    to M, forward stages, the table, inverse stages) the first N outputs are
    the oracle's FC derivative (periodic derivative for C = 0); the filter's
    table gives the oracle's filtered line; and with the wrapped kernel in
    double precision the transposed sequence (Delta^T of the padded
    cotangent, conjugate table, positions < N, tail fold) is the oracle's
    transpose, which needs the wrap to cover m - n up to N."""
    lib = L.lib()
    Lx = N + C
    assert not synth.smooth13(Lx)
    M = lib.fcsd_host_embed_length(ctypes.c_int(N + Lx))
    assert M >= N + Lx and synth.smooth13(M)
    rad = L.fft_plan(M)
    tw = np.exp(-2j * np.pi * np.arange(M) / M)
    rng = np.random.default_rng(N + C)
    F = synth.random_lines(rng, 2, N)
    f = F[0] + 1j * F[1]
    if C:
        ArQ = L.fc_matrix(5, C)
        ext = fcgram.extend(F, ArQ)
        want = fcgram.diff_lines(F, 5, C)
    else:
        ext = F
        want = fcgram.periodic_derivative(F, 1.0)
    e = ext[0] + 1j * ext[1]
    dz = np.concatenate([np.roll(e, -1) - e, np.zeros(M - Lx)])
    out = np.zeros(2 * M, np.float32)
    r = (ctypes.c_int * 8)(*rad)
    lib.fcsd_host_kmul_embedded(ctypes.c_int(N), ctypes.c_int(Lx), ctypes.c_int(M), ctypes.c_int(len(rad)), r,
                                out.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(1 if C == 0 else 0))
    km = out[0::2].astype(np.float64) + 1j * out[1::2]
    d = emulate_engine(km * emulate_engine(dz, rad, tw, False), rad, tw, True)[:N]
    assert np.abs(d.real - want[0]).max() <= 1e-5 * np.abs(want[0]).max()
    assert np.abs(d.imag - want[1]).max() <= 1e-5 * np.abs(want[1]).max()
    # the table is DFT_M of the wrapped first column of the length-L circulant
    kw = _position_wavenumbers(M, rad)
    ks = np.fft.fftfreq(Lx) * Lx
    period = 1.0 if C == 0 else Lx / (N - 1)
    with np.errstate(all="ignore"):
        mult = np.where(ks == 0, 0, 2j * np.pi * ks / period / (np.exp(2j * np.pi * ks / Lx) - 1))
    if Lx % 2 == 0:
        mult[Lx // 2] = 0
    h = np.fft.ifft(mult)
    kM = np.zeros(M, complex)
    for t in range(-(Lx - 1), N + 1):
        kM[t % M] = h[t % Lx]
    K = np.fft.fft(kM) / M
    assert np.abs(km - K[kw]).max() <= 2e-7 * np.abs(K).max()
    # filter factors: the filtered line through the same engine
    out = np.zeros(2 * M, np.float32)
    lib.fcsd_host_fmul_embedded(ctypes.c_int(N), ctypes.c_int(Lx), ctypes.c_int(M), ctypes.c_int(len(rad)), r,
                                ctypes.c_double(10.0), ctypes.c_int(14), out.ctypes.data_as(ctypes.c_void_p))
    kf = out[0::2].astype(np.float64) + 1j * out[1::2]
    fl = emulate_engine(kf * emulate_engine(np.concatenate([e, np.zeros(M - Lx)]), rad, tw, False), rad, tw,
                        True)[:N]
    from oracle import filter as flt
    wf = flt.filter_lines(F, 5, C, 10.0, 14)
    assert np.abs(fl.real - wf[0]).max() <= 1e-6 * np.abs(wf[0]).max()
    assert np.abs(fl.imag - wf[1]).max() <= 1e-6 * np.abs(wf[1]).max()
    # transposed sequence with the wrapped kernel in double precision
    y = synth.random_lines(rng, 2, N)
    yz = y[0] + 1j * y[1]
    v = np.zeros(M, complex)
    v[:N] = yz
    if C:
        v[N] = yz[N - 1]
        v[1:N] = yz[:N - 1] - yz[1:]
        v[0] = -yz[0]
    else:
        v[:N] = np.roll(yz, 1) - yz
    t = emulate_engine(np.conj(K[kw]) * emulate_engine(v, rad, tw, False), rad, tw, True)
    if C:
        # the tail positions N..Lx-1 of the length-L transpose, then the fold
        got = t[:N].copy()
        tail = t[N:Lx]
        got[N - 5:] += ArQ.T @ tail
        got[:5] += fcgram.left_matrix(ArQ).T @ tail
        want_adj = fcgram.diff_lines_adj(y, 5, C)
    else:
        got = t[:N]
        want_adj = -fcgram.periodic_derivative(y, 1.0)
    assert np.abs(got.real - want_adj[0]).max() <= 1e-9 * np.abs(want_adj[0]).max()
    assert np.abs(got.imag - want_adj[1]).max() <= 1e-9 * np.abs(want_adj[1]).max()
