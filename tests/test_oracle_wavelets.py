"""Pins for the oracle's directional wavelet transform on the sphere (CPU only)."""
import numpy as np
import pytest
from scipy import special

import synthetic as S
from oracle import filters, mw, wavelets


def _map(L, key):
    return np.real(mw.sht_inverse(S.sphere_flm(L, key), L))


@pytest.mark.parametrize("L,N,J0", [(8, 3, 0), (8, 4, 1), (32, 3, 0), (16, 2, 1), (13, 5, 0)])
def test_round_trip(L, N, J0):
    """synthesis(analysis(f)) = f on band-limited f (Section 4.1: exact synthesis)."""
    P = wavelets.Plan(L, N, 2.0, J0)
    f = _map(L, S.stream_key(1, L))
    wav, scal = wavelets.analysis(f, P)
    np.testing.assert_allclose(wavelets.synthesis(wav, scal, P), f, atol=1e-13 * np.abs(f).max())


def test_round_trip_L256_N4_J0_2():
    """L=256, N=4, lam=2, J0=2."""
    P = wavelets.Plan(256, 4, 2.0, 2)
    f = _map(256, S.stream_key(2))
    wav, scal = wavelets.analysis(f, P)
    f2 = wavelets.synthesis(wav, scal, P)
    assert np.abs(f2 - f).max() < 1e-13 * np.abs(f).max()


def test_coefficients_real():
    P = wavelets.Plan(16, 4, 2.0, 0)
    flm = S.sphere_flm(16, S.stream_key(5))
    wav, scal = wavelets.analysis_lm(flm, P, real=False)
    for w in wav:
        assert np.abs(w.imag).max() < 1e-15
    assert np.abs(scal.imag).max() < 1e-15


def test_tight_frame_energy():
    """sum_j int |W^j|^2 drho + int |W^Phi|^2 dOmega = sum_lm |f_lm|^2, integrals
    by Parseval with the exact MW transforms of each scale."""
    L, N = 24, 3
    P = wavelets.Plan(L, N, 2.0, 1)
    flm = S.sphere_flm(L, S.stream_key(6))
    wav, scal = wavelets.analysis_lm(flm, P)
    e = np.sum(np.abs(mw.sht_forward(scal, P.Lphi)) ** 2)
    for k, w in enumerate(wav):
        Lj, Nj = P.Lj[k], P.Nj[k]
        wh = mw.wigner_forward(w, Lj, Nj)
        lj = np.arange(Lj)
        e += np.sum((2 * lj + 1)[None, :, None] / (8 * np.pi ** 2) * np.abs(wh) ** 2)
    assert abs(e - np.sum(np.abs(flm) ** 2)) < 1e-13 * e


def test_alpha_shift_equivariance():
    """Rotating f about the pole by alpha0 = 2 pi a0/(2L_j-1) (f_lm -> e^{-i m alpha0} f_lm,
    from (R f)_lm = sum_n D^l_mn f_ln, Section 2.4) shifts W^j by a0 samples in alpha."""
    L, N = 16, 3
    P = wavelets.Plan(L, N, 2.0, 0)
    flm = S.sphere_flm(L, S.stream_key(8))
    k = len(P.scales) - 1
    Lj = P.Lj[k]
    a0 = 3
    al0 = 2 * np.pi * a0 / (2 * Lj - 1)
    ms = np.arange(-(L - 1), L)
    wav, _ = wavelets.analysis_lm(flm, P)
    wav2, _ = wavelets.analysis_lm(flm * np.exp(-1j * ms * al0)[None, :], P)
    np.testing.assert_allclose(wav2[k], np.roll(wav[k], a0, axis=2), atol=1e-13)


def test_gamma_shift_equivariance():
    """Psi_ln -> e^{-i n gamma0} Psi_ln with gamma0 = 2 pi g0/(2N_j-1) gives W^j(gamma + gamma0)."""
    L, N = 12, 3
    P = wavelets.Plan(L, N, 2.0, 0)
    flm = S.sphere_flm(L, S.stream_key(9))
    k = len(P.scales) - 1
    Nj = P.Nj[k]
    g0 = 2
    ga0 = 2 * np.pi * g0 / (2 * Nj - 1)
    wav, _ = wavelets.analysis_lm(flm, P)
    ns = np.arange(-(N - 1), N)
    P.Psi[k] = P.Psi[k] * np.exp(-1j * ns * ga0)[None, :]
    wav2, _ = wavelets.analysis_lm(flm, P, real=False)
    np.testing.assert_allclose(wav2[k], np.roll(wav[k], -g0, axis=0), atol=1e-13)


def _Y(l, m, th, ph):
    return special.sph_harm_y(l, m, th, ph)


@pytest.mark.parametrize("L,N", [(4, 3), (5, 2), (6, 4)])
def test_direct_convolution(L, N):
    """W^j(rho) = <f, R_rho Psi^j> (eq:direct_conv) by pixel-space Gauss-Legendre
    quadrature, with (R_rho Psi)_lm = sum_n D^l_mn(rho) Psi_ln (Section 2.4),
    D from Wigner's explicit sum and Y from scipy, at every grid point of the
    top scale."""
    P = wavelets.Plan(L, N, 2.0, 0)
    flm = S.sphere_flm(L, S.stream_key(10, L))
    wav, _ = wavelets.analysis_lm(flm, P)
    k = len(P.scales) - 1
    Lj, Nj = P.Lj[k], P.Nj[k]
    Psi = P.Psi[k]
    x, w = np.polynomial.legendre.leggauss(L + 1)
    th = np.arccos(x)[:, None]
    ph = mw.phis(L + 1)[None, :]
    wq = w[:, None] * (2 * np.pi / (2 * L + 1))
    fpix = sum(flm[l, m + L - 1] * _Y(l, m, th, ph) for l in range(L) for m in range(-l, l + 1))
    Ys = {(l, m): _Y(l, m, th, ph) for l in range(L) for m in range(-l, l + 1)}
    for g, gam in enumerate(mw.gammas(Nj)):
        for b, bet in enumerate(mw.thetas(Lj)):
            for a, alp in enumerate(mw.phis(Lj)):
                rpsi = 0j
                for l in range(Lj):
                    for m in range(-l, l + 1):
                        c = 0j
                        for n in range(-(N - 1), N):
                            if abs(n) > l or Psi[l, n + N - 1] == 0:
                                continue
                            D = np.exp(-1j * m * alp) * mw.wigner_d_sum(l, m, n, bet) * np.exp(-1j * n * gam)
                            c += D * Psi[l, n + N - 1]
                        rpsi = rpsi + c * Ys[(l, m)]
                val = np.sum(wq * fpix * np.conj(rpsi))
                assert abs(val - wav[k][g, b, a]) < 1e-13


@pytest.mark.parametrize("L,N,J0", [(8, 3, 0), (16, 4, 1), (12, 2, 0)])
def test_adjoint_dot(L, N, J0):
    """<A x, y> = <x, A^T y> on random, non-band-limited arrays; A^T is not the synthesis."""
    P = wavelets.Plan(L, N, 2.0, J0)
    rng = np.random.default_rng(L + N)
    x = rng.normal(size=(L, 2 * L - 1))
    Ax, As = wavelets.analysis(x, P)
    gw = [rng.normal(size=w.shape) for w in Ax]
    gs = rng.normal(size=As.shape)
    lhs = sum(np.sum(a * g) for a, g in zip(Ax, gw)) + np.sum(As * gs)
    ATy = wavelets.analysis_adjoint(gw, gs, P)
    assert abs(lhs - np.sum(x * ATy)) < 1e-12 * abs(lhs)
    assert np.abs(ATy - wavelets.synthesis(gw, gs, P)).max() > 1e-3


def test_gradient_central_differences():
    """Gradient of sum_j sum W^j^2 at L=16 via 2 A^T(W) vs central differences
    (quadratic loss, so central differences are exact up to rounding)."""
    L, N = 16, 4
    P = wavelets.Plan(L, N, 2.0, 0)
    f = _map(L, S.stream_key(4))

    def loss(x):
        wav, _ = wavelets.analysis(x, P)
        return sum(np.sum(w ** 2) for w in wav)

    wav, scal = wavelets.analysis(f, P)
    g = wavelets.analysis_adjoint([2 * w for w in wav], np.zeros_like(scal), P)
    rng = np.random.default_rng(0)
    h = 1e-3
    for _ in range(6):
        i, j = rng.integers(L), rng.integers(2 * L - 1)
        e = np.zeros_like(f)
        e[i, j] = h
        fd = (loss(f + e) - loss(f - e)) / (2 * h)
        assert abs(fd - g[i, j]) < 1e-9 * max(1.0, abs(g[i, j]))


@pytest.mark.parametrize("L,N,J0", [(8, 3, 0), (16, 4, 1), (12, 2, 0), (9, 5, 0)])
def test_synthesis_adjoint_dot(L, N, J0):
    """<S(w, s), g> = <w, S^T_w g> + <s, S^T_s g> on random, non-band-limited arrays
    (S the synthesis, a real-linear map of the sample arrays)."""
    P = wavelets.Plan(L, N, 2.0, J0)
    rng = np.random.default_rng(7 * L + N)
    f0 = rng.normal(size=(L, 2 * L - 1))
    w0, s0 = wavelets.analysis(f0, P)
    w = [rng.normal(size=a.shape) for a in w0]
    s = rng.normal(size=s0.shape)
    g = rng.normal(size=(L, 2 * L - 1))
    lhs = np.sum(wavelets.synthesis(w, s, P) * g)
    gw, gs = wavelets.synthesis_adjoint(g, P)
    rhs = sum(np.sum(a * b) for a, b in zip(w, gw)) + np.sum(s * gs)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # S^T is not the analysis (MW oversamples)
    aw, _ = wavelets.analysis(g, P)
    assert max(np.abs(a - b).max() for a, b in zip(aw, gw)) > 1e-3
