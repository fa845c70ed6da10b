"""Pins for the oracle's spin-s transforms (CPU only).

The spin-weighted harmonics are checked against Goldberg's closed-form sum
(binomial coefficients in sin and cos of theta/2), which shares nothing with the
oracle's d^l_mn route through the Delta = d(pi/2) tables; the forward transform against
Gauss-Legendre quadrature of f conj(sY); the wavelet transform of spin maps against
the pixel-space directional convolution <sf, R_rho sPsi> with D from Wigner's explicit
sum; and spin 0 against the real-map oracle by linearity."""
from math import comb, factorial

import numpy as np
import pytest

import synthetic as S
from oracle import mw, wavelets


def _sY(s, l, m, th, ph):
    """Goldberg et al. (1967): sY_lm = (-1)^m sqrt((l+m)!(l-m)!(2l+1) / (4pi (l+s)!(l-s)!))
    sum_r C(l-s, r) C(l+s, r+s-m) (-1)^{l-r-s} e^{imp} sin^{2l-k}(t/2) cos^k(t/2),
    k = 2r+s-m (the sin^{2l} cot^k form written without its removable singularity)."""
    shape = np.broadcast(th, ph).shape
    if l < max(abs(s), abs(m)):
        return np.zeros(shape, complex)
    pre = (-1) ** m * np.sqrt(factorial(l + m) * factorial(l - m) * (2 * l + 1)
                              / (4 * np.pi * factorial(l + s) * factorial(l - s)))
    acc = np.zeros(shape)
    for r in range(0, l - s + 1):
        j = r + s - m
        if j < 0 or j > l + s:
            continue
        k = 2 * r + s - m
        acc = acc + comb(l - s, r) * comb(l + s, j) * (-1) ** (l - r - s) \
            * np.sin(th / 2) ** (2 * l - k) * np.cos(th / 2) ** k
    return pre * acc * np.exp(1j * m * ph)


def test_spin_harmonics_match_goldberg():
    L = 6
    th, ph = mw.thetas(L)[:, None], mw.phis(L)[None, :]
    for s in range(-3, 4):
        for l in range(abs(s), L):
            for m in range(-l, l + 1):
                flm = np.zeros((L, 2 * L - 1), complex)
                flm[l, m + L - 1] = 1.0
                np.testing.assert_allclose(mw.spin_sht_inverse(flm, L, s), _sY(s, l, m, th, ph),
                                           atol=1e-14, err_msg=str((s, l, m)))


def test_spin_zero_is_the_scalar_transform():
    L = 9
    flm = S.spin_flm(L, 0, S.stream_key(80))
    np.testing.assert_allclose(mw.spin_sht_inverse(flm, L, 0), mw.sht_inverse(flm, L), atol=1e-14)
    f = mw.sht_inverse(flm, L)
    np.testing.assert_allclose(mw.spin_sht_forward(f, L, 0), mw.sht_forward(f, L), atol=1e-14)


@pytest.mark.parametrize("L,s", [(2, 1), (5, -2), (8, 1), (16, 3), (33, -1), (64, 2)])
def test_spin_round_trip(L, s):
    flm = S.spin_flm(L, s, S.stream_key(81, L))
    f = mw.spin_sht_inverse(flm, L, s)
    np.testing.assert_allclose(mw.spin_sht_forward(f, L, s), flm, atol=1e-13)


@pytest.mark.parametrize("L,s", [(4, 1), (6, -2), (7, 2)])
def test_spin_forward_against_gauss_legendre(L, s):
    """Brute force: the MW forward transform of a band-limited spin-s map equals the
    Gauss-Legendre (in cos t) x uniform-phi quadrature of f conj(sY_lm), with f and sY
    from Goldberg's formula."""
    flm = S.spin_flm(L, s, S.stream_key(82, L))

    def synth(th, ph):
        return sum(flm[l, m + L - 1] * _sY(s, l, m, th, ph)
                   for l in range(abs(s), L) for m in range(-l, l + 1))

    got = mw.spin_sht_forward(synth(mw.thetas(L)[:, None], mw.phis(L)[None, :]), L, s)
    x, w = np.polynomial.legendre.leggauss(L + 1)
    th, ph = np.arccos(x)[:, None], mw.phis(L)[None, :]
    fgl = synth(th, ph)
    want = np.zeros_like(flm)
    for l in range(abs(s), L):
        for m in range(-l, l + 1):
            want[l, m + L - 1] = np.sum(w[:, None] * (2 * np.pi / (2 * L - 1)) * fgl * np.conj(_sY(s, l, m, th, ph)))
    np.testing.assert_allclose(got, want, atol=1e-13)
    np.testing.assert_allclose(got, flm, atol=1e-13)


@pytest.mark.parametrize("s", [1, 2, -3])
def test_spin_conjugation(s):
    """conj(sf) is a spin -s map with coefficients (-1)^{s+m} conj(sf_{l,-m})."""
    L = 12
    flm = S.spin_flm(L, s, S.stream_key(83, abs(s)))
    f = mw.spin_sht_inverse(flm, L, s)
    got = mw.spin_sht_forward(np.conj(f), L, -s)
    ms = mw.mrange(L)
    want = ((-1.0) ** (s + ms))[None, :] * np.conj(flm[:, ::-1])
    np.testing.assert_allclose(got, want, atol=1e-13)


def test_spin0_complex_is_two_real_transforms():
    L, N = 16, 3
    P = wavelets.Plan(L, N, 2.0, 0)
    u = np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(84, 0)), L))
    v = np.real(mw.sht_inverse(S.sphere_flm(L, S.stream_key(84, 1)), L))
    wav, scal = wavelets.analysis_spin(u + 1j * v, P, 0)
    wu, su = wavelets.analysis(u, P)
    wv, sv = wavelets.analysis(v, P)
    for a, b, c in zip(wav, wu, wv):
        np.testing.assert_allclose(a, b + 1j * c, atol=1e-13)
    np.testing.assert_allclose(scal, su + 1j * sv, atol=1e-13)


@pytest.mark.parametrize("L,N,J0,s", [(8, 3, 0, 1), (16, 4, 1, -2), (32, 2, 0, 3), (12, 5, 0, 0)])
def test_spin_wavelet_round_trip(L, N, J0, s):
    P = wavelets.Plan(L, N, 2.0, J0)
    flm = S.spin_flm(L, s, S.stream_key(85, L))
    f = mw.spin_sht_inverse(flm, L, s)
    wav, scal = wavelets.analysis_spin(f, P, s)
    np.testing.assert_allclose(wavelets.synthesis_spin(wav, scal, P, s), f, atol=1e-12)


@pytest.mark.parametrize("L,N,s", [(4, 3, 1), (5, 2, 2), (4, 2, -1)])
def test_spin_direct_convolution(L, N, s):
    """W^j(rho) = <sf, R_rho sPsi^j> by pixel-space Gauss-Legendre quadrature, with
    (R_rho sPsi)_lm = sum_n D^l_mn(rho) Psi_ln and sY from Goldberg's formula, at every
    grid point of the top scale."""
    P = wavelets.Plan(L, N, 2.0, 0)
    flm = S.spin_flm(L, s, S.stream_key(86, L))
    f = mw.spin_sht_inverse(flm, L, s)
    wav, _ = wavelets.analysis_spin(f, P, s)
    k = len(P.scales) - 1
    Lj, Nj = P.Lj[k], P.Nj[k]
    Psi = P.Psi[k]
    x, w = np.polynomial.legendre.leggauss(L + 1)
    th = np.arccos(x)[:, None]
    ph = mw.phis(L + 1)[None, :]
    wq = w[:, None] * (2 * np.pi / (2 * L + 1))
    Ys = {(l, m): _sY(s, l, m, th, ph) for l in range(L) for m in range(-l, l + 1)}
    fpix = sum(flm[l, m + L - 1] * Ys[(l, m)] for l in range(L) for m in range(-l, l + 1))
    for g, gam in enumerate(mw.gammas(Nj)):
        for b, bet in enumerate(mw.thetas(Lj)):
            for a, alp in enumerate(mw.phis(Lj)):
                rpsi = 0j
                for l in range(max(abs(s), 0), Lj):
                    for m in range(-l, l + 1):
                        c = 0j
                        for n in range(-(N - 1), N):
                            if abs(n) > l or Psi[l, n + N - 1] == 0:
                                continue
                            D = np.exp(-1j * m * alp) * mw.wigner_d_sum(l, m, n, bet) * np.exp(-1j * n * gam)
                            c += D * Psi[l, n + N - 1]
                        rpsi = rpsi + c * Ys[(l, m)]
                val = np.sum(wq * fpix * np.conj(rpsi))
                assert abs(val - wav[k][g, b, a]) < 1e-13, (g, b, a)
