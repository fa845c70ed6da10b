"""Pins for the oracle's MW spherical-harmonic and Wigner transforms (CPU only)."""
import numpy as np
import pytest
from scipy import special

import synthetic as S
from oracle import mw


def _Y(l, m, theta, phi):
    return special.sph_harm_y(l, m, theta, phi)


def test_closed_form_harmonics():
    """Y_00 = 1/sqrt(4pi), Y_10 = sqrt(3/4pi) cos t, Y_11 = -sqrt(3/8pi) sin t e^{ip}."""
    L = 5
    th, ph = mw.thetas(L)[:, None], mw.phis(L)[None, :]
    cases = {(0, 0): np.full((L, 2 * L - 1), 1 / np.sqrt(4 * np.pi)) + 0j,
             (1, 0): np.sqrt(3 / (4 * np.pi)) * np.cos(th) * np.ones_like(ph) + 0j,
             (1, 1): -np.sqrt(3 / (8 * np.pi)) * np.sin(th) * np.exp(1j * ph)}
    for (l, m), want in cases.items():
        flm = np.zeros((L, 2 * L - 1), complex)
        flm[l, m + L - 1] = 1.0
        np.testing.assert_allclose(mw.sht_inverse(flm, L), want, atol=1e-15)


@pytest.mark.parametrize("L", [1, 2, 3, 8, 32, 128])
def test_sht_round_trip(L):
    flm = S.sphere_flm(L, S.stream_key(7, L))
    f = mw.sht_inverse(flm, L)
    assert np.abs(f.imag).max() < 1e-13
    np.testing.assert_allclose(mw.sht_forward(f.real, L), flm, atol=1e-13)


@pytest.mark.parametrize("L", [3, 6, 9])
def test_sht_forward_against_gauss_legendre(L):
    """Brute force: the MW forward transform of a band-limited map equals the
    Gauss-Legendre (in cos t) x uniform-phi quadrature of f Y*_lm, with f and
    Y evaluated by scipy (independent of the oracle's d and MW machinery)."""
    rng = np.random.default_rng(L)
    flm = np.zeros((L, 2 * L - 1), complex)
    for l in range(L):
        for m in range(-l, l + 1):
            flm[l, m + L - 1] = rng.normal() + 1j * rng.normal()

    def synth(th, ph):
        out = np.zeros(np.broadcast(th, ph).shape, complex)
        for l in range(L):
            for m in range(-l, l + 1):
                out += flm[l, m + L - 1] * _Y(l, m, th, ph)
        return out

    f_mw = synth(mw.thetas(L)[:, None], mw.phis(L)[None, :])
    got = mw.sht_forward(f_mw, L)
    x, w = np.polynomial.legendre.leggauss(L + 1)
    th = np.arccos(x)[:, None]
    ph = mw.phis(L)[None, :]
    f_gl = synth(th, ph)
    want = np.zeros_like(flm)
    for l in range(L):
        for m in range(-l, l + 1):
            want[l, m + L - 1] = np.sum(w[:, None] * (2 * np.pi / (2 * L - 1)) * f_gl * np.conj(_Y(l, m, th, ph)))
    np.testing.assert_allclose(got, want, atol=1e-13)
    np.testing.assert_allclose(got, flm, atol=1e-13)


@pytest.mark.parametrize("L,N", [(4, 2), (6, 3), (8, 3), (16, 4)])
def test_wigner_round_trip(L, N):
    rng = np.random.default_rng(L * 10 + N)
    fh = np.zeros((2 * N - 1, L, 2 * L - 1), complex)
    for n in range(-(N - 1), N):
        for l in range(abs(n), L):
            for m in range(-l, l + 1):
                fh[n + N - 1, l, m + L - 1] = rng.normal() + 1j * rng.normal()
    f = mw.wigner_inverse(fh, L, N)
    np.testing.assert_allclose(mw.wigner_forward(f, L, N), fh, atol=1e-13)


@pytest.mark.parametrize("L,N", [(3, 2), (4, 3)])
def test_wigner_inverse_brute_force(L, N):
    """f(a,b,g) = sum (2l+1)/(8pi^2) fh D* with D* = e^{ima} d(b) e^{ing}, d from
    Wigner's explicit sum, evaluated point by point."""
    rng = np.random.default_rng(3)
    fh = np.zeros((2 * N - 1, L, 2 * L - 1), complex)
    for n in range(-(N - 1), N):
        for l in range(abs(n), L):
            for m in range(-l, l + 1):
                fh[n + N - 1, l, m + L - 1] = rng.normal() + 1j * rng.normal()
    got = mw.wigner_inverse(fh, L, N)
    al, be, ga = mw.phis(L), mw.thetas(L), mw.gammas(N)
    for g in range(2 * N - 1):
        for b in range(L):
            for a in range(2 * L - 1):
                acc = 0j
                for n in range(-(N - 1), N):
                    for l in range(abs(n), L):
                        for m in range(-l, l + 1):
                            acc += ((2 * l + 1) / (8 * np.pi ** 2) * fh[n + N - 1, l, m + L - 1]
                                    * np.exp(1j * m * al[a]) * mw.wigner_d_sum(l, m, n, be[b])
                                    * np.exp(1j * n * ga[g]))
                assert abs(got[g, b, a] - acc) < 1e-13


def test_wigner_forward_against_gauss_legendre():
    """Forward Wigner on MW samples vs Gauss-Legendre in cos b with d from the
    explicit sum (exact for band-limited products)."""
    L, N = 4, 3
    rng = np.random.default_rng(11)
    fh = np.zeros((2 * N - 1, L, 2 * L - 1), complex)
    for n in range(-(N - 1), N):
        for l in range(abs(n), L):
            for m in range(-l, l + 1):
                fh[n + N - 1, l, m + L - 1] = rng.normal() + 1j * rng.normal()
    got = mw.wigner_forward(mw.wigner_inverse(fh, L, N), L, N)
    x, w = np.polynomial.legendre.leggauss(L + 1)
    bs = np.arccos(x)
    al, ga = mw.phis(L), mw.gammas(N)
    want = np.zeros_like(fh)
    for n in range(-(N - 1), N):
        for l in range(abs(n), L):
            for m in range(-l, l + 1):
                acc = 0j
                for kb, b in enumerate(bs):
                    # f at (a, b, g) by the inverse definition, integrated against D
                    for g in range(2 * N - 1):
                        for a in range(2 * L - 1):
                            fv = 0j
                            for n2 in range(-(N - 1), N):
                                for l2 in range(abs(n2), L):
                                    for m2 in (m,):
                                        if abs(m2) > l2:
                                            continue
                                        fv += ((2 * l2 + 1) / (8 * np.pi ** 2) * fh[n2 + N - 1, l2, m2 + L - 1]
                                               * np.exp(1j * m2 * al[a]) * mw.wigner_d_sum(l2, m2, n2, b)
                                               * np.exp(1j * n2 * ga[g]))
                            acc += (w[kb] * (2 * np.pi / (2 * L - 1)) * (2 * np.pi / (2 * N - 1)) * fv
                                    * np.exp(-1j * m * al[a]) * mw.wigner_d_sum(l, m, n, b) * np.exp(-1j * n * ga[g]))
                want[n + N - 1, l, m + L - 1] = acc
    np.testing.assert_allclose(got, want, atol=1e-13)
