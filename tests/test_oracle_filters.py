"""Pins for the oracle's wavelet filters (paper Appendix A), CPU only."""
import math

import mpmath
import numpy as np
import pytest

from oracle import filters


def _k_mp(t, lam):
    """k_lam(t) at 30 digits with mpmath (independent quadrature)."""
    mpmath.mp.dps = 30
    lam = mpmath.mpf(lam)

    def s2(x):
        u = 2 * lam / (lam - 1) * (x - 1 / lam) - 1
        if abs(u) >= 1:
            return mpmath.mpf(0)
        return mpmath.e ** (-2 / (1 - u * u)) / x

    if t <= 1 / lam:
        return 1.0
    if t >= 1:
        return 0.0
    num = mpmath.quad(s2, [mpmath.mpf(t), 1])
    den = mpmath.quad(s2, [1 / lam, (1 / lam + 1) / 2, 1])
    return float(num / den)


@pytest.mark.parametrize("lam", [2.0, 3.0, 1.5])
def test_k_lambda_against_mpmath(lam):
    for t in [0.3, 1 / lam + 1e-3, 0.55, 0.7, 0.8, 0.95, 0.999, 1.2]:
        assert abs(filters.k_lam(t, lam) - _k_mp(t, lam)) < 2e-15


def test_k_lambda_limits_and_monotone():
    lam = 2.0
    ts = np.linspace(0.4, 1.1, 57)
    ks = [filters.k_lam(t, lam) for t in ts]
    assert all(a >= b - 1e-16 for a, b in zip(ks, ks[1:]))
    assert filters.k_lam(0.5, lam) == 1.0 and filters.k_lam(1.0, lam) == 0.0


@pytest.mark.parametrize("L,N,lam,J0", [(32, 3, 2.0, 0), (64, 4, 2.0, 2), (33, 5, 2.0, 1),
                                        (40, 2, 3.0, 1), (1024, 8, 2.0, 0)])
def test_admissibility(L, N, lam, J0):
    """4pi/(2l+1)|Phi_l0|^2 + 8pi^2/(2l+1) sum_j sum_n |Psi^j_ln|^2 = 1 for all l (Section 3.1)."""
    np.testing.assert_allclose(filters.admissibility(L, N, lam, J0), 1.0, atol=1e-14)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 8])
def test_zeta_unit_energy(N):
    for l in range(1, 40):
        e = sum(abs(filters.zeta(l, n, N)) ** 2 for n in range(-(N - 1), N))
        assert abs(e - 1.0) < 1e-15
    # zero outside |n| < N, |n| <= l, and of the wrong parity
    for l in range(0, 12):
        for n in range(-12, 13):
            z = filters.zeta(l, n, N)
            if abs(n) >= N or abs(n) > l or (N + n) % 2 == 0:
                assert z == 0


def test_zeta_phase_gives_real_coefficients():
    """(-1)^n zeta_{l,-n} = conj(zeta_ln): makes W real for real f."""
    for N in (2, 3, 4, 7, 8):
        for l in range(0, 20):
            for n in range(-(N - 1), N):
                assert abs((-1) ** n * filters.zeta(l, -n, N) - np.conj(filters.zeta(l, n, N))) < 1e-16


def test_kappa_peak_and_support():
    lam = 2.0
    for j in range(1, 9):
        assert abs(filters.kappa(j, int(lam ** j), lam) - 1.0) < 1e-15   # kappa_j(lam^j) = 1
        for l in range(0, 600):
            k = filters.kappa(j, l, lam)
            if l <= lam ** (j - 1) or l >= lam ** (j + 1):
                assert k == 0.0
            elif abs(l - lam ** j) < 1e-9:
                assert abs(k - 1) < 1e-15


def test_band_limits():
    assert filters.scale_count(1024, 2.0) == 10
    assert [filters.scale_bandlimit(j, 1024, 2.0) for j in range(11)] == \
        [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 1024]
    assert filters.scaling_bandlimit(256, 2.0, 2) == 4
    assert filters.scaling_bandlimit(256, 2.0, 0) == 1
    # every l < L is covered by some scale or the scaling function
    for (L, lam, J0) in [(100, 2.0, 0), (100, 3.0, 1), (64, 2.0, 3)]:
        J = filters.scale_count(L, lam)
        assert lam ** J >= L - 1
        assert math.ceil(lam ** (J + 1)) >= L
