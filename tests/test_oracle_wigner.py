"""Pins for the oracle's Wigner d-functions (CPU only).

The oracle builds d^l_mn from Delta = d(pi/2) tables and the Fourier
expansion d = i^{n-m} sum_q Delta_qm Delta_qn e^{i q b}; these tests pin it to
textbook closed forms, Wigner's explicit sum, scipy's associated Legendre
functions and exact identities.
"""
import math
import os

import numpy as np
import pytest
from numpy import cos, sin, sqrt  # noqa: F401  (used by golden expressions)
from scipy import special

from oracle import mw

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "wigner_d_small.txt")
BETAS = np.array([0.0, 0.37, 1.1, np.pi / 2, 2.5, np.pi])


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        l, m, n, expr = line.split(None, 3)
        rows.append((int(l), int(m), int(n), expr))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"d{r[0]}_{r[1]}{r[2]}")
def test_closed_forms(row):
    l, m, n, expr = row
    for b in BETAS:
        c, s = math.cos(b), math.sin(b)  # noqa: F841
        want = eval(expr, {"c": c, "s": s, "sqrt": math.sqrt})
        # both symmetric partners of the table entry
        for (mm, nn, sign) in [(m, n, 1.0), (n, m, (-1.0) ** (m - n)), (-n, -m, 1.0)]:
            assert abs(mw.wigner_d_sum(l, mm, nn, b) - sign * want) < 1e-15
            assert abs(mw.wigner_d_fourier(l, mm, nn, b) - sign * want) < 1e-15


def test_delta_matches_explicit_sum():
    err = 0.0
    for l in range(9):
        for q in range(-l, l + 1):
            for m in range(-l, l + 1):
                err = max(err, abs(mw.delta(l, q, m) - mw.wigner_d_sum(l, q, m, np.pi / 2)))
    assert err < 1e-15


def test_fourier_d_matches_explicit_sum():
    b = np.array([0.21, 0.9, 1.7, 2.9])
    err = 0.0
    for l in range(8):
        for m in range(-l, l + 1):
            for n in range(-l, l + 1):
                d1 = mw.wigner_d_fourier(l, m, n, b)
                d2 = np.array([mw.wigner_d_sum(l, m, n, x) for x in b])
                err = max(err, np.abs(d1 - d2).max())
    assert err < 1e-14


def test_legendre_special_cases():
    """d^l_00 = P_l(cos b); d^l_m0 = sqrt((l-m)!/(l+m)!) P_l^m(cos b) with the
    Condon-Shortley phase (scipy.special.lpmv includes it)."""
    b = np.linspace(0.05, 3.1, 7)
    for l in range(0, 30, 3):
        np.testing.assert_allclose(mw.wigner_d_fourier(l, 0, 0, b),
                                   special.eval_legendre(l, np.cos(b)), atol=2e-14)
        for m in (1, 2, l // 2, l):
            if m > l or m < 1:
                continue
            norm = math.exp(0.5 * (math.lgamma(l - m + 1) - math.lgamma(l + m + 1)))
            want = norm * special.lpmv(m, l, np.cos(b))
            np.testing.assert_allclose(mw.wigner_d_fourier(l, m, 0, b), want, atol=5e-14)


def test_poles():
    """d^l_mn(0) = delta_mn and d^l_mn(pi) = (-1)^{l-n} delta_{m,-n}."""
    for l in (0, 1, 5, 17):
        for m in range(-l, l + 1):
            for n in range(-l, l + 1):
                assert abs(mw.wigner_d_fourier(l, m, n, 0.0) - (m == n)) < 2e-14
                want = (-1.0) ** (l - n) if m == -n else 0.0
                assert abs(mw.wigner_d_fourier(l, m, n, np.pi) - want) < 2e-14


def test_delta_orthogonal_at_large_degree():
    """Delta^l is a real orthogonal matrix; checked at l = 1023 (stability of the
    long-double ladder recursion over the whole column)."""
    mw.delta_table(1024)
    l = 1023
    cols = [0, 1, 2, 7, 300, 511, 1000, 1023]
    D = np.array([[mw.delta(l, q, m) for q in range(-l, l + 1)] for m in cols])
    assert np.abs(D @ D.T - np.eye(len(cols))).max() < 1e-14


def test_orthogonality_in_beta():
    """int_0^pi d^l_mn d^l'_mn sin b db = 2/(2l+1) delta_ll' (Gauss-Legendre in cos b)."""
    x, w = np.polynomial.legendre.leggauss(40)
    b = np.arccos(x)
    for (m, n) in [(0, 0), (2, 1), (3, -2), (5, 4)]:
        ls = range(max(abs(m), abs(n)), 12)
        D = np.array([mw.wigner_d_fourier(l, m, n, b) for l in ls])
        G = (D * w) @ D.T
        want = np.diag([2.0 / (2 * l + 1) for l in ls])
        np.testing.assert_allclose(G, want, atol=5e-14)


def test_mw_weight_closed_form():
    """w(k) = int_0^pi e^{ikt} sin t dt checked against Gauss-Legendre in t."""
    x, wt = np.polynomial.legendre.leggauss(80)
    t = 0.5 * np.pi * (x + 1)
    for k in range(-9, 10):
        num = 0.5 * np.pi * np.sum(wt * np.exp(1j * k * t) * np.sin(t))
        assert abs(mw.mw_weight(np.array([k]))[0] - num) < 1e-13
