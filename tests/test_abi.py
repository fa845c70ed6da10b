"""C-ABI library: loads, exports every declared symbol, and its host-side plan
arithmetic (filters, MW theta quadrature, Wigner-d recursion tables) agrees
with the oracle.  CPU only: no device work is issued here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import filters, mw, wavelets

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "s2w.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:s2w|b3w)_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2402_01282_amd as s2w
    lib = ctypes.CDLL(s2w.LIB_PATH)
    names = _declared_symbols()
    assert "s2w_analysis" in names and "s2w_plan_create" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(s2w.EXPORTS) == names


def test_header_is_plain_c():
    src = open(os.path.join(ROOT, "include", "s2w.h")).read()
    assert "torch" not in src and "hip_runtime" not in src and 'extern "C"' in src


@pytest.mark.parametrize("L,N,lam,J0", [(32, 3, 2.0, 0), (64, 4, 2.0, 2), (40, 2, 3.0, 1),
                                        (33, 5, 2.0, 1), (1024, 8, 2.0, 0), (128, 4, 2.0, 0)])
def test_host_filters_match_oracle(L, N, lam, J0):
    import paper_2402_01282_amd as s2w
    Lk, Nk, Lp = s2w.host_scales(L, N, lam, J0)
    P = wavelets.Plan(L, N, lam, J0)
    assert Lk == P.Lj and Nk == P.Nj and Lp == P.Lphi
    psi, phi = s2w.host_filters(L, N, lam, J0)
    for k in range(len(P.scales)):
        np.testing.assert_allclose(psi[k], P.Psi[k], atol=2e-15)
    np.testing.assert_allclose(phi, P.Phi, atol=2e-15)


@pytest.mark.parametrize("L", [1, 2, 3, 8, 33, 64])
@pytest.mark.parametrize("sigma", [1, -1])
def test_host_theta_matrix_matches_oracle_quadrature(L, sigma):
    """y^T T_sigma x = sum_q y^(q) G_x(q) for any x, y: the library's closed-form
    matrix equals the oracle's Fourier-space MW quadrature as a bilinear form."""
    import paper_2402_01282_amd as s2w
    T = s2w.host_theta_matrix(L, sigma)
    rng = np.random.default_rng(L)
    X = rng.normal(size=(6, L)) + 1j * rng.normal(size=(6, L))
    Y = rng.normal(size=(6, L))
    sig = np.full(6, float(sigma))
    G = mw.mw_quadrature_G(X, L, sig)
    Yh = mw.mw_fourier_coeffs(Y.astype(complex), L, sig)
    ref = np.sum(Yh * G, axis=1)
    got = np.einsum("rb,bc,rc->r", Y, T, X)
    assert np.abs(ref - got).max() < 1e-13 * max(1.0, np.abs(ref).max())
    np.testing.assert_allclose(T, T.T, atol=1e-15)


def _oracle_d(L, m, n):
    mw.delta_table(L)
    th = mw.thetas(L)
    out = np.zeros((L, L))
    for l in range(max(abs(m), abs(n)), L):
        qs = np.arange(-l, l + 1)
        dm = np.array([mw.delta(l, q, m) for q in qs])
        dn = np.array([mw.delta(l, q, n) for q in qs])
        out[l] = np.real((1j) ** ((n - m) % 4) * (np.exp(1j * np.outer(th, qs)) @ (dm * dn)))
    return out


@pytest.mark.parametrize("L,m,n", [(16, 0, 0), (16, 3, -2), (16, 5, 5), (16, 0, 3), (64, 40, -7),
                                   (64, 63, 1), (64, 2, -7), (128, 120, 7), (128, 64, -5), (96, 1, 0)])
def test_host_recursion_matches_oracle_d(L, m, n):
    """The scaled, log-rescaled l-recursion the kernels use (run on the host) against
    d from the oracle's Delta-matrix Fourier sums, including the deep-underflow start
    region (large m near the poles) and theta = pi."""
    import paper_2402_01282_amd as s2w
    got = s2w.host_wigner_d(L, m, n)
    ref = _oracle_d(L, m, n)
    assert np.abs(got - ref).max() < 6e-14


def test_host_argument_errors():
    import paper_2402_01282_amd as s2w
    lib = s2w.lib()
    for args in [(1, 1, 2.0, 0), (8, 0, 2.0, 0), (8, 9, 2.0, 0), (8, 2, 1.0, 0), (8, 2, 2.0, 9)]:
        st = lib.s2w_host_scales(*args, None, None, None, None)
        assert st == -1, args
        assert len(lib.s2w_last_error()) > 0
    assert lib.s2w_host_theta_matrix(8, 0, None) == -1
    with pytest.raises(s2w.S2WError):
        s2w.host_wigner_d(8, 9, 0)


def test_plan_create_rejects_bad_arguments_without_device_work():
    """Argument checks run before any device call."""
    import paper_2402_01282_amd as s2w
    lib = s2w.lib()
    h = ctypes.c_void_p()
    assert lib.s2w_plan_create(None, 8, 2, 2.0, 0, 1, 0, 0, 0) == -1
    assert lib.s2w_plan_create(ctypes.byref(h), 8, 2, 2.0, 0, 0, 0, 0, 0) == -1       # batch
    assert lib.s2w_plan_create(ctypes.byref(h), 8, 2, 2.0, 0, 1, 0, 0, 7) == -1       # flags
    assert lib.s2w_plan_create(ctypes.byref(h), 1, 1, 2.0, 0, 1, 0, 0, 0) == -1       # L
    assert lib.s2w_plan_create(ctypes.byref(h), 8, 2, 0.5, 0, 1, 0, 0, 0) == -1       # lambda
    assert lib.s2w_plan_create(ctypes.byref(h), 8, 2, 2.0, 5, 1, 0, 0, 0) == -1       # J0 > J
    assert h.value is None
    assert lib.s2w_plan_destroy(None) == 0
    assert lib.s2w_analysis(None, None, None, None, None) == -1


@pytest.mark.parametrize("m,n", [(0, 0), (1, 0), (7, 7), (8, -7), (300, -5)])
def test_host_recursion_with_polar_table_at_L1024(m, n):
    """At L=1024 the FP64 recursion alone drifts by ~1e-11 at the samples next to the
    poles (near-double characteristic root); with the long-double polar table the
    l-contraction sum_l a_l d^l_mn(theta_b) matches the oracle's to ~1e-13 relative
    (compared through the oracle's Delta-based Fourier sums)."""
    import paper_2402_01282_amd as s2w
    L = 1024
    got = s2w.host_wigner_d(L, m, n)            # [l][b]
    rng = np.random.default_rng(7)
    l0 = max(abs(m), abs(n))
    a = np.zeros((L, 1, 1), complex)
    a[l0:, 0, 0] = rng.normal(size=L - l0) / np.sqrt(np.arange(l0, L) + 1.0)
    ref = ((1j) ** ((n - m) % 4) * mw.eval_fourier(mw._fourier(L, [m], [n], a)[0], L))[0].real
    c = a[:, 0, 0].real @ got
    assert np.linalg.norm(c - ref) / np.linalg.norm(ref) < 1.5e-13
    # every sample, pole-adjacent ones included, within 4e-12 of the column's rms
    # (the recursion alone is off by ~1.4e-11 of it at the first sample)
    assert np.abs(c - ref).max() < 4e-12 * np.linalg.norm(ref) / np.sqrt(L)


@pytest.mark.parametrize("P,tau", [(1, 1.0), (7, 0.5), (64, 1.0), (128, 2.0)])
def test_host_laguerre_rule_matches_oracle(P, tau):
    """The library's radial rule (Sturm bisection on the Jacobi matrix + Newton, long
    double) against the oracle's (library eigenvalue estimate + Newton)."""
    import paper_2402_01282_amd as s2w
    from oracle import ball
    r, w = s2w.host_laguerre_rule(P, tau)
    R = ball.Radial(P, tau)
    np.testing.assert_allclose(r, R.r, rtol=1e-13)
    np.testing.assert_allclose(w, R.W, rtol=1e-12)
