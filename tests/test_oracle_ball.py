"""Pins for the ball oracle (radial Laguerre rule, ball filters, ball wavelets)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import eval_genlaguerre, roots_genlaguerre

import synthetic as S
from oracle import ball, mw, wavelets


def test_laguerre_functions_closed_forms():
    """psi_0..psi_2 against L^(2)_0 = 1, L^(2)_1 = 3 - x, L^(2)_2 = (x^2 - 8x + 12)/2."""
    x = np.linspace(0.0, 30.0, 41)
    ps = ball.laguerre_psi(3, x)
    e = np.exp(-x / 2)
    np.testing.assert_allclose(ps[0], e / math.sqrt(2), rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(ps[1], e * (3 - x) / math.sqrt(6), rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(ps[2], e * (x * x - 8 * x + 12) / 2 / math.sqrt(12), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("P", [1, 4, 10, 30])
def test_nodes_and_weights_match_library_rule(P):
    """Nodes are roots of L^(2)_P; tau^3 e^{x} w (our Christoffel form) equals the
    library's generalised Gauss-Laguerre weight times e^{x}."""
    R = ball.Radial(P)
    xs, ws = roots_genlaguerre(P, 2)
    np.testing.assert_allclose(R.x, np.sort(xs), rtol=1e-13)
    np.testing.assert_allclose(R.W, ws * np.exp(xs), rtol=1e-11)
    # Newton distance to the root, |L_P / L_P'| with L^(2)_P' = -L^(3)_{P-1}
    if P > 1:
        dx = np.abs(eval_genlaguerre(P, 2, R.x) / eval_genlaguerre(P - 1, 3, R.x))
        assert (dx / R.x).max() < 1e-12


@pytest.mark.parametrize("tau", [1.0, 1.7])
def test_basis_orthonormal_by_direct_integration(tau):
    """int_0^inf r^2 K_p(r) K_q(r) dr = delta_pq (adaptive quadrature, p, q < 4)."""
    def K(p, r):
        return ball.laguerre_psi(p + 1, np.array([r / tau]))[p, 0] / tau ** 1.5
    for p in range(4):
        for q in range(p, 4):
            v = quad(lambda r: r * r * K(p, r) * K(q, r), 0, np.inf, epsabs=1e-13, limit=200)[0]
            assert abs(v - (1.0 if p == q else 0.0)) < 1e-11, (p, q, v)


def test_rule_orthonormality_P128():
    """sum_k W_k K_p(r_k) K_q(r_k) = delta_pq for p, q < 128 (exactness of the rule)."""
    R = ball.Radial(128, tau=0.8)
    G = (R.K * R.W[None, :]) @ R.K.T
    assert np.abs(G - np.eye(128)).max() < 5e-13


def test_radial_transform_recovers_coefficients():
    rng = np.random.default_rng(3)
    R = ball.Radial(40, tau=2.0)
    c = rng.normal(size=(40, 3))
    np.testing.assert_allclose(R.forward(R.inverse(c)), c, atol=1e-12)


@pytest.mark.parametrize("L,N,P,J0,J0p", [(16, 3, 16, 0, 0), (32, 4, 24, 1, 2), (9, 2, 33, 2, 0)])
def test_ball_admissibility(L, N, P, J0, J0p):
    BP = ball.BallPlan(L, N, P, 2.0, 2.0, J0, J0p)
    assert np.abs(BP.admissibility() - 1.0).max() < 1e-13


def test_printed_ball_scaling_generator_is_not_admissible():
    """The hybrid scaling generator as printed (Appendix A.3) leaves an admissibility
    residual of order one, which is why the scaling filter is taken from the
    admissibility condition."""
    from oracle import filters
    lam = nu = 2.0
    BP = ball.BallPlan(16, 3, 16, lam, nu, 0, 0)
    k = filters.k_lam
    printed = np.array([[max(k(l / lam, lam) * k(p, nu) + k(l, lam) * k(p / nu, nu) - k(l, lam) * k(p, nu), 0.0)
                         for l in range(16)] for p in range(16)])
    tot = BP.admissibility() - BP.phi ** 2 + printed
    assert np.abs(tot - 1.0).max() > 0.5


@pytest.mark.parametrize("L,N,P,J0,J0p,tau", [(8, 3, 8, 0, 0, 1.0), (12, 4, 10, 1, 1, 0.7)])
def test_ball_round_trip(L, N, P, J0, J0p, tau):
    BP = ball.BallPlan(L, N, P, 2.0, 2.0, J0, J0p, tau)
    flmp = S.ball_flmp(L, P, S.stream_key(5))
    f = ball.sl_inverse(flmp, BP)
    wav, scal = ball.analysis(f, BP)
    f2 = ball.synthesis(wav, scal, BP)
    assert np.abs(f2 - f).max() < 1e-12 * np.abs(f).max()
    # the spherical-Laguerre transform itself is exact
    np.testing.assert_allclose(ball.sl_forward(f, BP), flmp, atol=1e-13 * np.abs(flmp).max())


def test_separable_input_factorises_into_sphere_wavelets():
    """For f_lmp = g_lm h_p, W^{jj'}(r'_k) = [sum_p K_p(r'_k) kappa_j'(p) h_p] W^j[g]: the ball
    coefficients are the sphere oracle's coefficients times a radial profile."""
    L, N, P = 10, 3, 12
    BP = ball.BallPlan(L, N, P)
    g = S.sphere_flm(L, S.stream_key(6))
    h = S.normals(S.stream_key(7), P)
    wav, _ = ball.analysis_lmp(h[:, None, None] * g[None], BP)
    wsph, _ = wavelets.analysis_lm(g, BP.ang)
    for i in range(len(BP.rscales)):
        prof = (BP.rad_j[i].basis(P) * BP.kappa_p[i][:, None]).T @ h      # [P_j']
        for k in range(len(BP.ang.scales)):
            ref = prof[:, None, None, None] * wsph[k][None]
            np.testing.assert_allclose(wav[(i, k)], ref, atol=1e-13 * (np.abs(ref).max() + 1e-300))


@pytest.mark.parametrize("L,N,P,J0,J0p,tau", [(6, 3, 5, 0, 0, 1.0), (8, 2, 6, 1, 1, 0.8)])
def test_ball_adjoints_dot(L, N, P, J0, J0p, tau):
    """<A x, y> = <x, A^T y> for the ball analysis, and <S y, x> = <y, S^T x> for the
    ball synthesis, on random non-band-limited arrays."""
    BP = ball.BallPlan(L, N, P, 2.0, 2.0, J0, J0p, tau)
    rng = np.random.default_rng(L * P + N)
    x = rng.normal(size=(P, L, 2 * L - 1))
    Aw, As = ball.analysis(x, BP)
    yw = {k: rng.normal(size=v.shape) for k, v in Aw.items()}
    ys = rng.normal(size=As.shape)
    lhs = sum(np.sum(Aw[k] * yw[k]) for k in Aw) + np.sum(As * ys)
    ATy = ball.analysis_adjoint(yw, ys, BP)
    assert abs(lhs - np.sum(x * ATy)) < 1e-11 * abs(lhs)
    Sy = ball.synthesis(yw, ys, BP)
    gw, gs = ball.synthesis_adjoint(x, BP)
    lhs2 = np.sum(Sy * x)
    rhs2 = sum(np.sum(yw[k] * gw[k]) for k in yw) + np.sum(ys * gs)
    assert abs(lhs2 - rhs2) < 1e-11 * abs(lhs2)


@pytest.mark.parametrize("L,N,P,tau", [(6, 3, 5, 1.0), (8, 1, 7, 0.8), (5, 4, 4, 1.2)])
def test_wigner_laguerre_round_trip_and_separability(L, N, P, tau):
    """Wigner-Laguerre transform: forward(inverse(c)) = c for band-limited real coefficients
    (the SO(3) MW sampling and the Laguerre rule are exact), the synthesised samples are real,
    and a separable function h(r) g(rho) has coefficients (radial coefficients of h) x (SO(3)
    coefficients of g)."""
    BP = ball.BallPlan(L, N, P, 2.0, 2.0, 0, 0, tau)
    c = S.wl_flmnp(L, N, P, S.stream_key(15))
    f = ball.wl_inverse(c, BP, N, real=False)
    assert np.abs(f.imag).max() < 1e-13 * np.abs(f.real).max()
    np.testing.assert_allclose(ball.wl_forward(f.real, BP, N), c, atol=1e-12 * np.abs(c).max())
    # separable input
    hp = S.normals(S.stream_key(16), P)                       # radial coefficients
    h = BP.rad.inverse(hp)                                    # h(r_k)
    g = S.so3_flmn(L, N, S.stream_key(17))
    gs = np.real(mw.wigner_inverse(g, L, N))
    sep = h[:, None, None, None] * gs[None]
    ref = hp[:, None, None, None] * g[None]
    np.testing.assert_allclose(ball.wl_forward(sep, BP, N), ref, atol=1e-12 * np.abs(ref).max())


def test_so3_generator_is_real_and_band_limited():
    L, N = 6, 3
    c = S.so3_flmn(L, N, S.stream_key(18))
    f = mw.wigner_inverse(c, L, N)
    assert np.abs(f.imag).max() < 1e-14 * np.abs(f.real).max()
    for i, n in enumerate(range(-(N - 1), N)):
        for l in range(L):
            for j, m in enumerate(range(-(L - 1), L)):
                if abs(m) > l or abs(n) > l:
                    assert c[i, l, j] == 0
