"""McEwen-Wiaux (MW) sampling, exact theta quadrature, spherical-harmonic and
Wigner transforms (oracle; test infrastructure only).

Transforms follow the paper's definitions:
  forward SHT     f_lm = int f Y*_lm dOmega                (Section 2.1, eq:fswsh)
  inverse SHT     f = sum f_lm Y_lm                        (Section 2.1, eq:iswsh)
  forward Wigner  f^l_mn = int f D^l_mn drho               (Section 2.2, eq:forward_wigner_transform)
  inverse Wigner  f = sum (2l+1)/(8 pi^2) f^l_mn D^{l*}_mn (Section 2.2, eq:inverse_wigner_transform)
with D^l_mn(a, b, g) = e^{-i m a} d^l_mn(b) e^{-i n g} (Section 5.2) and the
spin-0 harmonics Y_lm(t, p) = sqrt((2l+1)/(4 pi)) d^l_m0(t) e^{i m p}.

MW grids (the paper cites the MW sampling theorem for exactness, Section
4.4): theta_b = pi (2b+1)/(2L-1), b < L; phi_a = 2 pi a/(2L-1), a < 2L-1;
gamma_g = 2 pi g/(2N-1), g < 2N-1.

Theta quadrature: F(theta) of band limit L with parity F(2pi - t) = s F(t)
is extended to the 2L-1 torus points, its Fourier coefficients F^(p) are
taken exactly, and  int_0^pi F d sin(t) dt = sum_{p,q} F^(p) w(p+q) d^(q)
with w(k) = int_0^pi e^{ikt} sin t dt and d^(q) = i^{n-m} Delta_qm Delta_qn.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as _sfft

from . import _lib


def _fft(x, axis):
    return _sfft.fft(x, axis=axis, workers=-1)


def _ifft(x, axis):
    return _sfft.ifft(x, axis=axis, workers=-1)


def _to_wrapped(A, L):
    """Reorder the last axis from index k+L-1 (k = -(L-1)..L-1) to k mod (2L-1)."""
    return np.concatenate([A[..., L - 1:], A[..., :L - 1]], axis=-1)


def _from_wrapped(A, L):
    """Inverse of _to_wrapped."""
    return np.concatenate([A[..., L:], A[..., :L]], axis=-1)

_TABLE = {"L": 0, "T": None}


def delta_table(L: int) -> np.ndarray:
    """Packed Delta^l = d^l(pi/2) table for all l < L (cached; a larger table
    serves every smaller L because blocks depend on l only)."""
    if _TABLE["L"] < L:
        lib = _lib.lib()
        T = np.empty(lib.oracle_delta_size(L), dtype=np.float64)
        lib.oracle_delta_table(L, T)
        _TABLE["L"], _TABLE["T"] = L, T
    return _TABLE["T"]


def delta(l: int, q: int, m: int) -> float:
    T = delta_table(l + 1)
    return _lib.lib().oracle_delta_get(T, l, q, m)


def wigner_d_sum(l: int, m: int, n: int, beta: float) -> float:
    """Wigner's explicit sum formula (textbook; for small l)."""
    return _lib.lib().oracle_wigner_d_sum(l, m, n, float(beta))


def wigner_d_fourier(l: int, m: int, n: int, beta) -> np.ndarray:
    """d^l_mn(beta) = i^{n-m} sum_q Delta_qm Delta_qn e^{i q beta}."""
    beta = np.asarray(beta, dtype=np.float64)
    acc = np.zeros(beta.shape, dtype=np.complex128)
    for q in range(-l, l + 1):
        acc += delta(l, q, m) * delta(l, q, n) * np.exp(1j * q * beta)
    return np.real((1j) ** ((n - m) % 4) * acc)


def thetas(L: int) -> np.ndarray:
    return np.pi * (2.0 * np.arange(L) + 1.0) / (2.0 * L - 1.0)


def phis(L: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(2 * L - 1) / (2.0 * L - 1.0)


def gammas(N: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(2 * N - 1) / (2.0 * N - 1.0)


def mw_weight(k) -> np.ndarray:
    """w(k) = int_0^pi e^{i k t} sin t dt: +-i pi/2 at k = +-1, 2/(1-k^2) for even k, else 0."""
    k = np.asarray(k)
    out = np.zeros(k.shape, dtype=np.complex128)
    even = (k % 2) == 0
    out[even] = 2.0 / (1.0 - k[even].astype(np.float64) ** 2)
    out[k == 1] = 0.5j * np.pi
    out[k == -1] = -0.5j * np.pi
    return out


def _ipow(e):
    return (1j) ** (np.asarray(e) % 4)


def mw_fourier_coeffs(F: np.ndarray, L: int, sigma: np.ndarray) -> np.ndarray:
    """F [cols, L] sampled at theta_b -> F^(p) [cols, 2L-1], p = -(L-1)..L-1,
    after extending to the torus with F(theta_b) = sigma F(theta_{2L-2-b})."""
    n = 2 * L - 1
    Fe = np.empty((F.shape[0], n), dtype=np.complex128)
    Fe[:, :L] = F
    if L > 1:
        Fe[:, L:] = sigma[:, None] * F[:, L - 2::-1]
    X = _fft(Fe, 1) / n
    p = np.arange(-(L - 1), L)
    return np.exp(-1j * p * np.pi / n)[None, :] * _from_wrapped(X, L)


def mw_quadrature_G(F: np.ndarray, L: int, sigma: np.ndarray) -> np.ndarray:
    """G(q) = sum_p F^(p) w(p+q): integral against d becomes sum_q d^(q) G(q)."""
    Fh = mw_fourier_coeffs(F, L, sigma)
    return _hankel_w(Fh, L)


def _hankel_w(Fh: np.ndarray, L: int, conj: bool = False) -> np.ndarray:
    """G[:, q] = sum_p Fh[:, p] w(p+q) (conj: with conj(w)), evaluated as a real
    matrix product for the even-k part of w plus the two k = +-1 terms."""
    p = np.arange(-(L - 1), L)
    k = p[:, None] + p[None, :]
    kf = k.astype(np.float64)
    We = np.where(k % 2 == 0, 2.0 / np.where(k % 2 == 0, 1.0 - kf ** 2, 1.0), 0.0)
    G = (np.ascontiguousarray(Fh.real) @ We) + 1j * (np.ascontiguousarray(Fh.imag) @ We)
    s = -1.0 if conj else 1.0
    Q = 2 * L - 1
    # k = p + q = 1  ->  p = 1 - q;  k = -1  ->  p = -1 - q  (indices shift by L-1)
    qi = np.arange(Q)
    q = qi - (L - 1)
    i1 = 1 - q + (L - 1)
    im1 = -1 - q + (L - 1)
    ok1 = (i1 >= 0) & (i1 < Q)
    okm1 = (im1 >= 0) & (im1 < Q)
    G[:, qi[ok1]] += s * 0.5j * np.pi * Fh[:, i1[ok1]]
    G[:, qi[okm1]] -= s * 0.5j * np.pi * Fh[:, im1[okm1]]
    return G


def eval_fourier(G: np.ndarray, L: int) -> np.ndarray:
    """C[cols, b] = sum_q G[cols, q] e^{i q theta_b}, b < L."""
    n = 2 * L - 1
    q = np.arange(-(L - 1), L)
    Y = _to_wrapped(G * np.exp(1j * q * np.pi / n)[None, :], L)
    return (_ifft(Y, 1) * n)[:, :L]


def theta_transpose_sum(F: np.ndarray, L: int) -> np.ndarray:
    """H[cols, q] = sum_{b<L} e^{i q theta_b} F[cols, b]: with H, sum_b d(theta_b) F(theta_b)
    = i^{n-m} sum_q Delta_qm Delta_qn H(q) (used by the adjoints)."""
    q = np.arange(-(L - 1), L)
    E = np.exp(1j * np.outer(thetas(L), q))  # [b, q]
    return F @ E


def _fourier(L, ms, ns, a):
    """Fourier-space sum G[mi, ni, q] = sum_l a[l, mi, ni] Delta_qm Delta_qn."""
    lib = _lib.lib()
    T = delta_table(L)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    av = np.ascontiguousarray(a, dtype=np.complex128).view(np.float64).reshape(-1)
    G = np.empty(len(ms) * len(ns) * (2 * L - 1) * 2, dtype=np.float64)
    lib.oracle_wigner_fourier(L, len(ms), ms, len(ns), ns, np.ascontiguousarray(av), G, T)
    return G.view(np.complex128).reshape(len(ms), len(ns), 2 * L - 1)


def _project(L, ms, ns, H):
    """out[l, mi, ni] = sum_q Delta^l_qm Delta^l_qn H[mi, ni, q]."""
    lib = _lib.lib()
    T = delta_table(L)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    Hv = np.ascontiguousarray(H, dtype=np.complex128).view(np.float64).reshape(-1)
    out = np.empty(L * len(ms) * len(ns) * 2, dtype=np.float64)
    lib.oracle_wigner_project(L, len(ms), ms, len(ns), ns, np.ascontiguousarray(Hv), out, T)
    return out.view(np.complex128).reshape(L, len(ms), len(ns))


def mrange(L):
    return np.arange(-(L - 1), L)


def nrange(N):
    return np.arange(-(N - 1), N)


# ---------------------------------------------------------------- SO(3) ----

def wigner_inverse(fhat: np.ndarray, L: int, N: int) -> np.ndarray:
    """Inverse Wigner transform (Section 2.2, eq:inverse_wigner_transform) on the
    MW SO(3) grid.  fhat [2N-1, L, 2L-1] ("nlm", index n+N-1, l, m+L-1)
    -> f [2N-1 (gamma), L (beta), 2L-1 (alpha)] complex."""
    ms, ns = mrange(L), nrange(N)
    ls = np.arange(L)
    a = ((2 * ls + 1) / (8 * np.pi ** 2))[:, None, None] * np.transpose(fhat, (1, 2, 0))
    G = _fourier(L, ms, ns, a)  # [m, n, q]
    G *= _ipow(ns[None, :] - ms[:, None])[:, :, None]
    C = eval_fourier(G.reshape(-1, 2 * L - 1), L).reshape(len(ms), len(ns), L)
    na, ng = 2 * L - 1, 2 * N - 1
    X = np.zeros((ng, L, na), dtype=np.complex128)
    X[(ns % ng)[None, :, None], np.arange(L)[None, None, :], (ms % na)[:, None, None]] = C
    return _ifft(_ifft(X, 2), 0) * (na * ng)


def so3_fourier(f: np.ndarray, L: int, N: int, weighted: bool = True) -> np.ndarray:
    """F_mn(beta_b) = (2pi/(2L-1))(2pi/(2N-1)) sum_{a,g} f e^{-i m a} e^{-i n g}
    (unweighted: without the 2pi/(2L-1), 2pi/(2N-1) factors).  -> [m, n, b]."""
    na, ng = 2 * L - 1, 2 * N - 1
    X = _fft(_fft(f, 2), 0)
    ms, ns = mrange(L), nrange(N)
    F = X[(ns % ng)[None, :, None], np.arange(L)[None, None, :], (ms % na)[:, None, None]]
    if weighted:
        F = F * (2 * np.pi / na) * (2 * np.pi / ng)
    return F


def wigner_forward(f: np.ndarray, L: int, N: int) -> np.ndarray:
    """Forward Wigner transform (Section 2.2, eq:forward_wigner_transform),
    exact on the MW SO(3) grid.  f [2N-1, L, 2L-1] -> fhat [2N-1, L, 2L-1]."""
    ms, ns = mrange(L), nrange(N)
    F = so3_fourier(f, L, N)
    sigma = ((-1.0) ** (ms[:, None] + ns[None, :])).reshape(-1)
    G = mw_quadrature_G(F.reshape(-1, L), L, sigma).reshape(len(ms), len(ns), 2 * L - 1)
    raw = _project(L, ms, ns, G)  # [l, m, n]
    raw *= _ipow(ns[None, :] - ms[:, None])[None, :, :]
    return np.transpose(raw, (2, 0, 1))


# ---------------------------------------------------------------- S^2 ------

def sht_forward(f: np.ndarray, L: int) -> np.ndarray:
    """Forward spin-0 SHT (Section 2.1, eq:fswsh) on MW samples f [L, 2L-1]
    -> flm [L, 2L-1] (index m+L-1)."""
    ms = mrange(L)
    na = 2 * L - 1
    X = _fft(f, 1) * (2 * np.pi / na)   # [b, k]
    F = X[:, ms % na].T                              # [m, b]
    G = mw_quadrature_G(F, L, (-1.0) ** ms)
    raw = _project(L, ms, np.array([0]), G[:, None, :])[:, :, 0]  # [l, m]
    ls = np.arange(L)
    return np.sqrt((2 * ls + 1) / (4 * np.pi))[:, None] * _ipow(-ms)[None, :] * raw


def sht_inverse(flm: np.ndarray, L: int) -> np.ndarray:
    """Inverse spin-0 SHT (Section 2.1, eq:iswsh): flm [L, 2L-1] -> f [L, 2L-1] complex."""
    ms = mrange(L)
    ls = np.arange(L)
    a = (np.sqrt((2 * ls + 1) / (4 * np.pi))[:, None] * flm)[:, :, None]  # [l, m, 1]
    G = _fourier(L, ms, np.array([0]), a)[:, 0, :] * _ipow(-ms)[:, None]
    C = eval_fourier(G, L)  # [m, b]
    na = 2 * L - 1
    X = np.zeros((L, na), dtype=np.complex128)
    X[:, ms % na] = C.T
    return _ifft(X, 1) * na


# ------------------------------------------------------------ spin-s ------
# Spin-weighted harmonics (Section 2.1, eq:u1sym to eq:iswsh) in the convention
#   sY_lm(t, p) = (-1)^s sqrt((2l+1)/(4 pi)) D^{l*}_{m,-s}(p, t, 0)
#               = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(t) e^{i m p},
# which is Y_lm at s = 0 and gives 1Y_10 = sqrt(3/(8 pi)) sin t.  The spin-s
# transforms are the spin-0 ones with the d column n = -s in place of n = 0; the
# theta extension of the n = -s integrand has the parity (-1)^{m+s}.

def spin_sht_forward(f: np.ndarray, L: int, s: int) -> np.ndarray:
    """Forward spin-s SHT (Section 2.1, eq:fswsh) on MW samples of a complex spin-s
    map f [L, 2L-1] -> sflm [L, 2L-1] (index m+L-1; zero for l < |s|)."""
    ms = mrange(L)
    na = 2 * L - 1
    X = _fft(np.asarray(f, dtype=np.complex128), 1) * (2 * np.pi / na)   # [b, k]
    F = X[:, ms % na].T                                                   # [m, b]
    G = mw_quadrature_G(F, L, (-1.0) ** (ms + s))
    raw = _project(L, ms, np.array([-s]), G[:, None, :])[:, :, 0]         # [l, m]
    ls = np.arange(L)
    return (-1.0) ** s * np.sqrt((2 * ls + 1) / (4 * np.pi))[:, None] * _ipow(-s - ms)[None, :] * raw


def spin_sht_inverse(flm: np.ndarray, L: int, s: int) -> np.ndarray:
    """Inverse spin-s SHT (Section 2.1, eq:iswsh): sflm [L, 2L-1] -> complex map [L, 2L-1]."""
    ms = mrange(L)
    ls = np.arange(L)
    a = ((-1.0) ** s * np.sqrt((2 * ls + 1) / (4 * np.pi))[:, None] * flm)[:, :, None]   # [l, m, 1]
    G = _fourier(L, ms, np.array([-s]), a)[:, 0, :] * _ipow(-s - ms)[:, None]
    C = eval_fourier(G, L)                                                # [m, b]
    na = 2 * L - 1
    X = np.zeros((L, na), dtype=np.complex128)
    X[:, ms % na] = C.T
    return _ifft(X, 1) * na


# ------------------------------------------------------------- adjoints ----
# Literal (Hermitian) transposes of the discrete maps above, for real inner
# products <x, y> = Re sum conj(x) y.

def wigner_inverse_adjoint(g: np.ndarray, L: int, N: int) -> np.ndarray:
    """Adjoint of wigner_inverse: g [2N-1, L, 2L-1] -> [2N-1, L, 2L-1] ("nlm")."""
    ms, ns = mrange(L), nrange(N)
    F = so3_fourier(g, L, N, weighted=False)            # sum e^{-i m a} e^{-i n g}
    H = theta_transpose_sum(F.reshape(-1, L), L).reshape(len(ms), len(ns), 2 * L - 1)
    raw = _project(L, ms, ns, H)                         # sum_q Delta_qm Delta_qn H(q)
    raw *= _ipow(ns[None, :] - ms[:, None])[None, :, :]  # -> sum_b d(theta_b) F(theta_b)
    ls = np.arange(L)
    raw *= ((2 * ls + 1) / (8 * np.pi ** 2))[:, None, None]
    return np.transpose(raw, (2, 0, 1))


def sht_inverse_adjoint(g: np.ndarray, L: int) -> np.ndarray:
    """Adjoint of sht_inverse: g [L, 2L-1] -> [L, 2L-1] (flm layout)."""
    ms = mrange(L)
    na = 2 * L - 1
    X = _fft(g, 1)
    F = X[:, ms % na].T
    H = theta_transpose_sum(F, L)
    raw = _project(L, ms, np.array([0]), H[:, None, :])[:, :, 0]
    ls = np.arange(L)
    return np.sqrt((2 * ls + 1) / (4 * np.pi))[:, None] * _ipow(-ms)[None, :] * raw


def _mw_quadrature_G_adjoint(Gp: np.ndarray, L: int, sigma: np.ndarray) -> np.ndarray:
    """Adjoint of mw_quadrature_G: [cols, q] -> [cols, b < L]."""
    n = 2 * L - 1
    p = np.arange(-(L - 1), L)
    Fh = _hankel_w(Gp, L, conj=True)                           # w symmetric: adjoint uses conj(w)
    Fh = Fh * np.conj(np.exp(-1j * p * np.pi / n))[None, :]
    X = _to_wrapped(Fh, L)
    Fe = _ifft(X, 1)                                           # adjoint of fft(.)/n
    F = Fe[:, :L].copy()
    if L > 1:
        F[:, L - 2::-1] += sigma[:, None] * Fe[:, L:]
    return F


def sht_forward_adjoint(g: np.ndarray, L: int) -> np.ndarray:
    """Adjoint of sht_forward (as a map of complex samples): g [L, 2L-1] (flm) -> [L, 2L-1]."""
    ms = mrange(L)
    na = 2 * L - 1
    ls = np.arange(L)
    a = np.sqrt((2 * ls + 1) / (4 * np.pi))[:, None] * np.conj(_ipow(-ms))[None, :] * g
    Gp = _fourier(L, ms, np.array([0]), a[:, :, None])[:, 0, :]   # sum_l D_qm D_q0 a
    F = _mw_quadrature_G_adjoint(Gp, L, (-1.0) ** ms)              # [m, b]
    X = np.zeros((L, na), dtype=np.complex128)
    X[:, ms % na] = F.T * (2 * np.pi / na)
    return _ifft(X, 1) * na                              # adjoint of fft


def wigner_forward_adjoint(g: np.ndarray, L: int, N: int) -> np.ndarray:
    """Adjoint of wigner_forward: g ("nlm") -> [2N-1, L, 2L-1] complex samples."""
    ms, ns = mrange(L), nrange(N)
    a = np.transpose(g, (1, 2, 0)) * np.conj(_ipow(ns[None, :] - ms[:, None]))[None, :, :]
    Gp = _fourier(L, ms, ns, a)                                      # [m, n, q]
    sigma = ((-1.0) ** (ms[:, None] + ns[None, :])).reshape(-1)
    F = _mw_quadrature_G_adjoint(Gp.reshape(-1, 2 * L - 1), L, sigma).reshape(len(ms), len(ns), L)
    na, ng = 2 * L - 1, 2 * N - 1
    F = F * (2 * np.pi / na) * (2 * np.pi / ng)
    X = np.zeros((ng, L, na), dtype=np.complex128)
    X[(ns % ng)[None, :, None], np.arange(L)[None, None, :], (ms % na)[:, None, None]] = F
    return _ifft(_ifft(X, 2), 0) * (na * ng)
