"""Scale-discretised wavelet filters (oracle; test infrastructure only).

Paper Appendix A:
  s(t) = exp(-1/(1-t^2)) on |t| < 1                     (A.1, bump function)
  s_lam(t) = s(2 lam/(lam-1) (t - 1/lam) - 1)           (A.1, support [1/lam, 1])
  k_lam(t) = int_t^1 s_lam^2(t')/t' dt' / int_{1/lam}^1 s_lam^2(t')/t' dt'   (A.1)
  kappa_lam(t) = sqrt(k_lam(t/lam) - k_lam(t)),  eta_lam(t) = sqrt(k_lam(t))  (A.1)
      (the difference is evaluated as one integral over [t/lam, t]; see kappa2_lam)
  zeta_ln = xi mu sqrt(2^{-q} C(q, (q-n)/2)), xi = 1 (N-1 even) else i,
            mu = [1 - (-1)^{N+n}]/2, q = min(N-1, l - [1 + (-1)^{N+l}]/2)   (A.2)
  Psi^j_ln = sqrt((2l+1)/(8 pi^2)) kappa^j(l) zeta_ln                      (A.4)
  Phi_l0  = sqrt((2l+1)/(4 pi)) eta_lam(l/lam^J0)                          (A.4, sphere)

Readings (the paper is ambiguous or garbled here):
  * scale index runs upward: kappa^j(l) = kappa_lam(l/lam^j), support
    lam^{j-1} < l < lam^{j+1}, matching the multiresolution support of
    Section 3.3;
  * J is the smallest integer with lam^J >= L (admissibility needs lam^J >= L-1);
  * per-scale band limits L_j = min(ceil(lam^{j+1}), L), N_j = min(N, L_j);
    scaling band limit L_phi = ceil(lam^J0);
  * the sphere scaling function drops p and j' from the ball's three-case
    form, as the admissibility paragraph instructs.
k_lam uses adaptive Gauss-Kronrod quadrature (scipy.integrate.quad).
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.integrate import quad


def bump(t: float) -> float:
    return math.exp(-1.0 / (1.0 - t * t)) if abs(t) < 1.0 else 0.0


def s_lam(t: float, lam: float) -> float:
    return bump(2.0 * lam / (lam - 1.0) * (t - 1.0 / lam) - 1.0)


@lru_cache(maxsize=None)
def _k_den(lam: float) -> float:
    return quad(lambda x: s_lam(x, lam) ** 2 / x, 1.0 / lam, 1.0,
                epsabs=0.0, epsrel=2e-14, limit=400)[0]


@lru_cache(maxsize=None)
def k_lam(t: float, lam: float) -> float:
    if t <= 1.0 / lam:
        return 1.0
    if t >= 1.0:
        return 0.0
    num = quad(lambda x: s_lam(x, lam) ** 2 / x, t, 1.0, epsabs=0.0, epsrel=2e-14, limit=400)[0]
    return num / _k_den(lam)


@lru_cache(maxsize=None)
def kappa2_lam(t: float, lam: float) -> float:
    """kappa_lam(t)^2 = k_lam(t/lam) - k_lam(t).  Both terms are integrals of the
    same integrand s_lam^2/t' from their argument to 1, so the difference is the
    integral over [t/lam, t] (clipped to the support [1/lam, 1]); evaluating it
    that way avoids the cancellation of two numbers close to 1."""
    a, b = max(t / lam, 1.0 / lam), min(t, 1.0)
    if b <= a:
        return 0.0
    num = quad(lambda x: s_lam(x, lam) ** 2 / x, a, b, epsabs=0.0, epsrel=2e-14, limit=400)[0]
    return num / _k_den(lam)


def kappa(j: int, l: int, lam: float) -> float:
    t = l / lam ** j
    return math.sqrt(kappa2_lam(t, lam))


def eta(l: int, lam: float, J0: int) -> float:
    return math.sqrt(k_lam(l / lam ** J0, lam))


def zeta(l: int, n: int, N: int) -> complex:
    if abs(n) >= N or abs(n) > l:
        return 0.0
    if (N + n) % 2 == 0:          # mu = 0
        return 0.0
    q = min(N - 1, l - (1 + (-1) ** (N + l)) // 2)
    if q < 0 or abs(n) > q:
        return 0.0
    xi = 1.0 if (N - 1) % 2 == 0 else 1j
    return xi * math.sqrt(math.comb(q, (q - n) // 2) / 2.0 ** q)


def scale_count(L: int, lam: float) -> int:
    J = 0
    while lam ** J < L:
        J += 1
    return J


def scale_bandlimit(j: int, L: int, lam: float) -> int:
    return min(int(math.ceil(lam ** (j + 1) - 1e-12)), L)


def scale_azimuthal(j: int, L: int, N: int, lam: float) -> int:
    return min(N, scale_bandlimit(j, L, lam))


def scaling_bandlimit(L: int, lam: float, J0: int) -> int:
    return min(int(math.ceil(lam ** J0 - 1e-12)), L)


def wavelet_filter(j: int, L: int, N: int, lam: float) -> np.ndarray:
    """Psi^j_ln as [L, 2N-1] (index n+N-1), l < L."""
    out = np.zeros((L, 2 * N - 1), dtype=np.complex128)
    for l in range(L):
        kj = kappa(j, l, lam)
        if kj == 0.0:
            continue
        c = math.sqrt((2 * l + 1) / (8 * math.pi ** 2)) * kj
        for n in range(-(N - 1), N):
            out[l, n + N - 1] = c * zeta(l, n, N)
    return out


def scaling_filter(L: int, lam: float, J0: int) -> np.ndarray:
    """Phi_l0 as [L]."""
    return np.array([math.sqrt((2 * l + 1) / (4 * math.pi)) * eta(l, lam, J0) for l in range(L)])


def admissibility(L: int, N: int, lam: float, J0: int) -> np.ndarray:
    """4pi/(2l+1)|Phi_l0|^2 + 8pi^2/(2l+1) sum_{j>=J0} sum_n |Psi^j_ln|^2 (Section 3.1)."""
    J = scale_count(L, lam)
    Phi = scaling_filter(L, lam, J0)
    ls = np.arange(L)
    tot = 4 * np.pi / (2 * ls + 1) * np.abs(Phi) ** 2
    for j in range(J0, J + 1):
        Psi = wavelet_filter(j, L, N, lam)
        tot = tot + 8 * np.pi ** 2 / (2 * ls + 1) * np.sum(np.abs(Psi) ** 2, axis=1)
    return tot
