"""Directional scale-discretised wavelet transform on the sphere (oracle;
test infrastructure only).

Paper Section 4.1 and Algorithm 1:
  analysis   W^{Psi^j} = D^{-1}_j N Psi^j Y f      (eq:analysis_s2), with
             (W^{Psi^j})^l_mn = 8pi^2/(2l+1) f_lm Psi^{j*}_ln   (eq:wigner_wav_coeffs)
             W^Phi = Y^{-1} Phi Y f, (W^Phi)_lm = sqrt(4pi/(2l+1)) f_lm Phi*_l0
             (eq:harmonic_scal_coeffs)
  synthesis  f = Y^{-1}( Phi Y W^Phi + sum_j Psi^{j dagger} D W^{Psi^j} )   (eq:synthesis_s2)
Multiresolution (Section 3.3): scale j is transformed at its own band limits
(L_j, N_j); the scaling part at L_phi.  Scales run j = J0..J.

The adjoint is the literal transpose of the analysis under the real inner
product of sample arrays (what a gradient needs; it is not the synthesis).
"""
from __future__ import annotations

import numpy as np

from . import filters, mw


class Plan:
    """Filters and per-scale band limits for (L, N, lam, J0)."""

    def __init__(self, L: int, N: int, lam: float = 2.0, J0: int = 0):
        self.L, self.N, self.lam, self.J0 = L, N, float(lam), J0
        self.J = filters.scale_count(L, lam)
        self.scales = list(range(J0, self.J + 1))
        self.Lj = [filters.scale_bandlimit(j, L, lam) for j in self.scales]
        self.Nj = [filters.scale_azimuthal(j, L, N, lam) for j in self.scales]
        self.Lphi = filters.scaling_bandlimit(L, lam, J0)
        self.Psi = [filters.wavelet_filter(j, L, N, lam) for j in self.scales]  # [L, 2N-1]
        self.Phi = filters.scaling_filter(L, lam, J0)

    def psi(self, k: int) -> np.ndarray:
        """Psi^j_ln restricted to l < L_j, |n| < N_j: [L_j, 2N_j-1]."""
        Lj, Nj, N = self.Lj[k], self.Nj[k], self.N
        return self.Psi[k][:Lj, N - Nj:N + Nj - 1]


def _embed(flm: np.ndarray, L: int, Lsub: int) -> np.ndarray:
    """Restrict flm [L, 2L-1] to band limit Lsub: [Lsub, 2Lsub-1]."""
    return flm[:Lsub, L - Lsub:L + Lsub - 1]


def _extend(flm_sub: np.ndarray, Lsub: int, L: int) -> np.ndarray:
    out = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    out[:Lsub, L - Lsub:L + Lsub - 1] = flm_sub
    return out


def analysis(f: np.ndarray, P: Plan):
    """Real map f [L, 2L-1] -> (list of W^j [2N_j-1, L_j, 2L_j-1], W^Phi [L_phi, 2L_phi-1])."""
    L = P.L
    flm = mw.sht_forward(f, L)
    return analysis_lm(flm, P)


def analysis_lm(flm: np.ndarray, P: Plan, real: bool = True):
    """Analysis from harmonic coefficients flm [L, 2L-1]."""
    L = P.L
    ls = np.arange(L)
    Lp = P.Lphi
    wphi = np.sqrt(4 * np.pi / (2 * ls + 1))[:, None] * flm * np.conj(P.Phi)[:, None]
    scal = mw.sht_inverse(_embed(wphi, L, Lp), Lp)
    wav = []
    for k in range(len(P.scales)):
        Lj, Nj = P.Lj[k], P.Nj[k]
        fl = _embed(flm, L, Lj)                                   # [l, m]
        lj = np.arange(Lj)
        psi = np.conj(P.psi(k))                                   # [l, n]
        what = (8 * np.pi ** 2 / (2 * lj + 1))[None, :, None] * fl[None, :, :] * psi.T[:, :, None]
        wav.append(mw.wigner_inverse(what, Lj, Nj))
    if real:
        wav = [np.real(w) for w in wav]
        scal = np.real(scal)
    return wav, scal


def synthesis_lm(wav, scal, P: Plan) -> np.ndarray:
    """(W^j, W^Phi) -> harmonic coefficients flm [L, 2L-1] (before the final Y^{-1})."""
    L = P.L
    ls = np.arange(L)
    Lp = P.Lphi
    sphi = _extend(mw.sht_forward(scal, Lp), Lp, L)
    flm = np.sqrt(4 * np.pi / (2 * ls + 1))[:, None] * P.Phi[:, None] * sphi
    for k in range(len(P.scales)):
        Lj, Nj = P.Lj[k], P.Nj[k]
        what = mw.wigner_forward(wav[k], Lj, Nj)                   # [n, l, m]
        psi = P.psi(k)                                             # [l, n]
        contrib = np.einsum("nlm,ln->lm", what, psi)
        flm += _extend(contrib, Lj, L)
    return flm


def synthesis(wav, scal, P: Plan) -> np.ndarray:
    """(W^j, W^Phi) -> real map f [L, 2L-1]."""
    return np.real(mw.sht_inverse(synthesis_lm(wav, scal, P), P.L))


def analysis_adjoint(gwav, gscal, P: Plan) -> np.ndarray:
    """Transpose of the real-linear analysis map: (gW^j, gW^Phi) -> g f [L, 2L-1].

    Literal transposes of each stage of analysis(), in reverse order:
    W^j = D^{-1}_j(a^j), a^j = 8pi^2/(2l+1) conj(Psi) * Y f; W^Phi = Y^{-1}(c Phi* Y f).
    """
    L = P.L
    ls = np.arange(L)
    Lp = P.Lphi
    gflm = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    g = mw.sht_inverse_adjoint(np.asarray(gscal, dtype=np.complex128), Lp)
    gflm += np.sqrt(4 * np.pi / (2 * ls + 1))[:, None] * P.Phi[:, None] * _extend(g, Lp, L)
    for k in range(len(P.scales)):
        Lj, Nj = P.Lj[k], P.Nj[k]
        ga = mw.wigner_inverse_adjoint(np.asarray(gwav[k], dtype=np.complex128), Lj, Nj)  # [n,l,m]
        lj = np.arange(Lj)
        psi = P.psi(k)                                             # conj(conj(Psi)) = Psi
        contrib = np.einsum("nlm,ln->lm", ga, psi) * (8 * np.pi ** 2 / (2 * lj + 1))[:, None]
        gflm += _extend(contrib, Lj, L)
    return np.real(mw.sht_forward_adjoint(gflm, L))


def synthesis_adjoint(gf, P: Plan):
    """Transpose of the real-linear synthesis map: g f [L, 2L-1] -> (list of g W^j, g W^Phi).

    Literal transposes of each stage of synthesis(), in reverse order:
    f = Re Y^{-1} flm,  flm = sqrt(4pi/(2l+1)) Phi_l Y_{L_phi} W^Phi + sum_j sum_n Psi^j_ln (D_j W^j)^l_mn.
    """
    L = P.L
    ls = np.arange(L)
    Lp = P.Lphi
    gflm = mw.sht_inverse_adjoint(np.asarray(gf, dtype=np.complex128), L)
    gs = np.sqrt(4 * np.pi / (2 * ls + 1))[:, None] * P.Phi[:, None] * gflm
    gscal = np.real(mw.sht_forward_adjoint(_embed(gs, L, Lp), Lp))
    gwav = []
    for k in range(len(P.scales)):
        Lj, Nj = P.Lj[k], P.Nj[k]
        psi = P.psi(k)                                             # [l, n]
        gk = _embed(gflm, L, Lj)                                   # [l, m]
        g_nlm = np.conj(psi).T[:, :, None] * gk[None, :, :]        # transpose of the sum over n
        gwav.append(np.real(mw.wigner_forward_adjoint(g_nlm, Lj, Nj)))
    return gwav, gscal


# ------------------------------------------------------------ spin-s ------
# Spin-s maps (Section 4.1 with the spin subscripts kept, Section 2.1 eq:u1sym):
# the wavelet and scaling coefficients depend on the map only through its spin-s
# harmonic coefficients sf_lm (eq:wigner_wav_coeffs, eq:harmonic_scal_coeffs), with the
# same filters as for spin 0 (Appendix A: the dictionary's harmonic coefficients carry no
# spin-dependent factor).  The wavelet coefficients live on SO(3) and the scaling
# coefficients are a spin-0 map; both are complex.

def analysis_spin(f: np.ndarray, P: Plan, s: int):
    """Complex spin-s map f [L, 2L-1] -> (complex W^j, complex W^Phi)."""
    return analysis_lm(mw.spin_sht_forward(f, P.L, s), P, real=False)


def synthesis_spin(wav, scal, P: Plan, s: int) -> np.ndarray:
    """(complex W^j, complex W^Phi) -> complex spin-s map f [L, 2L-1]."""
    return mw.spin_sht_inverse(synthesis_lm(wav, scal, P), P.L, s)
