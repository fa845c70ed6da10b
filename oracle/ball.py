"""Directional scale-discretised wavelets on the ball B^3 = R+ x S^2 (oracle;
test infrastructure only).

Paper Section 2.3 (functions on the ball), Section 3.2 (ball wavelets),
Section 5 (eq:forward_ball_wavelet, eq:synthesis_b3, Algorithm 2) and
Appendix A.3-A.4:

  K_p(r) = sqrt(p!/(p+2)!) e^{-r/(2 tau)} tau^{-3/2} L^{(2)}_p(r/tau)       (Laguerre basis)
  f_p = int_0^inf r^2 f(r) K_p(r) dr   (eq:flag),   f(r) = sum_p f_p K_p(r)   (eq:ilag)
  Z: f(r, omega) -> f_lmp = sum_k W_k K_p(r_k) [Y f(r_k, .)]_lm              (eq:forward_spherical_laguerre)
  (W^{Psi^{jj'}})^l_mnp = 8pi^2/(2l+1) f_lmp Psi^{jj'*}_lnp                   (eq:wig_lag_wav_coeffs)
  (W^Phi)_lmp = sqrt(4pi/(2l+1)) f_lmp Phi*_l0p                              (eq:wig_lag_scal_coeffs)
  Psi^{jj'}_lmp = sqrt((2l+1)/(8pi^2)) kappa^j(l) kappa^{j'}(p) zeta_lm      (Appendix A.4)
  analysis   W^{jj'} = Q^{-1} N Psi^{jj'} Z f,  W^Phi = Z^{-1} Phi Z f       (eq:forward_ball_wavelet)
  synthesis  f = Z^{-1}( Phi Z W^Phi + sum_{jj'} Psi^{jj' dagger} Q W^{jj'} ) (eq:synthesis_b3)

Radial sampling: r_k = tau x_k with x_k the P roots of L^{(2)}_P (generalised
Gauss-Laguerre, weight x^2 e^{-x}); for a radially band-limited f (p < P) the
integrand r^2 f K_p is e^{-x} times a polynomial of degree <= 2P-2, so the
P-point rule is exact.  Weights are the Christoffel numbers of the rule,
W_k = tau^3 / sum_{p<P} psi_p(x_k)^2 with psi_p(x) = sqrt(p!/(p+2)!) e^{-x/2}
L^{(2)}_p(x) (the e^{x_k} of the Gauss weight is absorbed, so nothing
underflows), and psi_p comes from the three-term Laguerre recursion
    psi_{p+1} = ((2p+3-x) psi_p - sqrt(p(p+2)) psi_{p-1}) / sqrt((p+1)(p+3)).

Readings (the paper is silent, garbled or self-contradictory here):
  * radial band limit: P coefficients p = 0..P-1 on P nodes, tau = 1 unless given;
  * radial scales run upward like the angular ones: kappa^{j'}(p) =
    kappa_nu(p/nu^{j'}), J' the smallest integer with nu^{J'} >= P, scale j'
    sampled on the P_{j'} = min(ceil(nu^{j'+1}), P) nodes of its own rule;
  * the scaling function as printed does not satisfy the admissibility
    condition; it is taken from the condition itself:
      4pi/(2l+1) |Phi_l0p|^2 = a + b - a b,  a = k_lam(l/lam^J0), b = k_nu(p/nu^J0'),
    i.e. 1 - sum_{j>=J0, j'>=J0'} kappa_j(l)^2 kappa_{j'}(p)^2;
  * the scaling coefficients are kept at the full (L, P) resolution, since
    their support is the union of a low-l band over all p and a low-p band
    over all l;
  * Wigner-Laguerre basis Q^l_mnp = K_p D^l_mn with the SO(3) conventions of
    the sphere transform (forward against D, inverse with D*).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_genlaguerre

from . import filters, mw, wavelets


# ------------------------------------------------------------- radial ------

def laguerre_psi(P: int, x: np.ndarray) -> np.ndarray:
    """psi_p(x) = sqrt(p!/(p+2)!) e^{-x/2} L^{(2)}_p(x) for p < P: [P, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((P, x.size))
    if P == 0:
        return out
    out[0] = np.exp(-0.5 * x) / math.sqrt(2.0)
    if P > 1:
        out[1] = (3.0 - x) * out[0] / math.sqrt(3.0)
    for p in range(1, P - 1):
        out[p + 1] = ((2 * p + 3 - x) * out[p] - math.sqrt(p * (p + 2.0)) * out[p - 1]) \
            / math.sqrt((p + 1.0) * (p + 3.0))
    return out


def laguerre_nodes(P: int) -> np.ndarray:
    """Roots x_k of L^{(2)}_P (ascending): a library eigenvalue estimate, then
    Newton steps on psi_P (same roots, bounded values)."""
    if P == 0:
        return np.zeros(0)
    x, _ = roots_genlaguerre(P, 2)
    x = np.array(x, dtype=np.float64)
    for _ in range(3):
        ps = laguerre_psi(P + 1, x)
        # with psi_p = c_p e^{-x/2} L_p, c_p = 1/sqrt((p+1)(p+2)) and
        # x L_P' = P L_P - (P+2) L_{P-1}:  psi_P / psi_P' = psi_P / (D / x - psi_P / 2),
        # D = P psi_P - sqrt(P (P+2)) psi_{P-1}
        D = P * ps[P] - math.sqrt(P * (P + 2.0)) * ps[P - 1]
        x = x - ps[P] / (D / x - 0.5 * ps[P])
    return np.sort(x)


class Radial:
    """P-point Laguerre rule: nodes r_k, weights W_k, basis values K_p(r_k)."""

    def __init__(self, P: int, tau: float = 1.0):
        self.P, self.tau = P, float(tau)
        self.x = laguerre_nodes(P)
        self.r = self.tau * self.x
        psi = laguerre_psi(P, self.x)                              # [p, k]
        self.K = psi / self.tau ** 1.5                             # K_p(r_k)
        self.W = self.tau ** 3 / np.sum(psi ** 2, axis=0)          # tau^3 e^{x_k} x Christoffel number

    def basis(self, Pb: int) -> np.ndarray:
        """K_p(r_k) for p < Pb at this rule's nodes: [Pb, P]."""
        return laguerre_psi(Pb, self.x) / self.tau ** 1.5

    def forward(self, f: np.ndarray) -> np.ndarray:
        """f_p = sum_k W_k K_p(r_k) f(r_k) over the leading axis (eq:flag, exact for p < P)."""
        return np.tensordot(self.K * self.W[None, :], f, axes=(1, 0))

    def inverse(self, fp: np.ndarray) -> np.ndarray:
        """f(r_k) = sum_p f_p K_p(r_k) over the leading axis (eq:ilag)."""
        return np.tensordot(self.K.T, fp, axes=(1, 0))


# ------------------------------------------------------------ filters ------

class BallPlan:
    """Angular and radial scales, filters and rules for (L, N, P, lam, nu, J0, J0', tau)."""

    def __init__(self, L: int, N: int, P: int, lam: float = 2.0, nu: float = 2.0,
                 J0: int = 0, J0p: int = 0, tau: float = 1.0):
        self.L, self.N, self.P = L, N, P
        self.lam, self.nu, self.J0, self.J0p, self.tau = float(lam), float(nu), J0, J0p, float(tau)
        self.ang = wavelets.Plan(L, N, lam, J0)                    # angular scales and Psi^j
        self.Jp = filters.scale_count(P, nu)
        self.rscales = list(range(J0p, self.Jp + 1))
        self.Pj = [filters.scale_bandlimit(jp, P, nu) for jp in self.rscales]
        self.kappa_p = [np.array([filters.kappa(jp, p, nu) for p in range(P)]) for jp in self.rscales]
        self.rad = Radial(P, tau)
        self.rad_j = [Radial(Pj, tau) for Pj in self.Pj]
        a = np.array([filters.k_lam(l / self.lam ** J0, self.lam) for l in range(L)])
        b = np.array([filters.k_lam(p / self.nu ** J0p, self.nu) for p in range(P)])
        # sqrt(4pi/(2l+1)) Phi_l0p  [P, L]
        self.phi = np.sqrt(np.clip(a[None, :] + b[:, None] - a[None, :] * b[:, None], 0.0, None))

    def admissibility(self) -> np.ndarray:
        """4pi/(2l+1)|Phi|^2 + 8pi^2/(2l+1) sum_{j j' n} |Psi^{jj'}_lnp|^2 as [P, L] (Section 3.2)."""
        L = self.L
        ls = np.arange(L)
        tot = self.phi ** 2
        for k in range(len(self.ang.scales)):
            ang = 8 * np.pi ** 2 / (2 * ls + 1) * np.sum(np.abs(self.ang.Psi[k]) ** 2, axis=1)   # [L]
            for i in range(len(self.rscales)):
                tot = tot + self.kappa_p[i][:, None] ** 2 * ang[None, :]
        return tot


# -------------------------------------------------------- transforms -------

def sl_forward(f: np.ndarray, BP: BallPlan) -> np.ndarray:
    """Z: f [P, L, 2L-1] on the radial nodes -> f_lmp [P, L, 2L-1] (eq:forward_spherical_laguerre)."""
    L = BP.L
    flm = np.stack([mw.sht_forward(f[k], L) for k in range(BP.P)])
    return BP.rad.forward(flm)


def sl_inverse(flmp: np.ndarray, BP: BallPlan, real: bool = True) -> np.ndarray:
    """Z^{-1}: f_lmp -> f [P, L, 2L-1] (eq:inverse_spherical_laguerre)."""
    L = BP.L
    flm = BP.rad.inverse(flmp)
    out = np.stack([mw.sht_inverse(flm[k], L) for k in range(BP.P)])
    return np.real(out) if real else out


def _shell_coeffs(flmp: np.ndarray, BP: BallPlan, i: int) -> np.ndarray:
    """g^{j'}_lm(r'_k) = sum_p K_p(r'_k) kappa^{j'}(p) f_lmp on the P_{j'} nodes of scale j'."""
    Pj = BP.Pj[i]
    Kb = BP.rad_j[i].basis(BP.P)                                  # [p < P, k < Pj]
    return np.tensordot((Kb * BP.kappa_p[i][:, None]).T, flmp, axes=(1, 0))   # [Pj, L, 2L-1]


def analysis_lmp(flmp: np.ndarray, BP: BallPlan, real: bool = True):
    """Analysis from spherical-Laguerre coefficients f_lmp [P, L, 2L-1].

    Returns (wav, scal): wav[(i, k)] = W^{j'_i j_k} [P_{j'}, 2N_j-1, L_j, 2L_j-1] on the
    nodes of the P_{j'}-point rule; scal = W^Phi [P, L, 2L-1] on the full rule."""
    L = BP.L
    scal = sl_inverse(BP.phi[:, :, None] * flmp, BP, real=real)
    wav = {}
    for i in range(len(BP.rscales)):
        g = _shell_coeffs(flmp, BP, i)
        for k in range(len(BP.ang.scales)):
            wav[(i, k)] = _angular_scale(g, BP, k, real)
    return wav, scal


def _angular_scale(g: np.ndarray, BP: BallPlan, k: int, real: bool) -> np.ndarray:
    """Per shell: W^j = D_j^{-1}[8pi^2/(2l+1) g_lm Psi^{j*}_ln]."""
    A = BP.ang
    L = BP.L
    Lj, Nj = A.Lj[k], A.Nj[k]
    lj = np.arange(Lj)
    psi = np.conj(A.psi(k))
    out = []
    for s in range(g.shape[0]):
        fl = g[s][:Lj, L - Lj:L + Lj - 1]
        what = (8 * np.pi ** 2 / (2 * lj + 1))[None, :, None] * fl[None, :, :] * psi.T[:, :, None]
        w = mw.wigner_inverse(what, Lj, Nj)
        out.append(np.real(w) if real else w)
    return np.stack(out)


def analysis(f: np.ndarray, BP: BallPlan):
    """Real ball map f [P, L, 2L-1] on the radial nodes -> (wav, scal) (eq:forward_ball_wavelet)."""
    return analysis_lmp(sl_forward(f, BP), BP)


def synthesis_lmp(wav, scal, BP: BallPlan) -> np.ndarray:
    """(W^{jj'}, W^Phi) -> f_lmp [P, L, 2L-1] before the final Z^{-1} (eq:synthesis_b3)."""
    L = BP.L
    A = BP.ang
    flmp = BP.phi[:, :, None] * sl_forward(scal, BP)
    for i in range(len(BP.rscales)):
        Pj = BP.Pj[i]
        acc = np.zeros((Pj, L, 2 * L - 1), dtype=np.complex128)    # sum_j Psi^dagger D W per shell
        for k in range(len(A.scales)):
            Lj, Nj = A.Lj[k], A.Nj[k]
            psi = A.psi(k)
            for s in range(Pj):
                what = mw.wigner_forward(wav[(i, k)][s], Lj, Nj)
                acc[s, :Lj, L - Lj:L + Lj - 1] += np.einsum("nlm,ln->lm", what, psi)
        Kb = BP.rad_j[i].basis(BP.P)                               # [p, k]
        Wk = BP.rad_j[i].W
        flmp += np.tensordot(Kb * Wk[None, :] * BP.kappa_p[i][:, None], acc, axes=(1, 0))
    return flmp


def synthesis(wav, scal, BP: BallPlan) -> np.ndarray:
    """(W^{jj'}, W^Phi) -> real ball map f [P, L, 2L-1]."""
    return sl_inverse(synthesis_lmp(wav, scal, BP), BP)


# ------------------------------------------------------------- adjoints ----
# Literal transposes of the real-linear ball maps above (the adjoint transforms of
# Section 5.2), stage by stage in reverse order, for the real inner product of the
# sample arrays.

def _sl_forward_adjoint(g: np.ndarray, BP: BallPlan) -> np.ndarray:
    """Transpose of sl_forward: cotangent of f_lmp [P, L, 2L-1] -> real map cotangent on the nodes."""
    L = BP.L
    y = np.tensordot((BP.rad.K * BP.rad.W[None, :]).T, g, axes=(1, 0))     # [k, L, 2L-1]
    return np.real(np.stack([mw.sht_forward_adjoint(y[k], L) for k in range(BP.P)]))


def _sl_inverse_adjoint(g: np.ndarray, BP: BallPlan) -> np.ndarray:
    """Transpose of sl_inverse (real maps): map cotangent on the nodes -> cotangent of f_lmp."""
    L = BP.L
    gl = np.stack([mw.sht_inverse_adjoint(np.asarray(g[k], dtype=np.complex128), L) for k in range(BP.P)])
    return np.tensordot(BP.rad.K, gl, axes=(1, 0))


def analysis_adjoint(gwav, gscal, BP: BallPlan) -> np.ndarray:
    """Transpose of analysis(): (g W^{jj'}, g W^Phi) -> g f [P, L, 2L-1]."""
    L, P = BP.L, BP.P
    A = BP.ang
    gflmp = BP.phi[:, :, None] * _sl_inverse_adjoint(gscal, BP)
    for i in range(len(BP.rscales)):
        Pj = BP.Pj[i]
        gg = np.zeros((Pj, L, 2 * L - 1), dtype=np.complex128)     # cotangent of g^{j'}_lm(r'_k)
        for k in range(len(A.scales)):
            Lj, Nj = A.Lj[k], A.Nj[k]
            lj = np.arange(Lj)
            psi = A.psi(k)
            for s in range(Pj):
                ga = mw.wigner_inverse_adjoint(np.asarray(gwav[(i, k)][s], dtype=np.complex128), Lj, Nj)
                gg[s, :Lj, L - Lj:L + Lj - 1] += np.einsum("nlm,ln->lm", ga, psi) \
                    * (8 * np.pi ** 2 / (2 * lj + 1))[:, None]
        Kb = BP.rad_j[i].basis(P)                                   # [p, k]
        gflmp += np.tensordot(Kb * BP.kappa_p[i][:, None], gg, axes=(1, 0))
    return _sl_forward_adjoint(gflmp, BP)


def synthesis_adjoint(gf, BP: BallPlan):
    """Transpose of synthesis(): g f [P, L, 2L-1] -> (g W^{jj'}, g W^Phi)."""
    L, P = BP.L, BP.P
    A = BP.ang
    gflmp = _sl_inverse_adjoint(gf, BP)
    gscal = _sl_forward_adjoint(BP.phi[:, :, None] * gflmp, BP)
    gwav = {}
    for i in range(len(BP.rscales)):
        Pj = BP.Pj[i]
        Kb = BP.rad_j[i].basis(P)                                   # [p, k]
        M = Kb * BP.rad_j[i].W[None, :] * BP.kappa_p[i][:, None]
        gacc = np.tensordot(M.T, gflmp, axes=(1, 0))               # [Pj, L, 2L-1]
        for k in range(len(A.scales)):
            Lj, Nj = A.Lj[k], A.Nj[k]
            psi = A.psi(k)
            out = []
            for s in range(Pj):
                gk = gacc[s, :Lj, L - Lj:L + Lj - 1]
                g_nlm = np.conj(psi).T[:, :, None] * gk[None, :, :]
                out.append(np.real(mw.wigner_forward_adjoint(g_nlm, Lj, Nj)))
            gwav[(i, k)] = np.stack(out)
    return gwav, gscal


# ------------------------------------------------------ Wigner-Laguerre -----

def wl_forward(f: np.ndarray, BP: BallPlan, N: int) -> np.ndarray:
    """Wigner-Laguerre transform (Section 2.5: basis Q^l_mnp = K_p D^l_mn, with the SO(3)
    conventions of the sphere transforms, reading 17): samples f [P, 2N-1, L, 2L-1] on the
    radial nodes x the MW SO(3) grid -> coefficients [P, 2N-1, L, 2L-1] ("nlm" per p).  The
    SO(3) forward transform on every shell, then the radial forward (eq:flag on the rule)."""
    per = np.stack([mw.wigner_forward(f[k], BP.L, N) for k in range(BP.P)])
    return BP.rad.forward(per)


def wl_inverse(fh: np.ndarray, BP: BallPlan, N: int, real: bool = True) -> np.ndarray:
    """Inverse Wigner-Laguerre transform (eq:wiglag_inverse): radial synthesis at the nodes,
    then the SO(3) inverse on every shell."""
    per = BP.rad.inverse(fh)
    out = np.stack([mw.wigner_inverse(per[k], BP.L, N) for k in range(BP.P)])
    return np.real(out) if real else out
