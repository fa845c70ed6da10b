// Host-side plan arithmetic for the s2w library: per-scale band limits,
// wavelet filters (paper Appendix A), the exact MW theta-quadrature matrices,
// Wigner-d recursion tables and DFT factorisations.  Pure C++ (no HIP).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace s2w {

struct ScaleInfo {
    int j = 0;              // wavelet scale index (J0..J)
    int L = 0;              // band limit of the scale, min(ceil(lambda^(j+1)), L)
    int N = 0;              // azimuthal band limit of the scale, min(N, L_j)
    std::vector<int> n;     // azimuthal orders n with nonzero filter: |n| < N_j, n = N-1 (mod 2)
};

struct Scales {
    int L = 0, N = 0, J0 = 0, J = 0, Lphi = 0;
    double lambda = 2.0;
    std::vector<ScaleInfo> s;   // k = j - J0
};

bool make_scales(int L, int N, double lambda, int J0, Scales &out, std::string &err);

// k_lambda(t) of Appendix A by tanh-sinh quadrature.
double k_lambda(double t, double lambda);

// Filters.  psi_mag[k][l * nn_k + i]: |Psi^j_{l, n_i}| (>= 0) for the scale's n list;
// the filter is Psi = xi * psi_mag with xi = 1 (N odd) or i (N even).
// phi[l] = Phi_l0.
struct Filters {
    std::vector<std::vector<double>> psi_mag;
    std::vector<double> phi;
    bool xi_imag = false;
};
void make_filters(const Scales &S, Filters &F);

// kappa_lambda(t)^2 = k_lambda(t/lambda) - k_lambda(t), as one integral over [t/lambda, t].
double kappa2_lambda(double t, double lambda);

// Radial Laguerre rule (ball, Section 2.3): nodes r_k = tau x_k with x_k the P roots
// of L^{(2)}_P, weights W_k = tau^3 e^{x_k} w_k (w_k the Gauss weights for x^2 e^{-x})
// so that f_p = sum_k W_k K_p(r_k) f(r_k) is exact for p < P.
struct LaguerreRule {
    int P = 0;
    double tau = 1.0;
    std::vector<double> x, r, W;
};
void laguerre_rule(int P, double tau, LaguerreRule &R);
// K_p(r_k) = sqrt(p!/(p+2)!) e^{-x_k/2} L^{(2)}_p(x_k) / tau^{3/2} for p < Pb: [Pb][nodes].
void laguerre_basis(const LaguerreRule &R, int Pb, std::vector<double> &K);

// Exact MW theta-quadrature matrix, row-major [L][L].
void theta_matrix(int L, int sigma, std::vector<double> &T);

// Grid tables for band limit L: cos(theta_b), cos(theta_b/2), sin(theta_b/2) and
// the relative rounding residuals of the half-angle values (for accurate powers).
struct ThetaTables {
    std::vector<double> cth, cth_lo, ch, sh, ch_eps, sh_eps;   // cos(theta) = cth + cth_lo (double-double)
};
void theta_tables(int L, ThetaTables &T);

// Scaled three-term l-recursion for d^l_mn(theta):
//   d^l = S_l e^l,  e^{l+1} = (A_l cos(theta) - B_l) e^l - e^{l-1},  l >= l0 = max(|m|,|n|),
//   e^{l0} = d^{l0}, e^{l0-1} = 0.
// Tables for n in `ns` and m = 0..L-1 laid out [ni][m][l] (l = 0..L-1, zero below l0),
// together with the start value d^{l0}_mn(theta) = sign * sqrt(C(2 l0, l0 + k))
// * cos^{|m+n|}(theta/2) sin^{|m-n|}(theta/2), with sign * sqrt(C) = start_mant * 2^start_exp.
struct RecTables {
    int L = 0;
    std::vector<int> ns;
    std::vector<double> A, B, S;      // [ni][m][l]
    std::vector<double> start_mant;   // [ni][m]
    std::vector<int> start_exp;       // [ni][m]
};
void rec_tables(int L, const std::vector<int> &ns, RecTables &R);

// Samples next to each pole whose d^l_mn come from the polar table instead of
// the FP64 recursion (0 for small L, where the recursion error stays small).
int polar_count(int L);
// d^l_mn(theta_b) at the 2 np samples nearest the poles (b < np and b >= L - np),
// layout [ni][m][p][l], p < np: b = p, else b = L - 2 np + p.
void polar_table(int L, const std::vector<int> &ns, int np, std::vector<double> &out);

// Host evaluation of d^l_mn(theta_b) as the device computes it: the FP64
// recursion, with the polar samples from the polar table (tests).
void host_wigner_d(int L, int m, int n, std::vector<double> &out);

// Prime-factor (Good-Thomas) factorisation n = n1 * n2, gcd(n1, n2) = 1.
struct PfaPlan {
    int n = 0, n1 = 0, n2 = 0;
    int e1 = 0, e2 = 0;               // output index a = (a1 * e1 + a2 * e2) mod n
    std::vector<double> w1, w2;       // cos, sin interleaved: w1[2k] = cos(2 pi k/n1), w1[2k+1] = sin(...)
};
void pfa_plan(int n, PfaPlan &P);

}  // namespace s2w
