// Host-side plan arithmetic (see s2w_host.h).
#include "s2w_host.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

namespace s2w {

namespace {

constexpr long double kPiL = 3.141592653589793238462643383279502884L;

int ceil_pow(double lambda, int e)
{
    // ceil(lambda^e) robust to rounding when lambda^e is an integer
    long double v = powl((long double)lambda, (long double)e);
    long double r = roundl(v);
    if (fabsl(v - r) < 1e-9L * std::max((long double)1, r)) return (int)r;
    return (int)ceill(v);
}

template <class F>
void parallel_for(int n, F &&f)
{
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 64 || nt == 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int i = (int)t; i < n; i += (int)nt) f(i);
        });
    for (auto &x : th) x.join();
}

}  // namespace

bool make_scales(int L, int N, double lambda, int J0, Scales &out, std::string &err)
{
    if (L < 2) { err = "L must be >= 2"; return false; }
    if (N < 1 || N > L) { err = "N must satisfy 1 <= N <= L"; return false; }
    if (!(lambda > 1.0) || !std::isfinite(lambda)) { err = "lambda must be > 1"; return false; }
    int J = 0;
    while (powl((long double)lambda, (long double)J) < (long double)L - 1e-9L) {
        ++J;
        if (J > 64) { err = "too many scales"; return false; }
    }
    if (J0 < 0 || J0 > J) { err = "J0 must satisfy 0 <= J0 <= J"; return false; }
    out = Scales{};
    out.L = L; out.N = N; out.J0 = J0; out.J = J; out.lambda = lambda;
    out.Lphi = std::min(ceil_pow(lambda, J0), L);
    for (int j = J0; j <= J; ++j) {
        ScaleInfo si;
        si.j = j;
        si.L = std::min(ceil_pow(lambda, j + 1), L);
        si.N = std::min(N, si.L);
        for (int n = -(si.N - 1); n <= si.N - 1; ++n)
            if (((n - (N - 1)) % 2 + 2) % 2 == 0) si.n.push_back(n);
        out.s.push_back(si);
    }
    return true;
}

// ---------------------------------------------------------------- filters ---

namespace {

long double bump2_over_t(long double x, long double lambda)
{
    long double u = 2.0L * lambda / (lambda - 1.0L) * (x - 1.0L / lambda) - 1.0L;
    if (fabsl(u) >= 1.0L) return 0.0L;
    return expl(-2.0L / (1.0L - u * u)) / x;
}

// tanh-sinh quadrature of bump^2/t on [a, b]
long double ts_integral(long double a, long double b, long double lambda)
{
    if (b <= a) return 0.0L;
    const long double h = 1.0L / 64.0L;
    const long double c = 0.5L * (a + b), r = 0.5L * (b - a);
    long double acc = 0.0L;
    for (int k = -260; k <= 260; ++k) {
        long double t = k * h;
        long double sh = sinhl(t), chh = coshl(t);
        long double u = 0.5L * kPiL * sh;
        long double cu = coshl(u);
        long double x = c + r * tanhl(u);
        long double w = r * h * 0.5L * kPiL * chh / (cu * cu);
        if (!(w > 0.0L) || !std::isfinite((double)w)) continue;
        if (x <= a || x >= b) continue;
        acc += w * bump2_over_t(x, lambda);
    }
    return acc;
}

}  // namespace

double k_lambda(double t, double lambda)
{
    const long double lam = lambda;
    if (t <= 1.0 / lambda) return 1.0;
    if (t >= 1.0) return 0.0;
    long double num = ts_integral((long double)t, 1.0L, lam);
    long double den = ts_integral(1.0L / lam, 1.0L, lam);
    return (double)(num / den);
}

void make_filters(const Scales &S, Filters &F)
{
    const int L = S.L, N = S.N;
    F.xi_imag = ((N - 1) % 2) != 0;
    // eta^2 = k_lambda(l / lambda^J0)
    std::vector<double> K(L);
    parallel_for(L, [&](int l) {
        long double t = (long double)l / powl((long double)S.lambda, (long double)S.J0);
        K[l] = k_lambda((double)t, S.lambda);
    });
    const long double kden = ts_integral(1.0L / (long double)S.lambda, 1.0L, S.lambda);
    F.phi.assign(L, 0.0);
    for (int l = 0; l < L; ++l)
        F.phi[l] = sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * sqrt(std::max(0.0, K[l]));
    F.psi_mag.clear();
    for (size_t k = 0; k < S.s.size(); ++k) {
        const ScaleInfo &si = S.s[k];
        const int nn = (int)si.n.size();
        std::vector<double> P((size_t)si.L * nn, 0.0);
        for (int l = 0; l < si.L; ++l) {
            // kappa^2 = k(t/lambda) - k(t) as one integral of s^2/t' over [t/lambda, t]
            const long double t = (long double)l / powl((long double)S.lambda, (long double)si.j);
            const long double lo = std::max(t / (long double)S.lambda, 1.0L / (long double)S.lambda);
            const long double hi = std::min(t, 1.0L);
            double kap2 = (hi > lo) ? (double)(ts_integral(lo, hi, S.lambda) / kden) : 0.0;
            if (!(kap2 > 0.0)) continue;
            double base = sqrt((2.0 * l + 1.0) / (8.0 * M_PI * M_PI)) * sqrt(kap2);
            int q = std::min(N - 1, l - ((((N + l) % 2) == 0) ? 1 : 0));
            for (int i = 0; i < nn; ++i) {
                int n = si.n[i];
                if (q < 0 || std::abs(n) > q || ((q - n) % 2) != 0) continue;
                // sqrt(C(q, (q-n)/2) / 2^q)
                int kk = (q - n) / 2;
                long double lc = lgammal(q + 1.0L) - lgammal(kk + 1.0L) - lgammal(q - kk + 1.0L)
                                 - q * logl(2.0L);
                P[(size_t)l * nn + i] = base * (double)expl(0.5L * lc);
            }
        }
        F.psi_mag.push_back(std::move(P));
    }
}

double kappa2_lambda(double t, double lambda)
{
    const long double lam = lambda;
    const long double lo = std::max((long double)t / lam, 1.0L / lam), hi = std::min((long double)t, 1.0L);
    if (!(hi > lo)) return 0.0;
    return (double)(ts_integral(lo, hi, lam) / ts_integral(1.0L / lam, 1.0L, lam));
}

// ------------------------------------------------------- Laguerre rule -----
//
// The monic polynomials orthogonal for x^2 e^{-x} obey
//   pi_{k+1} = (x - (2k+3)) pi_k - k(k+2) pi_{k-1},
// so the rule's nodes are the eigenvalues of the symmetric tridiagonal matrix
// with diagonal 2k+3 and off-diagonal sqrt(k(k+2)) (Golub-Welsch).  They are
// found by Sturm-sequence bisection in long double and polished by Newton steps
// on the orthonormal functions psi_p(x) = sqrt(p!/(p+2)!) e^{-x/2} L^{(2)}_p(x),
//   psi_{p+1} = ((2p+3-x) psi_p - sqrt(p(p+2)) psi_{p-1}) / sqrt((p+1)(p+3)),
// whose squares also give the Christoffel numbers: e^{x_k} w_k = 1 / sum_p psi_p(x_k)^2.

namespace {

void laguerre_psi(int P, long double x, std::vector<long double> &ps)
{
    ps.assign(P + 1, 0.0L);
    ps[0] = expl(-0.5L * x) / sqrtl(2.0L);
    if (P >= 1) ps[1] = (3.0L - x) * ps[0] / sqrtl(3.0L);
    for (int p = 1; p < P; ++p)
        ps[p + 1] = ((2.0L * p + 3.0L - x) * ps[p] - sqrtl((long double)p * (p + 2.0L)) * ps[p - 1]) /
                    sqrtl((p + 1.0L) * (p + 3.0L));
}

int sturm_below(int P, long double x)
{
    int cnt = 0;
    long double q = 0.0L;
    for (int k = 0; k < P; ++k) {
        const long double d = 2.0L * k + 3.0L;
        const long double e2 = (long double)k * (k + 2.0L);
        q = (k == 0) ? d - x : d - x - e2 / q;
        if (q == 0.0L) q = -1e-4000L;
        if (q < 0.0L) ++cnt;
    }
    return cnt;
}

}  // namespace

void laguerre_rule(int P, double tau, LaguerreRule &R)
{
    R.P = P;
    R.tau = tau;
    R.x.assign(P, 0.0);
    R.r.assign(P, 0.0);
    R.W.assign(P, 0.0);
    if (P <= 0) return;
    long double hi = 0.0L;
    for (int k = 0; k < P; ++k)
        hi = std::max(hi, 2.0L * k + 3.0L + sqrtl((long double)k * (k + 2.0L)) + sqrtl((k + 1.0L) * (k + 3.0L)));
    std::vector<long double> ps;
    for (int i = 0; i < P; ++i) {
        long double a = 0.0L, b = hi;
        for (int it = 0; it < 200 && b - a > 1e-19L * b; ++it) {
            const long double m = 0.5L * (a + b);
            if (sturm_below(P, m) > i) b = m;
            else a = m;
        }
        long double x = 0.5L * (a + b);
        for (int it = 0; it < 3; ++it) {
            laguerre_psi(P, x, ps);
            // x d/dx (e^{-x/2} c_P L_P) = P psi_P - sqrt(P(P+2)) psi_{P-1} - x psi_P / 2
            const long double D = P * ps[P] - sqrtl((long double)P * (P + 2.0L)) * ps[P - 1] - 0.5L * x * ps[P];
            if (D != 0.0L) x -= x * ps[P] / D;
        }
        laguerre_psi(P, x, ps);
        long double s2 = 0.0L;
        for (int p = 0; p < P; ++p) s2 += ps[p] * ps[p];
        R.x[i] = (double)x;
        R.r[i] = (double)((long double)tau * x);
        R.W[i] = (double)(powl((long double)tau, 3.0L) / s2);
    }
}

void laguerre_basis(const LaguerreRule &R, int Pb, std::vector<double> &K)
{
    K.assign((size_t)Pb * R.P, 0.0);
    std::vector<long double> ps;
    const long double s = powl((long double)R.tau, -1.5L);
    for (int k = 0; k < R.P; ++k) {
        laguerre_psi(std::max(Pb, 1), (long double)R.x[k], ps);
        for (int p = 0; p < Pb; ++p) K[(size_t)p * R.P + k] = (double)(ps[p] * s);
    }
}

// -------------------------------------------------- theta quadrature (MW) ---
//
// For F, d of band limit L and parity sigma on the torus, with n = 2L-1 samples
// theta_b = pi(2b+1)/n (b < L; b >= L obtained by parity), the Fourier
// coefficients are F^(p) = (1/n) sum_b' E[p][b'] F(theta_b') with
// E[p][b'] = e^{-ip theta_b'} + sigma e^{+ip theta_b'} (b' < L-1) and (-1)^p (b' = L-1),
// and int_0^pi F d sin = sum_{p,q} F^(p) d^(q) w(p+q), w(k) = int_0^pi e^{ikt} sin t dt.
// Hence T = (1/n^2) E^T W E.  Only the even-k part of w survives for the
// cos.cos (sigma = +1) and sin.sin (sigma = -1) blocks; the k = +-1 part enters the
// sigma = -1 row/column at theta = pi.

void theta_matrix(int L, int sigma, std::vector<double> &T)
{
    T.assign((size_t)L * L, 0.0);
    const int n = 2 * L - 1;
    const long double n2 = (long double)n * (long double)n;
    auto we = [](int k) -> long double {
        return (k % 2 == 0) ? 2.0L / (1.0L - (long double)k * (long double)k) : 0.0L;
    };
    std::vector<long double> th(L);
    for (int b = 0; b < L; ++b) th[b] = kPiL * (2.0L * b + 1.0L) / n;
    // V[q][b'] for q = 0..L-1 (cos case: even in q) or U[q][b'] (sin case: odd in q)
    std::vector<long double> V((size_t)L * L);
    parallel_for(L, [&](int bp) {
        std::vector<long double> cs(L);
        for (int p = 0; p < L; ++p) cs[p] = (sigma > 0) ? cosl(p * th[bp]) : sinl(p * th[bp]);
        for (int q = 0; q < L; ++q) {
            long double acc = 0.0L;
            if (sigma > 0) {
                acc = we(q);
                for (int p = 1; p < L; ++p) acc += cs[p] * (we(q + p) + we(q - p));
            } else {
                for (int p = 1; p < L; ++p) acc += cs[p] * (we(q + p) - we(q - p));
            }
            V[(size_t)q * L + bp] = acc;
        }
    });
    parallel_for(L, [&](int b) {
        std::vector<long double> cs(L);
        for (int q = 0; q < L; ++q) cs[q] = (sigma > 0) ? cosl(q * th[b]) : sinl(q * th[b]);
        for (int bp = 0; bp < L; ++bp) {
            long double acc;
            if (sigma > 0) {
                acc = V[bp];
                for (int q = 1; q < L; ++q) acc += 2.0L * cs[q] * V[(size_t)q * L + bp];
                acc *= 4.0L / n2;
                // theta = pi column/row carries E = (-1)^p = (1/2) 2cos(p pi)
                if (bp == L - 1) acc *= 0.5L;
                if (b == L - 1) acc *= 0.5L;
            } else {
                acc = 0.0L;
                for (int q = 1; q < L; ++q) acc += cs[q] * V[(size_t)q * L + bp];
                acc *= -8.0L / n2;
            }
            T[(size_t)b * L + bp] = (double)acc;
        }
    });
    if (sigma < 0) {
        // row/column theta = pi: E[p][L-1] = (-1)^p
        const long double sgn = ((L - 1) % 2 == 0) ? 1.0L : -1.0L;
        for (int b = 0; b < L - 1; ++b) {
            long double v = -2.0L * kPiL / n2 * sgn * sinl((L - 1) * th[b]);
            T[(size_t)b * L + (L - 1)] = (double)v;
            T[(size_t)(L - 1) * L + b] = (double)v;
        }
        long double corner = 0.0L;   // (1/n^2) sum_{p,q} w_e(p+q)
        for (int k = -(2 * L - 2); k <= 2 * L - 2; ++k) corner += (long double)(n - std::abs(k)) * we(k);
        T[(size_t)(L - 1) * L + (L - 1)] = (double)(corner / n2);
    }
}

void theta_tables(int L, ThetaTables &T)
{
    const int n = 2 * L - 1;
    T.cth.resize(L); T.cth_lo.resize(L); T.ch.resize(L); T.sh.resize(L); T.ch_eps.resize(L); T.sh_eps.resize(L);
    for (int b = 0; b < L; ++b) {
        long double th = kPiL * (2.0L * b + 1.0L) / n;
        long double c = cosl(0.5L * th), s = sinl(0.5L * th);
        if (b == L - 1) { c = 0.0L; s = 1.0L; th = kPiL; }
        // cos(theta) from the half angle, measured from the nearer pole, so that 1 - |cos|
        // keeps its relative precision there (the recursion is most sensitive near the poles)
        const long double ct = (2 * (2 * b + 1) < n) ? 1.0L - 2.0L * s * s : 2.0L * c * c - 1.0L;
        T.cth[b] = (b == L - 1) ? -1.0 : (double)ct;
        T.cth_lo[b] = (b == L - 1) ? 0.0 : (double)(ct - (long double)T.cth[b]);
        T.ch[b] = (double)c;
        T.sh[b] = (double)s;
        T.ch_eps[b] = (c != 0.0L) ? (double)((c - (long double)T.ch[b]) / (long double)T.ch[b]) : 0.0;
        T.sh_eps[b] = (s != 0.0L) ? (double)((s - (long double)T.sh[b]) / (long double)T.sh[b]) : 0.0;
    }
}

// ------------------------------------------------------- recursion tables ---

namespace {

void rec_column(int L, int m, int n, double *A, double *B, double *S, double &mant, int &ex)
{
    const int l0 = std::max(std::abs(m), std::abs(n));
    for (int l = 0; l < L; ++l) { A[l] = 0.0; B[l] = 0.0; S[l] = 0.0; }
    mant = 0.0; ex = 0;
    if (l0 >= L) return;
    const long double mm = (long double)m * m, nn = (long double)n * n;
    auto rr = [&](int l) -> long double {  // sqrt((l^2 - m^2)(l^2 - n^2))
        long double l2 = (long double)l * l;
        return sqrtl((l2 - mm) * (l2 - nn));
    };
    std::vector<long double> s(L + 1, 0.0L);
    s[l0] = 1.0L;
    if (l0 + 1 <= L) s[l0 + 1] = 1.0L;
    for (int l = l0; l < L; ++l) {
        long double alpha, beta, gamma;
        if (l == 0) {
            alpha = 1.0L; beta = 0.0L; gamma = 0.0L;        // d^1_00 = cos(theta) d^0_00
        } else {
            long double den = rr(l + 1);
            alpha = (2.0L * l + 1.0L) * (l + 1.0L) / den;
            beta = (2.0L * l + 1.0L) * (long double)m * (long double)n / ((long double)l * den);
            gamma = (l == l0) ? 0.0L : ((l + 1.0L) / (long double)l) * rr(l) / den;
        }
        if (l >= l0 + 1 && l + 1 <= L) s[l + 1] = gamma * s[l - 1];
        long double ratio = s[l] / s[l + 1];
        A[l] = (double)(alpha * ratio);
        B[l] = (double)(beta * ratio);
        S[l] = (double)s[l];
    }
    // start value sign * sqrt(C(2 l0, l0 + k)), k the smaller-magnitude index
    const int k = (std::abs(m) >= std::abs(n)) ? n : m;
    long double lg2 = 0.5L * (lgammal(2.0L * l0 + 1.0L) - lgammal((long double)(l0 + k) + 1.0L)
                              - lgammal((long double)(l0 - k) + 1.0L)) / logl(2.0L);
    int e = (int)floorl(lg2);
    long double mt = powl(2.0L, lg2 - e);
    int sign = 1;
    if (std::abs(m) >= std::abs(n)) {
        if (m >= 0 && ((m - n) % 2 != 0)) sign = -1;          // d^m_{m,n}: (-1)^{m-n}
    } else {
        if (n < 0 && (((m - n) % 2 + 2) % 2 != 0)) sign = -1; // d^{|n|}_{m,-|n|}: (-1)^{m-n}
    }
    mant = (double)(sign * mt);
    ex = e;
}

}  // namespace

void rec_tables(int L, const std::vector<int> &ns, RecTables &R)
{
    R.L = L;
    R.ns = ns;
    const int nn = (int)ns.size();
    R.A.assign((size_t)nn * L * L, 0.0);
    R.B.assign((size_t)nn * L * L, 0.0);
    R.S.assign((size_t)nn * L * L, 0.0);
    R.start_mant.assign((size_t)nn * L, 0.0);
    R.start_exp.assign((size_t)nn * L, 0);
    parallel_for(nn * L, [&](int idx) {
        int ni = idx / L, m = idx % L;
        size_t off = ((size_t)ni * L + m) * L;
        rec_column(L, m, ns[ni], &R.A[off], &R.B[off], &R.S[off], R.start_mant[idx], R.start_exp[idx]);
    });
}

int polar_count(int L) { return L >= 64 ? 4 : 0; }

// Near theta = 0 and pi the characteristic roots of the three-term recursion
// nearly coincide, and FP64 rounding grows like u l^2 there (about 1e-11 at
// l ~ 10^3 on the first and last samples).  The few samples next to the poles are
// therefore taken from this table: the unscaled recursion
//   l sqrt(((l+1)^2-m^2)((l+1)^2-n^2)) d^{l+1}
//       = (2l+1)(l(l+1) cos(theta) - mn) d^l - (l+1) sqrt((l^2-m^2)(l^2-n^2)) d^{l-1}
// in long double (64-bit mantissa), from the closed-form start at l0 = max(|m|,|n|),
// with cos(theta) from the half angle and a power-of-two exponent carried aside.
namespace {
// one (m, n) column: out[p][l], p < 2 np, already zeroed
void polar_column(int L, int m, int n, int np, double *out)
{
    const int P = 2 * np, nsamp = 2 * L - 1;
    {
        const int l0 = std::max(std::abs(m), std::abs(n));
        if (l0 >= L) return;
        std::vector<double> A(L), B(L), S(L);
        double mant;
        int ex;
        rec_column(L, m, n, A.data(), B.data(), S.data(), mant, ex);
        if (mant == 0.0) return;
        const int p1 = std::abs(m + n), p2 = std::abs(m - n);
        const long double mm = (long double)m * m, nq = (long double)n * n, mn = (long double)m * n;
        for (int p = 0; p < P; ++p) {
            const int b = p < np ? p : L - P + p;
            const long double th = kPiL * (2.0L * b + 1.0L) / nsamp;
            long double c = cosl(0.5L * th), s = sinl(0.5L * th), x;
            if (b == L - 1) { c = 0.0L; s = 1.0L; x = -1.0L; }
            else x = (2 * (2 * b + 1) < nsamp) ? 1.0L - 2.0L * s * s : 2.0L * c * c - 1.0L;
            if ((c == 0.0L && p1 > 0) || (s == 0.0L && p2 > 0)) continue;
            double *o = out + (size_t)p * L;
            const long double lg = log2l(fabsl((long double)mant)) + ex + (p1 ? p1 * log2l(c) : 0.0L) +
                                   (p2 ? p2 * log2l(s) : 0.0L);
            int E = (int)floorl(lg);
            long double d = copysignl(exp2l(lg - E), (long double)mant), dm = 0.0L;
            for (int l = l0; l < L; ++l) {
                o[l] = (double)ldexpl(d, E);
                if (l + 1 >= L) break;
                long double dn;
                if (l == 0) {
                    dn = x * d;
                } else {
                    const long double l1 = (long double)(l + 1) * (l + 1), lq = (long double)l * l;
                    const long double den = l * sqrtl((l1 - mm) * (l1 - nq));
                    const long double a1 = (2.0L * l + 1.0L) * ((long double)l * (l + 1) * x - mn);
                    const long double a2 = (l + 1.0L) * sqrtl((lq - mm) * (lq - nq));
                    dn = (a1 * d - a2 * dm) / den;
                }
                dm = d;
                d = dn;
                if (d != 0.0L) {
                    int f;
                    frexpl(d, &f);
                    if (f > 64 || f < -64) {
                        d = ldexpl(d, -f);
                        dm = ldexpl(dm, -f);
                        E += f;
                    }
                }
            }
        }
    }
}
}  // namespace

void polar_table(int L, const std::vector<int> &ns, int np, std::vector<double> &out)
{
    const int nn = (int)ns.size(), P = 2 * np;
    out.assign((size_t)nn * L * P * L, 0.0);
    if (np == 0) return;
    parallel_for(nn * L, [&](int idx) {
        const int ni = idx / L, m = idx % L;
        polar_column(L, m, ns[ni], np, &out[((size_t)ni * L + m) * P * L]);
    });
}

void host_wigner_d(int L, int m, int n, std::vector<double> &out)
{
    out.assign((size_t)L * L, 0.0);
    std::vector<double> A(L), B(L), S(L);
    double mant;
    int ex;
    rec_column(L, m, n, A.data(), B.data(), S.data(), mant, ex);
    const int l0 = std::max(std::abs(m), std::abs(n));
    if (l0 >= L) return;
    ThetaTables T;
    theta_tables(L, T);
    const int p1 = std::abs(m + n), p2 = std::abs(m - n);
    for (int b = 0; b < L; ++b) {
        // start value with log-scaling: value = e * 2^(512 k)
        double c = T.ch[b], s = T.sh[b];
        double v;
        int E;
        if ((c == 0.0 && p1 > 0) || (s == 0.0 && p2 > 0)) {
            v = 0.0; E = 0;
        } else {
            int ec = 0, es = 0;
            double mc = 1.0, ms = 1.0;
            // powers by repeated squaring with exponent extraction
            auto pw = [](double x, int p, double &mt, int &et) {
                mt = 1.0; et = 0;
                if (p == 0) return;
                int bx;
                double bm = frexp(x, &bx);
                while (p) {
                    if (p & 1) { int t; mt = frexp(mt * bm, &t); et += t + bx; }
                    int t2; bm = frexp(bm * bm, &t2); bx = 2 * bx + t2;
                    p >>= 1;
                }
            };
            pw(c, p1, mc, ec);
            pw(s, p2, ms, es);
            mc *= 1.0 + p1 * T.ch_eps[b];
            ms *= 1.0 + p2 * T.sh_eps[b];
            v = mant * mc * ms;
            E = ex + ec + es;
        }
        int k = (int)std::floor((E + 256.0) / 512.0);
        if (k > 0) k = 0;
        double e = ldexp(v, E - 512 * k), ep = 0.0;
        const double cth = T.cth[b], ctl = T.cth_lo[b];
        for (int l = l0; l < L; ++l) {
            out[(size_t)l * L + b] = (k == 0) ? S[l] * e : 0.0;
            const double en = std::fma(std::fma(A[l], ctl, std::fma(A[l], cth, -B[l])), e, -ep);
            ep = e;
            e = en;
            if (k < 0 && std::fabs(e) > 0x1p256) {
                e *= 0x1p-512; ep *= 0x1p-512; ++k;
            }
        }
    }    const int np = polar_count(L);
    if (np > 0) {
        const int P = 2 * np;
        std::vector<double> pt((size_t)P * L, 0.0);
        polar_column(L, m, n, np, pt.data());
        for (int p = 0; p < P; ++p) {
            const int b = p < np ? p : L - P + p;
            for (int l = 0; l < L; ++l) out[(size_t)l * L + b] = pt[(size_t)p * L + l];
        }
    }
}

// -------------------------------------------------------------------- DFT ---

namespace {
int modinv(int a, int m)
{
    if (m == 1) return 0;
    a %= m;
    for (int x = 1; x < m; ++x)
        if ((long long)a * x % m == 1) return x;
    return 0;
}
}  // namespace

void pfa_plan(int n, PfaPlan &P)
{
    P.n = n;
    int best1 = 1, best2 = n;
    for (int d = 1; d <= n; ++d) {
        if (n % d) continue;
        int e = n / d;
        if (std::gcd(d, e) != 1) continue;
        if (d > e) continue;
        if (d + e < best1 + best2) { best1 = d; best2 = e; }
    }
    P.n1 = best1;
    P.n2 = best2;
    // a = a1 e1 + a2 e2 mod n with e1 = 1 (mod n1), 0 (mod n2); e2 = 0 (mod n1), 1 (mod n2)
    P.e1 = (int)((long long)P.n2 * modinv(P.n2 % std::max(P.n1, 1), P.n1) % n);
    P.e2 = (int)((long long)P.n1 * modinv(P.n1 % std::max(P.n2, 1), P.n2) % n);
    if (P.n1 == 1) { P.e1 = 0; P.e2 = 1 % n; }
    P.w1.resize(2 * P.n1);
    P.w2.resize(2 * P.n2);
    for (int k = 0; k < P.n1; ++k) {
        long double a = 2.0L * kPiL * k / P.n1;
        P.w1[2 * k] = (double)cosl(a);
        P.w1[2 * k + 1] = (double)sinl(a);
    }
    for (int k = 0; k < P.n2; ++k) {
        long double a = 2.0L * kPiL * k / P.n2;
        P.w2[2 * k] = (double)cosl(a);
        P.w2[2 * k + 1] = (double)sinl(a);
    }
}

}  // namespace s2w
