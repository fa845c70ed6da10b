// Self-check of the host plan arithmetic (s2w_host.cpp) for sanitizer builds: every
// routine runs over a range of sizes, including the degenerate ones, and basic invariants
// are checked (finite values, symmetric quadrature matrices, bijective prime-factor index
// maps, positive Laguerre weights, filters that tile the harmonic line).  Built and run on
// the host with AddressSanitizer and UndefinedBehaviorSanitizer by the test suite; exits
// nonzero on the first violated invariant.
#include <cmath>
#include <cstdio>
#include <set>
#include <string>
#include <vector>

#include "s2w_host.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what, int a = 0, int b = 0)
{
    if (!ok) {
        std::fprintf(stderr, "host_check: %s (%d, %d)\n", what, a, b);
        ++failures;
    }
}

bool finite(const std::vector<double> &v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

}  // namespace

int main()
{
    using namespace s2w;
    // band limits and filters
    const double lams[] = {2.0, 3.0, 1.5, 2.5};
    for (int L : {2, 3, 8, 33, 64, 130}) {
        for (int N : {1, 2, 3, 5, 8}) {
            if (N > L) continue;
            for (double lam : lams)
                for (int J0 : {0, 1, 2}) {
                    Scales S;
                    std::string err;
                    if (!make_scales(L, N, lam, J0, S, err)) continue;
                    Filters F;
                    make_filters(S, F);
                    expect((int)F.phi.size() == L, "phi size", L, N);
                    // admissibility: |Phi|^2 4 pi / (2l+1) + sum_j 8 pi^2/(2l+1) sum_n |Psi|^2 = 1
                    for (int l = 0; l < L; ++l) {
                        double tot = F.phi[l] * F.phi[l] * 4.0 * M_PI / (2.0 * l + 1.0);
                        for (size_t k = 0; k < S.s.size(); ++k) {
                            const int nn = (int)S.s[k].n.size();
                            if (l >= S.s[k].L) continue;
                            for (int i = 0; i < nn; ++i) {
                                const double v = F.psi_mag[k][(size_t)l * nn + i];
                                tot += 8.0 * M_PI * M_PI / (2.0 * l + 1.0) * v * v;
                            }
                        }
                        expect(std::fabs(tot - 1.0) < 1e-12, "admissibility", L, l);
                    }
                }
        }
    }
    // quadrature matrices and grid tables
    for (int L : {1, 2, 3, 8, 33, 64, 129}) {
        for (int sg : {1, -1}) {
            std::vector<double> T;
            theta_matrix(L, sg, T);
            expect((int)T.size() == L * L && finite(T), "theta matrix", L, sg);
            for (int i = 0; i < L; ++i)
                for (int j = 0; j < i; ++j)
                    expect(std::fabs(T[(size_t)i * L + j] - T[(size_t)j * L + i]) < 1e-12, "theta symmetry", i, j);
        }
        ThetaTables tt;
        theta_tables(L, tt);
        expect(finite(tt.cth) && finite(tt.ch) && finite(tt.sh), "theta tables", L);
    }
    // recursion and polar tables, device-form d
    for (int L : {2, 5, 64, 100, 256}) {
        std::vector<int> ns = {0, 1, -1, 3, -3};
        RecTables R;
        rec_tables(L, ns, R);
        expect(finite(R.A) && finite(R.B) && finite(R.S), "recursion tables", L);
        const int np = polar_count(L);
        if (np > 0) {
            std::vector<double> pt;
            polar_table(L, ns, np, pt);
            expect(finite(pt), "polar table", L, np);
        }
        std::vector<double> d;
        host_wigner_d(L, L / 2, L > 3 ? 3 : 0, d);
        expect((int)d.size() == L * L && finite(d), "host d", L);
    }
    // prime-factor plans: the input and output index maps are bijections
    for (int n : {1, 3, 5, 7, 15, 63, 127, 255, 511, 1023, 1999, 2047}) {
        PfaPlan P;
        pfa_plan(n, P);
        expect(P.n1 * P.n2 == n, "pfa factors", n);
        std::set<long> in, out;
        for (int m1 = 0; m1 < P.n1; ++m1)
            for (int m2 = 0; m2 < P.n2; ++m2) {
                in.insert(((long)m1 * P.n2 + (long)m2 * P.n1) % n);
                out.insert(((long)m1 * P.e1 + (long)m2 * P.e2) % n);
            }
        expect((int)in.size() == n && (int)out.size() == n, "pfa bijection", n);
        expect(finite(P.w1) && finite(P.w2), "pfa twiddles", n);
    }
    // Laguerre rules
    for (int P : {1, 2, 5, 64, 256})
        for (double tau : {1.0, 0.7}) {
            LaguerreRule R;
            laguerre_rule(P, tau, R);
            bool pos = true;
            for (double w : R.W) pos = pos && w > 0.0 && std::isfinite(w);
            expect(pos && (int)R.r.size() == P, "laguerre weights", P);
            std::vector<double> K;
            laguerre_basis(R, P, K);
            expect(finite(K), "laguerre basis", P);
        }
    if (failures) return 1;
    std::printf("host_check ok\n");
    return 0;
}
