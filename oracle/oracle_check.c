/* Self-check of the oracle's C core (wigner_oracle.c) for sanitizer builds (test
 * infrastructure only): the Delta tables, the Fourier-space Wigner sums and the explicit
 * sum formula over small sizes, with finiteness and the orthogonality of each Delta block
 * checked.  Built and run on the host with AddressSanitizer and UndefinedBehaviorSanitizer
 * by the test suite (serial: OpenMP off); exits nonzero on a violated check. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

size_t oracle_delta_size(int L);
void oracle_delta_table(int L, double *T);
double oracle_delta_get(const double *T, int l, int q, int m);
void oracle_wigner_fourier(int L, int nm, const int *ms, int nn, const int *ns, const double *a, double *G,
                           const double *T);
void oracle_wigner_project(int L, int nm, const int *ms, int nn, const int *ns, const double *H, double *out,
                           const double *T);
double oracle_wigner_d_sum(int l, int m, int n, double beta);

int main(void)
{
    int bad = 0;
    for (int L = 1; L <= 24; L += 7) {
        double *T = malloc(sizeof(double) * oracle_delta_size(L));
        oracle_delta_table(L, T);
        /* rows of Delta^l are orthonormal: sum_q Delta_qm Delta_qm' = delta_mm' */
        for (int l = 0; l < L; ++l)
            for (int m = -l; m <= l; ++m)
                for (int mp = -l; mp <= l; ++mp) {
                    double s = 0.0;
                    for (int q = -l; q <= l; ++q) s += oracle_delta_get(T, l, q, m) * oracle_delta_get(T, l, q, mp);
                    if (fabs(s - (m == mp ? 1.0 : 0.0)) > 1e-12) bad = 1;
                }
        int ms[3] = {0, L > 1 ? 1 : 0, -(L - 1)}, ns[2] = {0, L > 2 ? -2 : 0};
        const int nm = 3, nn = 2, Q = 2 * L - 1;
        double *a = calloc((size_t)L * nm * nn * 2, sizeof(double));
        double *G = calloc((size_t)nm * nn * Q * 2, sizeof(double));
        double *out = calloc((size_t)L * nm * nn * 2, sizeof(double));
        for (size_t i = 0; i < (size_t)L * nm * nn * 2; ++i) a[i] = sin(0.37 * (double)i);
        oracle_wigner_fourier(L, nm, ms, nn, ns, a, G, T);
        oracle_wigner_project(L, nm, ms, nn, ns, G, out, T);
        for (size_t i = 0; i < (size_t)nm * nn * Q * 2; ++i)
            if (!isfinite(G[i])) bad = 1;
        for (size_t i = 0; i < (size_t)L * nm * nn * 2; ++i)
            if (!isfinite(out[i])) bad = 1;
        free(a);
        free(G);
        free(out);
        free(T);
    }
    for (int l = 0; l <= 8; ++l)
        for (int m = -l; m <= l; ++m)
            if (!isfinite(oracle_wigner_d_sum(l, m, -m, 0.7))) bad = 1;
    if (bad) {
        fprintf(stderr, "oracle_check: a check failed\n");
        return 1;
    }
    printf("oracle_check ok\n");
    return 0;
}
