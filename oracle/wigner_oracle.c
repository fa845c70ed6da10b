/*
 * FP64 CPU oracle core for the directional wavelet transform on MW sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only tests/, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the GPU library.
 *
 * Wigner d-functions are obtained here WITHOUT the three-term recursion in the
 * degree l that the GPU path uses:
 *   - Delta^l_{qm} = d^l_{qm}(pi/2) is built column by column (fixed second
 *     index m, first index q running down from l) from the angular-momentum
 *     ladder identity  2 m Delta_{q,m} = sqrt((l-q+1)(l+q)) Delta_{q-1,m}
 *     + sqrt((l+q+1)(l-q)) Delta_{q+1,m}, started from the closed form
 *     Delta_{l,m} = (-1)^{l-m} sqrt(C(2l, l+m)) 2^{-l}; long double throughout;
 *   - d^l_{mn}(beta) = i^{n-m} sum_q Delta_{qm} Delta_{qn} e^{i q beta}, the
 *     Fourier expansion used by the separation of variables D = d e^{-i(n g + m a)}
 *     (paper Section 5.2, equation for D^l_mn in terms of d^l_mn).
 * Wigner's explicit sum formula is provided for small l as an independent pin.
 *
 * Conventions: d^1_{10}(beta) = -sin(beta)/sqrt(2) (Wigner's explicit sum).
 * Complex arrays are interleaved (re, im) doubles.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Packed table of Delta^l for l = 0..L-1: block l has (l+1)^2 entries,
 * entry [m*(l+1) + q] = Delta^l_{q,m} for q, m in [0, l]. */
size_t oracle_delta_offset(int l) { return (size_t)l * (l + 1) * (2 * l + 1) / 6; }
size_t oracle_delta_size(int L) { return oracle_delta_offset(L); }

static void delta_block(int l, double *out)
{
    long double *col = (long double *)malloc(sizeof(long double) * (size_t)(l + 2));
    long double *s1 = (long double *)malloc(sizeof(long double) * (size_t)(l + 2));
    long double *s2 = (long double *)malloc(sizeof(long double) * (size_t)(l + 2));
    for (int q = 1; q <= l; ++q) {
        s1[q] = sqrtl((long double)(l - q + 1) * (long double)(l + q));   /* coefficient of Delta_{q-1} */
        s2[q] = sqrtl((long double)(l + q + 1) * (long double)(l - q));   /* coefficient of Delta_{q+1} */
    }
    for (int m = 0; m <= l; ++m) {
        /* start: Delta_{l,m} = (-1)^{l-m} sqrt(C(2l,l+m)) 2^{-l} */
        long double lg = 0.5L * (lgammal(2.0L * l + 1.0L) - lgammal((long double)(l + m) + 1.0L)
                                 - lgammal((long double)(l - m) + 1.0L)) - (long double)l * logl(2.0L);
        long double v = expl(lg);
        if ((l - m) & 1) v = -v;
        col[l] = v;
        col[l + 1] = 0.0L;
        for (int q = l; q >= 1; --q)
            col[q - 1] = (2.0L * m * col[q] - s2[q] * col[q + 1]) / s1[q];
        double *dst = out + (size_t)m * (l + 1);
        for (int q = 0; q <= l; ++q) dst[q] = (double)col[q];
    }
    free(col);
    free(s1);
    free(s2);
}

/* Fill the packed Delta table for all l < L (uses OpenMP over l). */
void oracle_delta_table(int L, double *T)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int l = L - 1; l >= 0; --l) delta_block(l, T + oracle_delta_offset(l));
}

/* Delta^l_{q,m} for any q, m in [-l, l], from the stored quadrant using
 * Delta_{q,-m} = (-1)^{l+q} Delta_{q,m} and Delta_{-q,m} = (-1)^{l+m} Delta_{q,m}. */
static inline double dget(const double *T, int l, int q, int m)
{
    double s = 1.0;
    if (m < 0) { m = -m; if ((l + q) & 1) s = -s; }
    if (q < 0) { q = -q; if ((l + m) & 1) s = -s; }
    return s * T[oracle_delta_offset(l) + (size_t)m * (l + 1) + q];
}

double oracle_delta_get(const double *T, int l, int q, int m) { return dget(T, l, q, m); }

/* Fill column c[q + l] = Delta^l_{q,m}, q in [-l, l], from the stored
 * quadrant (same symmetry rules as dget, applied to a whole column). */
static void column(const double *T, int l, int m, double *c)
{
    const int am = m < 0 ? -m : m;
    const double *src = T + oracle_delta_offset(l) + (size_t)am * (l + 1);
    const double sneg = ((l + am) & 1) ? -1.0 : 1.0;     /* Delta_{-q,|m|} = (-1)^{l+|m|} Delta_{q,|m|} */
    for (int q = 0; q <= l; ++q) {
        c[l + q] = src[q];
        c[l - q] = sneg * src[q];
    }
    if (m < 0)                                           /* Delta_{q,-m} = (-1)^{l+q} Delta_{q,m} */
        for (int q = -l; q <= l; ++q)
            if ((l + q) & 1) c[q + l] = -c[q + l];
}

/* Columns for a list of n values at every l < L: out[(ni * L + l) * Q + (q + l)]. */
static double *ncolumns(const double *T, int L, int nn, const int *ns)
{
    const int Q = 2 * L - 1;
    double *out = (double *)calloc((size_t)nn * L * Q, sizeof(double));
    for (int ni = 0; ni < nn; ++ni)
        for (int l = abs(ns[ni]); l < L; ++l) column(T, l, ns[ni], out + ((size_t)ni * L + l) * Q);
    return out;
}

/*
 * Fourier-space form of sum_l a_lmn d^l_mn(beta):
 *   G[mi][ni][q + L-1] = sum_{l >= max(|m|,|n|)}^{L-1} a[l][mi][ni] Delta^l_{qm} Delta^l_{qn}
 * for q in [-(L-1), L-1].  The caller multiplies by i^{n-m} and evaluates
 * sum_q G(q) e^{i q beta}.  a and G are complex interleaved.
 */
void oracle_wigner_fourier(int L, int nm, const int *ms, int nn, const int *ns,
                           const double *a, double *G, const double *T)
{
    const int Q = 2 * L - 1;
    double *cnall = ncolumns(T, L, nn, ns);
#pragma omp parallel
    {
        double *cm = (double *)malloc(sizeof(double) * Q);
#pragma omp for schedule(dynamic, 1)
        for (int mi = 0; mi < nm; ++mi) {
            const int m = ms[mi];
            double *Gm = G + (size_t)mi * nn * Q * 2;
            memset(Gm, 0, sizeof(double) * (size_t)nn * Q * 2);
            for (int l = abs(m); l < L; ++l) {
                column(T, l, m, cm);
                for (int ni = 0; ni < nn; ++ni) {
                    const int n = ns[ni];
                    if (abs(n) > l) continue;
                    const double ar = a[(((size_t)l * nm + mi) * nn + ni) * 2];
                    const double ai = a[(((size_t)l * nm + mi) * nn + ni) * 2 + 1];
                    if (ar == 0.0 && ai == 0.0) continue;
                    const double *c2 = cnall + ((size_t)ni * L + l) * Q;
                    double *g = Gm + ((size_t)ni * Q + (L - 1 - l)) * 2;
                    for (int k = 0; k <= 2 * l; ++k) {
                        const double p = cm[k] * c2[k];
                        g[2 * k] += ar * p;
                        g[2 * k + 1] += ai * p;
                    }
                }
            }
        }
        free(cm);
    }
    free(cnall);
}

/*
 * Projection onto the Fourier coefficients of d:
 *   out[l][mi][ni] = sum_{q=-l}^{l} Delta^l_{qm} Delta^l_{qn} H[mi][ni][q + L-1]
 * for l >= max(|m|,|n|), zero otherwise.  The caller multiplies by i^{n-m}.
 */
void oracle_wigner_project(int L, int nm, const int *ms, int nn, const int *ns,
                           const double *H, double *out, const double *T)
{
    const int Q = 2 * L - 1;
    memset(out, 0, sizeof(double) * 2 * (size_t)L * nm * nn);
    double *cnall = ncolumns(T, L, nn, ns);
#pragma omp parallel
    {
        double *cm = (double *)malloc(sizeof(double) * Q);
#pragma omp for schedule(dynamic, 1)
        for (int mi = 0; mi < nm; ++mi) {
            const int m = ms[mi];
            for (int l = abs(m); l < L; ++l) {
                column(T, l, m, cm);
                for (int ni = 0; ni < nn; ++ni) {
                    const int n = ns[ni];
                    if (abs(n) > l) continue;
                    const double *cn = cnall + ((size_t)ni * L + l) * Q;
                    const double *h = H + (((size_t)mi * nn + ni) * Q + (L - 1 - l)) * 2;
                    double sr = 0.0, si = 0.0;
                    for (int k = 0; k <= 2 * l; ++k) {
                        const double p = cm[k] * cn[k];
                        sr += p * h[2 * k];
                        si += p * h[2 * k + 1];
                    }
                    out[(((size_t)l * nm + mi) * nn + ni) * 2] = sr;
                    out[(((size_t)l * nm + mi) * nn + ni) * 2 + 1] = si;
                }
            }
        }
        free(cm);
    }
    free(cnall);
}

/* Wigner's explicit sum for d^l_{mn}(beta) (long double; intended for small l). */
double oracle_wigner_d_sum(int l, int m, int n, double beta)
{
    if (abs(m) > l || abs(n) > l) return 0.0;
    const long double c = cosl(0.5L * beta), s = sinl(0.5L * beta);
    const long double lf = 0.5L * (lgammal(l + m + 1.0L) + lgammal(l - m + 1.0L)
                                   + lgammal(l + n + 1.0L) + lgammal(l - n + 1.0L));
    long double acc = 0.0L;
    for (int k = 0; k <= 2 * l; ++k) {
        if (l + n - k < 0 || m - n + k < 0 || l - m - k < 0) continue;
        long double lt = lf - lgammal(l + n - k + 1.0L) - lgammal(k + 1.0L)
                         - lgammal(m - n + k + 1.0L) - lgammal(l - m - k + 1.0L);
        long double t = expl(lt) * powl(c, 2 * l + n - m - 2 * k) * powl(s, m - n + 2 * k);
        if ((m - n + k) & 1) t = -t;
        acc += t;
    }
    return (double)acc;
}
