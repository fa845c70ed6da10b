// HIP kernels for the directional wavelet transform on MW sampling (gfx950).
//
// Per-scale Wigner transform, split into:
//   k_lsum   sum over degree l of a_lmn d^l_mn(theta) for every (m >= 0, n, theta):
//            lanes own theta samples; d generated on the fly by the scaled
//            three-term recursion in l, started from the closed form at
//            l0 = max(|m|,|n|) with per-lane power-of-two rescaling (FP64).
//            cos(theta) enters as a double-double pair (hi + lo, one extra FMA
//            per step): near the poles a single rounding of cos(theta) shifts
//            d^l by about l^2 u / 2, far above the FP64 target at l ~ 10^3
//   k_tsum   sum over theta of d^l_mn(theta) h(theta) for every l (the
//            transposed contraction), same recursion, cross-lane reduction
//            through LDS
//   k_gemm   exact MW theta quadrature h = T_sigma F (MFMA, FP64 or FP32)
//   k_dft_*  odd-length DFTs (2L-1, 2N-1 points) by the prime-factor algorithm
//   k_gamma_* azimuthal (gamma) DFT over the few nonzero n, fused with the
//            layout change between the l-stage ((m, n) rows over theta) and
//            the alpha-stage (rows over m)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "s2w_dev.h"
#include "s2w_kern.h"

namespace s2w {

// theta samples next to the poles whose d come from the polar table
__device__ inline bool is_polar(int th, int L, int npol) { return th < npol || th >= L - npol; }
__device__ inline int polar_theta(int p, int L, int npol) { return p < npol ? p : L - 2 * npol + p; }

// ------------------------------------------------------------- k_lsum ------
//
// C_s[b][ni][m][theta] = sum_{l=l0}^{L-1} u_s(l) e^l(theta),
// u_s(l) = S_l w_s[ni][l] flm[b][m][l]   (so that u e^l = w flm d^l).
// PRE (precompute mode): d^l(theta) is read from the grid's table instead of being
// recursed, and u_s(l) = w_s[ni][l] flm[b][m][l].

template <int T, int NS, bool PRE>
__global__ __launch_bounds__(64) void k_lsum(const LsumArgs a)
{
    const int m = blockIdx.x, ni = blockIdx.y;
    const int nch = (a.L + 64 * T - 1) / (64 * T);
    const int b = blockIdx.z / nch, chk = blockIdx.z % nch;
    const int lane = threadIdx.x;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int am = m, an = n < 0 ? -n : n;
    const int l0 = am > an ? am : an;
    const int lmax = a.L;

    __shared__ double2 sAB[64];
    __shared__ double2 sU[NS][64];

    double c[T], cl[T], e[T], ep[T], acc[NS][2][T];
    int k[T];
    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    const double mant = a.smant[(size_t)ng * a.Lrec + m];
    const int ex = a.sexp[(size_t)ng * a.Lrec + m];
    const int p1 = (m + n) < 0 ? -(m + n) : (m + n);
    const int p2 = (m - n) < 0 ? -(m - n) : (m - n);
    bool asleep_any = false;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int th = chk * 64 * T + t * 64 + lane;
        e[t] = 0.0;
        ep[t] = 0.0;
        k[t] = 0;
        c[t] = 0.0;
        cl[t] = 0.0;
        if (!PRE && th < a.L && l0 < lmax) {
            c[t] = a.cth[th];
            cl[t] = a.ctl[th];
            start_value(mant, ex, p1, p2, a.ch[th], a.sh[th], a.ceps[th], a.seps[th], e[t], k[t]);
        }
        asleep_any |= (k[t] < 0);
#pragma unroll
        for (int s = 0; s < NS; ++s) { acc[s][0][t] = 0.0; acc[s][1][t] = 0.0; }
    }
    bool anyAsleep = __any(asleep_any);
    // precompute mode: this (n, m) row block of the table, and this lane's theta samples
    const double *drow = PRE ? a.dtab + a.doff[(size_t)ng * a.L + m] : nullptr;

    for (int lb = l0; lb < lmax; lb += 64) {
        {
            const int l = lb + lane;
            double A = 0.0, Bv = 0.0;
            double ur[NS], ui[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) { ur[s] = 0.0; ui[s] = 0.0; }
            if (l < lmax) {
                A = a.A[tabm + l];
                Bv = a.B[tabm + l];
                const double S = PRE ? 1.0 : a.S[tabm + l];
                const double *fl = a.flm + (((size_t)b * a.flm_m + m) * a.flm_l + l + ni * a.flm_nstride) * 2;
                const double fr = fl[0], fi = fl[1];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const double w = S * a.w[s][(size_t)ni * a.wstride + l];
                    ur[s] = w * fr;
                    ui[s] = w * fi;
                }
            }
            __syncthreads();
            sAB[lane] = make_double2(A, Bv);
#pragma unroll
            for (int s = 0; s < NS; ++s) sU[s][lane] = make_double2(ur[s], ui[s]);
            __syncthreads();
        }
        const int cnt = (lmax - lb) < 64 ? (lmax - lb) : 64;
        for (int g = 0; g < cnt; g += 8) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double2 ab = sAB[g + i];
                double2 u[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) u[s] = sU[s][g + i];
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    if (PRE) {
                        // table row of degree lb + g + i (past the last degree u is zero)
                        const int th = chk * 64 * T + t * 64 + lane;
                        const int li = lb + g + i - l0;
                        e[t] = (th < a.L && lb + g + i < lmax) ? drow[(size_t)li * a.L + th] : 0.0;
                    }
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        acc[s][0][t] = fma(u[s].x, e[t], acc[s][0][t]);
                        acc[s][1][t] = fma(u[s].y, e[t], acc[s][1][t]);
                    }
                    if (!PRE) {
                        const double en = fma(fma(ab.x, cl[t], fma(ab.x, c[t], -ab.y)), e[t], -ep[t]);
                        ep[t] = e[t];
                        e[t] = en;
                    }
                }
            }
            if (!PRE && anyAsleep) {
                bool any = false;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    if (k[t] < 0) {
                        if (fabs(e[t]) > 0x1p256) {
                            e[t] *= 0x1p-512;
                            ep[t] *= 0x1p-512;
                            k[t] += 1;
                            if (k[t] == 0) {
#pragma unroll
                                for (int s = 0; s < NS; ++s) { acc[s][0][t] = 0.0; acc[s][1][t] = 0.0; }
                            }
                        }
                    }
                    any |= (k[t] < 0);
                }
                anyAsleep = __any(any);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int th = chk * 64 * T + t * 64 + lane;
        if (th >= a.L) continue;
        const bool live = (k[t] == 0) && (l0 < lmax);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double *o = a.out[s] + ((((size_t)b * a.nn + ni) * a.mcount + m) * a.L + th) * 2;
            o[0] = live ? acc[s][0][t] : 0.0;
            o[1] = live ? acc[s][1][t] : 0.0;
        }
    }
}

// ------------------------------------------------------------- k_tsum ------
//
// P_s[b][m][ni][l] = S_l w_s[ni][l] sum_theta e^l(theta) h_s(theta)   (l >= l0, else 0)
// h_s rows (re, im) come from the sigma-grouped layout [sig][b][m'][ni][c][theta].

template <int T, int NS, bool PRE>
__global__ __launch_bounds__(256) void k_tsum(const TsumArgs a)
{
    constexpr int LB = 16 / NS;          // l-steps per reduction block: 2*NS*LB = 32 entries
    constexpr int K = 2 * NS * LB;
    constexpr int MAXW = 4;
    const int m = blockIdx.x, ni = blockIdx.y;
    const int b = blockIdx.z;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n;
    const int l0 = m > an ? m : an;
    const int lmax = a.L;

    // wave w owns theta = 64 (w T + t) + lane, t < T; each wave reduces its lanes
    // through red[w], then wave 0 adds the waves' partials in a fixed order
    __shared__ double red[MAXW][64][K + 1];
    __shared__ double part[MAXW][K];
    __shared__ double2 sAB[LB];

    // input rows
    const int sig = (m + a.npar) & 1;
    const int mp = m >> 1;
    const size_t rbase = (sig == 0 ? 0 : (size_t)a.B * a.M0 * a.nn * 2)
                         + ((((size_t)b * (sig == 0 ? a.M0 : a.M1) + mp) * a.nn + ni) * 2);

    double c[T], cl[T], e[T], ep[T], hr[NS][T], hi[NS][T];
    int k[T];
    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    const double mant = a.smant[(size_t)ng * a.Lrec + m];
    const int ex = a.sexp[(size_t)ng * a.Lrec + m];
    const int p1 = (m + n) < 0 ? -(m + n) : (m + n);
    const int p2 = (m - n) < 0 ? -(m - n) : (m - n);
    bool asleep_any = false;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int th = (w * T + t) * 64 + lane;
        e[t] = 0.0;
        ep[t] = 0.0;
        k[t] = 0;
        c[t] = 0.0;
        cl[t] = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) { hr[s][t] = 0.0; hi[s][t] = 0.0; }
        if (th < a.L && l0 < lmax) {
            if (!PRE) {
                c[t] = a.cth[th];
                cl[t] = a.ctl[th];
                start_value(mant, ex, p1, p2, a.ch[th], a.sh[th], a.ceps[th], a.seps[th], e[t], k[t]);
            }
            if (k[t] == 0 && !is_polar(th, a.L, a.npol)) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    hr[s][t] = a.h[s][(rbase + 0) * a.L + th];
                    hi[s][t] = a.h[s][(rbase + 1) * a.L + th];
                }
            }
        }
        asleep_any |= (k[t] < 0);
    }
    bool anyAsleep = __any(asleep_any);
    const double *drow = PRE ? a.dtab + a.doff[(size_t)ng * a.L + m] : nullptr;

    for (int lb = l0; lb < lmax; lb += LB) {
        __syncthreads();
        if (threadIdx.x < LB) {
            const int l = lb + threadIdx.x;
            double A = 0.0, Bv = 0.0;
            if (l < lmax) { A = a.A[tabm + l]; Bv = a.B_[tabm + l]; }
            sAB[threadIdx.x] = make_double2(A, Bv);
        }
        __syncthreads();
        for (int i = 0; i < LB; ++i) {
            const double2 ab = sAB[i];
            double pr[NS], pi[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) { pr[s] = 0.0; pi[s] = 0.0; }
#pragma unroll
            for (int t = 0; t < T; ++t) {
                if (PRE) {
                    const int th = (w * T + t) * 64 + lane;
                    e[t] = (th < a.L && lb + i < lmax) ? drow[(size_t)(lb + i - l0) * a.L + th] : 0.0;
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    pr[s] = fma(e[t], hr[s][t], pr[s]);
                    pi[s] = fma(e[t], hi[s][t], pi[s]);
                }
                if (!PRE) {
                    const double en = fma(fma(ab.x, cl[t], fma(ab.x, c[t], -ab.y)), e[t], -ep[t]);
                    ep[t] = e[t];
                    e[t] = en;
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                red[w][lane][(s * LB + i) * 2 + 0] = pr[s];
                red[w][lane][(s * LB + i) * 2 + 1] = pi[s];
            }
            if (!PRE && anyAsleep && ((i & 7) == 7)) {
                bool any = false;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    if (k[t] < 0) {
                        if (fabs(e[t]) > 0x1p256) {
                            e[t] *= 0x1p-512;
                            ep[t] *= 0x1p-512;
                            k[t] += 1;
                            const int th = (w * T + t) * 64 + lane;
                            if (k[t] == 0 && !is_polar(th, a.L, a.npol)) {
#pragma unroll
                                for (int s = 0; s < NS; ++s) {
                                    hr[s][t] = a.h[s][(rbase + 0) * a.L + th];
                                    hi[s][t] = a.h[s][(rbase + 1) * a.L + th];
                                }
                            }
                        }
                    }
                    any |= (k[t] < 0);
                }
                anyAsleep = __any(any);
            }
        }
        __syncthreads();
        // lane j < K of each wave sums entry j over the wave's 64 lanes
        if (lane < K) {
            double v = 0.0;
#pragma unroll 8
            for (int src = 0; src < 64; ++src) v += red[w][src][lane];
            part[w][lane] = v;
        }
        __syncthreads();
        if (w == 0 && lane < K) {
            const int j = lane;
            double v = 0.0;
            for (int ww = 0; ww < nw; ++ww) v += part[ww][j];
            const int s = j / (2 * LB);
            const int i = (j / 2) % LB;
            const int cc = j & 1;
            const int l = lb + i;
            if (l < lmax) {
                const double S = PRE ? 1.0 : a.S[tabm + l];
                const double wgt = a.w[s][(size_t)ni * a.wstride + l];
                a.out[s][((((size_t)b * a.mcount + m) * a.nn + ni) * a.L + l) * 2 + cc] = v * S * wgt;
            }
        }
    }
    // zero the l < l0 part of the output rows
    for (int l = threadIdx.x; l < l0 && l < lmax; l += blockDim.x) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double *o = a.out[s] + ((((size_t)b * a.mcount + m) * a.nn + ni) * a.L + l) * 2;
            o[0] = 0.0;
            o[1] = 0.0;
        }
    }
}

// ------------------------------------------------------------- d tables ----
// Precompute mode: d^l_mn(theta_b) = S_l e^l(theta_b) of one grid for every (n, m) and
// l0 <= l < L, rows over theta: tab[doff[nglob L + m] + (l - l0) L + theta], by the same
// scaled, log-rescaled recursion the contraction kernels run (a sample whose scaled value
// has not reached the representable range holds 0, as those kernels treat it).  One lane
// per theta sample, one block per (m, n, 64 samples).
__global__ __launch_bounds__(64) void k_dtable(const LsumArgs a, double *tab, const int64_t *doff)
{
    const int m = blockIdx.x, ni = blockIdx.y;
    const int th = blockIdx.z * 64 + threadIdx.x;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n, l0 = m > an ? m : an;
    if (l0 >= a.L || th >= a.L) return;
    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    const int p1 = (m + n) < 0 ? -(m + n) : (m + n);
    const int p2 = (m - n) < 0 ? -(m - n) : (m - n);
    const double c = a.cth[th], cl = a.ctl[th];
    double e = 0.0, ep = 0.0;
    int k = 0;
    start_value(a.smant[(size_t)ng * a.Lrec + m], a.sexp[(size_t)ng * a.Lrec + m], p1, p2, a.ch[th], a.sh[th],
                a.ceps[th], a.seps[th], e, k);
    double *row = tab + doff[(size_t)ng * a.L + m] + th;
    for (int l = l0; l < a.L; ++l) {
        row[(size_t)(l - l0) * a.L] = k == 0 ? a.S[tabm + l] * e : 0.0;
        const double A = a.A[tabm + l], Bv = a.B[tabm + l];
        const double en = fma(fma(A, cl, fma(A, c, -Bv)), e, -ep);
        ep = e;
        e = en;
        if (k < 0 && fabs(e) > 0x1p256) {
            e *= 0x1p-512;
            ep *= 0x1p-512;
            k += 1;
        }
    }
}

// --------------------------------------------------------- polar samples ----
//
// The 2 npol samples next to the poles take d from the long-double table (the
// FP64 recursion loses about u l^2 there).  k_lsum_polar overwrites k_lsum's
// output at those samples; k_tsum skips them and k_tsum_polar adds their terms.

template <int NS>
__global__ __launch_bounds__(64) void k_lsum_polar(const LsumArgs a)
{
    constexpr int PM = 8;                // 2 npol <= PM
    const int m = blockIdx.x, ni = blockIdx.y, b = blockIdx.z, lane = threadIdx.x;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n, l0 = m > an ? m : an;
    const int P = 2 * a.npol;
    double acc[PM][NS][2];
#pragma unroll
    for (int p = 0; p < PM; ++p)
#pragma unroll
        for (int s = 0; s < NS; ++s) { acc[p][s][0] = 0.0; acc[p][s][1] = 0.0; }
    const double *tab = a.pol + ((size_t)ng * a.L + m) * P * a.L;
    for (int l = l0 + lane; l < a.L; l += 64) {
        const double *fl = a.flm + (((size_t)b * a.flm_m + m) * a.flm_l + l + ni * a.flm_nstride) * 2;
        const double fr = fl[0], fi = fl[1];
        double ur[NS], ui[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double w = a.w[s][(size_t)ni * a.wstride + l];
            ur[s] = w * fr;
            ui[s] = w * fi;
        }
#pragma unroll
        for (int p = 0; p < PM; ++p) {
            if (p >= P) break;
            const double d = tab[(size_t)p * a.L + l];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                acc[p][s][0] = fma(ur[s], d, acc[p][s][0]);
                acc[p][s][1] = fma(ui[s], d, acc[p][s][1]);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < PM; ++p)
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) acc[p][s][c] += __shfl_xor(acc[p][s][c], off, 64);
    if (lane == 0) {
#pragma unroll
        for (int p = 0; p < PM; ++p) {
            if (p >= P) break;
            const int th = polar_theta(p, a.L, a.npol);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                double *o = a.out[s] + ((((size_t)b * a.nn + ni) * a.mcount + m) * a.L + th) * 2;
                o[0] = acc[p][s][0];
                o[1] = acc[p][s][1];
            }
        }
    }
}

template <int NS>
__global__ __launch_bounds__(64) void k_tsum_polar(const TsumArgs a)
{
    constexpr int PM = 8;
    const int m = blockIdx.x, ni = blockIdx.y, b = blockIdx.z, lane = threadIdx.x;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n, l0 = m > an ? m : an;
    const int P = 2 * a.npol;
    const int sig = (m + a.npar) & 1, mp = m >> 1;
    const size_t rbase = (sig == 0 ? 0 : (size_t)a.B * a.M0 * a.nn * 2)
                         + ((((size_t)b * (sig == 0 ? a.M0 : a.M1) + mp) * a.nn + ni) * 2);
    double hr[PM][NS], hi[PM][NS];
#pragma unroll
    for (int p = 0; p < PM; ++p) {
        const int th = polar_theta(p < P ? p : 0, a.L, a.npol);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            hr[p][s] = p < P ? a.h[s][(rbase + 0) * a.L + th] : 0.0;
            hi[p][s] = p < P ? a.h[s][(rbase + 1) * a.L + th] : 0.0;
        }
    }
    const double *tab = a.pol + ((size_t)ng * a.L + m) * P * a.L;
    for (int l = l0 + lane; l < a.L; l += 64) {
        double vr[NS], vi[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) { vr[s] = 0.0; vi[s] = 0.0; }
#pragma unroll
        for (int p = 0; p < PM; ++p) {
            if (p >= P) break;
            const double d = tab[(size_t)p * a.L + l];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                vr[s] = fma(d, hr[p][s], vr[s]);
                vi[s] = fma(d, hi[p][s], vi[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double w = a.w[s][(size_t)ni * a.wstride + l];
            double *o = a.out[s] + ((((size_t)b * a.mcount + m) * a.nn + ni) * a.L + l) * 2;
            o[0] += w * vr[s];
            o[1] += w * vi[s];
        }
    }
}

// ------------------------------------------------------------ k_tsum_mm64 ----
// Batched form of k_tsum on FP64 matrix cores (16x16x4), for launches of many maps:
// the recursion runs once per (m, n, theta) for 32 columns (scale, map, re/im) instead
// of once per map.  grid (m, ni, groups of 32 columns); NW = ceil(L/64) waves per block,
// wave w owns theta = 64 w + lane and keeps its 64 x 32 (theta x column) slice of h in
// registers as MFMA B operands; per chunk of 16 degrees it writes d (FP64) to its LDS
// slice, forms the 16 x 32 partial product and stores it over that slice, and the
// waves' partials are summed in a fixed order.  Polar samples are left to k_tsum_polar.

typedef double d4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int TS64_RS = 64 * 16;       // doubles per wave slice: d [64][16] or partial [32 col][17]

template <int NS>
__global__ __launch_bounds__(1024) void k_tsum_mm64(const TsumArgs a, const double *__restrict__ rA,
                                                    const double *__restrict__ rB)
{
    // rA, rB alias a.A, a.B_: as restrict arguments their wave-uniform reads become scalar loads
    extern __shared__ double smd[];    // [NW][TS64_RS]
    const int m = blockIdx.x, ni = blockIdx.y, g = blockIdx.z;
    const int L = a.L;
    const int NW = blockDim.x >> 6;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n;
    const int l0 = m > an ? m : an;
    const int B = a.B, ncols = 2 * B * NS;
    const int th = w * 64 + lane;
    const bool valid = th < L && !is_polar(th, L, a.npol);

    // h slice: hb[ks][j] = h[theta = 64 w + 4 ks + lane / 16][col = 32 g + 16 j + lane % 16]
    const int sig = (m + a.npar) & 1;
    const int mp = m >> 1;
    const size_t sigoff = (sig == 0 ? 0 : (size_t)B * a.M0 * a.nn * 2);
    const int Msig = (sig == 0 ? a.M0 : a.M1);
    double hb[16][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int cg = g * 32 + 16 * j + (lane & 15);
        int s = 0, b = 0, cc = 0;
        const bool cok = cg < ncols;
        if (cok) {
            s = cg / (2 * B);
            const int rem = cg - s * 2 * B;
            b = rem >> 1;
            cc = rem & 1;
        }
        const double *hs = a.h[s < NS ? s : 0];
        const size_t row = sigoff + (((size_t)b * Msig + mp) * a.nn + ni) * 2 + cc;
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int t2 = w * 64 + 4 * ks + (lane >> 4);
            hb[ks][j] = (cok && t2 < L) ? hs[row * L + t2] : 0.0;
        }
    }

    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    double c = 0.0, cl = 0.0, e = 0.0, ep = 0.0;
    int k = 0;
    if (th < L && l0 < L) {
        c = a.cth[th];
        cl = a.ctl[th];
        const int p1 = (m + n) < 0 ? -(m + n) : (m + n);
        const int p2 = (m - n) < 0 ? -(m - n) : (m - n);
        start_value(a.smant[(size_t)ng * a.Lrec + m], a.sexp[(size_t)ng * a.Lrec + m], p1, p2, a.ch[th],
                    a.sh[th], a.ceps[th], a.seps[th], e, k);
    }

    double *Dw = smd + (size_t)w * TS64_RS;
    for (int lb = l0; lb < L; lb += 16) {
        // d chunk, swizzled [theta][l ^ (theta & 15)]
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
            const int l = lb + i;
            double A = 0.0, Bv = 0.0;
            if (l < L) { A = rA[tabm + l]; Bv = rB[tabm + l]; }
            Dw[lane * 16 + (i ^ (lane & 15))] = (valid && k == 0) ? e : 0.0;
            const double en = fma(fma(A, cl, fma(A, c, -Bv)), e, -ep);
            ep = e;
            e = en;
            if ((i & 7) == 7 && k < 0 && fabs(e) > 0x1p256) {
                e *= 0x1p-512;
                ep *= 0x1p-512;
                k += 1;
            }
        }
        wave_lds_fence();
        d4v pacc[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) pacc[j] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int tl = 4 * ks + (lane >> 4);
            const double av = Dw[tl * 16 + ((lane & 15) ^ (tl & 15))];   // A[l = lane%16][theta = tl]
#pragma unroll
            for (int j = 0; j < 2; ++j) pacc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, hb[ks][j], pacc[j], 0, 0, 0);
        }
        wave_lds_fence();
        // partial 16 (l) x 32 (col), stored [col][l] with stride 17: register r of lane ->
        // l = lane / 16 + 4 r (FP64 result layout), col = 16 j + lane % 16
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) Dw[(16 * j + (lane & 15)) * 17 + (lane >> 4) + 4 * r] = pacc[j][r];
        __syncthreads();
        for (int t = threadIdx.x; t < 512; t += blockDim.x) {
            const int col = 2 * (t >> 5) + (t & 1), li = (t >> 1) & 15;
            const int l = lb + li, cg = g * 32 + col;
            double v = 0.0;
            for (int ww = 0; ww < NW; ++ww) v += smd[(size_t)ww * TS64_RS + col * 17 + li];
            if (l < L && cg < ncols) {
                const int s = cg / (2 * B);
                const int rem = cg - s * 2 * B;
                const int b = rem >> 1, cc = rem & 1;
                const double sc = a.S[tabm + l] * a.w[s][(size_t)ni * a.wstride + l];
                a.out[s][((((size_t)b * a.mcount + m) * a.nn + ni) * L + l) * 2 + cc] = v * sc;
            }
        }
        __syncthreads();   // the next chunk's d overwrites the slices
    }
    // zero l < l0: each of the block's 16 column pairs (re, im of one scale and map) owns a
    // contiguous run of nz (re, im) values, written by blockDim / 16 threads along l
    const int nz = (l0 < L ? l0 : L);
    const int tpp = blockDim.x >> 4;
    const int pz = threadIdx.x / tpp, qz = threadIdx.x - pz * tpp;
    const int cz = g * 32 + 2 * pz;
    if (cz < ncols) {
        const int s = cz / (2 * B), b = (cz - s * 2 * B) >> 1;
        double *row = a.out[s] + (((size_t)b * a.mcount + m) * a.nn + ni) * L * 2;
        for (int l = qz; l < nz; l += tpp) {
            row[2 * l] = 0.0;
            row[2 * l + 1] = 0.0;
        }
    }
}

// ------------------------------------------------------------ k_lsum_mm64 ----
// Batched form of k_lsum on FP64 matrix cores, for launches of many maps: the
// recursion runs once per (m, n, theta) for 32 columns (scale, map, re/im).  W waves
// per block, wave w owns the 64-theta tile (tb W + w) of one (m, n, 32 columns) unit;
// per chunk of 16 degrees the waves share one staged coefficient tile (16-byte
// (re, im) loads, 16 consecutive degrees per column pair), each writes its d chunk
// (S_l d, FP64) to LDS and accumulates its 64 x 32 output on the matrix cores.
// Polar samples are overwritten afterwards by k_lsum_polar.

constexpr int LS64_DS = 64 + 1;        // row stride (doubles) of the d and staging tiles

template <int NS, int W>
__global__ __launch_bounds__(64 * W) void k_lsum_mm64(const LsumArgs a, const double *__restrict__ rA,
                                                      const double *__restrict__ rB, const double *__restrict__ rS,
                                                      int B)
{
    constexpr int R = 4 / W;           // staging slots per thread (16 column pairs x 16 degrees)
    const int L = a.L;
    const int ntt = (L + 63) >> 6;
    const int ntb = (ntt + W - 1) / W;
    const int ncols = 2 * B * NS;
    const int ngrp = (ncols + 31) >> 5;
    const int nunit = a.mcount * a.nn * ngrp;
    // XCD-aware order: the ntb theta blocks of one unit get consecutive slots on one XCD
    const int bid = blockIdx.x, xcd = bid & 7, kx = bid >> 3;
    const int tb = kx % ntb, unit = (kx / ntb) * 8 + xcd;
    if (unit >= nunit) return;
    const int m = unit % a.mcount, ni = (unit / a.mcount) % a.nn, g = unit / (a.mcount * a.nn);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n;
    const int l0 = m > an ? m : an;
    const int th = (tb * W + w) * 64 + lane;
    const bool valid = th < L;

    __shared__ double Ds[W][16 * LS64_DS];   // d chunk [l][theta]; output staging [col][theta] at the end
    __shared__ double Us[16][32 + 2];        // coefficient chunk [l][column]

    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    double c = 0.0, cl = 0.0, e = 0.0, ep = 0.0;
    int k = 0;
    if (valid && l0 < L) {
        c = a.cth[th];
        cl = a.ctl[th];
        const int p1 = (m + n) < 0 ? -(m + n) : (m + n);
        const int p2 = (m - n) < 0 ? -(m - n) : (m - n);
        start_value(a.smant[(size_t)ng * a.Lrec + m], a.sexp[(size_t)ng * a.Lrec + m], p1, p2, a.ch[th],
                    a.sh[th], a.ceps[th], a.seps[th], e, k);
    }

    // staging slot q = tid + 64 W r: column pair p = q / 16 (re, im of one map and scale), degree lb + q % 16
    int iq[R], pc[R];
    bool cok[R];
    const double *wv[R];
    const double2 *fl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = tid + 64 * W * r;
        pc[r] = q >> 4;
        iq[r] = q & 15;
        const int cg = g * 32 + 2 * pc[r];
        cok[r] = cg < ncols;
        int cs = 0, cb = 0;
        if (cok[r]) {
            cs = cg / (2 * B);
            cb = (cg - cs * 2 * B) >> 1;
        }
        wv[r] = a.w[cs < NS ? cs : 0] + (size_t)ni * a.wstride;
        fl[r] = reinterpret_cast<const double2 *>(a.flm) + ((size_t)cb * a.flm_m + m) * a.flm_l + ni * a.flm_nstride;
    }

    typedef double d4 __attribute__((ext_vector_type(4)));
    d4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    for (int lb = l0; lb < L; lb += 16) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int l = lb + iq[r];
            double2 f = make_double2(0.0, 0.0);
            double wt = 0.0;
            if (cok[r] && l < L) {
                f = fl[r][l];
                wt = wv[r][l];
            }
            Us[iq[r]][2 * pc[r]] = wt * f.x;
            Us[iq[r]][2 * pc[r] + 1] = wt * f.y;
        }
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
            const int l = lb + i;
            double A = 0.0, Bv = 0.0, S = 0.0;
            if (l < L) { A = rA[tabm + l]; Bv = rB[tabm + l]; S = rS[tabm + l]; }
            Ds[w][i * LS64_DS + lane] = (valid && k == 0) ? S * e : 0.0;
            const double en = fma(fma(A, cl, fma(A, c, -Bv)), e, -ep);
            ep = e;
            e = en;
            if ((i & 7) == 7 && k < 0 && fabs(e) > 0x1p256) {
                e *= 0x1p-512;
                ep *= 0x1p-512;
                k += 1;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            double af[4], bf[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = Ds[w][(kk + (lane >> 4)) * LS64_DS + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = Us[kk + (lane >> 4)][j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // output: one 16-column tile at a time through this wave's Ds slice ([col][theta]),
    // register r of tile (i, j) holding theta = 16 i + lane / 16 + 4 r, column 16 j + lane % 16
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) Ds[w][(lane & 15) * LS64_DS + i * 16 + (lane >> 4) + 4 * r] = acc[i][j][r];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int cgp = g * 32 + 16 * j + 2 * q;
            if (cgp < ncols && valid) {
                const int s = cgp / (2 * B);
                const int b = (cgp - s * 2 * B) >> 1;
                double2 *dst = reinterpret_cast<double2 *>(a.out[s]);
                dst[(((size_t)b * a.nn + ni) * a.mcount + m) * L + th] =
                    make_double2(Ds[w][(2 * q) * LS64_DS + lane], Ds[w][(2 * q + 1) * LS64_DS + lane]);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- k_gemm ------
// C[M][N] = A[M][K] * Bm[K][N], row-major, on matrix cores (16x16x4 MFMA, FP64 or FP32).
// MFMA operand layout (both types): A fragment lane l holds
// A[l % 16][l / 16], B fragment B[l / 16][l % 16].  Result register j of lane l holds
// column l % 16 and row 4 (l / 16) + j for FP32 but row l / 16 + 4 j for FP64
// (checked on the device).

template <typename Tp>
struct Mfma16;
template <>
struct Mfma16<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int j) { return (lane >> 4) + 4 * j; }
};
template <>
struct Mfma16<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int j) { return 4 * (lane >> 4) + j; }
};

template <typename Tp>
struct GemmCfg;
template <>
struct GemmCfg<float> {
    static constexpr int BN = 128, BK = 16, VEC = 4, APAD = 4, BPAD = 16;
    typedef float4 V;
};
template <>
struct GemmCfg<double> {
    // 64 columns per block: a wave's 64 x 32 FP64 tile keeps its accumulators in 64 registers
    static constexpr int BN = 64, BK = 16, VEC = 2, APAD = 2, BPAD = 16;
    typedef double2 V;
};

// Workgroup tile 128 x BN (four waves of 64 x BN/2; BN = 128 for FP32, 64 for FP64), K staged
// BK at a time through two LDS buffers: the next K slice is fetched from global
// memory into registers (16-byte vector loads when K and N allow) while the current
// one feeds the matrix cores.  A is kept [m][k] with row stride BK + APAD and B [k][n]
// with row stride BN + BPAD, chosen so that the fragment reads of each half-wave fall
// on distinct banks (FP32: strides 36 and 144 words; FP64: 36 and 160 words, 8-byte reads).  Tiles
// are assigned XCD-aware: consecutive workgroups go to different XCDs (each with its
// own L2), so workgroup b runs tile (m, n) = (b % 8 + 8 ((b / 8) / nt), (b / 8) % nt),
// and all column tiles of a 128-row block of A are read on one XCD.
template <typename Tp>
__global__ __launch_bounds__(256) void k_gemm(const Tp *__restrict__ A, const Tp *__restrict__ Bm,
                                              Tp *__restrict__ C, int M, int N, int K, int accum, int mt, int nt,
                                              int vec)
{
    constexpr int BM = 128, BN = GemmCfg<Tp>::BN, BK = GemmCfg<Tp>::BK, VEC = GemmCfg<Tp>::VEC;
    constexpr int WN = BN / 32;        // 16-column MFMA tiles per wave (two waves across the block)
    constexpr int AS = BK + GemmCfg<Tp>::APAD, BS = BN + GemmCfg<Tp>::BPAD;
    constexpr int AV = BM * BK / VEC / 256, BV = BK * BN / VEC / 256;   // vectors per thread
    typedef typename GemmCfg<Tp>::V V;
    typedef typename Mfma16<Tp>::v4 v4;
    extern __shared__ __align__(16) unsigned char gemm_smem[];
    Tp *As = reinterpret_cast<Tp *>(gemm_smem);          // [2][BM][AS]
    Tp *Bs = As + 2 * BM * AS;                            // [2][BK][BS]
    const int bid = blockIdx.x, kx = bid >> 3;
    const int mtile = (bid & 7) + 8 * (kx / nt), ntile = kx % nt;
    if (mtile >= mt) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row0 = mtile * BM, col0 = ntile * BN;
    V ra[AV], rb[BV];
    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < AV; ++r) {
            const int f = tid + 256 * r;
            const int am = f / (BK / VEC), aq = f % (BK / VEC);
            const int gr = row0 + am, gk = k0 + aq * VEC;
            Tp t[VEC];
            if (vec && gr < M && gk < K) {
                const V x = *reinterpret_cast<const V *>(A + (size_t)gr * K + gk);
                __builtin_memcpy(t, &x, sizeof(V));
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) t[e] = (gr < M && gk + e < K) ? A[(size_t)gr * K + gk + e] : Tp(0);
            }
            __builtin_memcpy(&ra[r], t, sizeof(V));
        }
#pragma unroll
        for (int r = 0; r < BV; ++r) {
            const int f = tid + 256 * r;
            const int bk = f / (BN / VEC), bq = f % (BN / VEC);
            const int gk = k0 + bk, gc = col0 + bq * VEC;
            Tp t[VEC];
            if (vec && gk < K && gc < N) {
                const V x = *reinterpret_cast<const V *>(Bm + (size_t)gk * N + gc);
                __builtin_memcpy(t, &x, sizeof(V));
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) t[e] = (gk < K && gc + e < N) ? Bm[(size_t)gk * N + gc + e] : Tp(0);
            }
            __builtin_memcpy(&rb[r], t, sizeof(V));
        }
    };
    auto sstore = [&](int buf) {
        Tp *a = As + buf * BM * AS;
        Tp *b = Bs + buf * BK * BS;
#pragma unroll
        for (int r = 0; r < AV; ++r) {
            const int f = tid + 256 * r;
            const int am = f / (BK / VEC), aq = f % (BK / VEC);
            *reinterpret_cast<V *>(a + am * AS + aq * VEC) = ra[r];
        }
#pragma unroll
        for (int r = 0; r < BV; ++r) {
            const int f = tid + 256 * r;
            const int bk = f / (BN / VEC), bq = f % (BN / VEC);
            *reinterpret_cast<V *>(b + bk * BS + bq * VEC) = rb[r];
        }
    };
    v4 acc[4][WN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = v4{0, 0, 0, 0};
    const int nk = (K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const int cur = t & 1;
        if (t + 1 < nk) gload((t + 1) * BK);
        const Tp *a = As + cur * BM * AS;
        const Tp *b = Bs + cur * BK * BS;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            Tp af[4], bf[WN];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = a[(wr * 64 + i * 16 + (lane & 15)) * AS + kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < WN; ++j) bf[j] = b[(kk + (lane >> 4)) * BS + wc * (BN / 2) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) acc[i][j] = Mfma16<Tp>::op(af[i], bf[j], acc[i][j]);
        }
        if (t + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    // accumulate into C only when asked (a uniform branch: the plain store never reads C)
    if (accum) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gr = row0 + wr * 64 + i * 16 + Mfma16<Tp>::row(lane, r);
                    const int gc = col0 + wc * (BN / 2) + j * 16 + (lane & 15);
                    if (gr < M && gc < N) C[(size_t)gr * N + gc] += acc[i][j][r];
                }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gr = row0 + wr * 64 + i * 16 + Mfma16<Tp>::row(lane, r);
                    const int gc = col0 + wc * (BN / 2) + j * 16 + (lane & 15);
                    if (gr < M && gc < N) C[(size_t)gr * N + gc] = acc[i][j][r];
                }
    }
}

// -------------------------------------------------------------- DFTs -------
//
// Prime-factor DFT of length n = n1 n2 (gcd(n1, n2) = 1) of complex rows held
// in LDS.  Input index (m1 n2 + m2 n1) mod n sits at LDS position m1 n2 + m2
// (table inpos maps the index to its position); stage 1 transforms over m1
// (length n1), stage 2 over m2 (length n2), with no twiddles between stages;
// output frequency (a1 e1 + a2 e2) mod n ends at position a1 n2 + a2 (table
// outpos).  Each stage pairs indices k and p-k of an odd length p:
//   u_k = x_k + x_{p-k},  v_k = x_k - x_{p-k},  h = (p-1)/2,
//   A_j = x_0 + sum_{k=1..h} u_k cos(2 pi jk/p),  B_j = sum_{k=1..h} v_k sin(2 pi jk/p),
//   X_j = A_j + i sgn B_j,  X_{p-j} = A_j - i sgn B_j,
// a quarter of the real multiplications of the plain sum.  A thread owns a
// block of J outputs j by C sequences (DftBlk); when every thread of the block
// holds at most one such task per stage, a stage reads its buffer, waits at a
// barrier and overwrites it in place (one LDS buffer of n per row pair).
// Rows are paired as z = x1 + i x2 (two real rows per complex DFT).  Tr is the
// arithmetic type; only FP64 is defined (DftBlk has no other specialisation, so
// the paired kernels cannot be instantiated for FP32: the FP32 path uses the
// matrix-core DFT and the direct prime-factor kernels below).

template <typename Tr>
struct DftBlk;
template <>
struct DftBlk<double> {
    static constexpr int J = 2, C = 3;
};

template <typename Tr>
struct DftTask {
    typedef typename V2<Tr>::t C2;
    static constexpr int DJB = DftBlk<Tr>::J, DCB = DftBlk<Tr>::C;
    C2 A[DJB][DCB], Bv[DJB][DCB];
};

// Compute the task (jb, cb) of one stage: element (k, c) at buf[k*sj + c*sc].
template <typename Tr>
__device__ inline void dft_task(const typename V2<Tr>::t *buf, const typename V2<Tr>::t *tw, int p, int q, int sj,
                                int sc, int jb, int cb, DftTask<Tr> &T)
{
    typedef typename V2<Tr>::t C2;
    constexpr int DJB = DftBlk<Tr>::J, DCB = DftBlk<Tr>::C;
    const int h = (p - 1) / 2, j0 = jb * DJB, c0 = cb * DCB;
    int off[DCB];
#pragma unroll
    for (int c = 0; c < DCB; ++c) off[c] = (c0 + c < q ? c0 + c : q - 1) * sc;
#pragma unroll
    for (int c = 0; c < DCB; ++c) {
        const C2 x0 = buf[off[c]];
#pragma unroll
        for (int j = 0; j < DJB; ++j) {
            T.A[j][c] = x0;
            T.Bv[j][c] = mk2<Tr>(0, 0);
        }
    }
    int t[DJB];
#pragma unroll
    for (int j = 0; j < DJB; ++j) t[j] = 0;
#pragma unroll 1
    for (int k = 1; k <= h; ++k) {
        C2 u[DCB], v[DCB];
#pragma unroll
        for (int c = 0; c < DCB; ++c) {
            const C2 z1 = buf[k * sj + off[c]], z2 = buf[(p - k) * sj + off[c]];
            u[c] = mk2<Tr>(z1.x + z2.x, z1.y + z2.y);
            v[c] = mk2<Tr>(z1.x - z2.x, z1.y - z2.y);
        }
#pragma unroll
        for (int j = 0; j < DJB; ++j) {
            t[j] += j0 + j;
            if (t[j] >= p) t[j] -= p;
            const C2 w = tw[t[j]];
#pragma unroll
            for (int c = 0; c < DCB; ++c) {
                T.A[j][c].x = fma(u[c].x, w.x, T.A[j][c].x);
                T.A[j][c].y = fma(u[c].y, w.x, T.A[j][c].y);
                T.Bv[j][c].x = fma(v[c].x, w.y, T.Bv[j][c].x);
                T.Bv[j][c].y = fma(v[c].y, w.y, T.Bv[j][c].y);
            }
        }
    }
}

template <typename Tr>
__device__ inline void dft_task_store(typename V2<Tr>::t *buf, int p, int q, int sj, int sc, int jb, int cb,
                                      const DftTask<Tr> &T, Tr sgn)
{
    constexpr int DJB = DftBlk<Tr>::J, DCB = DftBlk<Tr>::C;
    const int h = (p - 1) / 2, j0 = jb * DJB, c0 = cb * DCB;
#pragma unroll
    for (int j = 0; j < DJB; ++j) {
        const int jj = j0 + j;
        if (jj > h) continue;
#pragma unroll
        for (int c = 0; c < DCB; ++c) {
            if (c0 + c >= q) continue;
            const int o = (c0 + c) * sc;
            const auto &A = T.A[j][c];
            const auto &B = T.Bv[j][c];
            buf[jj * sj + o] = mk2<Tr>(A.x - sgn * B.y, A.y + sgn * B.x);
            if (jj > 0) buf[(p - jj) * sj + o] = mk2<Tr>(A.x + sgn * B.y, A.y - sgn * B.x);
        }
    }
}

template <typename Tr>
__host__ __device__ inline int dft_tasks(int p, int q)
{
    return ((p - 1) / 2 + DftBlk<Tr>::J) / DftBlk<Tr>::J * ((q + DftBlk<Tr>::C - 1) / DftBlk<Tr>::C);
}

// One stage over R slots of n elements: src -> dst (dst == src when every thread
// holds at most one task, else a separate buffer; then tasks loop).
template <typename Tr>
__device__ inline void pfa_stage(typename V2<Tr>::t *src, typename V2<Tr>::t *dst, const typename V2<Tr>::t *tw,
                                 int n, int p, int q, int sj, int sc, int R, Tr sgn)
{
    const int t1 = dft_tasks<Tr>(p, q), nc = (q + DftBlk<Tr>::C - 1) / DftBlk<Tr>::C;
    if (src == dst) {
        const bool act = (int)threadIdx.x < R * t1;
        const int s = act ? threadIdx.x / t1 : 0, t = act ? threadIdx.x % t1 : 0;
        DftTask<Tr> T;
        if (act) dft_task<Tr>(src + (size_t)s * n, tw, p, q, sj, sc, t / nc, t % nc, T);
        __syncthreads();
        if (act) dft_task_store<Tr>(dst + (size_t)s * n, p, q, sj, sc, t / nc, t % nc, T, sgn);
    } else {
        for (int task = threadIdx.x; task < R * t1; task += blockDim.x) {
            const int s = task / t1, t = task % t1;
            DftTask<Tr> T;
            dft_task<Tr>(src + (size_t)s * n, tw, p, q, sj, sc, t / nc, t % nc, T);
            dft_task_store<Tr>(dst + (size_t)s * n, p, q, sj, sc, t / nc, t % nc, T, sgn);
        }
    }
    __syncthreads();
}

// Both stages on R row pairs (slots) held at Z + s n; the result ends in Z.  Y is
// Z itself when every thread holds at most one task per stage, else R n more
// elements of LDS.  tw1, tw2: twiddles in LDS.
template <typename Tr>
__device__ inline void pfa_stages(typename V2<Tr>::t *Z, typename V2<Tr>::t *Y, const typename V2<Tr>::t *tw1,
                                  const typename V2<Tr>::t *tw2, int n, int n1, int n2, int R, Tr sgn)
{
    pfa_stage<Tr>(Z, Y, tw1, n, n1, n2, n2, 1, R, sgn);
    pfa_stage<Tr>(Y, Z, tw2, n, n2, n1, 1, n2, R, sgn);
}

template <typename Tr>
__device__ inline typename V2<Tr>::t *dft_smem_setup(const DftArgs &a, unsigned char *raw)
{
    typedef typename V2<Tr>::t C2;
    C2 *tw = reinterpret_cast<C2 *>(raw);
    const double2 *w1 = reinterpret_cast<const double2 *>(a.w1), *w2 = reinterpret_cast<const double2 *>(a.w2);
    for (int i = threadIdx.x; i < a.n1 + a.n2; i += blockDim.x) {
        const double2 w = i < a.n1 ? w1[i] : w2[i - a.n1];
        tw[i] = mk2<Tr>((Tr)w.x, (Tr)w.y);
    }
    return tw + a.n1 + a.n2;
}

// c2r: two Hermitian rows E1, E2 (m = 0..Lh-1, complex) -> two real rows of length n.
// x(a) = scale * (Re E_0 + 2 Re sum_{m>=1} E_m e^{+2 pi i m a/n})
template <typename Tr>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_dft_c2r(const DftArgs a)
{
    typedef typename V2<Tr>::t C2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2 *Z = dft_smem_setup<Tr>(a, smem_raw);
    const C2 *tw1 = reinterpret_cast<const C2 *>(smem_raw), *tw2 = tw1 + a.n1;
    const int n = a.n, Lh = (n + 1) / 2, R = a.rpb;
    const long pair0 = (long)blockIdx.x * R;
    const Tr sc = (Tr)a.scale;
    for (int idx = threadIdx.x; idx < R * Lh; idx += blockDim.x) {
        const int s = idx / Lh, mm = idx - s * Lh;
        const long r1 = 2 * (pair0 + s);
        if (r1 >= a.nrows) continue;
        const bool has2 = r1 + 1 < a.nrows;
        C2 z1 = reinterpret_cast<const C2 *>(a.in)[r1 * a.istride + mm];
        C2 z2 = has2 ? reinterpret_cast<const C2 *>(a.in)[(r1 + 1) * a.istride + mm] : mk2<Tr>(0, 0);
        C2 *Zs = Z + (size_t)s * n;
        if (mm == 0) {
            Zs[a.inpos[0]] = mk2<Tr>(sc * z1.x, sc * z2.x);
        } else {
            Zs[a.inpos[mm]] = mk2<Tr>(sc * (z1.x - z2.y), sc * (z1.y + z2.x));       // z1 + i z2
            Zs[a.inpos[n - mm]] = mk2<Tr>(sc * (z1.x + z2.y), sc * (z2.x - z1.y));   // conj(z1) + i conj(z2)
        }
    }
    __syncthreads();
    pfa_stages<Tr>(Z, a.inplace ? Z : Z + (size_t)R * n, tw1, tw2, n, a.n1, a.n2, R, (Tr)1);
    for (int idx = threadIdx.x; idx < R * n; idx += blockDim.x) {
        const int s = idx / n, aa = idx - s * n;
        const long r1 = 2 * (pair0 + s);
        if (r1 >= a.nrows) continue;
        const C2 z = Z[(size_t)s * n + a.outpos[aa]];
        reinterpret_cast<Tr *>(a.out)[r1 * a.ostride + aa] = z.x;
        if (r1 + 1 < a.nrows) reinterpret_cast<Tr *>(a.out)[(r1 + 1) * a.ostride + aa] = z.y;
    }
}

// r2c: two real rows x1, x2 of length n -> X_m = scale * sum_a x(a) e^{-2 pi i m a/n}, m = 0..Lh-1.
// Tin: element type of the input rows.
template <typename Tr, typename Tin>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_dft_r2c(const DftArgs a)
{
    typedef typename V2<Tr>::t C2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2 *Z = dft_smem_setup<Tr>(a, smem_raw);
    const C2 *tw1 = reinterpret_cast<const C2 *>(smem_raw), *tw2 = tw1 + a.n1;
    const int n = a.n, Lh = (n + 1) / 2, R = a.rpb;
    const long pair0 = (long)blockIdx.x * R;
    for (int idx = threadIdx.x; idx < R * n; idx += blockDim.x) {
        const int s = idx / n, mm = idx - s * n;
        const long r1 = 2 * (pair0 + s);
        if (r1 >= a.nrows) continue;
        const Tin *x = reinterpret_cast<const Tin *>(a.in);
        const Tr x1 = (Tr)x[r1 * a.istride + mm];
        const Tr x2 = r1 + 1 < a.nrows ? (Tr)x[(r1 + 1) * a.istride + mm] : (Tr)0;
        Z[(size_t)s * n + a.inpos[mm]] = mk2<Tr>(x1, x2);
    }
    __syncthreads();
    pfa_stages<Tr>(Z, a.inplace ? Z : Z + (size_t)R * n, tw1, tw2, n, a.n1, a.n2, R, (Tr)-1);
    const Tr h = (Tr)(0.5 * a.scale);
    for (int idx = threadIdx.x; idx < R * Lh; idx += blockDim.x) {
        const int s = idx / Lh, mm = idx - s * Lh;
        const long r1 = 2 * (pair0 + s);
        if (r1 >= a.nrows) continue;
        const C2 *Zs = Z + (size_t)s * n;
        const C2 X = Zs[a.outpos[mm]];
        const C2 Xc = Zs[a.outpos[mm == 0 ? 0 : n - mm]];
        C2 *O = reinterpret_cast<C2 *>(a.out);
        O[r1 * a.ostride + mm] = mk2<Tr>(h * (X.x + Xc.x), h * (X.y - Xc.y));
        if (r1 + 1 < a.nrows) O[(r1 + 1) * a.ostride + mm] = mk2<Tr>(h * (X.y + Xc.y), -h * (X.x - Xc.x));
    }
}

// Plain prime-factor stages (direct length-n1 and length-n2 sums, twiddles read
// from global memory, two LDS buffers per row pair); used by the FP32 (mixed)
// path for lengths the matrix-core DFT does not cover (a prime factor above 95, e.g.
// 1999 at L = 1000).  The sums accumulate in FP64 whatever the element type: a direct
// sum of a prime length takes up to 2L - 1 terms, whose FP32 accumulation alone would
// approach 1e-6 of the result.  Position p holds input index pin[p] and, after both
// stages, output frequency pout[p].

template <typename Tr>
__device__ inline void pfa_stages_direct(typename V2<Tr>::t *Z, typename V2<Tr>::t *Y, const double2 *w1,
                                  const double2 *w2, int n1, int n2, Tr sgn)
{
    typedef typename V2<Tr>::t C2;
    const int tid = threadIdx.x, nt = blockDim.x;
    {
        const int nb1 = (n1 + 3) / 4, nb2 = (n2 + 3) / 4;
        for (int task = tid; task < nb1 * nb2; task += nt) {
            const int a1b = (task / nb2) * 4, m2b = (task % nb2) * 4;
            double2 acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
            int tw[4], st[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) { st[i] = (a1b + i) % n1; tw[i] = 0; }
            for (int m1 = 0; m1 < n1; ++m1) {
                double2 z[4], w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int m2 = m2b + j < n2 ? m2b + j : n2 - 1;
                    const C2 zt = Z[m1 * n2 + m2];
                    z[j] = make_double2((double)zt.x, (double)zt.y);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double2 wd = w1[tw[i]];
                    w[i] = make_double2(wd.x, (double)sgn * wd.y);
                    tw[i] += st[i];
                    if (tw[i] >= n1) tw[i] -= n1;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[i][j].x = fma(z[j].x, w[i].x, fma(-z[j].y, w[i].y, acc[i][j].x));
                        acc[i][j].y = fma(z[j].x, w[i].y, fma(z[j].y, w[i].x, acc[i][j].y));
                    }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (a1b + i < n1 && m2b + j < n2) Y[(a1b + i) * n2 + m2b + j] = mk2<Tr>((Tr)acc[i][j].x, (Tr)acc[i][j].y);
        }
    }
    __syncthreads();
    {
        const int nb1 = (n1 + 3) / 4, nb2 = (n2 + 3) / 4;
        for (int task = tid; task < nb1 * nb2; task += nt) {
            const int a1b = (task / nb2) * 4, a2b = (task % nb2) * 4;
            double2 acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
            int tw[4], st[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) { st[j] = (a2b + j) % n2; tw[j] = 0; }
            for (int m2 = 0; m2 < n2; ++m2) {
                double2 y[4], w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int a1 = a1b + i < n1 ? a1b + i : n1 - 1;
                    const C2 yt = Y[a1 * n2 + m2];
                    y[i] = make_double2((double)yt.x, (double)yt.y);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double2 wd = w2[tw[j]];
                    w[j] = make_double2(wd.x, (double)sgn * wd.y);
                    tw[j] += st[j];
                    if (tw[j] >= n2) tw[j] -= n2;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[i][j].x = fma(y[i].x, w[j].x, fma(-y[i].y, w[j].y, acc[i][j].x));
                        acc[i][j].y = fma(y[i].x, w[j].y, fma(y[i].y, w[j].x, acc[i][j].y));
                    }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (a1b + i < n1 && a2b + j < n2) Z[(a1b + i) * n2 + a2b + j] = mk2<Tr>((Tr)acc[i][j].x, (Tr)acc[i][j].y);
        }
    }
    __syncthreads();
}

// c2r: two Hermitian rows E1, E2 (m = 0..Lh-1, complex) -> two real rows of length n.
// x(a) = scale * (Re E_0 + 2 Re sum_{m>=1} E_m e^{+2 pi i m a/n})
template <typename Tr>
__global__ __launch_bounds__(128) void k_dft_c2r_direct(const DftArgs a)
{
    typedef typename V2<Tr>::t C2;
    extern __shared__ unsigned char smem_raw[];
    C2 *smem = reinterpret_cast<C2 *>(smem_raw);
    const int n = a.n, n1 = a.n1, n2 = a.n2, Lh = (n + 1) / 2;
    C2 *Z = smem, *Y = smem + n;
    const double2 *w1 = reinterpret_cast<const double2 *>(a.w1), *w2 = reinterpret_cast<const double2 *>(a.w2);
    const int tid = threadIdx.x;
    const long r1 = 2L * blockIdx.x, r2 = r1 + 1;
    const bool has2 = r2 < a.nrows;
    const C2 *E1 = reinterpret_cast<const C2 *>(a.in) + r1 * a.istride;
    const C2 *E2 = reinterpret_cast<const C2 *>(a.in) + r2 * a.istride;
    const Tr sc = (Tr)a.scale;
    for (int p = tid; p < n; p += blockDim.x) {
        const int mm = a.pin[p];
        C2 z1, z2 = mk2<Tr>(0, 0);
        if (mm < Lh) {
            z1 = E1[mm];
            if (has2) z2 = E2[mm];
            if (mm == 0) { z1.y = 0; z2.y = 0; }
        } else {
            z1 = E1[n - mm];
            z1.y = -z1.y;
            if (has2) { z2 = E2[n - mm]; z2.y = -z2.y; }
        }
        Z[p] = mk2<Tr>(sc * (z1.x - z2.y), sc * (z1.y + z2.x));   // z1 + i z2
    }
    __syncthreads();
    pfa_stages_direct<Tr>(Z, Y, w1, w2, n1, n2, (Tr)1);
    Tr *o1 = reinterpret_cast<Tr *>(a.out) + r1 * a.ostride, *o2 = reinterpret_cast<Tr *>(a.out) + r2 * a.ostride;
    for (int p = tid; p < n; p += blockDim.x) {
        const int aa = a.pout[p];
        o1[aa] = Z[p].x;
        if (has2) o2[aa] = Z[p].y;
    }
}

// r2c: two real rows x1, x2 of length n -> X_m = scale * sum_a x(a) e^{-2 pi i m a/n}, m = 0..Lh-1.
// Tin: element type of the input rows (the mixed path reads FP64 maps into FP32 arithmetic).
template <typename Tr, typename Tin>
__global__ __launch_bounds__(128) void k_dft_r2c_direct(const DftArgs a)
{
    typedef typename V2<Tr>::t C2;
    extern __shared__ unsigned char smem_raw[];
    C2 *smem = reinterpret_cast<C2 *>(smem_raw);
    const int n = a.n, n1 = a.n1, n2 = a.n2, Lh = (n + 1) / 2;
    C2 *Z = smem, *Y = smem + n;
    const double2 *w1 = reinterpret_cast<const double2 *>(a.w1), *w2 = reinterpret_cast<const double2 *>(a.w2);
    const int tid = threadIdx.x;
    const long r1 = 2L * blockIdx.x, r2 = r1 + 1;
    const bool has2 = r2 < a.nrows;
    const Tin *x1 = reinterpret_cast<const Tin *>(a.in) + r1 * a.istride;
    const Tin *x2 = reinterpret_cast<const Tin *>(a.in) + r2 * a.istride;
    for (int p = tid; p < n; p += blockDim.x) {
        const int mm = a.pin[p];
        Z[p] = mk2<Tr>((Tr)x1[mm], has2 ? (Tr)x2[mm] : (Tr)0);
    }
    __syncthreads();
    pfa_stages_direct<Tr>(Z, Y, w1, w2, n1, n2, (Tr)-1);
    C2 *O1 = reinterpret_cast<C2 *>(a.out) + r1 * a.ostride;
    C2 *O2 = reinterpret_cast<C2 *>(a.out) + r2 * a.ostride;
    const Tr h = (Tr)(0.5 * a.scale);
    for (int mm = tid; mm < Lh; mm += blockDim.x) {
        const C2 X = Z[a.outpos[mm]];
        const C2 Xc = Z[a.outpos[mm == 0 ? 0 : n - mm]];
        O1[mm] = mk2<Tr>(h * (X.x + Xc.x), h * (X.y - Xc.y));
        if (has2) O2[mm] = mk2<Tr>(h * (X.y + Xc.y), -h * (X.x - Xc.x));
    }
}

// --------------------------------------------------------- gamma stages ----
//
// Both sides transpose (m, theta) tiles through LDS.  Every global load of a tile is
// issued before the first is used (the n and gamma loops are unrolled to their
// maxima and predicated), so a block keeps its whole tile in flight, and the
// twiddles e^{+-i n gamma_g} are staged once per block in LDS.

constexpr int GAMMA_MAXG = 2 * GAMMA_MAXN - 1;

template <typename Tr, int NN, int NG>
__device__ __forceinline__ void gamma_twiddles(const GammaArgs &a, typename V2<Tr>::t (*tw)[NG])
{
    const int tid = threadIdx.x;
    if (tid < NN * NG) {
        const int ni = tid / NG, g = tid % NG;
        Tr c = 0, sn = 0;
        if (ni < a.nn && g < a.ng) {
            int idx = (a.nval[ni] * g) % a.ng;
            if (idx < 0) idx += a.ng;
            c = (Tr)a.tw[2 * idx];
            sn = (Tr)(a.sgn * a.tw[2 * idx + 1]);
        }
        tw[ni][g] = mk2<Tr>(c, sn);
    }
}

// c2r side: E[b][g][theta][m] = ph * fm(m) * sum_ni C[b][ni][m][theta] e^{+i n_ni gamma_g} (complex)
// TM x TT (m x theta) tile per block: loaded theta-fastest, written m-fastest.
template <typename Tr, int TM, int TT, int NN, int NG>
__global__ __launch_bounds__(256) void k_gamma_c2r(const GammaArgs a)
{
    typedef typename V2<Tr>::t C2;
    constexpr int EPT = TM * TT / 256;
    __shared__ C2 tile[NN][TM][TT + 1];
    __shared__ C2 tw[NN][NG];
    const int tid = threadIdx.x;
    const int m0 = blockIdx.x * TM, th0 = blockIdx.y * TT, b = blockIdx.z;
    const C2 *src = reinterpret_cast<const C2 *>(a.src);
    gamma_twiddles<Tr, NN, NG>(a, tw);
    {
        C2 v[EPT][NN];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int idx = tid + 256 * e, tt = idx % TT, tm = idx / TT;
            const int m = m0 + tm, th = th0 + tt;
            const bool ok = m < a.M && th < a.L;
#pragma unroll
            for (int ni = 0; ni < NN; ++ni)
                v[e][ni] = (ok && ni < a.nn) ? src[(((size_t)b * a.nn + ni) * a.M + m) * a.L + th] : mk2<Tr>(0, 0);
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int idx = tid + 256 * e, tt = idx % TT, tm = idx / TT;
#pragma unroll
            for (int ni = 0; ni < NN; ++ni) tile[ni][tm][tt] = v[e][ni];
        }
    }
    __syncthreads();
    const Tr phr = (Tr)a.phr, phi = (Tr)a.phi;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + 256 * e, tm = idx % TM, tt = idx / TM;
        const int m = m0 + tm, th = th0 + tt;
        if (m >= a.M || th >= a.L) continue;
        C2 x[NN];
#pragma unroll
        for (int ni = 0; ni < NN; ++ni) x[ni] = tile[ni][tm][tt];
        const Tr fm = (Tr)((m == 0) ? a.fm0 : a.fm1) * (Tr)a.wscale;
        C2 *dst = reinterpret_cast<C2 *>(a.dst) + ((size_t)b * a.ng * a.L + th) * a.Mout + m;
        for (int g = 0; g < a.ng; ++g) {
            Tr re = 0, im = 0;
#pragma unroll
            for (int ni = 0; ni < NN; ++ni) {
                const C2 w = tw[ni][g];
                re += x[ni].x * w.x - x[ni].y * w.y;
                im += x[ni].x * w.y + x[ni].y * w.x;
            }
            dst[(size_t)g * a.L * a.Mout] = mk2<Tr>(fm * (phr * re - phi * im), fm * (phr * im + phi * re));
        }
    }
}

// r2c side: F[sig][b][m'][ni][c][theta] = w * fm(m) * ph * sum_g X[b][g][theta][m] e^{-i n_ni gamma_g}
// TM x TT tile per block: loaded m-fastest, written theta-fastest.
template <typename Tr, int TM, int TT, int NN, int NG>
__global__ __launch_bounds__(256) void k_gamma_r2c(const GammaArgs a)
{
    typedef typename V2<Tr>::t C2;
    constexpr int EPT = TM * TT / 256;
    __shared__ Tr tile[NN][2][TM][TT + 1];
    __shared__ C2 tw[NN][NG];
    const int tid = threadIdx.x;
    const int m0 = blockIdx.x * TM, th0 = blockIdx.y * TT, b = blockIdx.z;
    const C2 *src = reinterpret_cast<const C2 *>(a.src);
    Tr *dst = reinterpret_cast<Tr *>(a.dst);
    gamma_twiddles<Tr, NN, NG>(a, tw);
    C2 x[EPT][NG];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + 256 * e, tm = idx % TM, tt = idx / TM;
        const int m = m0 + tm, th = th0 + tt;
        const bool ok = m < a.M && th < a.L;
#pragma unroll
        for (int g = 0; g < NG; ++g)
            x[e][g] = (ok && g < a.ng) ? src[(((size_t)b * a.ng + g) * a.L + th) * a.Min + m] : mk2<Tr>(0, 0);
    }
    __syncthreads();
    const Tr phr = (Tr)a.phr, phi = (Tr)a.phi;
    // gamma outermost: one sample's twiddles are live at a time
    Tr ar[EPT][NN], ai[EPT][NN];
#pragma unroll
    for (int e = 0; e < EPT; ++e)
#pragma unroll
        for (int ni = 0; ni < NN; ++ni) { ar[e][ni] = 0; ai[e][ni] = 0; }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        C2 w[NN];
#pragma unroll
        for (int ni = 0; ni < NN; ++ni) w[ni] = tw[ni][g];
#pragma unroll
        for (int e = 0; e < EPT; ++e)
#pragma unroll
            for (int ni = 0; ni < NN; ++ni) {
                ar[e][ni] += x[e][g].x * w[ni].x - x[e][g].y * w[ni].y;
                ai[e][ni] += x[e][g].x * w[ni].y + x[e][g].y * w[ni].x;
            }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + 256 * e, tm = idx % TM, tt = idx / TM;
        const int m = m0 + tm;
        const Tr fm = (Tr)((m == 0) ? a.fm0 : a.fm1) * (Tr)a.wscale;
#pragma unroll
        for (int ni = 0; ni < NN; ++ni) {
            tile[ni][0][tm][tt] = fm * (phr * ar[e][ni] - phi * ai[e][ni]);
            tile[ni][1][tm][tt] = fm * (phr * ai[e][ni] + phi * ar[e][ni]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + 256 * e, tt = idx % TT, tm = idx / TT;
        const int m = m0 + tm, th = th0 + tt;
        if (m >= a.M || th >= a.L) continue;
        const int sig = (m + a.npar) & 1;
        const int mp = m >> 1;
        const size_t base = (sig == 0 ? 0 : (size_t)a.B * a.M0 * a.nn * 2)
                            + (((size_t)b * (sig == 0 ? a.M0 : a.M1) + mp) * a.nn) * 2;
#pragma unroll
        for (int ni = 0; ni < NN; ++ni) {
            if (ni >= a.nn) break;
            dst[(base + (size_t)ni * 2 + 0) * a.L + th] = tile[ni][0][tm][tt];
            dst[(base + (size_t)ni * 2 + 1) * a.L + th] = tile[ni][1][tm][tt];
        }
    }
}

// -------------------------------------------------------------- combine ----
// fhat[b][m][l] = sum_terms ph_t * sum_ni P_t[b][m][ni][l]   (FP64, fixed order; a term's P
// may hold FP32 values, widened as they are read)
__global__ __launch_bounds__(256) void k_combine(const CombineArgs a)
{
    const int l = blockIdx.x * 256 + threadIdx.x;
    const int m = blockIdx.y, b = blockIdx.z;
    if (l >= a.L) return;
    double re = 0.0, im = 0.0;
    if (l >= m) {
        for (int t = 0; t < a.nterms; ++t) {
            const CombineTerm &c = a.t[t];
            if (m >= c.L || l >= c.L) continue;
            double sr = 0.0, si = 0.0;
            for (int ni = 0; ni < c.nn; ++ni) {
                const size_t e = ((((size_t)b * c.L + m) * c.nn + ni) * c.L + l) * 2;
                if (c.f32) {
                    const float *p = static_cast<const float *>(c.P) + e;
                    sr += (double)p[0];
                    si += (double)p[1];
                } else {
                    const double *p = static_cast<const double *>(c.P) + e;
                    sr += p[0];
                    si += p[1];
                }
            }
            re += c.phr * sr - c.phi * si;
            im += c.phr * si + c.phi * sr;
        }
    }
    double *o = a.out + (((size_t)b * a.L + m) * a.L + l) * 2;
    o[0] = re;
    o[1] = im;
}

// ------------------------------------------------- sigma-grouped rows ----
// [b][ni][m][theta] complex  <->  [sig][b][m'][ni][c][theta] real rows, sig = (m + npar) & 1
template <typename Tr>
__global__ void k_pack_sigma(const Tr *in, Tr *out, int B, int nn, int M, int L, int npar,
                             int M0, int M1, int dir)
{
    const int th = blockIdx.x * 256 + threadIdx.x;
    const int m = blockIdx.y;
    const int bn = blockIdx.z;          // b * nn + ni
    if (th >= L) return;
    const int b = bn / nn, ni = bn % nn;
    const int sig = (m + npar) & 1, mp = m >> 1;
    const size_t base = (sig == 0 ? 0 : (size_t)B * M0 * nn * 2)
                        + ((((size_t)b * (sig == 0 ? M0 : M1) + mp) * nn + ni) * 2);
    const size_t ci = (((size_t)b * nn + ni) * M + m) * L + th;
    if (dir == 0) {
        out[(base + 0) * L + th] = in[ci * 2 + 0];
        out[(base + 1) * L + th] = in[ci * 2 + 1];
    } else {
        out[ci * 2 + 0] = in[(base + 0) * L + th];
        out[ci * 2 + 1] = in[(base + 1) * L + th];
    }
}

// out[b][p][m][l] = phi[p][l] in[b][p][m][l] (complex), rows of L x L harmonic
// coefficients per radial index p (ball scaling filter, applied elementwise).
__global__ void k_scale_pl(const double *in, double *out, const double *phi, int P, int L, size_t total)
{
    const size_t LL = (size_t)L * L;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int l = (int)(i % L);
        const int p = (int)((i / LL) % P);
        const double f = phi[(size_t)p * L + l];
        out[2 * i] = f * in[2 * i];
        out[2 * i + 1] = f * in[2 * i + 1];
    }
}

__global__ void k_convert_f64_f32(const double *in, float *out, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

__global__ void k_convert_f32_f64(const float *in, double *out, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}

// ----------------------------------------------------- harmonic layouts ----
// internal [b][m][l] (m >= 0)  <->  external [b][l][m + L - 1] (all m)
__global__ void k_flm_to_ext(const double *in, double *out, int L, int B)
{
    const int l = blockIdx.x, b = blockIdx.y;
    for (int mm = threadIdx.x; mm < 2 * L - 1; mm += blockDim.x) {
        const int m = mm - (L - 1);
        double re = 0.0, im = 0.0;
        if (l >= (m < 0 ? -m : m)) {
            const int am = m < 0 ? -m : m;
            const double *p = in + (((size_t)b * L + am) * L + l) * 2;
            re = p[0];
            im = p[1];
            if (m < 0) {  // f_{l,-m} = (-1)^m conj(f_lm)
                im = -im;
                if (am & 1) { re = -re; im = -im; }
            }
        }
        double *o = out + (((size_t)b * L + l) * (2 * L - 1) + mm) * 2;
        o[0] = re;
        o[1] = im;
    }
}

__global__ void k_flm_from_ext(const double *in, double *out, int L, int B)
{
    const int m = blockIdx.x, b = blockIdx.y;
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        double re = 0.0, im = 0.0;
        if (l >= m) {
            const double *p = in + (((size_t)b * L + l) * (2 * L - 1) + (m + L - 1)) * 2;
            re = p[0];
            im = p[1];
        }
        double *o = out + (((size_t)b * L + m) * L + l) * 2;
        o[0] = re;
        o[1] = im;
    }
}

// ------------------------------------------------------------ spin-s maps ----
// A complex spin-s map f = u + i v is held as the two real maps u, v (batch entries 2b and
// 2b + 1).  Its spin-s harmonic coefficients g_lm (all m) use d^l_{m,-s} for m >= 0 and,
// through d^l_{-m,-s} = (-1)^{m+s} d^l_{m,s}, d^l_{m,s} for the negative orders.  On the
// real side every sum runs over m >= 0 with two n slots: slot 0 for n = -s, slot 1 for
// n = +s.

// X [2B][m][2][l] complex: the forward sums of u and v (weights sqrt((2l+1)/(4 pi)) applied),
// so that g_lm = (-1)^s (XU0 + i XV0) and h_lm = (-1)^m conj(g_{l,-m}) = XU1 - i XV1 (m >= 0).
// pairs [2B][m][l]: the coefficients of the real maps A, B with g = A + i B,
//   a = (g + h) / 2, b = (g - h) / (2i); ext [B][l][2L-1] complex: g itself.
__global__ void k_spin_combine(const double *X, double *pairs, double *ext, int L, int s)
{
    const int m = blockIdx.x, b = blockIdx.y;
    const int as = s < 0 ? -s : s, l0 = m > as ? m : as;
    const double ss = (as & 1) ? -1.0 : 1.0;
    const double2 *X2 = reinterpret_cast<const double2 *>(X);
    const double2 *xu = X2 + (((size_t)(2 * b) * L + m) * 2) * L;
    const double2 *xv = X2 + (((size_t)(2 * b + 1) * L + m) * 2) * L;
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        double2 g = make_double2(0.0, 0.0), h = make_double2(0.0, 0.0);
        if (l >= l0) {
            const double2 u0 = xu[l], v0 = xv[l], u1 = xu[L + l], v1 = xv[L + l];
            g = make_double2(ss * (u0.x - v0.y), ss * (u0.y + v0.x));
            h = make_double2(u1.x + v1.y, u1.y - v1.x);
        }
        if (pairs) {
            double2 *pa = reinterpret_cast<double2 *>(pairs);
            pa[((size_t)(2 * b) * L + m) * L + l] = make_double2(0.5 * (g.x + h.x), 0.5 * (g.y + h.y));
            pa[((size_t)(2 * b + 1) * L + m) * L + l] = make_double2(0.5 * (g.y - h.y), -0.5 * (g.x - h.x));
        }
        if (ext) {
            double2 *e = reinterpret_cast<double2 *>(ext) + ((size_t)b * L + l) * (2 * L - 1) + (L - 1);
            e[m] = g;
            if (m > 0) {   // g_{l,-m} = (-1)^m conj(h)
                const double sm = (m & 1) ? -1.0 : 1.0;
                e[-m] = make_double2(sm * h.x, -sm * h.y);
            }
        }
    }
}

// The inverse: from g (ext [B][l][2L-1], or pairs [2B][m][l] with g = a + i b, h = a - i b)
// to the coefficient rows cin [2B][2][m][l] of the two real maps u = Re f, v = Im f:
//   u: slot 0 = (-1)^s g / 2, slot 1 = h / 2;  v: slot 0 = -i (-1)^s g / 2, slot 1 = i h / 2,
// so that summing the two slots after the l-sums gives the m >= 0 Fourier rows of u and v.
__global__ void k_spin_split(const double *pairs, const double *ext, double *cin, int L, int s)
{
    const int m = blockIdx.x, b = blockIdx.y;
    const int as = s < 0 ? -s : s, l0 = m > as ? m : as;
    const double hs = (as & 1) ? -0.5 : 0.5;
    const double sm = (m & 1) ? -1.0 : 1.0;
    double2 *c2 = reinterpret_cast<double2 *>(cin);
    double2 *cu = c2 + (((size_t)(2 * b) * 2) * L + m) * L;
    double2 *cv = c2 + (((size_t)(2 * b + 1) * 2) * L + m) * L;
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        double2 g = make_double2(0.0, 0.0), h = make_double2(0.0, 0.0);
        if (l >= l0) {
            if (pairs) {
                const double2 *pa = reinterpret_cast<const double2 *>(pairs);
                const double2 a = pa[((size_t)(2 * b) * L + m) * L + l], c = pa[((size_t)(2 * b + 1) * L + m) * L + l];
                g = make_double2(a.x - c.y, a.y + c.x);
                h = make_double2(a.x + c.y, a.y - c.x);
            } else {
                const double2 *e = reinterpret_cast<const double2 *>(ext) + ((size_t)b * L + l) * (2 * L - 1) + (L - 1);
                g = e[m];
                const double2 n = e[-m];
                h = make_double2(sm * n.x, -sm * n.y);
            }
        }
        cu[l] = make_double2(hs * g.x, hs * g.y);
        cu[(size_t)L * L + l] = make_double2(0.5 * h.x, 0.5 * h.y);
        cv[l] = make_double2(hs * g.y, -hs * g.x);
        cv[(size_t)L * L + l] = make_double2(-0.5 * h.y, 0.5 * h.x);
    }
}

// ----------------------------------------------------------- SO(3) layouts ----
// external "nlm" -> internal [b][n index][m >= 0][l] (the inverse transform reads m >= 0)
__global__ void k_wig_ext_to_int(const double *ext, double *in, int L, int N)
{
    const int m = blockIdx.x, ni = blockIdx.y, b = blockIdx.z;
    const int ng = 2 * N - 1;
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        const double *src = ext + ((((size_t)b * ng + ni) * L + l) * (2 * L - 1) + (m + L - 1)) * 2;
        double *dst = in + ((((size_t)b * ng + ni) * L + m) * L + l) * 2;
        dst[0] = src[0];
        dst[1] = src[1];
    }
}

// theta-sum outputs P[b][m][qi][l] (defined at l >= m; zero at m <= l < max(m, |n|)) of the
// n values nval[qi] -> external "nlm": entry (n, l, m >= 0), and for m >= 1 the entry
// (-n, l, -m) = (-1)^(m+n) conj(n, l, m) of a real function on SO(3); zero at l < max(|m|, |n|)
struct WigNvals {
    int v[8];
};
__global__ void k_wig_sum_to_ext(const double *P, double *ext, int L, int N, int nq, const WigNvals nv)
{
    const int m = blockIdx.x, qi = blockIdx.y, b = blockIdx.z;
    const int n = nv.v[qi], an = n < 0 ? -n : n;
    const int ng = 2 * N - 1, na = 2 * L - 1;
    const double sg = ((m + n) & 1) ? -1.0 : 1.0;
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        double re = 0.0, im = 0.0;
        if (l >= m && l >= an) {
            const double *src = P + ((((size_t)b * L + m) * nq + qi) * L + l) * 2;
            re = src[0];
            im = src[1];
        }
        double *d = ext + ((((size_t)b * ng + (n + N - 1)) * L + l) * na + (m + L - 1)) * 2;
        d[0] = re;
        d[1] = im;
        if (m >= 1) {
            double *e = ext + ((((size_t)b * ng + (-n + N - 1)) * L + l) * na + (-m + L - 1)) * 2;
            e[0] = sg * re;
            e[1] = -sg * im;
        }
    }
}

void launch_wig_ext_to_int(const double *ext, double *in, int L, int N, int B, hipStream_t st)
{
    hipLaunchKernelGGL(k_wig_ext_to_int, dim3(L, 2 * N - 1, B), dim3(256), 0, st, ext, in, L, N);
}

void launch_wig_sum_to_ext(const double *P, double *ext, int L, int N, int B, int nq, const int *nval,
                           hipStream_t st)
{
    WigNvals nv{};
    for (int i = 0; i < nq && i < 8; ++i) nv.v[i] = nval[i];
    hipLaunchKernelGGL(k_wig_sum_to_ext, dim3(L, nq, B), dim3(256), 0, st, P, ext, L, N, nq, nv);
}

// ------------------------------------------------------------- launchers ---

template <int T, int NS>
static void launch_lsum_t(const LsumArgs &a, int B, hipStream_t st)
{
    const int nch = (a.L + 64 * T - 1) / (64 * T);
    dim3 grid(a.mcount, a.nn, B * nch);
    if (a.dtab) hipLaunchKernelGGL((k_lsum<T, NS, true>), grid, dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_lsum<T, NS, false>), grid, dim3(64), 0, st, a);
}

void launch_dtable(const LsumArgs &a, double *tab, const int64_t *doff, hipStream_t st)
{
    if (a.L <= 0 || a.nn <= 0) return;
    dim3 grid(a.L, a.nn, (a.L + 63) / 64);
    hipLaunchKernelGGL(k_dtable, grid, dim3(64), 0, st, a, tab, doff);
}

void launch_lsum(const LsumArgs &a, int NS, int B, hipStream_t st)
{
    if (B >= 16 && a.mcount > 0) {
        // many maps: one recursion for 32 columns on FP64 matrix cores
        const int ntt = (a.L + 63) / 64;
        const int W = ntt >= 4 ? 4 : (ntt >= 2 ? 2 : 1);
        const int ntb = (ntt + W - 1) / W;
        const long nunit = (long)a.mcount * a.nn * ((2 * B * NS + 31) / 32);
        dim3 grid((unsigned)(8L * ntb * ((nunit + 7) / 8)));
        const dim3 blk(64 * W);
        if (NS == 1) {
            if (W == 4) hipLaunchKernelGGL((k_lsum_mm64<1, 4>), grid, blk, 0, st, a, a.A, a.B, a.S, B);
            else if (W == 2) hipLaunchKernelGGL((k_lsum_mm64<1, 2>), grid, blk, 0, st, a, a.A, a.B, a.S, B);
            else hipLaunchKernelGGL((k_lsum_mm64<1, 1>), grid, blk, 0, st, a, a.A, a.B, a.S, B);
        } else {
            if (W == 4) hipLaunchKernelGGL((k_lsum_mm64<2, 4>), grid, blk, 0, st, a, a.A, a.B, a.S, B);
            else if (W == 2) hipLaunchKernelGGL((k_lsum_mm64<2, 2>), grid, blk, 0, st, a, a.A, a.B, a.S, B);
            else hipLaunchKernelGGL((k_lsum_mm64<2, 1>), grid, blk, 0, st, a, a.A, a.B, a.S, B);
        }
        if (a.npol > 0) {
            dim3 pgrid(a.mcount, a.nn, B);
            if (NS == 1) hipLaunchKernelGGL(k_lsum_polar<1>, pgrid, dim3(64), 0, st, a);
            else hipLaunchKernelGGL(k_lsum_polar<2>, pgrid, dim3(64), 0, st, a);
        }
        return;
    }
    int T = a.L > 512 ? 8 : (a.L > 256 ? 8 : (a.L > 128 ? 4 : (a.L > 64 ? 2 : 1)));
    if (a.tileT == 1 || a.tileT == 2 || a.tileT == 4 || a.tileT == 8) T = a.tileT;
    if (NS == 1) {
        switch (T) {
            case 1: launch_lsum_t<1, 1>(a, B, st); break;
            case 2: launch_lsum_t<2, 1>(a, B, st); break;
            case 4: launch_lsum_t<4, 1>(a, B, st); break;
            default: launch_lsum_t<8, 1>(a, B, st); break;
        }
    } else {
        switch (T) {
            case 1: launch_lsum_t<1, 2>(a, B, st); break;
            case 2: launch_lsum_t<2, 2>(a, B, st); break;
            case 4: launch_lsum_t<4, 2>(a, B, st); break;
            default: launch_lsum_t<8, 2>(a, B, st); break;
        }
    }
    if (a.npol > 0 && a.mcount > 0) {
        dim3 grid(a.mcount, a.nn, B);
        if (NS == 1) hipLaunchKernelGGL(k_lsum_polar<1>, grid, dim3(64), 0, st, a);
        else hipLaunchKernelGGL(k_lsum_polar<2>, grid, dim3(64), 0, st, a);
    }
}

template <int T, int NS>
static void launch_tsum_t(const TsumArgs &a, int B, int nw, hipStream_t st)
{
    dim3 grid(a.mcount, a.nn, B);
    if (a.dtab) hipLaunchKernelGGL((k_tsum<T, NS, true>), grid, dim3(64 * nw), 0, st, a);
    else hipLaunchKernelGGL((k_tsum<T, NS, false>), grid, dim3(64 * nw), 0, st, a);
}

void launch_tsum_vec(const TsumArgs &a, int NS, int B, hipStream_t st);

void launch_tsum(const TsumArgs &a, int NS, int B, hipStream_t st)
{
    if (B >= 16 && a.L <= 1024 && a.mcount > 0) {
        // many maps: one recursion for 32 columns on FP64 matrix cores
        const int NW = (a.L + 63) / 64;
        const int ngrp = (2 * B * NS + 31) / 32;
        dim3 grid(a.mcount, a.nn, ngrp);
        const size_t smem = sizeof(double) * TS64_RS * (size_t)NW;   // 128 KB at NW = 16
        if (NS == 1) hipLaunchKernelGGL(k_tsum_mm64<1>, grid, dim3(64 * NW), smem, st, a, a.A, a.B_);
        else hipLaunchKernelGGL(k_tsum_mm64<2>, grid, dim3(64 * NW), smem, st, a, a.A, a.B_);
    } else {
        launch_tsum_vec(a, NS, B, st);
    }
    if (a.npol > 0 && a.mcount > 0) {
        dim3 grid(a.mcount, a.nn, B);
        if (NS == 1) hipLaunchKernelGGL(k_tsum_polar<1>, grid, dim3(64), 0, st, a);
        else hipLaunchKernelGGL(k_tsum_polar<2>, grid, dim3(64), 0, st, a);
    }
}

void launch_tsum_vec(const TsumArgs &a, int NS, int B, hipStream_t st)
{
    // T theta samples per lane (at most 4, keeping the lane state in registers) and
    // up to 4 waves per block: T = ceil(L / (64 nw)) with nw = ceil(L / 256)
    const int nw = std::min(4, std::max(1, (a.L + 255) / 256));
    const int T = (a.L + 64 * nw - 1) / (64 * nw);
    if (NS == 1) {
        if (T <= 1) launch_tsum_t<1, 1>(a, B, nw, st);
        else if (T <= 2) launch_tsum_t<2, 1>(a, B, nw, st);
        else launch_tsum_t<4, 1>(a, B, nw, st);
    } else {
        if (T <= 1) launch_tsum_t<1, 2>(a, B, nw, st);
        else if (T <= 2) launch_tsum_t<2, 2>(a, B, nw, st);
        else launch_tsum_t<4, 2>(a, B, nw, st);
    }
}

void launch_scale_pl(const double *in, double *out, const double *phi, int P, int L, size_t total, hipStream_t st)
{
    if (total == 0) return;
    const size_t blocks = std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_scale_pl, dim3((unsigned)blocks), dim3(256), 0, st, in, out, phi, P, L, total);
}

// Precompute mode, forward SHT (FP64): the theta quadrature and the theta sums fold into
// one table per m, Dt^l_m(theta) = sum_theta' d^l_m0(theta') T_sigma[theta][theta'] (rows
// l = m..L-1, theta contiguous), so that f_lm = w_l sum_theta F_m(theta) Dt^l_m(theta) with
// F the sigma-grouped rows before the quadrature.  A batched product over m: the 2B
// columns (map, re/im) of m against its L - m table rows, with the tiling, double buffering
// and FP64 16x16x4 products of k_gemm<double>; the table slab [64 l][16 theta] is
// transposed into the [k][n] LDS layout as it is staged.  Tiles (m, column tile, degree
// tile) come from eight per-XCD lists.  Output: the internal flm [B][m][l] complex.
__global__ __launch_bounds__(256) void k_sht_tab(const ShtTab a)
{
    constexpr int BM = 128, BN = 64, BK = 16, WN = BN / 32;
    constexpr int AS = BK + 2, BS = BN + 16;
    typedef double v4 __attribute__((ext_vector_type(4)));
    __shared__ __align__(16) double As[2 * BM * AS];
    __shared__ __align__(16) double Bs[2 * BK * BS];
    const int xc = blockIdx.x & 7, kx = blockIdx.x >> 3;
    if (kx >= a.cnt[xc]) return;
    const int4 tl = a.tiles[a.off[xc] + kx];
    const int m = tl.x, L = a.L, M = 2 * a.B, N = L - m, K = L;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row0 = tl.y * BM, col0 = tl.z * BN;
    const int sig = m & 1, mp = m >> 1;
    const size_t sigoff = sig == 0 ? 0 : (size_t)a.B * a.M0 * 2;
    const int Msig = sig == 0 ? a.M0 : a.M1;
    const double *Bt = a.tab + a.toff[m];
    // staging: A 128 rows x 16 k as double2 (4 per thread); B 64 rows (l) x 16 k (4 per thread)
    const double *arow[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int f = tid + 256 * r, am = f >> 3, gr = row0 + am;
        arow[r] = gr < M ? a.F + (sigoff + ((size_t)(gr >> 1) * Msig + mp) * 2 + (gr & 1)) * L : nullptr;
    }
    const int bl = tid >> 2, bq = tid & 3;
    double2 ra[4], rb[2];
    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = tid + 256 * r, aq = f & 7, gk = k0 + 2 * aq;
            ra[r] = (arow[r] && gk < K) ? *reinterpret_cast<const double2 *>(arow[r] + gk) : make_double2(0.0, 0.0);
        }
        const int gl = col0 + bl, gk = k0 + 4 * bq;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            rb[h] = (gl < N && gk < K) ? *reinterpret_cast<const double2 *>(Bt + (size_t)gl * K + gk + 2 * h)
                                       : make_double2(0.0, 0.0);
    };
    auto sstore = [&](int buf) {
        double *as = As + buf * BM * AS;
        double *bs = Bs + buf * BK * BS;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = tid + 256 * r, am = f >> 3, aq = f & 7;
            *reinterpret_cast<double2 *>(as + am * AS + 2 * aq) = ra[r];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bs[(4 * bq + 2 * h) * BS + bl] = rb[h].x;
            bs[(4 * bq + 2 * h + 1) * BS + bl] = rb[h].y;
        }
    };
    v4 acc[4][WN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = v4{0, 0, 0, 0};
    const int nk = (K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const int cur = t & 1;
        if (t + 1 < nk) gload((t + 1) * BK);
        const double *as = As + cur * BM * AS;
        const double *bs = Bs + cur * BK * BS;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double af[4], bf[WN];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = as[(wr * 64 + i * 16 + (lane & 15)) * AS + kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < WN; ++j) bf[j] = bs[(kk + (lane >> 4)) * BS + wc * (BN / 2) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (t + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    // result register r of lane: column lane % 16, row lane / 16 + 4 r (FP64 layout)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gr = row0 + wr * 64 + i * 16 + (lane >> 4) + 4 * r;
                const int gc = col0 + wc * (BN / 2) + j * 16 + (lane & 15);
                if (gr < M && gc < N) {
                    const int l = m + gc;
                    a.out[(((size_t)(gr >> 1) * L + m) * L + l) * 2 + (gr & 1)] = acc[i][j][r] * a.w[l];
                }
            }
}

// The inverse SHT's theta rows from the table of d^l_m0(theta) (rows l = m..L-1, theta
// contiguous): C_m(theta) = sum_l (w_l f_lm) d^l_m0(theta) for the 2B columns (map, re/im) of
// each m, batched over m as k_sht_tab (the table is the [k][n] operand as it is; the
// coefficients are staged from the internal flm, times w_l).  Output: rows [B][m][theta]
// complex, as the l-sum writes them for the gamma and DFT stages.
__global__ __launch_bounds__(256) void k_shti_tab(const ShtTab a)
{
    constexpr int BM = 128, BN = 64, BK = 16, WN = BN / 32;
    constexpr int AS = BK + 2, BS = BN + 16;
    typedef double v4 __attribute__((ext_vector_type(4)));
    __shared__ __align__(16) double As[2 * BM * AS];
    __shared__ __align__(16) double Bs[2 * BK * BS];
    const int xc = blockIdx.x & 7, kx = blockIdx.x >> 3;
    if (kx >= a.cnt[xc]) return;
    const int4 tl = a.tiles[a.off[xc] + kx];
    const int m = tl.x, L = a.L, M = 2 * a.B, N = L, K = L - m;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row0 = tl.y * BM, col0 = tl.z * BN;
    const double *Bt = a.tab + a.toff[m];
    const double2 *flm = reinterpret_cast<const double2 *>(a.F);
    double2 ra[4], rb[2];
    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = tid + 256 * r, bm = f >> 4, kq = f & 15;
            const int b = (row0 >> 1) + bm, k = k0 + kq;
            double2 v = make_double2(0.0, 0.0);
            if (2 * b < M && k < K) {
                v = flm[((size_t)b * L + m) * L + m + k];
                const double wl = a.w[m + k];
                v.x *= wl;
                v.y *= wl;
            }
            ra[r] = v;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int f = tid + 256 * h, bk = f >> 5, bq = f & 31;
            const int k = k0 + bk, n = col0 + 2 * bq;
            rb[h] = (k < K && n < N) ? *reinterpret_cast<const double2 *>(Bt + (size_t)k * L + n)
                                     : make_double2(0.0, 0.0);
        }
    };
    auto sstore = [&](int buf) {
        double *as = As + buf * BM * AS;
        double *bs = Bs + buf * BK * BS;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = tid + 256 * r, bm = f >> 4, kq = f & 15;
            as[(2 * bm) * AS + kq] = ra[r].x;
            as[(2 * bm + 1) * AS + kq] = ra[r].y;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int f = tid + 256 * h, bk = f >> 5, bq = f & 31;
            *reinterpret_cast<double2 *>(bs + bk * BS + 2 * bq) = rb[h];
        }
    };
    v4 acc[4][WN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = v4{0, 0, 0, 0};
    const int nk = (K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const int cur = t & 1;
        if (t + 1 < nk) gload((t + 1) * BK);
        const double *as = As + cur * BM * AS;
        const double *bs = Bs + cur * BK * BS;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double af[4], bf[WN];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = as[(wr * 64 + i * 16 + (lane & 15)) * AS + kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < WN; ++j) bf[j] = bs[(kk + (lane >> 4)) * BS + wc * (BN / 2) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (t + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gr = row0 + wr * 64 + i * 16 + (lane >> 4) + 4 * r;
                const int gc = col0 + wc * (BN / 2) + j * 16 + (lane & 15);
                if (gr < M && gc < N) a.out[(((size_t)(gr >> 1) * L + m) * L + gc) * 2 + (gr & 1)] = acc[i][j][r];
            }
}

void launch_shti_tab(const ShtTab &a, hipStream_t st)
{
    int mx = 0;
    for (int x = 0; x < 8; ++x) mx = std::max(mx, a.cnt[x]);
    if (mx == 0) return;
    hipLaunchKernelGGL(k_shti_tab, dim3(8u * (unsigned)mx), dim3(256), 0, st, a);
}

void launch_sht_tab(const ShtTab &a, hipStream_t st)
{
    int mx = 0;
    for (int x = 0; x < 8; ++x) mx = std::max(mx, a.cnt[x]);
    if (mx == 0) return;
    hipLaunchKernelGGL(k_sht_tab, dim3(8u * (unsigned)mx), dim3(256), 0, st, a);
}

template <typename Tp>
static void launch_gemm_t(const Tp *A, const Tp *Bm, Tp *C, int M, int N, int K, hipStream_t st, bool accum)
{
    if (M <= 0 || N <= 0) return;
    constexpr int VEC = GemmCfg<Tp>::VEC, BK = GemmCfg<Tp>::BK, BN = GemmCfg<Tp>::BN;
    const int mt = (M + 127) / 128, nt = (N + BN - 1) / BN;
    const bool vec = (K % VEC == 0) && (N % VEC == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)Bm % 16 == 0);
    const size_t lds = sizeof(Tp) * 2 * ((size_t)128 * (BK + GemmCfg<Tp>::APAD) + (size_t)BK * (BN + GemmCfg<Tp>::BPAD));
    const unsigned blocks = 8u * (unsigned)nt * (unsigned)((mt + 7) / 8);
    hipLaunchKernelGGL(k_gemm<Tp>, dim3(blocks), dim3(256), lds, st, A, Bm, C, M, N, K, accum ? 1 : 0, mt, nt,
                       vec ? 1 : 0);
}

void launch_gemm(const double *A, const double *Bm, double *C, int M, int N, int K, hipStream_t st, bool accum)
{
    launch_gemm_t<double>(A, Bm, C, M, N, K, st, accum);
}

void launch_gemm_f32(const float *A, const float *Bm, float *C, int M, int N, int K, hipStream_t st)
{
    launch_gemm_t<float>(A, Bm, C, M, N, K, st, false);
}

// Row pairs per block and threads per block for a DFT launch.  In-place stages
// when every thread holds at most one task per stage (up to 4 row pairs, 32 KB of
// rows per block); otherwise one row pair, 256 threads and a second buffer.
template <typename Tr>
static void dft_shape(DftArgs &a, int &threads, size_t &lds)
{
    const size_t elem = 2 * sizeof(Tr);
    const int t = std::max(dft_tasks<Tr>(a.n1, a.n2), dft_tasks<Tr>(a.n2, a.n1));
    int R = 1;
    if (t <= 256) {
        while (R < 4 && (R + 1) * t <= 256 && (size_t)(R + 1) * a.n * elem <= 32768) ++R;
        threads = std::max(64, (R * t + 63) / 64 * 64);
        a.inplace = 1;
    } else {
        threads = 256;
        a.inplace = 0;
    }
    a.rpb = R;
    lds = ((size_t)R * a.n * (a.inplace ? 1 : 2) + a.n1 + a.n2) * elem;
}

void launch_dft_c2r(DftArgs a, hipStream_t st, bool f32)
{
    if (a.nrows <= 0) return;
    if (f32) {
        if (dft_mm_ok(a)) {
            launch_dft_mm_c2r(a, st);
            return;
        }
        hipLaunchKernelGGL(k_dft_c2r_direct<float>, dim3((a.nrows + 1) / 2), dim3(128),
                           sizeof(float2) * 2 * (size_t)a.n, st, a);
        return;
    }
    int thr;
    size_t lds;
    dft_shape<double>(a, thr, lds);
    dim3 grid((unsigned)(((a.nrows + 1) / 2 + a.rpb - 1) / a.rpb));
    hipLaunchKernelGGL(k_dft_c2r<double>, grid, dim3(thr), lds, st, a);
}

void launch_dft_r2c(DftArgs a, hipStream_t st, bool f32, bool in64, bool in32)
{
    if (a.nrows <= 0) return;
    if (f32) {
        if (!in64 && dft_mm_ok(a)) {
            launch_dft_mm_r2c(a, st);
            return;
        }
        const size_t lds = sizeof(float2) * 2 * (size_t)a.n;
        if (in64)
            hipLaunchKernelGGL((k_dft_r2c_direct<float, double>), dim3((a.nrows + 1) / 2), dim3(128), lds, st, a);
        else
            hipLaunchKernelGGL((k_dft_r2c_direct<float, float>), dim3((a.nrows + 1) / 2), dim3(128), lds, st, a);
        return;
    }
    int thr;
    size_t lds;
    dft_shape<double>(a, thr, lds);
    dim3 grid((unsigned)(((a.nrows + 1) / 2 + a.rpb - 1) / a.rpb));
    if (in32)
        hipLaunchKernelGGL((k_dft_r2c<double, float>), grid, dim3(thr), lds, st, a);
    else
        hipLaunchKernelGGL((k_dft_r2c<double, double>), grid, dim3(thr), lds, st, a);
}

// tiles: FP32 c2r 32 m x 16 theta (256-byte row segments on the larger, written side),
// FP32 r2c 16 m x 32 theta, FP64 16 x 16; each about 35 KB of LDS
void launch_gamma_c2r(const GammaArgs &a, hipStream_t st, bool f32)
{
    // the loops over n and gamma are unrolled to NN, NG; nn = ng = 1 (harmonic transforms)
    // has its own instantiation
    const bool one = a.nn == 1 && a.ng == 1;
    if (f32) {
        dim3 grid((a.M + 31) / 32, (a.L + 15) / 16, a.B);
        if (one) hipLaunchKernelGGL((k_gamma_c2r<float, 32, 16, 1, 1>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_gamma_c2r<float, 32, 16, GAMMA_MAXN, GAMMA_MAXG>), grid, dim3(256), 0, st, a);
    } else {
        dim3 grid((a.M + 15) / 16, (a.L + 15) / 16, a.B);
        if (one) hipLaunchKernelGGL((k_gamma_c2r<double, 16, 16, 1, 1>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_gamma_c2r<double, 16, 16, GAMMA_MAXN, GAMMA_MAXG>), grid, dim3(256), 0, st, a);
    }
}

void launch_gamma_r2c(const GammaArgs &a, hipStream_t st, bool f32)
{
    const bool one = a.nn == 1 && a.ng == 1;
    if (f32) {
        // 32 x 32 tiles: 256-byte reads of the rows over m (218 VGPRs, two blocks per CU)
        dim3 grid((a.M + 31) / 32, (a.L + 31) / 32, a.B);
        if (one) hipLaunchKernelGGL((k_gamma_r2c<float, 32, 32, 1, 1>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_gamma_r2c<float, 32, 32, GAMMA_MAXN, GAMMA_MAXG>), grid, dim3(256), 0, st, a);
    } else {
        dim3 grid((a.M + 15) / 16, (a.L + 15) / 16, a.B);
        if (one) hipLaunchKernelGGL((k_gamma_r2c<double, 16, 16, 1, 1>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_gamma_r2c<double, 16, 16, GAMMA_MAXN, GAMMA_MAXG>), grid, dim3(256), 0, st, a);
    }
}

void launch_convert(const void *in, void *out, size_t n, bool to_f32, hipStream_t st)
{
    if (n == 0) return;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
    if (to_f32) hipLaunchKernelGGL(k_convert_f64_f32, dim3(blocks), dim3(256), 0, st, (const double *)in, (float *)out, n);
    else hipLaunchKernelGGL(k_convert_f32_f64, dim3(blocks), dim3(256), 0, st, (const float *)in, (double *)out, n);
}

void launch_combine(const CombineArgs &a, int B, hipStream_t st)
{
    dim3 grid((a.L + 255) / 256, a.L, B);
    hipLaunchKernelGGL(k_combine, grid, dim3(256), 0, st, a);
}

void launch_pack_sigma(const double *in, double *out, int B, int nn, int M, int L, int npar, int M0,
                       int M1, int dir, hipStream_t st)
{
    dim3 grid((L + 255) / 256, M, B * nn);
    hipLaunchKernelGGL(k_pack_sigma<double>, grid, dim3(256), 0, st, in, out, B, nn, M, L, npar, M0, M1, dir);
}

void launch_pack_sigma_f32(const float *in, float *out, int B, int nn, int M, int L, int npar, int M0,
                           int M1, int dir, hipStream_t st)
{
    dim3 grid((L + 255) / 256, M, B * nn);
    hipLaunchKernelGGL(k_pack_sigma<float>, grid, dim3(256), 0, st, in, out, B, nn, M, L, npar, M0, M1, dir);
}

void launch_flm_to_ext(const double *in, double *out, int L, int B, hipStream_t st)
{
    hipLaunchKernelGGL(k_flm_to_ext, dim3(L, B), dim3(256), 0, st, in, out, L, B);
}

void launch_flm_from_ext(const double *in, double *out, int L, int B, hipStream_t st)
{
    hipLaunchKernelGGL(k_flm_from_ext, dim3(L, B), dim3(256), 0, st, in, out, L, B);
}

void launch_spin_combine(const double *X, double *pairs, double *ext, int L, int s, int B, hipStream_t st)
{
    hipLaunchKernelGGL(k_spin_combine, dim3(L, B), dim3(256), 0, st, X, pairs, ext, L, s);
}

void launch_spin_split(const double *pairs, const double *ext, double *cin, int L, int s, int B, hipStream_t st)
{
    hipLaunchKernelGGL(k_spin_split, dim3(L, B), dim3(256), 0, st, pairs, ext, cin, L, s);
}

}  // namespace s2w
