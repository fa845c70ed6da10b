// Mixed-precision, batched Wigner contractions (gfx950).
//
// The Wigner-d recursion runs in FP64 (one lane per theta sample, log-rescaled
// start, same tables as the FP64 kernels) and is shared by every map of the
// batch; d is rounded to FP32 in chunks of 16 degrees, staged in LDS, and
// contracted on FP32 matrix cores (16x16x4 MFMA) against coefficient tiles of
// 64 columns, a column being (scale, map, real/imaginary part).  Partial sums
// are promoted to FP64: every 64 degrees for the sum over l, and in the
// fixed-order cross-wave reduction for the sum over theta.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "s2w_dev.h"
#include "s2w_kern.h"

namespace s2w {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ k_lsum_mm ----
// C_s[b][ni][m][theta] (complex FP32) = sum_{l >= l0} d^l_mn(theta) w_s[ni][l] flm[b][m][l]
// grid (m, ni, theta tiles x column groups of 16 NC columns), one wave per block.

template <int NS, int NC>
__global__ __launch_bounds__(64) void k_lsum_mm(const LsumArgs a, const MixOut o)
{
    constexpr int CW = 16 * NC;        // columns per wave
    const int m = blockIdx.x, ni = blockIdx.y;
    const int L = a.L;
    const int ntt = (L + 63) >> 6;
    const int tt = blockIdx.z % ntt, g = blockIdx.z / ntt;
    const int lane = threadIdx.x;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n;
    const int l0 = m > an ? m : an;
    const int B = o.B, ncols = 2 * B * NS;
    const int th = tt * 64 + lane;
    const bool valid = th < L;

    __shared__ float Ds[16][64 + 4];
    __shared__ float Us[16][CW + 4];
    __shared__ float Ot[CW][64 + 1];

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
    f4 acc[4][NC];
    double accd[4][NC][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            acc[i][j] = f4{0, 0, 0, 0};
#pragma unroll
            for (int r = 0; r < 4; ++r) accd[i][j][r] = 0.0;
        }

    // this lane stages column (lane % CW) for degrees i = lane / CW + (64 / CW) * q
    const int ccol = lane % CW, cpart = lane / CW;
    constexpr int NPART = 64 / CW;
    const int cg = g * CW + ccol;
    int cs = 0, cb = 0, ccc = 0;
    const bool cok = cg < ncols;
    if (cok) {
        cs = cg / (2 * B);
        const int rem = cg - cs * 2 * B;
        cb = rem >> 1;
        ccc = rem & 1;
    }
    const double *wv = a.w[cs < NS ? cs : 0] + (size_t)ni * a.wstride;
    const double *fl = a.flm + ((size_t)cb * a.flm_m + m) * a.flm_l * 2 + ccc;

    int chunk = 0;
    for (int lb = l0; lb < L; lb += 16, ++chunk) {
#pragma unroll
        for (int q = 0; q < 16 / NPART; ++q) {
            const int i = cpart + NPART * q;
            const int l = lb + i;
            float v = 0.f;
            if (cok && l < L) v = (float)(wv[l] * fl[(size_t)l * 2]);
            Us[i][ccol] = v;
        }
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
            const int l = lb + i;
            double A = 0.0, Bv = 0.0, S = 0.0;
            if (l < L) { A = a.A[tabm + l]; Bv = a.B[tabm + l]; S = a.S[tabm + l]; }
            Ds[i][lane] = (valid && k == 0) ? (float)(S * e) : 0.f;
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
            float af[4], bf[NC];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = Ds[kk + (lane >> 4)][i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NC; ++j) bf[j] = Us[kk + (lane >> 4)][j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < NC; ++j) acc[i][j] = mfma16(af[i], bf[j], acc[i][j]);
        }
        __syncthreads();
        if ((chunk & 3) == 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < NC; ++j) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) accd[i][j][r] += (double)acc[i][j][r];
                    acc[i][j] = f4{0, 0, 0, 0};
                }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Ot[j * 16 + (lane & 15)][i * 16 + 4 * (lane >> 4) + r] = (float)(accd[i][j][r] + (double)acc[i][j][r]);
    __syncthreads();
    // write (re, im) pairs with theta contiguous
    for (int p = 0; p < CW / 2; ++p) {
        const int cgp = g * CW + 2 * p;
        if (cgp >= ncols) break;
        const int s = cgp / (2 * B);
        const int b = (cgp - s * 2 * B) >> 1;
        if (valid) {
            float2 *dst = reinterpret_cast<float2 *>(o.out[s]);
            dst[(((size_t)b * a.nn + ni) * a.mcount + m) * L + th] = make_float2(Ot[2 * p][lane], Ot[2 * p + 1][lane]);
        }
    }
}

// ------------------------------------------------------------ k_tsum_mm ----
// P_s[b][m][ni][l] (complex FP64) = S_l w_s[ni][l] sum_theta d^l_mn(theta) h_s[b](theta)
// with h rows (FP32) in the sigma-grouped layout [sig][b][m'][ni][c][theta].
// grid (m, ni, column groups), NW = ceil(L/64) waves per block, wave w owns theta = 64 w + lane.
// Each wave keeps its 64 x 64 (theta x column) slice of h in registers as MFMA
// B operands; per chunk of 16 degrees it writes d (FP32) to LDS, forms the
// 16 x 64 partial product on matrix cores, and the waves' partials are summed
// in FP64 in a fixed order.

template <int NS>
__global__ __launch_bounds__(1024) void k_tsum_mm(const TsumArgs a, const MixIn in)
{
    extern __shared__ float sm[];      // NW x 1024 floats: d chunks, then the partial products
    const int m = blockIdx.x, ni = blockIdx.y, g = blockIdx.z;
    const int L = a.L;
    const int NW = blockDim.x >> 6;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n;
    const int l0 = m > an ? m : an;
    const int B = in.B, ncols = 2 * B * NS;
    const int th = w * 64 + lane;
    const bool valid = th < L;
    float *Dw = sm + (size_t)w * 1024;

    // h slice: hb[ks][j] = h[theta = 64 w + 4 ks + lane / 16][col = 64 g + 16 j + lane % 16]
    const int sig = (m + a.npar) & 1;
    const int mp = m >> 1;
    const size_t sigoff = (sig == 0 ? 0 : (size_t)B * a.M0 * a.nn * 2);
    const int Msig = (sig == 0 ? a.M0 : a.M1);
    float hb[16][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int cg = g * 64 + 16 * j + (lane & 15);
        int s = 0, b = 0, cc = 0;
        const bool cok = cg < ncols;
        if (cok) {
            s = cg / (2 * B);
            const int rem = cg - s * 2 * B;
            b = rem >> 1;
            cc = rem & 1;
        }
        const float *hs = in.h[s < NS ? s : 0];
        const size_t row = sigoff + (((size_t)b * Msig + mp) * a.nn + ni) * 2 + cc;
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int t2 = w * 64 + 4 * ks + (lane >> 4);
            hb[ks][j] = (cok && t2 < L) ? hs[row * L + t2] : 0.f;
        }
    }

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

    for (int lb = l0; lb < L; lb += 16) {
        // d chunk, swizzled [theta][l ^ (theta & 15)] so that both the per-step writes and the
        // MFMA A-operand reads avoid bank conflicts
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
            const int l = lb + i;
            double A = 0.0, Bv = 0.0;
            if (l < L) { A = a.A[tabm + l]; Bv = a.B_[tabm + l]; }
            Dw[lane * 16 + (i ^ (lane & 15))] = (valid && k == 0) ? (float)e : 0.f;
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
        f4 pacc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pacc[j] = f4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int tl = 4 * ks + (lane >> 4);
            const float av = Dw[tl * 16 + ((lane & 15) ^ (tl & 15))];   // A[l = lane%16][theta = tl]
#pragma unroll
            for (int j = 0; j < 4; ++j) pacc[j] = mfma16(av, hb[ks][j], pacc[j]);
        }
        __syncthreads();
        // partial 16 (l) x 64 (col) of this wave: register r of lane -> l = 4 (lane/16) + r, col = 16 j + lane%16
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) Dw[(4 * (lane >> 4) + r) * 64 + 16 * j + (lane & 15)] = pacc[j][r];
        __syncthreads();
        for (int t = threadIdx.x; t < 1024; t += blockDim.x) {
            const int li = t >> 6, col = t & 63;
            const int l = lb + li, cg = g * 64 + col;
            double v = 0.0;
            for (int ww = 0; ww < NW; ++ww) v += (double)sm[(size_t)ww * 1024 + t];
            if (l < L && cg < ncols) {
                const int s = cg / (2 * B);
                const int rem = cg - s * 2 * B;
                const int b = rem >> 1, cc = rem & 1;
                const double sc = a.S[tabm + l] * a.w[s][(size_t)ni * a.wstride + l];
                in.out[s][((((size_t)b * a.mcount + m) * a.nn + ni) * L + l) * 2 + cc] = v * sc;
            }
        }
        __syncthreads();
    }
    // zero l < l0
    const int nz = (l0 < L ? l0 : L);
    for (int t = threadIdx.x; t < nz * 64; t += blockDim.x) {
        const int l = t >> 6, col = t & 63, cg = g * 64 + col;
        if (cg >= ncols) continue;
        const int s = cg / (2 * B);
        const int rem = cg - s * 2 * B;
        const int b = rem >> 1, cc = rem & 1;
        in.out[s][((((size_t)b * a.mcount + m) * a.nn + ni) * L + l) * 2 + cc] = 0.0;
    }
}

// ------------------------------------------------------------- launchers ---

void launch_lsum_mm(const LsumArgs &a, const MixOut &o, int NS, hipStream_t st)
{
    constexpr int NC = 2;
    const int ntt = (a.L + 63) / 64;
    const int ngrp = (2 * o.B * NS + 16 * NC - 1) / (16 * NC);
    dim3 grid(a.mcount, a.nn, ntt * ngrp);
    if (NS == 1) hipLaunchKernelGGL((k_lsum_mm<1, NC>), grid, dim3(64), 0, st, a, o);
    else hipLaunchKernelGGL((k_lsum_mm<2, NC>), grid, dim3(64), 0, st, a, o);
}

void launch_tsum_mm(const TsumArgs &a, const MixIn &in, int NS, hipStream_t st)
{
    const int NW = (a.L + 63) / 64;
    const int ngrp = (2 * in.B * NS + 63) / 64;
    dim3 grid(a.mcount, a.nn, ngrp);
    const size_t smem = sizeof(float) * 1024 * (size_t)NW;
    if (NS == 1) hipLaunchKernelGGL(k_tsum_mm<1>, grid, dim3(64 * NW), smem, st, a, in);
    else hipLaunchKernelGGL(k_tsum_mm<2>, grid, dim3(64 * NW), smem, st, a, in);
}

}  // namespace s2w
