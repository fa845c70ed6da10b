// Mixed-precision, batched Wigner contractions (gfx950).
//
// The Wigner-d recursion runs in FP64 (one lane per theta sample, log-rescaled
// start, same tables as the FP64 kernels) and is shared by every map of the
// batch; d is rounded to FP32 in chunks of 16 degrees, staged in LDS, and
// contracted on FP32 matrix cores (16x16x4 MFMA) against coefficient tiles of
// 64 columns, a column being (scale, map, real/imaginary part).  The sum over l
// is carried from the matrix-core accumulator into a second FP32 accumulator
// every 64 degrees; the sum over theta is completed in FP64 in a fixed-order
// cross-wave reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "s2w_dev.h"
#include "s2w_kern.h"

namespace s2w {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ k_lsum_mm ----

// C_s[b][ni][m][theta] (complex FP32) = sum_{l >= l0} d^l_mn(theta) w_s[ni][l] flm[b][m][l]
// W waves per block: wave w owns the 64-theta tile
// (tb W + w) of one (m, n, group of 64 columns) unit, and the waves share one staged
// 16-degree x 64-column coefficient tile per chunk.  The coefficient loads for the next
// chunk are issued before the current chunk's recursion and matrix-core work, as
// 16-byte (re, im) pairs.  Sums over l accumulate in FP32 on the matrix cores and are
// carried into a second FP32 accumulator every 64 degrees.

constexpr int LS_CPAD = 16;            // coefficient entries past L (zero) read by the last chunk

template <int NS, int W>
__global__ __launch_bounds__(64 * W, 2) void k_lsum_mm(const LsumArgs a, const MixOut o)
{
    constexpr int R = 4 / W;           // staging slots per thread
    const int L = a.L;
    const int ntt = (L + 63) >> 6;
    const int ntb = (ntt + W - 1) / W;
    const int B = o.B, ncols = 2 * B * NS;
    const int ngrp = (ncols + 63) >> 6;
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

    __shared__ float Ds[2][W][16][64 + 4];   // d chunks of each wave [l][theta]; output staging at the end
    __shared__ float Us[2][16][64 + 4];      // coefficient chunks [l][column]
    // recursion coefficients of this (m, n) row: (A_l, B_l) and S_l for l0 <= l < L + LS_CPAD
    // (zero past L), staged once per block
    extern __shared__ double2 lsab[];
    double *lss = reinterpret_cast<double *>(lsab + L + LS_CPAD);

    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    for (int l = l0 + tid; l < L + LS_CPAD; l += 64 * W) {
        double2 v = {0.0, 0.0};
        double sv = 0.0;
        if (l < L) {
            v.x = a.A[tabm + l];
            v.y = a.B[tabm + l];
            sv = a.S[tabm + l];
        }
        lsab[l] = v;
        lss[l] = sv;
    }
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

    // staging: slot q = tid + 64 W r (r < R) of the 32 column pairs x 8 degree pairs of a
    // chunk is column pair p = q / 8 (re, im of one map and scale), degrees lb + iq, lb + iq + 1
    int iq[R], pc[R];
    bool cok[R];
    const double *wv[R];
    const double2 *fl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = tid + 64 * W * r;
        pc[r] = q >> 3;
        iq[r] = (q & 7) * 2;
        const int cg = g * 64 + 2 * pc[r];
        cok[r] = cg < ncols;
        int cs = 0, cb = 0;
        if (cok[r]) {
            cs = cg / (2 * B);
            cb = (cg - cs * 2 * B) >> 1;
        }
        wv[r] = a.w[cs < NS ? cs : 0] + (size_t)ni * a.wstride;
        fl[r] = reinterpret_cast<const double2 *>(a.flm) + ((size_t)cb * a.flm_m + m) * a.flm_l + ni * a.flm_nstride;
    }
    double2 f0[R], f1[R];
    double w0[R], w1[R];
    auto fetch = [&](int lb) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int la = lb + iq[r];
            f0[r] = make_double2(0.0, 0.0);
            f1[r] = make_double2(0.0, 0.0);
            w0[r] = 0.0;
            w1[r] = 0.0;
            if (cok[r] && la < L) { f0[r] = fl[r][la]; w0[r] = wv[r][la]; }
            if (cok[r] && la + 1 < L) { f1[r] = fl[r][la + 1]; w1[r] = wv[r][la + 1]; }
        }
    };
    if (l0 < L) fetch(l0);

    f4 acc[4][4], acc2[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[i][j] = f4{0, 0, 0, 0};
            acc2[i][j] = f4{0, 0, 0, 0};
        }

    // The recursion and the coefficient staging run one chunk ahead of the matrix-core
    // work, into the other of two LDS buffers: chunk c's products are issued between
    // the recursion steps of chunk c + 1 (independent instructions that overlap on the
    // VALU and the matrix cores), and one block barrier per chunk suffices (a buffer is
    // rewritten only after the barrier that follows its last reads).
    auto stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            Us[buf][iq[r]][2 * pc[r]] = (float)(w0[r] * f0[r].x);
            Us[buf][iq[r]][2 * pc[r] + 1] = (float)(w0[r] * f0[r].y);
            Us[buf][iq[r] + 1][2 * pc[r]] = (float)(w1[r] * f1[r].x);
            Us[buf][iq[r] + 1][2 * pc[r] + 1] = (float)(w1[r] * f1[r].y);
        }
    };
    // recursion step i of the chunk starting at degree lc (wave-uniform LDS reads)
    auto rstep = [&](int buf, int lc, int i) {
        const double2 ab = lsab[lc + i];
        const double A = ab.x, Bv = ab.y, S = lss[lc + i];
        Ds[buf][w][i][lane] = (valid && k == 0) ? (float)(S * e) : 0.f;
        const double en = fma(fma(A, cl, fma(A, c, -Bv)), e, -ep);
        ep = e;
        e = en;
        if ((i & 7) == 7 && k < 0 && fabs(e) > 0x1p256) {
            e *= 0x1p-512;
            ep *= 0x1p-512;
            k += 1;
        }
    };
    __syncthreads();                   // coefficient row staged
    if (l0 < L) {
        stage(0);
        if (l0 + 16 < L) fetch(l0 + 16);
#pragma unroll 4
        for (int i = 0; i < 16; ++i) rstep(0, l0, i);
    }
    __syncthreads();
    int chunk = 0;
    for (int lb = l0; lb < L; lb += 16, ++chunk) {
        const int cb = chunk & 1, nb = cb ^ 1;
        const bool nxt = lb + 16 < L;
        if (nxt) {
            stage(nb);
            if (lb + 32 < L) fetch(lb + 32);
        }
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            float af[4], bf[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = Ds[cb][w][kk + (lane >> 4)][i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) bf[j] = Us[cb][kk + (lane >> 4)][j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(af[i], bf[j], acc[i][j]);
            if (nxt) {
#pragma unroll
                for (int i = 0; i < 4; ++i) rstep(nb, lb + 16, kk + i);
            }
        }
        __syncthreads();
        if ((chunk & 3) == 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc2[i][j] += acc[i][j];
                    acc[i][j] = f4{0, 0, 0, 0};
                }
        }
    }
    // output: one 16-column tile at a time through this wave's Ds slice, then
    // (re, im) pairs written with theta contiguous
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Ds[0][w][lane & 15][i * 16 + 4 * (lane >> 4) + r] = acc2[i][j][r] + acc[i][j][r];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int cgp = g * 64 + 16 * j + 2 * q;
            if (cgp < ncols && valid) {
                const int s = cgp / (2 * B);
                const int b = (cgp - s * 2 * B) >> 1;
                float2 *dst = reinterpret_cast<float2 *>(o.out[s]);
                dst[(((size_t)b * a.nn + ni) * a.mcount + m) * L + th] = make_float2(Ds[0][w][2 * q][lane], Ds[0][w][2 * q + 1][lane]);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ k_tsum_mm ----
// P_s[b][m][ni][l] (complex FP64) = S_l w_s[ni][l] sum_theta d^l_mn(theta) h_s[b](theta)
// with h rows (FP32) in the sigma-grouped layout [sig][b][m'][ni][c][theta].
// grid (m, ni, column groups), NW = ceil(L/64) waves per block, wave w owns theta = 64 w + lane.
// Each wave keeps its 64 x 64 (theta x column) slice of h in registers as MFMA
// B operands; per chunk of 16 degrees it writes d (FP32) to its own LDS slice,
// forms the 16 x 64 partial product on matrix cores and stores it over that
// slice, and the waves' partials are summed in FP64 in a fixed order.  The
// slices alternate between two buffers by chunk parity: a wave orders its own
// slice with a wave-level fence, and one block barrier per chunk separates the
// partial products from their sum (the next chunk writes the other buffer, whose
// last readers finished before this chunk's barrier).  The (m, n) row of
// recursion coefficients is staged in LDS once per block, and every LDS address
// of the chunk loop is a per-lane base plus a constant (rows of 17 floats), so
// that the loop holds no per-step address registers.

constexpr int TS_RS = 64 * 17;         // floats per wave slice: d [64 theta][17] or partial [64 col][17]
constexpr int TS_CPAD = 16;            // coefficient entries past L (zero) read by the last chunk

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// wave w's h slice as MFMA B operands: hb[ks][j] = h[theta = 64 w + 4 ks + lane / 16][col =
// 64 g + 16 j + lane % 16], zero for theta >= L or col >= 2 B NS.  A column's h row is
// contiguous in theta, so each 16-column group is read one row per load (lane = theta,
// 256 bytes per row), written to the wave's LDS slice T [16][65] and read back in the
// operand layout.  T (at least 1040 floats) is the wave's own slice, not yet in use.
template <int NS>
__device__ __forceinline__ void tsum_h_slice(const TsumArgs &a, const MixIn &in, int m, int ni, int g, int w,
                                             int lane, float (&hb)[16][4], float *T)
{
    const int L = a.L, B = in.B, ncols = 2 * B * NS;
    const int sig = (m + a.npar) & 1;
    const int mp = m >> 1;
    const size_t sigoff = (sig == 0 ? 0 : (size_t)B * a.M0 * a.nn * 2);
    const int Msig = (sig == 0 ? a.M0 : a.M1);
    const int th = w * 64 + lane;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float t[16];
        // wave-uniform column cg = 64 g + 16 j + c: scale s, and rem = 2 (map) + part, stepped
        int s = (g * 64 + 16 * j) / (2 * B), rem = g * 64 + 16 * j - s * 2 * B;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int cg = g * 64 + 16 * j + c;
            t[c] = 0.f;
            if (cg < ncols && th < L) {
                const size_t row = sigoff + (((size_t)(rem >> 1) * Msig + mp) * a.nn + ni) * 2 + (rem & 1);
                t[c] = in.h[s][row * L + th];
            }
            if (++rem == 2 * B) {
                rem = 0;
                ++s;
            }
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) T[c * 65 + lane] = t[c];
        wave_lds_sync();
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) hb[ks][j] = T[(lane & 15) * 65 + 4 * ks + (lane >> 4)];
        wave_lds_sync();               // read before the next group overwrites T
    }
}

// out[s][b][m][ni][l] = 0 for m <= l < nz (d^l_mn vanishes below max(|m|, |n|)) for this
// block's 32 column pairs: a pair (re, im of one scale and map) owns a contiguous run of
// (re, im) values, written as 16-byte stores by blockDim / 32 threads.  The rows are read
// only at l >= m (by the sum over n and scales), so entries below m are left as they are.
__device__ __forceinline__ void tsum_zero_head(const TsumArgs &a, const MixIn &in, int m, int ni, int g, int nz,
                                               int ncols)
{
    const int tpp = blockDim.x >> 5;
    const int pr = threadIdx.x / tpp, q = threadIdx.x - pr * tpp;
    const int cg = g * 64 + 2 * pr;
    if (cg >= ncols) return;
    const int s = cg / (2 * in.B), b = (cg - s * 2 * in.B) >> 1;
    double2 *row = reinterpret_cast<double2 *>(in.out[s]) + (((size_t)b * a.mcount + m) * a.nn + ni) * a.L;
    for (int l = m + q; l < nz; l += tpp) row[l] = make_double2(0.0, 0.0);
}

template <int NS>
__global__ __launch_bounds__(1024) void k_tsum_mm(const TsumArgs a, const MixIn in, const double *__restrict__ rA,
                                                  const double *__restrict__ rB)
{
    // rA, rB alias a.A, a.B_ (restrict: not written by this kernel)
    extern __shared__ double2 smc[];   // [L + TS_CPAD] (A_l, B_l), then [2][NW][TS_RS] floats
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

    float *sm = reinterpret_cast<float *>(smc + L + TS_CPAD);
    float hb[16][4];
    tsum_h_slice<NS>(a, in, m, ni, g, w, lane, hb, sm + (size_t)w * TS_RS);

    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    double2 *cf = smc;
    for (int l = l0 + (int)threadIdx.x; l < L + TS_CPAD; l += blockDim.x) {
        double2 v = {0.0, 0.0};
        if (l < L) {
            v.x = rA[tabm + l];
            v.y = rB[tabm + l];
        }
        cf[l] = v;
    }
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

    // this thread's first reduction output (column rcol, degree lb + rli of each chunk):
    // its scale-factor rows and output row are resolved once per block
    const int rcol = 2 * ((int)threadIdx.x >> 5) + ((int)threadIdx.x & 1), rli = ((int)threadIdx.x >> 1) & 15;
    const int rcg = g * 64 + rcol;
    const bool rok = rcg < ncols;
    const int rs = rok ? rcg / (2 * B) : 0;
    const int rrem = rok ? rcg - rs * 2 * B : 0;
    const double *Srow = a.S + tabm;
    const double *wrow = a.w[rs] + (size_t)ni * a.wstride;
    double *orow = in.out[rs] + ((((size_t)(rrem >> 1) * a.mcount + m) * a.nn + ni) * L) * 2 + (rrem & 1);

    __syncthreads();                   // coefficient row staged

    int glmin = 1 << 30;
    {
        const int s0 = (g * 64) / (2 * B), s1 = min(NS - 1, (min(g * 64 + 63, ncols - 1)) / (2 * B));
        for (int s = s0; s <= s1; ++s) glmin = min(glmin, a.lmin[s]);
    }
    int par = 0;
    for (int lb = l0; lb < L; lb += 16, par ^= 1) {
        const bool live = lb + 16 > glmin;   // chunks below the filter support issue no products
        float *Dw = sm + (size_t)(par * NW + w) * TS_RS;
        // scale factors of this thread's first output of the chunk, loaded (without a
        // branch, degree clamped) before the chunk's recursion and matrix-core work
        const int lr = lb + rli < L ? lb + rli : L - 1;
        const double s0 = Srow[lr], w0 = wrow[lr];
        // d chunk [theta][17]: lane theta writes its row (the odd row length spreads the
        // 64 lanes over distinct banks); coefficients past L are zero
        float *Dl = Dw + lane * 17;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const double2 ab = cf[lb + i];
            Dl[i] = (valid && k == 0) ? (float)e : 0.f;
            const double en = fma(fma(ab.x, cl, fma(ab.x, c, -ab.y)), e, -ep);
            ep = e;
            e = en;
            if ((i & 7) == 7 && k < 0 && fabs(e) > 0x1p256) {
                e *= 0x1p-512;
                ep *= 0x1p-512;
                k += 1;
            }
        }
        wave_lds_sync();
        f4 pacc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pacc[j] = f4{0, 0, 0, 0};
        // A[l = lane%16][theta = 4 ks + lane/16]
        const float *Da = Dw + (lane >> 4) * 17 + (lane & 15);
        if (live) {
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) {
                const float av = Da[68 * ks];
#pragma unroll
                for (int j = 0; j < 4; ++j) pacc[j] = mfma16(av, hb[ks][j], pacc[j]);
            }
        }
        wave_lds_sync();
        // partial 16 (l) x 64 (col) of this wave, stored [col][l] (stride 17): register r of
        // lane -> l = 4 (lane/16) + r, col = 16 j + lane%16
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) Dw[(16 * j + (lane & 15)) * 17 + 4 * (lane >> 4) + r] = pacc[j][r];
        __syncthreads();
        // the scale product is formed here: the empty asm keeps the compiler from waiting
        // on the two loads before the matrix-core section
        double sc0 = s0, wc0 = w0;
        asm volatile("" : "+v"(sc0), "+v"(wc0));
        // thread -> (column pair, l, re/im) so that a map's 16 degrees x (re, im) are written contiguously
        const float *Pb = sm + (size_t)par * NW * TS_RS;
        for (int t = threadIdx.x; t < 1024; t += 64 * NW) {
            const int col = 2 * (t >> 5) + (t & 1), li = (t >> 1) & 15;
            const int l = lb + li, cg = g * 64 + col;
            // all NW (<= 16) partials are read before the sum, which runs in wave order
            const float *pp = Pb + col * 17 + li;
            float pv[16];
#pragma unroll
            for (int ww = 0; ww < 16; ++ww) {
                const float x = pp[(ww < NW ? ww : 0) * TS_RS];
                pv[ww] = ww < NW ? x : 0.f;
            }
            double v = 0.0;
#pragma unroll
            for (int ww = 0; ww < 16; ++ww) v += (double)pv[ww];
            if (l < L && cg < ncols) {
                if (t == (int)threadIdx.x) {
                    orow[(size_t)l * 2] = v * (sc0 * wc0);
                } else {
                    const int s = cg / (2 * B);
                    const int rem = cg - s * 2 * B;
                    const int b = rem >> 1, cc = rem & 1;
                    const double sc = a.S[tabm + l] * a.w[s][(size_t)ni * a.wstride + l];
                    in.out[s][((((size_t)b * a.mcount + m) * a.nn + ni) * L + l) * 2 + cc] = v * sc;
                }
            }
        }
    }
    tsum_zero_head(a, in, m, ni, g, l0 < L ? l0 : L, ncols);
}

// 16-wave form (L > 960) with the phases of consecutive chunks overlapped.  Per chunk the
// matrix-core products of k steps 0-7 are issued between the reads and FP64 additions of
// the cross-wave sum of the previous chunk's partials; k steps 8-11 follow; the A operands
// of k steps 12-15 are then read together, after which their products are issued between
// the recursion steps of the next chunk, which overwrite the wave's d rows.  The partials
// have their own LDS buffer: one barrier before they are written (every wave has finished
// summing the previous ones) and one after.  Same arithmetic and summation order as
// k_tsum_mm.

constexpr int TS16_CPAD = 32;          // coefficient entries past L (zero): the recursion runs for
                                       // every chunk, including the one after the last

template <int NS>
__global__ __launch_bounds__(1024) void k_tsum_mm16(const TsumArgs a, const MixIn in, const double *__restrict__ rA,
                                                    const double *__restrict__ rB)
{
    // rA, rB alias a.A, a.B_ (restrict: not written by this kernel)
    extern __shared__ double2 smc[];   // [L + TS16_CPAD] (A_l, B_l), d rows [16][TS_RS], partials [16][TS_RS]
    constexpr int NW = 16;
    const int m = blockIdx.x, ni = blockIdx.y, g = blockIdx.z;
    const int L = a.L;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n;
    const int l0 = m > an ? m : an;
    const int B = in.B, ncols = 2 * B * NS;
    const int th = w * 64 + lane;
    const bool valid = th < L;

    float *Dw = reinterpret_cast<float *>(smc + L + TS16_CPAD) + w * TS_RS;
    float hb[16][4];
    tsum_h_slice<NS>(a, in, m, ni, g, w, lane, hb, Dw);

    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    double2 *cf = smc;
    const float *P = reinterpret_cast<const float *>(smc + L + TS16_CPAD) + NW * TS_RS;
    float *Pw = reinterpret_cast<float *>(smc + L + TS16_CPAD) + (NW + w) * TS_RS;
    for (int l = l0 + (int)threadIdx.x; l < L + TS16_CPAD; l += 64 * NW) {
        double2 v = {0.0, 0.0};
        if (l < L) {
            v.x = rA[tabm + l];
            v.y = rB[tabm + l];
        }
        cf[l] = v;
    }
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
    // this thread's reduction output (column rcol, degree lb + rli of each chunk)
    const int rcol = 2 * ((int)threadIdx.x >> 5) + ((int)threadIdx.x & 1), rli = ((int)threadIdx.x >> 1) & 15;
    const int rcg = g * 64 + rcol;
    const bool rok = rcg < ncols;
    const int rs = rok ? rcg / (2 * B) : 0;
    const int rrem = rok ? rcg - rs * 2 * B : 0;
    const double *Srow = a.S + tabm;
    const double *wrow = a.w[rs] + (size_t)ni * a.wstride;
    double *orow = in.out[rs] + ((((size_t)(rrem >> 1) * a.mcount + m) * a.nn + ni) * L) * 2 + (rrem & 1);
    const float *Pr = P + rcol * 17 + rli;

    __syncthreads();                   // coefficient row staged

    // recursion step i of the chunk starting at degree lc: d into row `lane` of this wave's slice
    float *Dl = Dw + lane * 17;
    auto rstep = [&](int lc, int i) {
        const double2 ab = cf[lc + i];
        Dl[i] = (valid && k == 0) ? (float)e : 0.f;
        const double en = fma(fma(ab.x, cl, fma(ab.x, c, -ab.y)), e, -ep);
        ep = e;
        e = en;
        if ((i & 7) == 7 && k < 0 && fabs(e) > 0x1p256) {
            e *= 0x1p-512;
            ep *= 0x1p-512;
            k += 1;
        }
    };
    if (l0 < L) {
#pragma unroll
        for (int i = 0; i < 16; ++i) rstep(l0, i);
    }

    const float *Da = Dw + (lane >> 4) * 17 + (lane & 15);   // A[l = lane%16][theta = 4 ks + lane/16]
    // first degree with a nonzero weight in this column group: chunks below it have zero
    // outputs and issue no products (their partials are zero)
    int glmin = 1 << 30;
    {
        const int s0 = (g * 64) / (2 * B), s1 = min(NS - 1, (min(g * 64 + 63, ncols - 1)) / (2 * B));
        for (int s = s0; s <= s1; ++s) glmin = min(glmin, a.lmin[s]);
    }
    // one chunk; LIVE: with the matrix-core products
    auto chunk_body = [&](int lb, auto LIVE) {
        // scale factors of the previous chunk's output, stored after this chunk's first 8 k steps
        // (degree clamped to [0, L): on the first chunk there is no previous output)
        const int lq = lb - 16 + rli;
        const int lr = lq < 0 ? 0 : (lq < L ? lq : L - 1);
        const double s0 = Srow[lr], w0 = wrow[lr];
        wave_lds_sync();               // this wave's d rows of the chunk are written
        f4 pacc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pacc[j] = f4{0, 0, 0, 0};
        // k steps 0..7, with the sum of the previous chunk's partials (read even on the first
        // chunk, where the result is not stored), then its store
        double v = 0.0;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            if constexpr (decltype(LIVE)::value) {
                const float av = Da[68 * ks];
#pragma unroll
                for (int j = 0; j < 4; ++j) pacc[j] = mfma16(av, hb[ks][j], pacc[j]);
            }
            v += (double)Pr[(2 * ks) * TS_RS];
            v += (double)Pr[(2 * ks + 1) * TS_RS];
            // keeps each k step's partial reads beside its products (hoisting all of them
            // ahead would cost 16 registers at the 128-register budget)
            __builtin_amdgcn_sched_barrier(0);
        }
        if (lb > l0) {
            const int l = lb - 16 + rli;
            if (l < L && rok) orow[(size_t)l * 2] = v * (s0 * w0);
        }
        float av[4];
        if constexpr (decltype(LIVE)::value) {
            // k steps 8..11
#pragma unroll
            for (int ks = 8; ks < 12; ++ks) {
                const float a8 = Da[68 * ks];
#pragma unroll
                for (int j = 0; j < 4; ++j) pacc[j] = mfma16(a8, hb[ks][j], pacc[j]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) av[q] = Da[68 * (q + 12)];
        }
        wave_lds_sync();               // all A operands read: the rows may be overwritten
        // k steps 12..15, with the recursion of the next chunk
#pragma unroll
        for (int ks = 12; ks < 16; ++ks) {
            if constexpr (decltype(LIVE)::value) {
#pragma unroll
                for (int j = 0; j < 4; ++j) pacc[j] = mfma16(av[ks - 12], hb[ks][j], pacc[j]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) rstep(lb + 16, 4 * (ks - 12) + i);
        }
        __syncthreads();               // every wave has summed the previous partials
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) Pw[(16 * j + (lane & 15)) * 17 + 4 * (lane >> 4) + r] = pacc[j][r];
        __syncthreads();               // this chunk's partials are visible
    };
    // the chunks below the support come first: two loops, each with its own body
    int lb = l0;
    for (; lb < L && lb + 16 <= glmin; lb += 16) chunk_body(lb, std::integral_constant<bool, false>());
    for (; lb < L; lb += 16) chunk_body(lb, std::integral_constant<bool, true>());
    if (l0 < L) {
        const int lb = l0 + ((L - 1 - l0) & ~15);  // the last chunk
        const int l = lb + rli;
        const double sc = Srow[l < L ? l : L - 1] * wrow[l < L ? l : L - 1];
        double v = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) v += (double)Pr[ww * TS_RS];
        if (l < L && rok) orow[(size_t)l * 2] = v * sc;
    }
    tsum_zero_head(a, in, m, ni, g, l0 < L ? l0 : L, ncols);
}

// ----------------------------------------------------------- k_lsum_bf3 ----
// The mixed l-contraction on BF16 matrix cores.  Same work split and output as
// k_lsum_mm (unit = (m, n, 64 columns), W waves per block each owning a 64-theta tile,
// the block sharing one staged coefficient tile per chunk), with d and the coefficients
// split into three BF16 parts (x0 + x1 + x2 = x to 2^-27 |x|, from the FP32 value) and
// contracted as x0 y0 + x0 y1 + x1 y0 + x0 y2 + x2 y0 + x1 y1 on 32x32x16 BF16 MFMA
// with FP32 accumulation, 16 degrees per chunk: 6 x 32 matrix-core cycles per 32 x 32
// tile and chunk where the FP32 16x16x4 form takes 4 x 4 x 32.  A wave's 64 x 64 output
// is 2 x 2 tiles of 32 x 32.  d parts are written by each lane to its own row of the
// wave's LDS slice ([theta][l], 16 degrees + 8 of padding, so that a lane's 8 degrees
// of one row are a 16-byte read and the 8 lanes served together hit distinct banks);
// the wave reads its A operands into registers before the recursion of the next chunk
// overwrites the slice.  The coefficient tile [column][l] is split as it is staged and
// double-buffered across the block (one barrier per chunk).  Chunks that lie below the
// filter support of every scale in the column group (zero coefficients) issue no
// products; the recursion runs through them.  Operand layout of the 32x32x16 BF16
// instruction: A lane l holds row l % 32 and 8 consecutive k of block l / 32, B the same
// k for column l % 32; result register r of lane l is column l % 32, row
// 8 (r / 4) + 4 (l / 32) + r % 4 (checked on the device).

typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int LB_RS = 24;              // bf16 per LDS row (16 degrees + padding)
constexpr int LB_SLICE = 3 * 64 * LB_RS;   // bf16 per wave slice (three parts of 64 rows)

__device__ __forceinline__ void bsplit(float x, __bf16 &p0, __bf16 &p1, __bf16 &p2)
{
    p0 = (__bf16)x;
    const float r1 = x - (float)p0;
    p1 = (__bf16)r1;
    p2 = (__bf16)(r1 - (float)p1);
}

__device__ __forceinline__ f16v mfma32(const bf16x8 &a, const bf16x8 &b, const f16v &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// One unit (m, n index ni, column group g) on the theta block tb: the body of the
// l-contraction, shared by the per-group launch (k_lsum_bf3) and the persistent launch over
// a work list (k_lsum_bf3_list).  Dp, Up: the block's d slices and coefficient buffers;
// lsab: the dynamic LDS of the coefficient row (sized for the largest band limit).
template <int W>
__device__ __forceinline__ void lsum_bf3_unit(const LsumArgs &a, const MixOut &o, const int NS, const int m,
                                              const int ni, const int g, const int tb, __bf16 *Dp,
                                              __bf16 (*Up)[3 * 64 * LB_RS], double2 *lsab)
{
    constexpr int R = 4 / W;           // staging slots per thread
    const int L = a.L;
    const int B = o.B, ncols = 2 * B * NS;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int n = a.nval[ni], ng = a.nglob[ni];
    const int an = n < 0 ? -n : n;
    const int l0 = m > an ? m : an;
    const int th = (tb * W + w) * 64 + lane;
    const bool valid = th < L;
    // first degree with a nonzero coefficient in this column group
    int glmin = 1 << 30;
    {
        const int s0 = (g * 64) / (2 * B), s1 = min(NS - 1, (min(g * 64 + 63, ncols - 1)) / (2 * B));
        for (int s = s0; s <= s1; ++s) glmin = min(glmin, a.lmin[s]);
    }

    double *lss = reinterpret_cast<double *>(lsab + L + LS_CPAD);   // (A_l, B_l), then S_l

    const size_t tabm = ((size_t)ng * a.Lrec + m) * a.Lrec;
    for (int l = l0 + tid; l < L + LS_CPAD; l += 64 * W) {
        double2 v = {0.0, 0.0};
        double sv = 0.0;
        if (l < L) {
            v.x = a.A[tabm + l];
            v.y = a.B[tabm + l];
            sv = a.S[tabm + l];
        }
        lsab[l] = v;
        lss[l] = sv;
    }
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

    // staging: slot q = tid + 64 W r of the 32 column pairs x 8 degree pairs of a chunk is
    // column pair p = q / 8 (re, im of one map and scale), degrees lb + iq, lb + iq + 1
    int iq[R], pc[R];
    bool cok[R];
    const double *wv[R];
    const double2 *fl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = tid + 64 * W * r;
        pc[r] = q >> 3;
        iq[r] = (q & 7) * 2;
        const int cg = g * 64 + 2 * pc[r];
        cok[r] = cg < ncols;
        int cs = 0, cb = 0;
        if (cok[r]) {
            cs = cg / (2 * B);
            cb = (cg - cs * 2 * B) >> 1;
        }
        wv[r] = a.w[cs < NS ? cs : 0] + (size_t)ni * a.wstride;
        fl[r] = reinterpret_cast<const double2 *>(a.flm) + ((size_t)cb * a.flm_m + m) * a.flm_l + ni * a.flm_nstride;
    }
    double2 f0[R], f1[R];
    double w0[R], w1[R];
    auto fetch = [&](int lb) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int la = lb + iq[r];
            f0[r] = make_double2(0.0, 0.0);
            f1[r] = make_double2(0.0, 0.0);
            w0[r] = 0.0;
            w1[r] = 0.0;
            if (cok[r] && la < L) { f0[r] = fl[r][la]; w0[r] = wv[r][la]; }
            if (cok[r] && la + 1 < L) { f1[r] = fl[r][la + 1]; w1[r] = wv[r][la + 1]; }
        }
    };
    // the (re, im) columns of a slot at two degrees, split into parts: U[part][col][l]
    auto stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            __bf16 re0[3], re1[3], im0[3], im1[3];
            bsplit((float)(w0[r] * f0[r].x), re0[0], re0[1], re0[2]);
            bsplit((float)(w1[r] * f1[r].x), re1[0], re1[1], re1[2]);
            bsplit((float)(w0[r] * f0[r].y), im0[0], im0[1], im0[2]);
            bsplit((float)(w1[r] * f1[r].y), im1[0], im1[1], im1[2]);
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                __bf16 *u = &Up[buf][(p * 64 + 2 * pc[r]) * LB_RS + iq[r]];
                typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
                bf16x2 vr, vi;
                vr[0] = re0[p];
                vr[1] = re1[p];
                vi[0] = im0[p];
                vi[1] = im1[p];
                *reinterpret_cast<bf16x2 *>(u) = vr;
                *reinterpret_cast<bf16x2 *>(u + LB_RS) = vi;
            }
        }
    };
    // recursion over the 16 degrees of the chunk at lc; d parts into this lane's rows
    __bf16 *Dme = Dp + w * LB_SLICE + lane * LB_RS;
    bf16x8 dq[3];
    auto rstep = [&](int lc, int i) {
        const double2 ab = lsab[lc + i];
        const double S = lss[lc + i];
        const float x = (valid && k == 0) ? (float)(S * e) : 0.f;
        __bf16 q0, q1, q2;
        bsplit(x, q0, q1, q2);
        dq[0][i & 7] = q0;
        dq[1][i & 7] = q1;
        dq[2][i & 7] = q2;
        if ((i & 7) == 7) {
#pragma unroll
            for (int p = 0; p < 3; ++p) *reinterpret_cast<bf16x8 *>(Dme + p * 64 * LB_RS + (i & 8)) = dq[p];
        }
        const double en = fma(fma(ab.x, cl, fma(ab.x, c, -ab.y)), e, -ep);
        ep = e;
        e = en;
        if ((i & 7) == 7 && k < 0 && fabs(e) > 0x1p256) {
            e *= 0x1p-512;
            ep *= 0x1p-512;
            k += 1;
        }
    };

    f16v acc[2][2], acc2[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc[i][j][r] = 0.f;
                acc2[i][j][r] = 0.f;
            }
        }

    if (l0 < L) fetch(l0);
    __syncthreads();                   // coefficient row staged
    if (l0 < L) {
        stage(0);
        if (l0 + 16 < L) fetch(l0 + 16);
#pragma unroll
        for (int i = 0; i < 16; ++i) rstep(l0, i);
    }
    __syncthreads();
    // fragment offsets: A row (theta) lane % 32 of tile i, B row (column) lane % 32 of tile j;
    // 8 degrees from 8 (lane / 32)
    const int fo = (lane & 31) * LB_RS + (lane >> 5) * 8;
    const __bf16 *Dw = Dp + w * LB_SLICE;
    int chunk = 0;
    for (int lb = l0; lb < L; lb += 16, ++chunk) {
        const int cb = chunk & 1, nb = cb ^ 1;
        const bool nxt = lb + 16 < L;
        const bool live = lb + 16 > glmin;   // some coefficient of the chunk is nonzero
        // A operands (this wave's d rows) are all read before the next chunk's recursion
        // overwrites the rows; B operands are read per column tile (the other coefficient
        // buffer is the one restaged during this chunk)
        bf16x8 af[2][3];
        if (live) {
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    af[t][p] = *reinterpret_cast<const bf16x8 *>(Dw + p * 64 * LB_RS + t * 32 * LB_RS + fo);
        }
        wave_lds_sync();               // this wave's d rows are read: the next chunk may overwrite them
        if (nxt) {
            stage(nb);
            if (lb + 32 < L) fetch(lb + 32);
        }
        if (live) {
            // per column tile: six products per row tile (small terms first), four steps of the
            // next chunk's recursion after each row tile's products
            constexpr int PA[6] = {1, 0, 2, 0, 1, 0}, PB[6] = {1, 2, 0, 1, 0, 0};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                bf16x8 bfr[3];
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    bfr[p] = *reinterpret_cast<const bf16x8 *>(&Up[cb][(p * 64 + j * 32) * LB_RS + fo]);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
#pragma unroll
                    for (int q = 0; q < 6; ++q) acc[i][j] = mfma32(af[i][PA[q]], bfr[PB[q]], acc[i][j]);
                    if (nxt) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) rstep(lb + 16, 4 * (2 * j + i) + r);
                    }
                }
            }
        } else if (nxt) {
#pragma unroll
            for (int i = 0; i < 16; ++i) rstep(lb + 16, i);
        }
        __syncthreads();
        if ((chunk & 3) == 3) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc2[i][j] += acc[i][j];
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
                }
        }
    }
    // output: one 32-column tile at a time through this wave's slice ([col][theta], rows of
    // 65 floats), then (re, im) pairs written with theta contiguous
    float *St = reinterpret_cast<float *>(Dp + w * LB_SLICE);   // 32 x 65 floats fit the slice
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                St[(lane & 31) * 65 + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)] = acc2[i][j][r] + acc[i][j][r];
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int cgp = g * 64 + 32 * j + 2 * q;
            if (cgp < ncols && valid) {
                const int s = cgp / (2 * B);
                const int b = (cgp - s * 2 * B) >> 1;
                float2 *dst = reinterpret_cast<float2 *>(o.out[s]);
                dst[(((size_t)b * a.nn + ni) * a.mcount + m) * L + th] =
                    make_float2(St[(2 * q) * 65 + lane], St[(2 * q + 1) * 65 + lane]);
            }
        }
        wave_lds_sync();
    }
}

template <int NS, int W>
__global__ __launch_bounds__(64 * W, 2) void k_lsum_bf3(const LsumArgs a, const MixOut o)
{
    __shared__ __align__(16) __bf16 Dp[W * LB_SLICE];       // per wave: [part][theta][l]
    __shared__ __align__(16) __bf16 Up[2][3 * 64 * LB_RS];  // per buffer: [part][column][l]
    extern __shared__ double2 lsab[];
    const int ntt = (a.L + 63) >> 6;
    const int ntb = (ntt + W - 1) / W;
    const int ngrp = (2 * o.B * NS + 63) >> 6;
    const int nunit = a.mcount * a.nn * ngrp;
    // XCD-aware order: the ntb theta blocks of one unit get consecutive slots on one XCD
    const int bid = blockIdx.x, xcd = bid & 7, kx = bid >> 3;
    const int tb = kx % ntb, unit = (kx / ntb) * 8 + xcd;
    if (unit >= nunit) return;
    const int m = unit % a.mcount, ni = (unit / a.mcount) % a.nn, g = unit / (a.mcount * a.nn);
    lsum_bf3_unit<W>(a, o, NS, m, ni, g, tb, Dp, Up, lsab);
}

// Persistent l-contraction over every degree group of a transform: one launch of
// about two blocks per CU, each taking work items (group, m, n, column group, theta block)
// from the list of its XCD (blocks are dispatched to the eight XCDs in turn) through an
// atomic counter.  Each list is sorted by decreasing cost (degrees L_j - max(m, |n|)), so
// the cheap items of every group fill the end of the launch, and all theta blocks of a
// unit are on one list (their coefficient rows are read through one L2).  The counters
// are zero at launch (k_zero_counters).
template <int W>
__global__ __launch_bounds__(64 * W, 2) void k_lsum_bf3_list(const LsumList gl, const uint2 *__restrict__ items,
                                                             unsigned *counters)
{
    __shared__ __align__(16) __bf16 Dp[W * LB_SLICE];
    __shared__ __align__(16) __bf16 Up[2][3 * 64 * LB_RS];
    __shared__ int item_sh;
    extern __shared__ double2 lsab[];
    const int x = blockIdx.x & 7;
    for (;;) {
        if (threadIdx.x == 0) item_sh = (int)atomicAdd(&counters[x], 1u);
        __syncthreads();               // the previous item is finished by every wave
        const int i = item_sh;
        __syncthreads();               // every thread has read the item index
        if (i >= gl.cnt[x]) break;
        const uint2 it = items[gl.off[x] + i];
        const int gi = it.x & 15, ni = (it.x >> 4) & 15, tb = (it.x >> 8) & 255, g = it.x >> 16, m = (int)it.y;
        lsum_bf3_unit<W>(gl.a[gi], gl.o[gi], gl.NS[gi], m, ni, g, tb, Dp, Up, lsab);
    }
}

__global__ void k_zero_counters(unsigned *c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

// ------------------------------------------------------------- launchers ---

void launch_lsum_bf3(const LsumArgs &a, const MixOut &o, int NS, hipStream_t st)
{
    const int ntt = (a.L + 63) / 64;
    const int W = (a.tileW == 2 || ntt < 4) ? 2 : 4;
    const int ntb = (ntt + W - 1) / W;
    const int ngrp = (2 * o.B * NS + 63) / 64;
    const long nunit = (long)a.mcount * a.nn * ngrp;
    dim3 grid((unsigned)(8L * ntb * ((nunit + 7) / 8)));
    const dim3 blk(64 * W);
    const size_t smem = (sizeof(double2) + sizeof(double)) * (size_t)(a.L + LS_CPAD);
    if (NS == 1) {
        if (W == 2) hipLaunchKernelGGL((k_lsum_bf3<1, 2>), grid, blk, smem, st, a, o);
        else hipLaunchKernelGGL((k_lsum_bf3<1, 4>), grid, blk, smem, st, a, o);
    } else {
        if (W == 2) hipLaunchKernelGGL((k_lsum_bf3<2, 2>), grid, blk, smem, st, a, o);
        else hipLaunchKernelGGL((k_lsum_bf3<2, 4>), grid, blk, smem, st, a, o);
    }
}

void launch_lsum_list(const LsumList &gl, const uint2 *items, unsigned *counters, int nblocks, hipStream_t st)
{
    int Lmax = 0;
    for (int i = 0; i < gl.ngroups; ++i) Lmax = std::max(Lmax, gl.a[i].L);
    const size_t smem = (sizeof(double2) + sizeof(double)) * (size_t)(Lmax + LS_CPAD);
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, counters, 8);
    hipLaunchKernelGGL(k_lsum_bf3_list<4>, dim3((unsigned)nblocks), dim3(256), smem, st, gl, items, counters);
}

void launch_lsum_mm(const LsumArgs &a, const MixOut &o, int NS, hipStream_t st)
{
    if (a.L >= 64) {
        launch_lsum_bf3(a, o, NS, st);
        return;
    }
    const int ntt = (a.L + 63) / 64;
    int W = a.tileW == 1 || a.tileW == 2 || a.tileW == 4 ? a.tileW : 4;
    if (W > ntt) W = ntt < 2 ? 1 : (ntt < 4 ? 2 : 4);
    const int ntb = (ntt + W - 1) / W;
    const int ngrp = (2 * o.B * NS + 63) / 64;
    const long nunit = (long)a.mcount * a.nn * ngrp;
    dim3 grid((unsigned)(8L * ntb * ((nunit + 7) / 8)));
    const dim3 blk(64 * W);
    // coefficient row: 24.6 KB at L = 1024
    const size_t smem = (sizeof(double2) + sizeof(double)) * (size_t)(a.L + LS_CPAD);
    if (NS == 1) {
        if (W == 1) hipLaunchKernelGGL((k_lsum_mm<1, 1>), grid, blk, smem, st, a, o);
        else if (W == 2) hipLaunchKernelGGL((k_lsum_mm<1, 2>), grid, blk, smem, st, a, o);
        else hipLaunchKernelGGL((k_lsum_mm<1, 4>), grid, blk, smem, st, a, o);
    } else {
        if (W == 1) hipLaunchKernelGGL((k_lsum_mm<2, 1>), grid, blk, smem, st, a, o);
        else if (W == 2) hipLaunchKernelGGL((k_lsum_mm<2, 2>), grid, blk, smem, st, a, o);
        else hipLaunchKernelGGL((k_lsum_mm<2, 4>), grid, blk, smem, st, a, o);
    }
}

void launch_tsum_mm(const TsumArgs &a, const MixIn &in, int NS, hipStream_t st)
{
    const int NW = (a.L + 63) / 64;
    const int ngrp = (2 * in.B * NS + 63) / 64;
    dim3 grid(a.mcount, a.nn, ngrp);
    if (NW == 16) {
        // 156 KB: coefficient row 16.9 KB + d rows 69.6 KB + partials 69.6 KB
        const size_t smem = sizeof(double2) * (size_t)(a.L + TS16_CPAD) + sizeof(float) * 2 * TS_RS * 16;
        if (NS == 1) hipLaunchKernelGGL(k_tsum_mm16<1>, grid, dim3(1024), smem, st, a, in, a.A, a.B_);
        else hipLaunchKernelGGL(k_tsum_mm16<2>, grid, dim3(1024), smem, st, a, in, a.A, a.B_);
    } else {
        const size_t smem = sizeof(double2) * (size_t)(a.L + TS_CPAD) + sizeof(float) * 2 * TS_RS * (size_t)NW;
        if (NS == 1) hipLaunchKernelGGL(k_tsum_mm<1>, grid, dim3(64 * NW), smem, st, a, in, a.A, a.B_);
        else hipLaunchKernelGGL(k_tsum_mm<2>, grid, dim3(64 * NW), smem, st, a, in, a.A, a.B_);
    }
}

// ------------------------------------------------------------ k_dft_mm -----
// FP32 odd-length DFTs of the mixed path on matrix cores.  Same prime-factor
// order as the FP64 kernels (input index (m1 n2 + m2 n1) mod n at LDS position
// m1 n2 + m2; output frequency (a1 e1 + a2 e2) mod n at a1 n2 + a2), R row pairs
// per block iteration, two real rows per complex row.  Each length-p stage pairs
// k with p-k (u_k = x_k + x_{p-k}, u_0 = x_0, v_k = x_k - x_{p-k}) and forms, as
// dense products on 16x16x4 FP32 MFMA,
//   A = C u,  B = S v,  C[j][k] = cos(2 pi jk/p),  S[j][k] = sin(2 pi jk/p),  0 <= j, k <= h,
// then X_j = A_j + i sgn B_j and X_{p-j} = A_j - i sgn B_j (h = (p-1)/2).  A wave
// takes 16 whole sequences at a time, their real and imaginary parts as two MFMA
// column tiles fed by the same 8-byte LDS reads, so the combination above happens
// within each lane; the wave that reads a sequence is the one that overwrites it,
// so each stage works in place.  C and S come from a per-plan table already in
// A-operand lane order and stay in registers for all the row groups a block takes
// (blocks loop over row groups); MT, KS bound the stage's j tiles and k steps.

// copy a stage's fragment table (MT x KS x 64 lanes of (cos, sin)) into LDS
template <int MT, int KS>
__device__ __forceinline__ void dft_frag_load(const float *tab, float2 *F)
{
    const float2 *t = reinterpret_cast<const float2 *>(tab);
    for (int e = threadIdx.x; e < MT * KS * 64; e += blockDim.x) {
        const int i = e / (KS * 64), r = e - i * KS * 64, s = r >> 6, lane = r & 63;
        F[e] = t[((size_t)i * DFT_FRAG_KS + s) * 64 + lane];
    }
}

template <int MT, int KS>
__device__ __forceinline__ void dft_mm_stage(float2 *Z, const float2 *F, int n, int R, int p, int q,
                                             int sj, int sc, float sgn)
{
    if (p == 1) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int h = (p - 1) / 2, mt = (h + 16) / 16;
    const int nseq = R * q, ngrp = (nseq + 15) >> 4;
    for (int gi = w; gi < ngrp; gi += nw) {
        const int sq = 16 * gi + (lane & 15);
        const bool ok = sq < nseq;
        const int s = ok ? sq / q : 0;
        const int c = ok ? sq - s * q : 0;
        const int base = s * n + c * sc;    // element k of this lane's sequence at base + k sj
        f4 aR[MT], aI[MT], bR[MT], bI[MT];
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            aR[i] = f4{0.f, 0.f, 0.f, 0.f};
            aI[i] = f4{0.f, 0.f, 0.f, 0.f};
            bR[i] = f4{0.f, 0.f, 0.f, 0.f};
            bI[i] = f4{0.f, 0.f, 0.f, 0.f};
        }
        // every k step and j tile up to KS, MT is issued (no branch around the products, so the
        // accumulators stay in place): fragments and u, v are zero beyond j, k <= h
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int k = 4 * st + (lane >> 4);
            float2 u = make_float2(0.f, 0.f), v = make_float2(0.f, 0.f);
            if (ok && k <= h) {
                const float2 x1 = Z[base + k * sj];
                if (k == 0) {
                    u = x1;
                } else {
                    const float2 x2 = Z[base + (p - k) * sj];
                    u = make_float2(x1.x + x2.x, x1.y + x2.y);
                    v = make_float2(x1.x - x2.x, x1.y - x2.y);
                }
            }
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const float2 f = F[(i * KS + st) * 64 + lane];   // (cos, sin) A-operand fragment
                aR[i] = mfma16(f.x, u.x, aR[i]);
                aI[i] = mfma16(f.x, u.y, aI[i]);
                bR[i] = mfma16(f.y, v.x, bR[i]);
                bI[i] = mfma16(f.y, v.y, bI[i]);
            }
        }
        // register r of tile i: j = 16 i + 4 (lane / 16) + r for this lane's sequence
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            if (i >= mt) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * i + 4 * (lane >> 4) + r;
                if (ok && j <= h) {
                    const float ar = aR[i][r], ai = aI[i][r], br = bR[i][r], bi = bI[i][r];
                    Z[base + j * sj] = make_float2(ar - sgn * bi, ai + sgn * br);
                    if (j > 0) Z[base + (p - j) * sj] = make_float2(ar + sgn * bi, ai - sgn * br);
                }
            }
        }
    }
}

// c2r (DIR = +1): Hermitian rows E (m < Lh, complex FP32) -> real rows of length n.
// r2c (DIR = -1): real rows (Tin) -> X_m = scale sum_a x(a) e^{-2 pi i m a/n}, m < Lh.
// N1C, N2C, RC: the factors n1, n2 and the row pairs per block when fixed at compile time
// (then every index map, stride and stage bound folds to constants), else 0
template <int DIR, typename Tin, int MT1, int KS1, int MT2, int KS2, int N1C = 0, int N2C = 0, int RC = 0>
__global__ __launch_bounds__(256, 3) void k_dft_mm(const DftArgs a)
{
    extern __shared__ __align__(16) unsigned char dmm_smem[];
    float2 *Z = reinterpret_cast<float2 *>(dmm_smem);
    const int n1 = N1C > 0 ? N1C : a.n1, n2 = N2C > 0 ? N2C : a.n2;
    const int n = N1C > 0 ? N1C * N2C : a.n, Lh = (n + 1) / 2, R = RC > 0 ? RC : a.rpb;
    const int tid = threadIdx.x, NT = blockDim.x;
    float2 *F1 = Z + (size_t)R * n, *F2 = F1 + MT1 * KS1 * 64;
    dft_frag_load<MT1, KS1>(a.frag1, F1);
    dft_frag_load<MT2, KS2>(a.frag2, F2);
    // index maps stepped in registers (tid + NT t for t = 0, 1, ...): input index x sits at
    // position m1 n2 + m2 (m1 = x n2^-1 mod n1, m2 = x n1^-1 mod n2); output frequency k
    // at (k mod n1) n2 + (k mod n2); -x has the negated residues
    const int d1 = (int)((long)NT * a.inv21 % n1), d2 = (int)((long)NT * a.inv12 % n2);
    const int e1 = NT % n1, e2 = NT % n2;
    const int m1t = (int)((long)tid * a.inv21 % n1), m2t = (int)((long)tid * a.inv12 % n2);
    const int k1t = tid % n1, k2t = tid % n2;
    const long npairs = (a.nrows + 1) / 2, ngroups = (npairs + R - 1) / R;
    constexpr int U = 4;
    // With the sizes fixed at compile time (256 threads), the next row group's input is
    // fetched into registers while the current group runs its two stages, so the global
    // loads overlap the matrix-core work (block barriers wait on LDS only).
    constexpr bool PF = N1C > 0 && RC > 0;
    constexpr int NTC = 256, NC = N1C * N2C;
    constexpr int NP = PF ? ((DIR > 0 ? (NC + 1) / 2 : NC) + U * NTC - 1) / (U * NTC) : 1;
    constexpr int RP = PF ? RC : 1;
    typedef typename std::conditional<(DIR > 0), float2, Tin>::type PT;
    PT pf1[NP][RP][U], pf2[NP][RP][U];
    auto fetch = [&](long grp) {
        const long pair0 = grp * RP;
#pragma unroll
        for (int ps = 0; ps < NP; ++ps)
#pragma unroll
            for (int s = 0; s < RP; ++s) {
                const long r1 = 2 * (pair0 + s);
                const PT *in1 = reinterpret_cast<const PT *>(a.in) + r1 * a.istride;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = ps * U * NTC + tid + NTC * u;
                    PT z1{}, z2{};
                    if (e < (DIR > 0 ? (NC + 1) / 2 : NC) && r1 < a.nrows) {
                        z1 = in1[e];
                        if (r1 + 1 < a.nrows) z2 = in1[a.istride + e];
                    }
                    pf1[ps][s][u] = z1;
                    pf2[ps][s][u] = z2;
                }
            }
    };
    if constexpr (PF) {
        if ((long)blockIdx.x < ngroups) fetch(blockIdx.x);
    }
    for (long grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const long pair0 = grp * R;
        if constexpr (PF) {
            // scatter the fetched group into prime-factor order, then fetch the next one
            int m1 = m1t, m2 = m2t;
#pragma unroll
            for (int ps = 0; ps < NP; ++ps) {
                int pos[U], posc[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    pos[u] = m1 * n2 + m2;
                    posc[u] = (m1 == 0 ? 0 : n1 - m1) * n2 + (m2 == 0 ? 0 : n2 - m2);
                    m1 += d1;
                    if (m1 >= n1) m1 -= n1;
                    m2 += d2;
                    if (m2 >= n2) m2 -= n2;
                }
#pragma unroll
                for (int s = 0; s < RP; ++s) {
                    float2 *Zs = Z + (size_t)s * n;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int e = ps * U * NTC + tid + NTC * u;
                        if constexpr (DIR > 0) {
                            if (e >= Lh) continue;
                            const float sc = (float)a.scale;
                            const float2 z1 = pf1[ps][s][u], z2 = pf2[ps][s][u];
                            if (e == 0) {
                                Zs[0] = make_float2(sc * z1.x, sc * z2.x);
                            } else {
                                Zs[pos[u]] = make_float2(sc * (z1.x - z2.y), sc * (z1.y + z2.x));
                                Zs[posc[u]] = make_float2(sc * (z1.x + z2.y), sc * (z2.x - z1.y));
                            }
                        } else {
                            if (e < n) Zs[pos[u]] = make_float2((float)pf1[ps][s][u], (float)pf2[ps][s][u]);
                        }
                    }
                }
            }
            if (grp + gridDim.x < ngroups) fetch(grp + gridDim.x);
        } else if (DIR > 0) {
            const float sc = (float)a.scale;
            int m1 = m1t, m2 = m2t;
            for (int mb = 0; mb < Lh; mb += U * NT) {
                int pos[U], posc[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    pos[u] = m1 * n2 + m2;
                    posc[u] = (m1 == 0 ? 0 : n1 - m1) * n2 + (m2 == 0 ? 0 : n2 - m2);
                    m1 += d1;
                    if (m1 >= n1) m1 -= n1;
                    m2 += d2;
                    if (m2 >= n2) m2 -= n2;
                }
                for (int s = 0; s < R; ++s) {
                    const long r1 = 2 * (pair0 + s);
                    const float2 *in1 = reinterpret_cast<const float2 *>(a.in) + r1 * a.istride;
                    float2 z1[U], z2[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int mm = mb + tid + NT * u;
                        z1[u] = make_float2(0.f, 0.f);
                        z2[u] = make_float2(0.f, 0.f);
                        if (mm < Lh && r1 < a.nrows) {
                            z1[u] = in1[mm];
                            if (r1 + 1 < a.nrows) z2[u] = in1[a.istride + mm];
                        }
                    }
                    float2 *Zs = Z + (size_t)s * n;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int mm = mb + tid + NT * u;
                        if (mm >= Lh) continue;
                        if (mm == 0) {
                            Zs[0] = make_float2(sc * z1[u].x, sc * z2[u].x);
                        } else {
                            Zs[pos[u]] = make_float2(sc * (z1[u].x - z2[u].y), sc * (z1[u].y + z2[u].x));
                            Zs[posc[u]] = make_float2(sc * (z1[u].x + z2[u].y), sc * (z2[u].x - z1[u].y));
                        }
                    }
                }
            }
        } else {
            int m1 = m1t, m2 = m2t;
            for (int xb = 0; xb < n; xb += U * NT) {
                int pos[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    pos[u] = m1 * n2 + m2;
                    m1 += d1;
                    if (m1 >= n1) m1 -= n1;
                    m2 += d2;
                    if (m2 >= n2) m2 -= n2;
                }
                for (int s = 0; s < R; ++s) {
                    const long r1 = 2 * (pair0 + s);
                    const Tin *x = reinterpret_cast<const Tin *>(a.in) + r1 * a.istride;
                    float x1[U], x2[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int xi = xb + tid + NT * u;
                        x1[u] = 0.f;
                        x2[u] = 0.f;
                        if (xi < n && r1 < a.nrows) {
                            x1[u] = (float)x[xi];
                            if (r1 + 1 < a.nrows) x2[u] = (float)x[a.istride + xi];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (xb + tid + NT * u < n) Z[(size_t)s * n + pos[u]] = make_float2(x1[u], x2[u]);
                }
            }
        }
        __syncthreads();
        const float sgn = DIR > 0 ? 1.f : -1.f;
        dft_mm_stage<MT1, KS1>(Z, F1, n, R, n1, n2, n2, 1, sgn);
        __syncthreads();
        dft_mm_stage<MT2, KS2>(Z, F2, n, R, n2, n1, 1, n2, sgn);
        __syncthreads();
        int k1 = k1t, k2 = k2t;
        if (DIR > 0) {
            for (int ab = 0; ab < n; ab += U * NT) {
                int pos[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    pos[u] = k1 * n2 + k2;
                    k1 += e1;
                    if (k1 >= n1) k1 -= n1;
                    k2 += e2;
                    if (k2 >= n2) k2 -= n2;
                }
                for (int s = 0; s < R; ++s) {
                    const long r1 = 2 * (pair0 + s);
                    if (r1 >= a.nrows) break;
                    float *o1 = reinterpret_cast<float *>(a.out) + r1 * a.ostride;
                    const float2 *Zs = Z + (size_t)s * n;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int aa = ab + tid + NT * u;
                        if (aa >= n) continue;
                        const float2 z = Zs[pos[u]];
                        o1[aa] = z.x;
                        if (r1 + 1 < a.nrows) o1[a.ostride + aa] = z.y;
                    }
                }
            }
        } else {
            const float hs = (float)(0.5 * a.scale);
            for (int mb = 0; mb < Lh; mb += U * NT) {
                int pos[U], posc[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    pos[u] = k1 * n2 + k2;
                    posc[u] = (k1 == 0 ? 0 : n1 - k1) * n2 + (k2 == 0 ? 0 : n2 - k2);
                    k1 += e1;
                    if (k1 >= n1) k1 -= n1;
                    k2 += e2;
                    if (k2 >= n2) k2 -= n2;
                }
                for (int s = 0; s < R; ++s) {
                    const long r1 = 2 * (pair0 + s);
                    if (r1 >= a.nrows) break;
                    const float2 *Zs = Z + (size_t)s * n;
                    float2 *O = reinterpret_cast<float2 *>(a.out) + r1 * a.ostride;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int mm = mb + tid + NT * u;
                        if (mm >= Lh) continue;
                        const float2 X = Zs[pos[u]];
                        const float2 Xc = Zs[posc[u]];
                        O[mm] = make_float2(hs * (X.x + Xc.x), hs * (X.y - Xc.y));
                        if (r1 + 1 < a.nrows) O[a.ostride + mm] = make_float2(hs * (X.y + Xc.y), -hs * (X.x - Xc.x));
                    }
                }
            }
        }
        __syncthreads();   // the next group's loads overwrite Z
    }
}

// Matrix-core DFT usable for this length: both prime-factor lengths within the
// fragment tables (p <= 95), which the plan builds for FP32 plans.
bool dft_mm_ok(const DftArgs &a) { return a.n1 <= 95 && a.n2 <= 95 && a.n >= 15 && a.frag1 && a.frag2; }

// tile shape (j tiles MT, 4-deep k steps KS) of a stage of length p: MT = ceil((h+1)/16),
// KS = ceil((h+1)/4), h = (p - 1) / 2; the class bounds (1, 4), (2, 8), (3, 12) cover any p <= 95
static void dft_shape(int p, int &mt, int &ks)
{
    const int h = (p - 1) / 2;
    mt = (h + 16) / 16;
    ks = (h + 4) / 4;
}

template <int DIR, int MT1, int KS1, int MT2, int KS2>
static void launch_dft_mm_t(DftArgs a, hipStream_t st)
{
    // row pairs per block iteration: LDS for them and the two fragment tables within 54 KB,
    // so that three blocks fit on a compute unit
    const size_t frag = (size_t)(MT1 * KS1 + MT2 * KS2) * 64 * sizeof(float2);
    int R = 1;
    while (R < 8 && (size_t)(2 * R) * a.n * sizeof(float2) + frag <= 55296) R *= 2;
    a.rpb = R;
    const size_t lds = (size_t)R * a.n * sizeof(float2) + frag;
    const long ngroups = ((a.nrows + 1) / 2 + R - 1) / R;
    // blocks loop over row groups: enough for every CU several times over
    const int blocks = (int)std::min<long>(ngroups, 2048);
    // 2047 = 23 x 89 (L = 1024, the two top scales) with all sizes as constants
    constexpr bool top = MT1 == 1 && KS1 == 3 && MT2 == 3 && KS2 == 12;
    if constexpr (top) if (a.n1 == 23 && a.n2 == 89 && R == 2) {
        if (DIR > 0) hipLaunchKernelGGL((k_dft_mm<1, float, MT1, KS1, MT2, KS2, 23, 89, 2>), dim3(blocks), dim3(256), lds, st, a);
        else hipLaunchKernelGGL((k_dft_mm<-1, float, MT1, KS1, MT2, KS2, 23, 89, 2>), dim3(blocks), dim3(256), lds, st, a);
        return;
    }
    // 1023 = 31 x 33 (L = 512)
    constexpr bool l512 = MT1 == 1 && KS1 == 4 && MT2 == 2 && KS2 == 5;
    if constexpr (l512) if (a.n1 == 31 && a.n2 == 33 && R == 4) {
        if (DIR > 0) hipLaunchKernelGGL((k_dft_mm<1, float, MT1, KS1, MT2, KS2, 31, 33, 4>), dim3(blocks), dim3(256), lds, st, a);
        else hipLaunchKernelGGL((k_dft_mm<-1, float, MT1, KS1, MT2, KS2, 31, 33, 4>), dim3(blocks), dim3(256), lds, st, a);
        return;
    }
    if (DIR > 0) hipLaunchKernelGGL((k_dft_mm<1, float, MT1, KS1, MT2, KS2>), dim3(blocks), dim3(256), lds, st, a);
    else hipLaunchKernelGGL((k_dft_mm<-1, float, MT1, KS1, MT2, KS2>), dim3(blocks), dim3(256), lds, st, a);
}

template <int DIR>
static void launch_dft_mm_dir(DftArgs a, hipStream_t st)
{
    if (a.nrows <= 0) return;
    int m1, k1, m2, k2;
    dft_shape(a.n1, m1, k1);
    dft_shape(a.n2, m2, k2);
    const auto is = [&](int a1, int b1, int a2, int b2) { return m1 == a1 && k1 == b1 && m2 == a2 && k2 == b2; };
    // exact shapes of the lengths 2L - 1 for L = 1024, 512, 256, 128, 32 (23 89, 31 33, 7 73, 15 17, 7 9)
    if (is(1, 3, 3, 12)) launch_dft_mm_t<DIR, 1, 3, 3, 12>(a, st);
    else if (is(1, 4, 2, 5)) launch_dft_mm_t<DIR, 1, 4, 2, 5>(a, st);
    else if (is(1, 1, 3, 10)) launch_dft_mm_t<DIR, 1, 1, 3, 10>(a, st);
    else if (is(1, 2, 1, 3)) launch_dft_mm_t<DIR, 1, 2, 1, 3>(a, st);
    else if (is(1, 1, 1, 2)) launch_dft_mm_t<DIR, 1, 1, 1, 2>(a, st);
    else {
        // any other shape within the class bounds (products beyond h add zeros)
        const int c1 = m1 - 1, c2 = m2 - 1;
        switch (3 * c1 + c2) {
        case 0: launch_dft_mm_t<DIR, 1, 4, 1, 4>(a, st); break;
        case 1: launch_dft_mm_t<DIR, 1, 4, 2, 8>(a, st); break;
        case 2: launch_dft_mm_t<DIR, 1, 4, 3, 12>(a, st); break;
        case 3: launch_dft_mm_t<DIR, 2, 8, 1, 4>(a, st); break;
        case 4: launch_dft_mm_t<DIR, 2, 8, 2, 8>(a, st); break;
        case 5: launch_dft_mm_t<DIR, 2, 8, 3, 12>(a, st); break;
        case 6: launch_dft_mm_t<DIR, 3, 12, 1, 4>(a, st); break;
        case 7: launch_dft_mm_t<DIR, 3, 12, 2, 8>(a, st); break;
        default: launch_dft_mm_t<DIR, 3, 12, 3, 12>(a, st); break;
        }
    }
}

// ------------------------------------------------------- k_gemm_bf3 -------
// C[M][N] = sum_k A[M][k] Bt[N][k] (FP32 in, FP32 out) on BF16 matrix cores.  Every
// operand is split into three BF16 parts x = x0 + x1 + x2, each the round-to-nearest
// BF16 value of what the previous parts leave (exact FP32 differences), so that
// |x - x0 - x1 - x2| <= 2^-27 |x|; the products x0 y0 + x0 y1 + x1 y0 + x0 y2 + x2 y0 +
// x1 y1 are exact in FP32 and accumulate in FP32 on 16x16x32 BF16 MFMA (the omitted
// terms x1 y2, x2 y1, x2 y2 are below 2^-26 of a product).  Bt comes pre-split (three
// [N][K] BF16 matrices); A is split as it is staged.  Six 16x16x32 BF16 products take
// 96 matrix-core cycles where the FP32 product of the same 16x16x32 tile takes 256.
//
// Workgroup tile 128 x 128, four waves of 64 x 64 (4 x 4 tiles of 16 x 16); K in slices
// of 32 through one LDS buffer per part ([row][k] with rows of 40 BF16, k contiguous, so
// that a lane's 8 consecutive k of one row are a 16-byte read and the 8 lanes served
// together hit distinct banks); the next slice is fetched into registers while the
// current one feeds the matrix cores; two workgroups per CU (60 KB of LDS each).  A
// fragment lane holds row lane % 16 and 8 consecutive k from 8 (lane / 16); the B
// fragment pairs the same k with column lane % 16, so the product sums over every k of
// the slice whatever order the instruction takes them in; result register r of a lane
// is row 4 (lane / 16) + r, column lane % 16.  XCD-aware tile order as in k_gemm.
// Requires K % 8 == 0 (whole 16-byte vectors along k); rows and columns are bounded.

constexpr int G3_BM = 128, G3_BN = 128, G3_BK = 32, G3_RS = 40;

// three BF16 parts of four FP32 values
__device__ __forceinline__ void split3(const float4 &x, bf16x4 &p0, bf16x4 &p1, bf16x4 &p2)
{
    const float v[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const __bf16 a = (__bf16)v[e];
        const float r1 = v[e] - (float)a;
        const __bf16 b = (__bf16)r1;
        const float r2 = r1 - (float)b;
        p0[e] = a;
        p1[e] = b;
        p2[e] = (__bf16)r2;
    }
}

__global__ __launch_bounds__(256, 2) void k_gemm_bf3(const float *__restrict__ A, const __bf16 *__restrict__ B0,
                                                     const __bf16 *__restrict__ B1, const __bf16 *__restrict__ B2,
                                                     float *__restrict__ C, int M, int N, int K, int mt, int nt)
{
    __shared__ __align__(16) __bf16 As[3][G3_BM * G3_RS];
    __shared__ __align__(16) __bf16 Bs[3][G3_BN * G3_RS];
    const int bid = blockIdx.x, kx = bid >> 3;
    const int mtile = (bid & 7) + 8 * (kx / nt), ntile = kx % nt;
    if (mtile >= mt) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row0 = mtile * G3_BM, col0 = ntile * G3_BN;
    const __bf16 *Bp[3] = {B0, B1, B2};
    // staging: A 128 rows x 8 float4 (thread: rows tid / 8 + 32 r, float4 tid % 8);
    // B per part 128 rows x 4 vectors of 8 BF16 (thread: rows tid / 4 + 64 r, vector tid % 4)
    const int aq = tid & 7, ar = tid >> 3;
    const int bq = tid & 3, br = tid >> 2;
    float4 ra[4];
    bf16x8 rb[3][2];
    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gr = row0 + ar + 32 * r, gk = k0 + aq * 4;
            ra[r] = (gr < M && gk < K) ? *reinterpret_cast<const float4 *>(A + (size_t)gr * K + gk)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int gn = col0 + br + 64 * r, gk = k0 + bq * 8;
                if (gn < N && gk < K) rb[p][r] = *reinterpret_cast<const bf16x8 *>(Bp[p] + (size_t)gn * K + gk);
                else
#pragma unroll
                    for (int e = 0; e < 8; ++e) rb[p][r][e] = (__bf16)0.f;
            }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bf16x4 p0, p1, p2;
            split3(ra[r], p0, p1, p2);
            const int o = (ar + 32 * r) * G3_RS + aq * 4;
            *reinterpret_cast<bf16x4 *>(&As[0][o]) = p0;
            *reinterpret_cast<bf16x4 *>(&As[1][o]) = p1;
            *reinterpret_cast<bf16x4 *>(&As[2][o]) = p2;
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = 0; r < 2; ++r)
                *reinterpret_cast<bf16x8 *>(&Bs[p][(br + 64 * r) * G3_RS + bq * 8]) = rb[p][r];
    };
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0, 0, 0, 0};
    const int nk = (K + G3_BK - 1) / G3_BK;
    const int fo = (lane & 15) * G3_RS + (lane >> 4) * 8;   // this lane's fragment offset in a 16-row tile
    gload(0);
    for (int t = 0; t < nk; ++t) {
        __syncthreads();               // the previous slice's fragment reads are done
        sstore();
        __syncthreads();
        if (t + 1 < nk) gload((t + 1) * G3_BK);
        bf16x8 bf[3][4];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bf[p][j] = *reinterpret_cast<const bf16x8 *>(&Bs[p][(wc * 64 + j * 16) * G3_RS + fo]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bf16x8 af[3];
#pragma unroll
            for (int p = 0; p < 3; ++p)
                af[p] = *reinterpret_cast<const bf16x8 *>(&As[p][(wr * 64 + i * 16) * G3_RS + fo]);
            // small terms first; consecutive products go to the four independent accumulators
            constexpr int PA[6] = {1, 0, 2, 0, 1, 0}, PB[6] = {1, 2, 0, 1, 0, 0};
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[PA[q]], bf[PB[q]][j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gr = row0 + wr * 64 + i * 16 + 4 * (lane >> 4) + r;
                const int gc = col0 + wc * 64 + j * 16 + (lane & 15);
                if (gr < M && gc < N) C[(size_t)gr * N + gc] = acc[i][j][r];
            }
}

// ------------------------------------------------------- k_tsum_tab -------
// Precompute mode of the mixed synthesis: the theta quadrature T_sigma and the theta
// contraction with d^l_mn fold into one table, Dt^l_mn(theta) = sum_theta' d^l_mn(theta')
// T_sigma[theta][theta'] (T_sigma is symmetric), so that
//   out[col][l] = w_l sum_theta F[col][theta] Dt^l_mn(theta)
// with F the rows before the quadrature.  One (m, n) problem is a product of its columns
// (2 x maps x scales) by its L - max(m, |n|) table rows over the L theta samples, run
// with the tiling, operand split and product order of k_gemm_bf3 (F split as it is
// staged, the table stored as three BF16 parts).  Tiles (128 columns x 128 degrees) come
// from eight per-XCD lists in which the tiles of one problem are consecutive, so that the
// column tiles sharing the table rows of a degree tile run back to back on one XCD.
// Result register r of a lane holds column 4 (lane / 16) + r: registers (0, 1) and (2, 3)
// are the real and imaginary parts of one map, written as one 16-byte (re, im) pair.
__global__ __launch_bounds__(256, 2) void k_tsum_tab(const TsumTab a)
{
    __shared__ __align__(16) __bf16 As[3][G3_BM * G3_RS];
    __shared__ __align__(16) __bf16 Bs[3][G3_BN * G3_RS];
    const int xc = blockIdx.x & 7, kx = blockIdx.x >> 3;
    if (kx >= a.cnt[xc]) return;
    const int4 tl = a.tiles[a.off[xc] + kx];
    const int m = tl.x, ni = tl.y;
    const int L = a.L, B = a.B, ncols = 2 * B * a.NS;
    const int n = a.nval[ni], an = n < 0 ? -n : n, l0 = m > an ? m : an;
    const int rows = L - l0;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int row0 = tl.z * G3_BM, col0 = tl.w * G3_BN;   // column rows of F, degree rows of the table
    const int sig = (m + a.npar) & 1, mp = m >> 1;
    const size_t sigoff = sig == 0 ? 0 : (size_t)B * a.M0 * a.nn * 2;
    const int Msig = sig == 0 ? a.M0 : a.M1;
    const int aq = tid & 7, ar = tid >> 3;
    const int bq = tid & 3, br = tid >> 2;
    const float *arow[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int cg = row0 + ar + 32 * r;
        arow[r] = nullptr;
        if (cg < ncols) {
            const int s = cg / (2 * B), rem = cg - s * 2 * B;
            arow[r] = a.h[s] + (sigoff + (((size_t)(rem >> 1) * Msig + mp) * a.nn + ni) * 2 + (rem & 1)) * L;
        }
    }
    const __bf16 *tb = reinterpret_cast<const __bf16 *>(a.tab) + a.toff[(size_t)ni * a.mcount + m];
    const size_t pstride = (size_t)rows * L;
    float4 ra[4];
    bf16x8 rb[3][2];
    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gk = k0 + aq * 4;
            ra[r] = (arow[r] && gk < L) ? *reinterpret_cast<const float4 *>(arow[r] + gk) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int gn = col0 + br + 64 * r, gk = k0 + bq * 8;
                if (gn < rows && gk < L) rb[p][r] = *reinterpret_cast<const bf16x8 *>(tb + p * pstride + (size_t)gn * L + gk);
                else
#pragma unroll
                    for (int e = 0; e < 8; ++e) rb[p][r][e] = (__bf16)0.f;
            }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bf16x4 p0, p1, p2;
            split3(ra[r], p0, p1, p2);
            const int o = (ar + 32 * r) * G3_RS + aq * 4;
            *reinterpret_cast<bf16x4 *>(&As[0][o]) = p0;
            *reinterpret_cast<bf16x4 *>(&As[1][o]) = p1;
            *reinterpret_cast<bf16x4 *>(&As[2][o]) = p2;
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = 0; r < 2; ++r)
                *reinterpret_cast<bf16x8 *>(&Bs[p][(br + 64 * r) * G3_RS + bq * 8]) = rb[p][r];
    };
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0, 0, 0, 0};
    const int nk = (L + G3_BK - 1) / G3_BK;
    const int fo = (lane & 15) * G3_RS + (lane >> 4) * 8;
    gload(0);
    for (int t = 0; t < nk; ++t) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (t + 1 < nk) gload((t + 1) * G3_BK);
        bf16x8 bf[3][4];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bf[p][j] = *reinterpret_cast<const bf16x8 *>(&Bs[p][(wc * 64 + j * 16) * G3_RS + fo]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bf16x8 af[3];
#pragma unroll
            for (int p = 0; p < 3; ++p)
                af[p] = *reinterpret_cast<const bf16x8 *>(&As[p][(wr * 64 + i * 16) * G3_RS + fo]);
            constexpr int PA[6] = {1, 0, 2, 0, 1, 0}, PB[6] = {1, 2, 0, 1, 0, 0};
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[PA[q]], bf[PB[q]][j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int lr = col0 + wc * 64 + j * 16 + (lane & 15);
            if (lr >= rows) continue;
            const int l = l0 + lr;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cg = row0 + wr * 64 + i * 16 + 4 * (lane >> 4) + 2 * h;   // even: the real part
                if (cg >= ncols) continue;
                const int s = cg / (2 * B), b = (cg - s * 2 * B) >> 1;
                const double wt = a.w[s][(size_t)ni * a.wstride + l];
                float2 *o = reinterpret_cast<float2 *>(a.out[s]) + (((size_t)b * a.mcount + m) * a.nn + ni) * L + l;
                *o = make_float2((float)((double)acc[i][j][2 * h] * wt), (float)((double)acc[i][j][2 * h + 1] * wt));
            }
        }
    // m <= l < l0: zero (d^l_mn vanishes below max(|m|, |n|)); the first degree tile's blocks
    if (tl.w == 0 && l0 > m) {
        for (int e = tid; e < 64 * (l0 - m); e += 256) {
            const int pr = e / (l0 - m), l = m + e - pr * (l0 - m);
            const int cg = row0 + 2 * pr;
            if (cg >= ncols) continue;
            const int s = cg / (2 * B), b = (cg - s * 2 * B) >> 1;
            reinterpret_cast<float2 *>(a.out[s])[(((size_t)b * a.mcount + m) * a.nn + ni) * L + l] = make_float2(0.f, 0.f);
        }
    }
}

void launch_tsum_tab(const TsumTab &a, hipStream_t st)
{
    int mx = 0;
    for (int x = 0; x < 8; ++x) mx = std::max(mx, a.cnt[x]);
    if (mx == 0) return;
    hipLaunchKernelGGL(k_tsum_tab, dim3(8u * (unsigned)mx), dim3(256), 0, st, a);
}

__global__ void k_split3_f64(const double *__restrict__ in, __bf16 *__restrict__ out, size_t count)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const double x = in[i];
        const __bf16 p0 = (__bf16)(float)x;
        const double r1 = x - (double)(float)p0;
        const __bf16 p1 = (__bf16)(float)r1;
        const double r2 = r1 - (double)(float)p1;
        out[i] = p0;
        out[count + i] = p1;
        out[2 * count + i] = (__bf16)(float)r2;
    }
}

void launch_split3_f64(const double *in, uint16_t *out, size_t count, hipStream_t st)
{
    if (count == 0) return;
    const unsigned blocks = (unsigned)std::min<size_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(k_split3_f64, dim3(blocks), dim3(256), 0, st, in, reinterpret_cast<__bf16 *>(out), count);
}

bool gemm_bf3_ok(int K) { return K % 8 == 0; }

void launch_gemm_bf3(const float *A, const void *B0, const void *B1, const void *B2, float *C, int M, int N, int K,
                     hipStream_t st)
{
    if (M <= 0 || N <= 0) return;
    const int mt = (M + G3_BM - 1) / G3_BM, nt = (N + G3_BN - 1) / G3_BN;
    const unsigned blocks = 8u * (unsigned)nt * (unsigned)((mt + 7) / 8);
    hipLaunchKernelGGL(k_gemm_bf3, dim3(blocks), dim3(256), 0, st, A, (const __bf16 *)B0, (const __bf16 *)B1,
                       (const __bf16 *)B2, C, M, N, K, mt, nt);
}

void launch_dft_mm_c2r(DftArgs a, hipStream_t st) { launch_dft_mm_dir<1>(a, st); }

void launch_dft_mm_r2c(DftArgs a, hipStream_t st) { launch_dft_mm_dir<-1>(a, st); }

}  // namespace s2w
