// Kernel argument blocks and launchers shared by the s2w entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace s2w {

constexpr int MAX_NS = 2;        // scales sharing one recursion pass
constexpr int MAX_NN = 8;        // azimuthal orders per launch
constexpr int GAMMA_MAXN = 8;

// sum over l (lanes own theta)
struct LsumArgs {
    int L;                       // grid band limit (theta samples, l < L)
    int mcount;                  // m = 0..mcount-1
    int nn;                      // number of n values
    int Lrec;                    // leading size of the recursion tables
    int nval[MAX_NN], nglob[MAX_NN];
    const double *A, *B, *S;     // [NG][Lrec][Lrec]
    const double *smant;         // [NG][Lrec]
    const int *sexp;
    const double *cth, *ctl, *ch, *sh, *ceps, *seps;   // [L]; cos(theta) = cth + ctl
    const double *pol;           // d at the 2 npol samples next to the poles [NG][L][2 npol][L]
    int npol;
    const double *flm;           // [B][flm_m][flm_l] complex
    int flm_m, flm_l;
    long flm_nstride;            // complex elements between the coefficient rows of consecutive n
                                 // indices (0: one row per m shared by every n)
    const double *w[MAX_NS];     // weights [nn][wstride] (wstride 0: shared by all n)
    int wstride;
    double *out[MAX_NS];         // [B][nn][mcount][L] complex
    int tileT;                   // theta samples per lane of k_lsum (1, 2, 4, 8; 0: default)
    int tileW;                   // waves per block of k_lsum_mm (1, 2, 4; 0: default)
    int lmin[MAX_NS];            // mixed kernels: first degree of each scale's filter support (the
                                 // weights are zero below it; 0 when unknown)
    const double *dtab;          // precompute mode (FP64 vector kernels): d^l_mn(theta) of this grid,
    const int64_t *doff;         // row l0 of (n, m) at dtab + doff[nglob L + m]; nullptr: recursion
};

// sum over theta (reduction across lanes)
struct TsumArgs {
    int L, mcount, nn, Lrec, B;
    int nval[MAX_NN], nglob[MAX_NN];
    const double *A, *B_, *S;
    const double *smant;
    const int *sexp;
    const double *cth, *ctl, *ch, *sh, *ceps, *seps;   // [L]; cos(theta) = cth + ctl
    const double *pol;           // d at the 2 npol samples next to the poles [NG][L][2 npol][L]
    int npol;
    int npar;                    // parity of n in this launch: sigma index = (m + npar) & 1
    int M0, M1;                  // number of m with sigma index 0 / 1
    int lmin[MAX_NS];            // mixed kernels: first degree of each scale's filter support (the
                                 // weights are zero below it; 0 when unknown)
    const double *dtab;          // precompute mode, as in LsumArgs
    const int64_t *doff;
    const double *h[MAX_NS];     // rows [sig][b][m'][ni][c][L]
    const double *w[MAX_NS];
    int wstride;
    double *out[MAX_NS];         // [B][mcount][nn][L] complex
};

struct DftArgs {
    const void *in;
    void *out;
    long istride, ostride;       // in elements of the row type (complex or real)
    int nrows;
    int n, n1, n2;
    const int *pin;              // input index held at LDS position p (prime-factor order)
    const int *pout;             // output frequency held at LDS position p after both stages
    const int *inpos;            // LDS position of input index i
    const int *outpos;           // LDS position holding output frequency k
    const double *w1, *w2;       // cos, sin of 2 pi k / n1 and 2 pi k / n2
    double scale;
    int rpb;                     // row pairs per block (set by the launcher)
    int inplace;                 // stages overwrite their input (set by the launcher)
    int inv21, inv12;            // n2^-1 mod n1 and n1^-1 mod n2 (0 for a factor of 1)
    const float *frag1, *frag2;  // matrix-core DFT: cos, sin of 2 pi j k / p of the stage over n1 (n2) in
                                 // MFMA A-operand lane order, [DFT_FRAG_MT][DFT_FRAG_KS][64][2] (FP32 plans)
};

constexpr int DFT_FRAG_MT = 3, DFT_FRAG_KS = 12;   // 16-row tiles of j and 4-deep k steps (p <= 95)

struct GammaArgs {
    const void *src;
    void *dst;
    int B, M, L;                 // maps, m count, theta count
    int Min, Mout;               // row lengths (m) of the rows over m
    int nn, ng;                  // n values, gamma samples (2N-1)
    int nval[GAMMA_MAXN];
    const double *tw;            // cos/sin of 2 pi k / ng, k < ng
    double sgn;                  // +1: e^{+i n g}, -1: e^{-i n g}
    double phr, phi;             // complex phase factor
    double wscale;               // real scale factor
    double fm0, fm1;             // r2c side: factor for m = 0 and m >= 1
    int npar, M0, M1;            // sigma grouping on the r2c side
};

struct CombineTerm {
    const void *P;               // [B][L][nn][L] complex, read at l >= m only
    int L, nn;
    int f32;                     // P holds FP32 values (else FP64)
    double phr, phi;
};

struct CombineArgs {
    double *out;                 // [B][L][L] complex
    int L;
    int nterms;
    CombineTerm t[24];
};

// mixed-precision batched contractions
struct MixOut {
    int B;
    float *out[MAX_NS];          // [B][nn][mcount][L] complex FP32
};
struct MixIn {
    int B;
    const float *h[MAX_NS];      // sigma-grouped rows, FP32
    double *out[MAX_NS];         // [B][mcount][nn][L] complex FP64, defined for l >= m
};
void launch_lsum_mm(const LsumArgs &a, const MixOut &o, int NS, hipStream_t st);

// persistent mixed l-contraction over several degree groups (band limit >= 64, 4 waves per
// block): per group its arguments, outputs and scale count; work items in eight per-XCD
// lists (cnt[x] items from off[x]), each item (x: group | n index << 4 | theta block << 8 |
// column group << 16, y: m)
constexpr int MAX_LGROUPS = 8;
struct LsumList {
    int ngroups;
    int NS[MAX_LGROUPS];
    int cnt[8], off[8];
    LsumArgs a[MAX_LGROUPS];
    MixOut o[MAX_LGROUPS];
};
void launch_lsum_list(const LsumList &gl, const uint2 *items, unsigned *counters, int nblocks, hipStream_t st);
void launch_tsum_mm(const TsumArgs &a, const MixIn &in, int NS, hipStream_t st);
// precompute mode, mixed plans: the theta contraction of the synthesis through a table of
// (d T_sigma)^l_mn(theta) in three BF16 parts, as a batched product over (m, n) problems
struct TsumTab {
    int L, mcount, nn, B, NS, npar, M0, M1;
    int nval[MAX_NN];
    const float *h[MAX_NS];      // sigma-grouped rows before the theta quadrature, FP32
    float *out[MAX_NS];          // [B][mcount][nn][L] complex FP32 (the products accumulate in FP32)
    const double *w[MAX_NS];     // filter weights [nn][wstride]
    int wstride;
    const uint16_t *tab;         // per (n index, m): three BF16 parts, each [L - l0][L]
    const int64_t *toff;         // [nn][mcount]: offset of the first part
    const int4 *tiles;           // (m, n index, column tile, degree tile) in eight per-XCD lists
    int cnt[8], off[8];
};
void launch_tsum_tab(const TsumTab &a, hipStream_t st);
// precompute mode, forward SHT in FP64: f_lm = w_l sum_theta F_m(theta) Dt^l_m(theta) with the
// folded table Dt^l_m = d^l_m0 T_sigma (per m: rows l = m..L-1, theta contiguous), batched over m
struct ShtTab {
    int L, B, M0, M1;
    const double *F;             // sigma-grouped rows before the quadrature (n = 0)
    double *out;                 // internal flm [B][L][L] complex
    const double *w;             // sqrt((2l+1)/(4 pi))
    const double *tab;           // per m: [L - m][L]
    const int64_t *toff;         // [L]
    const int4 *tiles;           // (m, column tile, degree tile, 0) in eight per-XCD lists
    int cnt[8], off[8];
};
void launch_sht_tab(const ShtTab &a, hipStream_t st);
// the inverse: rows C_m(theta) = sum_l w_l f_lm d^l_m0(theta) ([B][m][theta] complex) from the
// table of d^l_m0 (per m: [L - m][L]); F is the internal flm, tiles (m, column tile, theta tile)
void launch_shti_tab(const ShtTab &a, hipStream_t st);
// three BF16 parts of FP64 values (x0 + x1 + x2 = x to 2^-27 |x|): part p of element i at
// out[p * count + i]
void launch_split3_f64(const double *in, uint16_t *out, size_t count, hipStream_t st);

void launch_lsum(const LsumArgs &a, int NS, int B, hipStream_t st);
// precompute mode: d table of one grid for the n values of a (nval, nglob), all m < L
void launch_dtable(const LsumArgs &a, double *tab, const int64_t *doff, hipStream_t st);
void launch_tsum(const TsumArgs &a, int NS, int B, hipStream_t st);
void launch_gemm(const double *A, const double *Bm, double *C, int M, int N, int K, hipStream_t st,
                 bool accum = false);
void launch_scale_pl(const double *in, double *out, const double *phi, int P, int L, size_t total, hipStream_t st);
void launch_gemm_f32(const float *A, const float *Bm, float *C, int M, int N, int K, hipStream_t st);
// C[M][N] = A[M][K] Bt[N][K]^T in FP32 on BF16 matrix cores, Bt given as its three BF16
// parts (each [N][K], 16-bit words); needs K % 8 == 0 (gemm_bf3_ok)
bool gemm_bf3_ok(int K);
void launch_gemm_bf3(const float *A, const void *B0, const void *B1, const void *B2, float *C, int M, int N, int K,
                     hipStream_t st);
void launch_dft_c2r(DftArgs a, hipStream_t st, bool f32 = false);
// f32: FP32 arithmetic (in64: FP64 input rows); otherwise FP64 arithmetic (in32: FP32 input rows)
void launch_dft_r2c(DftArgs a, hipStream_t st, bool f32 = false, bool in64 = true, bool in32 = false);
// FP32 DFTs on matrix cores (mixed path); dft_mm_ok tells whether the length is supported
bool dft_mm_ok(const DftArgs &a);
void launch_dft_mm_c2r(DftArgs a, hipStream_t st);
void launch_dft_mm_r2c(DftArgs a, hipStream_t st);
void launch_gamma_c2r(const GammaArgs &a, hipStream_t st, bool f32 = false);
void launch_gamma_r2c(const GammaArgs &a, hipStream_t st, bool f32 = false);
void launch_convert(const void *in, void *out, size_t n, bool to_f32, hipStream_t st);
void launch_combine(const CombineArgs &a, int B, hipStream_t st);
void launch_pack_sigma(const double *in, double *out, int B, int nn, int M, int L, int npar, int M0,
                       int M1, int dir, hipStream_t st);
void launch_pack_sigma_f32(const float *in, float *out, int B, int nn, int M, int L, int npar, int M0,
                           int M1, int dir, hipStream_t st);
void launch_flm_to_ext(const double *in, double *out, int L, int B, hipStream_t st);
void launch_flm_from_ext(const double *in, double *out, int L, int B, hipStream_t st);
// spin-s maps held as real pairs (B = user maps; pairs and cin hold 2B real maps)
void launch_spin_combine(const double *X, double *pairs, double *ext, int L, int s, int B, hipStream_t st);
void launch_spin_split(const double *pairs, const double *ext, double *cin, int L, int s, int B, hipStream_t st);
// SO(3) coefficient layouts: external "nlm" [B][2N-1][L][2L-1] complex (index n+N-1, l, m+L-1)
// <-> internal [B][2N-1][m < L][l < L]; outputs of the theta sum [B][m][nq][l] for the n
// values nval[0..nq) -> external, with the m < 0 entries from the real-function symmetry
void launch_wig_ext_to_int(const double *ext, double *in, int L, int N, int B, hipStream_t st);
void launch_wig_sum_to_ext(const double *P, double *ext, int L, int N, int B, int nq, const int *nval,
                           hipStream_t st);

}  // namespace s2w
