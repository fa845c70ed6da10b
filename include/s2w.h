/*
 * s2w — directional scale-discretised wavelet transform on the sphere S^2
 * (and, through radial shells, the ball B^3) on McEwen-Wiaux sampling,
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: Price, Polanska, Whitney & McEwen, "Differentiable and accelerated
 * directional wavelet transforms on the sphere and ball".
 *   analysis   W^{Psi^j} = D_j^{-1} N Psi^j Y f          (Section 4.1, eq:analysis_s2)
 *              W^Phi = Y^{-1} Phi Y f                    (Section 4.1)
 *   synthesis  f = Y^{-1}(Phi Y W^Phi + sum_j Psi^{j dagger} D_j W^{Psi^j})   (eq:synthesis_s2)
 *   filters    Appendix A (kappa, eta, zeta, Psi, Phi); multiresolution band
 *              limits per scale (Section 3.3).
 *
 * Conventions (all arrays row-major, FP64 unless stated):
 *   map f              [B][L][2L-1]     theta_b = pi(2b+1)/(2L-1), phi_a = 2 pi a/(2L-1)
 *   harmonic flm       [B][L][2L-1]     complex interleaved (re, im), index m+L-1 ("lm" layout
 *                                       of Algorithm 1), zero where |m| > l
 *   wavelet coeffs     scales j = J0..J packed one after another; scale k = j-J0 occupies
 *                      [B][2N_k-1][L_k][2L_k-1] (gamma, beta, alpha) starting at element
 *                      wav_offset[k]; FP64 for S2W_FP64 plans, FP32 for S2W_MIXED plans
 *   scaling coeffs     [B][L_phi][2L_phi-1]
 *   per-scale limits   L_k = min(ceil(lambda^(j+1)), L), N_k = min(N, L_k), L_phi = ceil(lambda^J0),
 *                      J = smallest integer with lambda^J >= L
 *
 * Ownership and asynchrony: the caller owns every input/output device buffer.
 * The plan owns its tables and workspace, all allocated in s2w_plan_create; the
 * transform entry points allocate nothing, never synchronise, and enqueue their
 * work on `stream` (a hipStream_t, or NULL for the default stream).  Argument
 * errors are reported synchronously; device faults surface as S2W_EHIP at a later
 * call.  Calls never abort: failures return a negative status and set a
 * thread-local message readable with s2w_last_error().
 *
 * Streams: the calls on one plan share its workspace, so the library orders them: a call
 * on a stream other than the previous call's waits (on the device) for that call to end.
 * Calls on one stream run in order anyway.  A stream under graph capture is left alone;
 * the capturing program orders the captured work.  A plan is used from one host thread
 * at a time.
 *
 * Allocation failure can be injected for tests of the error paths: with the environment
 * variable S2W_FAIL_ALLOC_AT=k, the k-th device allocation (counting from 1) of each plan
 * creation fails, and the creation returns S2W_ENOMEM having freed what it allocated.
 */
#ifndef S2W_H
#define S2W_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    S2W_OK = 0,
    S2W_EINVAL = -1,        /* invalid argument (sizes, null pointers, plan) */
    S2W_ENOMEM = -2,        /* device or host allocation failed at plan creation */
    S2W_EHIP = -3,          /* HIP runtime error */
    S2W_EUNSUPPORTED = -4,  /* valid but unsupported configuration */
    S2W_ESTATE = -5         /* handle is not a live plan (destroyed, destroyed twice, or never
                               created); a handle whose memory a later plan reuses is that plan */
} s2w_status;

typedef enum {
    S2W_FP64 = 0,           /* FP64 end to end */
    S2W_MIXED = 1           /* FP64 Wigner-d recursion and scale sums; FP32 coefficients */
} s2w_precision;

typedef struct s2w_plan_s *s2w_plan;

/* Plan flags (bitwise or). */
enum {
    S2W_PLAN_TUNE = 1,      /* time the l-contraction tile shapes on the device at creation and
                               keep the fastest per grid (creation then synchronises the device) */
    S2W_PLAN_GRAPH = 2,     /* s2w_analysis / s2w_synthesis capture their launches into a HIP graph
                               on the first call with a given (input, output, output) pointer triple
                               and replay it afterwards (up to 16 triples per plan; kernel timing is
                               not recorded for graph replays) */
    S2W_PLAN_NO_WORKSPACE = 4, /* allocate no workspace (tables only): the plan runs only through
                               s2w_analysis_noalloc; other transform entry points return S2W_ESTATE.
                               Excludes S2W_PLAN_TUNE and S2W_PLAN_GRAPH. */
    S2W_PLAN_PERSISTENT = 8, /* mixed plans: the l-contraction of the analysis runs as one
                               persistent launch over every degree group of band limit >= 64 on
                               matrix cores, its work items (degree group, m, n, column group,
                               theta block) in per-XCD lists sorted by decreasing cost
                               L_j - max(m, |n|) (Section 3.3: the top scales dominate).  With
                               S2W_PLAN_TUNE alone the autotuner chooses between this and one
                               launch per degree group by timing both. */
    S2W_PLAN_WIGNER = 32,   /* recursion tables for every |n| < N (N <= 4) and buffers for the
                               standalone SO(3) transforms (s2w_wigner_*; on ball plans, the
                               Wigner-Laguerre transforms b3w_wl_*) */
    S2W_PLAN_PRECOMPUTE = 16 /* precompute mode (Section 4.2): for every grid of band limit <= 512,
                               Wigner d^l_mn(theta_b) is tabulated in device memory at plan
                               creation (all n of the plan, m < L, l >= max(m, |n|): about
                               N L^3 / 2 doubles per grid, 4.8 GB at L = 512, N = 8) and the FP64
                               vector contractions (FP64 plans below 16 maps, the vector route of
                               mixed plans) read d from it instead of running the recursion.
                               Mixed plans also fold the theta quadrature of the synthesis into a
                               table: for every scale group on a grid with L >= 64 and L % 8 == 0,
                               sum_theta' d^l_mn(theta') T_sigma[theta][theta'] in three BF16
                               parts (3 N L^3 / 2 bytes per grid: 26 GB at L = 1024, N = 8), and
                               the synthesis contracts its rows with it on matrix cores (no
                               quadrature product, no recursion).  The product's tile lists are
                               built for the plan's batch. */
};

/* Size of the static device scratch that s2w_analysis_noalloc works in (one copy per
 * device, held until the process ends). */
#define S2W_SCRATCH_BYTES (64ull << 20)

/* Create a plan for band limit L >= 2, azimuthal band limit 1 <= N <= L, dilation
 * lambda > 1, lowest wavelet scale 0 <= J0 <= J, batch >= 1 maps per call, on HIP
 * device `device`, with flags from S2W_PLAN_*.  Computes filters (Appendix A), the
 * exact MW theta-quadrature matrices, recursion tables and allocates all workspace. */
s2w_status s2w_plan_create(s2w_plan *out, int L, int N, double lambda, int J0, int batch,
                           s2w_precision precision, int device, unsigned flags);

/* Release a plan (NULL is accepted). */
s2w_status s2w_plan_destroy(s2w_plan plan);

/* Query the packed layout.  Any pointer may be NULL.  Arrays Lk, Nk have
 * nscales = J - J0 + 1 entries, wav_offset has nscales + 1 (the last is the total
 * element count per call, all maps included). */
s2w_status s2w_plan_layout(s2w_plan plan, int *nscales, int *J0, int *Lk, int *Nk,
                           int64_t *wav_offset, int *L_phi);

/* Wavelet analysis (Algorithm 1, analysis): real maps f -> wavelet and scaling
 * coefficients.  f: device [B][L][2L-1]; wav: device, packed (see above);
 * scal: device [B][L_phi][2L_phi-1]. */
s2w_status s2w_analysis(s2w_plan plan, const double *f, void *wav, double *scal, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): s2w_analysis with its workspace in a
 * static device array of S2W_SCRATCH_BYTES instead of the plan's own buffers.  It calls no
 * hipMalloc, hipFree or allocating routine; the caller passes inputs and outputs as for
 * s2w_analysis, on any plan (typically one created with S2W_PLAN_NO_WORKSPACE).  Plans
 * whose workspace exceeds the scratch are rejected with S2W_EUNSUPPORTED (the batch-1 FP64
 * plan at L = 256, N = 4 needs about 37 MB; L = 512, N = 8 needs more than 64 MiB).  Every
 * call on a device shares that device's scratch and leaves its contents behind: calls that
 * overlap on one device (on different streams, or host threads) race and must be ordered
 * by the caller.  Runs eagerly (no graph replay). */
s2w_status s2w_analysis_noalloc(s2w_plan plan, const double *f, void *wav, double *scal, void *stream);

/* Wavelet synthesis (Algorithm 1, synthesis): coefficients -> real maps. */
s2w_status s2w_synthesis(s2w_plan plan, const void *wav, const double *scal, double *f, void *stream);

/* Wavelet analysis from harmonic coefficients (Algorithm 1 without its first Y; Section
 * 4.1, eq:wigner_wav_coeffs and eq:harmonic_scal_coeffs): flm -> wavelet and scaling
 * coefficients.  flm: device, complex interleaved [B][L][2L-1] in the "lm" layout above,
 * describing real maps (f_{l,-m} = (-1)^m conj(f_lm)); only the m >= 0 entries are read.
 * wav, scal as for s2w_analysis. */
s2w_status s2w_analysis_lm(s2w_plan plan, const double *flm, void *wav, double *scal, void *stream);

/* Gradients.  The paper differentiates its transforms automatically (Section 4.3, and
 * Section 5.2 for the adjoint transforms the ball library provides); here each transform
 * has a hand-written transpose under the real inner product of the sample arrays (the
 * gradient of a loss with respect to the transform's input, given its gradient with
 * respect to the output).  The transposes recompute Wigner d, never store it, and run in
 * the plan's precision split: FP64 end to end for S2W_FP64 plans; for S2W_MIXED plans the
 * wavelet-coefficient cotangents are FP32 and their contractions and DFTs run on FP32
 * matrix cores with the FP64 recursion, harmonic transforms and scale sums, as in the
 * forward maps.  Buffers and errors as for the forward entry points.
 *
 * s2w_analysis_adjoint: (gwav, gscal) -> gf [B][L][2L-1]: transpose of s2w_analysis.  It
 * is not the synthesis: MW sampling oversamples, so A^T A != I.
 * s2w_synthesis_adjoint: gf -> (gwav, gscal): transpose of s2w_synthesis. */
s2w_status s2w_analysis_adjoint(s2w_plan plan, const void *gwav, const double *gscal, double *gf,
                                void *stream);
s2w_status s2w_synthesis_adjoint(s2w_plan plan, const double *gf, void *gwav, double *gscal,
                                 void *stream);

/* Wigner (SO(3)) transforms of real functions on the plan's MW grid (Section 2.2,
 * eq:forward_wigner_transform and eq:inverse_wigner_transform) at band limits (L, N), FP64
 * for either precision; the plan needs S2W_PLAN_WIGNER (N <= 4, else creation fails with
 * S2W_EUNSUPPORTED), otherwise S2W_ESTATE.  Samples f [B][2N-1][L][2L-1] (gamma, beta, alpha);
 * coefficients flmn complex interleaved [B][2N-1][L][2L-1] in the "nlm" layout of Algorithm 1
 * (index n+N-1, l, m+L-1), zero where |m| > l or |n| > l.  Inputs to s2w_wigner_inverse must
 * describe real functions (f^l_{-m,-n} = (-1)^(m+n) conj(f^l_mn)); only m >= 0 entries are read.
 * The forward transform is exact on MW samples of band-limited functions. */
s2w_status s2w_wigner_forward(s2w_plan plan, const double *f, double *flmn, void *stream);
s2w_status s2w_wigner_inverse(s2w_plan plan, const double *flmn, double *f, void *stream);

/* Spin-0 spherical-harmonic transforms on the plan's grid (Section 2.1,
 * eq:fswsh / eq:iswsh; the S^2 case of the Wigner transforms).  flm is complex
 * interleaved [B][L][2L-1].  Inputs to s2w_sht_inverse must describe real maps
 * (f_{l,-m} = (-1)^m conj(f_lm)); only m >= 0 entries are read. */
s2w_status s2w_sht_forward(s2w_plan plan, const double *f, double *flm, void *stream);
s2w_status s2w_sht_inverse(s2w_plan plan, const double *flm, double *f, void *stream);

/* Complex spin-s maps (Section 2.1, eq:u1sym to eq:iswsh; Section 4.1 with the spin kept:
 * eq:wigner_wav_coeffs, eq:harmonic_scal_coeffs, eq:s2_cont_synthesis).  Spin-weighted
 * harmonics in the convention sY_lm = (-1)^s sqrt((2l+1)/(4 pi)) e^{i m phi} d^l_{m,-s}(theta)
 * (Y_lm at s = 0; 1Y_10 = sqrt(3/(8 pi)) sin theta).  The filters are those of spin 0 (the
 * dictionary's harmonic coefficients carry no spin factor, Appendix A).
 *
 * s2w_plan_create_spin makes a plan for `batch` complex spin-`spin` maps (|spin| < L; spin 0
 * gives complex scalar maps); other arguments as for s2w_plan_create, flags limited to
 * S2W_PLAN_TUNE, S2W_PLAN_PERSISTENT and S2W_PLAN_PRECOMPUTE.  Such a plan runs only the
 * s2w_spin_* calls (the real-map calls return S2W_ESTATE on it, and the s2w_spin_* calls on
 * a real-map plan).  Layouts, B = batch:
 *   f    planar complex [B][2][L][2L-1]: real part, then imaginary part of each map;
 *   flm  complex interleaved [B][L][2L-1] (index m+L-1), zero for l < max(|m|, |spin|);
 *   wav  the packed layout that s2w_plan_layout reports for the plan (2B real maps per
 *        scale): map 2b holds Re W^j, map 2b+1 holds Im W^j of input b;
 *   scal [B][2][L_phi][2L_phi-1]: Re and Im of the (spin-0) scaling map.
 * The wavelet coefficients are linear in the spin-s coefficients g_lm, so with g = A + i B
 * for real maps A and B they are W(A) + i W(B): the plan computes the real transforms of A
 * and B (the same precision split as a real plan) and the spin-s harmonic transforms in
 * FP64.  s2w_spin_synthesis reconstructs f exactly (to rounding) from the coefficients of
 * s2w_spin_analysis for maps band-limited at L.  Device buffers, stream-ordered. */
s2w_status s2w_plan_create_spin(s2w_plan *out, int L, int N, double lambda, int J0, int spin, int batch,
                                s2w_precision precision, int device, unsigned flags);
s2w_status s2w_spin_sht_forward(s2w_plan plan, const double *f, double *flm, void *stream);
s2w_status s2w_spin_sht_inverse(s2w_plan plan, const double *flm, double *f, void *stream);
s2w_status s2w_spin_analysis(s2w_plan plan, const double *f, void *wav, double *scal, void *stream);
s2w_status s2w_spin_synthesis(s2w_plan plan, const void *wav, const double *scal, double *f, void *stream);

/* Kernel timing (for measurement).  s2w_plan_profile(plan, capacity) with capacity > 0
 * creates `capacity` pairs of HIP events and from then on records one pair around
 * every kernel launch of the transform entry points, on the stream of the call, together
 * with the launch's algorithmic work; capacity 0 stops recording and releases the events.
 * Not to be used under graph capture.  Algorithmic work counts what the method needs:
 * 6 FP64 flop per Wigner-d recursion step (theta, l, m, n), once for all maps and scales of
 * a launch; 4 flop per complex-by-real multiply-add of a contraction, per map, only at the
 * degrees inside the scale's filter support; 5 n log2 n per length-n complex DFT (2.5 n
 * log2 n per real row); for the exact MW theta quadrature, its Fourier route per complex
 * column (a DFT of the extended column, the Hankel product with the quadrature weights as
 * a convolution through two FFTs of twice the length, the inverse DFT).  flop64 is the part
 * on the FP64 units in a mixed-precision kernel (the recursion); dense is what a dense
 * product issues in place of a cheaper algorithm (2 flop per multiply-add of the theta-
 * quadrature matrix product; 0 for other kernels).
 * s2w_plan_profile_read synchronises the device, then reports per kernel name (up to `max`
 * names, each at most 31 characters, written to names + 32*i): total milliseconds, launch
 * count, total flop, flop64 and dense since profiling started, and clears the record.  Any
 * output pointer may be NULL.  Launches beyond the capacity are not recorded (dropped
 * reports their number). */
s2w_status s2w_plan_profile(s2w_plan plan, int capacity);
s2w_status s2w_plan_profile_read(s2w_plan plan, int max, char *names, double *total_ms,
                                 int64_t *launches, double *flop, double *flop64, double *dense,
                                 int *count, int64_t *dropped);

/* ---- ball B^3 = R+ x S^2 (Section 3.2, Section 5: eq:forward_ball_wavelet,
 * eq:synthesis_b3; radial Laguerre basis of Section 2.3; filters of Appendix A.3-A.4) ----
 *
 *   analysis   W^{Psi^{jj'}} = Q^{-1} N Psi^{jj'} Z f,   W^Phi = Z^{-1} Phi Z f
 *   synthesis  f = Z^{-1}(Phi Z W^Phi + sum_{jj'} Psi^{jj' dagger} Q W^{jj'})
 *   Psi^{jj'}_lmp = sqrt((2l+1)/(8 pi^2)) kappa_lambda(l/lambda^j) kappa_nu(p/nu^j') zeta_lm,
 *   4pi/(2l+1)|Phi_l0p|^2 = a + b - ab,  a = k_lambda(l/lambda^J0), b = k_nu(p/nu^J0')
 *   (the scaling filter is taken from the admissibility condition of Section 3.2).
 *
 * Radial sampling: P nodes r_k = tau x_k, x_k the roots of the Laguerre polynomial
 * L^{(2)}_P (exact quadrature for radial band limit P, p = 0..P-1).  Radial scale j'
 * (J0' <= j' <= J', J' the smallest integer with nu^J' >= P) has band limit
 * P_j' = min(ceil(nu^(j'+1)), P) and is sampled on the P_j' nodes of its own rule.
 *
 * Layouts (row-major):
 *   map f, scaling coeffs  [B][P][L][2L-1] FP64 on the P radial nodes (shell k = r_k)
 *   wavelet coeffs         blocks (i, k), radial scale i = j'-J0' outer, angular scale
 *                          k = j-J0 inner, block (i, k) = [B][P_j'][2N_k-1][L_k][2L_k-1]
 *                          starting at element wav_offset[i * nang + k]; FP64, or FP32 for
 *                          S2W_MIXED plans (radial stages stay FP64).
 * Ownership, asynchrony and errors as for s2w plans.  Each transform runs the sphere
 * transform of the plan on B P_j' shells at a time (one internal s2w plan). */
typedef struct b3w_plan_s *b3w_plan;

/* Create a ball plan: L >= 2, 1 <= N <= L, P >= 1, lambda > 1, nu > 1, 0 <= J0 <= J,
 * 0 <= J0p <= J', tau > 0, batch >= 1, flags from S2W_PLAN_TUNE, S2W_PLAN_WIGNER.  Errors: S2W_EINVAL,
 * S2W_EUNSUPPORTED (N > 8), S2W_ENOMEM, S2W_EHIP. */
s2w_status b3w_plan_create(b3w_plan *out, int L, int N, int P, double lambda, double nu, int J0,
                           int J0p, double tau, int batch, s2w_precision precision, int device,
                           unsigned flags);
s2w_status b3w_plan_destroy(b3w_plan plan);

/* Layout: nang angular and nrad radial scales; Lk, Nk need J - J0 + 1 entries, Pk
 * J' - J0' + 1, wav_offset nrad * nang + 1 (the last is the total element count),
 * nodes P (radial nodes r_k).  Any output pointer may be NULL. */
s2w_status b3w_plan_layout(b3w_plan plan, int *nang, int *nrad, int *Lk, int *Nk, int *Pk,
                           int64_t *wav_offset, double *nodes);

/* Ball wavelet analysis and synthesis (Algorithm 2; device buffers as laid out above). */
s2w_status b3w_analysis(b3w_plan plan, const double *f, void *wav, double *scal, void *stream);
s2w_status b3w_synthesis(b3w_plan plan, const void *wav, const double *scal, double *f, void *stream);

/* Transposes of b3w_analysis and b3w_synthesis under the real inner product of the
 * sample arrays (the adjoint ball transforms of Section 5.2; gradients as for the sphere
 * entry points above): b3w_analysis_adjoint (gwav, gscal) -> gf, b3w_synthesis_adjoint
 * gf -> (gwav, gscal).  Radial stages FP64; the angular stages in the plan's precision
 * split.  Buffers and errors as for b3w_analysis / b3w_synthesis. */
s2w_status b3w_analysis_adjoint(b3w_plan plan, const void *gwav, const double *gscal, double *gf,
                                void *stream);
s2w_status b3w_synthesis_adjoint(b3w_plan plan, const double *gf, void *gwav, double *gscal,
                                 void *stream);

/* Spherical-Laguerre transform on the plan's grid (Section 2.3, eq:forward_spherical_laguerre
 * and eq:inverse_spherical_laguerre): f on the P radial nodes, [B][P][L][2L-1] FP64, and
 * its coefficients f_lmp, complex interleaved [B][P][L][2L-1] (per p the harmonic layout
 * of s2w_sht_forward).  Both run in FP64 for either precision of the plan.  Inputs to
 * b3w_sl_inverse must describe real maps (f_{l,-m,p} = (-1)^m conj(f_lmp)); only m >= 0
 * entries are read.  Device buffers, stream-ordered; errors as for s2w plans. */
s2w_status b3w_sl_forward(b3w_plan plan, const double *f, double *flmp, void *stream);
s2w_status b3w_sl_inverse(b3w_plan plan, const double *flmp, double *f, void *stream);

/* Wigner-Laguerre transform of real functions on R+ x SO(3), the SO(3) analogue of the ball
 * (Section 2.5: basis Q^l_mnp = K_p D^l_mn, its decomposition and synthesis eq:wiglag_inverse),
 * FP64 for either precision; the ball plan needs S2W_PLAN_WIGNER (else S2W_ESTATE).  Samples f
 * [B][P][2N-1][L][2L-1] on the radial nodes x the MW SO(3) grid; coefficients f^l_mnp complex
 * interleaved [B][P][2N-1][L][2L-1], per p the layout of s2w_wigner_forward.  Inputs to
 * b3w_wl_inverse must describe real functions; only m >= 0 entries are read. */
s2w_status b3w_wl_forward(b3w_plan plan, const double *f, double *flmnp, void *stream);
s2w_status b3w_wl_inverse(b3w_plan plan, const double *flmnp, double *f, void *stream);

/* Kernel timing for ball transforms: as s2w_plan_profile / s2w_plan_profile_read. */
s2w_status b3w_plan_profile(b3w_plan plan, int capacity);
s2w_status b3w_plan_profile_read(b3w_plan plan, int max, char *names, double *total_ms,
                                 int64_t *launches, double *flop, double *flop64, double *dense,
                                 int *count, int64_t *dropped);

/* Message for the last failure on the calling thread. */
const char *s2w_last_error(void);

/* ---- host-only helpers (no device work; used to test the plan arithmetic) ---- */

/* Per-scale band limits for (L, N, lambda, J0).  Lk, Nk need room for J - J0 + 1 entries
 * (J <= 64). */
s2w_status s2w_host_scales(int L, int N, double lambda, int J0, int *nscales, int *Lk, int *Nk,
                           int *L_phi);

/* Wavelet filters Psi^j_ln (complex interleaved, [nscales][L][2N-1], index n+N-1) and
 * scaling filter Phi_l0 ([L]) from Appendix A. */
s2w_status s2w_host_filters(int L, int N, double lambda, int J0, double *psi, double *phi);

/* Exact MW theta-quadrature matrix T_sigma ([L][L], row-major): for F of band limit L
 * with parity F(2pi - t) = sigma F(t) and any d of band limit L with the same parity,
 * int_0^pi F d sin t dt = sum_b d(theta_b) (T_sigma F)(theta_b). sigma = +1 or -1. */
s2w_status s2w_host_theta_matrix(int L, int sigma, double *T);

/* Radial Laguerre rule of the ball (Section 2.3): the P nodes r_k = tau x_k (roots of
 * L^{(2)}_P) and weights W_k with f_p = sum_k W_k K_p(r_k) f(r_k) exact for p < P. */
s2w_status s2w_host_laguerre_rule(int P, double tau, double *nodes, double *weights);

/* Wigner d^l_mn(theta_b) for l = 0..L-1 on the MW grid of band limit L, computed on the
 * host by the same scaled, log-rescaled three-term recursion the device uses
 * (out: [L][L] as out[l*L + b]; zero for l < max(|m|,|n|)).  For tests of the
 * recursion tables. */
s2w_status s2w_host_wigner_d(int L, int m, int n, double *out);

#ifdef __cplusplus
}
#endif

#endif /* S2W_H */
