// C-ABI of the s2w library: plans and transform entry points (see include/s2w.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/s2w.h"
#include "s2w_host.h"
#include "s2w_kern.h"

// Static scratch for s2w_analysis_noalloc: the workspace of a plan created with
// S2W_PLAN_NO_WORKSPACE is carved out of this array, one copy per device, held until
// the process ends.  In host code `scratch` names a host-side stand-in; its device
// address is resolved once per device (hipGetSymbolAddress with that device current, at
// plan creation) and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[S2W_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

s2w_status fail(s2w_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

// Live plan handles.  A handle is looked up here before it is dereferenced, so a
// destroyed (or never created) handle is reported as S2W_ESTATE instead of being
// read.  A handle whose memory was reused by a later plan is indistinguishable
// from that plan.
std::mutex g_reg_mu;
std::unordered_set<const void *> g_live;

void reg_add(const void *h)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_live.insert(h);
}

bool reg_has(const void *h)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    return g_live.count(h) != 0;
}

// removes h; false when it was not live
bool reg_remove(const void *h)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    return g_live.erase(h) != 0;
}

// Injected allocation failure, for tests of the error paths: with S2W_FAIL_ALLOC_AT=k in
// the environment, the k-th device allocation (counting from 1) of a plan creation fails
// as if the device were out of memory.  Counted per creating thread; the sphere plan a
// ball plan creates counts in the ball plan's sequence.
thread_local int g_alloc_depth = 0, g_alloc_seq = 0, g_alloc_fail_at = 0;

struct AllocSeq {
    AllocSeq()
    {
        if (g_alloc_depth++ == 0) {
            g_alloc_seq = 0;
            const char *e = std::getenv("S2W_FAIL_ALLOC_AT");
            g_alloc_fail_at = e ? std::atoi(e) : 0;
        }
    }
    ~AllocSeq() { --g_alloc_depth; }
};

hipError_t dev_malloc(void **v, size_t bytes)
{
    ++g_alloc_seq;
    if (g_alloc_fail_at > 0 && g_alloc_seq == g_alloc_fail_at) return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(v, bytes);
    if (e != hipSuccess) (void)hipGetLastError();   // reported as S2W_ENOMEM, not left for a later call
    return e;
}

// device address of the static scratch per device (resolved at plan creation)
std::mutex g_scr_mu;
std::map<int, unsigned char *> g_scr;

// Resolves the current device's scratch address once; false on failure.
bool scratch_resolve(int device)
{
    std::lock_guard<std::mutex> lk(g_scr_mu);
    auto it = g_scr.find(device);
    if (it != g_scr.end()) return it->second != nullptr;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
    }
    g_scr[device] = (unsigned char *)ptr;
    return ptr != nullptr;
}

unsigned char *scratch_ptr(int device)
{
    std::lock_guard<std::mutex> lk(g_scr_mu);
    auto it = g_scr.find(device);
    return it == g_scr.end() ? nullptr : it->second;
}

struct DevDft {
    int n = 0, n1 = 0, n2 = 0;
    int *pin = nullptr, *pout = nullptr, *inpos = nullptr, *outpos = nullptr;
    double *w1 = nullptr, *w2 = nullptr;
    float *frag1 = nullptr, *frag2 = nullptr;
};

// cos, sin of 2 pi j k / p for the matrix-core DFT stage of length p, laid out as the
// MFMA A operand: entry (i, s, lane) holds j = 16 i + lane % 16, k = 4 s + lane / 16
// (zero outside j, k <= (p - 1) / 2); w holds cos, sin of 2 pi t / p for t < p
std::vector<float> dft_fragments(int p, const std::vector<double> &w)
{
    std::vector<float> f((size_t)s2w::DFT_FRAG_MT * s2w::DFT_FRAG_KS * 64 * 2, 0.0f);
    const int h = (p - 1) / 2;
    for (int i = 0; i < s2w::DFT_FRAG_MT; ++i)
        for (int st = 0; st < s2w::DFT_FRAG_KS; ++st)
            for (int lane = 0; lane < 64; ++lane) {
                const int j = 16 * i + lane % 16, k = 4 * st + lane / 16;
                if (p <= 1 || j > h || k > h) continue;
                const int t = (int)(((long)j * k) % p);
                const size_t o = (((size_t)i * s2w::DFT_FRAG_KS + st) * 64 + lane) * 2;
                f[o] = (float)w[2 * t];
                f[o + 1] = (float)w[2 * t + 1];
            }
    return f;
}

// BF16 bits of f, rounded to nearest (ties to even)
uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// x = x0 + x1 + x2 + O(2^-27 x) in BF16 parts, each the rounding of what the previous leave
void bf16_split3(const std::vector<double> &x, std::vector<uint16_t> (&part)[3])
{
    for (auto &v : part) v.resize(x.size());
    for (size_t i = 0; i < x.size(); ++i) {
        double r = x[i];
        for (int k = 0; k < 3; ++k) {
            part[k][i] = bf16_bits((float)r);
            r -= bf16_value(part[k][i]);
        }
    }
}

struct DevGrid {
    int L = 0;
    double *pol = nullptr;
    int npol = 0;
    double *cth = nullptr, *ctl = nullptr, *ch = nullptr, *sh = nullptr, *ceps = nullptr, *seps = nullptr;
    double *T[2] = {nullptr, nullptr};
    float *T32[2] = {nullptr, nullptr};
    uint16_t *T3[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};   // BF16 parts of T
    DevDft dft;
};

struct Group {
    std::vector<int> scales;   // plan scale indices sharing one grid
    int L = 0;
};

}  // namespace

struct s2w_plan_s {
    int L = 0, N = 0, J0 = 0, J = 0, B = 1, device = 0;
    double lambda = 2.0;
    s2w_precision prec = S2W_FP64;
    s2w::Scales S;
    s2w::Filters F;
    int Lphi = 1;
    std::vector<int64_t> wav_off;
    std::map<int, DevGrid> grids;
    std::map<int, double *> gamma_tw;       // per ng = 2N_k-1
    std::vector<int> nglob;                  // global n values of the recursion tables
    double *A = nullptr, *Bt = nullptr, *S_ = nullptr, *smant = nullptr;
    int *sexp = nullptr;
    std::vector<double *> wpsi;              // per scale [nn][L_k]
    std::vector<int> lmin;                   // per scale: first degree with a nonzero filter weight
    double *wphi = nullptr, *wsht = nullptr;
    double *flm = nullptr, *fhat = nullptr;
    double *bufA = nullptr, *bufB = nullptr, *bufC = nullptr;
    size_t szA = 0, szB = 0, szC = 0;
    // every workspace buffer (its pointer in this plan, size in doubles), in layout order;
    // ws_bytes: their total with each start rounded up to 256 bytes
    std::vector<std::pair<double **, size_t>> ws;
    size_t ws_bytes = 0;
    bool no_ws = false;                      // created with S2W_PLAN_NO_WORKSPACE
    // complex spin-s maps (s2w_plan_create_spin): B counts real maps, two per complex map
    bool cplx = false;
    int spin = 0;
    std::vector<double *> P;                 // per scale [B][L_k][nn][L_k] complex
    double *Pphi = nullptr;
    std::vector<Group> groups;
    std::vector<void *> allocs;
    // kernel timing
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<int> rec_name;
    std::vector<double> rec_flop, rec_flop64, rec_dense;
    std::vector<std::string> prof_names;
    int64_t prof_dropped = 0;
    int prof_cap = 0;
    // tuned tile shapes per grid band limit (S2W_PLAN_TUNE)
    std::map<int, int> tile_lsum, tile_lsum_mm;
    // mixed plans, per grid band limit: contraction route, 1 = FP64 vector kernels with an
    // FP32 conversion at the boundary (fastest for very small batches), 0 = matrix cores
    std::map<int, int> route_lsum, route_tsum;
    // standalone SO(3) (Wigner) transforms, S2W_PLAN_WIGNER: internal coefficients
    // [B][2N-1][L][L], degree weights (2l+1)/(8 pi^2) and ones
    bool wigner = false;
    double *wint = nullptr, *w8pi = nullptr, *wone = nullptr;
    // precompute mode: per grid band limit (<= PRE_MAX_L), the d table and its row offsets
    std::map<int, std::pair<double *, int64_t *>> dtabs;
    // precompute mode of mixed plans: per scale group (index into groups), the BF16 parts of
    // the folded theta quadrature and contraction table, and the tile lists of the product
    struct TTab {
        uint16_t *tab = nullptr;
        int64_t *toff = nullptr;
        int4 *tiles = nullptr;
        int cnt[8] = {0}, off[8] = {0};
        size_t bytes = 0;
    };
    std::map<int, TTab> ttabs;
    // precompute mode, batched plans: the folded forward-SHT table of the full grid (FP64)
    double *shttab = nullptr;
    int64_t *shtoff = nullptr;
    int4 *shttiles = nullptr;
    int shtcnt[8] = {0}, shtoffx[8] = {0};
    // ... and the d^l_m0 table of the inverse SHT (same offsets), with its tile lists
    double *shtitab = nullptr;
    int4 *shtitiles = nullptr;
    int shticnt[8] = {0}, shtioffx[8] = {0};
    // persistent l-contraction of the mixed analysis (one launch over the degree groups in
    // lgroups, work items in eight per-XCD lists sorted by cost); used when lsum_list is set
    // and the batch is the one the list was built for
    bool lsum_list = false;
    int list_B = 0, list_blocks = 0;
    std::vector<int> lgroups;                // indices into groups
    std::vector<size_t> lgroup_off;          // each group's output offset in bufA (floats)
    size_t list_end = 0;                     // end of those outputs: other groups write from here
    uint2 *items = nullptr;
    unsigned *counters = nullptr;
    int list_cnt[8] = {0}, list_off[8] = {0};
    // graph replay (S2W_PLAN_GRAPH)
    bool graph = false, capturing = false;
    hipStream_t cap_stream = nullptr;
    // ordering of calls across streams: recorded at the end of every call
    hipEvent_t order_ev = nullptr;
    hipStream_t order_stream = nullptr;
    bool order_used = false;
    struct GraphEntry {
        int kind;
        const void *a, *b, *c;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
};

struct b3w_plan_s {
    int L = 0, N = 0, P = 0, B = 1, J0 = 0, J0p = 0, Jp = 0;
    double lambda = 2.0, nu = 2.0, tau = 1.0;
    s2w_precision prec = S2W_FP64;
    s2w_plan sp = nullptr;                   // sphere plan over B * P shells
    int nang = 0, nrad = 0;
    std::vector<int> Pj;                     // radial band limit per radial scale
    std::vector<int64_t> wav_off;            // [nrad * nang + 1]
    std::vector<double> nodes;
    double *Zf = nullptr, *Zi = nullptr;     // [P][P]: W_k K_p(r_k) and K_p(r_k) (as [k][p])
    double *Zft = nullptr, *Zit = nullptr;   // their transposes (adjoints)
    double *phi = nullptr;                   // [P][L]: sqrt(4pi/(2l+1)) Phi_l0p
    std::vector<double *> G, H;              // per radial scale: [P_j'][P], [P][P_j']
    std::vector<double *> Gt, Ht;            // their transposes: [P][P_j'], [P_j'][P]
    double *flmp = nullptr, *shell = nullptr, *shell2 = nullptr;
    double *wltmp = nullptr;                 // Wigner-Laguerre transforms: [B][P][2N-1][L][2L-1] complex
    std::vector<void *> allocs;
};

namespace {

using s2w::CombineArgs;
using s2w::DftArgs;
using s2w::GammaArgs;
using s2w::LsumArgs;
using s2w::TsumArgs;

// Algorithmic work of a launch: all floating-point operations the method needs
// (flop), the part of them that runs on the FP64 units in a mixed-precision kernel
// (flop64: the Wigner-d recursion), and the operations of a dense product that stands in
// for a cheaper algorithm (dense: the theta-quadrature matrix product; 0 elsewhere).
struct Work {
    double flop = 0.0, flop64 = 0.0, dense = 0.0;
};

// Orders the calls on one plan across streams.  The calls of a plan share its workspace,
// so a call on a stream other than the previous call's first waits for the end of that
// call (an event recorded at the end of every call).  Skipped on a stream under graph
// capture, where the capturing program orders the work.
struct StreamOrder {
    s2w_plan p;
    hipStream_t st;
    bool on = false;
    StreamOrder(s2w_plan p_, hipStream_t st_) : p(p_), st(st_)
    {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        if (cs != hipStreamCaptureStatusNone) return;
        on = true;
        if (p->order_used && p->order_stream != st) (void)hipStreamWaitEvent(st, p->order_ev, 0);
    }
    ~StreamOrder()
    {
        if (!on) return;
        if (hipEventRecord(p->order_ev, st) == hipSuccess) {
            p->order_stream = st;
            p->order_used = true;
        }
    }
};

// One HIP event pair around a kernel launch when profiling is on.
struct Prof {
    s2w_plan p;
    hipStream_t st;
    int idx = -1;
    Prof(s2w_plan p_, const char *name, double flop, hipStream_t st_) : Prof(p_, name, Work{flop, 0.0, 0.0}, st_) {}
    Prof(s2w_plan p_, const char *name, const Work &wk, hipStream_t st_) : p(p_), st(st_)
    {
        if (p->prof_cap == 0 || p->capturing) return;
        if ((int)p->rec_name.size() >= p->prof_cap) { ++p->prof_dropped; return; }
        int id = -1;
        for (size_t i = 0; i < p->prof_names.size(); ++i)
            if (p->prof_names[i] == name) id = (int)i;
        if (id < 0) { p->prof_names.push_back(name); id = (int)p->prof_names.size() - 1; }
        idx = (int)p->rec_name.size();
        p->rec_name.push_back(id);
        p->rec_flop.push_back(wk.flop);
        p->rec_flop64.push_back(wk.flop64);
        p->rec_dense.push_back(wk.dense);
        (void)hipEventRecord(p->ev0[idx], st);
    }
    ~Prof()
    {
        if (idx >= 0) (void)hipEventRecord(p->ev1[idx], st);
    }
};

// Algorithmic work of one recursion + contraction launch on the theta grid of band
// limit L (L samples): 6 FP64 flop per Wigner-d recursion step (theta, l, m, n; l from
// max(m, |n|) to L - 1), counted once for all maps and scales of the launch, plus 4 flop
// per complex-by-real multiply-add, per map, at the degrees where the scale's weight is
// nonzero (the filter's support; products with zero coefficients are not counted).
// wt(s, i, l): weight of scale s, n index i, degree l.
template <class Wt>
Work rec_work(int L, int mcount, const std::vector<int> &ns, int NS, int B, Wt wt)
{
    double steps = 0.0, macs = 0.0;
    for (size_t i = 0; i < ns.size(); ++i) {
        const int an = std::abs(ns[i]);
        for (int m = 0; m < mcount; ++m) {
            const int l0 = std::max(m, an);
            if (l0 < L) steps += (double)(L - l0);
        }
        for (int s = 0; s < NS; ++s)
            for (int l = an; l < L; ++l)
                if (wt(s, (int)i, l) != 0.0) macs += (double)std::min(l + 1, mcount);
    }
    Work w;
    w.flop64 = 6.0 * steps * L;
    w.flop = w.flop64 + 4.0 * macs * L * B;
    return w;
}

// ... with the wavelet filters of the given scales (one group: same n set)
Work rec_work_psi(s2w_plan p, const std::vector<int> &scales, int L, int mcount, const std::vector<int> &ns, int B)
{
    const int nn = (int)ns.size();
    return rec_work(L, mcount, ns, (int)scales.size(), B, [&](int s, int i, int l) {
        return p->F.psi_mag[scales[s]][(size_t)l * nn + i];
    });
}

// ... for n = 0 with the weights of a harmonic transform: wt the device table p->wphi
// (scaling filter) or p->wsht (no zero weights)
Work rec_work_n0(s2w_plan p, const double *wt, int L, int mcount, int B)
{
    const bool phi = wt == p->wphi;
    return rec_work(L, mcount, std::vector<int>{0}, 1, B, [&](int, int, int l) {
        return phi ? p->F.phi[l] : 1.0;
    });
}

// The theta quadrature by its Fourier route, per complex column (m, n, map) on the grid
// of band limit L: the length-(2L-1) DFT of the extended column, the Hankel product with
// the weights w(p+q) as a linear convolution through two FFTs of length 2(2L-1) and a
// pointwise product, and the inverse length-(2L-1) DFT (5 n log2 n per complex FFT).
double theta_fft_flop(int L)
{
    const double n = 2.0 * L - 1.0;
    return 10.0 * n * std::log2(n) + 10.0 * (2.0 * n) * std::log2(2.0 * n) + 12.0 * n;
}

double dft_flop(int n, long rows) { return n > 1 ? 2.5 * n * std::log2((double)n) * (double)rows : 0.0; }

template <class Tp>
bool dalloc(s2w_plan p, Tp *&ptr, size_t count)
{
    void *v = nullptr;
    if (count == 0) count = 1;
    if (dev_malloc(&v, count * sizeof(Tp)) != hipSuccess) return false;
    p->allocs.push_back(v);
    ptr = (Tp *)v;
    return true;
}

template <class Tp>
bool upload(s2w_plan p, Tp *&ptr, const std::vector<Tp> &h)
{
    if (!dalloc(p, ptr, h.size())) return false;
    return hipMemcpy(ptr, h.data(), h.size() * sizeof(Tp), hipMemcpyHostToDevice) == hipSuccess;
}

void free_plan(s2w_plan p)
{
    for (void *v : p->allocs) (void)hipFree(v);
    p->allocs.clear();
}

int nglob_index(s2w_plan p, int n)
{
    for (size_t i = 0; i < p->nglob.size(); ++i)
        if (p->nglob[i] == n) return (int)i;
    return -1;
}

bool make_grid(s2w_plan p, int L)
{
    if (p->grids.count(L)) return true;
    DevGrid g;
    g.L = L;
    s2w::ThetaTables tt;
    s2w::theta_tables(L, tt);
    if (!upload(p, g.cth, tt.cth) || !upload(p, g.ctl, tt.cth_lo) || !upload(p, g.ch, tt.ch) || !upload(p, g.sh, tt.sh) ||
        !upload(p, g.ceps, tt.ch_eps) || !upload(p, g.seps, tt.sh_eps))
        return false;
    g.npol = s2w::polar_count(L);
    if (g.npol > 0) {
        std::vector<double> pt;
        s2w::polar_table(L, p->nglob, g.npol, pt);
        if (!upload(p, g.pol, pt)) return false;
    }
    for (int si = 0; si < 2; ++si) {
        std::vector<double> T;
        s2w::theta_matrix(L, si == 0 ? 1 : -1, T);
        if (!upload(p, g.T[si], T)) return false;
        if (p->prec == S2W_MIXED) {
            std::vector<float> T32(T.begin(), T.end());
            if (!upload(p, g.T32[si], T32)) return false;
            if (s2w::gemm_bf3_ok(L)) {
                std::vector<uint16_t> parts[3];
                bf16_split3(T, parts);   // T_sigma is applied as h = T F with T stored [theta][theta']
                for (int k = 0; k < 3; ++k)
                    if (!upload(p, g.T3[si][k], parts[k])) return false;
            }
        }
    }
    const int n = 2 * L - 1;
    s2w::PfaPlan pp;
    s2w::pfa_plan(n, pp);
    // input index (m1 n2 + m2 n1) mod n sits at LDS position m1 n2 + m2; output
    // frequency (a1 e1 + a2 e2) mod n ends at position a1 n2 + a2
    std::vector<int> pin(n), pout(n), inpos(n), outpos(n);
    for (int m1 = 0; m1 < pp.n1; ++m1)
        for (int m2 = 0; m2 < pp.n2; ++m2) {
            const int pos = m1 * pp.n2 + m2;
            pin[pos] = (int)(((long long)m1 * pp.n2 + (long long)m2 * pp.n1) % n);
            pout[pos] = (int)(((long long)m1 * pp.e1 + (long long)m2 * pp.e2) % n);
            inpos[pin[pos]] = pos;
            outpos[pout[pos]] = pos;
        }
    g.dft.n = n;
    g.dft.n1 = pp.n1;
    g.dft.n2 = pp.n2;
    if (!upload(p, g.dft.pin, pin) || !upload(p, g.dft.pout, pout) || !upload(p, g.dft.inpos, inpos) ||
        !upload(p, g.dft.outpos, outpos) ||
        !upload(p, g.dft.w1, pp.w1) || !upload(p, g.dft.w2, pp.w2))
        return false;
    if (p->prec == S2W_MIXED && pp.n1 <= 95 && pp.n2 <= 95 &&
        (!upload(p, g.dft.frag1, dft_fragments(pp.n1, pp.w1)) || !upload(p, g.dft.frag2, dft_fragments(pp.n2, pp.w2))))
        return false;
    p->grids[L] = g;
    return true;
}

bool make_gamma_tw(s2w_plan p, int ng)
{
    if (p->gamma_tw.count(ng)) return true;
    std::vector<double> tw(2 * ng);
    for (int k = 0; k < ng; ++k) {
        long double a = 2.0L * 3.141592653589793238462643383279502884L * k / ng;
        tw[2 * k] = (double)cosl(a);
        tw[2 * k + 1] = (double)sinl(a);
    }
    double *d = nullptr;
    if (!upload(p, d, tw)) return false;
    p->gamma_tw[ng] = d;
    return true;
}

DftArgs dft_args(const DevGrid &g, const void *in, long istride, void *out, long ostride, int nrows,
                 double scale)
{
    DftArgs a{};
    a.in = in;
    a.out = out;
    a.istride = istride;
    a.ostride = ostride;
    a.nrows = nrows;
    a.n = g.dft.n;
    a.n1 = g.dft.n1;
    a.n2 = g.dft.n2;
    a.pin = g.dft.pin;
    a.pout = g.dft.pout;
    a.inpos = g.dft.inpos;
    a.outpos = g.dft.outpos;
    a.w1 = g.dft.w1;
    a.w2 = g.dft.w2;
    a.frag1 = g.dft.frag1;
    a.frag2 = g.dft.frag2;
    a.scale = scale;
    // modular inverses for the index maps: input index x sits at position m1 n2 + m2 with
    // m1 = x n2^-1 mod n1, m2 = x n1^-1 mod n2; output frequency k at (k mod n1) n2 + k mod n2
    a.inv21 = a.inv12 = 0;
    for (int v = 1; v < a.n1; ++v)
        if ((long)v * a.n2 % a.n1 == 1) { a.inv21 = v; break; }
    for (int v = 1; v < a.n2; ++v)
        if ((long)v * a.n1 % a.n2 == 1) { a.inv12 = v; break; }
    return a;
}

void sig_counts(int M, int npar, int &M0, int &M1)
{
    M0 = M1 = 0;
    for (int m = 0; m < M; ++m) ((m + npar) & 1) ? ++M1 : ++M0;
}

LsumArgs lsum_args(s2w_plan p, const DevGrid &g, int mcount, const std::vector<int> &ns)
{
    LsumArgs a{};
    a.L = g.L;
    a.mcount = mcount;
    a.nn = (int)ns.size();
    a.Lrec = p->L;
    for (int i = 0; i < a.nn; ++i) {
        a.nval[i] = ns[i];
        a.nglob[i] = nglob_index(p, ns[i]);
    }
    {
        auto it = p->tile_lsum.find(g.L);
        a.tileT = it == p->tile_lsum.end() ? 0 : it->second;
        auto jt = p->tile_lsum_mm.find(g.L);
        a.tileW = jt == p->tile_lsum_mm.end() ? 0 : jt->second;
    }
    a.A = p->A;
    a.B = p->Bt;
    a.S = p->S_;
    a.smant = p->smant;
    a.sexp = p->sexp;
    a.cth = g.cth;
    a.ctl = g.ctl;
    a.pol = g.pol;
    a.npol = g.npol;
    a.ch = g.ch;
    a.sh = g.sh;
    a.ceps = g.ceps;
    a.seps = g.seps;
    auto dt = p->dtabs.find(g.L);
    if (dt != p->dtabs.end()) {
        a.dtab = dt->second.first;
        a.doff = dt->second.second;
    }
    return a;
}

TsumArgs tsum_args(s2w_plan p, const DevGrid &g, int mcount, const std::vector<int> &ns, int npar)
{
    TsumArgs a{};
    a.L = g.L;
    a.mcount = mcount;
    a.nn = (int)ns.size();
    a.Lrec = p->L;
    a.B = p->B;
    for (int i = 0; i < a.nn; ++i) {
        a.nval[i] = ns[i];
        a.nglob[i] = nglob_index(p, ns[i]);
    }
    a.A = p->A;
    a.B_ = p->Bt;
    a.S = p->S_;
    a.smant = p->smant;
    a.sexp = p->sexp;
    a.cth = g.cth;
    a.ctl = g.ctl;
    a.pol = g.pol;
    a.npol = g.npol;
    a.ch = g.ch;
    a.sh = g.sh;
    a.ceps = g.ceps;
    a.seps = g.seps;
    a.npar = npar;
    sig_counts(mcount, npar, a.M0, a.M1);
    auto dt = p->dtabs.find(g.L);
    if (dt != p->dtabs.end()) {
        a.dtab = dt->second.first;
        a.doff = dt->second.second;
    }
    return a;
}

// Precompute mode (S2W_PLAN_PRECOMPUTE): for every grid of band limit <= PRE_MAX_L, the table
// d^l_mn(theta_b) for all n of the recursion tables, m < L and max(m, |n|) <= l < L, filled
// on the device by the recursion (one launch per n).  The FP64 vector contractions then read
// d from it; grids above PRE_MAX_L keep the recursion.
constexpr int PRE_MAX_L = 512;

bool make_dtables(s2w_plan p)
{
    const int NG = (int)p->nglob.size();
    for (auto &kv : p->grids) {
        const int L = kv.first;
        if (L > PRE_MAX_L) continue;
        std::vector<int64_t> off((size_t)NG * L, 0);
        int64_t tot = 0;
        for (int ng = 0; ng < NG; ++ng)
            for (int m = 0; m < L; ++m) {
                off[(size_t)ng * L + m] = tot;
                const int l0 = std::max(m, std::abs(p->nglob[ng]));
                if (l0 < L) tot += (int64_t)(L - l0) * L;
            }
        double *tab = nullptr;
        int64_t *doff = nullptr;
        if (!dalloc(p, tab, (size_t)tot) || !upload(p, doff, off)) return false;
        for (int ng = 0; ng < NG; ++ng) {
            LsumArgs la = lsum_args(p, kv.second, L, std::vector<int>{p->nglob[ng]});
            s2w::launch_dtable(la, tab, doff, nullptr);
        }
        p->dtabs[L] = {tab, doff};
    }
    return hipDeviceSynchronize() == hipSuccess && hipGetLastError() == hipSuccess;
}

// Precompute mode of mixed plans: for every scale group on a grid of band limit L >= 64
// with L % 8 == 0, the table Dt^l_mn(theta) = sum_theta' d^l_mn(theta') T_sigma[theta][theta']
// (sigma = parity of m + n) for the group's n values, m < L and max(m, |n|) <= l < L, in
// three BF16 parts: 3 N L^3 / 2 bytes per grid (26 GB at L = 1024, N = 8).  Built from the
// FP64 recursion and the FP64 quadrature matrices one n at a time (temporary FP64 d rows of
// that n: L^3 / 2 doubles), then the tile lists of the synthesis product for the plan's batch.
bool make_ttables(s2w_plan p)
{
    const int npar = (p->N - 1) & 1;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const auto &grp = p->groups[gi];
        const int L = grp.L;
        if (L < 64 || L % 8 != 0) continue;
        const DevGrid &g = p->grids[L];
        const auto &si = p->S.s[grp.scales[0]];
        const int nn = (int)si.n.size(), NS = (int)grp.scales.size();
        s2w_plan_s::TTab tt;
        std::vector<int64_t> toff((size_t)nn * L, 0);
        int64_t tot = 0;
        size_t dmax = 0;
        for (int ni = 0; ni < nn; ++ni) {
            size_t dn = 0;
            for (int m = 0; m < L; ++m) {
                toff[(size_t)ni * L + m] = tot;
                const int rows = L - std::max(m, std::abs(si.n[ni]));
                if (rows > 0) {
                    tot += 3 * (int64_t)rows * L;
                    dn += (size_t)rows * L;
                }
            }
            dmax = std::max(dmax, dn);
        }
        if (!dalloc(p, tt.tab, (size_t)tot) || !upload(p, tt.toff, toff)) return false;
        tt.bytes = (size_t)tot * sizeof(uint16_t);
        // temporaries: FP64 d rows of one n, the folded rows of one m, and the row offsets
        double *dtmp = nullptr, *ftmp = nullptr;
        int64_t *doffd = nullptr;
        const int NG = (int)p->nglob.size();
        bool ok = dev_malloc((void **)&dtmp, std::max<size_t>(dmax, 1) * sizeof(double)) == hipSuccess;
        ok = ok && dev_malloc((void **)&ftmp, (size_t)L * L * sizeof(double)) == hipSuccess;
        ok = ok && dev_malloc((void **)&doffd, (size_t)NG * L * sizeof(int64_t)) == hipSuccess;
        for (int ni = 0; ok && ni < nn; ++ni) {
            const int n = si.n[ni], ng = nglob_index(p, n);
            std::vector<int64_t> doff((size_t)NG * L, 0), moff(L, 0);
            int64_t t = 0;
            for (int m = 0; m < L; ++m) {
                doff[(size_t)ng * L + m] = moff[m] = t;
                const int rows = L - std::max(m, std::abs(n));
                if (rows > 0) t += (int64_t)rows * L;
            }
            ok = hipMemcpy(doffd, doff.data(), doff.size() * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess;
            if (!ok) break;
            LsumArgs la = lsum_args(p, g, L, std::vector<int>{n});
            s2w::launch_dtable(la, dtmp, doffd, nullptr);
            for (int m = 0; m < L; ++m) {
                const int rows = L - std::max(m, std::abs(n));
                if (rows <= 0) continue;
                s2w::launch_gemm(dtmp + moff[m], g.T[(m + npar) & 1], ftmp, rows, L, L, nullptr);
                s2w::launch_split3_f64(ftmp, tt.tab + toff[(size_t)ni * L + m], (size_t)rows * L, nullptr);
            }
        }
        ok = ok && hipDeviceSynchronize() == hipSuccess && hipGetLastError() == hipSuccess;
        if (dtmp) (void)hipFree(dtmp);
        if (ftmp) (void)hipFree(ftmp);
        if (doffd) (void)hipFree(doffd);
        if (!ok) return false;
        // tile lists: problems by decreasing row count dealt to the eight XCD lists, the tiles of
        // a problem consecutive (degree tile outer, column tile inner)
        const int ncols = 2 * p->B * NS, nct = (ncols + 127) / 128;
        std::vector<std::pair<int, int>> probs;   // (m, ni)
        for (int ni = 0; ni < nn; ++ni)
            for (int m = 0; m < L; ++m)
                if (L - std::max(m, std::abs(si.n[ni])) > 0) probs.push_back({m, ni});
        std::stable_sort(probs.begin(), probs.end(), [&](const std::pair<int, int> &u, const std::pair<int, int> &v) {
            return L - std::max(u.first, std::abs(si.n[u.second])) > L - std::max(v.first, std::abs(si.n[v.second]));
        });
        std::vector<int4> lists[8];
        for (size_t q = 0; q < probs.size(); ++q) {
            const int m = probs[q].first, ni = probs[q].second;
            const int rows = L - std::max(m, std::abs(si.n[ni])), nlt = (rows + 127) / 128;
            for (int lt = 0; lt < nlt; ++lt)
                for (int ct = 0; ct < nct; ++ct) lists[q % 8].push_back(make_int4(m, ni, ct, lt));
        }
        std::vector<int4> all;
        for (int x = 0; x < 8; ++x) {
            tt.off[x] = (int)all.size();
            tt.cnt[x] = (int)lists[x].size();
            all.insert(all.end(), lists[x].begin(), lists[x].end());
        }
        if (!upload(p, tt.tiles, all)) return false;
        p->ttabs[(int)gi] = tt;
    }
    return true;
}

// Precompute mode of batched plans (8 maps or more): the forward SHT of the full grid through
// the FP64 table Dt^l_m(theta) = sum_theta' d^l_m0(theta') T_sigma[theta][theta'] (per m,
// rows l = m..L-1): L^2 (L+1) / 2 doubles (4.3 GB at L = 1024), built from the FP64
// recursion rows of n = 0 and one quadrature product per m; then the tile lists for the
// plan's batch.  Needs an even L (16-byte loads).
bool make_shttab(s2w_plan p)
{
    const int L = p->L;
    if (L < 64 || L % 2 != 0 || p->B < 8 || p->cplx) return true;
    const DevGrid &g = p->grids[L];
    std::vector<int64_t> toff(L, 0);
    int64_t tot = 0;
    for (int m = 0; m < L; ++m) {
        toff[m] = tot;
        tot += (int64_t)(L - m) * L;
    }
    if (!dalloc(p, p->shttab, (size_t)tot) || !upload(p, p->shtoff, toff)) return false;
    const int NG = (int)p->nglob.size(), ng = nglob_index(p, 0);
    // the d rows stay as the inverse table
    if (!dalloc(p, p->shtitab, (size_t)tot)) return false;
    double *dtmp = p->shtitab;
    int64_t *doffd = nullptr;
    bool ok = true;
    ok = ok && dev_malloc((void **)&doffd, (size_t)NG * L * sizeof(int64_t)) == hipSuccess;
    if (ok) {
        std::vector<int64_t> doff((size_t)NG * L, 0);
        for (int m = 0; m < L; ++m) doff[(size_t)ng * L + m] = toff[m];
        ok = hipMemcpy(doffd, doff.data(), doff.size() * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (ok) {
        LsumArgs la = lsum_args(p, g, L, std::vector<int>{0});
        s2w::launch_dtable(la, dtmp, doffd, nullptr);
        for (int m = 0; m < L; ++m)
            s2w::launch_gemm(dtmp + toff[m], g.T[m & 1], p->shttab + toff[m], L - m, L, L, nullptr);
        ok = hipDeviceSynchronize() == hipSuccess && hipGetLastError() == hipSuccess;
    }
    if (doffd) (void)hipFree(doffd);
    if (!ok) return false;
    const int mt = (2 * p->B + 127) / 128;
    {
        std::vector<int4> il[8];
        for (int m = 0; m < L; ++m)
            for (int j = 0; j < (L + 63) / 64; ++j)
                for (int i = 0; i < mt; ++i) il[m % 8].push_back(make_int4(m, i, j, 0));
        std::vector<int4> iall;
        for (int x = 0; x < 8; ++x) {
            p->shtioffx[x] = (int)iall.size();
            p->shticnt[x] = (int)il[x].size();
            iall.insert(iall.end(), il[x].begin(), il[x].end());
        }
        if (!upload(p, p->shtitiles, iall)) return false;
    }
    std::vector<int4> lists[8];
    for (int m = 0; m < L; ++m) {   // rows decrease with m: dealt in order
        const int nt = (L - m + 63) / 64;
        for (int j = 0; j < nt; ++j)
            for (int i = 0; i < mt; ++i) lists[m % 8].push_back(make_int4(m, i, j, 0));
    }
    std::vector<int4> all;
    for (int x = 0; x < 8; ++x) {
        p->shtoffx[x] = (int)all.size();
        p->shtcnt[x] = (int)lists[x].size();
        all.insert(all.end(), lists[x].begin(), lists[x].end());
    }
    return upload(p, p->shttiles, all);
}

GammaArgs gamma_args(s2w_plan p, int M, int L, int Min, int Mout, const std::vector<int> &ns, int ng)
{
    GammaArgs a{};
    a.B = p->B;
    a.M = M;
    a.L = L;
    a.Min = Min;
    a.Mout = Mout;
    a.nn = (int)ns.size();
    a.ng = ng;
    for (int i = 0; i < a.nn; ++i) a.nval[i] = ns[i];
    a.tw = p->gamma_tw[ng];
    a.sgn = 1.0;
    a.phr = 1.0;
    a.phi = 0.0;
    a.wscale = 1.0;
    a.fm0 = 1.0;
    a.fm1 = 1.0;
    a.npar = 0;
    a.M0 = a.M1 = 0;
    return a;
}

// h = T_sigma F on sigma-grouped rows; nn n values per m, npar their parity
void theta_quadrature(s2w_plan p, const DevGrid &g, const double *F, double *H, int M, int nn, int npar,
                      hipStream_t st)
{
    int M0, M1;
    sig_counts(M, npar, M0, M1);
    const size_t r0 = (size_t)p->B * M0 * nn * 2, r1 = (size_t)p->B * M1 * nn * 2;
    {
        Prof pr_(p, "gemm_theta", Work{theta_fft_flop(g.L) * (r0 / 2), 0.0, 2.0 * (double)r0 * g.L * g.L}, st);
        s2w::launch_gemm(F, g.T[0], H, (int)r0, g.L, g.L, st);
    }
    {
        Prof pr_(p, "gemm_theta", Work{theta_fft_flop(g.L) * (r1 / 2), 0.0, 2.0 * (double)r1 * g.L * g.L}, st);
        s2w::launch_gemm(F + r0 * g.L, g.T[1], H + r0 * g.L, (int)r1, g.L, g.L, st);
    }
}

// f (maps) -> flm internal [B][L][L] (m-major), forward SHT (eq:fswsh on MW samples)
void sht_forward_internal(s2w_plan p, const double *f, double *flm_out, hipStream_t st)
{
    const DevGrid &g = p->grids[p->L];
    const int L = p->L, na = 2 * L - 1;
    { const DftArgs da_ = dft_args(g, f, na, p->bufA, L, p->B * L, 2.0 * M_PI / na); Prof pr_(p, "dft_r2c", dft_flop(da_.n, da_.nrows), st); s2w::launch_dft_r2c(da_, st); }
    std::vector<int> n0{0};
    GammaArgs ga = gamma_args(p, L, L, L, L, n0, 1);
    ga.src = p->bufA;
    ga.dst = p->bufB;
    ga.sgn = -1.0;
    sig_counts(L, 0, ga.M0, ga.M1);
    { Prof pr_(p, "gamma_r2c", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_r2c(ga, st); }
    if (p->shttab) {
        // precompute mode: quadrature and theta sums through the folded table
        s2w::ShtTab sa{};
        sa.L = L;
        sa.B = p->B;
        sa.M0 = ga.M0;
        sa.M1 = ga.M1;
        sa.F = p->bufB;
        sa.out = flm_out;
        sa.w = p->wsht;
        sa.tab = p->shttab;
        sa.toff = p->shtoff;
        sa.tiles = p->shttiles;
        for (int x = 0; x < 8; ++x) {
            sa.cnt[x] = p->shtcnt[x];
            sa.off[x] = p->shtoffx[x];
        }
        Work wk = rec_work_n0(p, p->wsht, L, L, p->B);
        wk.flop -= wk.flop64;   // no recursion: d comes from the table
        wk.flop64 = 0.0;
        Prof pr_(p, "sht_tab", wk, st);
        s2w::launch_sht_tab(sa, st);
        return;
    }
    theta_quadrature(p, g, p->bufB, p->bufC, L, 1, 0, st);
    TsumArgs ta = tsum_args(p, g, L, n0, 0);
    ta.h[0] = p->bufC;
    ta.w[0] = p->wsht;
    ta.wstride = 0;
    ta.out[0] = flm_out;
    {
        Prof pr_(p, "tsum", rec_work_n0(p, p->wsht, ta.L, ta.mcount, p->B), st);
        s2w::launch_tsum(ta, 1, p->B, st);
    }
}

// flm internal -> maps, inverse SHT (eq:iswsh)
void sht_inverse_internal(s2w_plan p, const double *flm_in, double *f, hipStream_t st)
{
    const DevGrid &g = p->grids[p->L];
    const int L = p->L, na = 2 * L - 1;
    std::vector<int> n0{0};
    if (p->shtitab) {
        // precompute mode: theta rows from the table of d^l_m0
        s2w::ShtTab sa{};
        sa.L = L;
        sa.B = p->B;
        sa.F = flm_in;
        sa.out = p->bufA;
        sa.w = p->wsht;
        sa.tab = p->shtitab;
        sa.toff = p->shtoff;
        sa.tiles = p->shtitiles;
        for (int x = 0; x < 8; ++x) {
            sa.cnt[x] = p->shticnt[x];
            sa.off[x] = p->shtioffx[x];
        }
        Work wk = rec_work_n0(p, p->wsht, L, L, p->B);
        wk.flop -= wk.flop64;
        wk.flop64 = 0.0;
        Prof pr_(p, "shti_tab", wk, st);
        s2w::launch_shti_tab(sa, st);
    } else {
        LsumArgs la = lsum_args(p, g, L, n0);
        la.flm = flm_in;
        la.flm_m = L;
        la.flm_l = L;
        la.w[0] = p->wsht;
        la.wstride = 0;
        la.out[0] = p->bufA;
        Prof pr_(p, "lsum", rec_work_n0(p, p->wsht, la.L, la.mcount, p->B), st);
        s2w::launch_lsum(la, 1, p->B, st);
    }
    GammaArgs ga = gamma_args(p, L, L, L, L, n0, 1);
    ga.src = p->bufA;
    ga.dst = p->bufB;
    { Prof pr_(p, "gamma_c2r", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_c2r(ga, st); }
    { const DftArgs da_ = dft_args(g, p->bufB, L, f, na, p->B * L, 1.0); Prof pr_(p, "dft_c2r", dft_flop(da_.n, da_.nrows), st); s2w::launch_dft_c2r(da_, st); }
}

// Spin-s maps (plans from s2w_plan_create_spin; B counts real maps, u = Re f at 2b and
// v = Im f at 2b + 1).  Forward spin-s SHT (eq:fswsh with sY_lm = (-1)^s sqrt((2l+1)/(4 pi))
// e^{i m phi} d^l_{m,-s}): the real DFTs of u and v, the theta quadrature with the parity
// (-1)^{m+s} of the n = -s integrand, the theta sums with d^l_{m,-s} and d^l_{m,s} (the
// negative orders), then the combination into the real-map pairs (A, B) with g = A + i B
// and / or g itself in the external layout.
void spin_sht_forward_internal(s2w_plan p, const double *f, double *pairs, double *ext, hipStream_t st)
{
    const DevGrid &g = p->grids[p->L];
    const int L = p->L, na = 2 * L - 1, s = p->spin, npar = s & 1;
    { const DftArgs da_ = dft_args(g, f, na, p->bufA, L, p->B * L, 2.0 * M_PI / na); Prof pr_(p, "dft_r2c", dft_flop(da_.n, da_.nrows), st); s2w::launch_dft_r2c(da_, st); }
    const std::vector<int> ns{-s, s};
    GammaArgs ga = gamma_args(p, L, L, L, L, ns, 1);
    ga.src = p->bufA;
    ga.dst = p->bufB;
    ga.sgn = -1.0;
    ga.npar = npar;
    sig_counts(L, npar, ga.M0, ga.M1);
    { Prof pr_(p, "gamma_r2c", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_r2c(ga, st); }
    theta_quadrature(p, g, p->bufB, p->bufC, L, 2, npar, st);
    TsumArgs ta = tsum_args(p, g, L, ns, npar);
    ta.h[0] = p->bufC;
    ta.w[0] = p->wsht;
    ta.wstride = 0;
    ta.out[0] = p->bufA;
    {
        Prof pr_(p, "tsum", rec_work(L, L, ns, 1, p->B, [](int, int, int) { return 1.0; }), st);
        s2w::launch_tsum(ta, 1, p->B, st);
    }
    s2w::launch_spin_combine(p->bufA, pairs, ext, L, s, p->B / 2, st);
}

// Inverse spin-s SHT (eq:iswsh) from the real-map pairs or from g in the external layout:
// the split into the coefficient rows of u and v (n = -s and n = +s slots), the l-sums, the
// sum over the two slots, and the real inverse DFTs.
void spin_sht_inverse_internal(s2w_plan p, const double *pairs, const double *ext, double *f, hipStream_t st)
{
    const DevGrid &g = p->grids[p->L];
    const int L = p->L, na = 2 * L - 1, s = p->spin;
    s2w::launch_spin_split(pairs, ext, p->bufC, L, s, p->B / 2, st);
    const std::vector<int> ns{-s, s};
    LsumArgs la = lsum_args(p, g, L, ns);
    la.flm = p->bufC;
    la.flm_m = 2 * L;
    la.flm_l = L;
    la.flm_nstride = (long)L * L;
    la.w[0] = p->wsht;
    la.wstride = 0;
    la.out[0] = p->bufA;
    {
        Prof pr_(p, "lsum", rec_work(L, L, ns, 1, p->B, [](int, int, int) { return 1.0; }), st);
        s2w::launch_lsum(la, 1, p->B, st);
    }
    GammaArgs ga = gamma_args(p, L, L, L, L, ns, 1);
    ga.src = p->bufA;
    ga.dst = p->bufB;
    { Prof pr_(p, "gamma_c2r", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_c2r(ga, st); }
    { const DftArgs da_ = dft_args(g, p->bufB, L, f, na, p->B * L, 1.0); Prof pr_(p, "dft_c2r", dft_flop(da_.n, da_.nrows), st); s2w::launch_dft_c2r(da_, st); }
}

// ---- mixed-precision stages (FP32 arrays, FP64 recursion and scale sums) ----

void theta_quadrature32(s2w_plan p, const DevGrid &g, const float *F, float *H, int M, int nn, int npar,
                        hipStream_t st)
{
    int M0, M1;
    sig_counts(M, npar, M0, M1);
    const size_t r0 = (size_t)p->B * M0 * nn * 2, r1 = (size_t)p->B * M1 * nn * 2;
    if (g.T3[0][0]) {
        // BF16x3 split on BF16 matrix cores (FP32 accuracy or better)
        {
            Prof pr_(p, "gemm_theta_bf3", Work{theta_fft_flop(g.L) * (r0 / 2), 0.0, 2.0 * (double)r0 * g.L * g.L}, st);
            s2w::launch_gemm_bf3(F, g.T3[0][0], g.T3[0][1], g.T3[0][2], H, (int)r0, g.L, g.L, st);
        }
        {
            Prof pr_(p, "gemm_theta_bf3", Work{theta_fft_flop(g.L) * (r1 / 2), 0.0, 2.0 * (double)r1 * g.L * g.L}, st);
            s2w::launch_gemm_bf3(F + r0 * g.L, g.T3[1][0], g.T3[1][1], g.T3[1][2], H + r0 * g.L, (int)r1, g.L, g.L, st);
        }
        return;
    }
    {
        Prof pr_(p, "gemm_theta_f32", Work{theta_fft_flop(g.L) * (r0 / 2), 0.0, 2.0 * (double)r0 * g.L * g.L}, st);
        s2w::launch_gemm_f32(F, g.T32[0], H, (int)r0, g.L, g.L, st);
    }
    {
        Prof pr_(p, "gemm_theta_f32", Work{theta_fft_flop(g.L) * (r1 / 2), 0.0, 2.0 * (double)r1 * g.L * g.L}, st);
        s2w::launch_gemm_f32(F + r0 * g.L, g.T32[1], H + r0 * g.L, (int)r1, g.L, g.L, st);
    }
}

// Runs a plan on its first nb <= B maps: the plan's batch and the packed scale
// offsets follow nb while the scope lives (workspace is sized for B).
struct BatchScope {
    s2w_plan p;
    int B0;
    std::vector<int64_t> off0;
    BatchScope(s2w_plan p_, int nb) : p(p_), B0(p_->B), off0(p_->wav_off)
    {
        p->B = nb;
        const int K = (int)p->S.s.size();
        for (int k = 0; k < K; ++k)
            p->wav_off[k + 1] = p->wav_off[k] + (int64_t)nb * (2 * p->S.s[k].N - 1) * p->S.s[k].L * (2 * p->S.s[k].L - 1);
    }
    ~BatchScope()
    {
        p->B = B0;
        p->wav_off = off0;
    }
};

// Graph replay: the launches of one entry point for a given pointer triple are
// captured once (on the plan's own stream, so that a default caller stream works)
// into a HIP graph, which is then launched on the caller's stream.
template <class Body>
s2w_status run_graph(s2w_plan p, int kind, const void *a, const void *b, const void *c, hipStream_t st,
                     Body &&body)
{
    for (auto &g : p->graphs)
        if (g.kind == kind && g.a == a && g.b == b && g.c == c) {
            if (hipGraphLaunch(g.exec, st) != hipSuccess) return fail(S2W_EHIP, "hipGraphLaunch failed");
            return S2W_OK;
        }
    if (p->graphs.size() >= 16) return fail(S2W_EINVAL, "graph cache full (16 pointer triples per plan)");
    if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(S2W_EHIP, "stream creation failed");
    (void)hipGetLastError();
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(S2W_EHIP, "hipStreamBeginCapture failed");
    p->capturing = true;
    body(p->cap_stream);
    p->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e1 = hipStreamEndCapture(p->cap_stream, &graph);
    const hipError_t e0 = hipGetLastError();
    if (e1 != hipSuccess || e0 != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(S2W_EHIP, "graph capture failed");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return fail(S2W_EHIP, "hipGraphInstantiate failed");
    p->graphs.push_back({kind, a, b, c, exec});
    if (hipGraphLaunch(exec, st) != hipSuccess) return fail(S2W_EHIP, "hipGraphLaunch failed");
    return S2W_OK;
}

// Mixed plans: does the contraction of the grid of band limit Lk take the FP64 vector route?
// The autotuner's choice when it timed this grid, else the batch heuristic: the matrix-core
// kernels work on 64 columns (2 x maps x scales), so at one or two maps they do mostly
// padding and the vector kernels (one theta sample per lane) are faster.
bool lsum_vector(s2w_plan p, int Lk)
{
    auto it = p->route_lsum.find(Lk);
    return it != p->route_lsum.end() ? it->second == 1 : p->B <= 2;
}

bool tsum_vector(s2w_plan p, int Lk)
{
    auto it = p->route_tsum.find(Lk);
    return it != p->route_tsum.end() ? it->second == 1 : p->B <= 1;
}

// Work list of the persistent l-contraction (mixed plans): every degree group with band
// limit >= 64 on the matrix-core route, up to MAX_LGROUPS, whose outputs fit side by side
// in bufA.  Units (m, n, column group) are sorted by decreasing cost L_j - max(m, |n|) and
// dealt to the eight XCD lists in turn; each unit's theta blocks stay on its list.
bool build_lsum_list(s2w_plan p)
{
    p->lgroups.clear();
    p->lgroup_off.clear();
    size_t off = 0;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const auto &grp = p->groups[gi];
        if (grp.L < 64 || lsum_vector(p, grp.L)) continue;
        const int nn = (int)p->S.s[grp.scales[0]].n.size();
        const size_t sz = grp.scales.size() * (size_t)p->B * nn * grp.L * grp.L * 2;   // floats
        if (p->lgroups.size() == (size_t)s2w::MAX_LGROUPS || off + sz > 2 * p->szA) break;
        p->lgroups.push_back((int)gi);
        p->lgroup_off.push_back(off);
        off += sz;
    }
    // the groups outside the list write their outputs after the listed ones
    size_t rest = 0;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        if (std::find(p->lgroups.begin(), p->lgroups.end(), (int)gi) != p->lgroups.end()) continue;
        const auto &grp = p->groups[gi];
        const int nn = (int)p->S.s[grp.scales[0]].n.size();
        rest = std::max(rest, grp.scales.size() * (size_t)p->B * nn * grp.L * grp.L * 2);
    }
    if (p->lgroups.size() < 2 || off + rest > 2 * p->szA) {
        p->lgroups.clear();
        p->lgroup_off.clear();
        return false;
    }
    p->list_end = off;
    struct U { int cost, gi, m, ni, g, ntb; };
    std::vector<U> units;
    for (size_t k = 0; k < p->lgroups.size(); ++k) {
        const auto &grp = p->groups[p->lgroups[k]];
        const auto &si = p->S.s[grp.scales[0]];
        const int NS = (int)grp.scales.size(), nn = (int)si.n.size();
        const int ngrp = (2 * p->B * NS + 63) / 64, ntb = ((grp.L + 63) / 64 + 3) / 4;
        for (int g = 0; g < ngrp; ++g)
            for (int ni = 0; ni < nn; ++ni)
                for (int m = 0; m < grp.L; ++m) {
                    const int l0 = std::max(m, std::abs(si.n[ni]));
                    if (l0 < grp.L) units.push_back({grp.L - l0, (int)k, m, ni, g, ntb});
                }
    }
    std::stable_sort(units.begin(), units.end(), [](const U &a, const U &b) { return a.cost > b.cost; });
    std::vector<uint2> lists[8];
    for (size_t u = 0; u < units.size(); ++u)
        for (int tb = 0; tb < units[u].ntb; ++tb) {
            uint2 it;
            it.x = (unsigned)units[u].gi | ((unsigned)units[u].ni << 4) | ((unsigned)tb << 8) | ((unsigned)units[u].g << 16);
            it.y = (unsigned)units[u].m;
            lists[u % 8].push_back(it);
        }
    std::vector<uint2> all;
    for (int x = 0; x < 8; ++x) {
        p->list_off[x] = (int)all.size();
        p->list_cnt[x] = (int)lists[x].size();
        all.insert(all.end(), lists[x].begin(), lists[x].end());
    }
    if (!upload(p, p->items, all)) return false;
    if (!p->counters && !dalloc(p, p->counters, 8)) return false;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || ncu <= 0) ncu = 256;
    p->list_blocks = 2 * ncu;
    p->list_B = p->B;
    return true;
}

// Launch arguments of the persistent l-contraction of the analysis from flm (bufA outputs at
// the groups' offsets)
s2w::LsumList lsum_list_args(s2w_plan p, const double *flm)
{
    s2w::LsumList gl{};
    gl.ngroups = (int)p->lgroups.size();
    for (int x = 0; x < 8; ++x) {
        gl.cnt[x] = p->list_cnt[x];
        gl.off[x] = p->list_off[x];
    }
    float *A32 = (float *)p->bufA;
    for (int k = 0; k < gl.ngroups; ++k) {
        const auto &grp = p->groups[p->lgroups[k]];
        const DevGrid &g = p->grids[grp.L];
        const auto &si = p->S.s[grp.scales[0]];
        const int NS = (int)grp.scales.size(), nn = (int)si.n.size();
        const size_t cstride = (size_t)p->B * nn * grp.L * grp.L * 2;
        LsumArgs la = lsum_args(p, g, grp.L, si.n);
        la.flm = flm;
        la.flm_m = p->L;
        la.flm_l = p->L;
        la.wstride = grp.L;
        gl.NS[k] = NS;
        gl.o[k].B = p->B;
        for (int s = 0; s < NS; ++s) {
            la.w[s] = p->wpsi[grp.scales[s]];
            la.lmin[s] = p->lmin[grp.scales[s]];
            gl.o[k].out[s] = A32 + p->lgroup_off[k] + s * cstride;
        }
        gl.a[k] = la;
    }
    return gl;
}

// S2W_PLAN_TUNE: time the candidate kernels of every scale group on the plan's own shapes and
// workspace, and keep the fastest.  FP64 plans (band limit >= 128): theta samples per lane of
// k_lsum (1, 2, 4, 8).  Mixed plans (band limit >= 64): for the l-contraction the matrix-core
// kernel with 2 or 4 waves per block, or the FP64 vector kernel plus its conversion to FP32;
// for the theta contraction the matrix-core kernel, or the conversion of its input to FP64
// plus the FP64 vector kernel.  Every candidate of a contraction gives the same sums to
// rounding.  Runs at plan creation (synchronises).
void autotune(s2w_plan p)
{
    const bool mixed = p->prec == S2W_MIXED;
    const int B = p->B;
    (void)hipMemset(p->flm, 0, sizeof(double) * (size_t)B * p->L * p->L * 2);
    (void)hipMemset(p->bufA, 0, sizeof(double) * p->szA);
    (void)hipMemset(p->bufC, 0, sizeof(double) * p->szC);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        if (e0) (void)hipEventDestroy(e0);
        return;
    }
    // best of the candidates (each launched once untimed, then twice timed); 0 if none ran
    auto pick = [&](const std::vector<int> &cands, const std::function<void(int)> &launch) {
        int best = 0;
        float best_ms = 0.0f;
        for (int c : cands) {
            launch(c);
            (void)hipEventRecord(e0, nullptr);
            launch(c);
            launch(c);
            (void)hipEventRecord(e1, nullptr);
            if (hipEventSynchronize(e1) != hipSuccess) continue;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (best == 0 || ms < best_ms) { best = c; best_ms = ms; }
        }
        return best;
    };
    for (auto &grp : p->groups) {
        const int Lk = grp.L, NS = (int)grp.scales.size();
        if (Lk < (mixed ? 64 : 128) || (mixed ? p->route_lsum.count(Lk) : p->tile_lsum.count(Lk))) continue;
        const DevGrid &g = p->grids[Lk];
        const auto &si = p->S.s[grp.scales[0]];
        const int nn = (int)si.n.size();
        const int npar = (p->N - 1) & 1;
        LsumArgs la = lsum_args(p, g, Lk, si.n);
        la.flm = p->flm;
        la.flm_m = p->L;
        la.flm_l = p->L;
        la.wstride = Lk;
        const size_t cstride = (size_t)B * nn * Lk * Lk * 2;
        s2w::MixOut mo{};
        mo.B = B;
        for (int s = 0; s < NS; ++s) {
            la.w[s] = p->wpsi[grp.scales[s]];
            la.lmin[s] = p->lmin[grp.scales[s]];
            la.out[s] = p->bufC + s * cstride;
            mo.out[s] = (float *)p->bufA + s * cstride;
        }
        if (!mixed) {
            const int best = pick({1, 2, 4, 8}, [&](int c) { la.tileT = c; s2w::launch_lsum(la, NS, B, nullptr); });
            if (best) p->tile_lsum[Lk] = best;
            continue;
        }
        // l-contraction: 2 or 4 waves per block on matrix cores, or (-1) the vector route
        const int bl = pick({2, 4, -1}, [&](int c) {
            if (c > 0) {
                la.tileW = c;
                s2w::launch_lsum_mm(la, mo, NS, nullptr);
            } else {
                s2w::launch_lsum(la, NS, B, nullptr);
                s2w::launch_convert(p->bufC, mo.out[0], NS * cstride, true, nullptr);
            }
        });
        if (bl) {
            p->route_lsum[Lk] = bl < 0 ? 1 : 0;
            if (bl > 0) p->tile_lsum_mm[Lk] = bl;
        }
        // theta contraction on zero quadrature rows: matrix cores (1) or the vector route (-1)
        TsumArgs ta = tsum_args(p, g, Lk, si.n, npar);
        ta.wstride = Lk;
        s2w::MixIn mi{};
        mi.B = B;
        for (int s = 0; s < NS; ++s) {
            const int k = grp.scales[s];
            ta.w[s] = p->wpsi[k];
            ta.lmin[s] = p->lmin[k];
            ta.h[s] = p->bufA + s * cstride;
            ta.out[s] = p->P[k];
            mi.h[s] = (const float *)p->bufC + s * cstride;
            mi.out[s] = p->P[k];
        }
        const int bt = pick({1, -1}, [&](int c) {
            if (c > 0) {
                s2w::launch_tsum_mm(ta, mi, NS, nullptr);
            } else {
                s2w::launch_convert(p->bufC, p->bufA, NS * cstride, false, nullptr);
                s2w::launch_tsum(ta, NS, B, nullptr);
            }
        });
        if (bt) p->route_tsum[Lk] = bt < 0 ? 1 : 0;
    }
    // the analysis l-contraction of all matrix-core groups: one launch per group (1) or the
    // persistent launch over the cost-sorted work list (2)
    if (mixed && !p->lsum_list && build_lsum_list(p)) {
        const s2w::LsumList gl = lsum_list_args(p, p->flm);
        const int best = pick({1, 2}, [&](int c) {
            if (c == 1)
                for (int k = 0; k < gl.ngroups; ++k) s2w::launch_lsum_mm(gl.a[k], gl.o[k], gl.NS[k], nullptr);
            else
                s2w::launch_lsum_list(gl, p->items, p->counters, p->list_blocks, nullptr);
        });
        p->lsum_list = best == 2;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipGetLastError();
}

s2w_status check_plan(s2w_plan p)
{
    if (!p) return fail(S2W_EINVAL, "null plan");
    if (!reg_has(p)) return fail(S2W_ESTATE, "not a live plan (destroyed, or never created)");
    return S2W_OK;
}

// real-map transform entry points that use the plan's own workspace
s2w_status check_ws(s2w_plan p)
{
    if (p->cplx) return fail(S2W_ESTATE, "plan made for complex spin maps: use the s2w_spin_* calls");
    if (p->no_ws)
        return fail(S2W_ESTATE, "plan created with S2W_PLAN_NO_WORKSPACE: only s2w_analysis_noalloc runs on it");
    return S2W_OK;
}

s2w_status check_spin(s2w_plan p)
{
    if (!p->cplx) return fail(S2W_ESTATE, "plan made for real maps: the s2w_spin_* calls need s2w_plan_create_spin");
    return S2W_OK;
}

s2w_status check_ball(b3w_plan p)
{
    if (!p) return fail(S2W_EINVAL, "null plan");
    if (!reg_has(p)) return fail(S2W_ESTATE, "not a live ball plan (destroyed, or never created)");
    return S2W_OK;
}

s2w_status post_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(S2W_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return S2W_OK;
}

}  // namespace

// ======================================================================== API

extern "C" {

const char *s2w_last_error(void) { return g_err.c_str(); }

s2w_status s2w_host_scales(int L, int N, double lambda, int J0, int *nscales, int *Lk, int *Nk, int *L_phi)
{
    s2w::Scales S;
    std::string err;
    if (!s2w::make_scales(L, N, lambda, J0, S, err)) return fail(S2W_EINVAL, err);
    if (nscales) *nscales = (int)S.s.size();
    for (size_t k = 0; k < S.s.size(); ++k) {
        if (Lk) Lk[k] = S.s[k].L;
        if (Nk) Nk[k] = S.s[k].N;
    }
    if (L_phi) *L_phi = S.Lphi;
    return S2W_OK;
}

s2w_status s2w_host_filters(int L, int N, double lambda, int J0, double *psi, double *phi)
{
    s2w::Scales S;
    std::string err;
    if (!s2w::make_scales(L, N, lambda, J0, S, err)) return fail(S2W_EINVAL, err);
    s2w::Filters F;
    s2w::make_filters(S, F);
    if (phi)
        for (int l = 0; l < L; ++l) phi[l] = F.phi[l];
    if (psi) {
        const size_t per = (size_t)L * (2 * N - 1) * 2;
        std::memset(psi, 0, sizeof(double) * per * S.s.size());
        for (size_t k = 0; k < S.s.size(); ++k) {
            const auto &si = S.s[k];
            const int nn = (int)si.n.size();
            for (int l = 0; l < si.L; ++l)
                for (int i = 0; i < nn; ++i) {
                    const double v = F.psi_mag[k][(size_t)l * nn + i];
                    double *o = psi + k * per + ((size_t)l * (2 * N - 1) + (si.n[i] + N - 1)) * 2;
                    if (F.xi_imag) o[1] = v;
                    else o[0] = v;
                }
        }
    }
    return S2W_OK;
}

s2w_status s2w_host_theta_matrix(int L, int sigma, double *T)
{
    if (L < 1 || !T || (sigma != 1 && sigma != -1)) return fail(S2W_EINVAL, "bad arguments");
    std::vector<double> t;
    s2w::theta_matrix(L, sigma, t);
    std::memcpy(T, t.data(), sizeof(double) * t.size());
    return S2W_OK;
}

s2w_status s2w_host_wigner_d(int L, int m, int n, double *out)
{
    if (L < 1 || !out || std::abs(m) >= L || std::abs(n) >= L) return fail(S2W_EINVAL, "bad arguments");
    std::vector<double> d;
    s2w::host_wigner_d(L, m, n, d);
    std::memcpy(out, d.data(), sizeof(double) * d.size());
    return S2W_OK;
}

// Plan creation for real maps (cplx false) or for complex spin-`spin` maps (cplx true:
// every map is held as its real and imaginary parts, so the internal batch is 2 batch).
static s2w_status plan_create(s2w_plan *out, int L, int N, double lambda, int J0, int batch,
                              s2w_precision precision, int device, unsigned flags, bool cplx, int spin)
{
    AllocSeq alloc_seq;
    if (!out) return fail(S2W_EINVAL, "null output pointer");
    *out = nullptr;
    if (batch < 1) return fail(S2W_EINVAL, "batch must be >= 1");
    if (cplx) {
        if (batch > (1 << 29)) return fail(S2W_EINVAL, "batch too large");
        if (L < 1 || spin <= -L || spin >= L) return fail(S2W_EINVAL, "spin must satisfy |spin| < L");
        if (flags & (S2W_PLAN_GRAPH | S2W_PLAN_NO_WORKSPACE | S2W_PLAN_WIGNER))
            return fail(S2W_EINVAL, "spin plans accept S2W_PLAN_TUNE, S2W_PLAN_PERSISTENT and S2W_PLAN_PRECOMPUTE only");
        batch *= 2;
    }
    if (flags & ~(unsigned)(S2W_PLAN_TUNE | S2W_PLAN_GRAPH | S2W_PLAN_NO_WORKSPACE | S2W_PLAN_PERSISTENT |
                            S2W_PLAN_PRECOMPUTE | S2W_PLAN_WIGNER))
        return fail(S2W_EINVAL, "unknown flags");
    if ((flags & S2W_PLAN_WIGNER) && 2 * N - 1 > s2w::MAX_NN)
        return fail(S2W_EUNSUPPORTED, "S2W_PLAN_WIGNER needs 2N - 1 <= 8 azimuthal orders (N <= 4)");
    if ((flags & S2W_PLAN_NO_WORKSPACE) && (flags & (S2W_PLAN_TUNE | S2W_PLAN_GRAPH)))
        return fail(S2W_EINVAL, "S2W_PLAN_NO_WORKSPACE excludes S2W_PLAN_TUNE and S2W_PLAN_GRAPH");
    if (precision != S2W_FP64 && precision != S2W_MIXED) return fail(S2W_EINVAL, "unknown precision");
    s2w::Scales S;
    std::string err;
    if (!s2w::make_scales(L, N, lambda, J0, S, err)) return fail(S2W_EINVAL, err);
    if (N > s2w::MAX_NN) return fail(S2W_EUNSUPPORTED, "N too large (max 8)");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(S2W_EHIP, "no HIP device");
    if (device < 0 || device >= ndev) return fail(S2W_EINVAL, "bad device index");
    if (hipSetDevice(device) != hipSuccess) return fail(S2W_EHIP, "hipSetDevice failed");
    if (!scratch_resolve(device) && (flags & S2W_PLAN_NO_WORKSPACE))
        return fail(S2W_EHIP, "hipGetSymbolAddress of the static scratch failed");

    s2w_plan p = new (std::nothrow) s2w_plan_s;
    if (!p) return fail(S2W_ENOMEM, "host allocation failed");
    p->L = L; p->N = N; p->J0 = J0; p->J = S.J; p->B = batch; p->device = device;
    p->lambda = lambda; p->prec = precision;
    p->cplx = cplx; p->spin = cplx ? spin : 0;
    p->S = S;
    p->Lphi = S.Lphi;
    s2w::make_filters(p->S, p->F);

    auto oom = [&](const char *what) {
        free_plan(p);
        delete p;
        return fail(S2W_ENOMEM, std::string("device allocation failed: ") + what);
    };

    // layout
    const int K = (int)S.s.size();
    p->wav_off.assign(K + 1, 0);
    for (int k = 0; k < K; ++k)
        p->wav_off[k + 1] = p->wav_off[k] + (int64_t)batch * (2 * S.s[k].N - 1) * S.s[k].L * (2 * S.s[k].L - 1);

    // global n list: top scale's n values plus n = 0 (and, for the standalone SO(3)
    // transforms, every |n| < N)
    p->nglob = S.s.back().n;
    if (std::find(p->nglob.begin(), p->nglob.end(), 0) == p->nglob.end()) p->nglob.push_back(0);
    if (cplx)
        for (int n : {-spin, spin})
            if (std::find(p->nglob.begin(), p->nglob.end(), n) == p->nglob.end()) p->nglob.push_back(n);
    p->wigner = (flags & S2W_PLAN_WIGNER) != 0;
    if (p->wigner)
        for (int n = -(N - 1); n <= N - 1; ++n)
            if (std::find(p->nglob.begin(), p->nglob.end(), n) == p->nglob.end()) p->nglob.push_back(n);

    // grids
    if (!make_grid(p, L) || !make_grid(p, p->Lphi)) return oom("grid tables");
    for (int k = 0; k < K; ++k) {
        if (!make_grid(p, S.s[k].L)) return oom("grid tables");
        if (!make_gamma_tw(p, 2 * S.s[k].N - 1)) return oom("gamma twiddles");
    }
    if (!make_gamma_tw(p, 1)) return oom("gamma twiddles");
    {
        s2w::RecTables R;
        s2w::rec_tables(L, p->nglob, R);
        if (!upload(p, p->A, R.A) || !upload(p, p->Bt, R.B) || !upload(p, p->S_, R.S) ||
            !upload(p, p->smant, R.start_mant) || !upload(p, p->sexp, R.start_exp))
            return oom("recursion tables");
    }
    // weights
    {
        std::vector<double> ws(L), wp(p->Lphi);
        for (int l = 0; l < L; ++l) ws[l] = sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
        for (int l = 0; l < p->Lphi; ++l) wp[l] = p->F.phi[l];
        if (!upload(p, p->wsht, ws) || !upload(p, p->wphi, wp)) return oom("weights");
        if (p->wigner) {
            std::vector<double> w8(L), w1(L, 1.0);
            for (int l = 0; l < L; ++l) w8[l] = (2.0 * l + 1.0) / (8.0 * M_PI * M_PI);
            if (!upload(p, p->w8pi, w8) || !upload(p, p->wone, w1)) return oom("weights");
        }
        p->wpsi.assign(K, nullptr);
        p->lmin.assign(K, 0);
        for (int k = 0; k < K; ++k) {
            const int Lk = S.s[k].L, nn = (int)S.s[k].n.size();
            std::vector<double> w((size_t)nn * Lk);
            int lm = Lk;
            for (int i = 0; i < nn; ++i)
                for (int l = 0; l < Lk; ++l) {
                    w[(size_t)i * Lk + l] = p->F.psi_mag[k][(size_t)l * nn + i];
                    if (w[(size_t)i * Lk + l] != 0.0) lm = std::min(lm, l);
                }
            p->lmin[k] = lm;
            if (!upload(p, p->wpsi[k], w)) return oom("weights");
        }
    }
    // scale groups (same grid)
    for (int k = 0; k < K; ++k) {
        if (!p->groups.empty() && p->groups.back().L == S.s[k].L && p->groups.back().scales.size() < 2)
            p->groups.back().scales.push_back(k);
        else {
            Group g;
            g.L = S.s[k].L;
            g.scales.push_back(k);
            p->groups.push_back(g);
        }
    }
    // workspace
    {
        size_t a = (size_t)batch * L * L * 2 * 2;   // SHT stages
        size_t bsz = a, c = a;
        for (auto &g : p->groups) {
            const int Lk = g.L, NS = (int)g.scales.size();
            const int nn = (int)S.s[g.scales[0]].n.size(), ng = 2 * S.s[g.scales[0]].N - 1;
            const size_t cbuf = (size_t)NS * batch * nn * Lk * Lk * 2;   // lsum out / sigma rows
            const size_t ebuf = (size_t)batch * ng * Lk * Lk * 2;        // rows over m
            a = std::max(a, std::max(cbuf, ebuf));
            bsz = std::max(bsz, std::max(cbuf, ebuf));
            c = std::max(c, cbuf);
        }
        p->szA = a; p->szB = bsz; p->szC = c;
        p->P.assign(K, nullptr);
        p->ws = {{&p->bufA, a}, {&p->bufB, bsz}, {&p->bufC, c}, {&p->flm, (size_t)batch * L * L * 2},
                 {&p->fhat, (size_t)batch * L * L * 2}};
        for (int k = 0; k < K; ++k) {
            const int Lk = S.s[k].L, nn = (int)S.s[k].n.size();
            p->ws.push_back({&p->P[k], (size_t)batch * Lk * nn * Lk * 2});
        }
        p->ws.push_back({&p->Pphi, (size_t)batch * p->Lphi * p->Lphi * 2});
        if (p->wigner) p->ws.push_back({&p->wint, (size_t)batch * (2 * N - 1) * L * L * 2});
        for (auto &it : p->ws) p->ws_bytes += (it.second * sizeof(double) + 255) / 256 * 256;
        p->no_ws = (flags & S2W_PLAN_NO_WORKSPACE) != 0;
        if (!p->no_ws)
            for (auto &it : p->ws)
                if (!dalloc(p, *it.first, it.second)) return oom("workspace");
    }
    if ((flags & S2W_PLAN_PRECOMPUTE) && !make_dtables(p)) return oom("precomputed d tables");
    if ((flags & S2W_PLAN_PRECOMPUTE) && precision == S2W_MIXED && !make_ttables(p))
        return oom("precomputed contraction tables");
    if ((flags & S2W_PLAN_PRECOMPUTE) && !p->no_ws && !make_shttab(p)) return oom("precomputed SHT table");
    if ((flags & S2W_PLAN_PERSISTENT) && precision == S2W_MIXED && !p->no_ws) {
        if (!build_lsum_list(p)) return oom("work list");
        p->lsum_list = true;
    }
    if (flags & S2W_PLAN_TUNE) autotune(p);
    p->graph = (flags & S2W_PLAN_GRAPH) != 0;
    if (hipEventCreateWithFlags(&p->order_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        delete p;
        return fail(S2W_EHIP, "event creation failed during plan creation");
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipEventDestroy(p->order_ev);
        free_plan(p);
        delete p;
        return fail(S2W_EHIP, "device synchronisation failed during plan creation");
    }
    reg_add(p);
    *out = p;
    return S2W_OK;
}

s2w_status s2w_plan_create(s2w_plan *out, int L, int N, double lambda, int J0, int batch,
                           s2w_precision precision, int device, unsigned flags)
{
    return plan_create(out, L, N, lambda, J0, batch, precision, device, flags, false, 0);
}

s2w_status s2w_plan_create_spin(s2w_plan *out, int L, int N, double lambda, int J0, int spin, int batch,
                                s2w_precision precision, int device, unsigned flags)
{
    return plan_create(out, L, N, lambda, J0, batch, precision, device, flags, true, spin);
}

s2w_status s2w_plan_destroy(s2w_plan p)
{
    if (!p) return S2W_OK;
    if (!reg_remove(p)) return fail(S2W_ESTATE, "not a live plan (destroyed twice, or never created)");
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (auto &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (auto e : p->ev0) (void)hipEventDestroy(e);
    for (auto e : p->ev1) (void)hipEventDestroy(e);
    if (p->order_ev) (void)hipEventDestroy(p->order_ev);
    free_plan(p);
    delete p;
    return S2W_OK;
}

s2w_status s2w_plan_layout(s2w_plan p, int *nscales, int *J0, int *Lk, int *Nk, int64_t *wav_offset, int *L_phi)
{
    if (s2w_status st = check_plan(p)) return st;
    const int K = (int)p->S.s.size();
    if (nscales) *nscales = K;
    if (J0) *J0 = p->J0;
    for (int k = 0; k < K; ++k) {
        if (Lk) Lk[k] = p->S.s[k].L;
        if (Nk) Nk[k] = p->S.s[k].N;
    }
    if (wav_offset)
        for (int k = 0; k <= K; ++k) wav_offset[k] = p->wav_off[k];
    if (L_phi) *L_phi = p->Lphi;
    return S2W_OK;
}

s2w_status s2w_sht_forward(s2w_plan p, const double *f, double *flm, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (!f || !flm) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    sht_forward_internal(p, f, p->flm, st);
    s2w::launch_flm_to_ext(p->flm, flm, p->L, p->B, st);
    return post_launch("s2w_sht_forward");
}

s2w_status s2w_sht_inverse(s2w_plan p, const double *flm, double *f, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (!f || !flm) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    s2w::launch_flm_from_ext(flm, p->flm, p->L, p->B, st);
    sht_inverse_internal(p, p->flm, f, st);
    return post_launch("s2w_sht_inverse");
}

// Scaling and wavelet coefficients from harmonic coefficients flm (internal
// layout [B][L][L], m-major); the scaling part is skipped when scal is null.
static void analysis_from_flm(s2w_plan p, const double *flm, void *wav_, double *scal, hipStream_t st)
{
    double *wav = (double *)wav_;
    const int B = p->B;
    const bool mixed = p->prec == S2W_MIXED;
    // scaling coefficients: W^Phi = Y^{-1}_{L_phi}(Phi f)
    if (scal) {
        const DevGrid &g = p->grids[p->Lphi];
        const int Lp = p->Lphi;
        std::vector<int> n0{0};
        LsumArgs la = lsum_args(p, g, Lp, n0);
        la.flm = flm;
        la.flm_m = p->L;
        la.flm_l = p->L;
        la.w[0] = p->wphi;
        la.wstride = 0;
        la.out[0] = p->bufA;
        { Prof pr_(p, "lsum", rec_work_n0(p, p->wphi, la.L, la.mcount, B), st); s2w::launch_lsum(la, 1, B, st); }
        GammaArgs ga = gamma_args(p, Lp, Lp, Lp, Lp, n0, 1);
        ga.src = p->bufA;
        ga.dst = p->bufB;
        { Prof pr_(p, "gamma_c2r", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_c2r(ga, st); }
        { const DftArgs da_ = dft_args(g, p->bufB, Lp, scal, 2 * Lp - 1, B * Lp, 1.0); Prof pr_(p, "dft_c2r", dft_flop(da_.n, da_.nrows), st); s2w::launch_dft_c2r(da_, st); }
    }
    // wavelet scales
    if (mixed) {
        float *wav32 = (float *)wav_;
        float *A32 = (float *)p->bufA, *B32 = (float *)p->bufB;
        const bool listed = p->lsum_list && p->B == p->list_B;
        if (listed) {
            const s2w::LsumList gl = lsum_list_args(p, flm);
            Work wk;
            for (int k = 0; k < gl.ngroups; ++k) {
                const auto &grp = p->groups[p->lgroups[k]];
                const Work w1 = rec_work_psi(p, grp.scales, grp.L, grp.L, p->S.s[grp.scales[0]].n, B);
                wk.flop += w1.flop;
                wk.flop64 += w1.flop64;
            }
            Prof pr_(p, "lsum_mm", wk, st);
            s2w::launch_lsum_list(gl, p->items, p->counters, p->list_blocks, st);
        }
        for (size_t gi = 0; gi < p->groups.size(); ++gi) {
            const auto &grp = p->groups[gi];
            // output offset of a group computed by the persistent launch (else 0: computed here)
            size_t goff = listed ? p->list_end : 0;
            bool done = false;
            if (listed)
                for (size_t k = 0; k < p->lgroups.size(); ++k)
                    if (p->lgroups[k] == (int)gi) { goff = p->lgroup_off[k]; done = true; }
            const DevGrid &g = p->grids[grp.L];
            const int Lk = grp.L, NS = (int)grp.scales.size();
            const auto &si = p->S.s[grp.scales[0]];
            const int nn = (int)si.n.size(), ng = 2 * si.N - 1;
            LsumArgs la = lsum_args(p, g, Lk, si.n);
            la.flm = flm;
            la.flm_m = p->L;
            la.flm_l = p->L;
            la.wstride = Lk;
            const size_t cstride = (size_t)B * nn * Lk * Lk * 2;   // floats
            s2w::MixOut mo{};
            mo.B = B;
            for (int s = 0; s < NS; ++s) {
                la.w[s] = p->wpsi[grp.scales[s]];
                la.lmin[s] = p->lmin[grp.scales[s]];
                la.out[s] = p->bufC + s * cstride;
                mo.out[s] = A32 + goff + s * cstride;
            }
            if (done) {
                // computed by the persistent launch
            } else if (lsum_vector(p, Lk)) {
                { Prof pr_(p, "lsum", rec_work_psi(p, grp.scales, la.L, la.mcount, si.n, B), st); s2w::launch_lsum(la, NS, B, st); }
                { Prof pr_(p, "convert", 0.0, st); s2w::launch_convert(p->bufC, A32 + goff, NS * cstride, true, st); }
            } else {
                Prof pr_(p, "lsum_mm", rec_work_psi(p, grp.scales, la.L, la.mcount, si.n, B), st);
                s2w::launch_lsum_mm(la, mo, NS, st);
            }
            for (int s = 0; s < NS; ++s) {
                const int k = grp.scales[s];
                GammaArgs ga = gamma_args(p, Lk, Lk, Lk, Lk, si.n, ng);
                ga.src = A32 + goff + s * cstride;
                ga.dst = B32;
                if (p->F.xi_imag) { ga.phr = 0.0; ga.phi = -1.0; }
                {
                    Prof pr_(p, "gamma_c2r_f32", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st);
                    s2w::launch_gamma_c2r(ga, st, true);
                }
                const DftArgs da = dft_args(g, B32, Lk, wav32 + p->wav_off[k], 2 * Lk - 1, B * ng * Lk, 1.0);
                Prof pr_(p, "dft_c2r_f32", dft_flop(da.n, da.nrows), st);
                s2w::launch_dft_c2r(da, st, true);
            }
        }
        return;
    }
    for (auto &grp : p->groups) {
        const DevGrid &g = p->grids[grp.L];
        const int Lk = grp.L, NS = (int)grp.scales.size();
        const auto &si = p->S.s[grp.scales[0]];
        const int nn = (int)si.n.size(), ng = 2 * si.N - 1;
        LsumArgs la = lsum_args(p, g, Lk, si.n);
        la.flm = flm;
        la.flm_m = p->L;
        la.flm_l = p->L;
        la.wstride = Lk;
        const size_t cstride = (size_t)B * nn * Lk * Lk * 2;
        for (int s = 0; s < NS; ++s) {
            la.w[s] = p->wpsi[grp.scales[s]];
            la.out[s] = p->bufA + s * cstride;
        }
        { Prof pr_(p, "lsum", rec_work_psi(p, grp.scales, la.L, la.mcount, si.n, B), st); s2w::launch_lsum(la, NS, B, st); }
        for (int s = 0; s < NS; ++s) {
            const int k = grp.scales[s];
            GammaArgs ga = gamma_args(p, Lk, Lk, Lk, Lk, si.n, ng);
            ga.src = p->bufA + s * cstride;
            ga.dst = p->bufB;
            if (p->F.xi_imag) { ga.phr = 0.0; ga.phi = -1.0; }   // conj(xi) = -i
            { Prof pr_(p, "gamma_c2r", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_c2r(ga, st); }
            { const DftArgs da_ = dft_args(g, p->bufB, Lk, wav + p->wav_off[k], 2 * Lk - 1, B * ng * Lk, 1.0); Prof pr_(p, "dft_c2r", dft_flop(da_.n, da_.nrows), st); s2w::launch_dft_c2r(da_, st); }
        }
    }
    }

s2w_status s2w_analysis(s2w_plan p, const double *f, void *wav_, double *scal, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (!f || !wav_ || !scal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    // the forward SHT of the input map runs in FP64 in both forms: it is shared by every
    // scale, and FP32 rounding here would spread as white noise across all degrees
    if (p->graph && !p->capturing)
        return run_graph(p, 0, f, wav_, scal, st, [&](hipStream_t cs) {
            sht_forward_internal(p, f, p->flm, cs);
            analysis_from_flm(p, p->flm, wav_, scal, cs);
        });
    sht_forward_internal(p, f, p->flm, st);
    analysis_from_flm(p, p->flm, wav_, scal, st);
    return post_launch("s2w_analysis");
}

// Points the plan's workspace buffers at consecutive 256-byte aligned slices of the
// device scratch while the scope lives (kernel arguments are taken at launch, so the
// plan's own pointers are restored on exit).
struct ScratchScope {
    s2w_plan p;
    std::vector<double *> saved;
    ScratchScope(s2w_plan p_, unsigned char *base) : p(p_)
    {
        size_t off = 0;
        for (auto &it : p->ws) {
            saved.push_back(*it.first);
            *it.first = reinterpret_cast<double *>(base + off);
            off += (it.second * sizeof(double) + 255) / 256 * 256;
        }
    }
    ~ScratchScope()
    {
        for (size_t i = 0; i < saved.size(); ++i) *p->ws[i].first = saved[i];
    }
};

s2w_status s2w_analysis_noalloc(s2w_plan p, const double *f, void *wav_, double *scal, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (p->cplx) return fail(S2W_ESTATE, "plan made for complex spin maps: use the s2w_spin_* calls");
    if (!f || !wav_ || !scal) return fail(S2W_EINVAL, "null buffer");
    if (p->ws_bytes > S2W_SCRATCH_BYTES)
        return fail(S2W_EUNSUPPORTED, "this plan needs " + std::to_string(p->ws_bytes) +
                                          " bytes of workspace, more than the static scratch (" +
                                          std::to_string((size_t)S2W_SCRATCH_BYTES) + " bytes)");
    unsigned char *base = scratch_ptr(p->device);
    if (!base) return fail(S2W_ESTATE, "the device scratch address was not resolved at plan creation");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    ScratchScope sc(p, base);
    sht_forward_internal(p, f, p->flm, st);
    analysis_from_flm(p, p->flm, wav_, scal, st);
    return post_launch("s2w_analysis_noalloc");
}

// Harmonic coefficients fhat (internal layout) of the synthesis before the
// final inverse SHT; the scaling part is left out when scal is null.
static void synthesis_to_fhat(s2w_plan p, const void *wav_, const double *scal, double *fhat, hipStream_t st)
{
    const double *wav = (const double *)wav_;
    const int B = p->B;
    const int npar = (p->N - 1) & 1;
    const bool mixed = p->prec == S2W_MIXED;
    std::vector<int> p32(p->S.s.size(), 0);   // scales whose P the folded-table product wrote in FP32
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        if (!mixed) continue;
        const auto &grp = p->groups[gi];
        const auto tti = p->ttabs.find((int)gi);
        const bool tab = tti != p->ttabs.end();
        const float *wav32 = (const float *)wav_;
        float *A32 = (float *)p->bufA, *B32 = (float *)p->bufB, *C32 = (float *)p->bufC;
        const DevGrid &g = p->grids[grp.L];
        const int Lk = grp.L, NS = (int)grp.scales.size();
        const auto &si = p->S.s[grp.scales[0]];
        const int nn = (int)si.n.size(), ng = 2 * si.N - 1;
        const size_t cstride = (size_t)B * nn * Lk * Lk * 2;   // floats
        TsumArgs ta = tsum_args(p, g, Lk, si.n, npar);
        ta.wstride = Lk;
        s2w::MixIn mi{};
        mi.B = B;
        for (int s = 0; s < NS; ++s) {
            const int k = grp.scales[s];
            {
                const DftArgs da = dft_args(g, wav32 + p->wav_off[k], 2 * Lk - 1, B32, Lk, B * ng * Lk, 1.0);
                Prof pr_(p, "dft_r2c_f32", dft_flop(da.n, da.nrows), st);
                s2w::launch_dft_r2c(da, st, true, false);
            }
            GammaArgs ga = gamma_args(p, Lk, Lk, Lk, Lk, si.n, ng);
            ga.src = B32;
            ga.dst = A32 + s * cstride;
            ga.sgn = -1.0;
            ga.wscale = (2.0 * M_PI / (2 * Lk - 1)) * (2.0 * M_PI / ng);
            ga.npar = npar;
            sig_counts(Lk, npar, ga.M0, ga.M1);
            {
                Prof pr_(p, "gamma_r2c_f32", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st);
                s2w::launch_gamma_r2c(ga, st, true);
            }
            if (!tab) theta_quadrature32(p, g, A32 + s * cstride, C32 + s * cstride, Lk, nn, npar, st);
            ta.w[s] = p->wpsi[k];
            ta.lmin[s] = p->lmin[k];
            mi.h[s] = C32 + s * cstride;
            mi.out[s] = p->P[k];
            ta.h[s] = p->bufA + s * cstride;
            ta.out[s] = p->P[k];
        }
        if (tab) {
            // precompute mode: quadrature and contraction through the folded table
            const auto &tt = tti->second;
            s2w::TsumTab tb{};
            tb.L = Lk;
            tb.mcount = Lk;
            tb.nn = nn;
            tb.B = B;
            tb.NS = NS;
            tb.npar = npar;
            sig_counts(Lk, npar, tb.M0, tb.M1);
            for (int i = 0; i < nn; ++i) tb.nval[i] = si.n[i];
            for (int s = 0; s < NS; ++s) {
                tb.h[s] = A32 + s * cstride;
                tb.out[s] = reinterpret_cast<float *>(p->P[grp.scales[s]]);
                tb.w[s] = p->wpsi[grp.scales[s]];
                p32[grp.scales[s]] = 1;
            }
            tb.wstride = Lk;
            tb.tab = tt.tab;
            tb.toff = tt.toff;
            tb.tiles = tt.tiles;
            for (int x = 0; x < 8; ++x) {
                tb.cnt[x] = tt.cnt[x];
                tb.off[x] = tt.off[x];
            }
            Work wk = rec_work_psi(p, grp.scales, ta.L, ta.mcount, si.n, B);
            wk.flop -= wk.flop64;   // no recursion: d comes from the table
            wk.flop64 = 0.0;
            Prof pr_(p, "tsum_tab", wk, st);
            s2w::launch_tsum_tab(tb, st);
        } else if (tsum_vector(p, Lk)) {
            // the quadrature rows of every scale are no longer needed in A32: widen them there
            { Prof pr_(p, "convert", 0.0, st); s2w::launch_convert(C32, p->bufA, NS * cstride, false, st); }
            Prof pr_(p, "tsum", rec_work_psi(p, grp.scales, ta.L, ta.mcount, si.n, B), st);
            s2w::launch_tsum(ta, NS, B, st);
        } else {
            Prof pr_(p, "tsum_mm", rec_work_psi(p, grp.scales, ta.L, ta.mcount, si.n, B), st);
            s2w::launch_tsum_mm(ta, mi, NS, st);
        }
    }
    for (auto &grp : p->groups) {
        if (mixed) continue;
        const DevGrid &g = p->grids[grp.L];
        const int Lk = grp.L, NS = (int)grp.scales.size();
        const auto &si = p->S.s[grp.scales[0]];
        const int nn = (int)si.n.size(), ng = 2 * si.N - 1;
        const size_t cstride = (size_t)B * nn * Lk * Lk * 2;
        TsumArgs ta = tsum_args(p, g, Lk, si.n, npar);
        ta.wstride = Lk;
        for (int s = 0; s < NS; ++s) {
            const int k = grp.scales[s];
            { const DftArgs da_ = dft_args(g, wav + p->wav_off[k], 2 * Lk - 1, p->bufB, Lk, B * ng * Lk, 1.0); Prof pr_(p, "dft_r2c", dft_flop(da_.n, da_.nrows), st); s2w::launch_dft_r2c(da_, st); }
            GammaArgs ga = gamma_args(p, Lk, Lk, Lk, Lk, si.n, ng);
            ga.src = p->bufB;
            ga.dst = p->bufA + s * cstride;
            ga.sgn = -1.0;
            ga.wscale = (2.0 * M_PI / (2 * Lk - 1)) * (2.0 * M_PI / ng);
            ga.npar = npar;
            sig_counts(Lk, npar, ga.M0, ga.M1);
            { Prof pr_(p, "gamma_r2c", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_r2c(ga, st); }
            theta_quadrature(p, g, p->bufA + s * cstride, p->bufC + s * cstride, Lk, nn, npar, st);
            ta.h[s] = p->bufC + s * cstride;
            ta.w[s] = p->wpsi[k];
            ta.out[s] = p->P[k];
        }
        { Prof pr_(p, "tsum", rec_work_psi(p, grp.scales, ta.L, ta.mcount, si.n, B), st); s2w::launch_tsum(ta, NS, B, st); }
    }
    // scaling: Phi * Y(W^Phi)
    if (scal) {
        const DevGrid &g = p->grids[p->Lphi];
        const int Lp = p->Lphi;
        std::vector<int> n0{0};
        { const DftArgs da_ = dft_args(g, scal, 2 * Lp - 1, p->bufB, Lp, B * Lp, 2.0 * M_PI / (2 * Lp - 1)); Prof pr_(p, "dft_r2c", dft_flop(da_.n, da_.nrows), st); s2w::launch_dft_r2c(da_, st); }
        GammaArgs ga = gamma_args(p, Lp, Lp, Lp, Lp, n0, 1);
        ga.src = p->bufB;
        ga.dst = p->bufA;
        ga.sgn = -1.0;
        sig_counts(Lp, 0, ga.M0, ga.M1);
        { Prof pr_(p, "gamma_r2c", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_r2c(ga, st); }
        theta_quadrature(p, g, p->bufA, p->bufC, Lp, 1, 0, st);
        TsumArgs ta = tsum_args(p, g, Lp, n0, 0);
        ta.h[0] = p->bufC;
        ta.w[0] = p->wphi;
        ta.wstride = 0;
        ta.out[0] = p->Pphi;
        { Prof pr_(p, "tsum", rec_work_n0(p, p->wphi, ta.L, ta.mcount, B), st); s2w::launch_tsum(ta, 1, B, st); }
    }
    CombineArgs ca{};
    ca.out = fhat;
    ca.L = p->L;
    ca.nterms = 0;
    for (size_t k = 0; k < p->S.s.size(); ++k) {
        auto &t = ca.t[ca.nterms++];
        t.P = p->P[k];
        t.f32 = p32[k];
        t.L = p->S.s[k].L;
        t.nn = (int)p->S.s[k].n.size();
        t.phr = p->F.xi_imag ? 0.0 : 1.0;
        t.phi = p->F.xi_imag ? 1.0 : 0.0;
    }
    if (scal) {
        auto &t = ca.t[ca.nterms++];
        t.P = p->Pphi;
        t.L = p->Lphi;
        t.nn = 1;
        t.phr = 1.0;
        t.phi = 0.0;
    }
    { Prof pr_(p, "combine", 0.0, st); s2w::launch_combine(ca, B, st); }
}

s2w_status s2w_synthesis(s2w_plan p, const void *wav_, const double *scal, double *f, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (!f || !wav_ || !scal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    if (p->graph && !p->capturing)
        return run_graph(p, 1, wav_, scal, f, st, [&](hipStream_t cs) {
            synthesis_to_fhat(p, wav_, scal, p->fhat, cs);
            sht_inverse_internal(p, p->fhat, f, cs);
        });
    synthesis_to_fhat(p, wav_, scal, p->fhat, st);
    sht_inverse_internal(p, p->fhat, f, st);
    return post_launch("s2w_synthesis");
}

// ---- transposes (gradients) -----------------------------------------------
// Each stage below is the transpose, under the real inner product of the stored
// real and imaginary parts, of a stage of the forward maps; the internal harmonic
// arrays [B][m >= 0][l] carry cotangents of their stored entries (l >= m).

// Transpose of Y^{-1} on the grid of band limit Lg with degree weights wt (n = 0):
// map cotangent [B][Lg][2Lg-1] -> out [B][Lg][1][Lg] (defined at l >= m).  The
// transpose of the Hermitian c2r is an unweighted r2c with the m >= 1 terms doubled;
// the sum over theta is taken against d directly (no quadrature matrix).
static void sht_inverse_T(s2w_plan p, int Lg, const double *wt, const double *gmap, double *out, hipStream_t st)
{
    const DevGrid &g = p->grids[Lg];
    const int B = p->B;
    std::vector<int> n0{0};
    {
        const DftArgs da_ = dft_args(g, gmap, 2 * Lg - 1, p->bufB, Lg, B * Lg, 1.0);
        Prof pr_(p, "dft_r2c", dft_flop(da_.n, da_.nrows), st);
        s2w::launch_dft_r2c(da_, st);
    }
    GammaArgs ga = gamma_args(p, Lg, Lg, Lg, Lg, n0, 1);
    ga.src = p->bufB;
    ga.dst = p->bufA;
    ga.sgn = -1.0;
    ga.fm0 = 1.0;
    ga.fm1 = 2.0;
    sig_counts(Lg, 0, ga.M0, ga.M1);
    { Prof pr_(p, "gamma_r2c", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_r2c(ga, st); }
    TsumArgs ta = tsum_args(p, g, Lg, n0, 0);
    ta.h[0] = p->bufA;
    ta.w[0] = wt;
    ta.wstride = 0;
    ta.out[0] = out;
    { Prof pr_(p, "tsum", rec_work_n0(p, wt, ta.L, ta.mcount, B), st); s2w::launch_tsum(ta, 1, B, st); }
}

// Transpose of the forward SHT (Y, weights wt) on the grid of band limit Lg: cotangent
// of an internal harmonic array ([B][flm_m][flm_l], read at m <= l < Lg) -> map
// cotangent [B][Lg][2Lg-1].  Sum over l against d (n = 0), the quadrature matrix
// (symmetric, so its own transpose), then the transpose of the weighted phi r2c: a
// c2r with the m >= 1 terms halved.
static void sht_forward_T(s2w_plan p, int Lg, const double *wt, const double *flm, int flm_m, int flm_l,
                          double *gmap, hipStream_t st)
{
    const DevGrid &g = p->grids[Lg];
    const int B = p->B, na = 2 * Lg - 1;
    std::vector<int> n0{0};
    LsumArgs la = lsum_args(p, g, Lg, n0);
    la.flm = flm;
    la.flm_m = flm_m;
    la.flm_l = flm_l;
    la.w[0] = wt;
    la.wstride = 0;
    la.out[0] = p->bufA;
    { Prof pr_(p, "lsum", rec_work_n0(p, wt, la.L, la.mcount, B), st); s2w::launch_lsum(la, 1, B, st); }
    int M0, M1;
    sig_counts(Lg, 0, M0, M1);
    { Prof pr_(p, "pack_sigma", 0.0, st); s2w::launch_pack_sigma(p->bufA, p->bufB, B, 1, Lg, Lg, 0, M0, M1, 0, st); }
    theta_quadrature(p, g, p->bufB, p->bufC, Lg, 1, 0, st);
    { Prof pr_(p, "pack_sigma", 0.0, st); s2w::launch_pack_sigma(p->bufC, p->bufA, B, 1, Lg, Lg, 0, M0, M1, 1, st); }
    GammaArgs ga = gamma_args(p, Lg, Lg, Lg, Lg, n0, 1);
    ga.src = p->bufA;
    ga.dst = p->bufB;
    ga.fm0 = 1.0;
    ga.fm1 = 0.5;
    { Prof pr_(p, "gamma_c2r", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_c2r(ga, st); }
    {
        const DftArgs da_ = dft_args(g, p->bufB, Lg, gmap, na, B * Lg, 2.0 * M_PI / na);
        Prof pr_(p, "dft_c2r", dft_flop(da_.n, da_.nrows), st);
        s2w::launch_dft_c2r(da_, st);
    }
}

// Transpose of analysis_from_flm: cotangents of the wavelet coefficients (and of the
// scaling coefficients when gscal is not null) -> cotangent of the internal harmonic
// array fhat [B][L][L].  Per scale: unweighted r2c over alpha (m >= 1 doubled), the
// gamma sum with the filter phase xi, the sum over theta against d with the filter
// weights (d recomputed, no quadrature matrix); FP64 sum over n and scales.  Mixed
// plans take FP32 cotangents and run the DFTs and the theta sum in the precision split
// of their forward maps (FP32 matrix cores, FP64 recursion and sums).
static void analysis_from_flm_T(s2w_plan p, const void *gwav_, const double *gscal, double *fhat, hipStream_t st)
{
    const bool mixed = p->prec == S2W_MIXED;
    const int B = p->B;
    const int npar = (p->N - 1) & 1;
    for (auto &grp : p->groups) {
        const DevGrid &g = p->grids[grp.L];
        const int Lk = grp.L, NS = (int)grp.scales.size();
        const auto &si = p->S.s[grp.scales[0]];
        const int nn = (int)si.n.size(), ng = 2 * si.N - 1;
        const size_t cstride = (size_t)B * nn * Lk * Lk * 2;   // elements of the coefficient type
        TsumArgs ta = tsum_args(p, g, Lk, si.n, npar);
        ta.wstride = Lk;
        s2w::MixIn mi{};
        mi.B = B;
        for (int s = 0; s < NS; ++s) {
            const int k = grp.scales[s];
            GammaArgs ga = gamma_args(p, Lk, Lk, Lk, Lk, si.n, ng);
            ga.sgn = -1.0;
            ga.fm0 = 1.0;
            ga.fm1 = 2.0;
            if (p->F.xi_imag) { ga.phr = 0.0; ga.phi = 1.0; }   // xi = i
            ga.npar = npar;
            sig_counts(Lk, npar, ga.M0, ga.M1);
            if (mixed) {
                const float *gw32 = (const float *)gwav_ + p->wav_off[k];
                float *A32 = (float *)p->bufA, *B32 = (float *)p->bufB;
                {
                    const DftArgs da = dft_args(g, gw32, 2 * Lk - 1, B32, Lk, B * ng * Lk, 1.0);
                    Prof pr_(p, "dft_r2c_f32", dft_flop(da.n, da.nrows), st);
                    s2w::launch_dft_r2c(da, st, true, false);
                }
                ga.src = B32;
                ga.dst = A32 + s * cstride;
                { Prof pr_(p, "gamma_r2c_f32", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_r2c(ga, st, true); }
                ta.w[s] = p->wpsi[k];
                ta.lmin[s] = p->lmin[k];
                mi.h[s] = A32 + s * cstride;
                mi.out[s] = p->P[k];
                ta.h[s] = p->bufC + s * cstride;
                ta.out[s] = p->P[k];
            } else {
                const double *gw = (const double *)gwav_ + p->wav_off[k];
                {
                    const DftArgs da_ = dft_args(g, gw, 2 * Lk - 1, p->bufB, Lk, B * ng * Lk, 1.0);
                    Prof pr_(p, "dft_r2c", dft_flop(da_.n, da_.nrows), st);
                    s2w::launch_dft_r2c(da_, st);
                }
                ga.src = p->bufB;
                ga.dst = p->bufA + s * cstride;
                { Prof pr_(p, "gamma_r2c", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_r2c(ga, st); }
                ta.h[s] = p->bufA + s * cstride;
                ta.w[s] = p->wpsi[k];
                ta.out[s] = p->P[k];
            }
        }
        if (mixed && tsum_vector(p, Lk)) {
            { Prof pr_(p, "convert", 0.0, st); s2w::launch_convert(p->bufA, p->bufC, NS * cstride, false, st); }
            Prof pr_(p, "tsum", rec_work_psi(p, grp.scales, ta.L, ta.mcount, si.n, B), st);
            s2w::launch_tsum(ta, NS, B, st);
        } else if (mixed) {
            Prof pr_(p, "tsum_mm", rec_work_psi(p, grp.scales, ta.L, ta.mcount, si.n, B), st);
            s2w::launch_tsum_mm(ta, mi, NS, st);
        } else {
            Prof pr_(p, "tsum", rec_work_psi(p, grp.scales, ta.L, ta.mcount, si.n, B), st);
            s2w::launch_tsum(ta, NS, B, st);
        }
    }
    if (gscal) sht_inverse_T(p, p->Lphi, p->wphi, gscal, p->Pphi, st);
    CombineArgs ca{};
    ca.out = fhat;
    ca.L = p->L;
    for (size_t k = 0; k < p->S.s.size(); ++k) {
        auto &t = ca.t[ca.nterms++];
        t.P = p->P[k];
        t.L = p->S.s[k].L;
        t.nn = (int)p->S.s[k].n.size();
        t.phr = 1.0;
        t.phi = 0.0;
    }
    if (gscal) {
        auto &t = ca.t[ca.nterms++];
        t.P = p->Pphi;
        t.L = p->Lphi;
        t.nn = 1;
        t.phr = 1.0;
        t.phi = 0.0;
    }
    { Prof pr_(p, "combine", 0.0, st); s2w::launch_combine(ca, B, st); }
}

// Transpose of synthesis_to_fhat: cotangent of the internal harmonic array fhat
// ([B][L][L], read at l >= m) -> cotangents of the wavelet coefficients (and of the
// scaling coefficients when gscal is not null).  Per scale: the sum over l against d
// with the filter weights (the transpose of the theta sum; the same fhat row serves
// every n, since the scale sum adds the n rows), the quadrature matrix, the gamma sum
// with conj(xi) and the alpha c2r, both with the forward DFT weights and the m >= 1
// terms halved.  Mixed plans run it in the precision split of the forward maps.
static void synthesis_to_fhat_T(s2w_plan p, const double *fhat, void *gwav_, double *gscal, hipStream_t st)
{
    const bool mixed = p->prec == S2W_MIXED;
    const int B = p->B;
    const int npar = (p->N - 1) & 1;
    for (auto &grp : p->groups) {
        const DevGrid &g = p->grids[grp.L];
        const int Lk = grp.L, NS = (int)grp.scales.size();
        const auto &si = p->S.s[grp.scales[0]];
        const int nn = (int)si.n.size(), ng = 2 * si.N - 1;
        const size_t cstride = (size_t)B * nn * Lk * Lk * 2;
        int M0, M1;
        sig_counts(Lk, npar, M0, M1);
        LsumArgs la = lsum_args(p, g, Lk, si.n);
        la.flm = fhat;
        la.flm_m = p->L;
        la.flm_l = p->L;
        la.wstride = Lk;
        if (mixed) {
            float *A32 = (float *)p->bufA, *B32 = (float *)p->bufB, *C32 = (float *)p->bufC;
            s2w::MixOut mo{};
            mo.B = B;
            for (int s = 0; s < NS; ++s) {
                la.w[s] = p->wpsi[grp.scales[s]];
                la.lmin[s] = p->lmin[grp.scales[s]];
                la.out[s] = p->bufC + s * cstride;
                mo.out[s] = A32 + s * cstride;
            }
            if (lsum_vector(p, Lk)) {
                { Prof pr_(p, "lsum", rec_work_psi(p, grp.scales, la.L, la.mcount, si.n, B), st); s2w::launch_lsum(la, NS, B, st); }
                { Prof pr_(p, "convert", 0.0, st); s2w::launch_convert(p->bufC, A32, NS * cstride, true, st); }
            } else {
                Prof pr_(p, "lsum_mm", rec_work_psi(p, grp.scales, la.L, la.mcount, si.n, B), st);
                s2w::launch_lsum_mm(la, mo, NS, st);
            }
            for (int s = 0; s < NS; ++s) {
                const int k = grp.scales[s];
                { Prof pr_(p, "pack_sigma_f32", 0.0, st); s2w::launch_pack_sigma_f32(A32 + s * cstride, C32, B, nn, Lk, Lk, npar, M0, M1, 0, st); }
                theta_quadrature32(p, g, C32, B32, Lk, nn, npar, st);
                { Prof pr_(p, "pack_sigma_f32", 0.0, st); s2w::launch_pack_sigma_f32(B32, C32, B, nn, Lk, Lk, npar, M0, M1, 1, st); }
                GammaArgs ga = gamma_args(p, Lk, Lk, Lk, Lk, si.n, ng);
                ga.src = C32;
                ga.dst = B32;
                ga.wscale = (2.0 * M_PI / (2 * Lk - 1)) * (2.0 * M_PI / ng);
                ga.fm0 = 1.0;
                ga.fm1 = 0.5;
                if (p->F.xi_imag) { ga.phr = 0.0; ga.phi = -1.0; }   // conj(xi) = -i
                { Prof pr_(p, "gamma_c2r_f32", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_c2r(ga, st, true); }
                const DftArgs da = dft_args(g, B32, Lk, (float *)gwav_ + p->wav_off[k], 2 * Lk - 1, B * ng * Lk, 1.0);
                Prof pr_(p, "dft_c2r_f32", dft_flop(da.n, da.nrows), st);
                s2w::launch_dft_c2r(da, st, true);
            }
        } else {
            for (int s = 0; s < NS; ++s) {
                la.w[s] = p->wpsi[grp.scales[s]];
                la.out[s] = p->bufA + s * cstride;
            }
            { Prof pr_(p, "lsum", rec_work_psi(p, grp.scales, la.L, la.mcount, si.n, B), st); s2w::launch_lsum(la, NS, B, st); }
            for (int s = 0; s < NS; ++s) {
                const int k = grp.scales[s];
                { Prof pr_(p, "pack_sigma", 0.0, st); s2w::launch_pack_sigma(p->bufA + s * cstride, p->bufC, B, nn, Lk, Lk, npar, M0, M1, 0, st); }
                theta_quadrature(p, g, p->bufC, p->bufB, Lk, nn, npar, st);
                { Prof pr_(p, "pack_sigma", 0.0, st); s2w::launch_pack_sigma(p->bufB, p->bufC, B, nn, Lk, Lk, npar, M0, M1, 1, st); }
                GammaArgs ga = gamma_args(p, Lk, Lk, Lk, Lk, si.n, ng);
                ga.src = p->bufC;
                ga.dst = p->bufB;
                ga.wscale = (2.0 * M_PI / (2 * Lk - 1)) * (2.0 * M_PI / ng);
                ga.fm0 = 1.0;
                ga.fm1 = 0.5;
                if (p->F.xi_imag) { ga.phr = 0.0; ga.phi = -1.0; }
                { Prof pr_(p, "gamma_c2r", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_c2r(ga, st); }
                const DftArgs da_ = dft_args(g, p->bufB, Lk, (double *)gwav_ + p->wav_off[k], 2 * Lk - 1, B * ng * Lk, 1.0);
                Prof pr_(p, "dft_c2r", dft_flop(da_.n, da_.nrows), st);
                s2w::launch_dft_c2r(da_, st);
            }
        }
    }
    if (gscal) sht_forward_T(p, p->Lphi, p->wphi, fhat, p->L, p->L, gscal, st);
}

s2w_status s2w_analysis_adjoint(s2w_plan p, const void *gwav_, const double *gscal, double *gf, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (!gf || !gwav_ || !gscal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    analysis_from_flm_T(p, gwav_, gscal, p->fhat, st);
    sht_forward_T(p, p->L, p->wsht, p->fhat, p->L, p->L, gf, st);
    return post_launch("s2w_analysis_adjoint");
}

s2w_status s2w_synthesis_adjoint(s2w_plan p, const double *gf, void *gwav_, double *gscal, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (!gf || !gwav_ || !gscal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    sht_inverse_T(p, p->L, p->wsht, gf, p->fhat, st);
    synthesis_to_fhat_T(p, p->fhat, gwav_, gscal, st);
    return post_launch("s2w_synthesis_adjoint");
}

s2w_status s2w_analysis_lm(s2w_plan p, const double *flm, void *wav_, double *scal, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (!flm || !wav_ || !scal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    if (p->graph && !p->capturing)
        return run_graph(p, 2, flm, wav_, scal, st, [&](hipStream_t cs) {
            s2w::launch_flm_from_ext(flm, p->flm, p->L, p->B, cs);
            analysis_from_flm(p, p->flm, wav_, scal, cs);
        });
    s2w::launch_flm_from_ext(flm, p->flm, p->L, p->B, st);
    analysis_from_flm(p, p->flm, wav_, scal, st);
    return post_launch("s2w_analysis_lm");
}

// ---- standalone SO(3) transforms of real functions (S2W_PLAN_WIGNER) --------------------
// Section 2.2, eq:inverse_wigner_transform and eq:forward_wigner_transform, at the plan's
// band limits (L, N), FP64: the same stages as a wavelet scale with every |n| < N and the
// degree weights (2l+1)/(8 pi^2) (inverse) or 1 (forward) in place of the filters.

// internal coefficients wint [B][2N-1][m][l] -> samples f [B][2N-1][L][2L-1]
static void wigner_inverse_internal(s2w_plan p, const double *cin, double *f, hipStream_t st)
{
    const DevGrid &g = p->grids[p->L];
    const int L = p->L, N = p->N, B = p->B, ng = 2 * N - 1;
    std::vector<int> nall;
    for (int n = -(N - 1); n <= N - 1; ++n) nall.push_back(n);
    LsumArgs la = lsum_args(p, g, L, nall);
    la.flm = cin;
    la.flm_m = ng * L;
    la.flm_l = L;
    la.flm_nstride = (long)L * L;
    la.w[0] = p->w8pi;
    la.wstride = 0;
    la.out[0] = p->bufA;
    { Prof pr_(p, "lsum", rec_work(L, L, nall, 1, B, [](int, int, int) { return 1.0; }), st); s2w::launch_lsum(la, 1, B, st); }
    GammaArgs ga = gamma_args(p, L, L, L, L, nall, ng);
    ga.src = p->bufA;
    ga.dst = p->bufB;
    { Prof pr_(p, "gamma_c2r", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_c2r(ga, st); }
    const DftArgs da_ = dft_args(g, p->bufB, L, f, 2 * L - 1, B * ng * L, 1.0);
    Prof pr_(p, "dft_c2r", dft_flop(da_.n, da_.nrows), st);
    s2w::launch_dft_c2r(da_, st);
}

// samples f [B][2N-1][L][2L-1] -> coefficients, external "nlm" layout [B][2N-1][L][2L-1]
// complex; the two parities of n run separately (the quadrature matrix depends on (-1)^(m+n))
static void wigner_forward_internal(s2w_plan p, const double *f, double *ext, hipStream_t st)
{
    const DevGrid &g = p->grids[p->L];
    const int L = p->L, N = p->N, B = p->B, ng = 2 * N - 1;
    {
        const DftArgs da_ = dft_args(g, f, 2 * L - 1, p->bufB, L, B * ng * L, 1.0);
        Prof pr_(p, "dft_r2c", dft_flop(da_.n, da_.nrows), st);
        s2w::launch_dft_r2c(da_, st);
    }
    double *Pout = p->P[p->S.s.size() - 1];
    for (int q = 0; q < 2; ++q) {
        std::vector<int> nq;
        for (int n = -(N - 1); n <= N - 1; ++n)
            if (((n % 2) + 2) % 2 == q) nq.push_back(n);
        if (nq.empty()) continue;
        GammaArgs ga = gamma_args(p, L, L, L, L, nq, ng);
        ga.src = p->bufB;
        ga.dst = p->bufA;
        ga.sgn = -1.0;
        ga.wscale = (2.0 * M_PI / (2 * L - 1)) * (2.0 * M_PI / ng);
        ga.npar = q;
        sig_counts(L, q, ga.M0, ga.M1);
        { Prof pr_(p, "gamma_r2c", 8.0 * ga.B * ga.M * ga.L * ga.ng * ga.nn, st); s2w::launch_gamma_r2c(ga, st); }
        theta_quadrature(p, g, p->bufA, p->bufC, L, (int)nq.size(), q, st);
        TsumArgs ta = tsum_args(p, g, L, nq, q);
        ta.h[0] = p->bufC;
        ta.w[0] = p->wone;
        ta.wstride = 0;
        ta.out[0] = Pout;
        { Prof pr_(p, "tsum", rec_work(L, L, nq, 1, B, [](int, int, int) { return 1.0; }), st); s2w::launch_tsum(ta, 1, B, st); }
        { Prof pr_(p, "wig_layout", 0.0, st); s2w::launch_wig_sum_to_ext(Pout, ext, L, N, B, (int)nq.size(), nq.data(), st); }
    }
}

static s2w_status check_wigner(s2w_plan p)
{
    if (!p->wigner) return fail(S2W_ESTATE, "plan created without S2W_PLAN_WIGNER");
    return S2W_OK;
}

s2w_status s2w_wigner_forward(s2w_plan p, const double *f, double *flmn, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (s2w_status st = check_wigner(p)) return st;
    if (!f || !flmn) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    wigner_forward_internal(p, f, flmn, st);
    return post_launch("s2w_wigner_forward");
}

s2w_status s2w_wigner_inverse(s2w_plan p, const double *flmn, double *f, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_ws(p)) return st;
    if (s2w_status st = check_wigner(p)) return st;
    if (!f || !flmn) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    s2w::launch_wig_ext_to_int(flmn, p->wint, p->L, p->N, p->B, st);
    wigner_inverse_internal(p, p->wint, f, st);
    return post_launch("s2w_wigner_inverse");
}

// ---- complex spin-s maps ----

s2w_status s2w_spin_sht_forward(s2w_plan p, const double *f, double *flm, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_spin(p)) return st;
    if (!f || !flm) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    spin_sht_forward_internal(p, f, nullptr, flm, st);
    return post_launch("s2w_spin_sht_forward");
}

s2w_status s2w_spin_sht_inverse(s2w_plan p, const double *flm, double *f, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_spin(p)) return st;
    if (!f || !flm) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    spin_sht_inverse_internal(p, nullptr, flm, f, st);
    return post_launch("s2w_spin_sht_inverse");
}

// The wavelet coefficients of a spin-s map depend on it only through its spin-s harmonic
// coefficients g_lm (eq:wigner_wav_coeffs, eq:harmonic_scal_coeffs, filters as for spin
// 0), and are linear in them: with g = A + i B for the real maps A, B, W(g) = W(A) + i W(B),
// where W(A) and W(B) are the real transforms of the plan's real machinery.
s2w_status s2w_spin_analysis(s2w_plan p, const double *f, void *wav, double *scal, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_spin(p)) return st;
    if (!f || !wav || !scal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    spin_sht_forward_internal(p, f, p->flm, nullptr, st);
    analysis_from_flm(p, p->flm, wav, scal, st);
    return post_launch("s2w_spin_analysis");
}

s2w_status s2w_spin_synthesis(s2w_plan p, const void *wav, const double *scal, double *f, void *stream)
{
    if (s2w_status st = check_plan(p)) return st;
    if (s2w_status st = check_spin(p)) return st;
    if (!f || !wav || !scal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p, st);
    synthesis_to_fhat(p, wav, scal, p->fhat, st);
    spin_sht_inverse_internal(p, p->fhat, nullptr, f, st);
    return post_launch("s2w_spin_synthesis");
}

s2w_status s2w_plan_profile(s2w_plan p, int capacity)
{
    if (s2w_status st = check_plan(p)) return st;
    if (capacity < 0) return fail(S2W_EINVAL, "capacity must be >= 0");
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (auto e : p->ev0) (void)hipEventDestroy(e);
    for (auto e : p->ev1) (void)hipEventDestroy(e);
    p->ev0.clear();
    p->ev1.clear();
    p->rec_name.clear();
    p->rec_flop.clear();
    p->rec_flop64.clear();
    p->rec_dense.clear();
    p->prof_names.clear();
    p->prof_dropped = 0;
    p->prof_cap = 0;
    for (int i = 0; i < capacity; ++i) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
            return fail(S2W_EHIP, "hipEventCreate failed");
        p->ev0.push_back(a);
        p->ev1.push_back(b);
    }
    p->prof_cap = capacity;
    return S2W_OK;
}

s2w_status s2w_plan_profile_read(s2w_plan p, int max, char *names, double *total_ms, int64_t *launches,
                                 double *flop, double *flop64, double *dense, int *count, int64_t *dropped)
{
    if (s2w_status st = check_plan(p)) return st;
    if (hipDeviceSynchronize() != hipSuccess) return fail(S2W_EHIP, "device synchronisation failed");
    const int nn = (int)p->prof_names.size();
    std::vector<double> ms(nn, 0.0), fl(nn, 0.0), f64(nn, 0.0), dn(nn, 0.0);
    std::vector<int64_t> cnt(nn, 0);
    for (size_t i = 0; i < p->rec_name.size(); ++i) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, p->ev0[i], p->ev1[i]) != hipSuccess) return fail(S2W_EHIP, "event timing failed");
        const int id = p->rec_name[i];
        ms[id] += t;
        fl[id] += p->rec_flop[i];
        f64[id] += p->rec_flop64[i];
        dn[id] += p->rec_dense[i];
        cnt[id] += 1;
    }
    const int k = std::min(nn, max);
    for (int i = 0; i < k; ++i) {
        if (names) {
            std::memset(names + 32 * i, 0, 32);
            std::strncpy(names + 32 * i, p->prof_names[i].c_str(), 31);
        }
        if (total_ms) total_ms[i] = ms[i];
        if (launches) launches[i] = cnt[i];
        if (flop) flop[i] = fl[i];
        if (flop64) flop64[i] = f64[i];
        if (dense) dense[i] = dn[i];
    }
    if (count) *count = k;
    if (dropped) *dropped = p->prof_dropped;
    p->rec_name.clear();
    p->rec_flop.clear();
    p->rec_flop64.clear();
    p->rec_dense.clear();
    p->prof_dropped = 0;
    return S2W_OK;
}


// ------------------------------------------------------------------ ball ---

s2w_status s2w_host_laguerre_rule(int P, double tau, double *nodes, double *weights)
{
    if (P < 1 || !(tau > 0.0) || !nodes || !weights) return fail(S2W_EINVAL, "bad arguments");
    s2w::LaguerreRule R;
    s2w::laguerre_rule(P, tau, R);
    std::memcpy(nodes, R.r.data(), sizeof(double) * P);
    std::memcpy(weights, R.W.data(), sizeof(double) * P);
    return S2W_OK;
}

static void free_ball(b3w_plan p)
{
    for (void *v : p->allocs) (void)hipFree(v);
    p->allocs.clear();
    if (p->sp) s2w_plan_destroy(p->sp);
    p->sp = nullptr;
}

static bool ball_upload(b3w_plan p, double *&ptr, const std::vector<double> &h)
{
    void *v = nullptr;
    if (dev_malloc(&v, std::max<size_t>(h.size(), 1) * sizeof(double)) != hipSuccess) return false;
    p->allocs.push_back(v);
    ptr = (double *)v;
    return hipMemcpy(ptr, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
}

// [c][r] from a row-major [r][c] matrix
static std::vector<double> transpose(const std::vector<double> &a, int r, int c)
{
    std::vector<double> t((size_t)r * c);
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) t[(size_t)j * r + i] = a[(size_t)i * c + j];
    return t;
}

static bool ball_alloc(b3w_plan p, double *&ptr, size_t count)
{
    void *v = nullptr;
    if (dev_malloc(&v, std::max<size_t>(count, 1) * sizeof(double)) != hipSuccess) return false;
    p->allocs.push_back(v);
    ptr = (double *)v;
    return true;
}

s2w_status b3w_plan_create(b3w_plan *out, int L, int N, int P, double lambda, double nu, int J0, int J0p,
                           double tau, int batch, s2w_precision precision, int device, unsigned flags)
{
    AllocSeq alloc_seq;
    if (!out) return fail(S2W_EINVAL, "null output pointer");
    *out = nullptr;
    if (P < 1) return fail(S2W_EINVAL, "P must be >= 1");
    if (!(nu > 1.0)) return fail(S2W_EINVAL, "nu must be > 1");
    if (!(tau > 0.0)) return fail(S2W_EINVAL, "tau must be > 0");
    if (batch < 1) return fail(S2W_EINVAL, "batch must be >= 1");
    if (flags & ~(unsigned)(S2W_PLAN_TUNE | S2W_PLAN_WIGNER))
        return fail(S2W_EINVAL, "ball plans accept S2W_PLAN_TUNE and S2W_PLAN_WIGNER only");
    int Jp = 0;
    while (std::pow(nu, (double)Jp) < (double)P) ++Jp;
    if (J0p < 0 || J0p > Jp) return fail(S2W_EINVAL, "J0p must satisfy 0 <= J0p <= J'");
    if ((long long)batch * P > (1LL << 30)) return fail(S2W_EINVAL, "batch * P too large");
    b3w_plan p = new (std::nothrow) b3w_plan_s;
    if (!p) return fail(S2W_ENOMEM, "host allocation failed");
    p->L = L; p->N = N; p->P = P; p->B = batch; p->J0 = J0; p->J0p = J0p; p->Jp = Jp;
    p->lambda = lambda; p->nu = nu; p->tau = tau; p->prec = precision;
    if (s2w_status st = s2w_plan_create(&p->sp, L, N, lambda, J0, batch * P, precision, device, flags)) {
        delete p;
        return st;
    }
    auto oom = [&](const char *what) {
        free_ball(p);
        delete p;
        return fail(S2W_ENOMEM, std::string("device allocation failed: ") + what);
    };
    s2w_plan sp = p->sp;
    p->nang = (int)sp->S.s.size();
    for (int jp = J0p; jp <= Jp; ++jp) {
        const double v = std::ceil(std::pow(nu, (double)jp + 1.0) - 1e-12);
        p->Pj.push_back((int)std::min<double>(v, (double)P));
    }
    p->nrad = (int)p->Pj.size();
    // layout
    p->wav_off.assign((size_t)p->nrad * p->nang + 1, 0);
    {
        int64_t off = 0;
        for (int i = 0; i < p->nrad; ++i)
            for (int k = 0; k < p->nang; ++k) {
                p->wav_off[(size_t)i * p->nang + k] = off;
                const auto &si = sp->S.s[k];
                off += (int64_t)batch * p->Pj[i] * (2 * si.N - 1) * si.L * (2 * si.L - 1);
            }
        p->wav_off.back() = off;
    }
    // radial rules and matrices
    s2w::LaguerreRule R;
    s2w::laguerre_rule(P, tau, R);
    p->nodes = R.r;
    std::vector<double> K;
    s2w::laguerre_basis(R, P, K);                       // [p][k]
    std::vector<double> zf((size_t)P * P), zi((size_t)P * P);
    for (int q = 0; q < P; ++q)
        for (int k = 0; k < P; ++k) {
            zf[(size_t)q * P + k] = R.W[k] * K[(size_t)q * P + k];
            zi[(size_t)k * P + q] = K[(size_t)q * P + k];
        }
    if (!ball_upload(p, p->Zf, zf) || !ball_upload(p, p->Zi, zi)) return oom("radial tables");
    if (!ball_upload(p, p->Zft, transpose(zf, P, P)) || !ball_upload(p, p->Zit, transpose(zi, P, P)))
        return oom("radial tables");
    p->G.assign(p->nrad, nullptr);
    p->H.assign(p->nrad, nullptr);
    p->Gt.assign(p->nrad, nullptr);
    p->Ht.assign(p->nrad, nullptr);
    for (int i = 0; i < p->nrad; ++i) {
        const int jp = J0p + i, Pi = p->Pj[i];
        std::vector<double> kap(P);
        for (int q = 0; q < P; ++q) kap[q] = std::sqrt(std::max(0.0, s2w::kappa2_lambda(q / std::pow(nu, (double)jp), nu)));
        s2w::LaguerreRule Ri;
        s2w::laguerre_rule(Pi, tau, Ri);
        std::vector<double> Ki;
        s2w::laguerre_basis(Ri, P, Ki);                 // [p < P][k < Pi]
        std::vector<double> g((size_t)Pi * P), h((size_t)P * Pi);
        for (int q = 0; q < P; ++q)
            for (int k = 0; k < Pi; ++k) {
                g[(size_t)k * P + q] = Ki[(size_t)q * Pi + k] * kap[q];
                h[(size_t)q * Pi + k] = kap[q] * Ri.W[k] * Ki[(size_t)q * Pi + k];
            }
        if (!ball_upload(p, p->G[i], g) || !ball_upload(p, p->H[i], h)) return oom("radial tables");
        if (!ball_upload(p, p->Gt[i], transpose(g, Pi, P)) || !ball_upload(p, p->Ht[i], transpose(h, P, Pi)))
            return oom("radial tables");
    }
    {
        std::vector<double> ph((size_t)P * L);
        for (int q = 0; q < P; ++q) {
            const double b = s2w::k_lambda(q / std::pow(nu, (double)J0p), nu);
            for (int l = 0; l < L; ++l) {
                const double a = s2w::k_lambda(l / std::pow(lambda, (double)J0), lambda);
                ph[(size_t)q * L + l] = std::sqrt(std::max(0.0, a + b - a * b));
            }
        }
        if (!ball_upload(p, p->phi, ph)) return oom("scaling filter");
    }
    const size_t per = (size_t)batch * P * L * L * 2;
    if (!ball_alloc(p, p->flmp, per) || !ball_alloc(p, p->shell, per) || !ball_alloc(p, p->shell2, per))
        return oom("workspace");
    if ((flags & S2W_PLAN_WIGNER) &&
        !ball_alloc(p, p->wltmp, (size_t)batch * P * (2 * N - 1) * L * (2 * L - 1) * 2))
        return oom("workspace");
    if (hipDeviceSynchronize() != hipSuccess) {
        free_ball(p);
        delete p;
        return fail(S2W_EHIP, "device synchronisation failed during plan creation");
    }
    reg_add(p);
    *out = p;
    return S2W_OK;
}

s2w_status b3w_plan_destroy(b3w_plan p)
{
    if (!p) return S2W_OK;
    if (!reg_remove(p)) return fail(S2W_ESTATE, "not a live ball plan (destroyed twice, or never created)");
    free_ball(p);
    delete p;
    return S2W_OK;
}

s2w_status b3w_plan_layout(b3w_plan p, int *nang, int *nrad, int *Lk, int *Nk, int *Pk, int64_t *wav_offset,
                           double *nodes)
{
    if (s2w_status st = check_ball(p)) return st;
    if (nang) *nang = p->nang;
    if (nrad) *nrad = p->nrad;
    for (int k = 0; k < p->nang; ++k) {
        if (Lk) Lk[k] = p->sp->S.s[k].L;
        if (Nk) Nk[k] = p->sp->S.s[k].N;
    }
    if (Pk)
        for (int i = 0; i < p->nrad; ++i) Pk[i] = p->Pj[i];
    if (wav_offset)
        for (size_t i = 0; i < p->wav_off.size(); ++i) wav_offset[i] = p->wav_off[i];
    if (nodes) std::memcpy(nodes, p->nodes.data(), sizeof(double) * p->P);
    return S2W_OK;
}

// Radial matrix A ([rows][kin]) applied to every map: out[b] = A in[b] (+ out[b] when acc),
// rows of `row` doubles (default: 2 L^2, the internal harmonic layout).
static void ball_radial(b3w_plan p, const double *A, const double *in, int kin, double *out, int rows, bool acc,
                        hipStream_t st, size_t row = 0)
{
    if (row == 0) row = (size_t)2 * p->L * p->L;
    for (int b = 0; b < p->B; ++b) {
        Prof pr_(p->sp, "gemm_radial", 2.0 * rows * kin * (double)row, st);
        s2w::launch_gemm(A, in + (size_t)b * kin * row, out + (size_t)b * rows * row, rows, (int)row, kin, st, acc);
    }
}

s2w_status b3w_analysis(b3w_plan p, const double *f, void *wav, double *scal, void *stream)
{
    if (s2w_status st = check_ball(p)) return st;
    if (!f || !wav || !scal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p->sp, st);
    s2w_plan sp = p->sp;
    const int B = p->B, P = p->P, L = p->L;
    const size_t esz = p->prec == S2W_MIXED ? sizeof(float) : sizeof(double);
    {
        BatchScope bs(sp, B * P);
        sht_forward_internal(sp, f, p->shell, st);                         // Y per shell
        ball_radial(p, p->Zf, p->shell, P, p->flmp, P, false, st);          // f_lmp
        { Prof pr_(sp, "scale_pl", 0.0, st); s2w::launch_scale_pl(p->flmp, p->shell2, p->phi, P, L, (size_t)B * P * L * L, st); }
        ball_radial(p, p->Zi, p->shell2, P, p->shell, P, false, st);        // Phi f at the nodes
        sht_inverse_internal(sp, p->shell, scal, st);                        // W^Phi
    }
    for (int i = 0; i < p->nrad; ++i) {
        const int Pi = p->Pj[i];
        BatchScope bs(sp, B * Pi);
        ball_radial(p, p->G[i], p->flmp, P, p->shell, Pi, false, st);        // g^{j'}_lm(r'_k)
        analysis_from_flm(sp, p->shell, (char *)wav + esz * p->wav_off[(size_t)i * p->nang], nullptr, st);
    }
    return post_launch("b3w_analysis");
}

s2w_status b3w_synthesis(b3w_plan p, const void *wav, const double *scal, double *f, void *stream)
{
    if (s2w_status st = check_ball(p)) return st;
    if (!f || !wav || !scal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p->sp, st);
    s2w_plan sp = p->sp;
    const int B = p->B, P = p->P, L = p->L;
    const size_t esz = p->prec == S2W_MIXED ? sizeof(float) : sizeof(double);
    {
        BatchScope bs(sp, B * P);
        sht_forward_internal(sp, scal, p->shell, st);
        ball_radial(p, p->Zf, p->shell, P, p->shell2, P, false, st);
        { Prof pr_(sp, "scale_pl", 0.0, st); s2w::launch_scale_pl(p->shell2, p->flmp, p->phi, P, L, (size_t)B * P * L * L, st); }
    }
    for (int i = 0; i < p->nrad; ++i) {
        const int Pi = p->Pj[i];
        BatchScope bs(sp, B * Pi);
        synthesis_to_fhat(sp, (const char *)wav + esz * p->wav_off[(size_t)i * p->nang], nullptr, p->shell, st);
        ball_radial(p, p->H[i], p->shell, Pi, p->flmp, P, true, st);        // f_lmp += Psi^dagger Q W
    }
    {
        BatchScope bs(sp, B * P);
        ball_radial(p, p->Zi, p->flmp, P, p->shell, P, false, st);
        sht_inverse_internal(sp, p->shell, f, st);
    }
    return post_launch("b3w_synthesis");
}

// Transpose of b3w_analysis (the gradient with respect to f): scaling part (transposes of
// Y^{-1}, Z^{-1} and the scaling filter), then per radial scale the transpose of the
// sphere analysis on its shells and of the radial projection onto its nodes, accumulated
// into the cotangent of f_lmp; finally the transposes of the radial forward and of Y.
s2w_status b3w_analysis_adjoint(b3w_plan p, const void *gwav, const double *gscal, double *gf, void *stream)
{
    if (s2w_status st = check_ball(p)) return st;
    if (!gf || !gwav || !gscal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p->sp, st);
    s2w_plan sp = p->sp;
    const int B = p->B, P = p->P, L = p->L;
    const size_t esz = p->prec == S2W_MIXED ? sizeof(float) : sizeof(double);
    {
        BatchScope bs(sp, B * P);
        sht_inverse_T(sp, L, sp->wsht, gscal, p->shell, st);
        ball_radial(p, p->Zit, p->shell, P, p->shell2, P, false, st);
        { Prof pr_(sp, "scale_pl", 0.0, st); s2w::launch_scale_pl(p->shell2, p->flmp, p->phi, P, L, (size_t)B * P * L * L, st); }
    }
    for (int i = 0; i < p->nrad; ++i) {
        const int Pi = p->Pj[i];
        BatchScope bs(sp, B * Pi);
        analysis_from_flm_T(sp, (const char *)gwav + esz * p->wav_off[(size_t)i * p->nang], nullptr, p->shell, st);
        ball_radial(p, p->Gt[i], p->shell, Pi, p->flmp, P, true, st);
    }
    {
        BatchScope bs(sp, B * P);
        ball_radial(p, p->Zft, p->flmp, P, p->shell, P, false, st);
        sht_forward_T(sp, L, sp->wsht, p->shell, L, L, gf, st);
    }
    return post_launch("b3w_analysis_adjoint");
}

// Transpose of b3w_synthesis: transposes of Y^{-1} and of the radial inverse give the
// cotangent of f_lmp; per radial scale, the transpose of its radial synthesis matrix and
// of the sphere synthesis on its shells; the scaling part through the scaling filter and
// the transposes of the radial forward and of Y.
s2w_status b3w_synthesis_adjoint(b3w_plan p, const double *gf, void *gwav, double *gscal, void *stream)
{
    if (s2w_status st = check_ball(p)) return st;
    if (!gf || !gwav || !gscal) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p->sp, st);
    s2w_plan sp = p->sp;
    const int B = p->B, P = p->P, L = p->L;
    const size_t esz = p->prec == S2W_MIXED ? sizeof(float) : sizeof(double);
    {
        BatchScope bs(sp, B * P);
        sht_inverse_T(sp, L, sp->wsht, gf, p->shell, st);
        ball_radial(p, p->Zit, p->shell, P, p->flmp, P, false, st);
    }
    for (int i = 0; i < p->nrad; ++i) {
        const int Pi = p->Pj[i];
        BatchScope bs(sp, B * Pi);
        ball_radial(p, p->Ht[i], p->flmp, P, p->shell, Pi, false, st);
        synthesis_to_fhat_T(sp, p->shell, (char *)gwav + esz * p->wav_off[(size_t)i * p->nang], nullptr, st);
    }
    {
        BatchScope bs(sp, B * P);
        { Prof pr_(sp, "scale_pl", 0.0, st); s2w::launch_scale_pl(p->flmp, p->shell2, p->phi, P, L, (size_t)B * P * L * L, st); }
        ball_radial(p, p->Zft, p->shell2, P, p->shell, P, false, st);
        sht_forward_T(sp, L, sp->wsht, p->shell, L, L, gscal, st);
    }
    return post_launch("b3w_synthesis_adjoint");
}

// Wigner-Laguerre transform of real functions on R+ x SO(3) (Section 2.5: Q^l_mnp = K_p D^l_mn,
// the decomposition and its synthesis eq:wiglag_inverse): the SO(3) transform on every radial
// node (B P at a time), then the radial forward f_p = sum_k W_k K_p(r_k) f(r_k) on the
// coefficient rows (and the inverse in reverse order).  FP64.
s2w_status b3w_wl_forward(b3w_plan p, const double *f, double *flmnp, void *stream)
{
    if (s2w_status st = check_ball(p)) return st;
    if (!p->wltmp) return fail(S2W_ESTATE, "ball plan created without S2W_PLAN_WIGNER");
    if (!f || !flmnp) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p->sp, st);
    s2w_plan sp = p->sp;
    const int B = p->B, P = p->P, L = p->L, ng = 2 * p->N - 1;
    {
        BatchScope bs(sp, B * P);
        wigner_forward_internal(sp, f, p->wltmp, st);
        ball_radial(p, p->Zf, p->wltmp, P, flmnp, P, false, st, (size_t)ng * L * (2 * L - 1) * 2);
    }
    return post_launch("b3w_wl_forward");
}

s2w_status b3w_wl_inverse(b3w_plan p, const double *flmnp, double *f, void *stream)
{
    if (s2w_status st = check_ball(p)) return st;
    if (!p->wltmp) return fail(S2W_ESTATE, "ball plan created without S2W_PLAN_WIGNER");
    if (!f || !flmnp) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p->sp, st);
    s2w_plan sp = p->sp;
    const int B = p->B, P = p->P, L = p->L, N = p->N, ng = 2 * N - 1;
    {
        BatchScope bs(sp, B * P);
        ball_radial(p, p->Zi, flmnp, P, p->wltmp, P, false, st, (size_t)ng * L * (2 * L - 1) * 2);
        s2w::launch_wig_ext_to_int(p->wltmp, sp->wint, L, N, B * P, st);
        wigner_inverse_internal(sp, sp->wint, f, st);
    }
    return post_launch("b3w_wl_inverse");
}

// Z and Z^{-1}: per-shell spherical-harmonic transforms (B P shells at a time) and the
// radial projection onto the Laguerre basis (quadrature weights folded into Zf)
s2w_status b3w_sl_forward(b3w_plan p, const double *f, double *flmp, void *stream)
{
    if (s2w_status st = check_ball(p)) return st;
    if (!f || !flmp) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p->sp, st);
    s2w_plan sp = p->sp;
    const int B = p->B, P = p->P, L = p->L;
    {
        BatchScope bs(sp, B * P);
        sht_forward_internal(sp, f, p->shell, st);
        ball_radial(p, p->Zf, p->shell, P, p->flmp, P, false, st);
        s2w::launch_flm_to_ext(p->flmp, flmp, L, B * P, st);
    }
    return post_launch("b3w_sl_forward");
}

s2w_status b3w_sl_inverse(b3w_plan p, const double *flmp, double *f, void *stream)
{
    if (s2w_status st = check_ball(p)) return st;
    if (!f || !flmp) return fail(S2W_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    StreamOrder order(p->sp, st);
    s2w_plan sp = p->sp;
    const int B = p->B, P = p->P, L = p->L;
    {
        BatchScope bs(sp, B * P);
        s2w::launch_flm_from_ext(flmp, p->flmp, L, B * P, st);
        ball_radial(p, p->Zi, p->flmp, P, p->shell, P, false, st);
        sht_inverse_internal(sp, p->shell, f, st);
    }
    return post_launch("b3w_sl_inverse");
}

s2w_status b3w_plan_profile(b3w_plan p, int capacity)
{
    if (s2w_status st = check_ball(p)) return st;
    return s2w_plan_profile(p->sp, capacity);
}

s2w_status b3w_plan_profile_read(b3w_plan p, int max, char *names, double *total_ms, int64_t *launches,
                                 double *flop, double *flop64, double *dense, int *count, int64_t *dropped)
{
    if (s2w_status st = check_ball(p)) return st;
    return s2w_plan_profile_read(p->sp, max, names, total_ms, launches, flop, flop64, dense, count, dropped);
}

}  // extern "C"
