// Host runtime and C ABI of the DFS spectral Poisson solver (see
// include/sphere_poisson.h).  Plans own every device buffer; solves only
// enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <sys/stat.h>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "../../include/sphere_poisson.h"
#include "sp_batch.hpp"
#include "sp_theta_real.hpp"
#include "sp_calculus.hpp"
#include "sp_lowrank.hpp"
#include "sp_tables.hpp"
#include "sp_stream.hpp"

using sp::Cx;
using sp::FftDesc;
using sp::kEPT;
using sp::kSmaxD;
using sp::kSmaxF;
using sp::kLayLog2;
using sp::kSmaxR;
using sp::kBatchThreads;
using sp::kBatchClasses;
using sp::kBatchSmallRadix;
using sp::kBatchRealThreads;
using sp::kBatchSmaxR;
using sp::kBatchWaveThreads;
using sp::kBatchScal;
using sp::kBatchMaxLaunches;
using sp::KernelSet;
using sp::MixedSet;
using sp::BatchKernels;
using sp::pick_kernels;
using sp::pick_mixed;
using sp::grad_kernel;
using sp::batch_kernels;

namespace {

thread_local std::string g_hip_err;

int hip_fail(hipError_t e, const char* what) {
    g_hip_err = std::string(what) + ": " + hipGetErrorString(e);
    return SP_ERR_HIP;
}

#define SP_HIP(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)


// ------------------------------------------------------------ twiddles
// (cos, -sin)(2 pi t / N) in extended precision with exact quadrant
// reduction of the angle; rounded once to double.
void cis_neg(long long t, long long N, double* re, double* im) {
    t %= N;
    if (t < 0) t += N;
    long long a = 4 * t;
    long long qd = a / N;            // quadrant
    long long r = a - qd * N;        // angle = (qd + r/N) * pi/2
    long double x = (long double)r / (long double)N * (3.141592653589793238462643383279502884L / 2.0L);
    long double c = cosl(x), s = sinl(x);
    if (r == 0) { c = 1.0L; s = 0.0L; }
    long double cc, ss;
    switch (qd) {
        case 0: cc = c; ss = s; break;
        case 1: cc = -s; ss = c; break;
        case 2: cc = -c; ss = -s; break;
        default: cc = s; ss = -c; break;
    }
    *re = (double)cc;
    *im = (double)(-ss);
}

// ------------------------------------------------------------ FFT planning
// The compiled-in transform of length 5000 (radices 10, 5, 10, 10): its
// radix-10 passes exist only in that fixed build.
bool is_fixed5000(const std::vector<int>& rad, int L) {
    return L == 5000 && rad == std::vector<int>(std::begin(sp::kFixed5000Radices), std::end(sp::kFixed5000Radices));
}

bool factorize(int L, std::vector<int>& radices) {
    radices.clear();
    if (L < 1) return false;
    int e = 0;
    while (L % 2 == 0) { L /= 2; ++e; }
    std::vector<int> p2;
    while (e >= 3) { p2.push_back(8); e -= 3; }
    if (e == 2) p2.push_back(4);
    if (e == 1) {
        if (!p2.empty()) p2[0] = 16;
        else p2.push_back(2);
    }
    // odd radices first: the first Stockham pass writes with stride R, which
    // for an odd R touches distinct LDS banks
    static const int odd[] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
    for (int p : odd) {
        while (L % p == 0) { radices.push_back(p); L /= p; }
    }
    radices.insert(radices.end(), p2.begin(), p2.end());
    return L == 1 && (int)radices.size() <= sp::kMaxPass;
}

int bpt(int R) { return std::max(1, kEPT / R); }

// Default radix order of a length: the fixed transform where one is compiled
// in, else factorize().
bool default_radices(int L, std::vector<int>& radices) {
    if (L == 5000) {
        radices.assign(std::begin(sp::kFixed5000Radices), std::end(sp::kFixed5000Radices));
        return true;
    }
    return factorize(L, radices);
}

int fft_threads(const std::vector<int>& rad, int L) {
    int t = 1;
    for (int R : rad) t = std::max(t, ((L / R) + bpt(R) - 1) / bpt(R));
    return t;
}

// Per-pass twiddle table of a Stockham DFT of length L: pass p (radix R, span
// Ns = product of earlier radices) stores e^{-2 pi i r k / (Ns R)} at
// off_p + (r - 1) Ns + k, r = 1..R-1, k = 0..Ns-1.
FftDesc make_desc(const std::vector<int>& rad, int L, std::vector<Cx<double>>* table) {
    FftDesc d{};
    d.N = L;
    d.npass = (int)rad.size();
    // compiled-in fixed transforms (used when the thread count also matches)
    if (is_fixed5000(rad, L)) d.fixed = sp::kFixed5000;
    table->clear();
    long long Ns = 1;
    for (size_t i = 0; i < rad.size(); ++i) {
        const int R = rad[i];
        d.radix[i] = R;
        d.tw_off[i] = (int)table->size();
        for (int r = 1; r < R; ++r)
            for (long long k = 0; k < Ns; ++k) {
                Cx<double> w;
                cis_neg((long long)r * k, Ns * R, &w.x, &w.y);
                table->push_back(w);
            }
        Ns *= R;
    }
    if (table->empty()) table->push_back(Cx<double>{1.0, 0.0});
    return d;
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }
int round_up(int a, int b) { return ceil_div(a, b) * b; }

struct ClassCounts { int ncA, ncB; };
ClassCounts classes(int m, bool sine, bool k0) {
    int qhi = sine ? m : m - 1;
    int qA = k0 ? 2 : (sine ? 2 : 0);
    ClassCounts c;
    c.ncA = qhi >= qA ? (qhi - qA) / 2 + 1 : 0;
    c.ncB = qhi >= 1 ? (qhi - 1) / 2 + 1 : 0;
    return c;
}

// Threads a solve needs: the chunks of both classes for k != 0 (one chunk
// length for both, as the kernels lay them out) and for the k = 0 system.
int solve_threads(int m, int smax) {
    int best = 0;
    for (int s = 0; s < 2; ++s) {
        const ClassCounts c = classes(m, s, false);
        const sp::SolveChunks ch = sp::solve_chunks(c.ncA, c.ncB, smax);
        best = std::max(best, ch.pA + ch.pB);
    }
    const ClassCounts z = classes(m, false, true);
    return std::max(best, ceil_div(z.ncA, smax) + ceil_div(z.ncB, smax));
}


// The radix set a transform needs (see kernel_set).
int radix_set(const FftDesc& d, int nthr, bool fixed_ok) {
    if (fixed_ok && d.fixed == sp::kFixed5000 && nthr == sp::kFixed5000Threads) return sp::kRadixFixed5000;
    int r = 1;
    for (int p = 0; p < d.npass; ++p) r = std::max(r, d.radix[p]);
    return r <= 16 ? 16 : 32;
}

template <typename T>
struct Tables {
    Cx<T>* tw_n = nullptr;   // n entries: e^{-2 pi i t/n}
    Cx<T>* pass_n = nullptr; // per-pass twiddles of the length-n/2 DFT
    Cx<T>* pass_m = nullptr; // per-pass twiddles of the length-m DFT
    Cx<T>* eq = nullptr;     // m entries: e^{-i pi q/(2m)}
    Cx<T>* ws = nullptr;     // m/4 + 1 entries: e^{-2 pi i q/m} (real-part theta pass)
};

}  // namespace

// A batch plan (sphere_poisson_batch_plan): every problem's workspace and
// tables in one allocation, the work lists, and the captured graph.
struct sp_batch_s {
    int count = 0, precision = 0, device = 0, max_refine = 0;
    double tol = 0.0;
    std::vector<int> n, m;
    void* block = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;   // recorded after every launch: destroy waits for it
    bool launched = false;
    double* scal = nullptr;      // [count][kBatchScal]: [0] integral of f, then per correction sums d^2, u^2
    ~sp_batch_s() {
        if (done && launched) (void)hipEventSynchronize(done);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (done) (void)hipEventDestroy(done);
        if (block) (void)hipFree(block);
    }
};

// ------------------------------------------------------------ plan
struct sp_plan_s {
    sp_desc desc{};
    int device = 0;
    int n = 0, m = 0, N = 0;
    int rw_log2 = 0;          // rows per lambda workgroup (log2)
    int lay_log2 = 0;         // spectrum run length (log2)
    int lam_grid = 0;         // lambda workgroups (a multiple of 8 runs when a run spans several)
    // forward lambda passes: half the rows per workgroup when a full tile leaves room for one
    // workgroup per compute unit only, so that two share it (one loads while the other computes)
    int fwd_rw_log2 = 0, fwd_grid = 0;
    size_t fwd_lds = 0;
    int lam_threads = 0;      // threads per row in the lambda kernels
    int theta_threads = 0;    // block size of the theta kernel
    int theta_fft_threads = 0;
    bool theta_real = false;  // even m: one real part per theta workgroup, DFT length m/2
    int theta_grid = 0;       // theta workgroups
    size_t lam_lds = 0, theta_lds64 = 0, theta_lds32 = 0;
    int upd_block = 0;        // threads of the mixed update pass
    int k8 = 0;
    FftDesc fft_lam{}, fft_theta{};
    KernelSet<double> kd{};
    KernelSet<float> kf{};
    MixedSet km{};
    // tangential gradient: lambda pass with two lines per row (null: the rows do not fit the LDS)
    void (*grad)(sp::GradArgs) = nullptr;
    int grad_rw_log2 = 0, grad_grid = 0, grad_block = 0;
    size_t grad_lds = 0;
    double* gradtab = nullptr;   // [2][m] cos(theta), sin(theta); then [2][n] sin(lambda), cos(lambda)
    double* intw = nullptr;      // [m] integration weights 2 pi W_j / n (sphere_poisson_integral)
    double* intpart = nullptr;   // [kIntegralBlocks] partial sums
    // device memory
    void* block = nullptr;    // one allocation holding everything below
    size_t block_bytes = 0;
    Cx<double>* spec64 = nullptr;
    Tables<double> t64;
    Tables<float> t32;
    double* sin2 = nullptr;
    double* k0tab = nullptr;
    double* fint_w = nullptr;
    // device scalars: [0] integral of f; [1..2] sums d^2, u^2 of the last correction; [3..4] sums r^2,
    // F^2 of the last correction pass's residual; [5..6] sums d^2, u^2 of the correction before the last
    double* scal = nullptr;
    size_t spec_elems = 0;
    int last_status = SP_OK, last_iters = 0;   // of the last solve or adjoint (sphere_poisson_get_info)
    // MIXED workspace
    Cx<double>* specB = nullptr;   // float64: theta output; mixed: spectrum of the current iterate
    Cx<float>* spec0 = nullptr;    // float32 spectrum of the first iterate
    Cx<float>* specd = nullptr;    // float32 spectrum of the correction
    double* partial = nullptr;     // per lambda block: sum d^2, sum u^2
    double* rnorm = nullptr;       // per theta tile: sums r^2, F^2 of the correction pass
    Cx<double>* fco = nullptr;     // theta coefficients F of sin^2 f per wavenumber (solve order)
    // profiling: event pairs around launches
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    int ev_used = 0;
};

namespace {

std::mutex g_plans_mu;
std::set<sp_plan> g_plans;   // live plans: a destroyed or foreign handle is rejected without a dereference

bool plan_ok(sp_plan p) {
    if (!p) return false;
    std::lock_guard<std::mutex> g(g_plans_mu);
    return g_plans.count(p) != 0;
}

std::mutex g_batches_mu;
std::set<sp_batch> g_batches;   // live batch plans (same rule as g_plans)

bool batch_ok(sp_batch b) {
    if (!b) return false;
    std::lock_guard<std::mutex> g(g_batches_mu);
    return g_batches.count(b) != 0;
}

void plan_register(sp_plan p) {
    std::lock_guard<std::mutex> g(g_plans_mu);
    g_plans.insert(p);
}

void plan_unregister(sp_plan p) {
    std::lock_guard<std::mutex> g(g_plans_mu);
    g_plans.erase(p);
}

int validate_desc(const sp_desc* d) {
    if (!d) return SP_ERR_INVALID_ARG;
    if (d->n_lambda < 4 || (d->n_lambda & 1) || d->m_theta < 4) return SP_ERR_INVALID_ARG;
    if (d->precision != SP_FP64 && d->precision != SP_MIXED) return SP_ERR_INVALID_ARG;
    if (d->max_refine < 0 || (d->flags & ~(SP_SYNC_INFO | SP_AUTOTUNE | SP_INFO))) return SP_ERR_INVALID_ARG;
    if (d->n_lambda > (1 << 20) || d->m_theta > (1 << 20)) return SP_ERR_UNSUPPORTED_SIZE;
    std::vector<int> r;
    if (!factorize(d->n_lambda / 2, r) || !factorize(d->m_theta, r)) return SP_ERR_UNSUPPORTED_SIZE;
    return SP_OK;
}

struct Layout {
    size_t off_spec, off_tw64n, off_tw64m, off_eq64, off_tw32n, off_tw32m, off_eq32, off_p64n, off_p32n;
    size_t off_ws64, off_ws32;
    size_t off_sin2, off_k0, off_fint, off_scal, total;
    size_t off_specB, off_spec0, off_specd, off_partial, off_fco, off_rnorm;
    size_t off_grad, off_intw, off_intpart;
    size_t spec_elems;
};

constexpr int kIntegralBlocks = 512;   // workgroups of the first integration pass

// rw: rows per lambda workgroup; rl: spectrum run length (rows), a multiple of rw
Layout layout_for(int n, int m, int rw, int rl, bool mixed) {
    Layout L{};
    size_t N = n / 2;
    size_t nblk = (size_t)(m + rw - 1) / rw;
    L.spec_elems = ((size_t)(m + rl - 1) / rl) * (N + 1) * rl;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) & ~(size_t)255; return o; };
    L.off_spec = take(L.spec_elems * sizeof(Cx<double>));
    L.off_tw64n = take((size_t)n * sizeof(Cx<double>));
    L.off_tw64m = take((size_t)m * sizeof(Cx<double>));
    L.off_eq64 = take((size_t)m * sizeof(Cx<double>));
    L.off_tw32n = take((size_t)n * sizeof(Cx<float>));
    L.off_tw32m = take((size_t)m * sizeof(Cx<float>));
    L.off_eq32 = take((size_t)m * sizeof(Cx<float>));
    L.off_ws64 = take((size_t)(m / 4 + 2) * sizeof(Cx<double>));
    L.off_ws32 = take((size_t)(m / 4 + 2) * sizeof(Cx<float>));
    L.off_p64n = take((size_t)n * sizeof(Cx<double>));
    L.off_p32n = take((size_t)n * sizeof(Cx<float>));
    L.off_sin2 = take((size_t)m * sizeof(double));
    L.off_k0 = take((size_t)2 * (m + 2) * sizeof(double));
    L.off_fint = take((size_t)m * sizeof(double));
    L.off_scal = take(16 * sizeof(double));
    L.off_grad = take((size_t)(2 * m + 2 * n) * sizeof(double));
    L.off_intw = take((size_t)m * sizeof(double));
    L.off_intpart = take((size_t)kIntegralBlocks * sizeof(double));
    // second float64 spectrum: the theta output of the float64 path (lambda
    // read layout), and in mixed plans the spectrum of the current iterate
    L.off_specB = take(L.spec_elems * sizeof(Cx<double>));
    if (mixed) {
        L.off_spec0 = take(L.spec_elems * sizeof(Cx<float>));
        L.off_specd = take(L.spec_elems * sizeof(Cx<float>));
        L.off_partial = take(2 * nblk * sizeof(double));
        L.off_rnorm = take(4 * (N + 1) * sizeof(double));
        L.off_fco = take((N + 1) * (size_t)sp::solve_slot_stride(m) * sizeof(Cx<double>));
    }
    L.total = off;
    return L;
}

// rows per lambda workgroup and threads per row
bool lambda_schedule(int N, int m, const std::vector<int>& rad, size_t lds_limit, int* rw_log2,
                     int* nthr, size_t* lds) {
    int t = fft_threads(rad, N);
    if (t > 1024) return false;
    int best = -1;
    for (int l = 0; l <= 5; ++l) {
        int rw = 1 << l;
        if (rw * t > 1024) break;
        if ((size_t)rw * N * sizeof(Cx<double>) > lds_limit) break;
        best = l;
        if (rw >= m) break;
        // enough threads; rows of short transforms stop there (more tiles per CU),
        // rows of long ones also fill a 128-byte spectrum run
        if (rw * t >= 256 && (t < 256 || rw * (int)sizeof(Cx<double>) >= 128)) break;
    }
    if (best < 0) return false;
    *rw_log2 = best;
    *nthr = t;
    *lds = (size_t)(1 << best) * N * sizeof(Cx<double>);
    return true;
}

template <typename T>
size_t theta_lds_bytes(int m, int ptot) {
    size_t a = (size_t)m * sizeof(Cx<T>);
    size_t b = (size_t)ptot * (sizeof(Cx<T>) + 3 * sizeof(T));
    size_t c = (size_t)ptot * (sizeof(Cx<double>) + sizeof(double));
    return (std::max(a, std::max(b, c)) + 15) & ~(size_t)15;
}

int query_device(int* dev, size_t* lds_limit) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return SP_ERR_NO_DEVICE;
    SP_HIP(hipGetDevice(dev));
    hipDeviceProp_t prop;
    SP_HIP(hipGetDeviceProperties(&prop, *dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_hip_err = std::string("device is ") + prop.gcnArchName + ", library is built for gfx950";
        return SP_ERR_NO_DEVICE;
    }
    *lds_limit = prop.sharedMemPerBlock;
    return SP_OK;
}

template <typename T>
void set_lds_attr(const KernelSet<T>& ks, size_t lam, size_t theta) {
    (void)hipFuncSetAttribute((const void*)ks.fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lam);
    (void)hipFuncSetAttribute((const void*)ks.inv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lam);
    for (const void* fn : {(const void*)ks.theta, (const void*)ks.theta_real})
        if (fn) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)theta);
    (void)hipGetLastError();
}

// LDS of the real-part theta pass: the float64 line (m reals, with its zero
// margins) or the solve scratch (separator rows; k = 0 scan values),
// whichever is larger.
size_t real_theta_lds_bytes(int m, int ptot) {
    size_t a = (size_t)m * sizeof(double) + 2 * sp::kRealLineMargin;
    size_t b = (size_t)ptot * 4 * sizeof(double);
    size_t c = (size_t)ptot * 2 * sizeof(double);
    return (std::max(a, std::max(b, c)) + 15) & ~(size_t)15;
}

}  // namespace


namespace {
// Theta tables of one m: e^{-i pi q/(2m)}, sin^2(theta_j), the k = 0 LU factors
// (extended precision) and the quadrature weights of the integral of f.
void host_theta_tables(int m, std::vector<Cx<double>>& eq, std::vector<double>& sin2, std::vector<double>& k0,
                       std::vector<double>& fint) {
    eq.resize(m);
    for (int t = 0; t < m; ++t) cis_neg(t, 4LL * m, &eq[t].x, &eq[t].y);
    const long double PI = 3.141592653589793238462643383279502884L;
    sin2.resize(m);
    fint.resize(m);
    for (int j = 0; j < m; ++j) {
        long double th = ((long double)j + 0.5L) * PI / (long double)m;
        long double s = sinl(th);
        sin2[j] = (double)(s * s);
        // Fejer-type weight: int_0^pi g sin = sum_j W_j g_j for g in span{cos q theta, q < m};
        // the k = 0 column holds sin^2 f, so the integral of f uses W_j / sin^2(theta_j), times 2 pi.
        long double W = 0.0L;
        for (int q = 0; q < m; q += 2) {
            long double cq = (q == 0 ? 1.0L : 2.0L) / (long double)m;
            W += cq * cosl((long double)q * th) * 2.0L / (1.0L - (long double)q * q);
        }
        fint[j] = (double)(2.0L * PI * W / (s * s));
    }
    k0.clear();
    ClassCounts c = classes(m, false, true);
    auto lu = [&](int q0, int nc) {
        std::vector<double> inv(nc), cpd(nc);
        long double cprev = 0.0L;
        for (int i = 0; i < nc; ++i) {
            long double q = q0 + 2.0L * i;
            long double sub = i == 0 ? 0.0L : (q - 2.0L) * (q - 1.0L) / 4.0L;
            long double diag = -q * q / 2.0L;
            long double sup = i == nc - 1 ? 0.0L : (q + 2.0L) * (q + 1.0L) / 4.0L;
            long double den = diag - sub * cprev;
            inv[i] = (double)(1.0L / den);
            long double cp = sup / den;
            cpd[i] = (double)cp;
            cprev = cp;
        }
        k0.insert(k0.end(), inv.begin(), inv.end());
        k0.insert(k0.end(), cpd.begin(), cpd.end());
    };
    lu(2, c.ncA);
    lu(1, c.ncB);
}
}  // namespace

extern "C" size_t sphere_poisson_workspace_bytes(const sp_desc* d) {
    if (validate_desc(d) != SP_OK) return 0;
    std::vector<int> rl;
    default_radices(d->n_lambda / 2, rl);
    int rwl = 0, nt = 0;
    size_t lds = 0;
    if (!lambda_schedule(d->n_lambda / 2, d->m_theta, rl, 160 * 1024, &rwl, &nt, &lds)) return 0;
    return layout_for(d->n_lambda, d->m_theta, 1 << rwl, 1 << std::max(rwl, kLayLog2), d->precision == SP_MIXED).total;
}

namespace {
// A launch schedule: radix order of both transforms and rows per lambda tile
// (rw_log2 < 0: the fixed rule).
struct Sched {
    std::vector<int> lam, theta;
    int rw_log2 = -1;
};

bool valid_radices(const std::vector<int>& r, int L);

int plan_create(const sp_desc* d, hipStream_t stream, const Sched& sc, sp_plan* out) {
    *out = nullptr;
    int dev = 0;
    size_t lds_limit = 0;
    int st = query_device(&dev, &lds_limit);
    if (st != SP_OK) return st;

    sp_plan p = new (std::nothrow) sp_plan_s();
    if (!p) return SP_ERR_OOM;
    p->desc = *d;
    p->device = dev;
    p->n = d->n_lambda;
    p->m = d->m_theta;
    p->N = p->n / 2;
    const int n = p->n, m = p->m, N = p->N;

    // theta pass: even m runs one real part per workgroup (cosine transform
    // through a DFT of length m/2) when its thread and LDS budgets allow;
    // otherwise the complex line (DFT of length m)
    const size_t static_lds = 16 * sizeof(Cx<double>);
    if ((m & 1) == 0) {
        const int M = m / 2, ptotR = solve_threads(m, kSmaxR);
        std::vector<int> r = sc.theta;
        if (!valid_radices(r, M)) r.clear();
        if (r.empty() && !default_radices(M, r)) r.clear();
        if (!r.empty()) {
            const int fthr = fft_threads(r, M);
            const int thr = round_up(std::max(std::max(fthr, ptotR), sp::real_theta_min_threads(m)), 64);
            const size_t lds = real_theta_lds_bytes(m, ptotR);
            if (thr <= 512 && lds + static_lds <= lds_limit) {
                p->theta_real = true;
                p->theta_fft_threads = fthr;
                p->theta_threads = thr;
                p->theta_lds64 = lds;
                p->theta_lds32 = lds;
            }
        }
    }
    std::vector<int> rl = sc.lam, rt = sc.theta;
    const int Lt = p->theta_real ? m / 2 : m;
    if (!valid_radices(rl, N)) rl.clear();
    if (!valid_radices(rt, Lt)) rt.clear();
    if (rl.empty()) default_radices(N, rl);
    if (rt.empty()) default_radices(Lt, rt);
    std::vector<Cx<double>> ptab_n, ptab_m;
    p->fft_lam = make_desc(rl, N, &ptab_n);
    p->fft_theta = make_desc(rt, Lt, &ptab_m);

    if (!lambda_schedule(N, m, rl, lds_limit, &p->rw_log2, &p->lam_threads, &p->lam_lds)) {
        delete p;
        return SP_ERR_UNSUPPORTED_SIZE;
    }
    if (sc.rw_log2 >= 0 && sc.rw_log2 <= 5 && (1 << sc.rw_log2) * p->lam_threads <= 1024 &&
        ((size_t)N << sc.rw_log2) * sizeof(Cx<double>) <= lds_limit) {
        p->rw_log2 = sc.rw_log2;
        p->lam_lds = ((size_t)N << sc.rw_log2) * sizeof(Cx<double>);
    }
    p->lay_log2 = std::max(p->rw_log2, kLayLog2);
    {
        const int nblk = (m + (1 << p->rw_log2) - 1) >> p->rw_log2;
        p->lam_grid = round_up(nblk, 8 << (p->lay_log2 - p->rw_log2));
    }
    if (!p->theta_real) {
        p->theta_fft_threads = fft_threads(rt, m);
        int ptotD = solve_threads(m, kSmaxD), ptotF = solve_threads(m, kSmaxF);
        p->theta_threads = round_up(std::max(std::max(p->theta_fft_threads, ceil_div(m, sp::kThetaHold)),
                                             std::max(ptotD, ptotF)), 64);
        p->theta_lds64 = theta_lds_bytes<double>(m, ptotD);
        p->theta_lds32 = theta_lds_bytes<float>(m, ptotF);
        if (p->theta_threads > 1024 || p->theta_lds64 + static_lds > lds_limit) {
            delete p;
            return SP_ERR_UNSUPPORTED_SIZE;
        }
    }
    p->k8 = (N + 1 + 7) / 8;
    p->theta_grid = (p->theta_real ? 16 : 8) * p->k8;
    // lambda and theta kernels are picked separately: either may run a fixed transform
    const int rs_lam = radix_set(p->fft_lam, p->lam_threads, true);
    const int rs_th = radix_set(p->fft_theta, p->theta_fft_threads, p->theta_real);
    // the fixed real-part kernels assume m = 2 * 5000 (full solve chunks); the
    // fixed transform is only chosen for a real-part line of that length
    if (rs_th == sp::kRadixFixed5000 && m != 2 * 5000) {
        delete p;
        return SP_ERR_UNSUPPORTED_SIZE;
    }
    {
        const KernelSet<double> L = pick_kernels<double>(rs_lam), T = pick_kernels<double>(rs_th);
        p->kd = KernelSet<double>{L.fwd, L.inv, T.theta, T.theta_real};
        p->kf = pick_kernels<float>(rs_lam);
        const MixedSet Lm = pick_mixed(rs_lam);
        p->km = pick_mixed(rs_th);
        p->km.mix = Lm.mix;
        p->km.update = Lm.update;
    }
    set_lds_attr(p->kd, p->lam_lds, p->theta_lds64);
    set_lds_attr(p->kf, p->lam_lds, p->theta_lds64);
    for (int v = 0; v < 2; ++v)
        for (const void* fn : {(const void*)p->km.theta_first[v], (const void*)p->km.theta_resid[v],
                               (const void*)p->km.theta_first_t[v], (const void*)p->km.theta_resid_t[v],
                               (const void*)p->km.theta_resid_norm[v], (const void*)p->km.theta_resid_t_norm[v]})
            if (fn) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->theta_lds64);
    for (const void* fn : {(const void*)p->km.mix, (const void*)p->km.update})
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lam_lds);
    // the fixed transform's update pass runs a tile's rows one after the other in one row's threads
    p->upd_block = round_up((rs_lam == sp::kRadixFixed5000 ? 1 : 1 << p->rw_log2) * p->lam_threads, 64);
    // forward lambda passes: when a tile of the plan's rows fills the LDS so that one workgroup
    // runs per compute unit, the forward pass takes half the rows (measured at n = m = 10^4:
    // 0.53 -> 0.47 ms); the passes that read a spectrum keep the full tile, whose reads take
    // whole runs
    p->fwd_rw_log2 = p->rw_log2;
    if (p->rw_log2 > 0 && 2 * p->lam_lds + static_lds > lds_limit) p->fwd_rw_log2 = p->rw_log2 - 1;
    p->fwd_lds = ((size_t)N << p->fwd_rw_log2) * sizeof(Cx<double>);
    {
        const int nblk = (m + (1 << p->fwd_rw_log2) - 1) >> p->fwd_rw_log2;
        p->fwd_grid = round_up(nblk, 8 << (p->lay_log2 - p->fwd_rw_log2));
    }
    // gradient pass: two float64 lines per row, as many rows per workgroup as fit (at most the plan's);
    // the fixed transform's build takes one row and one line (its two transforms run in turn);
    // the theta division by sin(theta) needs one thread per chunk of each parity class
    const int div_hold = p->theta_real ? sp::kRealLoadHold : sp::kThetaHold;
    const int div_threads = ceil_div((m + 1) / 2, div_hold) + ceil_div(m / 2, div_hold);
    const bool grad_one_line = rs_lam == sp::kRadixFixed5000;
    for (int g = grad_one_line ? 0 : p->rw_log2; g >= 0 && div_threads <= p->theta_threads; --g) {
        const size_t lds = ((size_t)(grad_one_line ? 1 : 2) * N << g) * sizeof(Cx<double>);
        if (lds + static_lds <= lds_limit) {
            p->grad = grad_kernel(rs_lam);
            p->grad_rw_log2 = g;
            p->grad_lds = lds;
            p->grad_block = round_up((1 << g) * p->lam_threads, 64);
            p->grad_grid = round_up((m + (1 << g) - 1) >> g, 8 << (p->lay_log2 - g));
            (void)hipFuncSetAttribute((const void*)p->grad, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            break;
        }
    }
    (void)hipGetLastError();

    // ---- device memory
    const bool mixed = d->precision == SP_MIXED;
    Layout L = layout_for(n, m, 1 << p->rw_log2, 1 << p->lay_log2, mixed);
    p->spec_elems = L.spec_elems;
    hipError_t e = hipMalloc(&p->block, L.total);
    if (e != hipSuccess) {
        delete p;
        (void)hipGetLastError();
        return SP_ERR_OOM;
    }
    p->block_bytes = L.total;
    unsigned char* b = (unsigned char*)p->block;
    p->spec64 = (Cx<double>*)(b + L.off_spec);
    p->t64.tw_n = (Cx<double>*)(b + L.off_tw64n);
    p->t64.pass_m = (Cx<double>*)(b + L.off_tw64m);
    p->t64.eq = (Cx<double>*)(b + L.off_eq64);
    p->t32.tw_n = (Cx<float>*)(b + L.off_tw32n);
    p->t32.pass_m = (Cx<float>*)(b + L.off_tw32m);
    p->t32.eq = (Cx<float>*)(b + L.off_eq32);
    p->t64.ws = (Cx<double>*)(b + L.off_ws64);
    p->t32.ws = (Cx<float>*)(b + L.off_ws32);
    p->t64.pass_n = (Cx<double>*)(b + L.off_p64n);
    p->t32.pass_n = (Cx<float>*)(b + L.off_p32n);
    p->sin2 = (double*)(b + L.off_sin2);
    p->k0tab = (double*)(b + L.off_k0);
    p->fint_w = (double*)(b + L.off_fint);
    p->scal = (double*)(b + L.off_scal);
    p->gradtab = (double*)(b + L.off_grad);
    p->intw = (double*)(b + L.off_intw);
    p->intpart = (double*)(b + L.off_intpart);
    p->specB = (Cx<double>*)(b + L.off_specB);
    if (mixed) {
        p->spec0 = (Cx<float>*)(b + L.off_spec0);
        p->specd = (Cx<float>*)(b + L.off_specd);
        p->partial = (double*)(b + L.off_partial);
        p->rnorm = (double*)(b + L.off_rnorm);
        p->fco = (Cx<double>*)(b + L.off_fco);
    }

    // ---- host tables
    std::vector<Cx<double>> twn(n), eq;
    for (int t = 0; t < n; ++t) cis_neg(t, n, &twn[t].x, &twn[t].y);
    std::vector<double> sin2, fint, k0;
    host_theta_tables(m, eq, sin2, k0, fint);
    auto to32 = [](const std::vector<Cx<double>>& v) {
        std::vector<Cx<float>> o(v.size());
        for (size_t i = 0; i < v.size(); ++i) o[i] = Cx<float>{(float)v[i].x, (float)v[i].y};
        return o;
    };
    std::vector<Cx<double>> ws(m / 4 + 1);
    for (int q = 0; q <= m / 4; ++q) cis_neg(q, m, &ws[q].x, &ws[q].y);
    std::vector<Cx<float>> twn32 = to32(twn), eq32 = to32(eq), pn32 = to32(ptab_n), pm32 = to32(ptab_m);
    std::vector<Cx<float>> ws32 = to32(ws);
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    };
    hipError_t ee = hipSuccess;
    if (ee == hipSuccess) ee = up(p->t64.tw_n, twn.data(), n * sizeof(Cx<double>));
    if (ee == hipSuccess) ee = up(p->t64.pass_m, ptab_m.data(), ptab_m.size() * sizeof(Cx<double>));
    if (ee == hipSuccess) ee = up(p->t64.eq, eq.data(), m * sizeof(Cx<double>));
    if (ee == hipSuccess) ee = up(p->t32.tw_n, twn32.data(), n * sizeof(Cx<float>));
    if (ee == hipSuccess) ee = up(p->t32.pass_m, pm32.data(), pm32.size() * sizeof(Cx<float>));
    if (ee == hipSuccess) ee = up(p->t32.eq, eq32.data(), m * sizeof(Cx<float>));
    if (ee == hipSuccess) ee = up(p->t64.ws, ws.data(), ws.size() * sizeof(Cx<double>));
    if (ee == hipSuccess) ee = up(p->t32.ws, ws32.data(), ws32.size() * sizeof(Cx<float>));
    if (ee == hipSuccess) ee = up(p->t64.pass_n, ptab_n.data(), ptab_n.size() * sizeof(Cx<double>));
    if (ee == hipSuccess) ee = up(p->t32.pass_n, pn32.data(), pn32.size() * sizeof(Cx<float>));
    if (ee == hipSuccess) ee = up(p->sin2, sin2.data(), m * sizeof(double));
    if (ee == hipSuccess) ee = up(p->k0tab, k0.data(), k0.size() * sizeof(double));
    if (ee == hipSuccess) ee = up(p->fint_w, fint.data(), m * sizeof(double));
    // gradient factors: cos(theta_j), sin(theta_j); sin(lambda_i), cos(lambda_i)
    // with lambda_i = -pi + 2 pi i/n, so (cos, sin)(lambda_i) = -(cos, sin)(2 pi i/n)
    std::vector<double> gtab((size_t)2 * m + 2 * n);
    for (int j = 0; j < m; ++j) {
        const long double th = ((long double)j + 0.5L) * 3.141592653589793238462643383279502884L / (long double)m;
        gtab[j] = (double)std::cos(th);
        gtab[m + j] = (double)std::sin(th);
    }
    for (int i = 0; i < n; ++i) {
        double c = 0.0, sn = 0.0;
        cis_neg(i, n, &c, &sn);                // e^{-2 pi i i/n} = (cos, -sin)
        gtab[2 * m + i] = sn;                  // sin(lambda_i) = -sin(2 pi i/n)
        gtab[2 * m + n + i] = -c;              // cos(lambda_i) = -cos(2 pi i/n)
    }
    if (ee == hipSuccess) ee = up(p->gradtab, gtab.data(), gtab.size() * sizeof(double));
    // integration: fint_w holds 2 pi W_j / sin^2(theta_j) (it is applied to the
    // spectrum of sin^2 f); the grid integral needs 2 pi W_j / n
    std::vector<double> intw(m);
    for (int j = 0; j < m; ++j) intw[j] = fint[j] * sin2[j] / n;
    if (ee == hipSuccess) ee = up(p->intw, intw.data(), intw.size() * sizeof(double));
    if (ee == hipSuccess) ee = hipStreamSynchronize(stream);
    if (ee != hipSuccess) {
        int r = hip_fail(ee, "uploading plan tables");
        (void)hipFree(p->block);
        delete p;
        return r;
    }
    plan_register(p);
    *out = p;
    return SP_OK;
}

// ------------------------------------------------------------ autotuner
// Per transform length: the lambda transform of n (radix order and rows per
// tile, any precision) and the theta transform of m (radix order of its DFT,
// length m/2 for even m and m for odd m, per
// precision).  Candidates are timed with HIP events on scratch problems; the
// fastest schedules are kept in a text cache, one line per entry:
//   <arch> lam <n> <rw_log2> <r1,r2,...>      <arch> theta <m> <precision> <r1,r2,...>
std::mutex g_tune_mu;
std::map<std::string, std::string> g_tune;   // key -> value, loaded lazily
bool g_tune_loaded = false;

std::string tune_path() {
    const char* e = std::getenv("SPHERE_POISSON_TUNE_CACHE");
    if (e && *e) return e;
    const char* h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/sphere_poisson_tune.txt";
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    FILE* fp = std::fopen(tune_path().c_str(), "r");
    if (!fp) return;
    char line[512];
    while (std::fgets(line, sizeof(line), fp)) {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        size_t cut = l.rfind(' ');
        if (cut == std::string::npos) continue;
        g_tune[l.substr(0, cut)] = l.substr(cut + 1);
    }
    std::fclose(fp);
}

void tune_save_locked() {
    std::string path = tune_path();
    size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash);
        (void)::mkdir(dir.c_str(), 0755);
    }
    std::string tmp = path + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;
    for (auto& kv : g_tune) std::fprintf(fp, "%s %s\n", kv.first.c_str(), kv.second.c_str());
    std::fclose(fp);
    std::rename(tmp.c_str(), path.c_str());
}

std::string radix_str(const std::vector<int>& r) {
    std::string s;
    for (size_t i = 0; i < r.size(); ++i) s += (i ? "," : "") + std::to_string(r[i]);
    return s;
}

std::vector<int> parse_radices(const std::string& s) {
    std::vector<int> r;
    size_t i = 0;
    while (i < s.size()) {
        size_t j = s.find(',', i);
        if (j == std::string::npos) j = s.size();
        r.push_back(std::atoi(s.substr(i, j - i).c_str()));
        i = j + 1;
    }
    return r;
}

std::string key_lam(int n) { return "gfx950 lam " + std::to_string(n); }
std::string key_theta(int m, int prec) { return "gfx950 theta " + std::to_string(m) + " " + std::to_string(prec); }

bool valid_radices(const std::vector<int>& r, int L) {
    if (is_fixed5000(r, L)) return true;
    long long prod = 1;
    for (int x : r) {
        static const int ok[] = {2, 3, 4, 5, 7, 8, 11, 13, 16, 17, 19, 23, 29, 31};
        if (std::find(std::begin(ok), std::end(ok), x) == std::end(ok)) return false;
        prod *= x;
    }
    return prod == L && (int)r.size() <= sp::kMaxPass;
}

// Radix orders to try for length L: power-of-two groupings (2, 4, 8, 16) with
// at most one pass more than the fewest, each combined with the odd primes in
// a few orders.
std::vector<std::vector<int>> radix_candidates(int L) {
    std::vector<std::vector<int>> out;
    if (L == 5000) out.push_back(std::vector<int>(std::begin(sp::kFixed5000Radices), std::end(sp::kFixed5000Radices)));
    int e = 0, odd = L;
    while (odd % 2 == 0) { odd /= 2; ++e; }
    std::vector<int> primes;
    for (int p : {3, 5, 7, 11, 13, 17, 19, 23, 29, 31})
        while (odd % p == 0) { primes.push_back(p); odd /= p; }
    if (odd != 1) return out;
    std::vector<std::vector<int>> groups;
    int minp = 1 << 30;
    for (int c16 = 0; 4 * c16 <= e; ++c16)
        for (int c8 = 0; 4 * c16 + 3 * c8 <= e; ++c8)
            for (int c4 = 0; 4 * c16 + 3 * c8 + 2 * c4 <= e; ++c4) {
                int c2 = e - 4 * c16 - 3 * c8 - 2 * c4;
                if (c2 > 1) continue;
                minp = std::min(minp, c16 + c8 + c4 + c2);
            }
    for (int c16 = 0; 4 * c16 <= e; ++c16)
        for (int c8 = 0; 4 * c16 + 3 * c8 <= e; ++c8)
            for (int c4 = 0; 4 * c16 + 3 * c8 + 2 * c4 <= e; ++c4) {
                int c2 = e - 4 * c16 - 3 * c8 - 2 * c4;
                if (c2 > 1 || c16 + c8 + c4 + c2 > minp + 1) continue;
                std::vector<int> g;
                g.insert(g.end(), c16, 16);
                g.insert(g.end(), c8, 8);
                g.insert(g.end(), c4, 4);
                g.insert(g.end(), c2, 2);
                groups.push_back(g);
            }
    for (auto& g : groups) {
        std::vector<int> pa = g, pb;
        pa.insert(pa.end(), primes.begin(), primes.end());        // powers of two first
        pb = primes;
        pb.insert(pb.end(), g.begin(), g.end());                  // odd primes first
        std::vector<int> pc(pa.rbegin(), pa.rend());             // reversed
        for (auto* v : {&pa, &pb, &pc})
            if (std::find(out.begin(), out.end(), *v) == out.end()) out.push_back(*v);
    }
    if (out.size() > 24) out.resize(24);
    return out;
}

float time_ms(hipStream_t s, const std::function<void()>& fn, int reps) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    fn();   // warm-up
    (void)hipEventRecord(a, s);
    for (int i = 0; i < reps; ++i) fn();
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

int run_fp64(sp_plan p, const double* in, double* out, int mode, double c0, bool fwd_sin2,
             bool adjoint_weights, bool want_fint, hipStream_t s);
int run_mixed(sp_plan p, const double* f, double* u, double c0, bool adjoint, hipStream_t s);

// Time one schedule: a full solve of a scratch problem (n, m, precision).
float time_schedule(const sp_desc& base, const Sched& sc, hipStream_t s, double* x, double* y) {
    sp_plan p = nullptr;
    if (plan_create(&base, s, sc, &p) != SP_OK || !p) {
        (void)hipGetLastError();
        return 1e30f;
    }
    auto fn = [&]() {
        if (base.precision == SP_MIXED) (void)run_mixed(p, x, y, 0.0, false, s);
        else (void)run_fp64(p, x, y, sp::kSolve, 0.0, true, false, false, s);
    };
    float ms = time_ms(s, fn, 3);
    if (hipGetLastError() != hipSuccess) ms = 1e30f;
    plan_unregister(p);
    (void)hipStreamSynchronize(s);
    (void)hipFree(p->block);
    delete p;
    return ms;
}

// Fill missing cache entries for (n, m, precision) by measurement.
int autotune(const sp_desc* d, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    const int n = d->n_lambda, m = d->m_theta, prec = d->precision;
    const bool need_lam = !g_tune.count(key_lam(n)), need_th = !g_tune.count(key_theta(m, prec));
    if (!need_lam && !need_th) return SP_OK;
    // scratch problems: n x 256 rows for the lambda transform, 512 x m for the theta transform
    const int mt = 256, nt = 512;
    const size_t cells = std::max((size_t)n * mt, (size_t)nt * m);
    double* x = nullptr;
    double* y = nullptr;
    if (hipMalloc(&x, cells * sizeof(double)) != hipSuccess || hipMalloc(&y, cells * sizeof(double)) != hipSuccess) {
        (void)hipFree(x);
        (void)hipGetLastError();
        return SP_ERR_OOM;
    }
    (void)hipMemsetAsync(x, 0, cells * sizeof(double), s);
    if (need_lam) {
        sp_desc b = *d;
        b.m_theta = mt;
        b.precision = SP_FP64;
        b.flags = 0;
        Sched best;
        float best_ms = 1e30f;
        for (auto& r : radix_candidates(n / 2)) {
            for (int rwl = 0; rwl <= 5; ++rwl) {
                Sched sc;
                sc.lam = r;
                sc.rw_log2 = rwl;
                const float ms = time_schedule(b, sc, s, x, y);
                if (ms < best_ms) { best_ms = ms; best = sc; }
            }
        }
        if (best_ms < 1e29f)
            g_tune[key_lam(n)] = std::to_string(best.rw_log2) + ":" + radix_str(best.lam);
    }
    if (need_th) {
        sp_desc b = *d;
        b.n_lambda = nt;
        b.flags = 0;
        Sched best;
        float best_ms = 1e30f;
        // even m: the real-part theta pass transforms length m/2
        for (auto& r : radix_candidates((m & 1) ? m : m / 2)) {
            Sched sc;
            sc.theta = r;
            const float ms = time_schedule(b, sc, s, x, y);
            if (ms < best_ms) { best_ms = ms; best = sc; }
        }
        if (best_ms < 1e29f) g_tune[key_theta(m, prec)] = radix_str(best.theta);
    }
    (void)hipFree(x);
    (void)hipFree(y);
    (void)hipGetLastError();
    tune_save_locked();
    return SP_OK;
}

// The schedule the cache holds for (n, m, precision) (empty fields: fixed rule).
Sched cached_schedule(int n, int m, int prec) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    Sched sc;
    auto it = g_tune.find(key_lam(n));
    if (it != g_tune.end()) {
        size_t c = it->second.find(':');
        if (c != std::string::npos) {
            std::vector<int> r = parse_radices(it->second.substr(c + 1));
            if (valid_radices(r, n / 2)) {
                sc.lam = r;
                sc.rw_log2 = std::atoi(it->second.substr(0, c).c_str());
            }
        }
    }
    it = g_tune.find(key_theta(m, prec));
    if (it != g_tune.end()) {
        std::vector<int> r = parse_radices(it->second);
        if (valid_radices(r, m) || ((m & 1) == 0 && valid_radices(r, m / 2))) sc.theta = r;
    }
    return sc;
}

bool autotune_requested(const sp_desc* d) {
    const char* e = std::getenv("SPHERE_POISSON_AUTOTUNE");
    return (d->flags & SP_AUTOTUNE) || (e && *e == '1');
}

}  // namespace

extern "C" int sphere_poisson_plan(sp_plan* out, const sp_desc* d, void* hip_stream) {
    if (!out) return SP_ERR_INVALID_ARG;
    *out = nullptr;
    int st = validate_desc(d);
    if (st != SP_OK) return st;
    int dev = 0;
    size_t lds_limit = 0;
    st = query_device(&dev, &lds_limit);
    if (st != SP_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;
    if (autotune_requested(d)) {
        st = autotune(d, stream);
        if (st != SP_OK) return st;
    }
    return plan_create(d, stream, cached_schedule(d->n_lambda, d->m_theta, d->precision), out);
}

namespace {
void free_events(sp_plan p) {
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    p->ev.clear();
    p->ev_kind.clear();
    p->ev_used = 0;
}
}  // namespace

extern "C" int sphere_poisson_profile_enable(sp_plan p, int capacity) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    if (capacity < 0) return SP_ERR_INVALID_ARG;
    SP_HIP(hipDeviceSynchronize());
    free_events(p);
    p->ev.resize(2 * (size_t)capacity);
    for (size_t i = 0; i < p->ev.size(); ++i) {
        hipError_t e = hipEventCreate(&p->ev[i]);
        if (e != hipSuccess) {
            p->ev.resize(i);
            free_events(p);
            return hip_fail(e, "hipEventCreate");
        }
    }
    p->ev_kind.assign(capacity, -1);
    return SP_OK;
}

extern "C" int sphere_poisson_profile_read(sp_plan p, double* total_ms, int* counts) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    double tot[SP_KERNEL_KINDS] = {0};
    int cnt[SP_KERNEL_KINDS] = {0};
    for (int i = 0; i < p->ev_used; ++i) {
        SP_HIP(hipEventSynchronize(p->ev[2 * i + 1]));
        float ms = 0.f;
        SP_HIP(hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]));
        int k = p->ev_kind[i];
        if (k >= 0 && k < SP_KERNEL_KINDS) { tot[k] += ms; cnt[k] += 1; }
    }
    p->ev_used = 0;
    for (int k = 0; k < SP_KERNEL_KINDS; ++k) {
        if (total_ms) total_ms[k] = tot[k];
        if (counts) counts[k] = cnt[k];
    }
    return SP_OK;
}

extern "C" int sphere_poisson_destroy(sp_plan p) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    plan_unregister(p);
    int st = SP_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) st = hip_fail(e, "hipDeviceSynchronize");
    free_events(p);
    if (p->block) {
        e = hipFree(p->block);
        if (e != hipSuccess && st == SP_OK) st = hip_fail(e, "hipFree");
    }
    delete p;
    return st;
}

namespace {

// Launch bracketing for the profiling calls (no-ops unless enabled).
struct ProfScope {
    sp_plan p;
    hipStream_t s;
    int slot = -1;
    ProfScope(sp_plan p_, int kind, hipStream_t s_) : p(p_), s(s_) {
        if (p->ev_used < (int)p->ev_kind.size()) {
            slot = p->ev_used++;
            p->ev_kind[slot] = kind;
            (void)hipEventRecord(p->ev[2 * slot], s);
        }
    }
    ~ProfScope() {
        if (slot >= 0) (void)hipEventRecord(p->ev[2 * slot + 1], s);
    }
};

bool overlap(const void* a, const void* b, size_t bytes) {
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

bool overlap(const void* a, const void* b, size_t abytes, size_t bbytes) {
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bbytes && y < x + abytes;
}

// The forward lambda pass (rows -> spectrum in runs of 8 rows) with the
// plan's forward tile.
template <typename T>
void launch_lambda_fwd(sp_plan p, void (*fn)(sp::LambdaArgs<T>), sp::LambdaArgs<T> a, hipStream_t s) {
    a.rw_log2 = p->fwd_rw_log2;
    hipLaunchKernelGGL(fn, dim3(p->fwd_grid), dim3(round_up((1 << p->fwd_rw_log2) * p->lam_threads, 64)), p->fwd_lds,
                       s, a);
}

// One FP64 pass over the three kernels: lambda forward, theta, lambda inverse.
int run_fp64(sp_plan p, const double* in, double* out, int mode, double c0, bool fwd_sin2,
             bool adjoint_weights, bool want_fint, hipStream_t s) {
    const int n = p->n, m = p->m, N = p->N;
    const int rw = 1 << p->rw_log2;
    sp::LambdaArgs<double> la{};
    la.x = in;
    la.y = out;
    la.spec = p->spec64;
    la.tw = p->t64.tw_n;
    la.ptw = p->t64.pass_n;
    la.n = n; la.m = m; la.N = N; la.rw_log2 = p->rw_log2; la.lay_log2 = p->lay_log2;
    la.fft = p->fft_lam;
    la.nthr = p->lam_threads;
    // forward lambda (in == nullptr: spec64 already holds the right-hand side's spectrum)
    la.rowscale = fwd_sin2 ? p->sin2 : nullptr;
    if (!adjoint_weights) { la.w_mid = 1.0 / n; la.w_end = 1.0 / n; }
    else { la.w_mid = 2.0; la.w_end = 1.0; }
    if (in) {
        ProfScope ps(p, SP_KERNEL_LAMBDA_FWD, s);
        launch_lambda_fwd(p, p->kd.fwd, la, s);
    }
    // theta
    sp::ThetaArgs<double> ta{};
    ta.spec = p->spec64;
    ta.tw = p->t64.pass_m;
    ta.eq = p->t64.eq;
    ta.ws = p->t64.ws;
    ta.spec_out = p->specB;
    ta.n = n; ta.m = m; ta.N = N; ta.lay_log2 = p->lay_log2; ta.lay_out_log2 = p->rw_log2;
    ta.fft = p->fft_theta;
    ta.nthr_fft = p->theta_fft_threads;
    ta.mode = mode;
    ta.k8 = p->k8;
    ta.c0 = c0;
    ta.k0tab = p->k0tab;
    ta.fint_w = want_fint ? p->fint_w : nullptr;
    ta.fint_out = p->scal;
    {
        ProfScope ps(p, SP_KERNEL_THETA, s);
        hipLaunchKernelGGL(p->theta_real ? p->kd.theta_real : p->kd.theta, dim3(p->theta_grid),
                           dim3(p->theta_threads), p->theta_lds64, s, ta);
    }
    // inverse lambda: reads the theta output, one contiguous block per workgroup
    la.spec = p->specB;
    la.lay_log2 = p->rw_log2;
    if (!adjoint_weights) { la.w_mid = 1.0; la.w_end = 1.0; la.out_scale = 1.0; la.rowscale = nullptr; }
    else { la.w_mid = 0.5; la.w_end = 1.0; la.out_scale = 1.0 / n; la.rowscale = p->sin2; }
    {
        ProfScope ps(p, SP_KERNEL_LAMBDA_INV, s);
        hipLaunchKernelGGL(p->kd.inv, dim3(p->lam_grid), dim3(round_up(rw * p->lam_threads, 64)), p->lam_lds, s, la);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return SP_OK;
}

// The info of a solve from the device scalars (after a synchronisation);
// `norms`: the plan collected them (SP_SYNC_INFO or SP_INFO), else they read -1.
int read_info(sp_plan p, hipStream_t s, sp_info* info, int status, int iters, bool norms) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    double sc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    e = hipMemcpy(sc, p->scal, sizeof(sc), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy info");
    double rel = 0.0, res = 0.0, est = 0.0;
    if (iters > 0 && norms) {
        rel = sc[2] > 0.0 ? std::sqrt(sc[1] / sc[2]) : 0.0;
        res = sc[4] > 0.0 ? std::sqrt(sc[3] / sc[4]) : 0.0;
        // contraction: the ratio of the last two corrections, or with one
        // correction its own relative size (the float32 solve's relative error)
        const double prev = (iters >= 2 && sc[6] > 0.0) ? std::sqrt(sc[5] / sc[6]) : 0.0;
        const double rho = iters >= 2 ? (prev > 0.0 ? rel / prev : 0.0) : rel;
        est = rel * rho;
    } else if (!norms && p->desc.precision == SP_MIXED) {
        rel = res = est = -1.0;
    }
    if (norms && iters > 0 && p->desc.tol > 0.0 && !(rel <= p->desc.tol)) status = SP_ERR_NOT_CONVERGED;
    if (norms && p->desc.precision == SP_MIXED && iters == 0 && p->desc.tol > 0.0) status = SP_ERR_NOT_CONVERGED;
    if (info) {
        info->iters = iters;
        info->rel_correction = rel;
        info->f_integral = sc[0];
        info->status = status;
        info->rel_residual = res;
        info->est_rel_err = est;
    }
    return status;
}

int finish_info(sp_plan p, hipStream_t s, sp_info* info, int status, int iters) {
    p->last_status = status;
    p->last_iters = iters;
    if (!(p->desc.flags & SP_SYNC_INFO)) return status;
    status = read_info(p, s, info, status, iters, true);
    p->last_status = status;
    return status;
}

// MIXED: float64 right-hand side transform, float32 bulk solve, `max_refine`
// float64-residual corrections (see the mixed kernels).
int run_mixed(sp_plan p, const double* f, double* u, double c0, bool adjoint, hipStream_t s) {
    const int n = p->n, m = p->m, N = p->N;
    const int rw = 1 << p->rw_log2;
    const int nblk = (m + rw - 1) / rw;
    const bool want = (p->desc.flags & (SP_SYNC_INFO | SP_INFO)) != 0;
    const dim3 lam_grid(p->lam_grid), lam_block(round_up(rw * p->lam_threads, 64));
    const dim3 th_grid(p->theta_grid), th_block(p->theta_threads);
    const int tv = p->theta_real ? 1 : 0;
    const int ntiles = p->theta_real ? 2 * (N + 1) : N + 1;   // theta tiles (residual-norm partials)
    // 1. float64 lambda transform of sin^2 f -> spec64
    sp::LambdaArgs<double> la{};
    // forward: sin^2 f with weight 1/n; adjoint: the transpose of the inverse real DFT
    // (weights 2 for 0 < k < n/2, 1 at the ends, no sin^2)
    la.x = f; la.spec = p->spec64; la.tw = p->t64.tw_n; la.ptw = p->t64.pass_n;
    la.rowscale = adjoint ? nullptr : p->sin2;
    la.n = n; la.m = m; la.N = N; la.rw_log2 = p->rw_log2; la.lay_log2 = p->lay_log2; la.fft = p->fft_lam;
    la.nthr = p->lam_threads;
    la.w_mid = adjoint ? 2.0 : 1.0 / n;
    la.w_end = adjoint ? 1.0 : 1.0 / n;
    if (f) {   // f == nullptr: spec64 already holds the right-hand side's spectrum
        ProfScope ps(p, SP_KERNEL_LAMBDA_FWD, s);
        launch_lambda_fwd(p, p->kd.fwd, la, s);
    }
    // 2. first solve
    sp::ThetaMixArgs ta{};
    ta.sa = p->spec64; ta.fco = p->fco; ta.su = p->specB; ta.out = p->spec0;
    ta.tw64 = p->t64.pass_m; ta.eq64 = p->t64.eq; ta.tw32 = p->t32.pass_m; ta.eq32 = p->t32.eq;
    ta.ws64 = p->t64.ws; ta.ws32 = p->t32.ws;
    // the float32 spectra keep theta's run length: written by halves (one real
    // part per workgroup), shorter runs fragment those writes more than they
    // help the lambda reads
    ta.n = n; ta.m = m; ta.N = N; ta.lay_log2 = p->lay_log2; ta.lay_out_log2 = p->lay_log2; ta.fft = p->fft_theta;
    ta.nthr_fft = p->theta_fft_threads; ta.k8 = p->k8; ta.c0 = c0; ta.k0tab = p->k0tab;
    ta.fint_w = p->fint_w; ta.fint_out = p->scal;
    ta.k64 = p->desc.low_k_fp64 < 0 ? std::max(16, m / 64) : std::max(1, p->desc.low_k_fp64);
    ta.rnorm = nullptr;
    {
        ProfScope ps(p, SP_KERNEL_THETA, s);
        hipLaunchKernelGGL(adjoint ? p->km.theta_first_t[tv] : p->km.theta_first[tv], th_grid, th_block, p->theta_lds64,
                           s, ta);
    }
    const int R = p->desc.max_refine;
    if (R == 0) {
        sp::LambdaArgs<float> lf{};
        lf.y = u; lf.spec = p->spec0; lf.tw = p->t32.tw_n; lf.ptw = p->t32.pass_n;
        lf.rowscale = adjoint ? p->sin2 : nullptr;
        lf.n = n; lf.m = m; lf.N = N; lf.rw_log2 = p->rw_log2; lf.lay_log2 = p->lay_log2; lf.fft = p->fft_lam;
        lf.nthr = p->lam_threads;
        lf.w_mid = adjoint ? 0.5f : 1.0f; lf.w_end = 1.0f; lf.out_scale = adjoint ? 1.0 / n : 1.0;
        ProfScope ps(p, SP_KERNEL_LAMBDA_INV, s);
        hipLaunchKernelGGL(p->kf.inv, lam_grid, lam_block, p->lam_lds, s, lf);
    } else {
        sp::MixLambdaArgs ma{};
        ma.s0 = p->spec0; ma.sd = p->specd; ma.su = p->specB; ma.u = u;
        ma.tw32 = p->t32.tw_n; ma.tw64 = p->t64.tw_n; ma.partial = want ? p->partial : nullptr;
        ma.ptw32 = p->t32.pass_n; ma.ptw64 = p->t64.pass_n;
        ma.n = n; ma.m = m; ma.N = N; ma.rw_log2 = p->rw_log2;
        ma.lay_log2 = p->lay_log2;      // float32 spectra written by theta
        ma.lay_out_log2 = p->lay_log2;  // float64 spectrum of the iterate, read by theta
        ma.fft = p->fft_lam; ma.nthr = p->lam_threads; ma.accumulate = 0;
        if (!adjoint) {
            ma.in_w_mid = 1.0f; ma.in_w_end = 1.0f; ma.mid_scale = 1.0;
            ma.out_w_mid = 1.0 / n; ma.out_w_end = 1.0 / n;
            ma.rowscale = nullptr; ma.out_scale = 1.0;
        } else {
            // h = (1/n) C2R(y / c) is the transposed real DFT; its coefficients for the
            // residual are c n R2C(h), i.e. the raw DFT with weights (1, 2, ..., 2, 1)
            ma.in_w_mid = 0.5f; ma.in_w_end = 1.0f; ma.mid_scale = 1.0 / n;
            ma.out_w_mid = 2.0; ma.out_w_end = 1.0;
            ma.rowscale = p->sin2; ma.out_scale = 1.0 / n;
        }
        {
            ProfScope ps(p, SP_KERNEL_LAMBDA_MIX, s);
            hipLaunchKernelGGL(p->km.mix, lam_grid, lam_block, p->lam_lds, s, ma);
        }
        ta.out = p->specd;
        ta.fint_w = nullptr;
        for (int it = 1; it <= R; ++it) {
            if (it > 1) {
                // float64 lambda transform of the current iterate (no sin^2) -> specB
                if (adjoint) return SP_ERR_INVALID_ARG;   // checked by the caller: adjoint uses one correction
                la.x = u; la.spec = p->specB; la.rowscale = nullptr;
                ProfScope ps(p, SP_KERNEL_LAMBDA_FWD, s);
                launch_lambda_fwd(p, p->kd.fwd, la, s);
            }
            // the last correction pass also sums the residual of its iterate (info builds)
            const bool norm = want && it == R;
            ta.rnorm = norm ? p->rnorm : nullptr;
            {
                ProfScope ps(p, SP_KERNEL_THETA_RESID, s);
                auto* fn = adjoint ? (norm ? p->km.theta_resid_t_norm[tv] : p->km.theta_resid_t[tv])
                                   : (norm ? p->km.theta_resid_norm[tv] : p->km.theta_resid[tv]);
                hipLaunchKernelGGL(fn, th_grid, th_block, p->theta_lds64, s, ta);
            }
            ma.accumulate = it > 1 ? 1 : 0;
            {
                ProfScope ps(p, SP_KERNEL_LAMBDA_UPD, s);
                // float32 correction lines only: half the LDS of the other lambda passes
                hipLaunchKernelGGL(p->km.update, lam_grid, dim3(p->upd_block), p->lam_lds / 2, s, ma);
            }
            // correction norms of the last two corrections: [1..2] last, [5..6] the one before
            if (want && it >= R - 1) {
                ProfScope ps(p, SP_KERNEL_REDUCE, s);
                hipLaunchKernelGGL(sp::k_reduce_partials, dim3(1), dim3(256), 0, s, (const double*)p->partial, nblk,
                                   p->scal + (it == R ? 1 : 5));
            }
        }
        if (want) {
            ProfScope ps(p, SP_KERNEL_REDUCE, s);
            hipLaunchKernelGGL(sp::k_reduce_partials, dim3(1), dim3(256), 0, s, (const double*)p->rnorm, ntiles,
                               p->scal + 3);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return SP_OK;
}

// The adjoint refinement recovers the coefficients of its iterate h through
// c n R2C(h) (h itself, not sin^2 h, is refined), so any number of corrections
// would need the sin^2-free iterate kept separately; one correction is used.
int run_mixed_adjoint(sp_plan p, const double* g, double* fbar, int R, hipStream_t s) {
    const int saved = p->desc.max_refine;
    p->desc.max_refine = R;
    int st = run_mixed(p, g, fbar, 0.0, true, s);
    p->desc.max_refine = saved;
    return st;
}

}  // namespace

extern "C" int sphere_poisson_solve(sp_plan p, const double* f, double* u, double integral,
                                    void* hip_stream, sp_info* info) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    if (!f || !u) return SP_ERR_INVALID_ARG;
    const size_t bytes = (size_t)p->n * p->m * sizeof(double);
    if (overlap(f, u, bytes)) return SP_ERR_ALIAS;
    hipStream_t s = (hipStream_t)hip_stream;
    const double PI = 3.14159265358979323846;
    if (p->desc.precision == SP_MIXED) {
        int st = run_mixed(p, f, u, integral / (4.0 * PI), false, s);
        if (st != SP_OK) return st;
        return finish_info(p, s, info, SP_OK, p->desc.max_refine);
    }
    int st = run_fp64(p, f, u, sp::kSolve, integral / (4.0 * PI), true, false, true, s);
    if (st != SP_OK) return st;
    return finish_info(p, s, info, SP_OK, 0);
}

// Low-rank right-hand side: the lambda pass on the K rows of r (row scale d,
// one row per workgroup, rows contiguous) into specB, then the rank-K product
// into spec64; specB is free until the theta pass writes it.
int lowrank_rhs(sp_plan p, int rank, const double* d, const double* c, const double* r, hipStream_t s) {
    const int n = p->n, N = p->N;
    sp::LambdaArgs<double> la{};
    la.x = r; la.spec = p->specB; la.tw = p->t64.tw_n; la.ptw = p->t64.pass_n;
    la.rowscale = d;
    la.n = n; la.m = rank; la.N = N; la.rw_log2 = 0; la.lay_log2 = 0;
    la.fft = p->fft_lam; la.nthr = p->lam_threads;
    la.w_mid = 1.0 / n; la.w_end = 1.0 / n;
    {
        ProfScope ps(p, SP_KERNEL_LAMBDA_FWD, s);
        hipLaunchKernelGGL(p->kd.fwd, dim3(round_up(rank, 8)), dim3(round_up(p->lam_threads, 64)),
                           p->lam_lds >> p->rw_log2, s, la);
    }
    {
        ProfScope ps(p, SP_KERNEL_LOWRANK, s);
        const dim3 grid(ceil_div(p->m, sp::kLowRankRows), ceil_div(N + 1, sp::kLowRankThreads));
        hipLaunchKernelGGL(sp::k_lowrank_rhs<sp::kLowRankRows>, grid, dim3(sp::kLowRankThreads), 0, s,
                           (const double*)c, (const double*)p->sin2, (const Cx<double>*)p->specB, p->spec64, rank,
                           p->m, N, p->lay_log2);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return SP_OK;
}

extern "C" int sphere_poisson_solve_lowrank(sp_plan p, int rank, const double* d, const double* c, const double* r,
                                            double* u, double integral, void* hip_stream, sp_info* info) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    if (!d || !c || !r || !u || rank < 1 || rank > p->m) return SP_ERR_INVALID_ARG;
    const size_t ub = (size_t)p->n * p->m * sizeof(double);
    if (overlap(u, c, ub, (size_t)rank * p->m * sizeof(double)) ||
        overlap(u, r, ub, (size_t)rank * p->n * sizeof(double)) || overlap(u, d, ub, (size_t)rank * sizeof(double)))
        return SP_ERR_ALIAS;
    hipStream_t s = (hipStream_t)hip_stream;
    int st = lowrank_rhs(p, rank, d, c, r, s);
    if (st != SP_OK) return st;
    const double PI = 3.14159265358979323846;
    if (p->desc.precision == SP_MIXED) {
        st = run_mixed(p, nullptr, u, integral / (4.0 * PI), false, s);
        if (st != SP_OK) return st;
        return finish_info(p, s, info, SP_OK, p->desc.max_refine);
    }
    st = run_fp64(p, nullptr, u, sp::kSolve, integral / (4.0 * PI), true, false, true, s);
    if (st != SP_OK) return st;
    return finish_info(p, s, info, SP_OK, 0);
}

extern "C" int sphere_poisson_eval_lowrank(sp_plan p, int rank, const double* d, const double* c, const double* r,
                                           int npts, const double* xyz, double* out, void* hip_stream) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    if (!d || !c || !r || rank < 1 || rank > p->m || rank > p->N + 1 || npts < 0) return SP_ERR_INVALID_ARG;
    if (npts == 0) return SP_OK;
    if (!xyz || !out) return SP_ERR_INVALID_ARG;
    const size_t ob = (size_t)npts * sizeof(double);
    if (overlap(out, xyz, ob, 3 * ob) || overlap(out, c, ob, (size_t)rank * p->m * sizeof(double)) ||
        overlap(out, r, ob, (size_t)rank * p->n * sizeof(double)) || overlap(out, d, ob, (size_t)rank * sizeof(double)))
        return SP_ERR_ALIAS;
    hipStream_t s = (hipStream_t)hip_stream;
    const int n = p->n, m = p->m, N = p->N;
    // lambda coefficients of the rows of r, times d and the real-series weights -> specB
    sp::LambdaArgs<double> la{};
    la.x = r; la.spec = p->specB; la.tw = p->t64.tw_n; la.ptw = p->t64.pass_n;
    la.rowscale = d;
    la.n = n; la.m = rank; la.N = N; la.rw_log2 = 0; la.lay_log2 = 0;
    la.fft = p->fft_lam; la.nthr = p->lam_threads;
    la.w_mid = 2.0 / n; la.w_end = 1.0 / n;
    {
        ProfScope ps(p, SP_KERNEL_LAMBDA_FWD, s);
        hipLaunchKernelGGL(p->kd.fwd, dim3(round_up(rank, 8)), dim3(round_up(p->lam_threads, 64)),
                           p->lam_lds >> p->rw_log2, s, la);
    }
    // cosine and sine coefficients of the theta factors -> spec64 (2 rank m <= 2 m (N + 1) doubles)
    double* alpha = reinterpret_cast<double*>(p->spec64);
    double* beta = alpha + (size_t)rank * m;
    {
        ProfScope ps(p, SP_KERNEL_EVAL_COEFFS, s);
        hipLaunchKernelGGL(sp::k_trig_coeffs, dim3(rank, ceil_div(m, 256)), dim3(256), 0, s, c, m, alpha, beta);
    }
    {
        ProfScope ps(p, SP_KERNEL_EVAL, s);
        hipLaunchKernelGGL(sp::k_eval_lowrank, dim3(ceil_div(npts, 256 * sp::kEvalPoints)), dim3(256), 0, s,
                           (const double*)alpha,
                           (const double*)beta, (const Cx<double>*)p->specB, rank, m, N, xyz, npts, out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return SP_OK;
}

extern "C" int sphere_poisson_solve_adjoint(sp_plan p, const double* g, double* fbar, void* hip_stream,
                                            sp_info* info) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    if (!g || !fbar) return SP_ERR_INVALID_ARG;
    const size_t bytes = (size_t)p->n * p->m * sizeof(double);
    if (overlap(g, fbar, bytes)) return SP_ERR_ALIAS;
    hipStream_t s = (hipStream_t)hip_stream;
    if (p->desc.precision == SP_MIXED) {
        // the adjoint refinement supports one correction (see run_mixed_adjoint)
        if (p->desc.max_refine > 1) return SP_ERR_INVALID_ARG;
        const int R = p->desc.max_refine;
        int st = run_mixed_adjoint(p, g, fbar, R, s);
        if (st != SP_OK) return st;
        return finish_info(p, s, info, SP_OK, R);
    }
    int st = run_fp64(p, g, fbar, sp::kSolveTransposed, 0.0, false, true, false, s);
    if (st != SP_OK) return st;
    return finish_info(p, s, info, SP_OK, 0);
}

extern "C" int sphere_poisson_get_info(sp_plan p, void* hip_stream, sp_info* info) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    if (!info) return SP_ERR_INVALID_ARG;
    const bool norms = (p->desc.flags & (SP_SYNC_INFO | SP_INFO)) != 0;
    const int st = read_info(p, (hipStream_t)hip_stream, info, p->last_status, p->last_iters, norms);
    // a HIP failure is the call's own error; otherwise the last solve's status
    return st == SP_ERR_HIP ? st : SP_OK;
}

extern "C" int sphere_poisson_transform_roundtrip(sp_plan p, const double* f, double* out, void* hip_stream) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    if (!f || !out) return SP_ERR_INVALID_ARG;
    const size_t bytes = (size_t)p->n * p->m * sizeof(double);
    if (overlap(f, out, bytes)) return SP_ERR_ALIAS;
    return run_fp64(p, f, out, sp::kTransformOnly, 0.0, true, false, false, (hipStream_t)hip_stream);
}

// ------------------------------------------------------------ tangential gradient
namespace {

// What the gradient pass writes from the gradient g of one scalar field
// (Section 4, Vector calculus): the gradient, n x g (the curl of a scalar),
// or the term that component c of a vector field adds to its divergence,
// surface curl or vorticity.
enum GradOut { kGradient = 0, kNormalCross = 1, kDivTerm = 2, kCurlTerm = 3, kVortTerm = 4 };

void grad_weights(int out_mode, int c, sp::GradArgs& ga) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) { ga.wg[a][b] = 0.0; ga.wn[a][b] = 0.0; }
    ga.nout = 3;
    switch (out_mode) {
        case kGradient: for (int a = 0; a < 3; ++a) ga.wg[a][a] = 1.0; break;
        case kNormalCross: for (int a = 0; a < 3; ++a) ga.wn[a][a] = 1.0; break;
        case kDivTerm: ga.wg[0][c] = 1.0; ga.nout = 1; break;
        case kCurlTerm:   // curl_a = sum_{b} eps_{a b c} d_b f_c
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const int e = (a - b) * (b - c) * (c - a);   // Levi-Civita: +2 / -2 / 0
                    ga.wg[a][b] = e > 0 ? 1.0 : e < 0 ? -1.0 : 0.0;
                }
            break;
        default: ga.wn[0][c] = 1.0; ga.nout = 1; break;   // kVortTerm: (n x grad f_c)_c
    }
}

// The tangential derivatives of one grid function f, written or added
// (accumulate) as the output mode asks.
int run_grad(sp_plan p, const double* f, int out_mode, int comp, bool accumulate, double* o0, double* o1,
             double* o2, hipStream_t s) {
    if (!p->grad) return SP_ERR_UNSUPPORTED_SIZE;
    const int n = p->n, m = p->m, N = p->N;
    const int rw = 1 << p->rw_log2;
    // 1. half spectrum of f (weights 1/n) -> spec64
    sp::LambdaArgs<double> la{};
    la.x = f; la.spec = p->spec64; la.tw = p->t64.tw_n; la.ptw = p->t64.pass_n; la.rowscale = nullptr;
    la.n = n; la.m = m; la.N = N; la.rw_log2 = p->rw_log2; la.lay_log2 = p->lay_log2; la.fft = p->fft_lam;
    la.nthr = p->lam_threads; la.w_mid = 1.0 / n; la.w_end = 1.0 / n;
    {
        ProfScope ps(p, SP_KERNEL_LAMBDA_FWD, s);
        hipLaunchKernelGGL(p->kd.fwd, dim3(p->lam_grid), dim3(round_up(rw * p->lam_threads, 64)), p->lam_lds, s, la);
    }
    // 2. theta derivative of every wavenumber's series -> specB (same run length);
    // 3. then each series divided by sin(theta), in place (every workgroup reads
    //    its whole column part before writing it)
    sp::ThetaArgs<double> ta{};
    ta.spec = p->spec64; ta.spec_out = p->specB; ta.tw = p->t64.pass_m; ta.eq = p->t64.eq; ta.ws = p->t64.ws;
    ta.n = n; ta.m = m; ta.N = N; ta.lay_log2 = p->lay_log2; ta.lay_out_log2 = p->lay_log2;
    ta.fft = p->fft_theta; ta.nthr_fft = p->theta_fft_threads; ta.mode = sp::kDerivative; ta.k8 = p->k8;
    ta.c0 = 0.0; ta.k0tab = p->k0tab; ta.fint_w = nullptr; ta.fint_out = p->scal;
    for (int mode : {(int)sp::kDerivative, (int)sp::kDivideSin}) {
        ta.mode = mode;
        ta.spec_out = mode == sp::kDerivative ? p->specB : p->spec64;
        ProfScope ps(p, SP_KERNEL_THETA, s);
        hipLaunchKernelGGL(p->theta_real ? p->kd.theta_real : p->kd.theta, dim3(p->theta_grid),
                           dim3(p->theta_threads), p->theta_lds64, s, ta);
    }
    // 4. both inverse lambda transforms per row, combined into the outputs
    sp::GradArgs ga{};
    ga.spec_q = p->spec64; ga.spec_t = p->specB; ga.gx = o0; ga.gy = o1; ga.gz = o2;
    grad_weights(out_mode, comp, ga);
    ga.accumulate = accumulate ? 1 : 0;
    ga.tw = p->t64.tw_n; ga.ptw = p->t64.pass_n; ga.rowtab = p->gradtab; ga.coltab = p->gradtab + 2 * (size_t)m;
    ga.n = n; ga.m = m; ga.N = N; ga.rw_log2 = p->grad_rw_log2; ga.lay_log2 = p->lay_log2;
    ga.fft = p->fft_lam; ga.nthr = p->lam_threads;
    {
        ProfScope ps(p, SP_KERNEL_LAMBDA_GRAD, s);
        hipLaunchKernelGGL(p->grad, dim3(p->grad_grid), dim3(p->grad_block), p->grad_lds, s, ga);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return SP_OK;
}

// Argument checks shared by the vector-calculus entry points: every pointer
// set, and no output overlapping an input or another output.
int check_fields(sp_plan p, const double* const* in, int nin, double* const* out, int nout) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    for (int a = 0; a < nin; ++a)
        if (!in[a]) return SP_ERR_INVALID_ARG;
    for (int a = 0; a < nout; ++a)
        if (!out[a]) return SP_ERR_INVALID_ARG;
    const size_t bytes = (size_t)p->n * p->m * sizeof(double);
    for (int a = 0; a < nout; ++a) {
        for (int b = 0; b < nin; ++b)
            if (overlap(out[a], in[b], bytes)) return SP_ERR_ALIAS;
        for (int b = a + 1; b < nout; ++b)
            if (overlap(out[a], out[b], bytes)) return SP_ERR_ALIAS;
    }
    return p->grad ? SP_OK : SP_ERR_UNSUPPORTED_SIZE;
}

// A vector field's three components, each through run_grad, the first
// writing the outputs and the others adding to them.
int run_vector_op(sp_plan p, const double* const* fc, int mode, double* o0, double* o1, double* o2,
                  hipStream_t s) {
    for (int c = 0; c < 3; ++c) {
        const int st = run_grad(p, fc[c], mode, c, c > 0, o0, o1, o2, s);
        if (st != SP_OK) return st;
    }
    return SP_OK;
}

}  // namespace

// ------------------------------------------------------------ tangential derivatives and vector calculus
extern "C" int sphere_poisson_tangential_gradient(sp_plan p, const double* f, double* gx, double* gy, double* gz,
                                                  void* hip_stream) {
    const double* in[1] = {f};
    double* out[3] = {gx, gy, gz};
    const int st = check_fields(p, in, 1, out, 3);
    if (st != SP_OK) return st;
    return run_grad(p, f, kGradient, 0, false, gx, gy, gz, (hipStream_t)hip_stream);
}

extern "C" int sphere_poisson_curl_scalar(sp_plan p, const double* f, double* ux, double* uy, double* uz,
                                          void* hip_stream) {
    const double* in[1] = {f};
    double* out[3] = {ux, uy, uz};
    const int st = check_fields(p, in, 1, out, 3);
    if (st != SP_OK) return st;
    return run_grad(p, f, kNormalCross, 0, false, ux, uy, uz, (hipStream_t)hip_stream);
}

extern "C" int sphere_poisson_divergence(sp_plan p, const double* fx, const double* fy, const double* fz,
                                         double* out, void* hip_stream) {
    const double* in[3] = {fx, fy, fz};
    double* outs[1] = {out};
    const int st = check_fields(p, in, 3, outs, 1);
    if (st != SP_OK) return st;
    return run_vector_op(p, in, kDivTerm, out, nullptr, nullptr, (hipStream_t)hip_stream);
}

extern "C" int sphere_poisson_curl(sp_plan p, const double* fx, const double* fy, const double* fz, double* cx,
                                   double* cy, double* cz, void* hip_stream) {
    const double* in[3] = {fx, fy, fz};
    double* outs[3] = {cx, cy, cz};
    const int st = check_fields(p, in, 3, outs, 3);
    if (st != SP_OK) return st;
    return run_vector_op(p, in, kCurlTerm, cx, cy, cz, (hipStream_t)hip_stream);
}

extern "C" int sphere_poisson_vorticity(sp_plan p, const double* fx, const double* fy, const double* fz,
                                        double* out, void* hip_stream) {
    const double* in[3] = {fx, fy, fz};
    double* outs[1] = {out};
    const int st = check_fields(p, in, 3, outs, 1);
    if (st != SP_OK) return st;
    return run_vector_op(p, in, kVortTerm, out, nullptr, nullptr, (hipStream_t)hip_stream);
}

// ------------------------------------------------------------ integration
extern "C" int sphere_poisson_integral(sp_plan p, const double* f, double* out, void* hip_stream) {
    if (!plan_ok(p)) return SP_ERR_BAD_PLAN;
    if (!f || !out) return SP_ERR_INVALID_ARG;
    if (overlap(f, out, (size_t)p->n * p->m * sizeof(double))) return SP_ERR_ALIAS;
    hipStream_t s = (hipStream_t)hip_stream;
    const int nb = std::min(p->m, kIntegralBlocks);
    hipLaunchKernelGGL(sp::k_integral_rows, dim3(nb), dim3(256), 0, s, f, (const double*)p->intw, p->n, p->m,
                       p->intpart);
    hipLaunchKernelGGL(sp::k_integral_total, dim3(1), dim3(256), 0, s, (const double*)p->intpart, nb, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return SP_OK;
}

// ------------------------------------------------------------ batches
namespace {

constexpr size_t kBatchLamLds = 64 * 1024;   // LDS budget of a lambda tile (rows per tile follow)

struct SizeTables {              // tables shared by every problem with the same n (or m)
    int len = 0;
    std::vector<int> radices;
    FftDesc desc{};
    size_t off64 = 0, off32 = 0, offp64 = 0, offp32 = 0;   // lambda: tw_n and pass tables
    size_t offeq64 = 0, offeq32 = 0, offsin2 = 0, offk0 = 0, offfint = 0;  // theta extras
    size_t offws64 = 0, offws32 = 0;   // theta: real-part split twiddles
};


// Builds of every stage (a problem's class per stage):
//   0: radices up to 16, 256 threads, 128 registers (168 for the complex
//      theta line, whose bodies hold two solves' state);
//   1: radices up to 31, 256 threads, 256 registers;
//   2, 3 (theta only): one real part per tile (even m), 128 threads and
//      chunks of up to 17 rows, radices up to 16 in 168 registers or up to 31
//      in 256;
//   4, 5 (theta only): the same in one wave (64 threads, chunks of up to 21
//      rows) for the lines that fit it (m up to 1344).
// A problem runs in the small-radix build of a stage when the transform of
// that stage's direction uses no radix above 16.  Small tiles keep more
// wavenumbers in flight per compute unit; a line of m <= 2048 gives few
// threads work in any phase.


int radix_class(const std::vector<int>& rad) {
    for (int r : rad)
        if (r > kBatchSmallRadix) return 1;
    return 0;
}

// per-problem launch parameters inside the batch tiles; rl / rt: radix
// orders (empty: fixed rule).  Even m runs one real part per theta tile (DFT
// length m/2) in one wave when the line fits it, else in 128 threads when it
// fits those; otherwise the complex line (DFT length m) in a 256-thread tile.
// *th_real: threads of the real-part tile, 0 for the complex line.
bool batch_schedule(int n, int m, std::vector<int>& rl, std::vector<int>& rt, int* rwl, int* lam_nthr,
                    int* th_fft, int* th_real) {
    const int N = n / 2;
    if (!valid_radices(rl, N)) rl.clear();
    if (rl.empty() && !factorize(N, rl)) return false;
    const int t = fft_threads(rl, N);
    if (t > kBatchThreads) return false;
    int best = 0;
    for (int l = 0; l <= 5; ++l) {
        const int rw = 1 << l;
        if (rw * t > kBatchThreads || (size_t)rw * N * sizeof(Cx<double>) > kBatchLamLds) break;
        best = l;
        if (rw >= m) break;
    }
    *rwl = best;
    *lam_nthr = t;
    *th_real = 0;
    if ((m & 1) == 0) {
        std::vector<int> r = rt;
        if (!valid_radices(r, m / 2)) r.clear();
        if (!r.empty() || factorize(m / 2, r)) {
            const int f = fft_threads(r, m / 2);
            const int base = std::max(f, sp::real_theta_min_threads(m));
            const int nt = std::max(base, solve_threads(m, kSmaxR)) <= kBatchWaveThreads ? kBatchWaveThreads
                         : std::max(base, solve_threads(m, kBatchSmaxR)) <= kBatchRealThreads ? kBatchRealThreads : 0;
            if (nt) {
                rt = r;
                *th_fft = f;
                *th_real = nt;
                return true;
            }
        }
    }
    if (!valid_radices(rt, m)) rt.clear();
    if (rt.empty() && !factorize(m, rt)) return false;
    *th_fft = fft_threads(rt, m);
    const int need = std::max(std::max(*th_fft, ceil_div(m, sp::kThetaHold)),
                              std::max(solve_threads(m, kSmaxD), solve_threads(m, kSmaxF)));
    return need <= kBatchThreads;
}

}  // namespace

namespace {

void host_theta_tables(int m, std::vector<Cx<double>>& eq, std::vector<double>& sin2, std::vector<double>& k0,
                       std::vector<double>& fint);

int build_batch(int count, const int* n, const int* m, const double* const* f, double* const* u, int precision,
                int R, double tol, bool tune, sp_batch_s** out) {
    int dev = 0;
    size_t lds_limit = 0;
    int st = query_device(&dev, &lds_limit);
    if (st != SP_OK) return st;
    hipDeviceProp_t prop;
    SP_HIP(hipGetDeviceProperties(&prop, dev));
    const bool mixed = precision == SP_MIXED;
    // radix orders per distinct n and m: the autotuner cache, measured first when requested
    const char* env = std::getenv("SPHERE_POISSON_AUTOTUNE");
    if (tune || (env && *env == '1')) {
        std::map<int, int> seen_n, seen_m;
        for (int r = 0; r < count; ++r) {
            if (seen_n.count(n[r]) && seen_m.count(m[r])) continue;
            seen_n[n[r]] = 1;
            seen_m[m[r]] = 1;
            sp_desc d{};
            d.n_lambda = n[r]; d.m_theta = m[r]; d.precision = precision; d.max_refine = 1;
            int st2 = autotune(&d, nullptr);
            if (st2 != SP_OK) return st2;
        }
    }
    std::vector<int> rwl(count), lnt(count), tft(count);
    std::vector<std::vector<int>> rls(count), rts(count);
    std::vector<int> treal(count);
    for (int r = 0; r < count; ++r) {
        Sched sc = cached_schedule(n[r], m[r], precision);
        rls[r] = sc.lam;
        rts[r] = sc.theta;
        int re = 0;
        if (!batch_schedule(n[r], m[r], rls[r], rts[r], &rwl[r], &lnt[r], &tft[r], &re)) {
            rls[r].clear();
            rts[r].clear();
            if (!batch_schedule(n[r], m[r], rls[r], rts[r], &rwl[r], &lnt[r], &tft[r], &re))
                return SP_ERR_UNSUPPORTED_SIZE;
        }
        treal[r] = re;
    }

    sp_batch_s* bp = new (std::nothrow) sp_batch_s();
    if (!bp) return SP_ERR_OOM;
    bp->count = count;
    bp->precision = precision;
    bp->device = dev;
    bp->max_refine = mixed ? R : 0;
    bp->tol = tol;
    bp->n.assign(n, n + count);
    bp->m.assign(m, m + count);

    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) & ~(size_t)255; return o; };
    // tables per distinct n and m
    // tables per distinct (size, radix order)
    std::map<std::string, SizeTables> lam, th;
    std::map<std::string, std::vector<Cx<double>>> lam_tw, lam_pass, th_pass, th_eq, th_ws;
    std::map<std::string, std::vector<double>> th_sin2, th_k0, th_fint;
    std::vector<std::string> lkey(count), tkey(count);
    for (int r = 0; r < count; ++r) {
        lkey[r] = std::to_string(n[r]) + "|" + radix_str(rls[r]);
        tkey[r] = std::to_string(m[r]) + (treal[r] ? "r|" : "c|") + radix_str(rts[r]);
    }
    for (int r = 0; r < count; ++r) {
        const std::string& lk = lkey[r];
        const std::string& tk = tkey[r];
        if (!lam.count(lk)) {
            SizeTables& t = lam[lk];
            t.len = n[r] / 2;
            t.radices = rls[r];
            t.desc = make_desc(t.radices, t.len, &lam_pass[lk]);
            std::vector<Cx<double>>& tw = lam_tw[lk];
            tw.resize(n[r]);
            for (int i = 0; i < n[r]; ++i) cis_neg(i, n[r], &tw[i].x, &tw[i].y);
            t.off64 = take(n[r] * sizeof(Cx<double>));
            t.off32 = take(n[r] * sizeof(Cx<float>));
            t.offp64 = take(lam_pass[lk].size() * sizeof(Cx<double>));
            t.offp32 = take(lam_pass[lk].size() * sizeof(Cx<float>));
        }
        if (!th.count(tk)) {
            SizeTables& t = th[tk];
            t.len = treal[r] ? m[r] / 2 : m[r];
            t.radices = rts[r];
            t.desc = make_desc(t.radices, t.len, &th_pass[tk]);
            host_theta_tables(m[r], th_eq[tk], th_sin2[tk], th_k0[tk], th_fint[tk]);
            std::vector<Cx<double>>& ws = th_ws[tk];
            ws.resize(m[r] / 4 + 1);
            for (int q = 0; q <= m[r] / 4; ++q) cis_neg(q, m[r], &ws[q].x, &ws[q].y);
            t.offws64 = take(ws.size() * sizeof(Cx<double>));
            t.offws32 = take(ws.size() * sizeof(Cx<float>));
            t.offp64 = take(th_pass[tk].size() * sizeof(Cx<double>));
            t.offp32 = take(th_pass[tk].size() * sizeof(Cx<float>));
            t.offeq64 = take(m[r] * sizeof(Cx<double>));
            t.offeq32 = take(m[r] * sizeof(Cx<float>));
            t.offsin2 = take(m[r] * sizeof(double));
            t.offk0 = take(th_k0[tk].size() * sizeof(double));
            t.offfint = take(m[r] * sizeof(double));
        }
    }
    // per-problem workspace
    std::vector<size_t> o64(count), oB(count), o0(count), od(count), opart(count), ofco(count);
    std::vector<int> nblk(count);
    for (int r = 0; r < count; ++r) {
        const int rw = 1 << rwl[r];
        nblk[r] = (m[r] + rw - 1) / rw;
        // spectrum runs of at least 8 rows (a 128-byte line per wavenumber in
        // float64), as in a single plan: the theta tiles' column reads need them
        const int rl = 1 << std::max(rwl[r], kLayLog2);
        const size_t elems = (size_t)((m[r] + rl - 1) / rl) * (n[r] / 2 + 1) * rl;
        o64[r] = take(elems * sizeof(Cx<double>));
        if (mixed) {
            oB[r] = take(elems * sizeof(Cx<double>));
            o0[r] = take(elems * sizeof(Cx<float>));
            od[r] = take(elems * sizeof(Cx<float>));
            opart[r] = take(2 * (size_t)nblk[r] * sizeof(double));
            ofco[r] = take((size_t)(n[r] / 2 + 1) * sp::solve_slot_stride(m[r]) * sizeof(Cx<double>));
        }
    }
    // work lists per kernel build: (rhs, tile) sorted by decreasing tile cost
    std::vector<int2> lam_items[kBatchClasses], th_items[kBatchClasses];
    size_t lam_lds_c[kBatchClasses] = {}, th_lds_c[kBatchClasses] = {};
    for (int r = 0; r < count; ++r) {
        const int lc = radix_class(rls[r]);
        const int tc = radix_class(rts[r]) + (treal[r] == kBatchWaveThreads ? 4 : treal[r] ? 2 : 0);
        for (int jb = 0; jb < nblk[r]; ++jb) lam_items[lc].push_back(make_int2(r, jb));
        for (int k = 0; k <= n[r] / 2; ++k) {
            if (treal[r]) {
                th_items[tc].push_back(make_int2(r, 2 * k));
                th_items[tc].push_back(make_int2(r, 2 * k + 1));
            } else {
                th_items[tc].push_back(make_int2(r, k));
            }
        }
        lam_lds_c[lc] = std::max(lam_lds_c[lc], ((size_t)n[r] / 2 << rwl[r]) * sizeof(Cx<double>));
        const int smaxr = treal[r] == kBatchWaveThreads ? kSmaxR : kBatchSmaxR;
        const size_t tl = treal[r] ? real_theta_lds_bytes(m[r], solve_threads(m[r], smaxr))
                                   : theta_lds_bytes<double>(m[r], std::max(solve_threads(m[r], kSmaxD),
                                                                            solve_threads(m[r], kSmaxF)));
        th_lds_c[tc] = std::max(th_lds_c[tc], tl);
    }
    for (int c = 0; c < kBatchClasses; ++c) {
        std::stable_sort(lam_items[c].begin(), lam_items[c].end(), [&](int2 x, int2 y) {
            return (long long)n[x.x] << rwl[x.x] > (long long)n[y.x] << rwl[y.x];
        });
        std::stable_sort(th_items[c].begin(), th_items[c].end(), [&](int2 x, int2 y) { return m[x.x] > m[y.x]; });
    }
    const size_t o_desc = take(count * sizeof(sp::RhsDesc));
    // per-stage argument arrays, one entry per problem
    const size_t o_lfwd = take(count * sizeof(sp::LambdaArgs<double>));
    const size_t o_linv = mixed ? 0 : take(count * sizeof(sp::LambdaArgs<double>));
    const size_t o_th64 = mixed ? 0 : take(count * sizeof(sp::ThetaArgs<double>));
    const size_t o_thf = mixed ? take(count * sizeof(sp::ThetaMixArgs)) : 0;
    const size_t o_thr = mixed ? take(count * sizeof(sp::ThetaMixArgs)) : 0;
    const size_t o_mix = mixed ? take(count * sizeof(sp::MixLambdaArgs)) : 0;
    // corrections after the first: float64 transform of the iterate, then an accumulating update
    const size_t o_lfwd2 = (mixed && R > 1) ? take(count * sizeof(sp::LambdaArgs<double>)) : 0;
    const size_t o_mix2 = (mixed && R > 1) ? take(count * sizeof(sp::MixLambdaArgs)) : 0;
    size_t o_lam_items[kBatchClasses], o_th_items[kBatchClasses];
    for (int c = 0; c < kBatchClasses; ++c) {
        o_lam_items[c] = take(lam_items[c].size() * sizeof(int2));
        o_th_items[c] = take(th_items[c].size() * sizeof(int2));
    }
    const size_t o_ctr = take(kBatchMaxLaunches * sizeof(int));
    const size_t o_scal = take(kBatchScal * (size_t)count * sizeof(double));
    const size_t o_nblk = take(count * sizeof(int));

    hipError_t e = hipMalloc(&bp->block, off);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete bp;
        return SP_ERR_OOM;
    }
    unsigned char* B = (unsigned char*)bp->block;
    bp->scal = (double*)(B + o_scal);
    std::vector<sp::RhsDesc> descs(count);
    for (int r = 0; r < count; ++r) {
        const SizeTables& L = lam[lkey[r]];
        const SizeTables& T = th[tkey[r]];
        sp::RhsDesc& d = descs[r];
        d.n = n[r]; d.m = m[r]; d.N = n[r] / 2; d.rw_log2 = rwl[r]; d.lay_log2 = std::max(rwl[r], kLayLog2);
        d.lam_nthr = lnt[r]; d.theta_nthr_fft = tft[r]; d.theta_real = treal[r] ? 1 : 0;
        d.k64 = std::max(16, m[r] / 64);
        d.c0 = 0.0;
        d.fl = L.desc; d.ft = T.desc;
        d.f = f[r]; d.u = u[r];
        d.spec64 = (Cx<double>*)(B + o64[r]);
        d.specB = mixed ? (Cx<double>*)(B + oB[r]) : nullptr;
        d.spec0 = mixed ? (Cx<float>*)(B + o0[r]) : nullptr;
        d.specd = mixed ? (Cx<float>*)(B + od[r]) : nullptr;
        d.partial = mixed ? (double*)(B + opart[r]) : nullptr;
        d.fco = mixed ? (Cx<double>*)(B + ofco[r]) : nullptr;
        d.tw64n = (const Cx<double>*)(B + L.off64);
        d.tw32n = (const Cx<float>*)(B + L.off32);
        d.p64n = (const Cx<double>*)(B + L.offp64);
        d.p32n = (const Cx<float>*)(B + L.offp32);
        d.p64m = (const Cx<double>*)(B + T.offp64);
        d.p32m = (const Cx<float>*)(B + T.offp32);
        d.eq64 = (const Cx<double>*)(B + T.offeq64);
        d.eq32 = (const Cx<float>*)(B + T.offeq32);
        d.ws64 = (const Cx<double>*)(B + T.offws64);
        d.ws32 = (const Cx<float>*)(B + T.offws32);
        d.sin2 = (const double*)(B + T.offsin2);
        d.k0tab = (const double*)(B + T.offk0);
        d.fint_w = (const double*)(B + T.offfint);
        d.scal = bp->scal + kBatchScal * r;
    }
    auto to32 = [](const std::vector<Cx<double>>& v) {
        std::vector<Cx<float>> o(v.size());
        for (size_t i = 0; i < v.size(); ++i) o[i] = Cx<float>{(float)v[i].x, (float)v[i].y};
        return o;
    };
    std::vector<std::pair<size_t, std::vector<unsigned char>>> uploads;
    auto stage = [&](size_t o, const void* src, size_t bytes) {
        std::vector<unsigned char> v((const unsigned char*)src, (const unsigned char*)src + bytes);
        uploads.emplace_back(o, std::move(v));
    };
    for (auto& kv : lam) {
        const std::string& nn = kv.first;
        auto t32 = to32(lam_tw[nn]);
        auto p32 = to32(lam_pass[nn]);
        stage(kv.second.off64, lam_tw[nn].data(), lam_tw[nn].size() * sizeof(Cx<double>));
        stage(kv.second.off32, t32.data(), t32.size() * sizeof(Cx<float>));
        stage(kv.second.offp64, lam_pass[nn].data(), lam_pass[nn].size() * sizeof(Cx<double>));
        stage(kv.second.offp32, p32.data(), p32.size() * sizeof(Cx<float>));
    }
    for (auto& kv : th) {
        const std::string& mm = kv.first;
        auto p32 = to32(th_pass[mm]);
        auto e32 = to32(th_eq[mm]);
        stage(kv.second.offp64, th_pass[mm].data(), th_pass[mm].size() * sizeof(Cx<double>));
        stage(kv.second.offp32, p32.data(), p32.size() * sizeof(Cx<float>));
        stage(kv.second.offeq64, th_eq[mm].data(), th_eq[mm].size() * sizeof(Cx<double>));
        stage(kv.second.offeq32, e32.data(), e32.size() * sizeof(Cx<float>));
        stage(kv.second.offsin2, th_sin2[mm].data(), th_sin2[mm].size() * sizeof(double));
        stage(kv.second.offk0, th_k0[mm].data(), th_k0[mm].size() * sizeof(double));
        stage(kv.second.offfint, th_fint[mm].data(), th_fint[mm].size() * sizeof(double));
        auto w32 = to32(th_ws[mm]);
        stage(kv.second.offws64, th_ws[mm].data(), th_ws[mm].size() * sizeof(Cx<double>));
        stage(kv.second.offws32, w32.data(), w32.size() * sizeof(Cx<float>));
    }
    stage(o_desc, descs.data(), descs.size() * sizeof(sp::RhsDesc));
    {
        std::vector<sp::LambdaArgs<double>> lf(count), li(count);
        std::vector<sp::ThetaArgs<double>> t64(count);
        std::vector<sp::ThetaMixArgs> tf(count), tr(count);
        std::vector<sp::MixLambdaArgs> mx(count), mx2(count);
        std::vector<sp::LambdaArgs<double>> lf2(count);
        for (int r = 0; r < count; ++r) {
            lf[r] = sp::batch_lambda_args(descs[r], true);
            li[r] = sp::batch_lambda_args(descs[r], false);
            t64[r] = sp::batch_theta_args(descs[r]);
            tf[r] = sp::batch_theta_mix_args(descs[r], false);
            tr[r] = sp::batch_theta_mix_args(descs[r], true);
            mx[r] = sp::batch_mix_args(descs[r]);
            // later corrections: the float64 spectrum of the current iterate u (no sin^2) into specB,
            // and an update that adds the correction to u
            lf2[r] = lf[r];
            lf2[r].x = descs[r].u;
            lf2[r].rowscale = nullptr;
            lf2[r].spec = descs[r].specB;
            mx2[r] = mx[r];
            mx2[r].accumulate = 1;
        }
        stage(o_lfwd, lf.data(), count * sizeof(lf[0]));
        if (mixed) {
            stage(o_thf, tf.data(), count * sizeof(tf[0]));
            stage(o_thr, tr.data(), count * sizeof(tr[0]));
            stage(o_mix, mx.data(), count * sizeof(mx[0]));
            if (R > 1) {
                stage(o_lfwd2, lf2.data(), count * sizeof(lf2[0]));
                stage(o_mix2, mx2.data(), count * sizeof(mx2[0]));
            }
        } else {
            stage(o_linv, li.data(), count * sizeof(li[0]));
            stage(o_th64, t64.data(), count * sizeof(t64[0]));
        }
    }
    for (int c = 0; c < kBatchClasses; ++c) {
        stage(o_lam_items[c], lam_items[c].data(), lam_items[c].size() * sizeof(int2));
        stage(o_th_items[c], th_items[c].data(), th_items[c].size() * sizeof(int2));
    }
    stage(o_nblk, nblk.data(), nblk.size() * sizeof(int));
    for (auto& up : uploads) {
        e = hipMemcpy(B + up.first, up.second.data(), up.second.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) { delete bp; return hip_fail(e, "batch upload"); }
    }

    // graph: counter reset, the stage kernels (the correction stages R times), per-problem norms
    BatchKernels K = batch_kernels();
    struct Step { int stg; size_t args; int norm_slot; };   // norm_slot >= 0: per-problem norms after it
    std::vector<Step> steps;
    if (mixed) {
        steps = {{sp::kBLamFwd, o_lfwd, -1}, {sp::kBThetaFirst, o_thf, -1}, {sp::kBLamMix, o_mix, -1},
                 {sp::kBThetaResid, o_thr, -1}, {sp::kBLamUpd, o_mix, 1}};
        for (int it = 2; it <= R; ++it) {
            steps.push_back({sp::kBLamFwd, o_lfwd2, -1});
            steps.push_back({sp::kBThetaResid, o_thr, -1});
            steps.push_back({sp::kBLamUpd, o_mix2, 1 + 2 * (it - 1)});
        }
    } else {
        steps = {{sp::kBLamFwd, o_lfwd, -1}, {sp::kBTheta64, o_th64, -1}, {sp::kBLamInv, o_linv, -1}};
    }
    e = hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking);
    if (e != hipSuccess) { delete bp; return hip_fail(e, "hipStreamCreate"); }
    e = hipEventCreateWithFlags(&bp->done, hipEventDisableTiming);
    if (e != hipSuccess) { delete bp; return hip_fail(e, "hipEventCreate"); }
    // each (step, build) with work: its LDS, occupancy, persistent grid and work-list counter
    struct Launch { void (*fn)(const void*, const int2*, int, int*); int grid, nt; size_t lds, items, args; int nit, ctr, norm_slot; };
    std::vector<Launch> launches;
    for (const Step& S : steps) {
        const int stg = S.stg;
        const bool is_theta = stg == sp::kBTheta64 || stg == sp::kBThetaFirst || stg == sp::kBThetaResid;
        for (int c = 0; c < kBatchClasses; ++c) {
            const int nit = (int)(is_theta ? th_items[c].size() : lam_items[c].size());
            if (nit == 0) continue;
            // the update holds float32 correction lines only: half a float64 lambda tile
            const size_t lds = is_theta ? th_lds_c[c] : stg == sp::kBLamUpd ? lam_lds_c[c] / 2 : lam_lds_c[c];
            if (lds + 1024 > lds_limit) { delete bp; return SP_ERR_UNSUPPORTED_SIZE; }
            Launch L;
            L.fn = K.st[stg][c];
            L.nt = c >= 4 ? kBatchWaveThreads : c >= 2 ? kBatchRealThreads : kBatchThreads;
            (void)hipFuncSetAttribute((const void*)L.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            int occ = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)L.fn, L.nt, lds) !=
                    hipSuccess || occ < 1)
                occ = 1;
            L.grid = std::max(1, std::min(nit, prop.multiProcessorCount * occ));
            L.lds = lds;
            L.items = is_theta ? o_th_items[c] : o_lam_items[c];
            L.nit = nit;
            L.ctr = (int)launches.size();
            L.args = S.args;
            L.norm_slot = -1;
            launches.push_back(L);
        }
        if (S.norm_slot >= 0 && !launches.empty()) launches.back().norm_slot = S.norm_slot;
    }
    if ((int)launches.size() > kBatchMaxLaunches) { delete bp; return SP_ERR_UNSUPPORTED_SIZE; }
    (void)hipGetLastError();
    e = hipStreamBeginCapture(bp->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { delete bp; return hip_fail(e, "hipStreamBeginCapture"); }
    int* ctr = (int*)(B + o_ctr);
    const sp::RhsDesc* dd = (const sp::RhsDesc*)(B + o_desc);
    hipLaunchKernelGGL(sp::k_batch_reset, dim3(1), dim3(64), 0, bp->cap, ctr, (int)launches.size());
    for (const Launch& L : launches) {
        hipLaunchKernelGGL(L.fn, dim3(L.grid), dim3(L.nt), L.lds, bp->cap, (const void*)(B + L.args),
                           (const int2*)(B + L.items), L.nit, ctr + L.ctr);
        if (L.norm_slot >= 0)
            hipLaunchKernelGGL(sp::k_batch_norms, dim3(count), dim3(256), 0, bp->cap, dd, (const int*)(B + o_nblk),
                               L.norm_slot);
    }
    e = hipStreamEndCapture(bp->cap, &bp->graph);
    if (e != hipSuccess) { delete bp; return hip_fail(e, "hipStreamEndCapture"); }
    e = hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { delete bp; return hip_fail(e, "hipGraphInstantiate"); }
    *out = bp;
    return SP_OK;
}


}  // namespace

namespace {
// Overlaps across a batch: no u[r] may overlap any other buffer of the batch
// (its own f included); f buffers may overlap each other (they are only
// read).  The u intervals are sorted and checked pairwise in order; each f
// interval is then checked against the first u interval ending after its
// start.  O(count log count), host pointers only.
bool batch_alias(int count, const int* n, const int* m, const double* const* f, double* const* u) {
    struct Iv { uintptr_t lo, hi; };
    std::vector<Iv> us(count);
    for (int r = 0; r < count; ++r) {
        const size_t bytes = (size_t)n[r] * m[r] * sizeof(double);
        us[r] = Iv{(uintptr_t)u[r], (uintptr_t)u[r] + bytes};
    }
    std::sort(us.begin(), us.end(), [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
    for (int r = 1; r < count; ++r)
        if (us[r].lo < us[r - 1].hi) return true;
    // disjoint and sorted by start, so the ends are sorted too
    for (int r = 0; r < count; ++r) {
        const uintptr_t lo = (uintptr_t)f[r], hi = lo + (size_t)n[r] * m[r] * sizeof(double);
        auto it = std::upper_bound(us.begin(), us.end(), lo, [](uintptr_t v, const Iv& x) { return v < x.hi; });
        if (it != us.end() && it->lo < hi) return true;
    }
    return false;
}
}  // namespace

extern "C" int sphere_poisson_batch_plan(sp_batch* out, int count, const int* n, const int* m, const double* const* f,
                                         double* const* u, const sp_desc* desc, void* hip_stream) {
    (void)hip_stream;   // the tables are uploaded synchronously
    if (!out) return SP_ERR_INVALID_ARG;
    *out = nullptr;
    if (count <= 0 || !n || !m || !f || !u || !desc) return SP_ERR_INVALID_ARG;
    const int precision = desc->precision;
    if (precision != SP_FP64 && precision != SP_MIXED) return SP_ERR_INVALID_ARG;
    if (desc->flags & ~(SP_SYNC_INFO | SP_AUTOTUNE | SP_INFO)) return SP_ERR_INVALID_ARG;
    const int R = precision == SP_MIXED ? desc->max_refine : 0;
    if (precision == SP_MIXED && (R < 1 || R > sp::kBatchMaxRefine)) return SP_ERR_INVALID_ARG;
    for (int r = 0; r < count; ++r) {
        if (!f[r] || !u[r] || n[r] < 4 || (n[r] & 1) || m[r] < 4) return SP_ERR_INVALID_ARG;
        if (n[r] > (1 << 20) || m[r] > (1 << 20)) return SP_ERR_UNSUPPORTED_SIZE;
    }
    if (batch_alias(count, n, m, f, u)) return SP_ERR_ALIAS;
    sp_batch_s* bp = nullptr;
    const int st = build_batch(count, n, m, f, u, precision, R, desc->tol, (desc->flags & SP_AUTOTUNE) != 0, &bp);
    if (st != SP_OK) return st;
    {
        std::lock_guard<std::mutex> g(g_batches_mu);
        g_batches.insert(bp);
    }
    *out = bp;
    return SP_OK;
}

extern "C" int sphere_poisson_solve_batch(sp_batch bp, void* hip_stream, sp_info* infos) {
    if (!batch_ok(bp)) return SP_ERR_BAD_PLAN;
    hipStream_t s = (hipStream_t)hip_stream;
    SP_HIP(hipGraphLaunch(bp->exec, s));
    SP_HIP(hipEventRecord(bp->done, s));
    bp->launched = true;
    if (!infos) return SP_OK;
    SP_HIP(hipStreamSynchronize(s));
    const int count = bp->count, R = bp->max_refine;
    std::vector<double> sc(sp::kBatchScal * (size_t)count);
    SP_HIP(hipMemcpy(sc.data(), bp->scal, sc.size() * sizeof(double), hipMemcpyDeviceToHost));
    int status = SP_OK;
    for (int r = 0; r < count; ++r) {
        const double* q = sc.data() + (size_t)sp::kBatchScal * r;
        auto rel_of = [&](int it) { return q[2 * it] > 0.0 ? std::sqrt(q[2 * it - 1] / q[2 * it]) : 0.0; };
        sp_info& in = infos[r];
        in.iters = R;
        in.f_integral = q[0];
        in.rel_residual = 0.0;
        in.rel_correction = R > 0 ? rel_of(R) : 0.0;
        // contraction as for a single solve: the ratio of the last two corrections, or the first's own size
        const double rho = R >= 2 ? (rel_of(R - 1) > 0.0 ? in.rel_correction / rel_of(R - 1) : 0.0) : in.rel_correction;
        in.est_rel_err = R > 0 ? in.rel_correction * rho : 0.0;
        in.status = SP_OK;
        if (R > 0 && bp->tol > 0.0 && !(in.rel_correction <= bp->tol)) {
            in.status = SP_ERR_NOT_CONVERGED;
            status = SP_ERR_NOT_CONVERGED;
        }
    }
    return status;
}

extern "C" int sphere_poisson_batch_destroy(sp_batch bp) {
    {
        std::lock_guard<std::mutex> g(g_batches_mu);
        if (!bp || !g_batches.erase(bp)) return SP_ERR_BAD_PLAN;
    }
    delete bp;   // waits for the last launch
    return SP_OK;
}

extern "C" size_t sphere_poisson_stream_partials(size_t count) {
    return (count + sp::kStreamChunk - 1) / sp::kStreamChunk;
}

extern "C" int sphere_poisson_stream(int kind, const double* x, double* y, size_t count, void* hip_stream) {
    const int op = kind & 0xf;
    const bool nt = (kind & SP_STREAM_NONTEMPORAL) != 0;
    if ((kind & ~(0xf | SP_STREAM_NONTEMPORAL)) || op > SP_STREAM_WRITE) return SP_ERR_INVALID_ARG;
    if (!y || (op != SP_STREAM_WRITE && !x)) return SP_ERR_INVALID_ARG;
    if (((uintptr_t)y & 15) || (x && ((uintptr_t)x & 15))) return SP_ERR_INVALID_ARG;
    if (count == 0) return SP_OK;
    const size_t blocks = sphere_poisson_stream_partials(count);
    if (blocks > 0x7fffffffu) return SP_ERR_UNSUPPORTED_SIZE;
    if (op == SP_STREAM_COPY && overlap(x, y, count * sizeof(double))) return SP_ERR_ALIAS;
    if (op == SP_STREAM_READ && overlap(x, y, count * sizeof(double), blocks * sizeof(double))) return SP_ERR_ALIAS;
    hipStream_t s = (hipStream_t)hip_stream;
    const dim3 grid((unsigned)blocks), block(sp::kStreamThreads);
    if (op == SP_STREAM_COPY) {
        if (nt) hipLaunchKernelGGL(sp::k_stream_copy<true>, grid, block, 0, s, x, y, count);
        else hipLaunchKernelGGL(sp::k_stream_copy<false>, grid, block, 0, s, x, y, count);
    } else if (op == SP_STREAM_READ) {
        if (nt) hipLaunchKernelGGL(sp::k_stream_read<true>, grid, block, 0, s, x, y, count);
        else hipLaunchKernelGGL(sp::k_stream_read<false>, grid, block, 0, s, x, y, count);
    } else {
        if (nt) hipLaunchKernelGGL(sp::k_stream_write<true>, grid, block, 0, s, y, 1.0, count);
        else hipLaunchKernelGGL(sp::k_stream_write<false>, grid, block, 0, s, y, 1.0, count);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "stream kernel launch");
    return SP_OK;
}

extern "C" const char* sphere_poisson_strerror(int code) {
    switch (code) {
        case SP_OK: return "success";
        case SP_ERR_INVALID_ARG: return "invalid argument";
        case SP_ERR_UNSUPPORTED_SIZE: return "unsupported size (prime factor > 31 or too large)";
        case SP_ERR_OOM: return "device out of memory";
        case SP_ERR_HIP: {
            static thread_local std::string msg;
            msg = "HIP error: " + g_hip_err;
            return msg.c_str();
        }
        case SP_ERR_NOT_CONVERGED: return "refinement did not reach the requested tolerance";
        case SP_ERR_ALIAS: return "input and output buffers overlap";
        case SP_ERR_NO_DEVICE: {
            static thread_local std::string msg;
            msg = "no usable gfx950 device" + (g_hip_err.empty() ? std::string() : ": " + g_hip_err);
            return msg.c_str();
        }
        case SP_ERR_BAD_PLAN: return "null or destroyed plan";
        default: return "unknown status";
    }
}
