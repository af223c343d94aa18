// Structure-preserving Gaussian elimination on the sampled grid (Section 3,
// Figure GaussianElimination, eq. GEstructurePreservingStepPseudoinverse):
// each step picks the 2 x 2 BMC pivot with the largest sigma_1 = |a| + |b|
// (a = e(lambda* - pi, theta*), b = e(lambda*, theta*); eq. SingularValues),
// inverts it through its eps-pseudoinverse (eps = alpha sigma_1), and removes
// the resulting rank-2 term from the residual.  The doubled function is never
// formed: its value at (lambda, -theta) is the sample at (lambda + pi, theta).
// The two rank-1 terms of a step are d (C0 +- C1)(R0 +- R1) with d = 1 / (2 (a +- b))
// (0 where |a +- b| <= eps), C0 / C1 the residual's columns at lambda* - pi /
// lambda*, R0 the row at theta* and R1 that row shifted by pi.
// A step is three launches: the pivot (one workgroup), the factor extraction
// (one thread per entry), and the rank-2 update of the residual fused with
// the next step's partial pivot search (HBM-bound: one read and one write of
// the grid); one search pass before the first step; once the loop has
// stopped, the updates return at once.
// This translation unit is separate from the solver's: it owns no plan and
// works in a workspace the caller provides.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>

#include "../../include/sphere_poisson.h"

namespace spge {

constexpr int kGeBlocks = 1024;   // workgroups of the partial pivot search
constexpr int kGeThreads = 256;

struct GeRecord {      // device state carried from step to step
    double s_first;    // sigma_1 of the first pivot
    int active;        // 0 once the loop has stopped
    int t, i;          // this step's pivot (row, column with lambda_i in [0, pi))
};

// candidate (score, flat index t * (n/2) + i - n/2): larger score wins, ties go
// to the smaller index (the first maximum in row-major order)
__device__ __forceinline__ void ge_better(double s, long long idx, double& best, long long& bidx) {
    if (s > best || (s == best && idx < bidx)) {
        best = s;
        bidx = idx;
    }
}

__device__ __forceinline__ void ge_block_argmax(double& best, long long& bidx) {
    __shared__ double sb[kGeThreads];
    __shared__ long long si[kGeThreads];
    sb[threadIdx.x] = best;
    si[threadIdx.x] = bidx;
    __syncthreads();
    for (int w = kGeThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double b = sb[threadIdx.x];
            long long i = si[threadIdx.x];
            ge_better(sb[threadIdx.x + w], si[threadIdx.x + w], b, i);
            sb[threadIdx.x] = b;
            si[threadIdx.x] = i;
        }
        __syncthreads();
    }
    best = sb[0];
    bidx = si[0];
}

// 1. workgroup g scans rows g, g + G, ...: partial (score, index) per workgroup
// (after the loop has stopped, every workgroup returns at once: no candidate)
__global__ void __launch_bounds__(kGeThreads) k_ge_scores(const double* __restrict__ e, int m, int n,
                                                         const GeRecord* __restrict__ rec, int k,
                                                         double* __restrict__ pscore, long long* __restrict__ pidx) {
    const int H = n / 2;
    double best = -1.0;
    long long bidx = 0x7fffffffffffffffLL;
    if (k > 0 && rec->active == 0) {
        if (threadIdx.x == 0) {
            pscore[blockIdx.x] = best;
            pidx[blockIdx.x] = bidx;
        }
        return;
    }
    for (int t = blockIdx.x; t < m; t += gridDim.x) {
        const double* row = e + (size_t)t * n;
        for (int ih = threadIdx.x; ih < H; ih += blockDim.x)
            ge_better(fabs(row[ih]) + fabs(row[ih + H]), (long long)t * H + ih, best, bidx);
    }
    ge_block_argmax(best, bidx);
    if (threadIdx.x == 0) {
        pscore[blockIdx.x] = best;
        pidx[blockIdx.x] = bidx;
    }
}

// 2. one workgroup: the pivot and its pseudoinverse (d of step k)
__global__ void __launch_bounds__(kGeThreads) k_ge_pivot(const double* __restrict__ e, int m, int n,
                                                        const double* __restrict__ pscore,
                                                        const long long* __restrict__ pidx, int nparts, int k,
                                                        double alpha, double tol, GeRecord* __restrict__ rec,
                                                        double* __restrict__ d, int* __restrict__ piv) {
    const int H = n / 2;
    double best = -1.0;
    long long bidx = 0x7fffffffffffffffLL;
    for (int g = threadIdx.x; g < nparts; g += blockDim.x) ge_better(pscore[g], pidx[g], best, bidx);
    ge_block_argmax(best, bidx);
    if (threadIdx.x == 0) {
        // no candidate at all (a residual of NaNs): stop, reading a valid point
        const bool found = bidx != 0x7fffffffffffffffLL;
        const int t = found ? (int)(bidx / H) : 0, i = found ? (int)(bidx % H) + H : H;
        const double a = e[(size_t)t * n + i - H], b = e[(size_t)t * n + i];
        const double s1 = found ? fabs(a) + fabs(b) : 0.0;
        if (k == 0) {
            rec->s_first = s1;
            rec->active = 1;
        }
        const int act = rec->active && s1 > 0.0 && !(s1 <= tol * rec->s_first);
        rec->active = act;
        rec->t = t;
        rec->i = i;
        const double eps = alpha * s1;
        const double gp = act && fabs(a + b) > eps ? 1.0 / (a + b) : 0.0;
        const double gm = act && fabs(a - b) > eps ? 1.0 / (a - b) : 0.0;
        if (piv) {
            piv[2 * k] = act ? t : -1;
            piv[2 * k + 1] = act ? i : -1;
        }
        d[2 * k] = 0.5 * gp;
        d[2 * k + 1] = 0.5 * gm;
    }
}

// 3. the factors of step k, one thread per entry: c+- = C0 +- C1 (the columns
// at lambda* - pi and lambda*), r+- = R0 +- R1 (the row at theta* and that row
// shifted by pi); zeros once the loop has stopped
__global__ void __launch_bounds__(kGeThreads) k_ge_extract(const double* __restrict__ e, int m, int n, int k,
                                                          const GeRecord* __restrict__ rec, double* __restrict__ c,
                                                          double* __restrict__ r) {
    const int H = n / 2;
    const int act = rec->active, t = rec->t, i = rec->i;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) {
        const double c0 = act ? e[(size_t)q * n + i - H] : 0.0, c1 = act ? e[(size_t)q * n + i] : 0.0;
        c[(size_t)(2 * k) * m + q] = c0 + c1;
        c[(size_t)(2 * k + 1) * m + q] = c0 - c1;
    } else if (q < m + n) {
        const int l = q - m;
        const int ls = l + H < n ? l + H : l - H;
        const double* row = e + (size_t)t * n;
        const double r0 = act ? row[l] : 0.0, r1 = act ? row[ls] : 0.0;
        r[(size_t)(2 * k) * n + l] = r0 + r1;
        r[(size_t)(2 * k + 1) * n + l] = r0 - r1;
    }
}

// 4. e -= d+ c+ r+^T + d- c- r-^T over the grid, fused with the next step's
// pivot search: each thread updates the pair of samples (lambda_i - pi,
// lambda_i) of a row and scores the updated pair, so a step reads and writes
// the grid once.  Rows go to workgroups as in k_ge_scores.
__global__ void __launch_bounds__(kGeThreads) k_ge_update(double* __restrict__ e, int m, int n,
                                                         const double* __restrict__ d, const double* __restrict__ c,
                                                         const double* __restrict__ r, int k,
                                                         const GeRecord* __restrict__ rec, double* __restrict__ pscore,
                                                         long long* __restrict__ pidx) {
    const int H = n / 2;
    double best = -1.0;
    long long bidx = 0x7fffffffffffffffLL;
    if (rec->active == 0) {   // uniform: the loop has stopped, no candidate
        if (threadIdx.x == 0) {
            pscore[blockIdx.x] = best;
            pidx[blockIdx.x] = bidx;
        }
        return;
    }
    const double dp = d[2 * k], dm = d[2 * k + 1];
    const double* cp = c + (size_t)(2 * k) * m;
    const double* cm = cp + m;
    const double* rp = r + (size_t)(2 * k) * n;
    const double* rm = rp + n;
    for (int t = blockIdx.x; t < m; t += gridDim.x) {
        double* row = e + (size_t)t * n;
        const double ap = dp * cp[t], am = dm * cm[t];
        for (int ih = threadIdx.x; ih < H; ih += blockDim.x) {
            double e0 = row[ih], e1 = row[ih + H];
            e0 -= ap * rp[ih] + am * rm[ih];
            e1 -= ap * rp[ih + H] + am * rm[ih + H];
            row[ih] = e0;
            row[ih + H] = e1;
            ge_better(fabs(e0) + fabs(e1), (long long)t * H + ih, best, bidx);
        }
    }
    ge_block_argmax(best, bidx);
    if (threadIdx.x == 0) {
        pscore[blockIdx.x] = best;
        pidx[blockIdx.x] = bidx;
    }
}

}  // namespace spge

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

struct GeLayout {
    size_t off_e, off_score, off_idx, off_rec, total;
};

GeLayout ge_layout(int n, int m) {
    GeLayout L{};
    L.off_e = 0;
    L.off_score = up((size_t)n * m * sizeof(double));
    L.off_idx = L.off_score + up(spge::kGeBlocks * sizeof(double));
    L.off_rec = L.off_idx + up(spge::kGeBlocks * sizeof(long long));
    L.total = L.off_rec + up(sizeof(spge::GeRecord));
    return L;
}

bool ge_sizes_ok(int n, int m) { return n >= 4 && !(n & 1) && m >= 1 && n <= (1 << 20) && m <= (1 << 20); }

bool disjoint(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return !(x < y + nb && y < x + na);
}

}  // namespace

extern "C" size_t sphere_poisson_ge_workspace_bytes(int n_lambda, int m_theta) {
    if (!ge_sizes_ok(n_lambda, m_theta)) return 0;
    return ge_layout(n_lambda, m_theta).total;
}

namespace {

// Validation common to both entry points: sizes, parameters, outputs (and,
// when given, the caller's workspace) before any device call.
int ge_check(int n, int m, const double* f, int steps, double alpha, double tol, const void* work, size_t work_bytes,
             const double* d, const double* c, const double* r, const int* pivots) {
    if (!ge_sizes_ok(n, m) || steps < 1 || !(alpha >= 0.0 && alpha <= 1.0) || !(tol >= 0.0)) return SP_ERR_INVALID_ARG;
    if (!f || !d || !c || !r) return SP_ERR_INVALID_ARG;
    if ((uintptr_t)r & 15) return SP_ERR_INVALID_ARG;   // double2 access to the rows
    const GeLayout L = ge_layout(n, m);
    if (work) {
        if (work_bytes < L.total) return SP_ERR_INVALID_ARG;
        if ((uintptr_t)work & 15) return SP_ERR_INVALID_ARG;   // double2 access to the grid
    }
    const size_t fb = (size_t)n * m * sizeof(double);
    const size_t db = 2 * (size_t)steps * sizeof(double), cb = db * m, rb = db * n, pb = 2 * (size_t)steps * sizeof(int);
    const void* outs[4] = {d, c, r, pivots};
    const size_t ob[4] = {db, cb, rb, pivots ? pb : 0};
    for (int a = 0; a < 4; ++a) {
        if (!outs[a]) continue;
        if (!disjoint(outs[a], ob[a], f, fb)) return SP_ERR_ALIAS;
        if (work && !disjoint(outs[a], ob[a], work, L.total)) return SP_ERR_ALIAS;
        for (int b = a + 1; b < 4; ++b)
            if (outs[b] && !disjoint(outs[a], ob[a], outs[b], ob[b])) return SP_ERR_ALIAS;
    }
    if (work && !disjoint(f, fb, work, L.total)) return SP_ERR_ALIAS;
    return SP_OK;
}

// The elimination in a workspace of ge_layout(n, m).total bytes (every part of
// it is written before it is read: the residual by the copy of f, the partials
// by the first search, the record by the first pivot).
int ge_run(int n, int m, const double* f, int steps, double alpha, double tol, void* work, double* d, double* c,
           double* r, int* pivots, hipStream_t s) {
    const GeLayout L = ge_layout(n, m);
    const size_t fb = (size_t)n * m * sizeof(double);
    unsigned char* w = static_cast<unsigned char*>(work);
    double* e = reinterpret_cast<double*>(w + L.off_e);
    double* ps = reinterpret_cast<double*>(w + L.off_score);
    long long* pi = reinterpret_cast<long long*>(w + L.off_idx);
    spge::GeRecord* rec = reinterpret_cast<spge::GeRecord*>(w + L.off_rec);
    if (hipMemcpyAsync(e, f, fb, hipMemcpyDeviceToDevice, s) != hipSuccess) return SP_ERR_HIP;
    // the first search reads the grid; afterwards each update pass scores the next step's candidates
    hipLaunchKernelGGL(spge::k_ge_scores, dim3(spge::kGeBlocks), dim3(spge::kGeThreads), 0, s, (const double*)e, m, n,
                       (const spge::GeRecord*)rec, 0, ps, pi);
    for (int k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(spge::k_ge_pivot, dim3(1), dim3(spge::kGeThreads), 0, s, (const double*)e, m, n,
                           (const double*)ps, (const long long*)pi, spge::kGeBlocks, k, alpha, tol, rec, d, pivots);
        hipLaunchKernelGGL(spge::k_ge_extract, dim3((m + n + spge::kGeThreads - 1) / spge::kGeThreads),
                           dim3(spge::kGeThreads), 0, s, (const double*)e, m, n, k, (const spge::GeRecord*)rec, c, r);
        hipLaunchKernelGGL(spge::k_ge_update, dim3(spge::kGeBlocks), dim3(spge::kGeThreads), 0, s, e, m, n,
                           (const double*)d, (const double*)c, (const double*)r, k, (const spge::GeRecord*)rec, ps, pi);
    }
    if (hipGetLastError() != hipSuccess) return SP_ERR_HIP;
    return SP_OK;
}

// The workspace of sphere_poisson_ge_lowrank_static: a file-scope device
// array, one copy on every device the library runs on, held until the
// process ends.  Host code never passes the array's name to a kernel (that is
// a host-side stand-in): it takes the array's device address once per device,
// with that device current, and uses that address.
constexpr size_t kGeStaticBytes = SP_GE_STATIC_BYTES;
__device__ __align__(256) unsigned char scratch[kGeStaticBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of its scratch

int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return SP_ERR_NO_DEVICE;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return SP_OK;
    }
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return SP_ERR_HIP;
    }
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return SP_OK;
}

}  // namespace

extern "C" int sphere_poisson_ge_lowrank(int n_lambda, int m_theta, const double* f, int steps, double alpha,
                                         double tol, void* work, size_t work_bytes, double* d, double* c, double* r,
                                         int* pivots, void* hip_stream) {
    if (!work) return SP_ERR_INVALID_ARG;
    const int st = ge_check(n_lambda, m_theta, f, steps, alpha, tol, work, work_bytes, d, c, r, pivots);
    if (st != SP_OK) return st;
    return ge_run(n_lambda, m_theta, f, steps, alpha, tol, work, d, c, r, pivots, (hipStream_t)hip_stream);
}

extern "C" int sphere_poisson_ge_lowrank_static(int n_lambda, int m_theta, const double* f, int steps, double alpha,
                                                double tol, double* d, double* c, double* r, int* pivots,
                                                void* hip_stream) {
    const int st = ge_check(n_lambda, m_theta, f, steps, alpha, tol, nullptr, 0, d, c, r, pivots);
    if (st != SP_OK) return st;
    if (ge_layout(n_lambda, m_theta).total > kGeStaticBytes) return SP_ERR_UNSUPPORTED_SIZE;
    void* work = nullptr;
    const int sa = scratch_address(&work);
    if (sa != SP_OK) return sa;
    return ge_run(n_lambda, m_theta, f, steps, alpha, tol, work, d, c, r, pivots, (hipStream_t)hip_stream);
}
