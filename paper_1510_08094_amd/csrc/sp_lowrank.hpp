// Right-hand side of the Poisson solve from a low-rank form (Section 3,
// eq. lowrankRepresentation; Section 4, Computation of Fourier coefficients):
// for f(lambda, theta_j) = sum_q d_q c_q(theta_j) r_q(lambda) the half
// spectrum in lambda of row j of sin^2(theta) f is
//   X_k(theta_j) = sin^2(theta_j) sum_q c_q(theta_j) (d_q rhat_q(k)),
// with rhat_q the half spectrum of r_q (the lambda pass run on the K rows of
// r, row scale d, the solve's 1/n weights).  This kernel forms that rank-K
// product and writes it in the j-blocked layout the theta pass reads, in
// place of the lambda transform of the full grid: it reads K (m + n) values
// instead of m n, and its cost is one write of the spectrum (HBM-bound for
// K up to a few tens, then bound by the float64 FMA rate).
//
// Thread (j group, k): RJ consecutive rows of one wavenumber.  The rhat
// loads are coalesced over k; the c loads are uniform over the workgroup
// (scalar loads); the accumulation order over q is fixed; the results leave
// through LDS in the order of the run layout.
#pragma once
#include "sp_kernels.hpp"

namespace sp {

constexpr int kLowRankRows = 16;      // rows per thread
constexpr int kLowRankThreads = 256;  // wavenumbers per workgroup

template <int RJ>
__global__ void __launch_bounds__(kLowRankThreads)
    k_lowrank_rhs(const double* __restrict__ c, const double* __restrict__ sin2,
                  const Cx<double>* __restrict__ rhat, Cx<double>* __restrict__ spec, int K, int m, int N,
                  int lay) {
    static_assert(RJ % 8 == 0, "rows per thread: whole groups of eight");
    __shared__ Cx<double> tile[kLowRankThreads * 8];
    const int j0 = blockIdx.x * RJ;
    const int k0 = blockIdx.y * kLowRankThreads;
    // threads past the last wavenumber recompute k = N; their values are not stored
    const int k = min(k0 + (int)threadIdx.x, N);
    const int rows = min(RJ, m - j0);
    Cx<double> acc[RJ];
#pragma unroll
    for (int r = 0; r < RJ; ++r) acc[r] = Cx<double>{0.0, 0.0};
    const Cx<double>* h = rhat + k;
    const double* cj = c + j0;
    if (rows == RJ) {
        // four rhat loads in flight before the first use
        constexpr int U = 4;
        int q = 0;
        for (; q + U <= K; q += U) {
            Cx<double> v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = h[(size_t)(q + u) * (N + 1)];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double* cq = cj + (size_t)(q + u) * m;
#pragma unroll
                for (int r = 0; r < RJ; ++r) {
                    acc[r].x = fma(cq[r], v[u].x, acc[r].x);
                    acc[r].y = fma(cq[r], v[u].y, acc[r].y);
                }
            }
        }
        for (; q < K; ++q) {
            const Cx<double> v = h[(size_t)q * (N + 1)];
            const double* cq = cj + (size_t)q * m;
#pragma unroll
            for (int r = 0; r < RJ; ++r) {
                acc[r].x = fma(cq[r], v.x, acc[r].x);
                acc[r].y = fma(cq[r], v.y, acc[r].y);
            }
        }
    } else {
        for (int q = 0; q < K; ++q) {
            const Cx<double> v = h[(size_t)q * (N + 1)];
            const double* cq = cj + (size_t)q * m;
#pragma unroll
            for (int r = 0; r < RJ; ++r) {
                if (r < rows) {
                    acc[r].x = fma(cq[r], v.x, acc[r].x);
                    acc[r].y = fma(cq[r], v.y, acc[r].y);
                }
            }
        }
    }
    // Stores: eight rows at a time through LDS, so that consecutive lanes
    // write consecutive (k, row) entries of the run layout (whole lines)
    // instead of one 16-byte entry per line and lane.
    const int nk = min(kLowRankThreads, N + 1 - k0);
#pragma unroll
    for (int g = 0; g < RJ / 8; ++g) {
        if (g) __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const double s = sin2[min(j0 + g * 8 + r, m - 1)];
            tile[threadIdx.x * 8 + r] = Cx<double>{acc[g * 8 + r].x * s, acc[g * 8 + r].y * s};
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nk * 8; e += kLowRankThreads) {
            const int j = j0 + g * 8 + (e & 7);
            if (j < m) spec[spec_at(j, k0 + (e >> 3), N, lay)] = tile[e];
        }
    }
}

// ------------------------------------------------------------ evaluation
// Pointwise evaluation of a low-rank function (Section 4, Pointwise
// evaluation): at a point p, projected radially to the sphere,
//   f(p) = sum_q d_q (c_q^e(theta) r_q^+(lambda) + c_q^o(theta) r_q^-(lambda)),
// the factors' trigonometric interpolants with the even/odd structure of the
// DFS split (eq. lowrankRepresentationSplit): c^e the cosine interpolant of the
// theta samples, c^o the sine interpolant, r^+- the even / odd wavenumbers of
// the real Fourier interpolant of the lambda samples.  Each series is summed
// by Horner's rule in e^{i theta} or e^{2 i (lambda + pi)}: O(K (m + n)) per
// point, bound by the float64 FMA rate.

// alpha[q][.] and beta[q][.] of factor q (one thread per coefficient index s):
//   alpha_s = (2/m) sum_t c_q(theta_t) cos(s theta_t)      (halved for s = 0),
//   beta_s  = (2/m) sum_t c_q(theta_t) sin((s+1) theta_t)  (halved for s = m-1),
// the inverses of the cosine and sine sums on the half-shifted nodes
// theta_t = (t + 1/2) pi / m; angles reduced exactly as s (2t + 1) mod 4m.
__global__ void __launch_bounds__(256) k_trig_coeffs(const double* __restrict__ c, int m,
                                                     double* __restrict__ alpha, double* __restrict__ beta) {
    const int q = blockIdx.x;
    const int s = blockIdx.y * 256 + threadIdx.x;
    if (s >= m) return;
    const double* cq = c + (size_t)q * m;
    const long long m4 = 4LL * m;
    const double inv2m = 1.0 / (2.0 * m);
    double a = 0.0, b = 0.0;
    for (int t = 0; t < m; ++t) {
        const double v = cq[t];
        const long long odd = 2LL * t + 1;
        const double ac = (double)(((long long)s * odd) % m4) * inv2m;
        const double as = (double)(((long long)(s + 1) * odd) % m4) * inv2m;
        a = fma(v, cospi(ac), a);
        b = fma(v, sinpi(as), b);
    }
    const double w = 2.0 / m;
    alpha[(size_t)q * m + s] = a * (s == 0 ? 0.5 * w : w);
    beta[(size_t)q * m + s] = b * (s == m - 1 ? 0.5 * w : w);
}

// One Horner step p <- p w + a with the coefficient folded into the FMA chain
// (four FMA-type instructions for a complex coefficient, four for a real one).
__device__ __forceinline__ Cx<double> horner_c(Cx<double> p, Cx<double> w, Cx<double> a) {
    return Cx<double>{fma(p.x, w.x, fma(-p.y, w.y, a.x)), fma(p.x, w.y, fma(p.y, w.x, a.y))};
}
__device__ __forceinline__ Cx<double> horner_r(Cx<double> p, Cx<double> w, double a) {
    return Cx<double>{fma(p.x, w.x, fma(-p.y, w.y, a)), fma(p.x, w.y, p.y * w.x)};
}

// Two points per thread (kEvalPoints): the coefficient loads are uniform over
// the workgroup and shared by both points, and the two points' chains are
// independent.  h: the lambda coefficients of the factors, already multiplied
// by d_q and by the real-series weights (1 at k = 0 and k = n/2, 2 between),
// contiguous rows of N + 1 values.
constexpr int kEvalPoints = 2;

__global__ void __launch_bounds__(256) k_eval_lowrank(const double* __restrict__ alpha,
                                                      const double* __restrict__ beta,
                                                      const Cx<double>* __restrict__ h, int K, int m, int N,
                                                      const double* __restrict__ xyz, int npts,
                                                      double* __restrict__ out) {
    const int p0 = (blockIdx.x * 256 + threadIdx.x) * kEvalPoints;
    if (p0 >= npts) return;   // no barrier below
    Cx<double> zt[kEvalPoints], v[kEvalPoints], u[kEvalPoints];
    double acc[kEvalPoints];
#pragma unroll
    for (int e = 0; e < kEvalPoints; ++e) {
        const int p = min(p0 + e, npts - 1);   // the last thread may repeat its point
        const double x = xyz[3 * (size_t)p], y = xyz[3 * (size_t)p + 1], z = xyz[3 * (size_t)p + 2];
        const double rho = sqrt(x * x + y * y + z * z);
        // e^{i theta} = (z, sqrt(x^2 + y^2)) / rho; e^{i (lambda + pi)} = -e^{i lambda}, lambda = atan2(y, x)
        zt[e] = Cx<double>{fmin(fmax(z / rho, -1.0), 1.0), sqrt(x * x + y * y) / rho};
        double sl, cl;
        sincos(atan2(y, x), &sl, &cl);
        v[e] = Cx<double>{-cl, -sl};
        u[e] = cmul(v[e], v[e]);
        acc[e] = 0.0;
    }
    for (int q = 0; q < K; ++q) {
        const double* aq = alpha + (size_t)q * m;
        const double* bq = beta + (size_t)q * m;
        Cx<double> pe[kEvalPoints], po[kEvalPoints];
#pragma unroll
        for (int e = 0; e < kEvalPoints; ++e) pe[e] = po[e] = Cx<double>{0.0, 0.0};
        int s = m - 1;
        for (; s >= 3; s -= 4) {   // four coefficients per scalar-load batch
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double a = aq[s - j], b = bq[s - j];
#pragma unroll
                for (int e = 0; e < kEvalPoints; ++e) {
                    pe[e] = horner_r(pe[e], zt[e], a);
                    po[e] = horner_r(po[e], zt[e], b);
                }
            }
        }
        for (; s >= 0; --s) {
            const double a = aq[s], b = bq[s];
#pragma unroll
            for (int e = 0; e < kEvalPoints; ++e) {
                pe[e] = horner_r(pe[e], zt[e], a);
                po[e] = horner_r(po[e], zt[e], b);
            }
        }
        // even terms h_{2j} and odd terms h_{2j+1} as polynomials in u; for even N
        // the top even term h_N has no odd partner and starts the even sum
        const Cx<double>* hq = h + (size_t)q * (N + 1);
        Cx<double> pp[kEvalPoints], pm[kEvalPoints];
        int k2 = N / 2;
        const Cx<double> top = (N & 1) ? Cx<double>{0.0, 0.0} : hq[N];
#pragma unroll
        for (int e = 0; e < kEvalPoints; ++e) {
            pp[e] = top;
            pm[e] = Cx<double>{0.0, 0.0};
        }
        if (!(N & 1)) --k2;
        for (; k2 >= 0; --k2) {
            const Cx<double> he = hq[2 * k2], ho = hq[2 * k2 + 1];
#pragma unroll
            for (int e = 0; e < kEvalPoints; ++e) {
                pp[e] = horner_c(pp[e], u[e], he);
                pm[e] = horner_c(pm[e], u[e], ho);
            }
        }
#pragma unroll
        for (int e = 0; e < kEvalPoints; ++e) {
            const double ce = pe[e].x;                    // sum alpha_s cos(s theta)
            const double co = cmul(po[e], zt[e]).y;       // sum beta_s sin((s + 1) theta)
            const double rp = pp[e].x;                    // even wavenumbers
            const double rm = cmul(pm[e], v[e]).x;        // odd wavenumbers
            acc[e] += ce * rp + co * rm;
        }
    }
#pragma unroll
    for (int e = 0; e < kEvalPoints; ++e)
        if (p0 + e < npts) out[p0 + e] = acc[e];
}

}  // namespace sp
