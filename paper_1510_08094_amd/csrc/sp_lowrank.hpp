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

}  // namespace sp
