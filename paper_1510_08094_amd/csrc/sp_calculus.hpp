// Tangential derivatives on the sphere (Section 4, "Differentiation"): the
// Cartesian components of the surface gradient,
//   d^t/dx = -(sin lambda / sin theta) d/dlambda + cos lambda cos theta d/dtheta,
//   d^t/dy =  (cos lambda / sin theta) d/dlambda + sin lambda cos theta d/dtheta,
//   d^t/dz = -sin theta d/dtheta
// (the z component's sign is the chain rule's, z = cos theta).  As in the
// paper, the division by sin(theta) is done on coefficients (eq. Msin): the
// theta pass in divide mode turns each wavenumber's series into that of the
// series divided by sin(theta), and the theta pass in derivative mode writes
// the theta derivative.  This pass runs both inverse lambda transforms of a
// row (the first with the factor i k of d/dlambda) and combines them with the
// node values of sin/cos lambda and cos/sin theta.  Dividing on the grid
// instead (the nodes never include a pole) amplifies rounding near the poles
// by up to 1/sin(theta_0) ~ 2m/pi.
#pragma once
#include "sp_kernels.hpp"

namespace sp {

// What the pass writes from the gradient g of one scalar field f (p = (x, y, z)
// the point of the unit sphere, n = p its normal; Section 4, Vector calculus):
//   out_a (+)= sum_b wg[a][b] g_b + wn[a][b] (n x g)_b,   a < nout.
// The host fills the weights: the gradient (wg = I), the curl of a scalar
// (eq. CurlScalarF, wn = I), and the terms that component c of a vector field
// adds to its divergence (wg[0][c] = 1), surface curl (wg[a][b] = eps_abc) and
// vorticity (wn[0][c] = 1).

struct GradArgs {
    const Cx<double>* spec_q;   // half spectrum of f / sin(theta) (theta pass, divide mode)
    const Cx<double>* spec_t;   // half spectrum of d f / d theta (theta pass, derivative mode)
    double* gx;                 // outputs [m][n] (out_0, out_1, out_2; unused ones may be null)
    double* gy;
    double* gz;
    double wg[3][3];            // output weights on g
    double wn[3][3];            // output weights on n x g
    int nout;                   // outputs written (1 or 3)
    int accumulate;             // 1: add to the outputs instead of writing them
    const Cx<double>* tw;       // e^{-2 pi i t/n}
    const Cx<double>* ptw;      // per-pass twiddles of the length-N DFT
    const double* rowtab;       // per row j: cos(theta_j), sin(theta_j)  ([2][m])
    const double* coltab;       // per column i: sin(lambda_i), cos(lambda_i)             ([2][n])
    int n, m, N, rw_log2;
    int lay_log2;               // run length (log2) of both spectra read
    FftDesc fft;
    int nthr;                   // threads per row
};

// LDS per row: two lines of N float64 complex ((d/dlambda) / sin(theta), then d/dtheta).
template <int EPT, int RMAX>
__device__ __forceinline__ void lambda_grad_body(const GradArgs& a, int jb, unsigned char* smem_raw) {
    Cx<double>* lines = reinterpret_cast<Cx<double>*>(smem_raw);
    const int N = a.N;
    const int line = threadIdx.x / a.nthr;
    const int t = threadIdx.x - line * a.nthr;
    const int j = (jb << a.rw_log2) + line;
    const bool active = line < (1 << a.rw_log2) && j < a.m;
    const size_t stride = 2 * (size_t)N;
    // length-5000 transform (one row per workgroup): one float64 line, the
    // two inverse transforms in turn, each leaving its last pass in registers
    // (the points t + 500 e the output loop takes), so that two workgroups
    // share a compute unit
    constexpr bool REGS = RMAX == kRadixFixed5000;
    Cx<double> v1[REGS ? 10 : 1], v2[REGS ? 10 : 1];
    if constexpr (REGS) {
        c2r_load_prepare<double, double, true>(lines, N, a.spec_q, a.tw, N, 0, a.lay_log2, a.m, jb, 1.0, 1.0);
        __syncthreads();
        fft5000_regs<double, true, false, true>(lines, a.ptw, t, active, v1);
        __syncthreads();   // every thread has read the line's last pass
        c2r_load_prepare<double, double>(lines, N, a.spec_t, a.tw, N, 0, a.lay_log2, a.m, jb, 1.0, 1.0);
        __syncthreads();
        fft5000_regs<double, true, false, true>(lines, a.ptw, t, active, v2);
    } else {
        c2r_load_prepare<double, double, true>(lines, stride, a.spec_q, a.tw, N, a.rw_log2, a.lay_log2, a.m, jb,
                                               1.0, 1.0);
        c2r_load_prepare<double, double>(lines + N, stride, a.spec_t, a.tw, N, a.rw_log2, a.lay_log2, a.m, jb, 1.0,
                                         1.0);
        __syncthreads();
        fft_lds<double, true, EPT, RMAX>(lines, line * 2 * N, a.fft, a.ptw, t, a.nthr, active);
        fft_lds<double, true, EPT, RMAX>(lines, line * 2 * N + N, a.fft, a.ptw, t, a.nthr, active);
    }
    if (active) {
        const Cx<double>* fl = lines + (size_t)line * stride;   // samples 2i, 2i+1 of (d f/d lambda) / sin(theta)
        const Cx<double>* ft = fl + N;                            // and of d f/d theta
        const double cst = a.rowtab[j], snt = a.rowtab[a.m + j];
        const double2* sl = reinterpret_cast<const double2*>(a.coltab);
        const double2* cl = reinterpret_cast<const double2*>(a.coltab + a.n);
        double2* ox = reinterpret_cast<double2*>(a.gx + (size_t)j * a.n);
        double2* oy = a.gy ? reinterpret_cast<double2*>(a.gy + (size_t)j * a.n) : nullptr;
        double2* oz = a.gz ? reinterpret_cast<double2*>(a.gz + (size_t)j * a.n) : nullptr;
        const bool acc = a.accumulate != 0;
        const int nout = a.nout;
        // (REGS: exactly ten points per thread, i = t + 500 e, a loop of fixed count)
        constexpr int EMAX = REGS ? 10 : 1 << 30;
        constexpr int kUnroll = REGS ? 10 : 1;
#pragma unroll kUnroll
        for (int e = 0; e < EMAX; ++e) {
            const int i = t + e * a.nthr;
            if (!REGS && i >= N) break;
            Cx<double> dl, dt;
            if constexpr (REGS) {
                dl = v1[e];
                dt = v2[e];
            } else {
                dl = fl[i];
                dt = ft[i];
            }
            const double2 s = sl[i], c = cl[i];
            double r[3][2];   // the three outputs at samples 2i, 2i+1
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double sl_ = h ? s.y : s.x, cl_ = h ? c.y : c.x;
                const double A = h ? dl.y : dl.x, Bt = h ? dt.y : dt.x;
                const double g[3] = {-sl_ * A + cl_ * cst * Bt,    // d^t/dx
                                     cl_ * A + sl_ * cst * Bt,     // d^t/dy
                                     -snt * Bt};                   // d^t/dz
                const double px = cl_ * snt, py = sl_ * snt, pz = cst;   // the point (and normal)
                const double nx[3] = {py * g[2] - pz * g[1], pz * g[0] - px * g[2], px * g[1] - py * g[0]};
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    double v = 0.0;
#pragma unroll
                    for (int b = 0; b < 3; ++b) v += a.wg[o][b] * g[b] + a.wn[o][b] * nx[b];
                    r[o][h] = v;
                }
            }
            double2* outs[3] = {ox, oy, oz};
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                if (o < nout) {
                    double2 v = double2{r[o][0], r[o][1]};
                    if (acc) { const double2 w = outs[o][i]; v.x += w.x; v.y += w.y; }
                    outs[o][i] = v;
                }
            }
        }
    }
}

// The length-5000 build runs one row per workgroup in 512 threads and one
// float64 line: its bound (128 registers) lets two workgroups share a
// compute unit.
template <int EPT, int RMAX>
__global__ void __launch_bounds__(RMAX == kRadixFixed5000 ? 512 : 1024, RMAX == kRadixFixed5000 ? 4 : 1)
    k_lambda_grad(GradArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int jb = lambda_tile(a.lay_log2 - a.rw_log2);
    if (jb << a.rw_log2 >= a.m) return;
    lambda_grad_body<EPT, RMAX>(a, jb, smem_raw);
}

// ---------------------------------------------------------------- integration
// Integral of f over the sphere (Section 4, "Integration", the sum2
// command): the lambda integral of row j is 2 pi times its mean, and the
// theta integral against sin(theta) uses weights W_j exact for cosine
// series of degree < m on the half-shifted nodes:
//   int f dS = sum_j W_j (2 pi / n) sum_i f[j][i]   (w[j] = 2 pi W_j / n).
// First pass: workgroup b sums rows b, b + G, ... (a fixed order, so the
// result is reproducible) into partial[b]; second pass: one workgroup adds
// the partials.
static __global__ void __launch_bounds__(256) k_integral_rows(const double* __restrict__ f, const double* __restrict__ w,
                                                       int n, int m, double* __restrict__ partial) {
    __shared__ Cx<double> red[8];
    double acc = 0.0;
    for (int j = blockIdx.x; j < m; j += gridDim.x) {
        const double2* row = reinterpret_cast<const double2*>(f + (size_t)j * n);
        double srow = 0.0;
        for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
            const double2 v = row[i];
            srow += v.x + v.y;
        }
        acc += srow * w[j];
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

static __global__ void __launch_bounds__(256) k_integral_total(const double* __restrict__ partial, int nb,
                                                        double* __restrict__ out) {
    __shared__ Cx<double> red[8];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[b];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace sp
