// Heterogeneous batches: many right-hand sides of different grid sizes solved
// by one graph launch.  Each stage of the solve (lambda forward, theta,
// lambda inverse; or the mixed-precision stages) is one persistent kernel:
// its resident workgroups take (rhs, tile) items from a work list, in list
// order, through an atomic counter, and run the same tile bodies as the
// single-problem kernels with that problem's descriptor.  Consecutive stages
// are separate kernels, so a stage sees the previous stage's results
// (kernel boundaries order and publish the memory of every XCD).
#pragma once
#include "sp_kernels.hpp"
#include "sp_theta_real.hpp"

namespace sp {

struct RhsDesc {
    int n, m, N, rw_log2, lay_log2;
    int lam_nthr, theta_nthr_fft, k64;
    int theta_real;    // 1: one real part per theta tile (even m, DFT length m/2); 0: complex line
    double c0;
    FftDesc fl, ft;
    const double* f;
    double* u;
    Cx<double>* spec64;
    Cx<double>* specB;
    Cx<double>* fco;
    Cx<float>* spec0;
    Cx<float>* specd;
    const Cx<double>* tw64n;
    const Cx<float>* tw32n;
    const Cx<double>* p64n;
    const Cx<float>* p32n;
    const Cx<double>* p64m;
    const Cx<float>* p32m;
    const Cx<double>* eq64;
    const Cx<float>* eq32;
    const Cx<double>* ws64;   // real-part split twiddles e^{-2 pi i q/m}, q <= m/4
    const Cx<float>* ws32;
    const double* sin2;
    const double* k0tab;
    const double* fint_w;
    double* scal;      // [0] integral of f, then per correction it: [2 it - 1] sum d^2, [2 it] sum u^2
    double* partial;   // 2 per lambda block
};

enum BatchStage {
    kBLamFwd = 0,      // float64 lambda transform of sin^2 f
    kBTheta64 = 1,     // float64 theta transform + solve + inverse
    kBLamInv = 2,      // float64 inverse lambda transform -> u
    kBThetaFirst = 3,  // mixed: first solve
    kBLamMix = 4,      // mixed: u0 and its float64 transform
    kBThetaResid = 5,  // mixed: residual and correction
    kBLamUpd = 6,      // mixed: u = u0 + correction
    kBStages = 7
};

// Stage arguments of one problem, built on the host and kept in device
// memory.  The kernels read them in place through a wave-uniform index, so
// every field (the transform descriptor's per-pass radix table included) is
// loaded by the scalar unit; a private copy would put the dynamically indexed
// pass table in per-lane scratch memory.
inline LambdaArgs<double> batch_lambda_args(const RhsDesc& d, bool forward) {
    LambdaArgs<double> la{};
    la.n = d.n; la.m = d.m; la.N = d.N; la.rw_log2 = d.rw_log2; la.lay_log2 = d.lay_log2;
    la.fft = d.fl; la.nthr = d.lam_nthr;
    la.tw = d.tw64n; la.ptw = d.p64n;
    la.spec = d.spec64;
    if (forward) {
        la.x = d.f; la.rowscale = d.sin2;
        la.w_mid = 1.0 / d.n; la.w_end = 1.0 / d.n;
    } else {
        la.y = d.u; la.rowscale = nullptr;
        la.w_mid = 1.0; la.w_end = 1.0; la.out_scale = 1.0;
    }
    return la;
}

inline ThetaArgs<double> batch_theta_args(const RhsDesc& d) {
    ThetaArgs<double> ta{};
    ta.spec = d.spec64; ta.spec_out = d.spec64; ta.tw = d.p64m; ta.eq = d.eq64; ta.ws = d.ws64;
    ta.n = d.n; ta.m = d.m; ta.N = d.N; ta.lay_log2 = d.lay_log2; ta.lay_out_log2 = d.lay_log2;
    ta.fft = d.ft; ta.nthr_fft = d.theta_nthr_fft; ta.mode = kSolve; ta.k8 = 0;
    ta.c0 = d.c0; ta.k0tab = d.k0tab; ta.fint_w = d.fint_w; ta.fint_out = d.scal;
    return ta;
}

inline MixLambdaArgs batch_mix_args(const RhsDesc& d) {
    MixLambdaArgs ma{};
    ma.s0 = d.spec0; ma.sd = d.specd; ma.su = d.specB; ma.u = d.u;
    ma.tw32 = d.tw32n; ma.tw64 = d.tw64n; ma.ptw32 = d.p32n; ma.ptw64 = d.p64n;
    ma.partial = d.partial; ma.rowscale = nullptr;
    ma.n = d.n; ma.m = d.m; ma.N = d.N; ma.rw_log2 = d.rw_log2; ma.lay_log2 = d.lay_log2;
    ma.lay_out_log2 = d.lay_log2;
    ma.in_w_mid = 1.0f; ma.in_w_end = 1.0f; ma.mid_scale = 1.0;
    ma.out_w_mid = 1.0 / d.n; ma.out_w_end = 1.0 / d.n; ma.out_scale = 1.0;
    ma.fft = d.fl; ma.nthr = d.lam_nthr; ma.accumulate = 0;
    return ma;
}

inline ThetaMixArgs batch_theta_mix_args(const RhsDesc& d, bool resid) {
    ThetaMixArgs ta{};
    ta.sa = d.spec64; ta.fco = d.fco; ta.su = d.specB; ta.out = resid ? d.specd : d.spec0;
    ta.tw64 = d.p64m; ta.eq64 = d.eq64; ta.tw32 = d.p32m; ta.eq32 = d.eq32;
    ta.ws64 = d.ws64; ta.ws32 = d.ws32;
    ta.n = d.n; ta.m = d.m; ta.N = d.N; ta.lay_log2 = d.lay_log2; ta.lay_out_log2 = d.lay_log2;
    ta.fft = d.ft; ta.nthr_fft = d.theta_nthr_fft; ta.k8 = 0;
    ta.c0 = d.c0; ta.k0tab = d.k0tab;
    ta.fint_w = resid ? nullptr : d.fint_w; ta.fint_out = d.scal;
    ta.k64 = d.k64;
    return ta;
}

// NT: threads per tile.  WPE: waves per SIMD the register budget is sized for
// (4: 128 registers, 2: 256), so that several tiles share a compute unit and
// hide each other's memory and barrier latency.  args: the stage's argument array, one entry per
// problem (LambdaArgs, ThetaArgs, MixLambdaArgs or ThetaMixArgs by stage).
// REAL (theta stages): items are (problem, 2k + part), one real part of
// wavenumber k per tile; otherwise (problem, k) on the complex line.
template <int EPT, int RMAX, int SMAXF, int SMAXD, int STAGE, int NT, int WPE, bool REAL>
__global__ void __launch_bounds__(NT, WPE) k_batch(const void* __restrict__ args, const int2* __restrict__ items,
                                                    int nitems, int* __restrict__ counter) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Cx<double> red[16];
    __shared__ double red2[2][16];
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(cur);
        __syncthreads();
        if (it >= nitems) break;          // every wave leaves once the list is exhausted
        const int2 w = items[it];
        if constexpr (STAGE == kBLamFwd) {
            lambda_fwd_body<double, EPT, RMAX>(static_cast<const LambdaArgs<double>*>(args)[w.x], w.y, smem_raw);
        } else if constexpr (STAGE == kBTheta64) {
            const ThetaArgs<double>& ta = static_cast<const ThetaArgs<double>*>(args)[w.x];
            if constexpr (REAL)
                theta_real_body<double, EPT, RMAX, SMAXD>(ta, w.y >> 1, w.y & 1, smem_raw, red);
            else
                theta_body<double, EPT, RMAX, SMAXD>(ta, w.y, smem_raw, red);
        } else if constexpr (STAGE == kBLamInv) {
            lambda_inv_body<double, EPT, RMAX>(static_cast<const LambdaArgs<double>*>(args)[w.x], w.y, smem_raw);
        } else if constexpr (STAGE == kBThetaFirst) {
            const ThetaMixArgs& ta = static_cast<const ThetaMixArgs*>(args)[w.x];
            if constexpr (REAL)
                theta_mixed_real_body<EPT, RMAX, SMAXF, SMAXD, false, false>(ta, w.y >> 1, w.y & 1, smem_raw, red);
            else
                theta_mixed_body<EPT, RMAX, SMAXF, SMAXD, false, false>(ta, w.y, smem_raw, red);
        } else if constexpr (STAGE == kBLamMix) {
            lambda_mix_body<EPT, RMAX>(static_cast<const MixLambdaArgs*>(args)[w.x], w.y, smem_raw);
        } else if constexpr (STAGE == kBThetaResid) {
            const ThetaMixArgs& ta = static_cast<const ThetaMixArgs*>(args)[w.x];
            if constexpr (REAL)
                theta_mixed_real_body<EPT, RMAX, SMAXF, SMAXD, true, false>(ta, w.y >> 1, w.y & 1, smem_raw, red);
            else
                theta_mixed_body<EPT, RMAX, SMAXF, SMAXD, true, false>(ta, w.y, smem_raw, red);
        } else {
            lambda_update_body<EPT, RMAX>(static_cast<const MixLambdaArgs*>(args)[w.x], w.y, smem_raw, red2);
        }
    }
}

// Counters of every stage back to zero (a kernel node, not a memset node).
static __global__ void __launch_bounds__(64) k_batch_reset(int* counters, int n) {
    if ((int)threadIdx.x < n) counters[threadIdx.x] = 0;
}

// One block per right-hand side: sums of the update partials -> scal[slot], scal[slot + 1].
static __global__ void __launch_bounds__(256) k_batch_norms(const RhsDesc* __restrict__ descs, const int* __restrict__ nblk,
                                                            int slot) {
    __shared__ double r0[256], r1[256];
    const RhsDesc& d = descs[blockIdx.x];
    const int nb = nblk[blockIdx.x];
    double x = 0.0, y = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) { x += d.partial[2 * b]; y += d.partial[2 * b + 1]; }
    r0[threadIdx.x] = x;
    r1[threadIdx.x] = y;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) { r0[threadIdx.x] += r0[threadIdx.x + h]; r1[threadIdx.x] += r1[threadIdx.x + h]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { d.scal[slot] = r0[0]; d.scal[slot + 1] = r1[0]; }
}

}  // namespace sp
