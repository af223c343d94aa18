// Transform and solve kernels of the DFS Poisson solver (Section 5 of the
// paper): lambda real transforms (rows of the grid), and the per-wavenumber
// theta pass (cosine/sine transform, banded solves, inverse transform).
//
// Spectrum layout in HBM ("j-blocked"): the half spectrum X_k(theta_j),
// k = 0..N (N = n/2), is stored as spec[((j / RL) * (N + 1) + k) * RL + j % RL]
// with RL = 2^lay a power of two, the run length.  Each buffer takes the
// layout its reader prefers: spectra read by a theta pass use runs of at
// least 8 rows (one 128-byte line of a wavenumber in float64; a lambda
// workgroup owns RW <= RL rows and writes its part of every run).  The float64
// solve's theta output, read by the lambda inverse, uses RL = RW (one
// contiguous block per lambda workgroup); the mixed solve's float32 spectra
// and every spectrum of a batch keep the theta runs, since the theta passes
// write them in halves (one real part per workgroup).
#pragma once
#include "sp_fft.hpp"

namespace sp {

// ---------------------------------------------------------------- lambda pass
// Real DFT of length n through a complex DFT of length N = n/2:
// z_i = x_{2i} + i x_{2i+1}, Z = DFT_N(z), then for the pair (k, N-k)
//   E = (Z_k + conj Z_{N-k})/2,  O = (Z_k - conj Z_{N-k})/(2i),  W = e^{-2 pi i k/n}
//   X_k = E + W O,  X_{N-k} = conj(E - W O);  X_0 = Re Z_0 + Im Z_0, X_N = Re Z_0 - Im Z_0.
// The inverse runs the same relations backwards:
//   P = X_k + conj X_{N-k}, Q = X_k - conj X_{N-k}
//   Z_k = P + i conj(W) Q,  Z_{N-k} = conj(P - i conj(W) Q),  z = IDFT_N(Z) (unnormalised).

template <typename T>
struct LambdaArgs {
    const double* x;        // forward: input rows [m][n]
    double* y;              // inverse: output rows [m][n]
    Cx<T>* spec;            // spectrum (forward: written; inverse: read)
    const Cx<T>* tw;        // e^{-2 pi i t/n}, t = 0..n-1 (real-spectrum split)
    const Cx<T>* ptw;       // per-pass twiddles of the length-N complex DFT
    const double* rowscale; // per-row multiplier or nullptr
    int n, m, N, rw_log2;   // rw_log2: rows per workgroup (log2)
    int lay_log2;           // run length (log2) of the spectrum written (forward) or read (inverse)
    T w_mid, w_end;         // forward: output weight for 0<k<N and for k in {0,N}; inverse: input weights
    double out_scale;       // inverse: multiplier of the written rows
    FftDesc fft;
    int nthr;               // threads per row
};

// Block layout helpers: a lambda workgroup owns rows jb*RW .. jb*RW+RW-1; row r
// of the block uses LDS line `lines + r * stride`.
__device__ __forceinline__ size_t spec_at(int j, int k, int N, int lay) {
    return ((((size_t)(j >> lay)) * (N + 1) + k) << lay) + (j & ((1 << lay) - 1));
}

// Lambda workgroup -> row block.  When one spectrum run spans g = 2^glog2 row
// blocks, the g blocks of a run go to consecutive workgroups of one XCD
// (workgroups are dealt round-robin over the 8 XCDs), so their writes to the
// same 128-byte lines meet in that XCD's L2.  The grid is a multiple of 8 g.
__device__ __forceinline__ int lambda_tile_of(int tile, int glog2) {
    const int x = tile & 7, i = tile >> 3;
    return ((x + ((i >> glog2) << 3)) << glog2) + (i & ((1 << glog2) - 1));
}
__device__ __forceinline__ int lambda_tile(int glog2) { return lambda_tile_of(blockIdx.x, glog2); }

// Split the length-N complex DFT of every row into the half spectrum X_0..X_N
// (times w_mid for 0<k<N, w_end for k in {0, N}) and store it (type TS).
// Lanes run over (pair, row) with the row fastest, so stores are contiguous.
template <typename T, typename TS>
__device__ __forceinline__ void r2c_split_store(const Cx<T>* lines, size_t stride, Cx<TS>* spec,
                                                const Cx<T>* tw, int N, int rwl, int lay, int m, int jb,
                                                T w_mid, T w_end) {
    const int rw = 1 << rwl;
    const int npairs = N / 2 + 1;
    for (int e = threadIdx.x; e < npairs * rw; e += blockDim.x) {
        const int jj = e & (rw - 1);
        const int k = e >> rwl;
        const int j = (jb << rwl) + jj;
        if (j >= m) continue;
        const Cx<T>* b = lines + (size_t)jj * stride;
        if (k == 0) {
            const Cx<T> z = b[0];
            spec[spec_at(j, 0, N, lay)] = Cx<TS>{(TS)((z.x + z.y) * w_end), (TS)0};
            spec[spec_at(j, N, N, lay)] = Cx<TS>{(TS)((z.x - z.y) * w_end), (TS)0};
            continue;
        }
        const Cx<T> zk = b[k], zn = b[N - k];
        const Cx<T> E = (zk + cconj(zn)) * (T)0.5;
        const Cx<T> O = mul_negi(zk - cconj(zn)) * (T)0.5;
        const Cx<T> WO = cmul(tw[k], O);
        const Cx<T> xk = (E + WO) * w_mid;
        spec[spec_at(j, k, N, lay)] = Cx<TS>{(TS)xk.x, (TS)xk.y};
        if (N - k != k) {
            const Cx<T> xn = cconj(E - WO) * w_mid;
            spec[spec_at(j, N - k, N, lay)] = Cx<TS>{(TS)xn.x, (TS)xn.y};
        }
    }
}

// Read the half spectrum of every row (type TS, times w_mid / w_end) and build
// the length-N complex sequence whose inverse DFT interleaves the real output.
// DLAM: the spectrum of d/dlambda instead, coefficient k times i k; the k = 0
// and k = n/2 terms vanish (the derivative of the real Nyquist mode is zero on
// the grid).  Element e of a thread's share (e = threadIdx.x + it blockDim.x
// < (N/2 + 1) RW, the row fastest) is the pair (k, N - k) of row e mod RW;
// c2r_fetch loads those pairs, c2r_build forms the two line entries.
template <typename TS>
__device__ __forceinline__ void c2r_fetch(const Cx<TS>* spec, int N, int rwl, int lay, int m, int jb, int e,
                                          Cx<TS>& sk, Cx<TS>& sn) {
    const int jj = e & ((1 << rwl) - 1);
    const int k = e >> rwl;
    const int j = (jb << rwl) + jj;
    if (j >= m) return;
    sk = spec[spec_at(j, k, N, lay)];
    sn = spec[spec_at(j, k == 0 ? N : N - k, N, lay)];
}

template <typename T, typename TS, bool DLAM = false>
__device__ __forceinline__ void c2r_build(Cx<T>* lines, size_t stride, const Cx<T>* tw, int N, int rwl, int m,
                                          int jb, int e, Cx<TS> sk, Cx<TS> sn, T w_mid, T w_end) {
    const int jj = e & ((1 << rwl) - 1);
    const int k = e >> rwl;
    const int j = (jb << rwl) + jj;
    if (j >= m) return;
    Cx<T>* b = lines + (size_t)jj * stride;
    if (k == 0) {
        if constexpr (DLAM) {
            b[0] = Cx<T>{(T)0, (T)0};
        } else {
            const T x0 = (T)sk.x * w_end;
            const T xN = (T)sn.x * w_end;
            b[0] = Cx<T>{x0 + xN, x0 - xN};
        }
        return;
    }
    Cx<T> xk = Cx<T>{(T)sk.x, (T)sk.y} * w_mid;
    Cx<T> xn = Cx<T>{(T)sn.x, (T)sn.y} * w_mid;
    if constexpr (DLAM) {
        xk = mul_i(xk) * (T)k;
        xn = mul_i(xn) * (T)(N - k);
    }
    const Cx<T> P = xk + cconj(xn);
    const Cx<T> Q = xk - cconj(xn);
    const Cx<T> iWQ = mul_i(cmulc(Q, tw[k]));   // i conj(W) Q
    b[k] = P + iWQ;
    if (N - k != k) b[N - k] = cconj(P - iWQ);
}

template <typename T, typename TS, bool DLAM = false>
__device__ __forceinline__ void c2r_load_prepare(Cx<T>* lines, size_t stride, const Cx<TS>* spec,
                                                 const Cx<T>* tw, int N, int rwl, int lay, int m, int jb,
                                                 T w_mid, T w_end) {
    const int total = (N / 2 + 1) << rwl;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        Cx<TS> sk{}, sn{};
        c2r_fetch<TS>(spec, N, rwl, lay, m, jb, e, sk, sn);
        c2r_build<T, TS, DLAM>(lines, stride, tw, N, rwl, m, jb, e, sk, sn, w_mid, w_end);
    }
}

// x_{2i}, x_{2i+1} (one double2 per complex input) times s into buf[i] for
// i = t, t + nthr, ... < N, ten loads in flight per thread (branch-free:
// the last one is re-read): the whole row of the length-5000 transform in one
// round trip (eight measured 4% slower there).
template <typename T>
__device__ __forceinline__ void load_row(Cx<T>* buf, const double2* __restrict__ src, double s, int t, int nthr,
                                         int N) {
    constexpr int kB = 10;
    const int cnt = t < N ? (N - 1 - t) / nthr + 1 : 0;
    for (int e0 = 0; e0 < cnt; e0 += kB) {
        double2 v[kB];
#pragma unroll
        for (int e = 0; e < kB; ++e) v[e] = src[t + min(e0 + e, cnt - 1) * nthr];
#pragma unroll
        for (int e = 0; e < kB; ++e)
            if (e0 + e < cnt) buf[t + (e0 + e) * nthr] = Cx<T>{(T)(v[e].x * s), (T)(v[e].y * s)};
    }
}

// Each kernel is a __device__ body taking its tile index (a block of rows, or
// one wavenumber) and its LDS; the __global__ wrappers map blockIdx to the
// tile, the batch kernels take tiles from a work list.
template <typename T, int EPT, int RMAX>
__device__ __forceinline__ void lambda_fwd_body(const LambdaArgs<T>& a, int jb, unsigned char* smem_raw) {
    Cx<T>* lines = reinterpret_cast<Cx<T>*>(smem_raw);
    const int N = a.N;
    const int line = threadIdx.x / a.nthr;
    const int t = threadIdx.x - line * a.nthr;
    const int j = (jb << a.rw_log2) + line;
    const bool active = line < (1 << a.rw_log2) && j < a.m;
    Cx<T>* buf = lines + (size_t)line * N;
    // (Feeding the fixed transform's first pass from these loads, without the
    // LDS round trip, measured no faster here and slowed the mixed solve.)
    if (active) {
        const double s = a.rowscale ? a.rowscale[j] : 1.0;
        load_row<T>(buf, reinterpret_cast<const double2*>(a.x + (size_t)j * a.n), s, t, a.nthr, N);
    }
    __syncthreads();
    fft_lds<T, false, EPT, RMAX>(lines, line * N, a.fft, a.ptw, t, a.nthr, active);
    r2c_split_store<T, T>(lines, N, a.spec, a.tw, N, a.rw_log2, a.lay_log2, a.m, jb, a.w_mid, a.w_end);
}

template <typename T, int EPT, int RMAX>
__global__ void __launch_bounds__(1024) k_lambda_fwd(LambdaArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int jb = lambda_tile(a.lay_log2 - a.rw_log2);
    if (jb << a.rw_log2 >= a.m) return;
    lambda_fwd_body<T, EPT, RMAX>(a, jb, smem_raw);
}

template <typename T, int EPT, int RMAX>
__device__ __forceinline__ void lambda_inv_body(const LambdaArgs<T>& a, int jb, unsigned char* smem_raw) {
    Cx<T>* lines = reinterpret_cast<Cx<T>*>(smem_raw);
    const int N = a.N;
    const int line = threadIdx.x / a.nthr;
    const int t = threadIdx.x - line * a.nthr;
    const int j = (jb << a.rw_log2) + line;
    const bool active = line < (1 << a.rw_log2) && j < a.m;
    c2r_load_prepare<T, T>(lines, N, a.spec, a.tw, N, a.rw_log2, a.lay_log2, a.m, jb, a.w_mid, a.w_end);
    __syncthreads();
    if constexpr (RMAX == kRadixFixed5000) {
        // the last pass's points t + 500 r go straight to the row
        Cx<T> v[10];
        fft5000_regs<T, true, false, true>(lines + (size_t)line * N, a.ptw, t, active, v);
        if (active) {
            const double s = a.out_scale * (a.rowscale ? a.rowscale[j] : 1.0);
            double2* dst = reinterpret_cast<double2*>(a.y + (size_t)j * a.n);
#pragma unroll
            for (int r = 0; r < 10; ++r)
                dst[t + r * kFixed5000Threads] = double2{(double)v[r].x * s, (double)v[r].y * s};
        }
    } else {
        fft_lds<T, true, EPT, RMAX>(lines, line * N, a.fft, a.ptw, t, a.nthr, active);
        if (active) {
            const Cx<T>* buf = lines + (size_t)line * N;
            const double s = a.out_scale * (a.rowscale ? a.rowscale[j] : 1.0);
            double2* dst = reinterpret_cast<double2*>(a.y + (size_t)j * a.n);
            for (int i = t; i < N; i += a.nthr) {
                const Cx<T> z = buf[i];
                dst[i] = double2{(double)z.x * s, (double)z.y * s};
            }
        }
    }
}

template <typename T, int EPT, int RMAX>
__global__ void __launch_bounds__(1024) k_lambda_inv(LambdaArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int jb = lambda_tile(a.lay_log2 - a.rw_log2);
    if (jb << a.rw_log2 >= a.m) return;
    lambda_inv_body<T, EPT, RMAX>(a, jb, smem_raw);
}

// ---------------------------------------------------------------- mixed lambda passes
struct MixLambdaArgs {
    const Cx<float>* s0;       // float32 spectrum of the first iterate
    const Cx<float>* sd;       // float32 spectrum of the correction
    Cx<double>* su;            // float64 spectrum written by k_lambda_mix
    double* u;                 // output rows [m][n]
    const Cx<float>* tw32;     // e^{-2 pi i t/n} (float32)
    const Cx<double>* tw64;    // e^{-2 pi i t/n} (float64)
    const Cx<float>* ptw32;    // per-pass twiddles of the length-N DFT (float32)
    const Cx<double>* ptw64;   // per-pass twiddles of the length-N DFT (float64)
    double* partial;           // per block: sum of correction^2 and of u^2 (or nullptr)
    const double* rowscale;    // update: per-row output multiplier (or nullptr)
    int n, m, N, rw_log2;
    int lay_log2;              // run length (log2) of the float32 spectra read
    int lay_out_log2;          // run length (log2) of the float64 spectrum written (mix)
    float in_w_mid, in_w_end;  // weights of the float32 spectra read by the inverse DFTs
    double mid_scale;          // mix: multiplier of the float32 inverse DFT before the float64 forward DFT
    double out_w_mid, out_w_end; // mix: weights of the float64 spectrum written
    double out_scale;          // update: multiplier of the written rows
    FftDesc fft;
    int nthr;
    int accumulate;            // 1: u += correction (u already holds the previous iterate)
};

// Every thread holds at most this many line values while a line changes precision.
template <int EPT, int RMAX>
struct LineHold {
    static constexpr int value = EPT > RMAX ? EPT : RMAX;
};

// u0 = mid_scale * (inverse float32 DFT of the weighted s0) per row, then the
// float64 forward DFT of u0 with weights out_w -> su.  Forward solve: weights
// 1, mid_scale 1, out_w 1/n.  Adjoint: in_w (1/2, 1), mid_scale 1/n, out_w
// (2, 1) (the transposes of the real DFT pair).  LDS per row: N float64 complex.
// The float32 inverse DFT itself (before mid_scale) is also kept, as n floats
// at the start of the row's own output row u[j], for the update pass: it reads
// 4 bytes per sample there instead of transforming s0 a second time.
template <int EPT, int RMAX>
__device__ __forceinline__ void lambda_mix_body(const MixLambdaArgs& a, int jb, unsigned char* smem_raw) {
    Cx<double>* lines = reinterpret_cast<Cx<double>*>(smem_raw);
    const int N = a.N;
    const int line = threadIdx.x / a.nthr;
    const int t = threadIdx.x - line * a.nthr;
    const int j = (jb << a.rw_log2) + line;
    const bool active = line < (1 << a.rw_log2) && j < a.m;
    // float32 view: row r uses the first N float32 complex slots of its float64 line
    Cx<float>* fl = reinterpret_cast<Cx<float>*>(lines);
    c2r_load_prepare<float, float>(fl, 2 * (size_t)N, a.s0, a.tw32, N, a.rw_log2, a.lay_log2, a.m, jb, a.in_w_mid,
                                   a.in_w_end);
    __syncthreads();
    Cx<float>* fbuf = fl + (size_t)line * 2 * N;
    if constexpr (RMAX == kRadixFixed5000) {
        // the float32 inverse's last pass stays in registers (the points
        // t + 500 r: kept, widened and fed to the float64 transform's first
        // pass without a round trip through the LDS)
        Cx<float> vf[10];
        fft5000_regs<float, true, false, true>(fbuf, a.ptw32, t, active, vf);
        Cx<double> vd[10];
        if (active) {
            Cx<float>* keep = reinterpret_cast<Cx<float>*>(a.u + (size_t)j * a.n);
#pragma unroll
            for (int r = 0; r < 10; ++r) {
                keep[t + r * kFixed5000Threads] = vf[r];
                vd[r] = Cx<double>{(double)vf[r].x * a.mid_scale, (double)vf[r].y * a.mid_scale};
            }
        }
        __syncthreads();   // every thread has read the float32 line the float64 line overwrites
        fft5000_regs<double, false, true, false>(lines + (size_t)line * N, a.ptw64, t, active, vd);
    } else {
        fft_lds<float, true, EPT, RMAX>(fl, line * 2 * N, a.fft, a.ptw32, t, a.nthr, active);
        constexpr int H = LineHold<EPT, RMAX>::value;
        Cx<float> hold[H];
#pragma unroll
        for (int e = 0; e < H; ++e) {
            const int i = t + e * a.nthr;
            if (active && i < N) hold[e] = fbuf[i];
        }
        if (active) {
            Cx<float>* keep = reinterpret_cast<Cx<float>*>(a.u + (size_t)j * a.n);
#pragma unroll
            for (int e = 0; e < H; ++e) {
                const int i = t + e * a.nthr;
                if (i < N) keep[i] = hold[e];
            }
        }
        __syncthreads();
        Cx<double>* dbuf = lines + (size_t)line * N;
#pragma unroll
        for (int e = 0; e < H; ++e) {
            const int i = t + e * a.nthr;
            if (active && i < N) dbuf[i] = Cx<double>{(double)hold[e].x * a.mid_scale, (double)hold[e].y * a.mid_scale};
        }
        __syncthreads();
        fft_lds<double, false, EPT, RMAX>(lines, line * N, a.fft, a.ptw64, t, a.nthr, active);
    }
    r2c_split_store<double, double>(lines, N, a.su, a.tw64, N, a.rw_log2, a.lay_out_log2, a.m, jb, a.out_w_mid,
                                    a.out_w_end);
}

template <int EPT, int RMAX>
__global__ void __launch_bounds__(1024) k_lambda_mix(MixLambdaArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int jb = lambda_tile(a.lay_out_log2 - a.rw_log2);
    if (jb << a.rw_log2 >= a.m) return;
    lambda_mix_body<EPT, RMAX>(a, jb, smem_raw);
}

// Per-block sums of (s d)^2 and u^2 of the update pass (when a.partial is set).
__device__ __forceinline__ void block_partials(const MixLambdaArgs& a, int jb, double sd2, double su2,
                                               double (*red)[16]) {
    if (!a.partial) return;
    for (int off = 32; off > 0; off >>= 1) {
        sd2 += __shfl_down(sd2, off, 64);
        su2 += __shfl_down(su2, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { red[0][wave] = sd2; red[1][wave] = su2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) { x += red[0][w]; y += red[1][w]; }
        a.partial[2 * jb] = x;
        a.partial[2 * jb + 1] = y;
    }
    __syncthreads();
}

// u = s (u0 + d) (or u += s d) with u0, d the float32 inverse DFTs of the
// weighted s0 and sd, summed in float64, s = out_scale * rowscale[j].  u0 is
// the copy the mix pass left at the start of each output row; every thread
// reads the values it combines into registers before a full barrier that
// precedes the row's first store, so no row is overwritten before it has
// been read.  LDS per row: N float32 complex (the correction line only).
// Optionally accumulates per-block sums of (s d)^2 and u^2.
// The fixed length-5000 transform runs the rows of a tile (at most two: two
// float64 rows fill the LDS in the other lambda passes) one after the other
// in the threads of one row, so that the tile takes 512 threads and two
// tiles share a compute unit; the general form runs the rows side by side.
template <int EPT, int RMAX>
__device__ __forceinline__ void lambda_update_body(const MixLambdaArgs& a, int jb, unsigned char* smem_raw,
                                                   double (*red)[16]) {
    Cx<float>* fl = reinterpret_cast<Cx<float>*>(smem_raw);   // row r: the correction line
    const int N = a.N;
    if constexpr (RMAX == kRadixFixed5000) {
        c2r_load_prepare<float, float>(fl, (size_t)N, a.sd, a.tw32, N, a.rw_log2, a.lay_log2, a.m, jb, a.in_w_mid,
                                       a.in_w_end);
        __syncthreads();
        double sd2 = 0.0, su2 = 0.0;
#pragma unroll 1
        for (int row = 0; row < (1 << a.rw_log2); ++row) {
            int t = threadIdx.x;
            asm volatile("" : "+v"(t));   // keeps each row's index arithmetic inside the row (no spills)
            const int j = (jb << a.rw_log2) + row;
            const bool act = t < kFixed5000Threads && j < a.m;
            // the last pass's points t + 500 r stay in registers
            Cx<float> vf[10];
            fft5000_regs<float, true, false, true>(fl + (size_t)row * N, a.ptw32, t, act, vf);
            Cx<float> u0[10];
            if (!a.accumulate && act) {
                const Cx<float>* keep = reinterpret_cast<const Cx<float>*>(a.u + (size_t)j * a.n);
#pragma unroll
                for (int r = 0; r < 10; ++r) u0[r] = keep[t + r * kFixed5000Threads];
            }
            __syncthreads();   // every thread holds its kept values of row j before any thread writes the row
            if (act) {
                const double sc = a.out_scale * (a.rowscale ? a.rowscale[j] : 1.0);
                double2* dst = reinterpret_cast<double2*>(a.u + (size_t)j * a.n);
#pragma unroll
                for (int r = 0; r < 10; ++r) {
                    const int i = t + r * kFixed5000Threads;
                    const double dx = (double)vf[r].x * sc, dy = (double)vf[r].y * sc;
                    double2 base;
                    if (a.accumulate) base = dst[i];
                    else base = double2{(double)u0[r].x * sc, (double)u0[r].y * sc};
                    const double2 v = double2{base.x + dx, base.y + dy};
                    dst[i] = v;
                    sd2 += dx * dx + dy * dy;
                    su2 += v.x * v.x + v.y * v.y;
                }
            }
        }
        block_partials(a, jb, sd2, su2, red);
        return;
    }
    const int line = threadIdx.x / a.nthr;
    const int t = threadIdx.x - line * a.nthr;
    const int j = (jb << a.rw_log2) + line;
    const bool active = line < (1 << a.rw_log2) && j < a.m;
    constexpr int H = LineHold<EPT, RMAX>::value;
    Cx<float> u0[H];
    if (!a.accumulate && active) {
        const Cx<float>* keep = reinterpret_cast<const Cx<float>*>(a.u + (size_t)j * a.n);
#pragma unroll
        for (int e = 0; e < H; ++e) {
            const int i = t + e * a.nthr;
            if (i < N) u0[e] = keep[i];
        }
    }
    c2r_load_prepare<float, float>(fl, (size_t)N, a.sd, a.tw32, N, a.rw_log2, a.lay_log2, a.m, jb, a.in_w_mid,
                                   a.in_w_end);
    __syncthreads();
    // fixed transform: the last pass's points t + 500 r stay in registers
    Cx<float> vf[RMAX == kRadixFixed5000 ? 10 : 1];
    if constexpr (RMAX == kRadixFixed5000)
        fft5000_regs<float, true, false, true>(fl + (size_t)line * N, a.ptw32, t, active, vf);
    else
        fft_lds<float, true, EPT, RMAX>(fl, line * N, a.fft, a.ptw32, t, a.nthr, active);
    const Cx<float>* b1 = fl + (size_t)line * N;
    double sd2 = 0.0, su2 = 0.0;
    if (active) {
        const double sc = a.out_scale * (a.rowscale ? a.rowscale[j] : 1.0);
        double2* dst = reinterpret_cast<double2*>(a.u + (size_t)j * a.n);
#pragma unroll
        for (int e = 0; e < H; ++e) {
            const int i = t + e * a.nthr;
            if (i < N) {
                Cx<float> d;
                if constexpr (RMAX == kRadixFixed5000) d = vf[e < 10 ? e : 0];
                else d = b1[i];
                const double dx = (double)d.x * sc, dy = (double)d.y * sc;
                double2 base;
                if (a.accumulate) base = dst[i];
                else base = double2{(double)u0[e].x * sc, (double)u0[e].y * sc};
                const double2 v = double2{base.x + dx, base.y + dy};
                dst[i] = v;
                sd2 += dx * dx + dy * dy;
                su2 += v.x * v.x + v.y * v.y;
            }
        }
    }
    block_partials(a, jb, sd2, su2, red);
}

template <int EPT, int RMAX>
__global__ void __launch_bounds__(1024) k_lambda_update(MixLambdaArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][16];
    const int jb = lambda_tile(a.lay_log2 - a.rw_log2);
    if (jb << a.rw_log2 >= a.m) return;
    lambda_update_body<EPT, RMAX>(a, jb, smem_raw, red);
}

// Sum of the per-block partials (one block): out[0] = sum of d^2, out[1] = sum of u^2.
static __global__ void __launch_bounds__(256) k_reduce_partials(const double* partial, int nblk, double* out) {
    __shared__ double r0[256], r1[256];
    double x = 0.0, y = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) { x += partial[2 * b]; y += partial[2 * b + 1]; }
    r0[threadIdx.x] = x;
    r1[threadIdx.x] = y;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) { r0[threadIdx.x] += r0[threadIdx.x + h]; r1[threadIdx.x] += r1[threadIdx.x + h]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = r0[0]; out[1] = r1[0]; }
}

// ---------------------------------------------------------------- theta pass
// Column k of the doubled function is even in theta for even k and odd for
// odd k (the even/odd split of Section 3.2), so it is expanded in cosines
// (q = 0..m-1) or sines (q = 1..m).  Both use one complex DFT of length m:
//   cosine analysis: v = x reordered (x_0, x_2, ..., x_5, x_3, x_1), V = DFT_m(v),
//     y_q = (E_q V_q + conj(E_q) V_{m-q}) / 2 = sum_j x_j cos(q theta_j), E_q = e^{-i pi q/(2m)};
//   sine analysis: sum_j x_j sin(q theta_j) = cosine analysis of (-1)^j x_j at m - q;
//   synthesis: V_q = conj(E_q) (y_q - i y_{m-q}), v = IDFT_m(V) / m, x = v un-reordered.
// The coefficient with index q sits at LDS position p = q (cosine) or m - q (sine);
// true coefficients are a_q = c_p y_q with c_0 = 1/m, c_p = 2/m otherwise.
//
// Per wavenumber the operator L - k^2 I of Section 5 couples q to q +- 2 only:
//   row q: (q-2)(q-1)/4 * a_{q-2} - (q^2/2 + k^2) a_q + (q+2)(q+1)/4 * a_{q+2},
// which splits into an even-q and an odd-q tridiagonal class.  Out-of-range
// neighbours are dropped.  For k = 0 (cosine) the q = 0 row is replaced by the
// integral constraint a_0 = c0 - sum_{q>=2 even} a_q / (1 - q^2).

enum ThetaMode { kSolve = 0, kSolveTransposed = 1, kTransformOnly = 2, kDerivative = 3, kDivideSin = 4 };

constexpr int kThetaHold = 16;   // positions per thread in the residual / conversion loops, complex-line derivative

// d/dtheta of a column held as true coefficients in position order (a cosine
// series, coefficient q at position q, for even k; a sine series, coefficient
// q at position m - q, for odd k).  The derivative of a cosine series is the
// sine series with coefficients -q a_q, and that of a sine series the cosine
// series with coefficients q b_q; in both cases the new value at position p
// comes from position m - p:
//   even k: out[p] = -(m - p) in[m - p],   odd k: out[p] = p in[m - p],
// and out[0] = 0: for even k it would be the sine coefficient q = m, which
// needs a cosine coefficient q = m that the series does not have; for odd k it
// is the constant term of the derivative.  (The derivative of the sine term
// q = m, at position 0, is a multiple of cos(m theta), zero at every grid
// node.)  The column is then synthesised with the other parity.
// HOLD >= m / nthr.
template <typename V> struct ScalarOf { using type = V; };
template <typename T> struct ScalarOf<Cx<T>> { using type = T; };

template <typename V, int HOLD>
__device__ __forceinline__ void theta_derivative_line(V* y, int m, bool sine, int tid, int nthr) {
    using S = typename ScalarOf<V>::type;
    V h[HOLD];
#pragma unroll
    for (int e = 0; e < HOLD; ++e) {
        const int p = tid + e * nthr;
        if (p < m) {
            const S w = p == 0 ? (S)0 : (sine ? (S)p : -(S)(m - p));
            h[e] = p == 0 ? V{} : y[m - p] * w;
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < HOLD; ++e) {
        const int p = tid + e * nthr;
        if (p < m) y[p] = h[e];
    }
    __syncthreads();
}

template <typename T>
struct ThetaArgs {
    Cx<T>* spec;
    const Cx<T>* tw;        // per-pass twiddles of the length-m complex DFT
    const Cx<T>* eq;        // e^{-i pi q/(2m)}, q = 0..m-1
    const Cx<T>* ws;        // real-part pass: e^{-2 pi i q/m}, q = 0..m/4
    Cx<T>* spec_out;        // spectrum written (may be spec when both layouts agree)
    int n, m, N;
    int lay_log2;           // run length (log2) of the spectrum read
    int lay_out_log2;       // run length (log2) of the spectrum written
    FftDesc fft;
    int nthr_fft;
    int mode;               // ThetaMode
    int k8;                 // wavenumbers per XCD slice (ceil((N+1)/8))
    double c0;              // k = 0 constraint value for a_0 (integral / (4 pi))
    const double* k0tab;    // k = 0 LU factors: invA[NA] cpA[NA] invB[NB] cpB[NB]
    const double* fint_w;   // quadrature weights of the integral of f (k = 0 column), or nullptr
    double* fint_out;
};

// Rows of (L - k^2 I) restricted to one parity class, with kk = k^2:
//   sub = (q-2)(q-1)/4 = q^2/4 - 3q/4 + 1/2,  sup = (q+2)(q+1)/4 = q^2/4 + 3q/4 + 1/2,
//   diag = -q^2/2 - k^2;
// the transpose has sub'(q) = sup(q-2) = q^2/4 - q/4 and sup'(q) = sub(q+2) = q^2/4 + q/4.
// In float64 every value is exact for the sizes supported (q^2 < 2^53).
template <typename T>
__device__ __forceinline__ void band_kk(T q, T kk, bool first, bool last, bool transposed, T& sub, T& diag,
                                        T& sup) {
    const T qq = q * q;
    const T base = qq * (T)0.25 + (transposed ? (T)0 : (T)0.5);
    const T lin = q * (transposed ? (T)0.25 : (T)0.75);
    diag = qq * (T)-0.5 - kk;
    sub = first ? (T)0 : base - lin;
    sup = last ? (T)0 : base + lin;
}

template <typename T>
__device__ __forceinline__ void band(int q, int k, bool first, bool last, bool transposed,
                                     T& sub, T& diag, T& sup) {
    band_kk<T>((T)q, (T)k * (T)k, first, last, transposed, sub, diag, sup);
}

// Reciprocals of the pivots (never tiny nor huge here): the hardware estimate
// refined by two Newton steps in float64 (about one ulp); float32 uses the
// estimate, which is within one ulp.
__device__ __forceinline__ double rcp_pivot(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp_pivot(float x) { return __builtin_amdgcn_rcpf(x); }

struct ClassInfo {
    int q0, nc, s, p;     // first q, rows, chunk length, chunks
};

// Chunks of at most SMAX rows, of odd length when possible: the rows of a
// class sit two line positions apart, so consecutive chunks start 2s
// positions apart, and an odd s spreads the threads' LDS accesses over the
// banks (at most two-way conflicts instead of up to 16-way).  The chunk count
// never exceeds ceil(rows / SMAX), and no chunk is empty.
template <int SMAX>
__device__ __forceinline__ ClassInfo make_class(int q0, int qhi) {
    ClassInfo c;
    c.q0 = q0;
    c.nc = qhi >= q0 ? (qhi - q0) / 2 + 1 : 0;
    c.p = (c.nc + SMAX - 1) / SMAX;
    c.s = c.p ? (c.nc + c.p - 1) / c.p : 0;
    if ((c.s & 1) == 0 && c.s < SMAX) {
        c.s += 1;
        c.p = (c.nc + c.s - 1) / c.s;
    }
    return c;
}

// ---------------------------------------------------------------- value types
// A right-hand side is real (V = T) or complex (V = Cx<T>); the systems are
// real, so both share the eliminations.
template <typename V> struct VTraits;
template <> struct VTraits<double> { using D = double; };
template <> struct VTraits<float> { using D = double; };
template <> struct VTraits<Cx<double>> { using D = Cx<double>; };
template <> struct VTraits<Cx<float>> { using D = Cx<double>; };

template <typename V> __device__ __forceinline__ V vcast(double x) { return (V)x; }
template <typename V> __device__ __forceinline__ V vcast(float x) { return (V)x; }
template <typename V> __device__ __forceinline__ V vcast(Cx<double> x) {
    using T = decltype(V{}.x);
    return V{(T)x.x, (T)x.y};
}
template <typename V> __device__ __forceinline__ V vcast(Cx<float> x) {
    using T = decltype(V{}.x);
    return V{(T)x.x, (T)x.y};
}
__device__ __forceinline__ double vreal(double v) { return v; }
__device__ __forceinline__ double vreal(Cx<double> v) { return v.x; }
template <typename VD> __device__ __forceinline__ VD vfrom_real(double x);
template <> __device__ __forceinline__ double vfrom_real<double>(double x) { return x; }
template <> __device__ __forceinline__ Cx<double> vfrom_real<Cx<double>>(double x) { return Cx<double>{x, 0.0}; }

// Partitioned solve of both parity classes for k != 0 (or the transposed
// systems).  Each thread owns a contiguous chunk of rows of one class: its
// first row is a separator, the others are interior rows.  A top-down
// elimination over the interior rows, with the chunk's separator S and the
// next separator S+ unknown, writes each interior row as
//   x_ii = dy_ii - S dv_ii - cp_ii x_{ii+1},
// which at the last interior row is an affine function of S and S+.
// Substituting these relations into one another from the top gives the first
// interior row the same way, in the same pass (a running product of the -cp).
// The separators then form a tridiagonal system, solved by parallel cyclic
// reduction, and one backward pass with S and S+ known rebuilds the interior
// rows: from the kept dy, dv and cp where they fit in registers (SPIKE is
// true), else by a forward and a backward substitution that recompute the
// band from the row index and keep only the right-hand sides and the
// reciprocal pivots.
//
// Every chunk of both classes has the same length s, so the row loops run a
// count that is the same for the whole workgroup.  The last chunk of a class
// is filled up with padding rows that continue the band past the class's last
// row.  That row's superdiagonal is zero, so the coupling runs from the real
// rows into the padding only: the real rows' elimination, their separator
// equations and their solution are those of the class alone, and the padding
// rows' values are finite and never stored.

// Rows per chunk (both classes) and chunks per class for classes of ncA and
// ncB rows and chunks of at most smax rows; the same on the host (thread
// counts, LDS sizes) and in the kernels.  The length is odd when possible:
// the rows of a class sit two line positions apart, so consecutive chunks
// start 2s positions apart, and an odd s spreads the threads' LDS accesses
// over the banks (at most two-way conflicts instead of up to 16-way).
struct SolveChunks {
    int s, pA, pB;
};
__host__ __device__ constexpr SolveChunks solve_chunks(int ncA, int ncB, int smax) {
    const int nc = ncA > ncB ? ncA : ncB;
    const int p = (nc + smax - 1) / smax;
    int s = p ? (nc + p - 1) / p : 0;
    if ((s & 1) == 0 && s < smax) s += 1;
    SolveChunks c{s, s ? (ncA + s - 1) / s : 0, s ? (ncB + s - 1) / s : 0};
    return c;
}

// Rows of the two classes of a k != 0 system: class A holds the even q from
// 0 (cosine) or 2 (sine), class B the odd q, up to m - 1 (cosine) or m (sine).
__host__ __device__ constexpr int class_rows(int q0, int qhi) { return qhi >= q0 ? (qhi - q0) / 2 + 1 : 0; }

// Right-hand-side slot of row ii of a thread's chunk in the "solve order"
// used for values kept between kernels: class A rows first, then class B,
// each interleaved over the chunks (consecutive threads, consecutive slots).
// A class of nc rows in p chunks of s rows (padding included) uses
// s p < nc + s <= nc + SMAX slots, so with SMAX <= 31 the slots of a line (both
// classes) stay below m + 64.
__host__ __device__ __forceinline__ int solve_slot_stride(int m) { return m + 64; }

// Whether a solve of SMAX-row chunks with right-hand sides of type V in
// precision T keeps the top-down multipliers and separator weights of every
// row: two more register arrays, at most 256 bytes per thread for all three
// (real and complex float; not double, whose chunks would spill).
template <typename T, typename V, int SMAX>
__host__ __device__ constexpr bool solve_keeps_spike() { return (int)(sizeof(V) + 2 * sizeof(T)) * SMAX <= 256; }

// fetch(slot) issues a row's global reads and returns them (NoFetch when a
// load reads only the LDS line); load(p, q, slot, own, fetched) returns the
// right-hand side of the row of coefficient
// q at line position p (q for cosine, m - q for sine) with solve-order slot
// `slot`.  For a padding row q lies past the class, p is clamped into the
// line (a valid position whose value is only a placeholder) and own is
// false, so a load that accumulates over the rows skips it; a load that also
// keeps its value writes the padding row's own slot.  store(p, x) receives
// the solution of the real rows (PAD: also the padding rows', at positions
// in the line's margins).  Every load happens before the first barrier and
// every store after the last use of the LDS scratch.
struct NoFetch {};

template <typename T, typename V, int SMAX, bool PAD = false, bool FULL = false, typename Fetch, typename Load,
          typename Store>
__device__ __forceinline__ void solve_partitioned_io(Fetch&& fetch, Load&& load, Store&& store,
                                                     unsigned char* __restrict__ scratch, int m, int k, bool sine,
                                                     bool transposed, int tid) {
    constexpr bool SPIKE = solve_keeps_spike<T, V, SMAX>();
    const int qhi = sine ? m : m - 1;
    ClassInfo A, B;
    A.q0 = sine ? 2 : 0;
    B.q0 = 1;
    A.nc = class_rows(A.q0, qhi);
    B.nc = class_rows(1, qhi);
    const SolveChunks ch = solve_chunks(A.nc, B.nc, SMAX);
    const int s = FULL ? SMAX : ch.s;            // rows per chunk, the same in every thread
    A.s = B.s = s;
    A.p = ch.pA;
    B.p = ch.pB;
    const int ptot = A.p + B.p;
    const bool inA = tid < A.p;
    const bool inB = !inA && tid < ptot;
    const ClassInfo& C = inA ? A : B;
    const int p = inA ? tid : tid - A.p;
    const int cls_lo = inA ? 0 : A.p;            // reduced-row range of this class
    const int cls_hi = inA ? A.p : ptot;
    const int lo = p * s;
    const int cnt = (inA || inB) ? min(s, C.nc - lo) : 0;   // real rows of the chunk; the rest are padding
    // row ii of the chunk: coefficient Q0 + 2 ii at line position P0 + ii dP, solve-order slot slot0 + ii C.p
    const int Q0 = C.q0 + 2 * lo;
    const int P0 = sine ? m - Q0 : Q0;
    const int dP = sine ? -2 : 2;
    const int slot0 = (inA ? 0 : s * A.p) + p;
    const int ilast = C.nc - 1 - lo;             // the class's last row as a chunk index
    const T kk = (T)k * (T)k;
    const T qT0 = (T)Q0;
    // q is carried as a running value (exact: q < 2^24) rather than converted per row
    auto rowband = [&](T qrow, int ii, bool first, T& a, T& b, T& c) {
        band_kk<T>(qrow, kk, first, ii == ilast, transposed, a, b, c);
    };

    V r[SMAX];                   // right-hand sides (SPIKE: then dy)
    T cp[SPIKE ? SMAX : 1];      // SPIKE: cp and dv of every interior row
    T dv[SPIKE ? SMAX : 1];
    T iv[SPIKE ? 1 : SMAX];      // otherwise: the reciprocal pivots
    // Branch-free within a thread: every row's global reads (fetch) are
    // issued before any row is formed (a branch per row, or a fetch next to
    // its use, waits on each row's reads in turn).  Padding rows, and rows at
    // or past s (which exist only when s < SMAX), re-read the chunk's first
    // row, with its slot (a load that also keeps its value writes the same
    // value again): their right-hand sides only need to be finite.
    // (The selects pick between the row's own value, linear in ii, and the
    // first row's, so no per-row multiply is needed; q is only used with the
    // row's position, so a padding row keeps its own.)  PAD: the line has
    // margins the padding rows may read and write (at least 2 SMAX + 2
    // entries on each side, the loads' values there finite), so a padding row
    // uses its own position and slot and rows need no selects; rows at or
    // past s still re-read the first row (a test of s, the same in every
    // thread).
    using PF = decltype(fetch(0u));
    if (cnt > 0) {
        PF pf[SMAX];
#pragma unroll
        for (int ii = 0; ii < SMAX; ++ii) {
            const int iu = ii < s ? ii : 0;
            const int sl = PAD ? slot0 + iu * C.p : (ii < cnt ? slot0 + ii * C.p : slot0);
            pf[ii] = fetch((unsigned)sl);
        }
#pragma unroll
        for (int ii = 0; ii < SMAX; ++ii) {
            const int iu = ii < s ? ii : 0;
            const bool own = ii < cnt;
            const int sl = PAD ? slot0 + iu * C.p : (own ? slot0 + ii * C.p : slot0);
            const int pos = PAD ? P0 + iu * dP : (own ? P0 + ii * dP : P0);
            r[ii] = load(pos, Q0 + 2 * ii, (unsigned)sl, own, pf[ii]);
        }
    }
    lds_barrier();   // B1: the line may now be overwritten by scratch

    // Top-down.  Last interior row: x = yL - S vL - S+ wL (with no interior
    // row the "last interior row" is the separator: yL = 0, vL = -1, wL = 0).
    // First interior row, composed along the way: x_1 = yF + S gv + x_{ii+1} g,
    // with g the product of the -cp so far; at the end x_1 = yF - S vF - S+ wF
    // (with no interior row it is the next separator: yF = 0, vF = 0, wF = -1).
    // FULL (the caller guarantees s == SMAX): no row tests.  (A second copy of
    // the loops for s == SMAX beside the tested ones made the kernels spill.)
    V yL{}, yF{};
    T vL = (T)-1, wL = (T)0, vF = (T)0, wF = (T)-1;
    if (cnt > 0) {
        T g = (T)1, gv = (T)0, qrow = qT0;
#pragma unroll
        for (int ii = 1; ii < SMAX; ++ii) {
            if (FULL || ii < s) {
                qrow += (T)2;
                T a, b, c;
                rowband(qrow, ii, false, a, b, c);
                const T inv = rcp_pivot(b - a * wL);
                wL = c * inv;
                yL = (r[ii] - yL * a) * inv;
                vL = -a * vL * inv;
                if constexpr (SPIKE) { r[ii] = yL; cp[ii] = wL; dv[ii] = vL; } else { iv[ii] = inv; }
                yF = yF + yL * g;
                gv = gv - vL * g;
                g = -wL * g;
            }
        }
        if (FULL || s > 1) { vF = -gv; wF = -g; }
    }
    // scratch: de[ptot] (V), al[ptot], be[ptot], ga[ptot] (T)
    V* de = reinterpret_cast<V*>(scratch);
    T* al = reinterpret_cast<T*>(de + ptot);
    T* be = al + ptot;
    T* ga = be + ptot;
    if (cnt > 0) { de[tid] = yL; al[tid] = vL; ga[tid] = wL; }
    lds_barrier();   // B2
    T nal = 0, nbe = 1, nga = 0;
    V nde{};
    if (cnt > 0) {
        T a0, b0, c0;
        rowband(qT0, 0, lo == 0, a0, b0, c0);
        V pyL{};
        T pvL = 0, pwL = 0;
        if (p > 0) { pyL = de[tid - 1]; pvL = al[tid - 1]; pwL = ga[tid - 1]; }
        nal = -a0 * pvL;
        nbe = b0 - a0 * pwL - c0 * vF;
        nga = -c0 * wF;
        nde = r[0] - pyL * a0 - yF * c0;
    }
    lds_barrier();   // B3
    if (cnt > 0) { al[tid] = nal; be[tid] = nbe; ga[tid] = nga; de[tid] = nde; }
    lds_barrier();   // B4
    // parallel cyclic reduction on the separators of each class
    const int pmax = max(A.p, B.p);
    for (int h = 1; h < pmax; h <<= 1) {
        T xal = nal, xbe = nbe, xga = nga;
        V xde = nde;
        if (cnt > 0) {
            const int im = tid - h, ip = tid + h;
            if (im >= cls_lo) {
                const T k1 = nal * rcp_pivot(be[im]);
                xal = -k1 * al[im];
                xbe = xbe - k1 * ga[im];
                xde = xde - de[im] * k1;
            } else {
                xal = 0;
            }
            if (ip < cls_hi) {
                const T k2 = nga * rcp_pivot(be[ip]);
                xga = -k2 * ga[ip];
                xbe = xbe - k2 * al[ip];
                xde = xde - de[ip] * k2;
            } else {
                xga = 0;
            }
        }
        lds_barrier();
        nal = xal; nbe = xbe; nga = xga; nde = xde;
        if (cnt > 0) { al[tid] = nal; be[tid] = nbe; ga[tid] = nga; de[tid] = nde; }
        lds_barrier();
    }
    const V S = nde * rcp_pivot(nbe);
    if (cnt > 0) de[tid] = S;
    lds_barrier();
    V Sn{};
    if (cnt > 0 && tid + 1 < cls_hi) Sn = de[tid + 1];
    lds_barrier();   // scratch no longer needed: write the solution
    if (cnt > 0) {
        store(P0, S);
        if constexpr (SPIKE) {
            V next = Sn;
#pragma unroll
            for (int ii = SMAX - 1; ii >= 1; --ii) {
                if (FULL || ii < s) {
                    r[ii] = r[ii] - S * dv[ii] - next * cp[ii];
                    next = r[ii];
                    if (PAD || ii < cnt) store(P0 + ii * dP, r[ii]);
                }
            }
        } else {
            // r still holds the right-hand sides: a forward substitution
            // from x_0 = S, then a backward one from S+
            V prev = S;
            T qrow = qT0;
#pragma unroll
            for (int ii = 1; ii < SMAX; ++ii) {
                if (FULL || ii < s) {
                    qrow += (T)2;
                    T a, b, c;
                    rowband(qrow, ii, false, a, b, c);
                    r[ii] = (r[ii] - prev * a) * iv[ii];
                    prev = r[ii];
                }
            }
            V next = Sn;
            qrow += (T)2;
#pragma unroll
            for (int ii = SMAX - 1; ii >= 1; --ii) {
                if (FULL || ii < s) {
                    qrow -= (T)2;
                    T a, b, c;
                    rowband(qrow, ii, false, a, b, c);
                    r[ii] = r[ii] - next * (c * iv[ii]);
                    next = r[ii];
                    if (PAD || ii < cnt) store(P0 + ii * dP, r[ii]);
                }
            }
        }
    }
}

// In place on a line held in LDS.
template <typename T, int SMAX, typename V>
__device__ __forceinline__ void solve_partitioned(V* __restrict__ buf, unsigned char* __restrict__ scratch,
                                                  int m, int k, bool sine, bool transposed, int tid) {
    solve_partitioned_io<T, V, SMAX>([](unsigned) { return NoFetch{}; },
                                     [&](int p, int, unsigned, bool, NoFetch) { return buf[p]; },
                                     [&](int p, V x) { buf[p] = x; }, scratch, m, k, sine, transposed, tid);
}

// Block-wide sum of one complex double per thread (result valid in every thread).
__device__ __forceinline__ Cx<double> block_sum(Cx<double> v, Cx<double>* red) {
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_down(v.x, off, 64);
        v.y += __shfl_down(v.y, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    lds_barrier();
    Cx<double> s{0.0, 0.0};
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s = s + red[w];
    lds_barrier();
    return s;
}
__device__ __forceinline__ double block_sum(double v, Cx<double>* red) {
    return block_sum(Cx<double>{v, 0.0}, red).x;
}

// k = 0: the two cosine classes (odd q, and even q >= 2) are solved with LU
// factors precomputed on the host in extended precision (the k = 0 systems
// are only weakly diagonally dominant), as two first-order recurrences each
// evaluated by a chunked scan of affine maps:
//   T x = r:   z_i = (r_i - sub_i z_{i-1}) inv_i,     x_i = z_i - cp_i x_{i+1}
//   T^T x = r: z_i = r_i - cp_{i-1} z_{i-1},           x_i = (z_i - sub_{i+1} x_{i+1}) inv_i
// a_0 then follows from the constraint (transposed: the constraint row feeds
// the even class and the q = 0 output is zero).  Always float64.
template <typename VD, int SMAX>
__device__ __forceinline__ void scan_affine(VD& A, double& Bm, unsigned char* scratch, int tid,
                                            int cls_lo, int cls_hi, int ptot, bool reverse, bool valid) {
    // inclusive scan of maps f_p(z) = A_p + B_p z over the chunks of a class
    // (forward: f_p applied after f_{p-1}; reverse: after f_{p+1}).
    VD* sa = reinterpret_cast<VD*>(scratch);
    double* sb = reinterpret_cast<double*>(sa + ptot);
    if (valid) { sa[tid] = A; sb[tid] = Bm; }
    lds_barrier();
    const int pmax = ptot;   // upper bound on class length
    for (int h = 1; h < pmax; h <<= 1) {
        VD nA = A;
        double nB = Bm;
        if (valid) {
            const int o = reverse ? tid + h : tid - h;
            if (reverse ? (o < cls_hi) : (o >= cls_lo)) {
                // compose: (this after other): A + B * A_o, B * B_o
                nA = A + sa[o] * Bm;
                nB = Bm * sb[o];
            }
        }
        lds_barrier();
        A = nA; Bm = nB;
        if (valid) { sa[tid] = A; sb[tid] = Bm; }
        lds_barrier();
    }
}

// load(q) returns the right-hand side of row q (position q of the cosine
// line; q = 0 is the constraint row, read only for the transposed system);
// store(q, x) receives the solution, q = 0 included.  Every load happens
// before the first barrier and every store after the last use of the LDS
// scratch.  V is real or complex.
template <typename T, int SMAX, typename V, typename Load, typename Store>
__device__ __forceinline__ void solve_k0_io(Load&& load, Store&& store, unsigned char* __restrict__ scratch,
                                            int m, bool transposed, double c0, const double* __restrict__ tab,
                                            Cx<double>* red, int tid) {
    using VD = typename VTraits<V>::D;
    const int qhi = m - 1;
    const ClassInfo A = make_class<SMAX>(2, qhi);   // even q >= 2
    const ClassInfo B = make_class<SMAX>(1, qhi);   // odd q
    const int ptot = A.p + B.p;
    const bool inA = tid < A.p;
    const bool inB = !inA && tid < ptot;
    const ClassInfo& C = inA ? A : B;
    const int p = inA ? tid : tid - A.p;
    const int cls_lo = inA ? 0 : A.p;
    const int cls_hi = inA ? A.p : ptot;
    const int lo = p * C.s;
    const int cnt = (inA || inB) ? min(C.s, C.nc - lo) : 0;
    const double* inv = tab + (inA ? 0 : 2 * A.nc);
    const double* cp = inv + C.nc;
    const VD a0bar = transposed ? vcast<VD>(load(0)) : VD{};

    VD r[SMAX];
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int q = C.q0 + 2 * (lo + ii);
            r[ii] = vcast<VD>(load(q));
            if (transposed && inA) {
                const double om = 1.0 / (1.0 - (double)q * (double)q);
                r[ii] = r[ii] - a0bar * om;
            }
        }
    }
    lds_barrier();
    auto sub_of = [&](int row) -> double {   // sub-diagonal of row `row` of the class
        if (row <= 0) return 0.0;
        const double q = (double)(C.q0 + 2 * row);
        return (q - 2.0) * (q - 1.0) * 0.25;
    };
    // forward recurrence z_i = alpha_i + beta_i z_{i-1}
    VD Af{};
    double Bf = 1.0;
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int row = lo + ii;
            VD al;
            double be;
            if (!transposed) { al = r[ii] * inv[row]; be = -sub_of(row) * inv[row]; }
            else { al = r[ii]; be = row > 0 ? -cp[row - 1] : 0.0; }
            Af = al + Af * be;
            Bf = be * Bf;
        }
    }
    scan_affine<VD, SMAX>(Af, Bf, scratch, tid, cls_lo, cls_hi, ptot, false, cnt > 0);
    // value entering this chunk = inclusive result of the previous chunk applied to 0
    VD* sa = reinterpret_cast<VD*>(scratch);
    VD zin{};
    if (cnt > 0 && tid - 1 >= cls_lo) zin = sa[tid - 1];
    lds_barrier();
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int row = lo + ii;
            VD al;
            double be;
            if (!transposed) { al = r[ii] * inv[row]; be = -sub_of(row) * inv[row]; }
            else { al = r[ii]; be = row > 0 ? -cp[row - 1] : 0.0; }
            zin = al + zin * be;
            r[ii] = zin;
        }
    }
    // backward recurrence x_i = gamma_i + delta_i x_{i+1}
    VD Ab{};
    double Bb = 1.0;
#pragma unroll
    for (int ii = SMAX - 1; ii >= 0; --ii) {
        if (ii < cnt) {
            const int row = lo + ii;
            VD ga;
            double de;
            if (!transposed) { ga = r[ii]; de = -cp[row]; }
            else { ga = r[ii] * inv[row]; de = row + 1 < C.nc ? -sub_of(row + 1) * inv[row] : 0.0; }
            Ab = ga + Ab * de;
            Bb = de * Bb;
        }
    }
    scan_affine<VD, SMAX>(Ab, Bb, scratch, tid, cls_lo, cls_hi, ptot, true, cnt > 0);
    VD xin{};
    if (cnt > 0 && tid + 1 < cls_hi) xin = sa[tid + 1];
    lds_barrier();
    VD part{};
#pragma unroll
    for (int ii = SMAX - 1; ii >= 0; --ii) {
        if (ii < cnt) {
            const int row = lo + ii;
            VD ga;
            double de;
            if (!transposed) { ga = r[ii]; de = -cp[row]; }
            else { ga = r[ii] * inv[row]; de = row + 1 < C.nc ? -sub_of(row + 1) * inv[row] : 0.0; }
            xin = ga + xin * de;
            r[ii] = xin;
            if (inA && !transposed) {
                const double q = (double)(C.q0 + 2 * row);
                part = part + xin * (1.0 / (1.0 - q * q));
            }
        }
    }
    const VD dot = block_sum(part, red);
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int q = C.q0 + 2 * (lo + ii);
            store(q, r[ii]);
        }
    }
    if (tid == 0) store(0, transposed ? VD{} : vfrom_real<VD>(c0) - dot);
}

// In place on a line held in LDS (position order).
template <typename T, int SMAX, typename V>
__device__ __forceinline__ void solve_k0(V* __restrict__ buf, unsigned char* __restrict__ scratch, int m,
                                         bool transposed, double c0, const double* __restrict__ tab,
                                         Cx<double>* red, int tid) {
    using VD = typename VTraits<V>::D;
    solve_k0_io<T, SMAX, V>([&](int q) { return buf[q]; }, [&](int q, VD x) { buf[q] = vcast<V>(x); }, scratch, m,
                            transposed, c0, tab, red, tid);
}

// Division of a column by sin(theta) in coefficient space (the paper's
// M_sin^{-1}, Section 4 eq. Msin, on the cosine / sine series of one
// wavenumber instead of the doubled Fourier series).  With true coefficients
// g_p in position order:
//   even k, g a cosine series: h = g / sin(theta) is the sine series with
//     c_{p+1} = 2 sum_{p' <= p, p' = p mod 2} g_p'   (from g_p = (c_{p+1} - c_{p-1}) / 2, g_0 = c_1 / 2),
//     written at position m - (p + 1);
//   odd k, g a sine series (g_p at position m - p, p = 1..m): h is the cosine series with
//     d_{p-1} = 2 sum_{p' >= p, p' = p mod 2} g_p'   (from g_p = (d_{p-1} - d_{p+1}) / 2, g_1 = d_0 - d_2 / 2),
//     halved for d_0, written at position p - 1.
// These are cumulative sums along each parity class: every thread takes a
// chunk of up to HOLD consecutive coefficients of one class, and the chunk
// sums are scanned across the class (scan_affine, forward for even k,
// backward for odd k).  The result is exact when g vanishes at both poles
// (every wavenumber k >= 1 of a function on the sphere); the k = 0 column is
// not divisible and its output is not used.  The column is then synthesised
// with the other parity.  Uses the LDS from scratch (the line is read into
// registers first).  2 ceil(ceil(m/2) / HOLD) <= blockDim.x.
template <typename V, int HOLD>
__device__ __forceinline__ void theta_divide_sin_line(V* y, unsigned char* scratch, int m, bool sine, int tid) {
    using VD = typename VTraits<V>::D;
    // coefficient range of the input: 0..m-1 (cosine) or 1..m (sine); classes by parity of p
    const int plo = sine ? 1 : 0, phi = sine ? m : m - 1;
    const int nE = (phi - (plo + (plo & 1)) ) / 2 + 1;                        // even p in [plo, phi]
    const int firstO = plo | 1;
    const int nO = phi >= firstO ? (phi - firstO) / 2 + 1 : 0;                // odd p
    const int pE = (nE + HOLD - 1) / HOLD, pO = (nO + HOLD - 1) / HOLD;
    const int ptot = pE + pO;
    const bool inE = tid < pE, inO = !inE && tid < ptot;
    const int c = inE ? tid : tid - pE;
    const int ncls = inE ? nE : nO;
    const int first = inE ? (plo + (plo & 1)) : firstO;   // first p of the class
    const int lo = c * HOLD;
    const int cnt = (inE || inO) ? min(HOLD, ncls - lo) : 0;
    auto pos_in = [&](int p) { return sine ? m - p : p; };
    V r[HOLD];
    VD sum{};
#pragma unroll
    for (int ii = 0; ii < HOLD; ++ii) {
        if (ii < cnt) {
            r[ii] = y[pos_in(first + 2 * (lo + ii))];
            sum = sum + vcast<VD>(r[ii]);
        }
    }
    __syncthreads();   // the line is in registers; the LDS becomes scan scratch
    double B = 1.0;
    const int cls_lo = inE ? 0 : pE, cls_hi = inE ? pE : ptot;
    scan_affine<VD, HOLD>(sum, B, scratch, tid, cls_lo, cls_hi, ptot, sine, cnt > 0);
    VD* sa = reinterpret_cast<VD*>(scratch);
    VD run{};
    if (cnt > 0) {
        const int o = sine ? tid + 1 : tid - 1;   // the neighbouring chunk already summed
        if (sine ? (o < cls_hi) : (o >= cls_lo)) run = sa[o];
    }
    __syncthreads();   // scratch read; the line is written below
    if (cnt > 0) {
        if (!sine) {
#pragma unroll
            for (int ii = 0; ii < HOLD; ++ii) {
                if (ii < cnt) {
                    const int p = first + 2 * (lo + ii);
                    run = run + vcast<VD>(r[ii]);
                    y[m - (p + 1)] = vcast<V>(run * 2.0);
                }
            }
        } else {
#pragma unroll
            for (int ii = HOLD - 1; ii >= 0; --ii) {
                if (ii < cnt) {
                    const int p = first + 2 * (lo + ii);
                    run = run + vcast<VD>(r[ii]);
                    y[p - 1] = vcast<V>(run * (p == 1 ? 1.0 : 2.0));
                }
            }
        }
    }
    __syncthreads();
}

template <typename T, int EPT, int RMAX, int SMAX>
__device__ __forceinline__ void theta_body(const ThetaArgs<T>& a, int k, unsigned char* smem_raw,
                                           Cx<double>* red) {
    Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
    const int m = a.m, N = a.N, lay = a.lay_log2, lay_out = a.lay_out_log2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool sine = (k & 1) != 0;
    const T invm = (T)1 / (T)m;

    double fpart = 0.0;
    for (int j = tid; j < m; j += nthr) {
        const size_t idx = spec_at(j, k, N, lay);
        Cx<T> x = a.spec[idx];
        if (sine && (j & 1)) x = Cx<T>{-x.x, -x.y};
        const int pos = (j & 1) ? m - ((j + 1) >> 1) : (j >> 1);
        buf[pos] = x;
        if (k == 0 && a.fint_w) fpart += a.fint_w[j] * (double)x.x;
    }
    if (k == 0 && a.fint_w) {
        const Cx<double> s = block_sum(Cx<double>{fpart, 0.0}, red);
        if (tid == 0) *a.fint_out = s.x;
    }
    __syncthreads();
    fft_lds<T, false, EPT, RMAX>(buf, 0, a.fft, a.tw, tid, a.nthr_fft, tid < a.nthr_fft);
    const bool scale = a.mode == kSolve || a.mode == kDerivative || a.mode == kDivideSin;
    for (int q = tid; q <= m / 2; q += nthr) {
        const int qq = q == 0 ? 0 : m - q;
        const Cx<T> A = buf[q], B = buf[qq];
        const Cx<T> Eq = a.eq[q];
        Cx<T> yq = (cmul(Eq, A) + cmulc(B, Eq)) * (T)0.5;
        if (scale) yq = yq * (q == 0 ? invm : (T)2 * invm);
        if (qq != q) {
            const Cx<T> Eqq = a.eq[qq];
            Cx<T> yqq = (cmul(Eqq, B) + cmulc(A, Eqq)) * (T)0.5;
            if (scale) yqq = yqq * ((T)2 * invm);
            buf[qq] = yqq;
        }
        buf[q] = yq;
    }
    __syncthreads();
    if (a.mode == kDerivative) {
        theta_derivative_line<Cx<T>, kThetaHold>(buf, m, sine, tid, nthr);
    } else if (a.mode == kDivideSin) {
        theta_divide_sin_line<Cx<T>, kThetaHold>(buf, smem_raw, m, sine, tid);
    } else if (a.mode != kTransformOnly) {
        unsigned char* scratch = smem_raw;
        if (k == 0) solve_k0<T, SMAX>(buf, scratch, m, a.mode == kSolveTransposed, a.c0, a.k0tab, red, tid);
        else solve_partitioned<T, SMAX>(buf, scratch, m, k, sine, a.mode == kSolveTransposed, tid);
    }
    __syncthreads();
    const bool sine_out = (a.mode == kDerivative || a.mode == kDivideSin) ? !sine : sine;
    for (int q = tid; q <= m / 2; q += nthr) {
        const int qq = q == 0 ? 0 : m - q;
        Cx<T> yq = buf[q], yqq = buf[qq];
        if (scale) {
            yq = yq * (q == 0 ? (T)m : (T)m * (T)0.5);
            yqq = yqq * ((T)m * (T)0.5);
        }
        if (q == 0) {
            buf[0] = yq;
        } else {
            const Cx<T> Eq = a.eq[q];
            buf[q] = cmulc(yq - mul_i(yqq), Eq);
            if (qq != q) {
                const Cx<T> Eqq = a.eq[qq];
                buf[qq] = cmulc(yqq - mul_i(yq), Eqq);
            }
        }
    }
    __syncthreads();
    fft_lds<T, true, EPT, RMAX>(buf, 0, a.fft, a.tw, tid, a.nthr_fft, tid < a.nthr_fft);
    for (int j = tid; j < m; j += nthr) {
        const size_t idx = spec_at(j, k, N, lay_out);
        const int pos = (j & 1) ? m - ((j + 1) >> 1) : (j >> 1);
        Cx<T> x = buf[pos] * invm;
        if (sine_out && (j & 1)) x = Cx<T>{-x.x, -x.y};
        a.spec_out[idx] = x;
    }
}

// Wavenumbers to workgroups, XCD-aware: consecutive workgroup ids go round-robin
// over the 8 XCDs, so slice x of the k range is given to XCD x.
__device__ __forceinline__ int theta_k_of_block(int k8) {
    return (blockIdx.x & 7) * k8 + (blockIdx.x >> 3);
}

template <typename T, int EPT, int RMAX, int SMAX>
__global__ void __launch_bounds__(1024) k_theta(ThetaArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Cx<double> red[16];
    const int k = theta_k_of_block(a.k8);
    if (k > a.N) return;
    theta_body<T, EPT, RMAX, SMAX>(a, k, smem_raw, red);
}

// ---------------------------------------------------------------- mixed theta pass
// Float32 bulk solve with float64 right-hand side / residual (iterative
// refinement).  Wavenumbers k < k64 (always including k = 0) are eliminated in
// float64: their systems are too ill-conditioned for float32 corrections.  RESID = false (first solve):
//   load the float64 spectrum of sin^2 b, float64 cosine/sine analysis -> F
//   (true coefficients, position order), store F in place of the input,
//   solve (L - k^2) a = F in float32 (k = 0: float64 with the constraint),
//   float32 synthesis -> float32 spectrum s0.
// RESID = true (correction):
//   load the float64 spectrum of the current iterate, float64 analysis -> X,
//   r = F - (L - k^2) X in float64 (k = 0: constraint row r_0 = c0 - (X_0 +
//   sum_{q>=2 even} X_q/(1 - q^2))), solve for the correction in float32
//   (k = 0 float64), float32 synthesis -> float32 spectrum sd.

struct ThetaMixArgs {
    const Cx<double>* sa;      // float64 spectrum of sin^2 b (first solve)
    Cx<double>* fco;           // F per wavenumber, stride solve_slot_stride(m): written by the first solve
    const Cx<double>* su;      // RESID: float64 spectrum of the current iterate
    Cx<float>* out;            // float32 spectrum written (s0 or sd)
    const Cx<double>* tw64;    // per-pass twiddles of the length-m DFT
    const Cx<double>* eq64;
    const Cx<float>* tw32;
    const Cx<float>* eq32;
    const Cx<double>* ws64;    // real-part pass: e^{-2 pi i q/m}, q = 0..m/4
    const Cx<float>* ws32;
    int n, m, N;
    int lay_log2;              // run length (log2) of sa / su
    int lay_out_log2;          // run length (log2) of out
    FftDesc fft;
    int nthr_fft;
    int k8;
    double c0;                 // integral / (4 pi)
    const double* k0tab;
    const double* fint_w;
    double* fint_out;
    int k64;                   // wavenumbers below this are eliminated in float64
    double* rnorm;             // RESID in the NORM builds: per tile (k on the complex line, 2k + part
                               // for real parts) the sums of r^2 and F^2 over its rows
};

// k = 0 of the mixed theta pass: the bordered constraint system, always in
// float64.  F is kept in position order.  RESID: r = F - (L) X with the
// constraint row r_0 = c0 - (X_0 + sum_{q>=2 even} X_q/(1 - q^2)); TRANS:
// the transposed bordered system (the constraint row feeds the even class
// through -w b_0 and the q = 0 entry of the solution is pinned to zero, so the
// correction there is minus the q = 0 coefficient of the current iterate).
// On return the float32 column buff holds the solution.
template <int SMAXD, bool RESID, bool TRANS>
__device__ __forceinline__ void theta_mixed_k0(const ThetaMixArgs& a, Cx<double>* bufd, Cx<float>* buff,
                                               Cx<double>* F, unsigned char* smem_raw, Cx<double>* red, int tid,
                                               double& acc_r, double& acc_f) {
    const int m = a.m, nthr = blockDim.x;
    Cx<double> rh[kThetaHold];
    double r0 = a.c0;
    Cx<double> x0_pin{0.0, 0.0};
    const int qhi = m - 1;
    if (!RESID) {
#pragma unroll
        for (int e = 0; e < kThetaHold; ++e) {
            const int p = tid + e * nthr;
            if (p < m) {
                rh[e] = bufd[p];
                F[p] = rh[e];
            }
        }
    } else {
        Cx<double> part{0.0, 0.0};
        // transposed: the even class starts at q = 2 (no coupling to q = 0), and its
        // right-hand side is B_q - w_q B_0 with w_q = 1/(1 - q^2)
        const Cx<double> b0 = TRANS ? F[0] : Cx<double>{0.0, 0.0};
#pragma unroll
        for (int e = 0; e < kThetaHold; ++e) {
            const int q = tid + e * nthr;
            if (q < m) {
                if (q == 0) {
                    rh[e] = Cx<double>{0.0, 0.0};
                    continue;
                }
                const int lo_q = (TRANS && (q & 1) == 0) ? 2 : 0;
                double sub, diag, sup;
                band<double>(q, 0, q - 2 < lo_q, q + 2 > qhi, TRANS, sub, diag, sup);
                Cx<double> ax = bufd[q] * diag;
                if (q - 2 >= lo_q) ax = ax + bufd[q - 2] * sub;
                if (q + 2 <= qhi) ax = ax + bufd[q + 2] * sup;
                Cx<double> rhs = F[q];
                if (TRANS && (q & 1) == 0) rhs = rhs - b0 * (1.0 / (1.0 - (double)q * (double)q));
                rh[e] = rhs - ax;
                if (!TRANS && (q & 1) == 0) part = part + bufd[q] * (1.0 / (1.0 - (double)q * (double)q));
                acc_r += rh[e].x * rh[e].x + rh[e].y * rh[e].y;
                acc_f += rhs.x * rhs.x + rhs.y * rhs.y;
            }
        }
        if (!TRANS) {
            const Cx<double> dot = block_sum(part, red);
            const Cx<double> x0 = bufd[0];
            r0 = a.c0 - (x0.x + dot.x);   // the imaginary part of the k = 0 column is zero
            if (tid == 0) {
                acc_r += r0 * r0;
                acc_f += a.c0 * a.c0;
            }
        }
        if (TRANS) x0_pin = bufd[0];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kThetaHold; ++e) {
        const int p = tid + e * nthr;
        if (p < m) bufd[p] = rh[e];
    }
    __syncthreads();
    solve_k0<double, SMAXD>(bufd, smem_raw, m, TRANS, r0, a.k0tab, red, tid);
    __syncthreads();
    if (TRANS && RESID && tid == 0) bufd[0] = Cx<double>{-x0_pin.x, -x0_pin.y};
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kThetaHold; ++e) {
        const int p = tid + e * nthr;
        if (p < m) rh[e] = bufd[p];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kThetaHold; ++e) {
        const int p = tid + e * nthr;
        if (p < m) buff[p] = Cx<float>{(float)rh[e].x, (float)rh[e].y};
    }
    __syncthreads();
}

// TRANS = true runs the same refinement for the transposed systems (the
// adjoint): no coefficient scaling around the solve (the transpose of
// "analysis with scaling" is the plain synthesis), transposed bands, and for
// k = 0 the transposed bordered system (the constraint row feeds the even
// class through -w a_0 and the q = 0 output is zero).
template <int EPT, int RMAX, int SMAXF, int SMAXD, bool RESID, bool TRANS, bool NORM = false>
__device__ __forceinline__ void theta_mixed_body(const ThetaMixArgs& a, int k, unsigned char* smem_raw,
                                                 Cx<double>* red) {
    Cx<double>* bufd = reinterpret_cast<Cx<double>*>(smem_raw);
    Cx<float>* buff = reinterpret_cast<Cx<float>*>(smem_raw);
    const int m = a.m, N = a.N, lay = a.lay_log2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool sine = (k & 1) != 0;
    const double invm = 1.0 / (double)m;
    auto idx = [&](int j) -> size_t {
        return spec_at(j, k, N, lay);
    };
    auto posj = [&](int j) -> int { return (j & 1) ? m - ((j + 1) >> 1) : (j >> 1); };

    // float64 analysis of the input column
    const Cx<double>* src = RESID ? a.su : a.sa;
    double fpart = 0.0;
    for (int j = tid; j < m; j += nthr) {
        Cx<double> x = src[idx(j)];
        if (sine && (j & 1)) x = Cx<double>{-x.x, -x.y};
        bufd[posj(j)] = x;
        if (!RESID && k == 0 && a.fint_w) fpart += a.fint_w[j] * x.x;
    }
    if (!RESID && k == 0 && a.fint_w) {
        const Cx<double> sm = block_sum(Cx<double>{fpart, 0.0}, red);
        if (tid == 0) *a.fint_out = sm.x;
    }
    __syncthreads();
    fft_lds<double, false, EPT, RMAX>(bufd, 0, a.fft, a.tw64, tid, a.nthr_fft, tid < a.nthr_fft);
    for (int q = tid; q <= m / 2; q += nthr) {
        const int qq = q == 0 ? 0 : m - q;
        const Cx<double> A = bufd[q], B = bufd[qq];
        const Cx<double> Eq = a.eq64[q];
        const double s0 = TRANS ? 0.5 : 0.5 * (q == 0 ? invm : 2.0 * invm);
        const Cx<double> yq = (cmul(Eq, A) + cmulc(B, Eq)) * s0;
        if (qq != q) {
            const Cx<double> Eqq = a.eq64[qq];
            bufd[qq] = (cmul(Eqq, B) + cmulc(A, Eqq)) * (TRANS ? 0.5 : invm);
        }
        bufd[q] = yq;
    }
    __syncthreads();

    const int qlo = sine ? 1 : 0, qhi = sine ? m : m - 1;
    Cx<double>* Fk = a.fco + (size_t)k * solve_slot_stride(m);
    // NORM (correction pass only): the residual sums for the info, in a build of its own so
    // that the plain pass carries no extra registers
    constexpr bool want_norm = RESID && NORM;
    double acc_r = 0.0, acc_f = 0.0;
    if (k != 0) {
        // The right-hand side of each row is formed as the solve loads it:
        // first solve, F itself (also kept, in solve order, for the
        // correction); correction, r = F - (L - k^2) X in float64 from the
        // analysed iterate X in LDS.  The solution goes straight to the
        // float32 column used by the synthesis.
        // The neighbours are read unconditionally (positions clamped into the
        // line; a missing neighbour's band entry is zero), so the reads of a
        // row do not wait on one another.
        // correction: F of the row, read from HBM ahead of the rows' LDS work
        auto fetch = [&](unsigned slot) -> Cx<double> { return RESID ? Fk[slot] : Cx<double>{}; };
        auto load = [&](int p, int q, unsigned slot, bool own, Cx<double> f) -> Cx<double> {
            if (!RESID) {
                f = bufd[p];
                Fk[slot] = f;
                return f;
            }
            double sub, diag, sup;
            band<double>(q, k, q - 2 < qlo, q + 2 > qhi, TRANS, sub, diag, sup);
            const Cx<double> ylo = bufd[max(p - 2, 0)], yhi = bufd[min(p + 2, m - 1)];
            const Cx<double> ax = bufd[p] * diag + ylo * (sine ? sup : sub) + yhi * (sine ? sub : sup);
            const Cx<double> r = f - ax;
            if (want_norm && own) {
                acc_r += r.x * r.x + r.y * r.y;
                acc_f += f.x * f.x + f.y * f.y;
            }
            return r;
        };
        if (k < a.k64) {   // ill-conditioned low wavenumbers: float64 elimination
            solve_partitioned_io<double, Cx<double>, SMAXD>(
                fetch, load, [&](int p, Cx<double> x) { buff[p] = Cx<float>{(float)x.x, (float)x.y}; }, smem_raw, m,
                k, sine, TRANS, tid);
        } else {
            solve_partitioned_io<float, Cx<float>, SMAXF>(
                fetch,
                [&](int p, int q, unsigned slot, bool own, Cx<double> f) {
                    const Cx<double> r = load(p, q, slot, own, f);
                    return Cx<float>{(float)r.x, (float)r.y};
                },
                [&](int p, Cx<float> x) { buff[p] = x; }, smem_raw, m, k, sine, TRANS, tid);
        }
        __syncthreads();
    } else {
        theta_mixed_k0<SMAXD, RESID, TRANS>(a, bufd, buff, Fk, smem_raw, red, tid, acc_r, acc_f);
    }
    if (want_norm) {
        const Cx<double> sm = block_sum(Cx<double>{acc_r, acc_f}, red);
        if (tid == 0) {
            a.rnorm[2 * k] = sm.x;
            a.rnorm[2 * k + 1] = sm.y;
        }
    }
    // float32 synthesis
    const float fm = (float)m;
    for (int q = tid; q <= m / 2; q += nthr) {
        const int qq = q == 0 ? 0 : m - q;
        const Cx<float> yq = buff[q] * (TRANS ? 1.0f : (q == 0 ? fm : fm * 0.5f));
        const Cx<float> yqq = buff[qq] * (TRANS ? 1.0f : fm * 0.5f);
        if (q == 0) {
            buff[0] = yq;
        } else {
            buff[q] = cmulc(yq - mul_i(yqq), a.eq32[q]);
            if (qq != q) buff[qq] = cmulc(yqq - mul_i(yq), a.eq32[qq]);
        }
    }
    __syncthreads();
    fft_lds<float, true, EPT, RMAX>(buff, 0, a.fft, a.tw32, tid, a.nthr_fft, tid < a.nthr_fft);
    const float finvm = 1.0f / fm;
    for (int j = tid; j < m; j += nthr) {
        Cx<float> x = buff[posj(j)] * finvm;
        if (sine && (j & 1)) x = Cx<float>{-x.x, -x.y};
        a.out[spec_at(j, k, N, a.lay_out_log2)] = x;
    }
}

template <int EPT, int RMAX, int SMAXF, int SMAXD, bool RESID, bool TRANS, bool NORM = false>
__global__ void __launch_bounds__(1024) k_theta_mixed(ThetaMixArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Cx<double> red[16];
    const int k = theta_k_of_block(a.k8);
    if (k > a.N) return;
    theta_mixed_body<EPT, RMAX, SMAXF, SMAXD, RESID, TRANS, NORM>(a, k, smem_raw, red);
}

}  // namespace sp
