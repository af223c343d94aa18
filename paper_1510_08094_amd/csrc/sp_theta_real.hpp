// Theta pass on ONE real part (Re or Im) of one wavenumber's column, for even m.
//
// The banded systems of Section 5 are real, so the real and imaginary parts
// of a column X_k(theta_j) are transformed and solved independently.  A
// workgroup owns one (k, part) pair: its line is m real values (8m bytes in
// float64), half of a complex column, so two workgroups share a compute unit
// and one's memory traffic overlaps the other's arithmetic.
//
// Cosine transform of a real line x (DCT-II, Makhoul's reordering): v = x
// permuted (even samples ascending, odd samples descending), V = DFT_m(v),
// y_q = Re(E_q V_q) with E_q = e^{-i pi q/(2m)}.  The real DFT_m goes through a
// complex DFT of length M = m/2 of z_p = v_2p + i v_2p+1:
//   E = (Z_q + conj Z_{M-q})/2,  O = -i (Z_q - conj Z_{M-q})/2,  w = e^{-2 pi i q/m}
//   V_q = E + w O,  V_{M-q} = conj(E - w O)
// and, as E_{m-q} = -i conj(E_q), y_{m-q} = -Im(E_q V_q).  One pair (q, M-q)
// of Z gives the four coefficients q, m-q, M-q, M+q.  The inverse runs the
// same relations backwards: V_q = conj(E_q)(y_q - i y_{m-q}),
//   Z_q = (V_q + conj V_{M-q}) + i conj(w) (V_q - conj V_{M-q}),
// z = IDFT_M(Z) (unnormalised) holds m times v.  The sine case (odd k) is the
// cosine transform of (-1)^j x_j read backwards, as in the complex kernels.
// Line positions: coefficient q sits at position q (cosine) or m - q (sine).
#pragma once
#include "sp_kernels.hpp"

namespace sp {

constexpr int kRealPairHold = 8;    // coefficient pairs per thread in the split steps
// LDS before and after the line of a real-part pass: 64 float64 entries on
// each side, zero on the solve's loads.  A row's residual reads both band
// neighbours without testing for the ends of the line, and the padding rows
// of a class's last chunk (at most 2 SMAX + 2 entries past the line, SMAX <=
// 31) read, and write their solution, in the margins.
constexpr int kRealLineMarginEntries = 64;
constexpr int kRealLineMargin = kRealLineMarginEntries * 8;

constexpr int kRealLoadHold = 24;   // line values per thread (at least m / threads) in the k = 0 steps

// Threads of a real-part workgroup must cover the split pairs and the loads.
__host__ __device__ __forceinline__ int real_theta_min_threads(int m) {
    const int pairs = (m >> 2) + 1;
    const int a = (pairs + kRealPairHold - 1) / kRealPairHold;
    const int b = (m + kRealLoadHold - 1) / kRealLoadHold;
    return a > b ? a : b;
}

// z (M complex, after the forward DFT) -> y (m reals, position order), in
// place; coefficient q times s0 (q = 0) or s1 (q > 0).
template <typename T>
__device__ __forceinline__ void rdct_split_forward(Cx<T>* z, const Cx<T>* __restrict__ eq,
                                                   const Cx<T>* __restrict__ ws, int m, T s0, T s1, int tid,
                                                   int nthr) {
    T* y = reinterpret_cast<T*>(z);
    const int M = m >> 1, P = (M >> 1) + 1;
    T o[kRealPairHold][4];
#pragma unroll
    for (int e = 0; e < kRealPairHold; ++e) {
        const int q = tid + e * nthr;
        if (q < P) {
            const int qq = q == 0 ? 0 : M - q;   // Z_M = Z_0
            const Cx<T> Zq = z[q], Zqq = z[qq];
            const Cx<T> Ev = (Zq + cconj(Zqq)) * (T)0.5;
            const Cx<T> wO = cmul(ws[q], mul_negi(Zq - cconj(Zqq)) * (T)0.5);
            const Cx<T> Wq = cmul(eq[q], Ev + wO);
            const Cx<T> Wqq = cmul(eq[M - q], cconj(Ev - wO));
            o[e][0] = Wq.x;
            o[e][1] = -Wq.y;
            o[e][2] = Wqq.x;
            o[e][3] = -Wqq.y;
        }
    }
    lds_barrier();
#pragma unroll
    for (int e = 0; e < kRealPairHold; ++e) {
        const int q = tid + e * nthr;
        if (q < P) {
            y[q] = o[e][0] * (q == 0 ? s0 : s1);
            if (q != 0) y[m - q] = o[e][1] * s1;
            if (M - q != q) {
                y[M - q] = o[e][2] * s1;
                if (q != 0) y[M + q] = o[e][3] * s1;
            }
        }
    }
    lds_barrier();
}

// y (m reals, position order; coefficient q times s0 / s1) -> Z (M complex), in place.
template <typename T>
__device__ __forceinline__ void rdct_split_inverse(T* y, const Cx<T>* __restrict__ eq,
                                                   const Cx<T>* __restrict__ ws, int m, T s0, T s1, int tid,
                                                   int nthr) {
    Cx<T>* z = reinterpret_cast<Cx<T>*>(y);
    const int M = m >> 1, P = (M >> 1) + 1;
    Cx<T> o[kRealPairHold][2];
#pragma unroll
    for (int e = 0; e < kRealPairHold; ++e) {
        const int q = tid + e * nthr;
        if (q < P) {
            const T yq = y[q] * (q == 0 ? s0 : s1);
            const T ymq = q == 0 ? (T)0 : y[m - q] * s1;
            const T yMq = y[M - q] * s1;
            const T yMpq = y[M + q] * s1;
            const Cx<T> Vq = cmulc(Cx<T>{yq, -ymq}, eq[q]);
            const Cx<T> Vqq = cmulc(Cx<T>{yMq, -yMpq}, eq[M - q]);
            const Cx<T> Pp = Vq + cconj(Vqq);
            const Cx<T> iwQ = mul_i(cmulc(Vq - cconj(Vqq), ws[q]));
            o[e][0] = Pp + iwQ;
            o[e][1] = cconj(Pp - iwQ);
        }
    }
    lds_barrier();
#pragma unroll
    for (int e = 0; e < kRealPairHold; ++e) {
        const int q = tid + e * nthr;
        if (q < P) {
            z[q] = o[e][0];
            if (q != 0 && M - q != q) z[M - q] = o[e][1];
        }
    }
    lds_barrier();
}

__device__ __forceinline__ int line_pos(int j, int m) { return (j & 1) ? m - ((j + 1) >> 1) : (j >> 1); }

// Load one part of column k (times the sine signs) into the line in Makhoul
// order; all loads of a thread are issued before the first LDS store.  The
// block size is a multiple of 64 and of the run length, so the rows
// j = tid + e nthr of a thread share j mod 2^lay and the parity of j: the
// spectrum index and the line position advance by fixed strides.
template <typename T, typename TS>
__device__ __forceinline__ double load_part(T* y, const Cx<TS>* __restrict__ spec, int part, int k, int m,
                                            int N, int lay, bool sine, const double* __restrict__ fint_w,
                                            int tid, int nthr) {
    constexpr int kBatch = 8;   // loads in flight per thread (24, all of them at m = 10^4, measured slower)
    const TS* sp = reinterpret_cast<const TS*>(spec) + part + 2 * spec_at(tid, k, N, lay);
    const size_t dj = (size_t)2 * (((size_t)(nthr >> lay) * (N + 1)) << lay);
    const bool odd = (tid & 1) != 0;
    const int dp = odd ? -(nthr >> 1) : (nthr >> 1);
    T* yp = y + line_pos(tid, m);
    const double* fw = fint_w ? fint_w + tid : nullptr;
    const int rows = tid < m ? (m - 1 - tid) / nthr + 1 : 0;
    double fpart = 0.0;
    for (int e0 = 0; e0 < rows; e0 += kBatch) {
        TS v[kBatch];
#pragma unroll
        for (int e = 0; e < kBatch; ++e)
            if (e0 + e < rows) v[e] = sp[(e0 + e) * dj];
#pragma unroll
        for (int e = 0; e < kBatch; ++e) {
            if (e0 + e < rows) {
                const TS x = (sine && odd) ? -v[e] : v[e];
                yp[(e0 + e) * dp] = (T)x;
                if (fw) fpart += fw[(e0 + e) * nthr] * (double)x;
            }
        }
    }
    return fpart;
}

template <typename T, typename TS>
__device__ __forceinline__ void store_part(const T* y, Cx<TS>* __restrict__ spec, int part, int k, int m, int N,
                                           int lay, bool sine, T scale, int tid, int nthr) {
    // the index arithmetic is redone here rather than kept from the load (it
    // would stay live in registers, or spill, across the whole pass)
    asm volatile("" : "+v"(tid));
    TS* sp = reinterpret_cast<TS*>(spec) + part + 2 * spec_at(tid, k, N, lay);
    const size_t dj = (size_t)2 * (((size_t)(nthr >> lay) * (N + 1)) << lay);
    const bool odd = (tid & 1) != 0;
    const int p0 = line_pos(tid, m), dp = odd ? -(nthr >> 1) : (nthr >> 1);
    const T sc = (sine && odd) ? -scale : scale;
    int e = 0;
    for (int j = tid; j < m; j += nthr, ++e) sp[e * dj] = (TS)(y[p0 + e * dp] * sc);
}

// Workgroup b -> (k, part): slice b mod 8 of the wavenumbers goes to XCD
// b mod 8, and the two parts of one wavenumber are neighbours on that XCD, so
// the halves of every 16-byte spectrum entry meet in its L2.
__device__ __forceinline__ void real_theta_tile(int k8, int* k, int* part) {
    const int i = blockIdx.x >> 3;
    *k = (blockIdx.x & 7) * k8 + (i >> 1);
    *part = i & 1;
}

// ---------------------------------------------------------------- float64 / float32 single precision pass
template <typename T, int EPT, int RMAX, int SMAX>
__device__ __forceinline__ void theta_real_body(const ThetaArgs<T>& a, int k, int part, unsigned char* smem_raw,
                                                Cx<double>* red) {
    T* y = reinterpret_cast<T*>(smem_raw);
    Cx<T>* z = reinterpret_cast<Cx<T>*>(smem_raw);
    const int m = a.m, N = a.N;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool sine = (k & 1) != 0;
    const bool want_fint = k == 0 && part == 0 && a.fint_w != nullptr;
    const double fpart = load_part<T, T>(y, a.spec, part, k, m, N, a.lay_log2, sine,
                                         want_fint ? a.fint_w : nullptr, tid, nthr);
    if (want_fint) {
        const double s = block_sum(fpart, red);
        if (tid == 0) *a.fint_out = s;
    }
    __syncthreads();
    fft_lds<T, false, EPT, RMAX>(z, 0, a.fft, a.tw, tid, a.nthr_fft, tid < a.nthr_fft);
    const bool scale = a.mode == kSolve || a.mode == kDerivative || a.mode == kDivideSin;
    const T invm = (T)1 / (T)m;
    rdct_split_forward<T>(z, a.eq, a.ws, m, scale ? invm : (T)1, scale ? (T)2 * invm : (T)1, tid, nthr);
    if (a.mode == kDerivative) {
        theta_derivative_line<T, kRealLoadHold>(y, m, sine, tid, nthr);
    } else if (a.mode == kDivideSin) {
        theta_divide_sin_line<T, kRealLoadHold>(y, smem_raw, m, sine, tid);
    } else if (a.mode != kTransformOnly) {
        const bool tr = a.mode == kSolveTransposed;
        if (k == 0) solve_k0<T, SMAX>(y, smem_raw, m, tr, part == 0 ? a.c0 : 0.0, a.k0tab, red, tid);
        else solve_partitioned<T, SMAX>(y, smem_raw, m, k, sine, tr, tid);
        lds_barrier();
    }
    rdct_split_inverse<T>(y, a.eq, a.ws, m, scale ? (T)m : (T)1, scale ? (T)m * (T)0.5 : (T)1, tid, nthr);
    fft_lds<T, true, EPT, RMAX>(z, 0, a.fft, a.tw, tid, a.nthr_fft, tid < a.nthr_fft);
    const bool flip = a.mode == kDerivative || a.mode == kDivideSin;
    store_part<T, T>(y, a.spec_out, part, k, m, N, a.lay_out_log2, flip ? !sine : sine, invm, tid, nthr);
}

template <typename T, int EPT, int RMAX, int SMAX>
__global__ void __launch_bounds__(512, 4) k_theta_real(ThetaArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Cx<double> red[8];
    int k, part;
    real_theta_tile(a.k8, &k, &part);
    if (k > a.N) return;
    theta_real_body<T, EPT, RMAX, SMAX>(a, k, part, smem_raw, red);
}

// ---------------------------------------------------------------- mixed precision pass
// k = 0 of the mixed real pass (see theta_mixed_k0 for the complex line): the
// bordered system in float64, F kept in position order; on return the
// float32 line yf holds the solution.  The right-hand side of each row is
// formed as the solve loads it (F on the first pass; on a correction pass
// the residual of the current iterate yd, whose constraint row needs the
// block sum of its even coefficients first), and the solution goes straight
// to the float32 line: no line values are held in registers across the solve.
template <int SMAXD, bool RESID, bool TRANS>
__device__ __forceinline__ void theta_mixed_real_k0(const ThetaMixArgs& a, int part, double* yd, float* yf,
                                                    double* F, unsigned char* smem_raw, Cx<double>* red,
                                                    int tid, double& acc_r, double& acc_f) {
    const int m = a.m, nthr = blockDim.x;
    const int qhi = m - 1;
    double r0 = part == 0 ? a.c0 : 0.0;
    if (RESID && !TRANS) {
        double dotp = 0.0;
        for (int q = 2 * tid + 2; q <= qhi; q += 2 * nthr) dotp += yd[q] * (1.0 / (1.0 - (double)q * (double)q));
        const double c = r0;
        r0 = r0 - (yd[0] + block_sum(dotp, red));
        if (tid == 0) {
            acc_r += r0 * r0;
            acc_f += c * c;
        }
    }
    const double x0_pin = (RESID && TRANS) ? yd[0] : 0.0;
    const double b0 = (RESID && TRANS) ? F[0] : 0.0;
    if (!RESID && tid == 0) F[0] = yd[0];
    auto load = [&](int q) -> double {
        if (!RESID) {
            const double f = yd[q];
            if (q != 0) F[q] = f;
            return f;
        }
        if (q == 0) return 0.0;
        const int lo_q = (TRANS && (q & 1) == 0) ? 2 : 0;
        double sub, diag, sup;
        band<double>(q, 0, q - 2 < lo_q, q + 2 > qhi, TRANS, sub, diag, sup);
        double ax = yd[q] * diag;
        if (q - 2 >= lo_q) ax += yd[q - 2] * sub;
        if (q + 2 <= qhi) ax += yd[q + 2] * sup;
        double rhs = F[q];
        if (TRANS && (q & 1) == 0) rhs -= b0 * (1.0 / (1.0 - (double)q * (double)q));
        acc_r += (rhs - ax) * (rhs - ax);
        acc_f += rhs * rhs;
        return rhs - ax;
    };
    auto store = [&](int q, double x) { yf[q] = (float)((TRANS && RESID && q == 0) ? -x0_pin : x); };
    solve_k0_io<double, SMAXD, double>(load, store, smem_raw, m, TRANS, r0, a.k0tab, red, tid);
    lds_barrier();
}

// Same refinement as theta_mixed_body, on one real part: float64 analysis
// of the part (F on the first pass; the current iterate on a correction
// pass), the right-hand side formed as the solve loads it, float32 (low k:
// float64) elimination, float32 synthesis written to that part of `out`.
template <int EPT, int RMAX, int SMAXF, int SMAXD, bool RESID, bool TRANS, bool NORM = false>
__device__ __forceinline__ void theta_mixed_real_body(const ThetaMixArgs& a, int k, int part,
                                                      unsigned char* smem_raw, Cx<double>* red) {
    unsigned char* line = smem_raw + kRealLineMargin;
    double* yd = reinterpret_cast<double*>(line);
    Cx<double>* zd = reinterpret_cast<Cx<double>*>(line);
    float* yf = reinterpret_cast<float*>(line);
    Cx<float>* zf = reinterpret_cast<Cx<float>*>(line);
    const int m = a.m, N = a.N;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool sine = (k & 1) != 0;
    const bool want_fint = !RESID && k == 0 && part == 0 && a.fint_w != nullptr;
    const double fpart = load_part<double, double>(yd, RESID ? a.su : a.sa, part, k, m, N, a.lay_log2, sine,
                                                   want_fint ? a.fint_w : nullptr, tid, nthr);
    if (want_fint) {
        const double s = block_sum(fpart, red);
        if (tid == 0) *a.fint_out = s;
    }
    static_assert(2 * SMAXF + 2 <= kRealLineMarginEntries && 2 * SMAXD + 2 <= kRealLineMarginEntries,
                  "the solve's padding rows must stay in the line's margins");
    // The kernels built for the length-5000 transform run m = 10^4 only (the
    // plan checks it): both classes have 5000 rows and every chunk is full.
    constexpr bool FULL = RMAX == kRadixFixed5000;
    static_assert(!FULL || (solve_chunks(5000, 5000, SMAXF).s == SMAXF && solve_chunks(5000, 5000, SMAXD).s == SMAXD),
                  "full chunks at m = 10^4");
    if (tid < kRealLineMarginEntries) {   // the zero margins (the LDS may hold another pass's data)
        yd[tid - kRealLineMarginEntries] = 0.0;
        yd[m + tid] = 0.0;
    }
    __syncthreads();
    fft_lds<double, false, EPT, RMAX>(zd, 0, a.fft, a.tw64, tid, a.nthr_fft, tid < a.nthr_fft);
    const double invm = 1.0 / (double)m;
    rdct_split_forward<double>(zd, a.eq64, a.ws64, m, TRANS ? 1.0 : invm, TRANS ? 1.0 : 2.0 * invm, tid, nthr);

    double* Fk = reinterpret_cast<double*>(a.fco) + (size_t)(2 * k + part) * solve_slot_stride(m);
    // NORM (correction pass only): the residual sums for the info, in a build of its own so
    // that the plain pass carries no extra registers
    constexpr bool want_norm = RESID && NORM;
    double acc_r = 0.0, acc_f = 0.0;
    if (k != 0) {
        // Row q of (L - k^2) X: diag X_q + sub X_{q-2} + sup X_{q+2}, with
        // sub = base - lin and sup = base + lin.  X_{q-2} sits at position
        // p - 2 for a cosine line and p + 2 for a sine line, so the weight of
        // position p - 2 is base - sigma lin with sigma = -1 for sine.  A
        // neighbour past either end of the class reads a margin zero.
        const double kkd = (double)k * (double)k;
        const double lin_w = (sine ? -1.0 : 1.0) * (TRANS ? 0.25 : 0.75);
        const double base_c = TRANS ? 0.0 : 0.5;
        // F of the row in solve order, at a 32-bit byte offset from the
        // wavenumber's (uniform) base; the correction reads it from HBM ahead of
        // the rows' LDS work
        auto fslot = [&](unsigned slot) { return reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(Fk) + slot * 8u); };
        auto fetch = [&](unsigned slot) -> double { return RESID ? *fslot(slot) : 0.0; };
        auto load = [&](int p, int q, unsigned slot, bool own, double f) -> double {
            if (!RESID) {
                f = yd[p];
                *fslot(slot) = f;
                return f;
            }
            const double qd = (double)q, qq = qd * qd;
            const double base = __builtin_fma(qq, 0.25, base_c);
            const double lin = qd * lin_w;
            const double diag = __builtin_fma(qq, -0.5, -kkd);
            double ax = yd[p] * diag;
            ax = __builtin_fma(yd[p - 2], base - lin, ax);
            ax = __builtin_fma(yd[p + 2], base + lin, ax);
            const double r = f - ax;
            if (want_norm && own) {
                acc_r += r * r;
                acc_f += f * f;
            }
            return r;
        };
        if (k < a.k64) {
            solve_partitioned_io<double, double, SMAXD, true, FULL>(
                fetch, load, [&](int p, double x) { yf[p] = (float)x; }, smem_raw, m, k, sine, TRANS, tid);
        } else {
            solve_partitioned_io<float, float, SMAXF, true, FULL>(
                fetch, [&](int p, int q, unsigned slot, bool own, double f) { return (float)load(p, q, slot, own, f); },
                [&](int p, float x) { yf[p] = x; }, smem_raw, m, k, sine, TRANS, tid);
        }
        lds_barrier();
    } else {
        theta_mixed_real_k0<SMAXD, RESID, TRANS>(a, part, yd, yf, Fk, smem_raw, red, tid, acc_r, acc_f);
    }
    if (want_norm) {
        const Cx<double> sm = block_sum(Cx<double>{acc_r, acc_f}, red);
        if (tid == 0) {
            a.rnorm[2 * (2 * k + part)] = sm.x;
            a.rnorm[2 * (2 * k + part) + 1] = sm.y;
        }
    }
    const float fm = (float)m;
    rdct_split_inverse<float>(yf, a.eq32, a.ws32, m, TRANS ? 1.0f : fm, TRANS ? 1.0f : 0.5f * fm, tid, nthr);
    fft_lds<float, true, EPT, RMAX>(zf, 0, a.fft, a.tw32, tid, a.nthr_fft, tid < a.nthr_fft);
    store_part<float, float>(yf, a.out, part, k, m, N, a.lay_out_log2, sine, 1.0f / fm, tid, nthr);
}

template <int EPT, int RMAX, int SMAXF, int SMAXD, bool RESID, bool TRANS, bool NORM = false>
__global__ void __launch_bounds__(512, 4) k_theta_mixed_real(ThetaMixArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Cx<double> red[8];
    int k, part;
    real_theta_tile(a.k8, &k, &part);
    if (k > a.N) return;
    theta_mixed_real_body<EPT, RMAX, SMAXF, SMAXD, RESID, TRANS, NORM>(a, k, part, smem_raw, red);
}

}  // namespace sp
