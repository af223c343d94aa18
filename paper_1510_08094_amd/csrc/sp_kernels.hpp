// Transform and solve kernels of the DFS Poisson solver (Section 5 of the
// paper): lambda real transforms (rows of the grid), and the per-wavenumber
// theta pass (cosine/sine transform, banded solves, inverse transform).
//
// Spectrum layout in HBM ("j-blocked"): the half spectrum X_k(theta_j),
// k = 0..N (N = n/2), is stored as spec[((j / RW) * (N + 1) + k) * RW + j % RW]
// with RW a power of two (rows per lambda workgroup).  A lambda workgroup
// reads or writes one contiguous block; a theta workgroup reads runs of RW
// consecutive rows of one wavenumber.
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
    const Cx<T>* tw;        // e^{-2 pi i t/n}, t = 0..n-1 (the length-N DFT uses stride 2)
    const double* rowscale; // per-row multiplier or nullptr
    int n, m, N, rw_log2;
    T w_mid, w_end;         // forward: output weight for 0<k<N and for k in {0,N}; inverse: input weights
    double out_scale;       // inverse: multiplier of the written rows
    FftDesc fft;
    int nthr;               // threads per row
};

template <typename T, int EPT, int RMAX>
__global__ void __launch_bounds__(1024) k_lambda_fwd(LambdaArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Cx<T>* lines = reinterpret_cast<Cx<T>*>(smem_raw);
    const int rw = 1 << a.rw_log2;
    const int N = a.N;
    const int line = threadIdx.x / a.nthr;
    const int t = threadIdx.x - line * a.nthr;
    const int jb = blockIdx.x;
    const int j = (jb << a.rw_log2) + line;
    const bool active = line < rw && j < a.m;
    Cx<T>* buf = lines + (size_t)line * N;
    if (active) {
        const double s = a.rowscale ? a.rowscale[j] : 1.0;
        const double2* src = reinterpret_cast<const double2*>(a.x + (size_t)j * a.n);
        for (int i = t; i < N; i += a.nthr) {
            const double2 p = src[i];
            buf[i] = Cx<T>{(T)(p.x * s), (T)(p.y * s)};
        }
    }
    __syncthreads();
    fft_lds<T, false, EPT, RMAX>(buf, a.fft, a.tw, t, a.nthr, active);
    // split into the real-input spectrum; lanes run over (pair, row) with the row fastest
    const int npairs = N / 2 + 1;
    const size_t blk = (size_t)jb * (N + 1);
    for (int e = threadIdx.x; e < npairs * rw; e += blockDim.x) {
        const int jj = e & (rw - 1);
        const int k = e >> a.rw_log2;
        if ((jb << a.rw_log2) + jj >= a.m) continue;
        const Cx<T>* b = lines + (size_t)jj * N;
        if (k == 0) {
            const Cx<T> z = b[0];
            a.spec[(blk + 0) * rw + jj] = Cx<T>{(z.x + z.y) * a.w_end, (T)0};
            a.spec[(blk + N) * rw + jj] = Cx<T>{(z.x - z.y) * a.w_end, (T)0};
            continue;
        }
        const Cx<T> zk = b[k], zn = b[N - k];
        const Cx<T> E = (zk + cconj(zn)) * (T)0.5;
        const Cx<T> O = mul_negi(zk - cconj(zn)) * (T)0.5;
        const Cx<T> WO = cmul(a.tw[k], O);
        a.spec[(blk + k) * rw + jj] = (E + WO) * a.w_mid;
        if (N - k != k) a.spec[(blk + N - k) * rw + jj] = cconj(E - WO) * a.w_mid;
    }
}

template <typename T, int EPT, int RMAX>
__global__ void __launch_bounds__(1024) k_lambda_inv(LambdaArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Cx<T>* lines = reinterpret_cast<Cx<T>*>(smem_raw);
    const int rw = 1 << a.rw_log2;
    const int N = a.N;
    const int line = threadIdx.x / a.nthr;
    const int t = threadIdx.x - line * a.nthr;
    const int jb = blockIdx.x;
    const int j = (jb << a.rw_log2) + line;
    const bool active = line < rw && j < a.m;
    const int npairs = N / 2 + 1;
    const size_t blk = (size_t)jb * (N + 1);
    for (int e = threadIdx.x; e < npairs * rw; e += blockDim.x) {
        const int jj = e & (rw - 1);
        const int k = e >> a.rw_log2;
        if ((jb << a.rw_log2) + jj >= a.m) continue;
        Cx<T>* b = lines + (size_t)jj * N;
        if (k == 0) {
            const T x0 = a.spec[(blk + 0) * rw + jj].x * a.w_end;
            const T xN = a.spec[(blk + N) * rw + jj].x * a.w_end;
            b[0] = Cx<T>{x0 + xN, x0 - xN};
            continue;
        }
        const Cx<T> xk = a.spec[(blk + k) * rw + jj] * a.w_mid;
        const Cx<T> xn = a.spec[(blk + N - k) * rw + jj] * a.w_mid;
        const Cx<T> P = xk + cconj(xn);
        const Cx<T> Q = xk - cconj(xn);
        const Cx<T> iWQ = mul_i(cmulc(Q, a.tw[k]));   // i conj(W) Q
        b[k] = P + iWQ;
        if (N - k != k) b[N - k] = cconj(P - iWQ);
    }
    __syncthreads();
    fft_lds<T, true, EPT, RMAX>(lines + (size_t)line * N, a.fft, a.tw, t, a.nthr, active);
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

enum ThetaMode { kSolve = 0, kSolveTransposed = 1, kTransformOnly = 2 };

template <typename T>
struct ThetaArgs {
    Cx<T>* spec;
    const Cx<T>* tw;        // e^{-2 pi i t/m}, t = 0..m-1
    const Cx<T>* eq;        // e^{-i pi q/(2m)}, q = 0..m-1
    int n, m, N, rw_log2;
    FftDesc fft;
    int nthr_fft;
    int mode;               // ThetaMode
    int k8;                 // wavenumbers per XCD slice (ceil((N+1)/8))
    double c0;              // k = 0 constraint value for a_0 (integral / (4 pi))
    const double* k0tab;    // k = 0 LU factors: invA[NA] cpA[NA] invB[NB] cpB[NB]
    const double* fint_w;   // quadrature weights of the integral of f (k = 0 column), or nullptr
    double* fint_out;
};

template <typename T>
__device__ __forceinline__ void band(int q, int k, bool first, bool last, bool transposed,
                                     T& sub, T& diag, T& sup) {
    const T qq = (T)q;
    diag = -(qq * qq) * (T)0.5 - (T)k * (T)k;
    if (!transposed) {
        sub = first ? (T)0 : (qq - (T)2) * (qq - (T)1) * (T)0.25;
        sup = last ? (T)0 : (qq + (T)2) * (qq + (T)1) * (T)0.25;
    } else {   // rows of the transpose: sub'(q) = sup(q-2), sup'(q) = sub(q+2)
        sub = first ? (T)0 : qq * (qq - (T)1) * (T)0.25;
        sup = last ? (T)0 : qq * (qq + (T)1) * (T)0.25;
    }
}

struct ClassInfo {
    int q0, nc, s, p;     // first q, rows, chunk length, chunks
};

template <int SMAX>
__device__ __forceinline__ ClassInfo make_class(int q0, int qhi) {
    ClassInfo c;
    c.q0 = q0;
    c.nc = qhi >= q0 ? (qhi - q0) / 2 + 1 : 0;
    c.p = (c.nc + SMAX - 1) / SMAX;
    c.s = c.p ? (c.nc + c.p - 1) / c.p : 0;
    return c;
}

// Partitioned solve of both parity classes for k != 0 (or the transposed
// systems).  Each thread owns a contiguous chunk of rows of one class: its
// first row is a separator, the interior rows are eliminated against the two
// neighbouring separators (spikes v, w), the separators form a tridiagonal
// system solved by parallel cyclic reduction, and the interiors are rebuilt.
template <typename T, int SMAX>
__device__ void solve_partitioned(Cx<T>* __restrict__ buf, unsigned char* __restrict__ scratch,
                                  int m, int k, bool sine, bool transposed, int tid) {
    const int qhi = sine ? m : m - 1;
    const ClassInfo A = make_class<SMAX>(sine ? 2 : 0, qhi);
    const ClassInfo B = make_class<SMAX>(1, qhi);
    const int ptot = A.p + B.p;
    const bool inA = tid < A.p;
    const bool inB = !inA && tid < ptot;
    const ClassInfo& C = inA ? A : B;
    const int p = inA ? tid : tid - A.p;
    const int cls_lo = inA ? 0 : A.p;            // reduced-row range of this class
    const int cls_hi = inA ? A.p : ptot;
    const int lo = p * C.s;
    const int cnt = (inA || inB) ? min(C.s, C.nc - lo) : 0;
    const int ni = cnt - 1;

    Cx<T> dr[SMAX];
    T vr[SMAX], cr[SMAX];
    // load the chunk (LDS position of coefficient q: q for cosine, m - q for sine)
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int q = C.q0 + 2 * (lo + ii);
            dr[ii] = buf[sine ? m - q : q];
        }
    }
    __syncthreads();   // B1: the column may now be overwritten by scratch

    T dwlast = 0;
    {
        T cpp = 0, dvp = 0;
        Cx<T> dyp{0, 0};
#pragma unroll
        for (int ii = 1; ii < SMAX; ++ii) {
            if (ii <= ni) {
                const int row = lo + ii;
                const int q = C.q0 + 2 * row;
                T a, b, c;
                band<T>(q, k, false, row == C.nc - 1, transposed, a, b, c);
                const T den = (ii == 1) ? b : b - a * cpp;
                const T inv = (T)1 / den;
                const T cp = c * inv;
                const Cx<T> dy = (ii == 1) ? dr[ii] * inv : (dr[ii] - dyp * a) * inv;
                const T dv = (ii == 1) ? a * inv : -a * dvp * inv;
                if (ii == ni) dwlast = c * inv;
                cr[ii] = cp; dr[ii] = dy; vr[ii] = dv;
                cpp = cp; dyp = dy; dvp = dv;
            }
        }
    }
    {
        Cx<T> yn{0, 0};
        T vn = 0, wn = 0;
#pragma unroll
        for (int ii = SMAX - 1; ii >= 1; --ii) {
            if (ii <= ni) {
                Cx<T> y;
                T v, w;
                if (ii == ni) { y = dr[ii]; v = vr[ii]; w = dwlast; }
                else { y = dr[ii] - yn * cr[ii]; v = vr[ii] - cr[ii] * vn; w = -cr[ii] * wn; }
                dr[ii] = y; vr[ii] = v; cr[ii] = w;
                yn = y; vn = v; wn = w;
            }
        }
    }
    // first / last interior value triples (a chunk of one row passes the neighbour through)
    Cx<T> yF{0, 0}, yL{0, 0};
    T vF = 0, wF = -1, vL = -1, wL = 0;
    if (ni >= 1) {
        yF = dr[1]; vF = vr[1]; wF = cr[1];
#pragma unroll
        for (int ii = 1; ii < SMAX; ++ii)
            if (ii == ni) { yL = dr[ii]; vL = vr[ii]; wL = cr[ii]; }
    }
    // scratch: de[ptot] (Cx), al[ptot], be[ptot], ga[ptot] (T)
    Cx<T>* de = reinterpret_cast<Cx<T>*>(scratch);
    T* al = reinterpret_cast<T*>(de + ptot);
    T* be = al + ptot;
    T* ga = be + ptot;
    if (cnt > 0) { de[tid] = yL; al[tid] = vL; ga[tid] = wL; }
    __syncthreads();   // B2
    T nal = 0, nbe = 1, nga = 0;
    Cx<T> nde{0, 0};
    if (cnt > 0) {
        T a0, b0, c0;
        band<T>(C.q0 + 2 * lo, k, lo == 0, lo == C.nc - 1, transposed, a0, b0, c0);
        Cx<T> pyL{0, 0};
        T pvL = 0, pwL = 0;
        if (p > 0) { pyL = de[tid - 1]; pvL = al[tid - 1]; pwL = ga[tid - 1]; }
        nal = -a0 * pvL;
        nbe = b0 - a0 * pwL - c0 * vF;
        nga = -c0 * wF;
        nde = dr[0] - pyL * a0 - yF * c0;
    }
    __syncthreads();   // B3
    if (cnt > 0) { al[tid] = nal; be[tid] = nbe; ga[tid] = nga; de[tid] = nde; }
    __syncthreads();   // B4
    // parallel cyclic reduction on the separators of each class
    const int pmax = max(A.p, B.p);
    for (int h = 1; h < pmax; h <<= 1) {
        T xal = nal, xbe = nbe, xga = nga;
        Cx<T> xde = nde;
        if (cnt > 0) {
            const int im = tid - h, ip = tid + h;
            if (im >= cls_lo) {
                const T k1 = nal / be[im];
                xal = -k1 * al[im];
                xbe = xbe - k1 * ga[im];
                xde = xde - de[im] * k1;
            } else {
                xal = 0;
            }
            if (ip < cls_hi) {
                const T k2 = nga / be[ip];
                xga = -k2 * ga[ip];
                xbe = xbe - k2 * al[ip];
                xde = xde - de[ip] * k2;
            } else {
                xga = 0;
            }
        }
        __syncthreads();
        nal = xal; nbe = xbe; nga = xga; nde = xde;
        if (cnt > 0) { al[tid] = nal; be[tid] = nbe; ga[tid] = nga; de[tid] = nde; }
        __syncthreads();
    }
    const Cx<T> S = nde * ((T)1 / nbe);
    if (cnt > 0) de[tid] = S;
    __syncthreads();
    Cx<T> Sn{0, 0};
    if (cnt > 0 && tid + 1 < cls_hi) Sn = de[tid + 1];
    __syncthreads();   // scratch no longer needed: write the solution
    if (cnt > 0) {
        buf[sine ? m - (C.q0 + 2 * lo) : C.q0 + 2 * lo] = S;
#pragma unroll
        for (int ii = 1; ii < SMAX; ++ii) {
            if (ii <= ni) {
                const int q = C.q0 + 2 * (lo + ii);
                buf[sine ? m - q : q] = dr[ii] - S * vr[ii] - Sn * cr[ii];
            }
        }
    }
}

// Block-wide sum of one complex double per thread (result valid in every thread).
__device__ __forceinline__ Cx<double> block_sum(Cx<double> v, Cx<double>* red) {
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_down(v.x, off, 64);
        v.y += __shfl_down(v.y, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    Cx<double> s{0.0, 0.0};
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s = s + red[w];
    __syncthreads();
    return s;
}

// k = 0: the two cosine classes (odd q, and even q >= 2) are solved with LU
// factors precomputed on the host in extended precision (the k = 0 systems
// are only weakly diagonally dominant), as two first-order recurrences each
// evaluated by a chunked scan of affine maps:
//   T x = r:   z_i = (r_i - sub_i z_{i-1}) inv_i,     x_i = z_i - cp_i x_{i+1}
//   T^T x = r: z_i = r_i - cp_{i-1} z_{i-1},           x_i = (z_i - sub_{i+1} x_{i+1}) inv_i
// a_0 then follows from the constraint (transposed: the constraint row feeds
// the even class and the q = 0 output is zero).  Always float64.
template <int SMAX>
__device__ void scan_affine(Cx<double>& A, double& Bm, unsigned char* scratch, int tid,
                            int cls_lo, int cls_hi, int ptot, bool reverse, bool valid) {
    // inclusive scan of maps f_p(z) = A_p + B_p z over the chunks of a class
    // (forward: f_p applied after f_{p-1}; reverse: after f_{p+1}).
    Cx<double>* sa = reinterpret_cast<Cx<double>*>(scratch);
    double* sb = reinterpret_cast<double*>(sa + ptot);
    if (valid) { sa[tid] = A; sb[tid] = Bm; }
    __syncthreads();
    const int pmax = ptot;   // upper bound on class length
    for (int h = 1; h < pmax; h <<= 1) {
        Cx<double> nA = A;
        double nB = Bm;
        if (valid) {
            const int o = reverse ? tid + h : tid - h;
            if (reverse ? (o < cls_hi) : (o >= cls_lo)) {
                // compose: (this after other): A + B * A_o, B * B_o
                nA = A + sa[o] * Bm;
                nB = Bm * sb[o];
            }
        }
        __syncthreads();
        A = nA; Bm = nB;
        if (valid) { sa[tid] = A; sb[tid] = Bm; }
        __syncthreads();
    }
}

template <typename T, int SMAX>
__device__ void solve_k0(Cx<T>* __restrict__ buf, unsigned char* __restrict__ scratch, int m,
                         bool transposed, double c0, const double* __restrict__ tab, Cx<double>* red,
                         int tid) {
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
    const Cx<double> a0bar{(double)buf[0].x, (double)buf[0].y};

    Cx<double> r[SMAX];
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int q = C.q0 + 2 * (lo + ii);
            const Cx<T> v = buf[q];
            r[ii] = Cx<double>{(double)v.x, (double)v.y};
            if (transposed && inA) {
                const double om = 1.0 / (1.0 - (double)q * (double)q);
                r[ii] = r[ii] - a0bar * om;
            }
        }
    }
    __syncthreads();
    auto sub_of = [&](int row) -> double {   // sub-diagonal of row `row` of the class
        if (row <= 0) return 0.0;
        const double q = (double)(C.q0 + 2 * row);
        return (q - 2.0) * (q - 1.0) * 0.25;
    };
    // forward recurrence z_i = alpha_i + beta_i z_{i-1}
    Cx<double> Af{0.0, 0.0};
    double Bf = 1.0;
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int row = lo + ii;
            Cx<double> al;
            double be;
            if (!transposed) { al = r[ii] * inv[row]; be = -sub_of(row) * inv[row]; }
            else { al = r[ii]; be = row > 0 ? -cp[row - 1] : 0.0; }
            Af = al + Af * be;
            Bf = be * Bf;
        }
    }
    scan_affine<SMAX>(Af, Bf, scratch, tid, cls_lo, cls_hi, ptot, false, cnt > 0);
    // value entering this chunk = inclusive result of the previous chunk applied to 0
    Cx<double>* sa = reinterpret_cast<Cx<double>*>(scratch);
    Cx<double> zin{0.0, 0.0};
    if (cnt > 0 && tid - 1 >= cls_lo) zin = sa[tid - 1];
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int row = lo + ii;
            Cx<double> al;
            double be;
            if (!transposed) { al = r[ii] * inv[row]; be = -sub_of(row) * inv[row]; }
            else { al = r[ii]; be = row > 0 ? -cp[row - 1] : 0.0; }
            zin = al + zin * be;
            r[ii] = zin;
        }
    }
    // backward recurrence x_i = gamma_i + delta_i x_{i+1}
    Cx<double> Ab{0.0, 0.0};
    double Bb = 1.0;
#pragma unroll
    for (int ii = SMAX - 1; ii >= 0; --ii) {
        if (ii < cnt) {
            const int row = lo + ii;
            Cx<double> ga;
            double de;
            if (!transposed) { ga = r[ii]; de = -cp[row]; }
            else { ga = r[ii] * inv[row]; de = row + 1 < C.nc ? -sub_of(row + 1) * inv[row] : 0.0; }
            Ab = ga + Ab * de;
            Bb = de * Bb;
        }
    }
    scan_affine<SMAX>(Ab, Bb, scratch, tid, cls_lo, cls_hi, ptot, true, cnt > 0);
    Cx<double> xin{0.0, 0.0};
    if (cnt > 0 && tid + 1 < cls_hi) xin = sa[tid + 1];
    __syncthreads();
    Cx<double> part{0.0, 0.0};
#pragma unroll
    for (int ii = SMAX - 1; ii >= 0; --ii) {
        if (ii < cnt) {
            const int row = lo + ii;
            Cx<double> ga;
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
    const Cx<double> dot = block_sum(part, red);
#pragma unroll
    for (int ii = 0; ii < SMAX; ++ii) {
        if (ii < cnt) {
            const int q = C.q0 + 2 * (lo + ii);
            buf[q] = Cx<T>{(T)r[ii].x, (T)r[ii].y};
        }
    }
    if (tid == 0) {
        if (!transposed) buf[0] = Cx<T>{(T)(c0 - dot.x), (T)(-dot.y)};
        else buf[0] = Cx<T>{(T)0, (T)0};
    }
}

template <typename T, int EPT, int RMAX, int SMAX>
__global__ void __launch_bounds__(1024) k_theta(ThetaArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Cx<double> red[16];
    Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem_raw);
    const int k = (blockIdx.x & 7) * a.k8 + (blockIdx.x >> 3);
    if (k > a.N) return;
    const int m = a.m, N = a.N, rwl = a.rw_log2, rw = 1 << rwl;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool sine = (k & 1) != 0;
    const T invm = (T)1 / (T)m;

    double fpart = 0.0;
    for (int j = tid; j < m; j += nthr) {
        const size_t idx = ((((size_t)(j >> rwl)) * (N + 1) + k) << rwl) + (j & (rw - 1));
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
    fft_lds<T, false, EPT, RMAX>(buf, a.fft, a.tw, tid, a.nthr_fft, tid < a.nthr_fft);
    const bool scale = a.mode == kSolve;
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
    if (a.mode != kTransformOnly) {
        unsigned char* scratch = smem_raw;
        if (k == 0) solve_k0<T, SMAX>(buf, scratch, m, a.mode == kSolveTransposed, a.c0, a.k0tab, red, tid);
        else solve_partitioned<T, SMAX>(buf, scratch, m, k, sine, a.mode == kSolveTransposed, tid);
    }
    __syncthreads();
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
    fft_lds<T, true, EPT, RMAX>(buf, a.fft, a.tw, tid, a.nthr_fft, tid < a.nthr_fft);
    for (int j = tid; j < m; j += nthr) {
        const size_t idx = ((((size_t)(j >> rwl)) * (N + 1) + k) << rwl) + (j & (rw - 1));
        const int pos = (j & 1) ? m - ((j + 1) >> 1) : (j >> 1);
        Cx<T> x = buf[pos] * invm;
        if (sine && (j & 1)) x = Cx<T>{-x.x, -x.y};
        a.spec[idx] = x;
    }
}

}  // namespace sp
