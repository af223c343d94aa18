// Device building blocks: complex arithmetic, compile-time roots of unity,
// radix-R DFT codelets held in registers, and one Stockham autosort pass over
// a line held in LDS.  Used by the lambda and theta transform kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sp {

// ---------------------------------------------------------------- complex
template <typename T>
struct alignas(2 * sizeof(T)) Cx {
    T x, y;
};

template <typename T> __device__ __forceinline__ Cx<T> cmake(T a, T b) { return Cx<T>{a, b}; }
template <typename T> __device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ Cx<T> operator*(Cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> __device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T> __device__ __forceinline__ Cx<T> cconj(Cx<T> a) { return {a.x, -a.y}; }
template <typename T> __device__ __forceinline__ Cx<T> mul_i(Cx<T> a) { return {-a.y, a.x}; }      // i * a
template <typename T> __device__ __forceinline__ Cx<T> mul_negi(Cx<T> a) { return {a.y, -a.x}; }  // -i * a

// ---------------------------------------------------------------- constants
// cos / sin of 2 pi num / den evaluated at compile time: exact octant
// reduction in integers, then Taylor series on [0, pi/4] summed from the
// smallest term (about one ulp).
namespace ct {
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
    double t[16] = {};
    double term = x;
    t[0] = x;
    for (int k = 1; k < 16; ++k) {
        term = term * (-(x * x)) / double((2 * k) * (2 * k + 1));
        t[k] = term;
    }
    double s = 0.0;
    for (int k = 15; k >= 0; --k) s += t[k];
    return s;
}

constexpr double taylor_cos(double x) {
    double t[16] = {};
    double term = 1.0;
    t[0] = 1.0;
    for (int k = 1; k < 16; ++k) {
        term = term * (-(x * x)) / double((2 * k - 1) * (2 * k));
        t[k] = term;
    }
    double s = 0.0;
    for (int k = 15; k >= 0; --k) s += t[k];
    return s;
}

struct CS { double c, s; };

constexpr CS cossin2pi(long long num, long long den) {
    long long t = num % den;
    if (t < 0) t += den;
    long long a = 8 * t;
    long long o = a / den;         // octant 0..7
    long long r = a - o * den;     // angle = (o + r/den) * pi/4
    double x = (double)r / (double)den * (kPi / 4.0);
    double y = (double)(den - r) / (double)den * (kPi / 4.0);
    double cx = taylor_cos(x), sx = taylor_sin(x), cy = taylor_cos(y), sy = taylor_sin(y);
    if (r == 0) { cx = 1.0; sx = 0.0; cy = 0.0; sy = 0.0; }
    switch (o) {
        case 0: return {cx, sx};
        case 1: return r == 0 ? CS{0.70710678118654752440, 0.70710678118654752440} : CS{sy, cy};
        case 2: return r == 0 ? CS{0.0, 1.0} : CS{-sx, cx};
        case 3: return r == 0 ? CS{-0.70710678118654752440, 0.70710678118654752440} : CS{-cy, sy};
        case 4: return r == 0 ? CS{-1.0, 0.0} : CS{-cx, -sx};
        case 5: return r == 0 ? CS{-0.70710678118654752440, -0.70710678118654752440} : CS{-sy, -cy};
        case 6: return r == 0 ? CS{0.0, -1.0} : CS{sx, -cx};
        default: return r == 0 ? CS{0.70710678118654752440, -0.70710678118654752440} : CS{cy, -sy};
    }
}

template <int R>
struct Roots {
    double c[R];
    double s[R];
    constexpr Roots() : c(), s() {
        for (int t = 0; t < R; ++t) {
            CS v = cossin2pi(t, R);
            c[t] = v.c;
            s[t] = v.s;
        }
    }
};
}  // namespace ct

// ---------------------------------------------------------------- codelets
// Forward DFT: X_k = sum_j x_j e^{-2 pi i jk/R}; inverse uses e^{+...}
// (unnormalised).  In place on v[0..R-1].

template <typename T, bool INV>
__device__ __forceinline__ void dft2(Cx<T>& a, Cx<T>& b) {
    Cx<T> t = a - b;
    a = a + b;
    b = t;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(Cx<T>& a0, Cx<T>& a1, Cx<T>& a2, Cx<T>& a3) {
    Cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3;
    Cx<T> t3 = INV ? mul_i(a1 - a3) : mul_negi(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(Cx<T>* v) {
    constexpr T r2 = (T)0.70710678118654752440;
    Cx<T> a0 = v[0] + v[4], a4 = v[0] - v[4];
    Cx<T> a1 = v[1] + v[5], a5 = v[1] - v[5];
    Cx<T> a2 = v[2] + v[6], a6 = v[2] - v[6];
    Cx<T> a3 = v[3] + v[7], a7 = v[3] - v[7];
    if (!INV) {
        a5 = Cx<T>{(a5.x + a5.y) * r2, (a5.y - a5.x) * r2};     // * e^{-i pi/4}
        a6 = mul_negi(a6);                                      // * -i
        a7 = Cx<T>{(a7.y - a7.x) * r2, -(a7.x + a7.y) * r2};    // * e^{-3 i pi/4}
    } else {
        a5 = Cx<T>{(a5.x - a5.y) * r2, (a5.x + a5.y) * r2};
        a6 = mul_i(a6);
        a7 = Cx<T>{-(a7.x + a7.y) * r2, (a7.x - a7.y) * r2};
    }
    dft4<T, INV>(a0, a1, a2, a3);
    dft4<T, INV>(a4, a5, a6, a7);
    v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
    v[1] = a4; v[3] = a5; v[5] = a6; v[7] = a7;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(Cx<T>* v) {
    // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle w16^{n2 k1}, DFT4 over n2
    constexpr ct::Roots<16> W{};
    Cx<T> y[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        Cx<T> a = v[n2], b = v[4 + n2], c = v[8 + n2], d = v[12 + n2];
        dft4<T, INV>(a, b, c, d);
        y[n2 * 4 + 0] = a; y[n2 * 4 + 1] = b; y[n2 * 4 + 2] = c; y[n2 * 4 + 3] = d;
    }
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) {
            const int t = n2 * k1;
            Cx<T> w{(T)W.c[t], INV ? (T)W.s[t] : (T)(-W.s[t])};
            y[n2 * 4 + k1] = cmul(y[n2 * 4 + k1], w);
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        Cx<T> a = y[0 * 4 + k1], b = y[1 * 4 + k1], c = y[2 * 4 + k1], d = y[3 * 4 + k1];
        dft4<T, INV>(a, b, c, d);
        v[k1 + 0] = a; v[k1 + 4] = b; v[k1 + 8] = c; v[k1 + 12] = d;
    }
}

// Odd R: pair the inputs j and R-j; X_r = x0 + sum_j (x_j + x_{R-j}) cos(2 pi rj/R)
//                                         -/+ i sum_j (x_j - x_{R-j}) sin(2 pi rj/R)
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_odd(Cx<T>* v) {
    constexpr int H = (R - 1) / 2;
    constexpr ct::Roots<R> W{};
    Cx<T> s[H], d[H];
    Cx<T> x0 = v[0];
    Cx<T> sum = x0;
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        s[j - 1] = v[j] + v[R - j];
        d[j - 1] = v[j] - v[R - j];
        sum = sum + s[j - 1];
    }
    v[0] = sum;
#pragma unroll
    for (int r = 1; r <= H; ++r) {
        Cx<T> A = x0, B{(T)0, (T)0};
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const int t = (r * j) % R;
            A = A + s[j - 1] * (T)W.c[t];
            B = B + d[j - 1] * (T)W.s[t];
        }
        // forward: X_r = A - iB, X_{R-r} = A + iB
        Cx<T> iB = mul_i(B);
        v[r] = INV ? A + iB : A - iB;
        v[R - r] = INV ? A - iB : A + iB;
    }
}

// The same odd-R transform with each output pair written to out[r * stride]
// as soon as it is formed, and the pair sums and differences built in place
// of the inputs: only the R inputs are held, not the inputs and the outputs
// (radix 31 in float64 would need about 250 registers otherwise).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_odd_store(Cx<T>* v, Cx<T>* __restrict__ out, int stride) {
    constexpr int H = (R - 1) / 2;
    constexpr ct::Roots<R> W{};
    const Cx<T> x0 = v[0];
    Cx<T> sum = x0;
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        const Cx<T> a = v[j], b = v[R - j];
        v[j] = a + b;
        v[R - j] = a - b;
        sum = sum + v[j];
    }
    out[0] = sum;
#pragma unroll
    for (int r = 1; r <= H; ++r) {
        Cx<T> A = x0, B{(T)0, (T)0};
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const int t = (r * j) % R;
            A = A + v[j] * (T)W.c[t];
            B = B + v[R - j] * (T)W.s[t];
        }
        const Cx<T> iB = mul_i(B);
        out[r * stride] = INV ? A + iB : A - iB;
        out[(R - r) * stride] = INV ? A - iB : A + iB;
    }
}

// R = 10 as 2 x 5 by the prime-factor (Good-Thomas) mapping, no twiddles:
// input n = (5 n1 + 2 n2) mod 10, output k = (5 k1 + 6 k2) mod 10; two DFT5
// over n2, then five DFT2 over n1.
template <typename T, bool INV>
__device__ __forceinline__ void dft10(Cx<T>* v) {
    Cx<T> a[5], b[5];
#pragma unroll
    for (int n2 = 0; n2 < 5; ++n2) {
        a[n2] = v[(2 * n2) % 10];
        b[n2] = v[(5 + 2 * n2) % 10];
    }
    dft_odd<T, 5, INV>(a);
    dft_odd<T, 5, INV>(b);
#pragma unroll
    for (int k2 = 0; k2 < 5; ++k2) {
        v[(6 * k2) % 10] = a[k2] + b[k2];
        v[(5 + 6 * k2) % 10] = a[k2] - b[k2];
    }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(Cx<T>* v) {
    if constexpr (R == 10) {
        dft10<T, INV>(v);
    } else if constexpr (R == 2) {
        dft2<T, INV>(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4<T, INV>(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        dft8<T, INV>(v);
    } else if constexpr (R == 16) {
        dft16<T, INV>(v);
    } else {
        static_assert(R % 2 == 1, "unsupported radix");
        dft_odd<T, R, INV>(v);
    }
}

// ---------------------------------------------------------------- barriers
// A workgroup barrier for LDS traffic: it waits for this wave's LDS operations
// only.  __syncthreads() also waits for every global load and store the wave
// has in flight, which would stall the transform passes on memory traffic
// issued before them (a persistent kernel's loads of its next block, the
// stores of its last one).  The "memory" clobber keeps the compiler from
// moving memory accesses across it.  Callers that hand global memory from one
// thread to another use __syncthreads().
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ---------------------------------------------------------------- plans
constexpr int kMaxPass = 16;

struct FftDesc {
    int N;                 // transform length
    int fixed;             // a compiled-in fixed transform (FixedFft), or 0
    int npass;
    int radix[kMaxPass];
    int tw_off[kMaxPass];  // offset of each pass's twiddles in the per-pass table
};

// Butterflies each thread owns in a radix-R pass when a thread holds at most
// EPT complex values in registers.
template <int R, int EPT>
struct Bpt {
    static constexpr int value = (EPT / R) > 0 ? (EPT / R) : 1;
};

// One Stockham pass (radix R) over buf[0..N) in LDS, threads t in [0, nthr)
// of this line.  Every thread of the workgroup must call it (it contains
// barriers); `active` = false makes a thread only take part in the barriers.
// Ns = product of the radices of the previous passes.
//   butterfly j (0 <= j < N/R), k = j mod Ns:
//     v_r = buf[j + r N/R] * w^{r k},  w = e^{-+2 pi i / (Ns R)}
//     V = DFT_R(v);  buf[(j - k) R + k + r Ns] = V_r
// The pass's twiddles are stored as tw[(r - 1) Ns + k] = e^{-2 pi i r k/(Ns R)},
// so neighbouring lanes (neighbouring k) read neighbouring entries.
template <typename T, int R, bool INV, int EPT>
__device__ __forceinline__ void stockham_pass(Cx<T>* __restrict__ buf, int N, int Ns,
                                              const Cx<T>* __restrict__ tw,
                                              int t, int nthr, bool active) {
    constexpr int B = Bpt<R, EPT>::value;
    const int nb = N / R;
    Cx<T> v[B][R];
    if (active) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = t + b * nthr;
            if (j < nb) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[b][r] = buf[j + r * nb];
            }
        }
    }
    lds_barrier();
    if (active) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = t + b * nthr;
            if (j < nb) {
                const int k = j % Ns;
                if (Ns > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        const Cx<T> w = tw[(r - 1) * Ns + k];
                        v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
                    }
                }
                const int base = (j - k) * R + k;
                if constexpr (R >= 11 && (R & 1)) {
                    dft_odd_store<T, R, INV>(v[b], buf + base, Ns);
                } else {
                    dft<T, R, INV>(v[b]);
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[b][r];
                }
            }
        }
    }
    lds_barrier();
}

// ---------------------------------------------------------------- fixed-size transforms
// The same Stockham passes with the length, the radices, the span Ns of each
// pass and the number of threads known at compile time: all index arithmetic
// folds into constants and immediate offsets (the generic passes spend about
// as many integer as floating-point instructions on it).
template <typename T, int R, bool INV, int N, int NS, int NT>
__device__ __forceinline__ void stockham_pass_ct(Cx<T>* __restrict__ buf, const Cx<T>* __restrict__ tw, int t,
                                                 bool active) {
    constexpr int NB = N / R;                 // butterflies
    constexpr int B = (NB + NT - 1) / NT;     // butterflies per thread; only the last can fall off the end
    Cx<T> v[B][R];
    if (active) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = t + b * NT;
            if (b < B - 1 || NB % NT == 0 || j < NB) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[b][r] = buf[j + r * NB];
            }
        }
    }
    lds_barrier();
    if (active) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const unsigned j = (unsigned)(t + b * NT);
            if (b < B - 1 || NB % NT == 0 || j < (unsigned)NB) {
                __builtin_assume(j < (unsigned)NB);
                const unsigned k = NS == 1 ? 0u : j % (unsigned)NS;
                if constexpr (NS > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        const Cx<T> w = tw[(r - 1) * NS + k];
                        v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
                    }
                }
                dft<T, R, INV>(v[b]);
                const unsigned base = (j - k) * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) buf[base + r * NS] = v[b][r];
            }
        }
    }
    lds_barrier();
}

template <typename T, bool INV, int N, int NT, int NS, int R, int... REST>
__device__ __forceinline__ void fft_ct_passes(Cx<T>* __restrict__ buf, const Cx<T>* __restrict__ tw, int t,
                                              bool active) {
    stockham_pass_ct<T, R, INV, N, NS, NT>(buf, tw, t, active);
    if constexpr (sizeof...(REST) > 0)
        fft_ct_passes<T, INV, N, NT, NS * R, REST...>(buf, tw + (R - 1) * NS, t, active);
}

// Fixed transforms compiled in.  A kernel instantiated with the radix-set
// parameter RMAX = kRadixFixed5000 runs only the fixed passes below; the plan
// chooses it when FftDesc::fixed says the length, radix order and thread
// count match.
enum FixedFft { kFixedNone = 0, kFixed5000 = 1 };
constexpr int kRadixFixed5000 = -5000;
// 5000 = 10 5 10 10: radix-10 passes with one butterfly per thread and a
// radix-5 pass with two.  The radix-5 pass comes second: placed there, every
// pass's LDS writes hit distinct banks, where after a first radix-5 pass the
// radix-10 writes of span 5 collide two to three ways in float64.
constexpr int kFixed5000Threads = 500;
constexpr int kFixed5000Radices[4] = {10, 5, 10, 10};

// The fixed transform with its first pass fed from registers (IN) and/or its
// last pass left in registers (OUT), for lines read from or written to HBM in
// natural order.  The first pass (radix 10, span 1) of butterfly t takes the
// points t + 500 r, r = 0..9, and the last pass (radix 10, span 500) of
// butterfly t produces the points t + 500 r in place: exactly the points a
// thread of the row loads and stores owns.  IN: v holds the inputs and the
// LDS line is only written (its first read and barrier are saved).  OUT: the
// outputs stay in v, nothing is written back, and no barrier follows the last
// pass's LDS reads: a caller that writes the LDS next synchronises first.
template <typename T, bool INV, bool IN, bool OUT>
__device__ __forceinline__ void fft5000_regs(Cx<T>* __restrict__ buf, const Cx<T>* __restrict__ tw, int t,
                                             bool active, Cx<T> (&v)[10]) {
    static_assert(kFixed5000Radices[0] == 10 && kFixed5000Radices[1] == 5 && kFixed5000Radices[2] == 10 &&
                  kFixed5000Radices[3] == 10, "pass layout of the fixed transform");
    constexpr int N = 5000, NT = kFixed5000Threads;
    if constexpr (IN) {
        if (active) {
            dft<T, 10, INV>(v);
#pragma unroll
            for (int r = 0; r < 10; ++r) buf[t * 10 + r] = v[r];
        }
        lds_barrier();
    } else {
        stockham_pass_ct<T, 10, INV, N, 1, NT>(buf, tw, t, active);
    }
    stockham_pass_ct<T, 5, INV, N, 10, NT>(buf, tw + 9, t, active);
    stockham_pass_ct<T, 10, INV, N, 50, NT>(buf, tw + 9 + 4 * 10, t, active);
    const Cx<T>* tw4 = tw + 9 + 4 * 10 + 9 * 50;
    if constexpr (OUT) {
        if (active) {
#pragma unroll
            for (int r = 0; r < 10; ++r) v[r] = buf[t + r * 500];
#pragma unroll
            for (int r = 1; r < 10; ++r) {
                const Cx<T> w = tw4[(r - 1) * 500 + t];
                v[r] = INV ? cmulc(v[r], w) : cmul(v[r], w);
            }
            dft<T, 10, INV>(v);
        }
    } else {
        stockham_pass_ct<T, 10, INV, N, 500, NT>(buf, tw4, t, active);
    }
}

// Whole transform: dispatch each pass on its (uniform) radix.  RMAX bounds the
// radices compiled into this instantiation.
// The line is base[off .. off + N).
template <typename T, bool INV, int EPT, int RMAX>
__device__ __forceinline__ void fft_lds(Cx<T>* __restrict__ base, int off, const FftDesc& d,
                                        const Cx<T>* __restrict__ ptw, int t0, int nthr, bool active) {
    if constexpr (RMAX == kRadixFixed5000) {
        (void)d;
        (void)nthr;
        fft_ct_passes<T, INV, 5000, kFixed5000Threads, 1, 10, 5, 10, 10>(base + off, ptw, t0, active);
    } else {
        int Ns = 1;
        for (int p = 0; p < d.npass; ++p) {
            const int R = d.radix[p];
            const Cx<T>* tw = ptw + d.tw_off[p];
            // The thread index and the line offset are made opaque on every pass:
            // otherwise the LDS addresses of all radix cases are hoisted out of the
            // loop and stay live across it, which costs tens of registers and
            // forces spills.
            int t = t0, o = off;
            asm volatile("" : "+v"(t), "+v"(o));
            Cx<T>* buf = base + o;
            switch (R) {
                case 2: stockham_pass<T, 2, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                case 3: stockham_pass<T, 3, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                case 4: stockham_pass<T, 4, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                case 5: stockham_pass<T, 5, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                case 7: stockham_pass<T, 7, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                case 8: stockham_pass<T, 8, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                case 11: stockham_pass<T, 11, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                case 13: stockham_pass<T, 13, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                case 16: stockham_pass<T, 16, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                default:
                    if constexpr (RMAX >= 17) {
                        switch (R) {
                            case 17: stockham_pass<T, 17, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                            case 19: stockham_pass<T, 19, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                            case 23: stockham_pass<T, 23, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                            case 29: stockham_pass<T, 29, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                            case 31: stockham_pass<T, 31, INV, EPT>(buf, d.N, Ns, tw, t, nthr, active); break;
                            default: break;
                        }
                    }
                    break;
            }
            Ns *= R;
        }
    }
}

}  // namespace sp
