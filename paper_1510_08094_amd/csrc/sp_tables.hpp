// Host-side kernel tables: the compile-time tile constants shared by the
// plans and the kernel builds, and the tables of kernel entry points.  The
// kernels are instantiated in their own translation units (sp_inst_*.hip) so
// the library's device code compiles in parallel; the plans pick entries
// from these tables by radix set.
#pragma once
#include "sp_batch.hpp"
#include "sp_calculus.hpp"
#include "sp_theta_real.hpp"

namespace sp {

constexpr int kEPT = 16;
constexpr int kSmaxD = 13;   // chunk rows per thread, float64 solves (odd: see make_class)
constexpr int kSmaxF = 15;   // chunk rows per thread, float32 solves
constexpr int kLayLog2 = 3;  // spectrum runs of 8 rows: one 128-byte line per float64 run
constexpr int kSmaxR = 21;   // chunk rows per thread, real-part theta pass (both precisions)

// batch tiles (see the build table in sphere_poisson.hip)
constexpr int kBatchThreads = 256;
constexpr int kBatchClasses = 6;
constexpr int kBatchSmallRadix = 16;
constexpr int kBatchRealThreads = 128;
constexpr int kBatchSmaxR = 17;    // chunk rows per thread in those tiles: the shortest that lets m = 2048 fit
constexpr int kBatchWaveThreads = 64;
constexpr int kBatchScal = 16;          // device scalars per problem: integral of f, correction norms
constexpr int kBatchMaxLaunches = 64;   // stage launches in one batch graph (one work-list counter each)
constexpr int kBatchMaxRefine = 4;      // corrections in a mixed batch

template <typename T>
struct KernelSet {
    void (*fwd)(LambdaArgs<T>);
    void (*inv)(LambdaArgs<T>);
    void (*theta)(ThetaArgs<T>);        // complex line (odd m), float64 only
    void (*theta_real)(ThetaArgs<T>);   // one real part per workgroup (even m), float64 only
};

struct MixedSet {
    // [0] complex line (odd m), [1] one real part per workgroup (even m)
    void (*theta_first[2])(ThetaMixArgs);
    void (*theta_resid[2])(ThetaMixArgs);
    void (*theta_first_t[2])(ThetaMixArgs);   // transposed systems (adjoint)
    void (*theta_resid_t[2])(ThetaMixArgs);
    void (*theta_resid_norm[2])(ThetaMixArgs);     // correction pass that also sums the residual norms
    void (*theta_resid_t_norm[2])(ThetaMixArgs);
    void (*mix)(MixLambdaArgs);
    void (*update)(MixLambdaArgs);
};

struct BatchKernels {
    void (*st[kBStages][kBatchClasses])(const void*, const int2*, int, int*);
};

typedef void (*GradKernel)(GradArgs);

// rs: the radix set compiled into a kernel: 16 (radices up to 16), 32 (up to
// 31) or kRadixFixed5000 (the fixed length-5000 transform).
template <typename T> KernelSet<T> pick_kernels(int rs);
template <> KernelSet<double> pick_kernels<double>(int rs);
template <> KernelSet<float> pick_kernels<float>(int rs);
GradKernel grad_kernel(int rs);
MixedSet pick_mixed(int rs);
// every stage's builds; filled stage group by stage group (one translation unit each)
void batch_kernels_lambda(BatchKernels& k);
void batch_kernels_theta64(BatchKernels& k);
void batch_kernels_theta_first(BatchKernels& k);
void batch_kernels_theta_resid(BatchKernels& k);
inline BatchKernels batch_kernels() {
    BatchKernels k;
    batch_kernels_lambda(k);
    batch_kernels_theta64(k);
    batch_kernels_theta_first(k);
    batch_kernels_theta_resid(k);
    return k;
}

}  // namespace sp
