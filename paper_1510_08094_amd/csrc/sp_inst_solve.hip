// Kernel builds of the single-problem float64 / float32 passes and the
// gradient pass (see sp_tables.hpp).
#include "sp_tables.hpp"

namespace sp {
namespace {
template <typename T, int RMAX>
KernelSet<T> kernel_set() {
    KernelSet<T> k{&k_lambda_fwd<T, kEPT, RMAX>, &k_lambda_inv<T, kEPT, RMAX>, nullptr, nullptr};
    if constexpr (std::is_same<T, double>::value) {
        if constexpr (RMAX != kRadixFixed5000) k.theta = &k_theta<double, kEPT, RMAX, kSmaxD>;
        k.theta_real = &k_theta_real<double, kEPT, RMAX, kSmaxR>;
    }
    return k;
}

template <typename T>
KernelSet<T> pick(int rs) {
    if (rs == kRadixFixed5000) return kernel_set<T, kRadixFixed5000>();
    return rs <= 16 ? kernel_set<T, 16>() : kernel_set<T, 32>();
}
}  // namespace

template <> KernelSet<double> pick_kernels<double>(int rs) { return pick<double>(rs); }
template <> KernelSet<float> pick_kernels<float>(int rs) { return pick<float>(rs); }

GradKernel grad_kernel(int rs) {
    if (rs == kRadixFixed5000) return &k_lambda_grad<kEPT, kRadixFixed5000>;
    return rs <= 16 ? &k_lambda_grad<kEPT, 16> : &k_lambda_grad<kEPT, 32>;
}

}  // namespace sp
