// One stage's builds of the persistent batch kernel (included by the
// sp_inst_batch_*.hip translation units; see sp_tables.hpp).
#pragma once
#include "sp_tables.hpp"

namespace sp {
template <int STG>
void batch_stage_kernels(BatchKernels& k) {
    constexpr bool theta = STG == kBTheta64 || STG == kBThetaFirst || STG == kBThetaResid;
    k.st[STG][0] = &k_batch<kEPT, kBatchSmallRadix, kSmaxF, kSmaxD, STG, kBatchThreads, theta ? 3 : 4, false>;
    k.st[STG][1] = &k_batch<kEPT, 32, kSmaxF, kSmaxD, STG, kBatchThreads, 2, false>;
    if constexpr (theta) {
        k.st[STG][2] = &k_batch<kEPT, kBatchSmallRadix, kBatchSmaxR, kBatchSmaxR, STG, kBatchRealThreads, 3, true>;
        k.st[STG][3] = &k_batch<kEPT, 32, kBatchSmaxR, kBatchSmaxR, STG, kBatchRealThreads, 2, true>;
        k.st[STG][4] = &k_batch<kEPT, kBatchSmallRadix, kSmaxR, kSmaxR, STG, kBatchWaveThreads, 3, true>;
        k.st[STG][5] = &k_batch<kEPT, 32, kSmaxR, kSmaxR, STG, kBatchWaveThreads, 2, true>;
    } else {
        for (int c = 2; c < kBatchClasses; ++c) k.st[STG][c] = nullptr;
    }
}
}  // namespace sp
