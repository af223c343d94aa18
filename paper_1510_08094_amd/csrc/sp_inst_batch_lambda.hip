// Batch builds of the lambda stages.
#include "sp_inst_batch.hpp"

void sp::batch_kernels_lambda(BatchKernels& k) {
    batch_stage_kernels<kBLamFwd>(k);
    batch_stage_kernels<kBLamInv>(k);
    batch_stage_kernels<kBLamMix>(k);
    batch_stage_kernels<kBLamUpd>(k);
}
