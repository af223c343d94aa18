// Batch builds of the first mixed-precision theta stage.
#include "sp_inst_batch.hpp"

void sp::batch_kernels_theta_first(BatchKernels& k) { batch_stage_kernels<kBThetaFirst>(k); }
