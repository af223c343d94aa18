// Batch builds of the correction theta stage.
#include "sp_inst_batch.hpp"

void sp::batch_kernels_theta_resid(BatchKernels& k) { batch_stage_kernels<kBThetaResid>(k); }
