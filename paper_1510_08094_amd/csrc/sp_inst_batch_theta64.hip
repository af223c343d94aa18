// Batch builds of the float64 theta stage.
#include "sp_inst_batch.hpp"

void sp::batch_kernels_theta64(BatchKernels& k) { batch_stage_kernels<kBTheta64>(k); }
