// Stage kernels of one reconstruction (minmod), compiled on their own so the
// reconstructions build in parallel.
#define GRMHD_STAGE_KERNELS
#include "grmhd_stage.h"

namespace gk {
template hipError_t launch_stage_recon<GRMHD_RECON_MINMOD>(const StageArgs& a, int precision, int64_t blocks, hipStream_t s);
}  // namespace gk
