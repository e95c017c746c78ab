// srhd_step_fp32.hip -- the patch-step kernels of one precision mode (FP32 bulk and inversion after the FP64 L).
#include "srhd_step_impl.hpp"

namespace srhd {

hipError_t step_launch_fp32(const StepArgs &a, bool gather, hipStream_t st)
{
  return step_launch_ti<float, float>(a, gather, st);
}

int step_occupancy_fp32(bool gather, int kind, bool occ2) { return occupancy_ti<float, float>(gather, kind, occ2); }

hipError_t grid_prims_fp32(int64_t n_patch, const double *cons, void *prims,
                         unsigned long long *smax_bits, unsigned int *net_mask,
                         const GuessArgs &g, hipStream_t st)
{
  return grid_prims_ti<float, float>(n_patch, cons, prims, smax_bits, net_mask, g, st);
}

}  // namespace srhd
