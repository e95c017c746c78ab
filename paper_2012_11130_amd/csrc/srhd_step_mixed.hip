// srhd_step_mixed.hip -- the patch-step kernels of one precision mode (FP32 bulk, FP64 inversion).
#include "srhd_step_impl.hpp"

namespace srhd {

hipError_t step_launch_mixed(const StepArgs &a, bool gather, hipStream_t st)
{
  return step_launch_ti<float, double>(a, gather, st);
}

int step_occupancy_mixed(bool gather, int kind, bool occ2) { return occupancy_ti<float, double>(gather, kind, occ2); }

hipError_t grid_prims_mixed(int64_t n_patch, const double *cons, void *prims,
                         unsigned long long *smax_bits, unsigned int *net_mask,
                         const GuessArgs &g, hipStream_t st)
{
  return grid_prims_ti<float, double>(n_patch, cons, prims, smax_bits, net_mask, g, st);
}

}  // namespace srhd
