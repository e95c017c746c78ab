// srhd_step_fp64.hip -- the patch-step kernels of one precision mode (FP64 bulk and inversion).
#include "srhd_step_impl.hpp"

namespace srhd {

hipError_t step_launch_fp64(const StepArgs &a, bool gather, hipStream_t st)
{
  return step_launch_ti<double, double>(a, gather, st);
}

int step_occupancy_fp64(bool gather, int kind, bool occ2) { return occupancy_ti<double, double>(gather, kind, occ2); }

hipError_t grid_prims_fp64(int64_t n_patch, const double *cons, void *prims,
                         unsigned long long *smax_bits, unsigned int *net_mask,
                         const GuessArgs &g, hipStream_t st)
{
  return grid_prims_ti<double, double>(n_patch, cons, prims, smax_bits, net_mask, g, st);
}

}  // namespace srhd
