// srhd_step.hip -- dispatch of the patch step to the kernels of each precision mode
// (srhd_step_fp64.hip, srhd_step_mixed.hip, srhd_step_fp32.hip; templates in srhd_step_impl.hpp).
#include "srhd_internal.hpp"

namespace srhd {

hipError_t launch_step(int prec, const StepArgs &a, hipStream_t st)
{
  if (a.integrator == SRHD_VL) return launch_step_vl(prec, a, st);
  if (prec == SRHD_PREC_MIXED) return step_launch_mixed(a, false, st);
  if (prec == SRHD_PREC_FP32) return step_launch_fp32(a, false, st);
  return step_launch_fp64(a, false, st);
}

hipError_t launch_step_grid(int prec, const StepArgs &a, hipStream_t st)
{
  if (prec == SRHD_PREC_MIXED) return step_launch_mixed(a, true, st);
  if (prec == SRHD_PREC_FP32) return step_launch_fp32(a, true, st);
  return step_launch_fp64(a, true, st);
}

int step_occupancy(int prec, bool gather, int kind, bool occ2)
{
  if (prec == SRHD_PREC_MIXED) return step_occupancy_mixed(gather, kind, occ2);
  if (prec == SRHD_PREC_FP32) return step_occupancy_fp32(gather, kind, occ2);
  return step_occupancy_fp64(gather, kind, occ2);
}

hipError_t launch_grid_prims(int prec, int64_t n_patch, const double *cons, void *prims,
                             unsigned long long *smax_bits, const GuessArgs &g, hipStream_t st)
{
  if (prec == SRHD_PREC_MIXED) return grid_prims_mixed(n_patch, cons, prims, smax_bits, g, st);
  if (prec == SRHD_PREC_FP32) return grid_prims_fp32(n_patch, cons, prims, smax_bits, g, st);
  return grid_prims_fp64(n_patch, cons, prims, smax_bits, g, st);
}

}  // namespace srhd
