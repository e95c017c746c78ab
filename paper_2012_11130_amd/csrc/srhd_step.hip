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
                             unsigned long long *smax_bits, unsigned int *net_mask,
                             const GuessArgs &g, hipStream_t st)
{
  if (prec == SRHD_PREC_MIXED) return grid_prims_mixed(n_patch, cons, prims, smax_bits, net_mask, g, st);
  if (prec == SRHD_PREC_FP32) return grid_prims_fp32(n_patch, cons, prims, smax_bits, net_mask, g, st);
  return grid_prims_fp64(n_patch, cons, prims, smax_bits, net_mask, g, st);
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_side_mutex;
SideStream g_side[kMaxDevices];
bool g_side_ready[kMaxDevices];
std::mutex g_side_lock[kMaxDevices];
}  // namespace

hipError_t side_stream(SideStream &out)
{
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(g_side_mutex);
  if (!g_side_ready[dev]) {
    SideStream s{};
    e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.join, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    s.lock = &g_side_lock[dev];
    g_side[dev] = s;
    g_side_ready[dev] = true;
  }
  out = g_side[dev];
  return hipSuccess;
}

}  // namespace srhd
