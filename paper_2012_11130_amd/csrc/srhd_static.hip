// srhd_static.hip -- srhd_fluid_step_static: the patch step with its work buffers (the patch lists
// of the precision guard and the learned-guess split, the persistent schedule's queue counters)
// in a device array of this library instead of caller memory, for callers that cannot allocate.
#include <mutex>

#include "srhd_internal.hpp"

namespace {

// [0 .. SRHD_QUEUE_WORDS): queue counters; then the patch lists of the precision guard and the
// learned-guess split, 2 SRHD_STATIC_MAX_PATCH + 4 words.  Each GPU holds its own copy, found by
// hipGetSymbolAddress (the host-side name is not a device address).
constexpr size_t kWords = SRHD_QUEUE_WORDS + 2 * (size_t)SRHD_STATIC_MAX_PATCH + 4;
static __device__ __align__(256) unsigned long long scratch[kWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned long long *g_ptr[kMaxDevices] = {};

// The device address of the current device's scratch (set up on the first call on a device).
int scratch_ptr(unsigned long long **out)
{
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return SRHD_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return SRHD_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return SRHD_EHIP;
    g_ptr[dev] = (unsigned long long *)p;
  }
  *out = g_ptr[dev];
  return SRHD_OK;
}

}  // namespace

extern "C" int srhd_fluid_step_static(const srhd_patches *in, void *out, const double *dt_lev,
                                      const srhd_step_params *prm, srhd_step_stats *stats,
                                      void *stream)
{
  if (!in || !prm) return srhd_fluid_step(in, out, dt_lev, prm, stats, stream);   // its message
  if (in->n_patch > SRHD_STATIC_MAX_PATCH)
    return srhd::set_error(SRHD_EINVAL, "srhd_fluid_step_static: n_patch %lld exceeds the static "
                          "work array (%d patches); use srhd_fluid_step",
                          (long long)in->n_patch, SRHD_STATIC_MAX_PATCH);
  if (prm->defer || prm->sched.queue)
    return srhd::set_error(SRHD_EINVAL, "srhd_fluid_step_static: defer and sched.queue must be NULL "
                          "(the library's static array stands in for them)");
  unsigned long long *w = nullptr;
  int rc = scratch_ptr(&w);
  if (rc == SRHD_EHIP)
    return srhd::set_error(rc, "srhd_fluid_step_static: hipGetSymbolAddress of the static work "
                          "array failed");
  if (rc) return srhd::set_error(rc, "srhd_fluid_step_static: device index beyond %d", kMaxDevices);
  srhd_step_params p = *prm;
  p.sched.queue = p.sched.groups > 0 ? (uint64_t *)w : nullptr;
  p.defer = (uint64_t *)(w + SRHD_QUEUE_WORDS);
  return srhd_fluid_step(in, out, dt_lev, &p, stats, stream);
}
