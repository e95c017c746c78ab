// srhd_internal.hpp -- launch interface between the C ABI (srhd_capi.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/srhd.h"
#include "srhd_mlp.hpp"

namespace srhd {

// Records the message that srhd_last_error() returns (this thread) and returns code.
int set_error(int code, const char *fmt, ...);

struct GuessArgs {
  int kind;                // srhd_guess_kind
  int max_iter;
  const uint16_t *w;       // MLP weights (BF16), NULL for the analytic guess
  const float *bias;
  const float *norm;
  int features;            // SRHD_FEAT_*
  double gate;             // the network is consulted for L > gate
  __host__ __device__ MlpDev dev() const { return MlpDev{w, bias, norm, features, gate}; }
};

struct LevelArgs {
  int n_level;
  double dh[SRHD_MAX_LEVEL];
};

// eos_k: (Gamma - 1) / Gamma of the polytropic EoS, or 0 for TM
hipError_t launch_prim2cons(int dtype, int64_t n, const void *prim, void *cons, double eos_k,
                            hipStream_t s);
hipError_t launch_cons2prim(int dtype, int64_t n, const void *cons, void *prim, int8_t *status,
                            uint8_t *iters, const GuessArgs &g, double eos_k, hipStream_t s);
hipError_t launch_fill_ghosts(int dtype, int64_t n_patch, int ghost, int64_t n_src, const void *interior,
                              const int32_t *neighbor, void *padded, hipStream_t s);
hipError_t launch_cfl(int dtype, int64_t n_patch, const void *interior, const LevelArgs &lv,
                      double c_cfl, double *dt_lev, void *work, double eos_k, hipStream_t s);
hipError_t launch_stats_reset(srhd_step_stats *st, hipStream_t s);

struct StepArgs {
  int64_t n_patch;
  int ghost;
  const double *padded;
  const int8_t *level;
  int n_level;
  const double *dt_lev;
  double dh[SRHD_MAX_LEVEL];
  double theta;
  int riemann;
  int max_retry;
  GuessArgs guess;
  double *out;
  srhd_step_stats *stats;
  // gather mode: same-level patches whose ghost cells are read from the neighbours' interiors
  const double *cons;                   // [P][5][512] conserved interiors (padded unused)
  const void *prims;                    // [P][5][512] primitives in the bulk type
  const int32_t *neighbor;              // [P][27]
  void *prims_out;                      // [P][5][512] primitives of the output
  const unsigned long long *smax_in;    // S_max of the input (bit pattern), used when !dt_lev
  unsigned long long *smax_out;         // S_max of the output (zeroed by the launcher)
  double c_cfl;
  double *dt_out;                       // optional [n_level]: the dt the step used
  int xcd_remap;                        // give each XCD a contiguous range of patches
  // persistent schedule (queue != NULL): `groups` workgroups claim `chunk` patches at a time
  // from SRHD_QUEUE_WORDS counters (zeroed by the launcher)
  unsigned long long *queue;
  int groups;
  int chunk;
  int occ2;                             // the kernel variant that fits two workgroups per CU
  int energy;                           // srhd_energy: SRHD_ENERGY_TOTAL runs the original scheme
  int integrator;                       // srhd_integrator: SRHD_VL runs srhd_step_vl.hip's kernel
  double *flux_out;                     // padded layout: [P][6][5][64] boundary fluxes, or NULL
  double eos_k;                         // polytropic EoS: (Gamma - 1) / Gamma; 0 selects TM
  // precision guard of the FP32-bulk kernels (NULL: off): a patch whose tile holds a cell with
  // 1 + M^2 > kappa_max is listed here ([0] count, [1] claim counter, [2..] patch indices) and
  // stepped by the FP64 kernel in a second launch
  unsigned long long *defer;
  double kappa_max;
  // learned-guess split (NULL: off): the kernel without the network lists here the patches whose
  // tile holds a cell with L > guess.gate, and the learned kernel steps them in a second launch
  unsigned long long *net_list;
  // gather layout: network masks of the input state (per patch, the regions holding a cell with
  // L > gate; with the split on they decide the list before the step) and of the output (NULL:
  // not written), formed from the updated cells whose L exceeds net_gate
  const unsigned int *net_in;
  unsigned int *net_out;
  double net_gate;
  // set by the launcher for a launch over a list: the list it walks and the step counter
  // (srhd_step_stats word) each listed patch increments
  unsigned long long *list;
  int list_counter;
};

// Fluxes of the interfaces on the two faces (lower, upper) of direction d from the step's
// two-direction ring F[slot][5][NIF] (interface numbering of the step kernels: x fastest, the
// coordinate along d in [0, 9)) to flux_out[p][2 d + u][5][b * 8 + a]; 128 threads.
template <class T>
__device__ __forceinline__ void write_boundary_fluxes(double *flux_out, int64_t p, int d,
                                                      const T *ring, int nif, int t)
{
  const int u = t >> 6, a = t & 7, b = (t >> 3) & 7, c = u ? 8 : 0;
  const int r = d == 0 ? (b * 8 + a) * 9 + c : (d == 1 ? (b * 9 + c) * 8 + a : (c * 8 + b) * 8 + a);
  double *o = flux_out + ((p * 6 + 2 * d + u) * 5) * 64 + b * 8 + a;
#pragma unroll
  for (int f = 0; f < 5; ++f) o[f * 64] = (double)ring[f * nif + r];
}

hipError_t launch_step(int prec, const StepArgs &a, hipStream_t s);
// the VL integrator (srhd_step_vl.hip): analytic guess, reduced energy; padded and gather layouts
hipError_t launch_step_vl(int prec, const StepArgs &a, hipStream_t s);
hipError_t launch_step_vl_grid(int prec, const StepArgs &a, hipStream_t s);
int step_occupancy_vl(int prec, bool gather, bool occ2);

// per-precision launchers of the step (srhd_step_fp64.hip, srhd_step_mixed.hip, srhd_step_fp32.hip)
#define SRHD_STEP_MODE(name)                                                                   \
  hipError_t step_launch_##name(const StepArgs &a, bool gather, hipStream_t st);               \
  int step_occupancy_##name(bool gather, int kind, bool occ2);                                 \
  hipError_t grid_prims_##name(int64_t n_patch, const double *cons, void *prims,               \
                               unsigned long long *smax_bits, unsigned int *net_mask,           \
                               const GuessArgs &g, hipStream_t st);
SRHD_STEP_MODE(fp64)
SRHD_STEP_MODE(mixed)
SRHD_STEP_MODE(fp32)
#undef SRHD_STEP_MODE
// workgroups per CU, 0 on error; kind: 0 analytic guess, 1 learned guess, 2 original scheme,
// 3 polytropic EoS
int step_occupancy(int prec, bool gather, int kind, bool occ2);

size_t mlp_workspace_bytes(int64_t batch);
hipError_t launch_mlp_features(int dtype, int features, int64_t n, const void *cons, const void *prim,
                               float *feat, float *target, hipStream_t s);
hipError_t launch_mlp_forward(const MlpDev &m, int64_t n, const float *feat, float *y, hipStream_t s);
hipError_t launch_mlp_grad(const MlpDev &m, int64_t n, const float *feat, const float *target,
                           float *grad, float *loss, void *ws, hipStream_t s);
hipError_t launch_mlp_adam(float *master, float *m1, float *m2, const float *grad, int step,
                           float lr, uint16_t *w, float *bias, hipStream_t s);
hipError_t launch_step_grid(int prec, const StepArgs &a, hipStream_t s);
hipError_t launch_grid_prims(int prec, int64_t n_patch, const double *cons, void *prims,
                             unsigned long long *smax_bits, unsigned int *net_mask,
                             const GuessArgs &g, hipStream_t s);

// A second stream of the current device (default priority, non-blocking; created on first use
// and kept until the process ends) with two events, for work forked off a caller's stream and
// joined back into it.  The caller holds *lock from the fork's record to the join's wait, so
// that concurrent calls do not interleave their records of the shared events.
struct SideStream {
  hipStream_t stream;
  hipEvent_t fork, join;
  std::mutex *lock;
};
hipError_t side_stream(SideStream &out);

// AMR neighbour operations (srhd_amr.hip)
hipError_t launch_fill_ghosts_coarse(int64_t n_fine, int ghost, const int32_t *neighbor,
                                     const int32_t *parent, const int8_t *octant, int64_t n_coarse,
                                     int ghost_c, const double *coarse_old, const double *coarse_new,
                                     double alpha, double theta, double *fine_padded,
                                     unsigned long long *counts, hipStream_t s);
hipError_t launch_restrict(int64_t n_parent, const int32_t *parent_of, const int32_t *child,
                           int64_t n_fine, const double *fine, int64_t n_coarse, double *coarse,
                           hipStream_t s);
hipError_t launch_flux_accumulate(int64_t n, double *acc, const double *flux, double beta,
                                  double weight, hipStream_t s);
hipError_t launch_flux_correct(int64_t n_face, const int32_t *faces, int64_t n_coarse,
                               double *coarse, const double *coarse_flux, int64_t n_fine,
                               const double *fine_flux, double dh_c, unsigned long long *skipped,
                               hipStream_t s);

}  // namespace srhd
