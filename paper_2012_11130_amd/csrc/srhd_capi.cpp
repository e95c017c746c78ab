// srhd_capi.cpp -- the extern "C" entry points of libsrhd (declared in include/srhd.h):
// argument validation, error reporting and kernel launches on the caller's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "srhd_internal.hpp"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace

namespace srhd {

int set_error(int code, const char *fmt, ...)
{
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace srhd

namespace {

int hip_status(hipError_t e, const char *what)
{
  if (e == hipSuccess) return SRHD_OK;
  return fail(SRHD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// [a, a + an) and [b, b + bn) share no byte
bool disjoint(const void *a, size_t an, const void *b, size_t bn)
{
  const char *x = (const char *)a, *y = (const char *)b;
  return !(x < y + bn && y < x + an);
}

size_t dsize(int dtype) { return dtype == SRHD_F64 ? 8 : 4; }

bool valid_dtype(int dtype) { return dtype == SRHD_F64 || dtype == SRHD_F32; }

int check_guess(const srhd_guess *g, srhd::GuessArgs &out)
{
  out = srhd::GuessArgs{SRHD_GUESS_ANALYTIC, 30, nullptr, nullptr, nullptr, 0, 0.0};
  if (!g) return SRHD_OK;
  if (g->max_iter > 255) return fail(SRHD_EINVAL, "guess.max_iter %d exceeds 255", g->max_iter);
  out.max_iter = g->max_iter > 0 ? g->max_iter : 30;
  if (g->kind == SRHD_GUESS_ANALYTIC) return SRHD_OK;
  if (g->kind == SRHD_GUESS_MLP) {
    if (!g->mlp || !g->mlp->w_bf16 || !g->mlp->bias || !g->mlp->norm)
      return fail(SRHD_EINVAL, "learned guess: missing network parameters");
    if (!aligned(g->mlp->w_bf16, 16) || !aligned(g->mlp->bias, 4) || !aligned(g->mlp->norm, 4))
      return fail(SRHD_EINVAL, "learned guess: misaligned parameters (weights need 16 bytes)");
    if (g->mlp->features != SRHD_FEAT_CONS && g->mlp->features != SRHD_FEAT_L)
      return fail(SRHD_EINVAL, "learned guess: unknown feature set %d", g->mlp->features);
    if (!(g->mlp->gate_L >= 0.0)) return fail(SRHD_EINVAL, "learned guess: gate_L must be >= 0");
    out.kind = SRHD_GUESS_MLP;
    out.w = g->mlp->w_bf16;
    out.bias = g->mlp->bias;
    out.norm = g->mlp->norm;
    out.features = g->mlp->features;
    out.gate = g->mlp->gate_L;
    return SRHD_OK;
  }
  return fail(SRHD_EINVAL, "unknown guess kind %d", g->kind);
}

// Equation of state (include/srhd.h, srhd_eos): k = (Gamma - 1) / Gamma of the polytropic EoS,
// 0 for TM (NULL or kind SRHD_EOS_TM).
int check_eos(const srhd_eos *eos, double &k, const char *who)
{
  k = 0.0;
  if (!eos || eos->kind == SRHD_EOS_TM) return SRHD_OK;
  if (eos->kind != SRHD_EOS_POLYTROPIC) return fail(SRHD_EINVAL, "%s: unknown EoS kind %d", who, eos->kind);
  if (!(eos->gamma > 1.0 && eos->gamma <= 2.0))
    return fail(SRHD_EINVAL, "%s: polytropic gamma %g not in (1, 2]", who, eos->gamma);
  k = (eos->gamma - 1.0) / eos->gamma;
  return SRHD_OK;
}

// Energy variable and integrator of a step (include/srhd.h, srhd_energy, srhd_integrator): the
// original scheme has kernels for the padded layout with equal bulk and inversion types and the
// analytic guess; the VL integrator for both layouts, the analytic guess and the reduced energy.
int check_variant(int energy, int integrator, int prec, int guess_kind, int gather, const char *who)
{
  if (integrator != SRHD_MHM && integrator != SRHD_VL)
    return fail(SRHD_EINVAL, "%s: unknown integrator %d", who, integrator);
  if (energy != SRHD_ENERGY_REDUCED && energy != SRHD_ENERGY_TOTAL)
    return fail(SRHD_EINVAL, "%s: unknown energy variable %d", who, energy);
  if (integrator == SRHD_VL) {
    if (energy != SRHD_ENERGY_REDUCED)
      return fail(SRHD_EUNSUPPORTED, "%s: the VL integrator evolves the reduced energy only", who);
    if (guess_kind != SRHD_GUESS_ANALYTIC)
      return fail(SRHD_EUNSUPPORTED, "%s: the VL integrator takes the analytic guess only", who);
    return SRHD_OK;
  }
  if (energy == SRHD_ENERGY_REDUCED) return SRHD_OK;
  if (gather) return fail(SRHD_EUNSUPPORTED, "%s: the total-energy scheme runs on padded patches only", who);
  if (prec == SRHD_PREC_MIXED)
    return fail(SRHD_EUNSUPPORTED, "%s: the total-energy scheme runs in FP64 or FP32 only", who);
  if (guess_kind != SRHD_GUESS_ANALYTIC)
    return fail(SRHD_EUNSUPPORTED, "%s: the total-energy scheme takes the analytic guess only", who);
  return SRHD_OK;
}

// The EoS of a step: the polytropic EoS runs in the padded MUSCL-Hancock kernels with the
// reduced energy and the analytic guess.
int check_eos_step(const srhd_step_params *prm, int gather, double &k, const char *who)
{
  int rc = check_eos(&prm->eos, k, who);
  if (rc || k == 0.0) return rc;
  if (gather) return fail(SRHD_EUNSUPPORTED, "%s: the polytropic EoS runs on padded patches only", who);
  if (prm->integrator != SRHD_MHM || prm->energy != SRHD_ENERGY_REDUCED || prm->guess.kind != SRHD_GUESS_ANALYTIC)
    return fail(SRHD_EUNSUPPORTED, "%s: the polytropic EoS runs with MUSCL-Hancock, the reduced energy "
                "and the analytic guess only", who);
  return SRHD_OK;
}

// Launch schedule of a step (include/srhd.h, srhd_sched).
int check_sched(const srhd_sched &sc, int prec, int guess_kind, srhd::StepArgs &s, const char *who)
{
  s.queue = nullptr;
  s.groups = 0;
  s.chunk = 1;
  s.occ2 = 0;
  if (sc.occupancy != 0 && sc.occupancy != 2)
    return fail(SRHD_EINVAL, "%s: sched.occupancy %d is neither 0 nor 2", who, sc.occupancy);
  if (sc.occupancy == 2) {
    if (prec == SRHD_PREC_FP64)
      return fail(SRHD_EUNSUPPORTED, "%s: sched.occupancy 2 needs an FP32 bulk", who);
    s.occ2 = 1;
  }
  if (sc.groups == 0) return SRHD_OK;
  if (sc.groups < 0 || sc.groups > 65535)
    return fail(SRHD_EINVAL, "%s: sched.groups %d not in [0, 65535]", who, sc.groups);
  if (sc.chunk < 1 || sc.chunk > 64)
    return fail(SRHD_EINVAL, "%s: sched.chunk %d not in [1, 64]", who, sc.chunk);
  if (!sc.queue || !aligned(sc.queue, 8))
    return fail(SRHD_EINVAL, "%s: a persistent schedule needs an 8-byte aligned sched.queue", who);
  s.queue = (unsigned long long *)sc.queue;
  s.groups = sc.groups;
  s.chunk = sc.chunk;
  return SRHD_OK;
}

// Patch lists of a MUSCL-Hancock step (include/srhd.h, srhd_step_params): the precision guard of
// an FP32 bulk (kappa_max 0, off, or >= 1) and the learned-guess split (learned_split 0 or 1; a
// learned guess with a positive gate, the reduced energy and the TM EoS).  Their workspace of
// 2 n_patch + 4 words must be 8-byte aligned and overlap none of the call's other arrays
// (regions, n_region of them, NULL entries skipped).
int check_lists(const srhd_step_params *prm, const srhd::GuessArgs &g, double eos_k, int64_t n_patch,
                const void *const *regions, const size_t *sizes, int n_region, srhd::StepArgs &s,
                const char *who)
{
  s.defer = nullptr;
  s.kappa_max = 0.0;
  s.net_list = nullptr;
  s.net_in = nullptr;
  s.net_out = nullptr;
  s.net_gate = __builtin_huge_val();
  s.list = nullptr;
  s.list_counter = 0;
  const double k = prm->kappa_max;
  if (!(k == 0.0 || k >= 1.0))
    return fail(SRHD_EINVAL, "%s: kappa_max %g is neither 0 nor at least 1", who, k);
  if (prm->learned_split != 0 && prm->learned_split != 1)
    return fail(SRHD_EINVAL, "%s: learned_split %d is neither 0 nor 1", who, prm->learned_split);
  const bool mhm = prm->integrator == SRHD_MHM;
  const bool guard = k > 0.0 && prm->prec != SRHD_PREC_FP64 && mhm;
  const bool split = prm->learned_split && g.kind == SRHD_GUESS_MLP && g.gate > 0.0 && mhm &&
                     prm->energy == SRHD_ENERGY_REDUCED && eos_k == 0.0;
  if (!guard && !split) return SRHD_OK;
  if (!prm->defer || !aligned(prm->defer, 8))
    return fail(SRHD_EINVAL, "%s: the precision guard and the learned-guess split need an 8-byte "
                "aligned defer workspace", who);
  const size_t db = (2 * (size_t)n_patch + 4) * 8;
  for (int i = 0; i < n_region; ++i)
    if (regions[i] && !disjoint(prm->defer, db, regions[i], sizes[i]))
      return fail(SRHD_EINVAL, "%s: defer overlaps another array of the call", who);
  unsigned long long *d = (unsigned long long *)prm->defer;
  if (guard) {
    s.defer = d;
    s.kappa_max = k;
  }
  if (split) s.net_list = d + n_patch + 2;
  return SRHD_OK;
}

}  // namespace

extern "C" {

const char *srhd_last_error(void) { return g_err; }

int srhd_abi_version(void) { return SRHD_ABI_VERSION; }

int srhd_prim2cons(int dtype, int64_t n, const void *prim, void *cons, const srhd_eos *eos,
                   void *stream)
{
  if (!valid_dtype(dtype)) return fail(SRHD_EINVAL, "srhd_prim2cons: bad dtype %d", dtype);
  double k;
  int rc = check_eos(eos, k, "srhd_prim2cons");
  if (rc) return rc;
  if (n < 0) return fail(SRHD_EINVAL, "srhd_prim2cons: n = %lld < 0", (long long)n);
  if (n == 0) return SRHD_OK;
  if (!prim || !cons) return fail(SRHD_EINVAL, "srhd_prim2cons: NULL array");
  if (!aligned(prim, dsize(dtype)) || !aligned(cons, dsize(dtype)))
    return fail(SRHD_EINVAL, "srhd_prim2cons: misaligned array");
  const char *a = (const char *)prim, *b = (const char *)cons;
  size_t bytes = (size_t)n * 5 * dsize(dtype);
  if (a < b + bytes && b < a + bytes) return fail(SRHD_EINVAL, "srhd_prim2cons: prim and cons overlap");
  return hip_status(srhd::launch_prim2cons(dtype, n, prim, cons, k, (hipStream_t)stream),
                    "srhd_prim2cons");
}

int srhd_cons2prim(int dtype, int64_t n, const void *cons, void *prim, int8_t *status,
                   uint8_t *iters, const srhd_guess *guess, const srhd_eos *eos, void *stream)
{
  if (!valid_dtype(dtype)) return fail(SRHD_EINVAL, "srhd_cons2prim: bad dtype %d", dtype);
  if (n < 0) return fail(SRHD_EINVAL, "srhd_cons2prim: n = %lld < 0", (long long)n);
  srhd::GuessArgs g;
  int rc = check_guess(guess, g);
  if (rc) return rc;
  double k;
  rc = check_eos(eos, k, "srhd_cons2prim");
  if (rc) return rc;
  if (k > 0.0 && g.kind == SRHD_GUESS_MLP)
    return fail(SRHD_EUNSUPPORTED, "srhd_cons2prim: the learned guess is for the TM EoS only");
  if (n == 0) return SRHD_OK;
  if (!prim || !cons) return fail(SRHD_EINVAL, "srhd_cons2prim: NULL array");
  if (!aligned(prim, dsize(dtype)) || !aligned(cons, dsize(dtype)))
    return fail(SRHD_EINVAL, "srhd_cons2prim: misaligned array");
  const char *a = (const char *)prim, *b = (const char *)cons;
  size_t bytes = (size_t)n * 5 * dsize(dtype);
  if (a < b + bytes && b < a + bytes) return fail(SRHD_EINVAL, "srhd_cons2prim: prim and cons overlap");
  return hip_status(srhd::launch_cons2prim(dtype, n, cons, prim, status, iters, g, k,
                                           (hipStream_t)stream),
                    "srhd_cons2prim");
}

int srhd_fill_ghosts(int dtype, int64_t n_patch, int ghost, int64_t n_src, const void *interior,
                     const int32_t *neighbor, void *padded, void *stream)
{
  if (n_src < 0) return fail(SRHD_EINVAL, "srhd_fill_ghosts: n_src < 0");
  if (!valid_dtype(dtype)) return fail(SRHD_EINVAL, "srhd_fill_ghosts: bad dtype %d", dtype);
  if (n_patch < 0) return fail(SRHD_EINVAL, "srhd_fill_ghosts: n_patch < 0");
  if (ghost < 0 || ghost > 8) return fail(SRHD_EINVAL, "srhd_fill_ghosts: ghost %d not in [0, 8]", ghost);
  if (n_patch == 0) return SRHD_OK;
  if (!interior || !neighbor || !padded) return fail(SRHD_EINVAL, "srhd_fill_ghosts: NULL array");
  if (!aligned(interior, dsize(dtype)) || !aligned(padded, dsize(dtype)) || !aligned(neighbor, 4))
    return fail(SRHD_EINVAL, "srhd_fill_ghosts: misaligned array");
  return hip_status(srhd::launch_fill_ghosts(dtype, n_patch, ghost, n_src, interior, neighbor, padded,
                                             (hipStream_t)stream),
                    "srhd_fill_ghosts");
}

// ---------------------------------------------------------------- AMR neighbour operations
int srhd_fill_ghosts_coarse(int64_t n_fine, int ghost, const int32_t *neighbor,
                            const int32_t *parent, const int8_t *octant, int64_t n_coarse,
                            int ghost_c, const double *coarse_old, const double *coarse_new,
                            double alpha, double theta, double *fine_padded, uint64_t *counts,
                            void *stream)
{
  const char *who = "srhd_fill_ghosts_coarse";
  if (n_fine < 0 || n_coarse < 0) return fail(SRHD_EINVAL, "%s: negative count", who);
  if (ghost < 1 || ghost > 8) return fail(SRHD_EINVAL, "%s: ghost %d not in [1, 8]", who, ghost);
  if (ghost_c < ghost / 2 + 2 || ghost_c > 8)
    return fail(SRHD_EINVAL, "%s: ghost_c %d not in [%d, 8]", who, ghost_c, ghost / 2 + 2);
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(SRHD_EINVAL, "%s: alpha %g not in [0, 1]", who, alpha);
  if (!(theta >= 0.0 && theta <= 2.0)) return fail(SRHD_EINVAL, "%s: theta %g not in [0, 2]", who, theta);
  if (n_fine == 0) return SRHD_OK;
  if (!neighbor || !parent || !octant || !coarse_old || !fine_padded)
    return fail(SRHD_EINVAL, "%s: NULL array", who);
  if (!aligned(neighbor, 4) || !aligned(parent, 4) || !aligned(coarse_old, 8) ||
      !aligned(fine_padded, 8) || (coarse_new && !aligned(coarse_new, 8)) || (counts && !aligned(counts, 8)))
    return fail(SRHD_EINVAL, "%s: misaligned array", who);
  const int N = 8 + 2 * ghost, Nc = 8 + 2 * ghost_c;
  const size_t fb = (size_t)n_fine * 5 * N * N * N * 8, cb = (size_t)n_coarse * 5 * Nc * Nc * Nc * 8;
  if (!disjoint(fine_padded, fb, coarse_old, cb) || (coarse_new && !disjoint(fine_padded, fb, coarse_new, cb)))
    return fail(SRHD_EINVAL, "%s: fine_padded overlaps a coarse array", who);
  return hip_status(srhd::launch_fill_ghosts_coarse(n_fine, ghost, neighbor, parent, octant, n_coarse,
                                                    ghost_c, coarse_old, coarse_new, alpha, theta,
                                                    fine_padded, (unsigned long long *)counts,
                                                    (hipStream_t)stream),
                    who);
}

int srhd_restrict(int64_t n_parent, const int32_t *parent_of, const int32_t *child,
                  int64_t n_fine, const double *fine, int64_t n_coarse, double *coarse,
                  void *stream)
{
  const char *who = "srhd_restrict";
  if (n_parent < 0 || n_fine < 0 || n_coarse < 0) return fail(SRHD_EINVAL, "%s: negative count", who);
  if (n_parent > 0x7fffffffLL) return fail(SRHD_EINVAL, "%s: too many parents", who);
  if (n_parent == 0) return SRHD_OK;
  if (!parent_of || !child || !fine || !coarse) return fail(SRHD_EINVAL, "%s: NULL array", who);
  if (!aligned(parent_of, 4) || !aligned(child, 4) || !aligned(fine, 8) || !aligned(coarse, 8))
    return fail(SRHD_EINVAL, "%s: misaligned array", who);
  if (!disjoint(fine, (size_t)n_fine * 5 * 512 * 8, coarse, (size_t)n_coarse * 5 * 512 * 8))
    return fail(SRHD_EINVAL, "%s: fine and coarse overlap", who);
  return hip_status(srhd::launch_restrict(n_parent, parent_of, child, n_fine, fine, n_coarse, coarse,
                                          (hipStream_t)stream),
                    who);
}

int srhd_flux_accumulate(int64_t n, double *acc, const double *flux, double beta, double weight,
                         void *stream)
{
  const char *who = "srhd_flux_accumulate";
  if (n < 0) return fail(SRHD_EINVAL, "%s: n < 0", who);
  if (n == 0) return SRHD_OK;
  if (!acc || !flux) return fail(SRHD_EINVAL, "%s: NULL array", who);
  if (!aligned(acc, 8) || !aligned(flux, 8)) return fail(SRHD_EINVAL, "%s: misaligned array", who);
  if (!disjoint(acc, (size_t)n * 8, flux, (size_t)n * 8)) return fail(SRHD_EINVAL, "%s: acc overlaps flux", who);
  return hip_status(srhd::launch_flux_accumulate(n, acc, flux, beta, weight, (hipStream_t)stream), who);
}

int srhd_flux_correct(int64_t n_face, const int32_t *faces, int64_t n_coarse, double *coarse,
                      const double *coarse_flux, int64_t n_fine, const double *fine_flux,
                      double dh_c, uint64_t *skipped, void *stream)
{
  const char *who = "srhd_flux_correct";
  if (n_face < 0 || n_coarse < 0 || n_fine < 0) return fail(SRHD_EINVAL, "%s: negative count", who);
  if (!(dh_c > 0.0)) return fail(SRHD_EINVAL, "%s: dh_c must be positive", who);
  if (n_face == 0) return SRHD_OK;
  if (!faces || !coarse || !coarse_flux || !fine_flux) return fail(SRHD_EINVAL, "%s: NULL array", who);
  if (!aligned(faces, 4) || !aligned(coarse, 8) || !aligned(coarse_flux, 8) || !aligned(fine_flux, 8) ||
      (skipped && !aligned(skipped, 8)))
    return fail(SRHD_EINVAL, "%s: misaligned array", who);
  const size_t cb = (size_t)n_coarse * 5 * 512 * 8;
  if (!disjoint(coarse, cb, coarse_flux, (size_t)n_coarse * 6 * 5 * 64 * 8) ||
      !disjoint(coarse, cb, fine_flux, (size_t)n_fine * 6 * 5 * 64 * 8))
    return fail(SRHD_EINVAL, "%s: coarse overlaps a flux array", who);
  return hip_status(srhd::launch_flux_correct(n_face, faces, n_coarse, coarse, coarse_flux, n_fine,
                                              fine_flux, dh_c, (unsigned long long *)skipped,
                                              (hipStream_t)stream),
                    who);
}

size_t srhd_cfl_work_bytes(void) { return 256; }

int srhd_cfl_dt(int dtype, int64_t n_patch, const void *interior, int n_level, const double *dh,
                double c_cfl, double *dt_lev, void *work, const srhd_eos *eos, void *stream)
{
  if (!valid_dtype(dtype)) return fail(SRHD_EINVAL, "srhd_cfl_dt: bad dtype %d", dtype);
  double k;
  int rc = check_eos(eos, k, "srhd_cfl_dt");
  if (rc) return rc;
  if (n_patch < 0) return fail(SRHD_EINVAL, "srhd_cfl_dt: n_patch < 0");
  if (n_level < 1 || n_level > SRHD_MAX_LEVEL)
    return fail(SRHD_EINVAL, "srhd_cfl_dt: n_level %d not in [1, %d]", n_level, SRHD_MAX_LEVEL);
  if (!dh || !dt_lev || !work || (n_patch > 0 && !interior))
    return fail(SRHD_EINVAL, "srhd_cfl_dt: NULL argument");
  if (!(c_cfl > 0.0)) return fail(SRHD_EINVAL, "srhd_cfl_dt: c_cfl must be positive");
  if (!aligned(work, 8) || !aligned(dt_lev, 8)) return fail(SRHD_EINVAL, "srhd_cfl_dt: misaligned buffer");
  srhd::LevelArgs lv;
  lv.n_level = n_level;
  for (int l = 0; l < SRHD_MAX_LEVEL; ++l) lv.dh[l] = l < n_level ? dh[l] : 0.0;
  for (int l = 0; l < n_level; ++l)
    if (!(dh[l] > 0.0)) return fail(SRHD_EINVAL, "srhd_cfl_dt: dh[%d] must be positive", l);
  return hip_status(srhd::launch_cfl(dtype, n_patch, interior, lv, c_cfl, dt_lev, work, k,
                                     (hipStream_t)stream),
                    "srhd_cfl_dt");
}

int srhd_stats_reset(srhd_step_stats *stats, void *stream)
{
  if (!stats) return fail(SRHD_EINVAL, "srhd_stats_reset: NULL stats");
  return hip_status(srhd::launch_stats_reset(stats, (hipStream_t)stream), "srhd_stats_reset");
}

int srhd_fluid_step(const srhd_patches *in, void *out, const double *dt_lev,
                    const srhd_step_params *prm, srhd_step_stats *stats, void *stream)
{
  if (!in || !prm) return fail(SRHD_EINVAL, "srhd_fluid_step: NULL descriptor");
  if (in->n_patch < 0) return fail(SRHD_EINVAL, "srhd_fluid_step: n_patch < 0");
  if (in->dtype != SRHD_F64)
    return fail(SRHD_EUNSUPPORTED, "srhd_fluid_step: patch storage must be FP64");
  if (in->ghost < 2 || in->ghost > 8)
    return fail(SRHD_EINVAL, "srhd_fluid_step: ghost %d not in [2, 8]", in->ghost);
  if (in->n_level < 1 || in->n_level > SRHD_MAX_LEVEL)
    return fail(SRHD_EINVAL, "srhd_fluid_step: n_level %d not in [1, %d]", in->n_level, SRHD_MAX_LEVEL);
  if (in->n_patch > 0x7fffffffLL) return fail(SRHD_EINVAL, "srhd_fluid_step: too many patches");
  if (prm->prec != SRHD_PREC_FP64 && prm->prec != SRHD_PREC_MIXED && prm->prec != SRHD_PREC_FP32)
    return fail(SRHD_EINVAL, "srhd_fluid_step: bad precision %d", prm->prec);
  if (prm->riemann != SRHD_HLLC && prm->riemann != SRHD_HLLE)
    return fail(SRHD_EINVAL, "srhd_fluid_step: bad Riemann solver %d", prm->riemann);
  if (!(prm->theta >= 0.0 && prm->theta <= 2.0))
    return fail(SRHD_EINVAL, "srhd_fluid_step: theta %g not in [0, 2]", prm->theta);
  if (prm->max_retry < 0 || prm->max_retry > 64)
    return fail(SRHD_EINVAL, "srhd_fluid_step: max_retry %d not in [0, 64]", prm->max_retry);
  srhd::GuessArgs g;
  int rc = check_guess(&prm->guess, g);
  if (rc) return rc;
  rc = check_variant(prm->energy, prm->integrator, prm->prec, g.kind, 0, "srhd_fluid_step");
  if (rc) return rc;
  double eos_k;
  rc = check_eos_step(prm, 0, eos_k, "srhd_fluid_step");
  if (rc) return rc;
  if (prm->integrator == SRHD_VL && in->ghost < 3)
    return fail(SRHD_EINVAL, "srhd_fluid_step: the VL integrator needs ghost >= 3 (got %d)", in->ghost);
  if (in->n_patch == 0) return SRHD_OK;
  if (!in->padded || !out || !dt_lev) return fail(SRHD_EINVAL, "srhd_fluid_step: NULL array");
  if (!aligned(in->padded, 8) || !aligned(out, 8) || !aligned(dt_lev, 8))
    return fail(SRHD_EINVAL, "srhd_fluid_step: misaligned array");
  for (int l = 0; l < in->n_level; ++l)
    if (!(in->dh[l] > 0.0)) return fail(SRHD_EINVAL, "srhd_fluid_step: dh[%d] must be positive", l);
  int N = 8 + 2 * in->ghost;
  const char *a = (const char *)in->padded, *b = (const char *)out;
  size_t abytes = (size_t)in->n_patch * 5 * N * N * N * 8, bbytes = (size_t)in->n_patch * 5 * 512 * 8;
  if (a < b + bbytes && b < a + abytes) return fail(SRHD_EINVAL, "srhd_fluid_step: out overlaps the input");
  srhd::StepArgs s;
  s.n_patch = in->n_patch;
  s.ghost = in->ghost;
  s.padded = (const double *)in->padded;
  s.level = in->level;
  s.n_level = in->n_level;
  s.dt_lev = dt_lev;
  for (int l = 0; l < SRHD_MAX_LEVEL; ++l) s.dh[l] = l < in->n_level ? in->dh[l] : 1.0;
  s.theta = prm->theta;
  s.riemann = prm->riemann;
  s.max_retry = prm->max_retry;
  s.guess = g;
  s.out = (double *)out;
  s.stats = stats;
  s.cons = nullptr;
  s.prims = nullptr;
  s.neighbor = nullptr;
  s.prims_out = nullptr;
  s.smax_in = nullptr;
  s.smax_out = nullptr;
  s.c_cfl = 0.0;
  s.dt_out = nullptr;
  s.xcd_remap = 0;
  s.energy = prm->energy;
  s.integrator = prm->integrator;
  s.eos_k = eos_k;
  s.flux_out = prm->flux_out;
  if (s.flux_out) {
    if (!aligned(s.flux_out, 8)) return fail(SRHD_EINVAL, "srhd_fluid_step: misaligned flux_out");
    if (!disjoint(s.flux_out, (size_t)in->n_patch * 6 * 5 * 64 * 8, a, abytes) ||
        !disjoint(s.flux_out, (size_t)in->n_patch * 6 * 5 * 64 * 8, b, bbytes))
      return fail(SRHD_EINVAL, "srhd_fluid_step: flux_out overlaps the patches");
  }
  rc = check_sched(prm->sched, prm->prec, g.kind, s, "srhd_fluid_step");
  if (rc) return rc;
  if (s.queue) {
    const char *q = (const char *)s.queue;
    if (q < b + bbytes && b < q + SRHD_QUEUE_WORDS * 8)
      return fail(SRHD_EINVAL, "srhd_fluid_step: sched.queue overlaps out");
  }
  {
    const void *reg[4] = {in->padded, out, s.flux_out, s.queue};
    const size_t sz[4] = {abytes, bbytes, (size_t)in->n_patch * 6 * 5 * 64 * 8, SRHD_QUEUE_WORDS * 8};
    rc = check_lists(prm, g, eos_k, in->n_patch, reg, sz, 4, s, "srhd_fluid_step");
    if (rc) return rc;
  }
  return hip_status(srhd::launch_step(prm->prec, s, (hipStream_t)stream), "srhd_fluid_step");
}

int srhd_step_occupancy(const srhd_step_params *prm, int gather)
{
  if (!prm) return fail(SRHD_EINVAL, "srhd_step_occupancy: NULL parameters");
  const int prec = prm->prec, guess_kind = prm->guess.kind, occupancy = prm->sched.occupancy;
  if (prec != SRHD_PREC_FP64 && prec != SRHD_PREC_MIXED && prec != SRHD_PREC_FP32)
    return fail(SRHD_EINVAL, "srhd_step_occupancy: bad precision %d", prec);
  if (guess_kind != SRHD_GUESS_ANALYTIC && guess_kind != SRHD_GUESS_MLP)
    return fail(SRHD_EINVAL, "srhd_step_occupancy: unknown guess kind %d", guess_kind);
  if (occupancy != 0 && occupancy != 2)
    return fail(SRHD_EINVAL, "srhd_step_occupancy: occupancy %d is neither 0 nor 2", occupancy);
  if (occupancy == 2 && prec == SRHD_PREC_FP64)
    return fail(SRHD_EUNSUPPORTED, "srhd_step_occupancy: occupancy 2 needs an FP32 bulk");
  int rc = check_variant(prm->energy, prm->integrator, prec, guess_kind, gather, "srhd_step_occupancy");
  if (rc) return rc;
  double eos_k;
  rc = check_eos_step(prm, gather, eos_k, "srhd_step_occupancy");
  if (rc) return rc;
  const int kind = prm->energy == SRHD_ENERGY_TOTAL ? 2
                 : (eos_k > 0.0 ? 3 : (guess_kind == SRHD_GUESS_MLP ? 1 : 0));
  int n = prm->integrator == SRHD_VL ? srhd::step_occupancy_vl(prec, gather != 0, occupancy == 2)
                                     : srhd::step_occupancy(prec, gather != 0, kind, occupancy == 2);
  if (n <= 0) return fail(SRHD_EHIP, "srhd_step_occupancy: occupancy query failed");
  return n;
}

}  // extern "C"

namespace {

// Times `run(trial)` for every candidate schedule and leaves the fastest in prm->sched.
template <class Run>
int autotune(srhd_step_params *prm, int gather, int reps, srhd_tune_entry *table, int table_cap,
             int *n_table, void *stream, const char *who, Run run)
{
  if (!prm) return fail(SRHD_EINVAL, "%s: NULL parameters", who);
  if (!prm->sched.queue) return fail(SRHD_EINVAL, "%s: prm->sched.queue must be set", who);
  if (reps < 1 || reps > 100) return fail(SRHD_EINVAL, "%s: reps %d not in [1, 100]", who, reps);
  if (table_cap < 0) return fail(SRHD_EINVAL, "%s: table_cap < 0", who);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_status(e, who);
  struct Cand { int groups, chunk, occ; };
  Cand cand[20];
  int nc = 0;
  const bool two = prm->prec != SRHD_PREC_FP64;
  for (int occ : {0, 2}) {
    if (occ == 2 && !two) continue;
    srhd_step_params q = *prm;
    q.sched.occupancy = occ;
    int per_cu = srhd_step_occupancy(&q, gather);
    if (per_cu <= 0) return per_cu < 0 ? per_cu : fail(SRHD_EHIP, "%s: occupancy 0", who);
    cand[nc++] = {0, 1, occ};
    for (int m : {1, 2, 4})
      for (int c : {1, 2, 4}) {
        long g = (long)m * per_cu * cus;
        cand[nc++] = {(int)(g > 65535 ? 65535 : g), c, occ};
      }
  }
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_status(e, who);
  }
  srhd_step_params trial = *prm;
  int best = -1, rc = SRHD_OK;
  float best_ms = 0.0f;
  if (n_table) *n_table = 0;
  for (int i = 0; i < nc && rc == SRHD_OK; ++i) {
    trial.sched.groups = cand[i].groups;
    trial.sched.chunk = cand[i].chunk;
    trial.sched.occupancy = cand[i].occ;
    rc = run(&trial);                                           // warm-up
    if (rc) break;
    e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && rc == SRHD_OK && e == hipSuccess; ++r) rc = run(&trial);
    if (rc) break;
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { rc = hip_status(e, who); break; }
    ms /= (float)reps;
    if (table && i < table_cap) table[i] = srhd_tune_entry{cand[i].groups, cand[i].chunk, cand[i].occ, ms};
    if (n_table && i < table_cap) *n_table = i + 1;
    if (best < 0 || ms < best_ms) { best = i; best_ms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  prm->sched.groups = cand[best].groups;
  prm->sched.chunk = cand[best].chunk;
  prm->sched.occupancy = cand[best].occ;
  return SRHD_OK;
}

}  // namespace

extern "C" {

int srhd_autotune_step(const srhd_patches *in, void *out, const double *dt_lev,
                       srhd_step_params *prm, int reps, srhd_tune_entry *table, int table_cap,
                       int *n_table, void *stream)
{
  return autotune(prm, 0, reps, table, table_cap, n_table, stream, "srhd_autotune_step",
                  [&](const srhd_step_params *t) { return srhd_fluid_step(in, out, dt_lev, t, nullptr, stream); });
}

int srhd_autotune_step_grid(const srhd_grid *in, const uint64_t *smax_in, double c_cfl,
                            const double *dt_lev, double *cons_out, void *prims_out,
                            uint64_t *smax_out, uint32_t *net_out, srhd_step_params *prm,
                            int reps, srhd_tune_entry *table, int table_cap, int *n_table,
                            void *stream)
{
  return autotune(prm, 1, reps, table, table_cap, n_table, stream, "srhd_autotune_step_grid",
                  [&](const srhd_step_params *t) {
                    return srhd_fluid_step_grid(in, smax_in, c_cfl, dt_lev, cons_out, prims_out,
                                                smax_out, net_out, nullptr, t, nullptr, stream);
                  });
}

int srhd_grid_prims(int prec, int64_t n_patch, const double *cons, void *prims,
                    uint64_t *smax_bits, uint32_t *net_mask, const srhd_guess *guess,
                    void *stream)
{
  srhd::GuessArgs g;
  int rc = check_guess(guess, g);
  if (rc) return rc;
  if (prec != SRHD_PREC_FP64 && prec != SRHD_PREC_MIXED && prec != SRHD_PREC_FP32)
    return fail(SRHD_EINVAL, "srhd_grid_prims: bad precision %d", prec);
  if (n_patch < 0) return fail(SRHD_EINVAL, "srhd_grid_prims: n_patch < 0");
  if (!smax_bits || (n_patch > 0 && (!cons || !prims)))
    return fail(SRHD_EINVAL, "srhd_grid_prims: NULL argument");
  size_t ps = prec == SRHD_PREC_FP64 ? 8 : 4;
  if (!aligned(cons, 8) || !aligned(prims, ps) || !aligned(smax_bits, 8) || !aligned(net_mask, 4))
    return fail(SRHD_EINVAL, "srhd_grid_prims: misaligned array");
  const char *a = (const char *)cons, *b = (const char *)prims;
  size_t ab = (size_t)n_patch * 5 * 512 * 8, bb = (size_t)n_patch * 5 * 512 * ps;
  if (n_patch > 0 && a < b + bb && b < a + ab)
    return fail(SRHD_EINVAL, "srhd_grid_prims: prims overlap cons");
  if (net_mask) {
    const size_t nb = (size_t)n_patch * 4;
    if (!disjoint(net_mask, nb, cons, ab) || !disjoint(net_mask, nb, prims, bb) ||
        !disjoint(net_mask, nb, smax_bits, 8))
      return fail(SRHD_EINVAL, "srhd_grid_prims: net_mask overlaps another array");
  }
  return hip_status(srhd::launch_grid_prims(prec, n_patch, cons, prims,
                                            (unsigned long long *)smax_bits, net_mask, g,
                                            (hipStream_t)stream),
                    "srhd_grid_prims");
}

static int check_mlp(const srhd_mlp *m, const char *who)
{
  if (!m || !m->w_bf16 || !m->bias || !m->norm) return fail(SRHD_EINVAL, "%s: missing network parameters", who);
  if (!aligned(m->w_bf16, 16) || !aligned(m->bias, 4) || !aligned(m->norm, 4))
    return fail(SRHD_EINVAL, "%s: misaligned parameters (weights need 16 bytes)", who);
  return SRHD_OK;
}

int srhd_mlp_features(int dtype, int features, int64_t n, const void *cons, const void *prim,
                      float *feat, float *target, void *stream)
{
  if (!valid_dtype(dtype)) return fail(SRHD_EINVAL, "srhd_mlp_features: bad dtype %d", dtype);
  if (features != SRHD_FEAT_CONS && features != SRHD_FEAT_L)
    return fail(SRHD_EINVAL, "srhd_mlp_features: unknown feature set %d", features);
  if (n < 0) return fail(SRHD_EINVAL, "srhd_mlp_features: n < 0");
  if (n == 0) return SRHD_OK;
  if (!cons || !feat) return fail(SRHD_EINVAL, "srhd_mlp_features: NULL array");
  if (!aligned(cons, dsize(dtype)) || !aligned(feat, 4) || !aligned(prim, dsize(dtype)) || !aligned(target, 4))
    return fail(SRHD_EINVAL, "srhd_mlp_features: misaligned array");
  if ((prim == nullptr) != (target == nullptr))
    return fail(SRHD_EINVAL, "srhd_mlp_features: prim and target go together");
  return hip_status(srhd::launch_mlp_features(dtype, features, n, cons, prim, feat, target, (hipStream_t)stream),
                    "srhd_mlp_features");
}

int srhd_mlp_forward(const srhd_mlp *m, int64_t n, const float *feat, float *y, void *stream)
{
  int rc = check_mlp(m, "srhd_mlp_forward");
  if (rc) return rc;
  if (n < 0) return fail(SRHD_EINVAL, "srhd_mlp_forward: n < 0");
  if (n == 0) return SRHD_OK;
  if (!feat || !y) return fail(SRHD_EINVAL, "srhd_mlp_forward: NULL array");
  if (!aligned(feat, 4) || !aligned(y, 4)) return fail(SRHD_EINVAL, "srhd_mlp_forward: misaligned array");
  srhd::MlpDev d = {m->w_bf16, m->bias, m->norm, m->features, m->gate_L};
  return hip_status(srhd::launch_mlp_forward(d, n, feat, y, (hipStream_t)stream), "srhd_mlp_forward");
}

size_t srhd_mlp_workspace_bytes(int64_t batch) { return batch > 0 ? srhd::mlp_workspace_bytes(batch) : 0; }

int srhd_mlp_grad(const srhd_mlp *m, int64_t batch, const float *feat, const float *target,
                  float *grad, float *loss, void *ws, void *stream)
{
  int rc = check_mlp(m, "srhd_mlp_grad");
  if (rc) return rc;
  if (batch <= 0 || batch > (1LL << 31)) return fail(SRHD_EINVAL, "srhd_mlp_grad: batch must be in [1, 2^31]");
  if (!feat || !target || !grad || !loss || !ws) return fail(SRHD_EINVAL, "srhd_mlp_grad: NULL array");
  if (!aligned(feat, 4) || !aligned(target, 4) || !aligned(grad, 4) || !aligned(loss, 4) || !aligned(ws, 4))
    return fail(SRHD_EINVAL, "srhd_mlp_grad: misaligned array");
  srhd::MlpDev d = {m->w_bf16, m->bias, m->norm, m->features, m->gate_L};
  return hip_status(srhd::launch_mlp_grad(d, batch, feat, target, grad, loss, ws, (hipStream_t)stream),
                    "srhd_mlp_grad");
}

int srhd_mlp_adam(float *master, float *m1, float *m2, const float *grad, int step, float lr,
                  uint16_t *w_bf16, float *bias, void *stream)
{
  if (!master || !m1 || !m2 || !grad || !w_bf16 || !bias) return fail(SRHD_EINVAL, "srhd_mlp_adam: NULL array");
  if (step < 1) return fail(SRHD_EINVAL, "srhd_mlp_adam: step counts from 1");
  if (!(lr > 0.0f)) return fail(SRHD_EINVAL, "srhd_mlp_adam: lr must be positive");
  return hip_status(srhd::launch_mlp_adam(master, m1, m2, grad, step, lr, w_bf16, bias, (hipStream_t)stream),
                    "srhd_mlp_adam");
}

int srhd_fluid_step_grid(const srhd_grid *in, const uint64_t *smax_in, double c_cfl,
                         const double *dt_lev, double *cons_out, void *prims_out,
                         uint64_t *smax_out, uint32_t *net_out, double *dt_used,
                         const srhd_step_params *prm, srhd_step_stats *stats, void *stream)
{
  if (!in || !prm) return fail(SRHD_EINVAL, "srhd_fluid_step_grid: NULL descriptor");
  if (in->n_patch < 0) return fail(SRHD_EINVAL, "srhd_fluid_step_grid: n_patch < 0");
  if (in->n_patch > (0x7fffffffLL / 8) * 8 - 8)
    return fail(SRHD_EINVAL, "srhd_fluid_step_grid: too many patches");
  if (in->n_level < 1 || in->n_level > SRHD_MAX_LEVEL)
    return fail(SRHD_EINVAL, "srhd_fluid_step_grid: n_level %d not in [1, %d]", in->n_level, SRHD_MAX_LEVEL);
  if (prm->prec != SRHD_PREC_FP64 && prm->prec != SRHD_PREC_MIXED && prm->prec != SRHD_PREC_FP32)
    return fail(SRHD_EINVAL, "srhd_fluid_step_grid: bad precision %d", prm->prec);
  if (prm->riemann != SRHD_HLLC && prm->riemann != SRHD_HLLE)
    return fail(SRHD_EINVAL, "srhd_fluid_step_grid: bad Riemann solver %d", prm->riemann);
  if (!(prm->theta >= 0.0 && prm->theta <= 2.0))
    return fail(SRHD_EINVAL, "srhd_fluid_step_grid: theta %g not in [0, 2]", prm->theta);
  if (prm->max_retry < 0 || prm->max_retry > 64)
    return fail(SRHD_EINVAL, "srhd_fluid_step_grid: max_retry %d not in [0, 64]", prm->max_retry);
  srhd::GuessArgs g;
  int rc = check_guess(&prm->guess, g);
  if (rc) return rc;
  rc = check_variant(prm->energy, prm->integrator, prm->prec, g.kind, 1, "srhd_fluid_step_grid");
  if (rc) return rc;
  double eos_k;
  rc = check_eos_step(prm, 1, eos_k, "srhd_fluid_step_grid");
  if (rc) return rc;
  if (!smax_out) return fail(SRHD_EINVAL, "srhd_fluid_step_grid: NULL smax_out");
  if (!dt_lev && (!smax_in || !(c_cfl > 0.0)))
    return fail(SRHD_EINVAL, "srhd_fluid_step_grid: need dt_lev, or smax_in and c_cfl > 0");
  for (int l = 0; l < in->n_level; ++l)
    if (!(in->dh[l] > 0.0)) return fail(SRHD_EINVAL, "srhd_fluid_step_grid: dh[%d] must be positive", l);
  size_t ps = prm->prec == SRHD_PREC_FP64 ? 8 : 4;
  if (in->n_patch > 0) {
    if (!in->cons || !in->prims || !in->neighbor || !cons_out || !prims_out)
      return fail(SRHD_EINVAL, "srhd_fluid_step_grid: NULL array");
    if (!aligned(in->cons, 8) || !aligned(cons_out, 8) || !aligned(in->prims, ps) ||
        !aligned(prims_out, ps) || !aligned(in->neighbor, 4) || !aligned(smax_out, 8) ||
        !aligned(net_out, 4) || !aligned(in->net_mask, 4))
      return fail(SRHD_EINVAL, "srhd_fluid_step_grid: misaligned array");
    size_t cb = (size_t)in->n_patch * 5 * 512 * 8, pb = (size_t)in->n_patch * 5 * 512 * ps;
    struct R { const char *p; size_t n; } ins[2] = {{(const char *)in->cons, cb}, {(const char *)in->prims, pb}},
        outs[2] = {{(const char *)cons_out, cb}, {(const char *)prims_out, pb}};
    for (auto &i : ins)
      for (auto &o : outs)
        if (i.p < o.p + o.n && o.p < i.p + i.n)
          return fail(SRHD_EINVAL, "srhd_fluid_step_grid: an output overlaps an input");
    if (outs[0].p < outs[1].p + outs[1].n && outs[1].p < outs[0].p + outs[0].n)
      return fail(SRHD_EINVAL, "srhd_fluid_step_grid: cons_out overlaps prims_out");
    if (net_out) {
      const size_t nb = (size_t)in->n_patch * 4;
      const void *others[6] = {in->cons, in->prims, cons_out, prims_out, smax_out, in->net_mask};
      const size_t osz[6] = {cb, pb, cb, pb, 8, nb};
      for (int i = 0; i < 6; ++i)
        if (others[i] && !disjoint(net_out, nb, others[i], osz[i]))
          return fail(SRHD_EINVAL, "srhd_fluid_step_grid: net_out overlaps another array");
    }
  }
  srhd::StepArgs s;
  s.n_patch = in->n_patch;
  s.ghost = 3;
  s.padded = nullptr;
  s.level = in->level;
  s.n_level = in->n_level;
  s.dt_lev = dt_lev;
  for (int l = 0; l < SRHD_MAX_LEVEL; ++l) s.dh[l] = l < in->n_level ? in->dh[l] : 1.0;
  s.theta = prm->theta;
  s.riemann = prm->riemann;
  s.max_retry = prm->max_retry;
  s.guess = g;
  s.out = cons_out;
  s.stats = stats;
  s.cons = in->cons;
  s.prims = in->prims;
  s.neighbor = in->neighbor;
  s.prims_out = prims_out;
  s.smax_in = (const unsigned long long *)smax_in;
  s.smax_out = (unsigned long long *)smax_out;
  s.c_cfl = c_cfl;
  s.dt_out = dt_used;
  s.xcd_remap = 1;
  s.energy = SRHD_ENERGY_REDUCED;
  s.integrator = prm->integrator;
  s.eos_k = 0.0;
  s.flux_out = nullptr;
  if (prm->flux_out)
    return fail(SRHD_EUNSUPPORTED, "srhd_fluid_step_grid: boundary fluxes are written by srhd_fluid_step only");
  rc = check_sched(prm->sched, prm->prec, g.kind, s, "srhd_fluid_step_grid");
  if (rc) return rc;
  {
    const size_t cb = (size_t)in->n_patch * 5 * 512 * 8, pb = (size_t)in->n_patch * 5 * 512 * ps;
    const size_t nb = (size_t)in->n_patch * 4;
    const void *reg[7] = {in->cons, in->prims, cons_out, prims_out, s.queue, in->net_mask, net_out};
    const size_t sz[7] = {cb, pb, cb, pb, SRHD_QUEUE_WORDS * 8, nb, nb};
    rc = check_lists(prm, g, eos_k, in->n_patch, reg, sz, 7, s, "srhd_fluid_step_grid");
    if (rc) return rc;
  }
  if (in->n_patch > 0) {
    s.net_out = net_out;
    s.net_gate = g.kind == SRHD_GUESS_MLP ? g.gate : __builtin_huge_val();
    if (s.net_list) s.net_in = in->net_mask;
  }
  if (s.integrator == SRHD_VL)
    return hip_status(srhd::launch_step_vl_grid(prm->prec, s, (hipStream_t)stream), "srhd_fluid_step_grid");
  return hip_status(srhd::launch_step_grid(prm->prec, s, (hipStream_t)stream),
                    "srhd_fluid_step_grid");
}

}  // extern "C"
