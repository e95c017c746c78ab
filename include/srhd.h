/*
 * srhd.h -- C ABI of libsrhd, an MI355X (gfx950) library for one finite-volume step of special
 * relativistic hydrodynamics with the Taub-Mathews equation of state over a batch of 8^3-cell
 * patches, after Tseng, Schive & Chiueh, arXiv:2012.11130 ("GAMER-SR").
 *
 * Conventions shared by every call
 *   - Units c = k_B = m = 1; Theta = k_B T / (m c^2).
 *   - Primitive variables (rho, Ux, Uy, Uz, p): proper density, four-velocity, pressure.
 *     Conserved variables (D, Mx, My, Mz, Et): lab density, momentum, reduced energy Et = E - D
 *     (Sec. 2.1, Eqs. 5a-5c and 6).
 *   - Every data pointer is a DEVICE pointer owned by the caller, unless the comment says host.
 *     The library never keeps a pointer after the call returns.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the default stream).  Results
 *     are valid once the stream is synchronised.  No call synchronises the device.
 *   - Return value: SRHD_OK (0) or a negative srhd_err.  Argument errors are detected before any
 *     launch and leave outputs untouched; srhd_last_error() then describes the problem.
 *   - Physical failures are data, not errors: they are reported per state (status codes) or in
 *     srhd_step_stats, and the affected outputs are NaN.
 *   - Arrays of states are structure-of-arrays, field-major: [5][n].  Patch arrays are
 *     [patch][field][z][y][x], x fastest; a padded patch has N = 8 + 2 ghost cells per side.
 *   - The library allocates no user-visible memory.  Work buffers are passed in by the caller.
 */
#ifndef SRHD_H
#define SRHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SRHD_ABI_VERSION 8

typedef enum { SRHD_F64 = 0, SRHD_F32 = 1 } srhd_dtype;

typedef enum {
  SRHD_OK = 0,
  SRHD_EINVAL = -1,       /* bad argument (NULL pointer, negative size, misaligned pointer...) */
  SRHD_EHIP = -2,         /* the HIP runtime reported an error at launch */
  SRHD_EUNSUPPORTED = -3  /* valid request that the library does not implement */
} srhd_err;

/* Per-state status of an inversion (int8). */
enum {
  SRHD_ST_OK = 0,
  SRHD_ST_UNPHYSICAL = 1, /* D <= 0, Et <= 0, non-finite input, or L <= eps (Eq. 30) */
  SRHD_ST_FALLBACK = 2,   /* the supplied initial guess failed; the analytic guess converged */
  SRHD_ST_NOCONV = 3      /* Newton did not converge within max_iter from either guess */
};

typedef enum { SRHD_GUESS_ANALYTIC = 0, SRHD_GUESS_MLP = 1 } srhd_guess_kind;
typedef enum { SRHD_HLLC = 0, SRHD_HLLE = 1 } srhd_riemann;
/* FP64: every stage in FP64.  MIXED: reconstruction, fluxes and the update increment in FP32;
 * the left-hand side L of Eq. 15 and the Newton iteration in FP64, the recovery of the
 * primitives from its root (whose results are stored in FP32) in FP32.  FP32: reconstruction,
 * fluxes, update increment and the Newton inversion in FP32; only the subtraction inside L
 * (the cancellation of Eq. 20) is formed in FP64 from the FP32 variables.  With an FP32 bulk, L
 * is the exact sum of exact products, or their plain FP64 sum where every lane of a wavefront
 * has a condition number of at most 1024 (relative error below 6e-13).  State storage stays
 * FP64 in every mode. */
typedef enum { SRHD_PREC_FP64 = 0, SRHD_PREC_MIXED = 1, SRHD_PREC_FP32 = 2 } srhd_prec;

/* The energy variable a step evolves (Sec. 4 compares the two).  REDUCED: Et = E - D (Eq. 23),
 * this paper's scheme, with the flux (Et + p) v_d and L formed without cancellation (Eq. 15).
 * TOTAL: the original scheme -- the fifth conserved slot holds the total energy E of Eq. 5c,
 * evolved with the flux M_d, and every inversion forms L = (E/D)^2 - (|M|/D)^2 - 1 from the
 * divided variables in the inversion's arithmetic (Eq. 21), whose relative error grows as
 * 4 eps / (3 Theta) for a cold gas (Eq. 32).  TOTAL runs in srhd_fluid_step with
 * SRHD_PREC_FP64 or SRHD_PREC_FP32 and the analytic guess only (else SRHD_EUNSUPPORTED); the
 * physical check of its states is D > 0, E > 0 and that L > DBL_EPSILON. */
typedef enum { SRHD_ENERGY_REDUCED = 0, SRHD_ENERGY_TOTAL = 1 } srhd_energy;

/* Time integrator of a step (Sec. 3.1 names both).  MHM: MUSCL-Hancock (Sec. 3.2), described at
 * srhd_fluid_step.  VL: the van Leer predictor-corrector (Falle 1991; van Leer 2006) -- a
 * first-order half step U* = U^n - (dt/2dh) sum_d [F_d(W_c, W_{c+d}) - F_d(W_{c-d}, W_c)] with
 * the cell-centre primitives as face states, W* = cons -> prim of U*, then the full step with
 * the fluxes of PLM face states of W*.  Only an updated cell failing Eq. 30 triggers the limiter
 * retry.  VL runs in srhd_fluid_step with ghost >= 3 and in srhd_fluid_step_grid, with the
 * analytic guess and the reduced energy, in every precision mode (else SRHD_EUNSUPPORTED).  A predictor state that fails the
 * inversion is replaced by the cell's state at t^n (W* = W^n: the half step is dropped for that
 * cell) and counted in n_pred_fallback. */
typedef enum { SRHD_MHM = 0, SRHD_VL = 1 } srhd_integrator;

/* Learned initial guess: device parameters of a 3-64-64-1 SiLU perceptron that maps three
 * standardised log-scaled invariants of the conserved state to the standardised log of the
 * Newton unknown ht (see srhd_mlp_*).  Feature sets:
 *   SRHD_FEAT_CONS: (log D, log max(|M|/D, 1e-300), log(Et/D));
 *   SRHD_FEAT_L:    (log L, log max(|M|/D, 1e-300), log(Et/D)), L the left-hand side of Eq. 15
 *                   as the inversion computes it (error-free, before any guess is needed).
 * The network is consulted only for states with L > gate_L (0: every state); the others, and
 * every state whose network guess fails, use the analytic guess of App. A.  Not in the paper: an
 * addition whose Newton refinement and analytic fallback keep the inversion's result unchanged. */
enum { SRHD_FEAT_CONS = 0, SRHD_FEAT_L = 1 };
typedef struct {
  const uint16_t *w_bf16;  /* BF16 weights, 16-byte aligned: W1[64][3], W2[64][64] (row = output
                              unit), W3[64] -- 4352 values */
  const float *bias;       /* FP32 biases: b1[64], b2[64], b3 -- 129 values */
  const float *norm;       /* FP32 [8]: input mean[3], input std[3], output mean, output std */
  int features;            /* SRHD_FEAT_CONS or SRHD_FEAT_L */
  double gate_L;           /* >= 0 */
} srhd_mlp;

typedef struct {
  int kind;                /* srhd_guess_kind */
  const srhd_mlp *mlp;     /* host pointer to device parameters; required when kind == MLP */
  int max_iter;            /* Newton iterations per guess; <= 0 selects 30 */
} srhd_guess;

/* Equation of state (Sec. 2.2).  SRHD_EOS_TM: the Taub-Mathews EoS of Eq. 10, the default
 * wherever an srhd_eos pointer is NULL or zero-initialised.  SRHD_EOS_POLYTROPIC: the polytropic
 * EoS h = 1 + Gamma Theta / (Gamma - 1) with 1 < gamma <= 2, whose sound speed is
 * c_s^2 = Gamma Theta / h; its inversion starts Newton from ht = L / ((1 - k)(2 + sqrt(L))),
 * k = (Gamma - 1) / Gamma (App. A's guess belongs to TM).  The polytropic EoS runs in the
 * conversions, the CFL time step and srhd_fluid_step with MUSCL-Hancock and the reduced energy
 * (every precision mode, analytic guess); elsewhere SRHD_EUNSUPPORTED. */
typedef enum { SRHD_EOS_TM = 0, SRHD_EOS_POLYTROPIC = 1 } srhd_eos_kind;
typedef struct {
  int kind;                /* srhd_eos_kind */
  double gamma;            /* ratio of specific heats (SRHD_EOS_POLYTROPIC only) */
} srhd_eos;

/* ---------------------------------------------------------------------------------------- */
/* Conversions (Sec. 2.3)                                                                   */
/* ---------------------------------------------------------------------------------------- */

/* prim[5][n] -> cons[5][n] by Eqs. 8, 5a, 22, 5b, 15 and 23 (no root finding).  dtype selects
 * FP64 or FP32 storage and arithmetic.  prim and cons must not overlap.  eos (host, may be
 * NULL: TM). */
int srhd_prim2cons(int dtype, int64_t n, const void *prim, void *cons, const srhd_eos *eos,
                   void *stream);

/* cons[5][n] -> prim[5][n]: L = x^2 + 2x - m^2 (x = Et/D, m = |M|/D) from error-free products
 * and a compensated sum, the physical check L > eps (Eq. 30), the root ht of f(ht) = L
 * (Eq. 15) by Newton's method (Eqs. A1-A2) from the guess selected by `guess` (NULL: the
 * analytic guess of App. A, Eqs. A3-A7), then Eqs. 17, 8, 5a, 16 and 18.
 * status[n] (int8, SRHD_ST_*) and iters[n] (uint8, Newton iterations) may be NULL.
 * FP32: L, Newton and recovery in FP32.  FP64: all in FP64.  eos (host, may be NULL: TM); the
 * learned guess is for TM only. */
int srhd_cons2prim(int dtype, int64_t n, const void *cons, void *prim, int8_t *status,
                   uint8_t *iters, const srhd_guess *guess, const srhd_eos *eos, void *stream);

/* ---------------------------------------------------------------------------------------- */
/* Patches (Sec. 3.1: 8^3-cell patches with ghost zones)                                    */
/* ---------------------------------------------------------------------------------------- */

#define SRHD_MAX_LEVEL 8

typedef struct {
  int64_t n_patch;
  int ghost;               /* ghost cells per side, >= 2 (3 in the GAMER layout) */
  int dtype;               /* storage type of `padded` (SRHD_F64 only for the step) */
  const void *padded;      /* [n_patch][5][N][N][N] conserved variables, N = 8 + 2 ghost */
  const int8_t *level;     /* [n_patch] refinement level, or NULL (all level 0) */
  int n_level;             /* 1 .. SRHD_MAX_LEVEL */
  double dh[SRHD_MAX_LEVEL];  /* host: cell size per level */
} srhd_patches;

/* Neighbour table neighbor[n_patch][27] (int32, device): slot (oz+1)*9 + (oy+1)*3 + (ox+1)
 * holds the index in `interior` of the same-level patch at offset (ox, oy, oz); slot 13 is the
 * patch's own index (so a table listing a subset of patches fills only those).  -1 in a face slot
 * marks a domain boundary: ghost cells beyond it copy the nearest interior cell (outflow,
 * zero gradient).  SRHD_NB_COARSE (-2) marks a region covered only by the next coarser level:
 * those ghost cells are left untouched here and filled by srhd_fill_ghosts_coarse.  Periodic
 * domains list wrapped neighbours.
 * Fills every ghost cell of padded[n_patch][5][N][N][N] (faces, edges and corners) from
 * interior[n_src][5][8][8][8]; also copies the interior.  A cell whose source index is outside
 * [0, n_src) and not SRHD_NB_COARSE -- e.g. -1 in an edge slot while no face slot marks a
 * boundary -- is set to NaN. */
#define SRHD_NB_COARSE (-2)
int srhd_fill_ghosts(int dtype, int64_t n_patch, int ghost, int64_t n_src, const void *interior,
                     const int32_t *neighbor, void *padded, void *stream);

/* CFL time step (Sec. 3.3, Eqs. 26-28, the sum taken over |Ux| + |Uy| + |Uz|): one global
 * maximum signal speed S_max over the interior cells of interior[n_patch][5][8^3] (inverted
 * with the analytic guess), then dt_lev[l] = c_cfl * dh[l] / S_max for l < n_level (so
 * dt_l = dt_0 / 2^l when dh_l = dh_0 / 2^l).  dt_lev: device double[n_level].
 * work: device buffer of srhd_cfl_work_bytes() bytes (reused across calls, contents scratch).
 * The maximum is exact (order independent), so the result is deterministic. */
size_t srhd_cfl_work_bytes(void);
int srhd_cfl_dt(int dtype, int64_t n_patch, const void *interior, int n_level,
                const double *dh /* host [n_level] */, double c_cfl, double *dt_lev,
                void *work, const srhd_eos *eos /* host, may be NULL: TM */, void *stream);

/* How the patches of a step are spread over the GPU (a launch choice, not part of the method;
 * results are identical for every schedule).  groups == 0: one workgroup per patch, each XCD
 * given a contiguous range of patch indices.  groups > 0: a persistent grid of `groups`
 * workgroups; each claims `chunk` patches at a time from one queue counter per XCD (over that
 * XCD's contiguous range, then the other XCDs' ranges in turn) until the list is exhausted.
 * queue: device memory of SRHD_QUEUE_WORDS uint64 words, required when groups > 0, zeroed by the
 * call on its stream; calls in flight at the same time must not share it.
 * occupancy: 0 selects the step kernel compiled for its natural register budget; 2 selects a
 * variant compiled for at most 128 VGPRs per lane so that two 512-thread workgroups share a
 * compute unit (an FP32 bulk, i.e. SRHD_PREC_MIXED or SRHD_PREC_FP32, only: otherwise
 * SRHD_EUNSUPPORTED). */
#define SRHD_QUEUE_WORDS 8
typedef struct {
  int groups;              /* 0, or 1 .. 65535 persistent workgroups */
  int chunk;               /* patches per claim, 1 .. 64 (ignored when groups == 0) */
  int occupancy;           /* 0 or 2 */
  uint64_t *queue;         /* device [SRHD_QUEUE_WORDS], or NULL when groups == 0 */
} srhd_sched;

typedef struct {
  double theta;            /* limiter coefficient of the generalized minmod (default 1.5) */
  int riemann;             /* srhd_riemann */
  int prec;                /* srhd_prec */
  int max_retry;           /* reductions theta *= 0.75 before the final theta = 0 attempt */
  srhd_guess guess;        /* initial guess for every inversion in the step */
  srhd_sched sched;        /* launch schedule; all-zero = one workgroup per patch */
  int energy;              /* srhd_energy (0: this paper's reduced energy) */
  int integrator;          /* srhd_integrator (0: MUSCL-Hancock) */
  srhd_eos eos;            /* equation of state (zero: TM) */
  double *flux_out;        /* device [n_patch][6][5][64] or NULL: the Riemann fluxes of the final
                              attempt through the six faces of each patch, face s = 2 d + u (axis
                              d; u = 1 the upper face), face cell b * 8 + a with (a, b) the two
                              transverse coordinates in increasing axis order.  Overwritten, not
                              accumulated (see srhd_flux_accumulate); for the flux correction of
                              coarse-fine interfaces.  Must not overlap the other arrays. */
  double kappa_max;        /* precision guard of the FP32-bulk modes (see below); 0: off */
  int learned_split;       /* learned guess by patch (see below); 0: one launch */
  uint64_t *defer;         /* device [2 n_patch + 4] workspace of the guard and the split, or NULL
                              when neither is on */
} srhd_step_params;

/* Precision guard (SRHD_PREC_MIXED and SRHD_PREC_FP32, MUSCL-Hancock).  Eq. 20 puts the error of
 * recovering the pressure from conserved variables that carry a relative rounding error eps at
 * (1 + M^2) eps, M = U / U_s the Mach number in four-velocities (U_s^2 = c_s^2 / (1 - c_s^2)).
 * An FP32 bulk rounds the half-step face states and the update increment to FP32, so a patch
 * holding a cell with kappa = 1 + M^2 near 1 / eps_32 (a gamma = 10^3 jet: kappa ~ 2e6) loses its
 * pressure there.  With kappa_max >= 1 every patch whose 12^3 primitive tile (after the
 * cell-centre inversions, or as gathered) holds a cell with kappa > kappa_max is stepped instead
 * by the FP64 kernel (FP64 bulk and inversion; in the gather layout from the gathered FP64
 * conserved variables), in a second launch over the list of such patches; the other patches keep the
 * FP32 bulk, whose one-step error is then of order kappa_max eps_32 per field.  kappa_max = 0
 * turns the guard off (the FP32 bulk everywhere, like a single-precision code).  Ignored by
 * SRHD_PREC_FP64 and by the VL integrator.
 *
 * Learned guess by patch (learned_split = 1, a learned guess with a gate_L > 0, MUSCL-Hancock with
 * the reduced energy and the TM EoS): the kernel without the network steps every patch and lists
 * those whose tile holds a cell with L > gate_L (Eq. 15's left-hand side of the cell's state); a
 * second launch steps the listed patches with the network, consulted as always where a state's
 * L > gate_L.  The other patches run no network code: where the gate keeps the network out of a
 * patch, its registers and code cost that patch nothing.  Results equal a single launch's up to
 * the Newton tolerance (a face state with L above the gate in an unlisted patch starts from the
 * analytic guess instead).  A patch the guard steps in FP64 is not listed.  In the gather layout
 * with the state's network masks (srhd_grid.net_mask) the list is known before the step: it holds
 * the patches whose 12^3 tile (the patch and the two layers of its 26 neighbours next to it)
 * holds a cell with L > gate_L, and the learned kernel steps them on a second stream of the
 * library's, concurrently with the kernel without the network, which skips them; the call joins
 * that stream back into `stream` before it returns (work queued later on `stream` waits for both).
 *
 * defer: device memory of 2 n_patch + 4 uint64 words (8-byte aligned), required when the guard or
 * the split is on; zeroed by the call on its stream.  Afterwards word 0 holds the number of
 * patches stepped in FP64 and words 2 .. their indices, word n_patch + 2 the number of patches
 * stepped with the network and words n_patch + 4 .. theirs, in no particular order.  Calls in
 * flight at the same time must not share it. */
#define SRHD_KAPPA_MAX_DEFAULT 1024.0

/* Device counters, accumulated (never reset by the step; see srhd_stats_reset). */
typedef struct {
  uint64_t n_unphysical;   /* failed inversions + failed output cells of the final attempts */
  uint64_t n_fallback;     /* inversions whose supplied guess failed (analytic rescue) */
  uint64_t n_noconv;       /* inversions that did not converge */
  uint64_t newton_iters;   /* Newton iterations over all inversions of all attempts */
  uint64_t n_inversions;   /* inversions performed (all attempts) */
  uint64_t n_retry;        /* extra attempts with a reduced limiter coefficient */
  uint64_t n_mlp;          /* learned-guess evaluations: lanes of wavefronts that ran the network */
  uint64_t n_pred_fallback; /* VL: predictor states that failed the inversion and were replaced
                               by the cell's state at t^n (final attempts) */
  uint64_t n_fp64_patch;   /* patches the precision guard stepped with the FP64 bulk */
  uint64_t n_learned_patch; /* patches the learned-guess split stepped with the network */
} srhd_step_stats;

int srhd_stats_reset(srhd_step_stats *stats, void *stream);

/* One unsplit MUSCL-Hancock step (Sec. 3.2) of every patch: cell-centre inversion, PLM in
 * (rho, Ux, Uy, Uz, p) with the hybrid van Leer / generalized minmod limiter, the half-step
 * face states, face inversions, HLLC or HLLE fluxes with the TM sound speed (Eq. 14) and the
 * reduced energy, and the conservative full update of the 8^3 interior:
 *   out[p] = U^n - dt_l/dh_l sum_d (F_{d,+1/2} - F_{d,-1/2}).
 * A patch meeting an unphysical state is redone with theta *= 0.75 (max_retry times) and then
 * theta = 0 (Sec. 3.4).  dt_lev: device double[n_level] (e.g. from srhd_cfl_dt).
 * out: [n_patch][5][8][8][8] FP64; must not overlap in->padded (nor prm->sched.queue).
 * stats may be NULL.  Precision (prm->prec), launch schedule (prm->sched) and energy variable
 * (prm->energy) are described at srhd_prec, srhd_sched and srhd_energy; every schedule gives the
 * same results bit for bit. */
int srhd_fluid_step(const srhd_patches *in, void *out, const double *dt_lev,
                    const srhd_step_params *prm, srhd_step_stats *stats, void *stream);
/* (prm->integrator selects MUSCL-Hancock or VL: see srhd_integrator.) */

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): srhd_fluid_step with its two work buffers -- the
 * patch lists of the precision guard and the learned-guess split (prm->defer) and the persistent
 * schedule's counters (prm->sched.queue) -- taken from a static device array of the library
 * instead of the caller.
 * The array holds SRHD_QUEUE_WORDS + 2 SRHD_STATIC_MAX_PATCH + 4 uint64 words (16 MiB) on
 * every GPU the library runs on, until the process ends; its device address is looked up on
 * the first call on each device.  Arguments and results as for srhd_fluid_step, except:
 * prm->defer and prm->sched.queue must be NULL, and n_patch may not exceed SRHD_STATIC_MAX_PATCH
 * (else SRHD_EINVAL before any launch).  The call allocates nothing.  Every call on one GPU
 * shares that GPU's array (the call clears what must start at zero, on its stream): calls that
 * overlap in time on one GPU -- on different streams, or from different threads -- race and
 * must not be issued. */
#define SRHD_STATIC_MAX_PATCH 1048576
int srhd_fluid_step_static(const srhd_patches *in, void *out, const double *dt_lev,
                           const srhd_step_params *prm, srhd_step_stats *stats, void *stream);

/* Workgroups of the step kernel that fit on one compute unit at once for the kernel that
 * prm (host) selects -- its precision, guess kind, register variant (prm->sched.occupancy),
 * energy variable and integrator -- and the layout (gather = 1: srhd_fluid_step_grid, 0:
 * srhd_fluid_step); multiplied by the device's compute-unit count it sizes a persistent
 * schedule.  prm->sched.groups and .queue are ignored.  Returns the count (> 0), or a negative
 * srhd_err (SRHD_EUNSUPPORTED for a combination that has no kernel). */
int srhd_step_occupancy(const srhd_step_params *prm, int gather);

/* Schedule autotuner for srhd_fluid_step.  Runs the step on `in` (writing `out`) once per
 * candidate schedule as a warm-up and then `reps` timed times, timed with events on `stream`,
 * and writes the fastest candidate into prm->sched (keeping prm->sched.queue, which must be
 * set).  Candidates, for each register variant the precision allows (occupancy 0, and 2 for
 * an FP32 bulk): one workgroup per patch, and persistent grids of
 * 1, 2 and 4 times the resident workgroups (srhd_step_occupancy x compute units) with chunk 1, 2
 * and 4.  table (host, may be NULL) receives up to table_cap entries {groups, chunk, occupancy,
 * ms per step} in trial order and *n_table their number.  Unlike the other calls this one
 * synchronises `stream`.  stats counters are not touched. */
typedef struct {
  int groups;
  int chunk;
  int occupancy;
  float ms;
} srhd_tune_entry;
int srhd_autotune_step(const srhd_patches *in, void *out, const double *dt_lev,
                       srhd_step_params *prm, int reps, srhd_tune_entry *table, int table_cap,
                       int *n_table, void *stream);

/* ---------------------------------------------------------------------------------------- */
/* The same step on a block of same-level patches without padded copies                     */
/* ---------------------------------------------------------------------------------------- */

/* A block of same-level patches: the step reads each patch's ghost cells directly from the
 * interiors of its 26 neighbours (the rule of srhd_fill_ghosts, including outflow clamping),
 * so no padded copy is written or read.  Primitives travel with the state: the step inverts
 * every updated cell once and returns its primitives and the maximum signal speed for the
 * next step's time step. */
typedef struct {
  int64_t n_patch;
  const double *cons;      /* [n_patch][5][8][8][8] FP64 conserved interiors */
  const void *prims;       /* [n_patch][5][8][8][8] primitives of `cons` in the step's bulk type:
                              float for SRHD_PREC_MIXED and SRHD_PREC_FP32, double for
                              SRHD_PREC_FP64 */
  const int32_t *neighbor; /* [n_patch][27] int32, as for srhd_fill_ghosts (indices < n_patch) */
  const int8_t *level;     /* [n_patch] or NULL */
  int n_level;
  double dh[SRHD_MAX_LEVEL];  /* host */
  const uint32_t *net_mask; /* [n_patch] or NULL: the state's network masks, as written by
                              srhd_grid_prims or the step that made the state (read only by the
                              learned-guess split) */
} srhd_grid;

/* Network mask of a patch of a gather-layout state: bit (rz + 1) 9 + (ry + 1) 3 + (rx + 1) is set
 * when the patch holds a cell whose L (Eq. 15's left-hand side, formed as for the cell's
 * inversion) exceeds the learned guess's gate_L in region (rx, ry, rz), where along each axis
 * r = 0 takes every cell, r = -1 the two lowest layers and r = +1 the two highest (the layers a
 * neighbour's step reads).  Zero with the analytic guess. */

/* Entry state of a chain of srhd_fluid_step_grid calls: inverts every interior cell (as
 * srhd_cons2prim, from the guess `guess` selects -- NULL: the analytic guess -- with the Newton
 * tolerance and inversion type of the step's precision), writes the
 * primitives in the step's bulk type, and the maximum S_max (Eqs. 26-27) over the cells as the
 * bit pattern of a positive double in *smax_bits (device; zeroed first).  Unphysical cells get
 * NaN primitives and do not enter the maximum.  net_mask (device uint32 [n_patch], or NULL)
 * receives the state's network masks. */
int srhd_grid_prims(int prec, int64_t n_patch, const double *cons, void *prims,
                    uint64_t *smax_bits, uint32_t *net_mask, const srhd_guess *guess,
                    void *stream);

/* One MUSCL-Hancock (or, prm->integrator = SRHD_VL, VL) step of a srhd_grid, the step of
 * srhd_fluid_step on the padded copies of the same patches: for the same dt bit for bit in FP64,
 * and with VL in every precision mode (MUSCL-Hancock with an FP32 bulk agrees to rounding: its
 * gather kernel refines the hardware reciprocals and square roots of its inversions and L).
 * The time step is dt_l = c_cfl * dh[l] / S_max with S_max read from *smax_in (the bits written
 * by srhd_grid_prims or by the previous step), unless dt_lev (device double[n_level]) is given.  Outputs: cons_out [n_patch][5][8][8][8] FP64,
 * prims_out (bulk type) and *smax_out (zeroed, then the maximum over the updated cells);
 * net_out (device uint32 [n_patch], or NULL) the updated state's network masks;
 * dt_used (device double[n_level], may be NULL) receives the time step used.
 * Outputs must not overlap the inputs.  Patches are mapped to workgroups so that each XCD works
 * on a contiguous range of patch indices (order patches along a space-filling curve).  The
 * reduced energy and the TM EoS only (prm->energy = SRHD_ENERGY_TOTAL or a polytropic EoS gives
 * SRHD_EUNSUPPORTED); VL takes the analytic guess, and its network masks (net_out) are zero. */
int srhd_fluid_step_grid(const srhd_grid *in, const uint64_t *smax_in, double c_cfl,
                         const double *dt_lev, double *cons_out, void *prims_out,
                         uint64_t *smax_out, uint32_t *net_out, double *dt_used,
                         const srhd_step_params *prm, srhd_step_stats *stats, void *stream);

/* The schedule autotuner of srhd_autotune_step for srhd_fluid_step_grid on the same arguments
 * (outputs written, prm->sched set to the fastest candidate; synchronises `stream`). */
int srhd_autotune_step_grid(const srhd_grid *in, const uint64_t *smax_in, double c_cfl,
                            const double *dt_lev, double *cons_out, void *prims_out,
                            uint64_t *smax_out, uint32_t *net_out, srhd_step_params *prm,
                            int reps, srhd_tune_entry *table, int table_cap, int *n_table,
                            void *stream);

/* ---------------------------------------------------------------------------------------- */
/* The learned guess: inference and training                                                */
/* ---------------------------------------------------------------------------------------- */

#define SRHD_MLP_NPARAM 4481   /* W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3 */

/* Features (feature set `features`, see srhd_mlp) of cons[5][n] into feat[3][n] (FP32).  With
 * prim[5][n] (the states' primitives, same dtype) also the training target target[n] = log ht,
 * ht from Eq. 22 at Theta = p/rho; prim and target are both NULL or both set.  States that are
 * not admissible (Eq. 30) get L = 0 (log L = -inf). */
int srhd_mlp_features(int dtype, int features, int64_t n, const void *cons, const void *prim,
                      float *feat, float *target, void *stream);

/* y[n] = de-standardised network output (the guess of log ht) for raw features feat[3][n]; the
 * hidden layer runs on the matrix cores (BF16 operands, FP32 accumulation). */
int srhd_mlp_forward(const srhd_mlp *m, int64_t n, const float *feat, float *y, void *stream);

/* Bytes of the workspace srhd_mlp_grad needs for a minibatch of `batch` samples. */
size_t srhd_mlp_workspace_bytes(int64_t batch);

/* Mean-squared-error gradient over a minibatch: targets target[batch] are log ht; the loss is
 * taken on the standardised output.  grad[SRHD_MLP_NPARAM] and loss[1] are FP32 device
 * outputs; the sum over samples is in sample order (bit-reproducible). */
int srhd_mlp_grad(const srhd_mlp *m, int64_t batch, const float *feat, const float *target,
                  float *grad, float *loss, void *ws, void *stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8; `step` counts from 1) on the FP32 master
 * parameters master[SRHD_MLP_NPARAM] with moments m1, m2; rewrites the BF16 weights w_bf16[4352]
 * and the FP32 biases bias[129] that inference reads. */
int srhd_mlp_adam(float *master, float *m1, float *m2, const float *grad, int step, float lr,
                  uint16_t *w_bf16, float *bias, void *stream);

/* Thread-local description of the last non-zero return. */
const char *srhd_last_error(void);
/* ---------------------------------------------------------------------------------------- */
/* AMR neighbours of the step (Sec. 3.4 items 3 and 4), refinement ratio 2                      */
/* ---------------------------------------------------------------------------------------- */

/* Coarse-to-fine ghost-zone interpolation (Sec. 3.4, "ghost-zone interpolation").  For each fine
 * patch p, every ghost cell of fine_padded[p] whose neighbour slot (after the outflow clamp of
 * srhd_fill_ghosts) is SRHD_NB_COARSE is filled from the parent coarse_old[parent[p]] (padded,
 * ghost_c layers, ghost_c >= ghost / 2 + 2): with I = 8 b + c the cell's fine index relative to
 * the parent (b the patch's octant bit along that axis, octant[p] = bx | by << 1 | bz << 2; c its
 * coordinate in the patch), the coarse cell is C = floor(I / 2) and the fine centre lies -1/4 or
 * +1/4 of a coarse cell from C's centre; the value is u_C plus, per axis, that offset times the
 * limited slope (the PLM limiter with coefficient theta) of u_{C-1}, u_C, u_{C+1} -- so the eight
 * children of a coarse cell average to it.  The coarse state is (1 - alpha) old + alpha new when
 * coarse_new is given (time interpolation for fine sub-steps).  The conserved variables are
 * interpolated first; where that state fails Eq. 30, the primitive variables of the same coarse
 * cells (FP64 inversions, analytic guess) are interpolated instead and converted back.
 * counts (device uint64[2], may be NULL) accumulates {cells interpolated, primitive fallbacks}.
 * Arrays FP64 on the device; fine_padded is read-modify-written (fill the same-level ghosts with
 * srhd_fill_ghosts first). */
int srhd_fill_ghosts_coarse(int64_t n_fine, int ghost, const int32_t *neighbor,
                            const int32_t *parent, const int8_t *octant, int64_t n_coarse,
                            int ghost_c, const double *coarse_old, const double *coarse_new,
                            double alpha, double theta, double *fine_padded, uint64_t *counts,
                            void *stream);

/* Restriction: coarse[parent_of[q]] = the average of its eight children (the volume-weighted
 * average that keeps a parent equal to its children, Sec. 3.4): child[q][o], o = bx | by << 1 |
 * bz << 2, indices into fine[n_fine][5][8][8][8]; parent_of[q] into coarse[n_coarse][5][8][8][8].
 * n_parent entries; FP64 device arrays; entries with indices out of range are skipped. */
int srhd_restrict(int64_t n_parent, const int32_t *parent_of, const int32_t *child,
                  int64_t n_fine, const double *fine, int64_t n_coarse, double *coarse,
                  void *stream);

/* acc[i] = beta * acc[i] + weight * flux[i] for i < n (device FP64): time-integrates the
 * boundary fluxes a step writes to flux_out (beta = 0 starts a sum). */
int srhd_flux_accumulate(int64_t n, double *acc, const double *flux, double beta, double weight,
                         void *stream);

/* Coarse-fine flux correction (Sec. 3.4 item 4).  faces[n_face][6] (device int32): coarse patch,
 * side s = 2 d + u of that patch, and the four fine patches across the face, fine[t] holding the
 * coarse face cells (a, b) with t = (a >= 4) + 2 (b >= 4).  coarse_flux [Pc][6][5][64] holds
 * dt_c F_c, fine_flux [Pf][6][5][64] the sum over the fine sub-steps of dt_f F_f (both from
 * flux_out through srhd_flux_accumulate).  Each coarse cell at such a face gets
 * dU = (u ? -1 : +1) (<fine> - coarse) / dh_c, <fine> the mean of the four fine face cells
 * covering it; a cell whose corrected state fails Eq. 30 keeps its state (counted in *skipped,
 * device uint64, may be NULL).  coarse: [Pc][5][8][8][8] FP64, updated in place.  The records are
 * applied side by side (s = 0 .. 5), so a cell touching faces on several sides gets each
 * correction in that order; at most one record per (coarse patch, side).  Records whose indices
 * fall outside [0, n_coarse) / [0, n_fine) are skipped. */
int srhd_flux_correct(int64_t n_face, const int32_t *faces, int64_t n_coarse, double *coarse,
                      const double *coarse_flux, int64_t n_fine, const double *fine_flux,
                      double dh_c, uint64_t *skipped, void *stream);

int srhd_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
