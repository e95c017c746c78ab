/*
 * srhd_oracle.h -- declarations of the CPU reference (oracle) for the SRHD step.
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the benchmark's
 * CPU-baseline leg; never by the product library.  All arrays are host memory, FP64.
 */
#ifndef SRHD_ORACLE_H
#define SRHD_ORACLE_H
#include <stdint.h>

enum { OR_ST_OK = 0, OR_ST_UNPHYSICAL = 1, OR_ST_FALLBACK = 2, OR_ST_NOCONV = 3 };
enum { OR_HLLC = 0, OR_HLLE = 1 };

double or_h_of_theta(double th);
double or_htilde_of_theta(double th);
double or_theta_of_htilde(double ht);
double or_dtheta_dhtilde(double ht);
double or_cs2(double th);
double or_f_given_theta(double ht, double th, double m2);
double or_f(double ht, double m2);
double or_dfdh(double ht, double m2);
double or_guess_cold(double L, double m2);
double or_guess_hot(double L);
double or_guess_threshold(double m2);
double or_guess_analytic(double L, double m2);
double or_sum_exact(const double *x, int n);
double or_L_exact(double D, double Mx, double My, double Mz, double Et);
double or_L_naive(double D, double Mx, double My, double Mz, double Et);
double or_L_total_energy(double D, double Mx, double My, double Mz, double E);
double or_solve_htilde(double L, double m2, int *iters);
void or_prim2cons_one(const double w[5], double u[5]);
int or_cons2prim_one(const double u[5], double w[5], double *ht_out, int *iters);
void or_prim2cons(int64_t n, const double *prim, double *cons);
void or_cons2prim(int64_t n, const double *cons, double *prim, int8_t *status, int32_t *iters);
void or_L_batch(int64_t n, const double *cons, int mode, double *L);
double or_smax_prim(const double w[5]);
void or_patch_smax(int64_t n_patch, const double *interior, double *smax, int64_t *n_unphys);
double or_slope(double wl, double wc, double wr, double theta);
void or_flux(int d, const double w[5], const double u[5], double F[5]);
void or_wavespeeds(int d, const double w[5], double *lm, double *lp);
void or_hlle(int d, const double wl[5], const double wr[5], double F[5]);
void or_hllc(int d, const double wl[5], const double wr[5], double F[5]);
int or_is_physical(const double u[5]);
int or_fluid_step(int64_t n_patch, int ghost, const double *padded, const int8_t *level,
                  const double *dh_lev, const double *dt_lev, double theta, int riemann,
                  int max_retry, int scheme, int integrator, double *out, int64_t *counts,
                  double *bflux);
/* EoS selection: 0 = TM, Gamma in (1, 2] = polytropic.  Returns -1 for another value. */
int or_set_eos(double gamma);
double or_get_eos(void);
/* AMR neighbour operations (refinement ratio 2). */
#define OR_NB_COARSE (-2)   /* neighbour slot covered by the next coarser level */
int or_fill_ghosts_coarse(int64_t n_fine, int ghost, const int32_t *neighbor, const int32_t *parent,
                          const int8_t *octant, int64_t n_coarse, int ghost_c,
                          const double *coarse_old, const double *coarse_new, double alpha,
                          double theta, double *fine_padded, int64_t *counts);
void or_restrict(int64_t n, const int32_t *parent_of, const int32_t *child, const double *fine,
                 double *coarse);
int64_t or_flux_correct(int64_t n_face, const int32_t *faces, double *coarse,
                        const double *coarse_flux, const double *fine_flux, double dh_c);
void or_prim2cons_total_one(const double w[5], double u[5]);
int or_cons2prim_total_one(const double u[5], double w[5], double *ht_out, int *iters);
void or_prim2cons_total(int64_t n, const double *prim, double *cons);
int or_fill_ghosts(int64_t n_patch, int ghost, int64_t n_src, const double *interior,
                   const int32_t *neighbor, double *padded);
void or_extract_interior(int64_t n_patch, int ghost, const double *padded, double *interior);
int or_num_threads(void);
void or_set_num_threads(int n);

#endif
