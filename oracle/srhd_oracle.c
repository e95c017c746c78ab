/*
 * srhd_oracle.c -- plain, slow, scalar FP64 CPU reference for one special-relativistic
 * hydrodynamics (SRHD) step with the Taub-Mathews (TM) equation of state, after
 * Tseng, Schive & Chiueh, "An adaptive mesh, GPU-accelerated, and error minimized special
 * relativistic hydrodynamics code" (arXiv:2012.11130).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load this library.  The product path (the HIP library) shares no code,
 * header, table or helper with it.
 *
 * Units: c = k_B = m = 1.  Theta = k_B T / (m c^2).  Reduced energy Et = E - D (Eq. 6),
 * reduced enthalpy ht = h - 1.  Build: -O2 -ffp-contract=off, no fast-math (so that every
 * expression below is evaluated exactly as written, one IEEE rounding per operation).
 *
 * Functions and the passage each follows:
 *   EoS                      Sec. 2.2, Eq. 10 (h), Eq. 22 (ht of Theta), Eq. 16 (Theta of ht),
 *                            Eq. 14 (sound speed), Eq. A2 (dTheta/dht); or the polytropic EoS
 *                            of Sec. 2.2 (or_set_eos), the same functions for h = 1 +
 *                            Gamma Theta / (Gamma - 1)
 *   inversion equation       Sec. 2.3, Eq. 15 (f), Eq. A1 (df/dht); its left-hand side L exactly
 *                            (error-free products, exact sum) and, to reproduce Eq. 20 and
 *                            App. B, as the plain expression of the divided variables
 *   initial guesses          App. A, Eqs. A3-A7 (A4 read as the positive root of A3)
 *   prim -> cons             Eqs. 8, 5a, 5b, 22, 15, 23
 *   cons -> prim             Eqs. 15, 30 (physical check), 17, 8, 5a, 16, 18; the root is
 *                            found by bisection-safeguarded Newton inside a bracket, which is
 *                            independent of the analytic or learned guess of the method
 *   CFL time step            Sec. 3.3, Eqs. 26 (sum over x, y, z), 27, 28
 *   PLM                      Sec. 3.2 / 4.2: hybrid van Leer / generalized minmod limiter
 *   Riemann fluxes           Sec. 3.2: relativistic HLLC / HLLE with the TM sound speed and
 *                            the reduced energy (E = Et + D); fluxes of Eqs. 4a, 4b, 7
 *   MUSCL-Hancock step       Sec. 3.2 (unsplit half step + full step)
 *   VL step                  Sec. 3.1 names the scheme (Falle 1991; van Leer 2006): a
 *                            first-order (piecewise-constant) half-step predictor, then PLM of
 *                            the half-step primitives and the full step with their fluxes
 *   ghost fill               Sec. 3.1 (8^3 patches), periodic or outflow (zero gradient)
 *   original scheme          Sec. 2.3 / 4: the total energy E (Eq. 5c) evolved with flux M
 *                            (Eq. 4b), L = (E/D)^2 - (|M|/D)^2 - 1 from the divided variables
 *                            (the cancellation Eq. 21 quantifies); kept to reproduce the
 *                            paper's comparison (Sec. 4.1, Eq. 32)
 *
 * "Parity unpinned" items: none of the functions above lacks a pin; see the test suite.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "srhd_oracle.h"

#define NF 5           /* number of fields */
#define PS 8           /* patch interior cells per side */

/* ===================================================================================== */
/* EoS (Sec. 2.2)                                                                        */
/* ===================================================================================== */

/* The equation of state of every function below: 0 selects TM (Eq. 10); Gamma in (1, 2]
 * selects the polytropic EoS h = 1 + Gamma Theta / (Gamma - 1) of Sec. 2.2.  Set before a call,
 * not while one runs. */
static double or_gamma = 0.0;

int or_set_eos(double gamma)
{
  if (gamma != 0.0 && !(gamma > 1.0 && gamma <= 2.0)) return -1;
  or_gamma = gamma;
  return 0;
}

double or_get_eos(void) { return or_gamma; }

/* Eq. 10: TM specific enthalpy h(Theta); polytropic: 1 + Gamma Theta / (Gamma - 1). */
double or_h_of_theta(double th)
{
  if (or_gamma != 0.0) return 1.0 + or_gamma * th / (or_gamma - 1.0);
  return 2.5 * th + sqrt(2.25 * th * th + 1.0);
}

/* Eq. 22: reduced enthalpy ht = h - 1 written without a subtraction. */
double or_htilde_of_theta(double th)
{
  if (or_gamma != 0.0) return or_gamma * th / (or_gamma - 1.0);
  double a = 2.25 * th * th;
  return 2.5 * th + a / (1.0 + sqrt(a + 1.0));
}

/* Eq. 16: Theta from the reduced enthalpy (inverse of Eq. 10). */
double or_theta_of_htilde(double ht)
{
  if (or_gamma != 0.0) return (or_gamma - 1.0) * ht / or_gamma;
  double num = 2.0 * ht * ht + 4.0 * ht;
  double den = 5.0 * ht + 5.0 + sqrt(9.0 * ht * ht + 18.0 * ht + 25.0);
  return num / den;
}

/* Eq. A2: dTheta/dht. */
double or_dtheta_dhtilde(double ht)
{
  if (or_gamma != 0.0) return (or_gamma - 1.0) / or_gamma;
  double s = sqrt(9.0 * ht * ht + 18.0 * ht + 25.0);
  double den = 5.0 * ht + 5.0 + s;
  return (4.0 * ht + 4.0) / den - (2.0 * ht * ht + 4.0 * ht) * ((9.0 * ht + 9.0) / s + 5.0) / (den * den);
}

/* Eq. 14: squared sound speed of the TM EoS; polytropic: Gamma Theta / h. */
double or_cs2(double th)
{
  if (or_gamma != 0.0) return or_gamma * th / or_h_of_theta(th);
  double h = or_h_of_theta(th);
  return th / (3.0 * h) * (5.0 * h - 8.0 * th) / (h - th);
}

/* ===================================================================================== */
/* The inversion equation (Eq. 15) and its derivative (Eq. A1)                           */
/* ===================================================================================== */

/* Eq. 15 right-hand side with Theta supplied (used by prim -> cons, where Theta = p/rho). */
double or_f_given_theta(double ht, double th, double m2)
{
  double h = ht + 1.0;
  return ht * ht + 2.0 * ht - 2.0 * th * h + th * th * h * h / (h * h + m2);
}

/* Eq. 15 with Theta = Theta(ht) from Eq. 16 (used by cons -> prim). */
double or_f(double ht, double m2) { return or_f_given_theta(ht, or_theta_of_htilde(ht), m2); }

/* Eq. A1: df/dht. */
double or_dfdh(double ht, double m2)
{
  double th = or_theta_of_htilde(ht);
  double dth = or_dtheta_dhtilde(ht);
  double h = ht + 1.0;
  double q = h * h + m2;
  double num = 2.0 * th * h * h * h * h * dth + 2.0 * th * h * m2 * (h * dth + th);
  return 2.0 * ht + 2.0 - 2.0 * th - 2.0 * h * dth + num / (q * q);
}

/* ===================================================================================== */
/* Analytic initial guesses (App. A)                                                     */
/* ===================================================================================== */

/* Cold gas: positive root of the second-order expansion Eq. A3,
 *   L = (6/5) ht + [43/125 + 4/(25 (1+m^2))] ht^2,
 * written without a subtraction.  The printed Eq. A4 puts the product under a square root in
 * the numerator; the positive root of A3 has the plain product there (and the factor
 * 43 m^2 + 63 cancels), which is the form used here. */
double or_guess_cold(double L, double m2)
{
  double a = 1.0 + m2;
  double b = 43.0 * m2 + 63.0;
  return 125.0 * a * L / (75.0 * a + sqrt(125.0 * a * b * L + 75.0 * 75.0 * a * a));
}

/* Hot gas, Eqs. A5-A6: L = (9/16) ht^2. */
double or_guess_hot(double L) { return 4.0 / 3.0 * sqrt(L); }

/* Eq. A7: threshold between the two guesses. */
double or_guess_threshold(double m2)
{
  double r = 1800.0 * (1.0 + m2) / (437.0 * m2 + 117.0);
  return r * r;
}

/* App. A: choose hot when L exceeds the threshold, cold otherwise. */
double or_guess_analytic(double L, double m2)
{
  return (L > or_guess_threshold(m2)) ? or_guess_hot(L) : or_guess_cold(L, m2);
}

/* ===================================================================================== */
/* Exact left-hand side of Eq. 15                                                        */
/* ===================================================================================== */

/* Correctly rounded sum of n doubles (n <= 32): keep a list of non-overlapping partial sums
 * that add up exactly to the running total (error-free two-sum), then round the exact total
 * to nearest-even by summing the partials from the largest, with the half-way correction
 * (Shewchuk 1997, "Adaptive precision floating-point arithmetic"). */
double or_sum_exact(const double *x, int n)
{
  double part[64];
  int np = 0;
  for (int i = 0; i < n; i++) {
    double v = x[i];
    int k = 0;
    for (int j = 0; j < np; j++) {
      double y = part[j];
      if (fabs(v) < fabs(y)) { double t = v; v = y; y = t; }
      double hi = v + y;
      double lo = y - (hi - v);
      if (lo != 0.0) part[k++] = lo;
      v = hi;
    }
    part[k++] = v;
    np = k;
  }
  if (np == 0) return 0.0;
  double hi = part[--np];
  double lo = 0.0;
  while (np > 0) {
    double v = hi;
    double y = part[--np];
    hi = v + y;
    double yr = hi - v;
    lo = y - yr;
    if (lo != 0.0) break;
  }
  if (np > 0 && ((lo < 0.0 && part[np - 1] < 0.0) || (lo > 0.0 && part[np - 1] > 0.0))) {
    double y = lo * 2.0;
    double v = hi + y;
    double yr = v - hi;
    if (y == yr) hi = v;
  }
  return hi;
}

/* L = (Et/D)^2 + 2 (Et/D) - (|M|/D)^2, the left-hand side of Eq. 15 and of the physical check
 * Eq. 30.  Its numerator N = Et^2 + 2 Et D - |M|^2 is summed exactly from error-free products
 * (a*b = p + e with e = fma(a, b, -p)) and rounded once; then L = (N / D) / D.  Computing L
 * this way removes the cancellation error (1 + Mach^2) eps of Eq. 20 from the conversion. */
double or_L_exact(double D, double Mx, double My, double Mz, double Et)
{
  double t[10];
  t[0] = Et * Et;        t[1] = fma(Et, Et, -t[0]);
  t[2] = 2.0 * Et * D;   t[3] = fma(2.0 * Et, D, -t[2]);
  t[4] = -(Mx * Mx);     t[5] = -fma(Mx, Mx, t[4]);
  t[6] = -(My * My);     t[7] = -fma(My, My, t[6]);
  t[8] = -(Mz * Mz);     t[9] = -fma(Mz, Mz, t[8]);
  double N = or_sum_exact(t, 10);
  return (N / D) / D;
}

/* The paper-literal evaluation from the divided variables, x = Et/D, m = |M|/D (Eq. 15 LHS);
 * its rounding error follows Eq. 20.  Kept to reproduce the error model of App. B. */
double or_L_naive(double D, double Mx, double My, double Mz, double Et)
{
  double x = Et / D;
  double mx = Mx / D, my = My / D, mz = Mz / D;
  return x * x + 2.0 * x - (mx * mx + my * my + mz * mz);
}

/* Original (total-energy) scheme: (E/D)^2 - (|M|/D)^2 - 1 with E = Et + D (Eq. 21). */
double or_L_total_energy(double D, double Mx, double My, double Mz, double E)
{
  double e = E / D;
  double mx = Mx / D, my = My / D, mz = Mz / D;
  return e * e - (mx * mx + my * my + mz * mz) - 1.0;
}

/* The physical-state criterion of Eq. 30 (strict), with D > 0, Et > 0 and finiteness. */
int or_is_physical(const double u[5])
{
  if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(u[3]) && isfinite(u[4])))
    return 0;
  if (!(u[0] > 0.0) || !(u[4] > 0.0)) return 0;
  return or_L_exact(u[0], u[1], u[2], u[3], u[4]) > DBL_EPSILON;
}

/* ===================================================================================== */
/* Root of f(ht) = L                                                                     */
/* ===================================================================================== */

/* f is increasing (Sec. 2.3); f <= ht^2 + 2 ht gives ht >= L / (1 + sqrt(1 + L)), and
 * f >= (6/5) ht (slope 6/5 at 0, Eq. A3) gives ht <= L / 1.2.  The bracket is checked and
 * widened if the floating-point f disagrees.  Newton steps (Eq. A1) are taken when they stay
 * strictly inside the bracket; otherwise the bracket is bisected. */
double or_solve_htilde(double L, double m2, int *iters)
{
  double lo = L / (1.0 + sqrt(1.0 + L));
  double hi = L / 1.2;
  int n = 0;
  while (or_f(lo, m2) > L && n < 2000) { lo *= 0.5; n++; }
  while (or_f(hi, m2) < L && n < 4000) { hi *= 2.0; n++; }
  double x = 0.5 * (lo + hi);
  int it;
  for (it = 1; it <= 300; it++) {
    double r = or_f(x, m2) - L;
    if (r == 0.0) break;
    if (r > 0.0) hi = x; else lo = x;
    double xn = x - r / or_dfdh(x, m2);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    double step = fabs(xn - x);
    x = xn;
    if (step <= 0x1p-52 * x) break;
    if (hi - lo <= 0x1p-53 * hi) break;
  }
  if (iters) *iters = it;
  return x;
}

/* ===================================================================================== */
/* Conversions                                                                           */
/* ===================================================================================== */

/* prim (rho, Ux, Uy, Uz, p) -> cons (D, Mx, My, Mz, Et): Eqs. 8, 5a, 22, 5b, 15, 23. */
void or_prim2cons_one(const double w[5], double u[5])
{
  double rho = w[0], ux = w[1], uy = w[2], uz = w[3], p = w[4];
  double U2 = ux * ux + uy * uy + uz * uz;
  double gam = sqrt(1.0 + U2);                 /* Eq. 8  */
  double D = rho * gam;                        /* Eq. 5a */
  double th = p / rho;                         /* Eq. 18 */
  double ht = or_htilde_of_theta(th);          /* Eq. 22 */
  double h = 1.0 + ht;
  double Dh = D * h;
  double m2 = h * h * U2;                      /* (|M|/D)^2 */
  double f = or_f_given_theta(ht, th, m2);     /* Eq. 15 */
  u[0] = D;
  u[1] = Dh * ux;                              /* Eq. 5b */
  u[2] = Dh * uy;
  u[3] = Dh * uz;
  u[4] = D * (m2 + f) / (1.0 + sqrt(1.0 + m2 + f));  /* Eq. 23 */
}

/* cons -> prim.  Returns a status code; on OR_ST_UNPHYSICAL the primitives are NaN.
 * Physical check (Eq. 30, strict): D > 0, Et > 0, all inputs finite and L > DBL_EPSILON. */
int or_cons2prim_one(const double u[5], double w[5], double *ht_out, int *iters)
{
  double D = u[0], Mx = u[1], My = u[2], Mz = u[3], Et = u[4];
  int it = 0;
  if (!(isfinite(D) && isfinite(Mx) && isfinite(My) && isfinite(Mz) && isfinite(Et)) ||
      !(D > 0.0) || !(Et > 0.0)) {
    for (int k = 0; k < 5; k++) w[k] = NAN;
    if (ht_out) *ht_out = NAN;
    if (iters) *iters = 0;
    return OR_ST_UNPHYSICAL;
  }
  double L = or_L_exact(D, Mx, My, Mz, Et);
  if (!(L > DBL_EPSILON)) {
    for (int k = 0; k < 5; k++) w[k] = NAN;
    if (ht_out) *ht_out = NAN;
    if (iters) *iters = 0;
    return OR_ST_UNPHYSICAL;
  }
  double mx = Mx / D, my = My / D, mz = Mz / D;
  double m2 = mx * mx + my * my + mz * mz;
  double ht = or_solve_htilde(L, m2, &it);
  double h = 1.0 + ht;
  double ux = Mx / (D * h), uy = My / (D * h), uz = Mz / (D * h);   /* Eq. 17 */
  double gam = sqrt(1.0 + ux * ux + uy * uy + uz * uz);            /* Eq. 8  */
  double rho = D / gam;                                              /* Eq. 5a */
  double th = or_theta_of_htilde(ht);                                /* Eq. 16 */
  w[0] = rho;
  w[1] = ux;
  w[2] = uy;
  w[3] = uz;
  w[4] = rho * th;                                                   /* Eq. 18 */
  if (ht_out) *ht_out = ht;
  if (iters) *iters = it;
  return OR_ST_OK;
}

/* Original scheme: prim -> (D, Mx, My, Mz, E) with E = rho h gamma^2 - p (Eq. 5c), h of Eq. 10. */
void or_prim2cons_total_one(const double w[5], double u[5])
{
  double rho = w[0], ux = w[1], uy = w[2], uz = w[3], p = w[4];
  double U2 = ux * ux + uy * uy + uz * uz;
  double gam = sqrt(1.0 + U2);
  double D = rho * gam;
  double h = or_h_of_theta(p / rho);
  double Dh = D * h;
  u[0] = D;
  u[1] = Dh * ux;
  u[2] = Dh * uy;
  u[3] = Dh * uz;
  u[4] = Dh * gam - p;
}

/* Original scheme: (D, M, E) -> prim with L = (E/D)^2 - (|M|/D)^2 - 1 evaluated from the divided
 * variables (Eq. 21's cancellation), the same root of Eq. 15 and the same recovery. */
int or_cons2prim_total_one(const double u[5], double w[5], double *ht_out, int *iters)
{
  double D = u[0], Mx = u[1], My = u[2], Mz = u[3], E = u[4];
  int it = 0;
  double L = (isfinite(D) && isfinite(Mx) && isfinite(My) && isfinite(Mz) && isfinite(E) &&
              D > 0.0 && E > 0.0) ? or_L_total_energy(D, Mx, My, Mz, E) : 0.0;
  if (!(L > DBL_EPSILON)) {
    for (int k = 0; k < 5; k++) w[k] = NAN;
    if (ht_out) *ht_out = NAN;
    if (iters) *iters = 0;
    return OR_ST_UNPHYSICAL;
  }
  double mx = Mx / D, my = My / D, mz = Mz / D;
  double m2 = mx * mx + my * my + mz * mz;
  double ht = or_solve_htilde(L, m2, &it);
  double h = 1.0 + ht;
  double ux = Mx / (D * h), uy = My / (D * h), uz = Mz / (D * h);
  double gam = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
  double rho = D / gam;
  double th = or_theta_of_htilde(ht);
  w[0] = rho;
  w[1] = ux;
  w[2] = uy;
  w[3] = uz;
  w[4] = rho * th;
  if (ht_out) *ht_out = ht;
  if (iters) *iters = it;
  return OR_ST_OK;
}

void or_prim2cons_total(int64_t n, const double *prim, double *cons)
{
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double w[5], u[5];
    for (int k = 0; k < 5; k++) w[k] = prim[k * n + i];
    or_prim2cons_total_one(w, u);
    for (int k = 0; k < 5; k++) cons[k * n + i] = u[k];
  }
}

/* Batch forms over structure-of-arrays [5][n]. */
void or_prim2cons(int64_t n, const double *prim, double *cons)
{
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double w[5], u[5];
    for (int k = 0; k < 5; k++) w[k] = prim[k * n + i];
    or_prim2cons_one(w, u);
    for (int k = 0; k < 5; k++) cons[k * n + i] = u[k];
  }
}

void or_cons2prim(int64_t n, const double *cons, double *prim, int8_t *status, int32_t *iters)
{
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; i++) {
    double w[5], u[5];
    int it = 0;
    for (int k = 0; k < 5; k++) u[k] = cons[k * n + i];
    int st = or_cons2prim_one(u, w, NULL, &it);
    for (int k = 0; k < 5; k++) prim[k * n + i] = w[k];
    if (status) status[i] = (int8_t)st;
    if (iters) iters[i] = it;
  }
}

void or_L_batch(int64_t n, const double *cons, int mode, double *L)
{
  for (int64_t i = 0; i < n; i++) {
    double D = cons[i], Mx = cons[n + i], My = cons[2 * n + i], Mz = cons[3 * n + i], Et = cons[4 * n + i];
    if (mode == 0) L[i] = or_L_exact(D, Mx, My, Mz, Et);
    else if (mode == 1) L[i] = or_L_naive(D, Mx, My, Mz, Et);
    else L[i] = or_L_total_energy(D, Mx, My, Mz, Et + D);
  }
}

/* ===================================================================================== */
/* CFL (Sec. 3.3)                                                                        */
/* ===================================================================================== */

/* Eqs. 26-27 for one cell: U_max = gamma_s (|Ux| + |Uy| + |Uz|) + 3 gamma U_s (the printed
 * Eq. 26 repeats |U_z|; the text sums every spatial component), S_max = U_max / sqrt(1 + U_max^2). */
double or_smax_prim(const double w[5])
{
  double th = w[4] / w[0];
  double cs2 = or_cs2(th);
  double gs = 1.0 / sqrt(1.0 - cs2);        /* gamma_s */
  double Us = sqrt(cs2) * gs;               /* U_s = c_s / sqrt(1 - c_s^2) */
  double gam = sqrt(1.0 + w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  double Umax = gs * (fabs(w[1]) + fabs(w[2]) + fabs(w[3])) + 3.0 * gam * Us;
  return Umax / sqrt(1.0 + Umax * Umax);
}

/* Max S_max over the interior cells of each patch of an interior array [P][5][8^3] of
 * conserved variables.  Unphysical cells are counted and skipped. */
void or_patch_smax(int64_t n_patch, const double *interior, double *smax, int64_t *n_unphys)
{
  int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int64_t p = 0; p < n_patch; p++) {
    const double *q = interior + p * NF * 512;
    double s = 0.0;
    for (int c = 0; c < 512; c++) {
      double u[5], w[5];
      for (int k = 0; k < 5; k++) u[k] = q[k * 512 + c];
      if (or_cons2prim_one(u, w, NULL, NULL) != OR_ST_OK) { bad++; continue; }
      double sc = or_smax_prim(w);
      if (sc > s) s = sc;
    }
    smax[p] = s;
  }
  if (n_unphys) *n_unphys = bad;
}

/* ===================================================================================== */
/* PLM (hybrid van Leer / generalized minmod)                                            */
/* ===================================================================================== */

/* Limited slope of a cell from its left and right neighbours: zero at an extremum, else the
 * smallest magnitude among the van Leer (harmonic) slope and theta times each one-sided
 * difference, with the sign of the differences. */
double or_slope(double wl, double wc, double wr, double theta)
{
  double dl = wc - wl;
  double dr = wr - wc;
  if (!((dl > 0.0 && dr > 0.0) || (dl < 0.0 && dr < 0.0))) return 0.0;
  double vl = fabs(2.0 * dl * dr / (dl + dr));
  double a = theta * fabs(dl);
  double b = theta * fabs(dr);
  double s = vl;
  if (a < s) s = a;
  if (b < s) s = b;
  return (dl > 0.0) ? s : -s;
}

/* ===================================================================================== */
/* Fluxes and Riemann solvers                                                            */
/* ===================================================================================== */

/* Physical flux along direction d (0, 1, 2) from Eqs. 4a, 4b and 7, with v_d = U_d / gamma. */
void or_flux(int d, const double w[5], const double u[5], double F[5])
{
  double gam = sqrt(1.0 + w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  double v = w[1 + d] / gam;
  F[0] = u[0] * v;
  F[1] = u[1] * v;
  F[2] = u[2] * v;
  F[3] = u[3] * v;
  F[1 + d] += w[4];
  F[4] = (u[4] + w[4]) * v;
}

/* Signal speeds along d of one state: the relativistic addition of flow and sound speed,
 * lambda_pm = [v_d (1 - cs^2) +- cs sqrt((1 - v^2)(1 - v^2 cs^2 - v_d^2 (1 - cs^2)))] / (1 - v^2 cs^2),
 * written here in four-velocity (multiply through by gamma^2):
 * lambda_pm = [gamma U_d (1 - cs^2) +- cs sqrt(1 + U_perp^2 (1 - cs^2))] / (1 + U^2 (1 - cs^2)). */
void or_wavespeeds(int d, const double w[5], double *lm, double *lp)
{
  double th = w[4] / w[0];
  double cs2 = or_cs2(th);
  double cs = sqrt(cs2);
  double Ud = w[1 + d];
  double Up2 = 0.0;
  for (int k = 0; k < 3; k++)
    if (k != d) Up2 += w[1 + k] * w[1 + k];
  double U2 = Ud * Ud + Up2;
  double gam = sqrt(1.0 + U2);
  double a = 1.0 - cs2;
  double den = 1.0 + U2 * a;
  double s = cs * sqrt(1.0 + Up2 * a);
  *lm = (gam * Ud * a - s) / den;
  *lp = (gam * Ud * a + s) / den;
}

/* The energy variable of a scheme: 0 the reduced energy Et (this paper), 1 the total energy E
 * (the original scheme, evolved with the flux M_d of Eq. 4b). */
static void sc_prim2cons(int scheme, const double w[5], double u[5])
{
  if (scheme) or_prim2cons_total_one(w, u);
  else or_prim2cons_one(w, u);
}

static int sc_cons2prim(int scheme, const double u[5], double w[5], int *iters)
{
  return scheme ? or_cons2prim_total_one(u, w, NULL, iters) : or_cons2prim_one(u, w, NULL, iters);
}

static void sc_flux(int scheme, int d, const double w[5], const double u[5], double F[5])
{
  or_flux(d, w, u, F);
  if (scheme) F[4] = u[1 + d];              /* (E + p) v_d = M_d */
}

static int sc_is_physical(int scheme, const double u[5])
{
  if (!scheme) return or_is_physical(u);
  if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(u[3]) && isfinite(u[4])))
    return 0;
  if (!(u[0] > 0.0) || !(u[4] > 0.0)) return 0;
  return or_L_total_energy(u[0], u[1], u[2], u[3], u[4]) > DBL_EPSILON;
}

/* HLLE flux along d between left/right primitive states. */
static void sc_hlle(int scheme, int d, const double wl[5], const double wr[5], double F[5])
{
  double ul[5], ur[5], fl[5], fr[5];
  double lmL, lpL, lmR, lpR;
  sc_prim2cons(scheme, wl, ul);
  sc_prim2cons(scheme, wr, ur);
  sc_flux(scheme, d, wl, ul, fl);
  sc_flux(scheme, d, wr, ur, fr);
  or_wavespeeds(d, wl, &lmL, &lpL);
  or_wavespeeds(d, wr, &lmR, &lpR);
  double sl = fmin(fmin(lmL, lmR), 0.0);
  double sr = fmax(fmax(lpL, lpR), 0.0);
  for (int k = 0; k < 5; k++)
    F[k] = (sr * fl[k] - sl * fr[k] + sr * sl * (ur[k] - ul[k])) / (sr - sl);
}

void or_hlle(int d, const double wl[5], const double wr[5], double F[5]) { sc_hlle(0, d, wl, wr, F); }

/* HLLC flux along d (Mignone & Bodo 2005, as adapted in Sec. 3.2 to the TM sound speed and to
 * the reduced energy).  The HLL average of the total energy E = Et + D (flux M_d) and of M_d
 * gives the contact speed lambda* as the root of F^E l^2 - (E + F^m) l + m = 0 that lies between
 * the signal speeds, written 2m / (B + sqrt(B^2 - 4 F^E m)), B = E + F^m; then p* = F^m - lambda* F^E.
 * Star state of side K (speed S, three-velocity v_d):
 *   D*  = D (S - v) / (S - l*),           M_perp* = M_perp (S - v) / (S - l*),
 *   M_d* = [M_d (S - v) + p* - p] / (S - l*),
 *   Et* = [Et (S - v) + p* l* - p v] / (S - l*)   (= E* - D*, no rest-mass cancellation),
 * and F* = F_K + S (U* - U_K). */
static void sc_hllc(int scheme, int d, const double wl[5], const double wr[5], double F[5])
{
  double ul[5], ur[5], fl[5], fr[5];
  double lmL, lpL, lmR, lpR;
  sc_prim2cons(scheme, wl, ul);
  sc_prim2cons(scheme, wr, ur);
  sc_flux(scheme, d, wl, ul, fl);
  sc_flux(scheme, d, wr, ur, fr);
  or_wavespeeds(d, wl, &lmL, &lpL);
  or_wavespeeds(d, wr, &lmR, &lpR);
  double sl = fmin(lmL, lmR);
  double sr = fmax(lpL, lpR);
  if (sl >= 0.0) { for (int k = 0; k < 5; k++) F[k] = fl[k]; return; }
  if (sr <= 0.0) { for (int k = 0; k < 5; k++) F[k] = fr[k]; return; }
  double uh[5], fh[5];
  for (int k = 0; k < 5; k++) {
    uh[k] = (sr * ur[k] - sl * ul[k] + fl[k] - fr[k]) / (sr - sl);
    fh[k] = (sl * sr * (ur[k] - ul[k]) + sr * fl[k] - sl * fr[k]) / (sr - sl);
  }
  double E = scheme ? uh[4] : uh[4] + uh[0];     /* total energy of the HLL state */
  double FE = scheme ? fh[4] : fh[4] + fh[0];    /* its flux */
  double m = uh[1 + d];
  double Fm = fh[1 + d];
  double B = E + Fm;
  double disc = B * B - 4.0 * FE * m;
  if (disc < 0.0) disc = 0.0;
  double ls = 2.0 * m / (B + sqrt(disc));
  double ps = Fm - ls * FE;
  const double *w, *u, *f;
  double S;
  if (ls >= 0.0) { w = wl; u = ul; f = fl; S = sl; }
  else           { w = wr; u = ur; f = fr; S = sr; }
  double gam = sqrt(1.0 + w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  double v = w[1 + d] / gam;
  double p = w[4];
  double inv = 1.0 / (S - ls);
  double us[5];
  us[0] = u[0] * (S - v) * inv;
  for (int k = 0; k < 3; k++) us[1 + k] = u[1 + k] * (S - v) * inv;
  us[1 + d] = (u[1 + d] * (S - v) + ps - p) * inv;
  us[4] = (u[4] * (S - v) + ps * ls - p * v) * inv;     /* the same form for Et* and E* */
  for (int k = 0; k < 5; k++) F[k] = f[k] + S * (us[k] - u[k]);
}

void or_hllc(int d, const double wl[5], const double wr[5], double F[5]) { sc_hllc(0, d, wl, wr, F); }

/* ===================================================================================== */
/* MUSCL-Hancock step on one padded patch                                                */
/* ===================================================================================== */

/* Padded patch geometry: cells (x, y, z) with interior coordinates i in [-g, 8+g); the array
 * index of interior coordinate i is i + g.  Layout [field][z][y][x]. */
typedef struct {
  int g, N;
  const double *q;          /* padded conserved variables of this patch */
} or_patch;

static double or_get(const or_patch *P, int f, int i, int j, int k)
{
  int N = P->N, g = P->g;
  return P->q[(((int64_t)f * N + (k + g)) * N + (j + g)) * N + (i + g)];
}

/* Cells whose half-step face states the full step needs: all interior cells and the cells
 * one step outside a face of the patch. */
static int or_in_half(int i, int j, int k)
{
  int c[3] = {i, j, k};
  int out = 0;
  for (int d = 0; d < 3; d++) {
    if (c[d] >= 0 && c[d] < PS) continue;
    if (c[d] == -1 || c[d] == PS) out++;
    else return 0;
  }
  return out <= 1;
}

/* Box of cells [-2, 10)^3 that the step can touch (2 ghost layers suffice for PLM + MHM). */
#define OB 12
#define OIDX(i, j, k) ((((k) + 2) * OB + ((j) + 2)) * OB + ((i) + 2))

typedef struct {
  int64_t unphys, noconv;
  int64_t iters;
  int centre_bad;           /* an input cell of the stencil is unphysical (no retry helps) */
  int face_bad;             /* a half-step face state failed the inversion */
  int64_t pred_fallback;    /* VL predictor states replaced by the cell's state at t^n */
} or_counts;

/* Centre primitives, computed once per needed cell. */
typedef struct {
  double w[OB * OB * OB][5];
  unsigned char have[OB * OB * OB];
  const or_patch *P;
  or_counts *cnt;
  int scheme;
} or_prim_cache;

static const double *or_cell_prim(or_prim_cache *C, int i, int j, int k)
{
  int id = OIDX(i, j, k);
  if (!C->have[id]) {
    double u[5];
    int it = 0;
    for (int f = 0; f < 5; f++) u[f] = or_get(C->P, f, i, j, k);
    int st = sc_cons2prim(C->scheme, u, C->w[id], &it);
    if (st == OR_ST_UNPHYSICAL) { C->cnt->unphys++; C->cnt->centre_bad = 1; }
    C->cnt->iters += it;
    C->have[id] = 1;
  }
  return C->w[id];
}

/* Step of one patch with limiter coefficient theta.  Writes out[5][512], the updated interior
 * conserved variables, and returns the number of them that fail the physical check (Eq. 30). */
/* Boundary fluxes of a patch: bflux[s][f][b * 8 + a] for face s = 2 d + u (u = 1: the upper
 * face), (a, b) the transverse coordinates in increasing axis order; interface fluxes fx are
 * indexed (d * 64 + a' * 8 + b') * 9 + c as in the steps below, with a' the higher and b' the
 * lower transverse axis. */
static void or_boundary_fluxes(const double (*fx)[5], double *bflux)
{
  if (!bflux) return;
  for (int d = 0; d < 3; d++)
    for (int u = 0; u < 2; u++)
      for (int b = 0; b < PS; b++)
        for (int a = 0; a < PS; a++)
          for (int f = 0; f < NF; f++)
            bflux[((2 * d + u) * NF + f) * 64 + b * 8 + a] = fx[(d * 64 + b * 8 + a) * 9 + (u ? PS : 0)][f];
}

static int or_step_patch(const or_patch *P, double dt, double dh, double theta, int riemann,
                          int scheme, double *out, or_counts *cnt, double *bflux)
{
  or_prim_cache *C = (or_prim_cache *)calloc(1, sizeof(or_prim_cache));
  C->P = P;
  C->cnt = cnt;
  C->scheme = scheme;
  /* Half-step face conserved states U_face^{n+1/2} of the cells that need them:
   * hf[cell][d][s][field], s = 0 for the minus face, 1 for the plus face. */
  double (*hf)[3][2][5] = (double (*)[3][2][5])calloc(OB * OB * OB, sizeof(*hf));
  double half = 0.5 * dt / dh;
  for (int k = -1; k <= PS; k++)
    for (int j = -1; j <= PS; j++)
      for (int i = -1; i <= PS; i++) {
        if (!or_in_half(i, j, k)) continue;
        const double *wc = or_cell_prim(C, i, j, k);
        double wf[3][2][5], uf[3][2][5], ff[3][2][5];
        for (int d = 0; d < 3; d++) {
          int di = (d == 0), dj = (d == 1), dk = (d == 2);
          const double *wm = or_cell_prim(C, i - di, j - dj, k - dk);
          const double *wp = or_cell_prim(C, i + di, j + dj, k + dk);
          for (int f = 0; f < 5; f++) {
            double s = or_slope(wm[f], wc[f], wp[f], theta);
            wf[d][0][f] = wc[f] - 0.5 * s;
            wf[d][1][f] = wc[f] + 0.5 * s;
          }
          for (int s = 0; s < 2; s++) {
            sc_prim2cons(scheme, wf[d][s], uf[d][s]);
            sc_flux(scheme, d, wf[d][s], uf[d][s], ff[d][s]);
          }
        }
        double corr[5];
        for (int f = 0; f < 5; f++) {
          double acc = 0.0;
          for (int d = 0; d < 3; d++) acc += ff[d][1][f] - ff[d][0][f];
          corr[f] = -half * acc;
        }
        int id = OIDX(i, j, k);
        for (int d = 0; d < 3; d++)
          for (int s = 0; s < 2; s++)
            for (int f = 0; f < 5; f++) hf[id][d][s][f] = uf[d][s][f] + corr[f];
      }
  /* Interface fluxes: x-interface (i - 1/2, j, k) for i in [0, 8], j, k in [0, 8), etc.
   * fl[d][interface][field] with interface index (a * 8 + b) * 9 + c, c along d. */
  double (*fx)[5] = (double (*)[5])calloc(3 * 9 * 64, sizeof(*fx));
  for (int d = 0; d < 3; d++)
    for (int a = 0; a < PS; a++)
      for (int b = 0; b < PS; b++)
        for (int c = 0; c <= PS; c++) {
          int cr[3], cl[3];
          /* the two transverse coordinates are (b, a) in increasing axis order */
          int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
          cr[d] = c; cr[t0] = b; cr[t1] = a;
          cl[0] = cr[0]; cl[1] = cr[1]; cl[2] = cr[2];
          cl[d] = c - 1;
          double wl[5], wr[5];
          int itl = 0, itr = 0;
          int stl = sc_cons2prim(scheme, hf[OIDX(cl[0], cl[1], cl[2])][d][1], wl, &itl);
          int str = sc_cons2prim(scheme, hf[OIDX(cr[0], cr[1], cr[2])][d][0], wr, &itr);
          cnt->unphys += (stl == OR_ST_UNPHYSICAL) + (str == OR_ST_UNPHYSICAL);
          if (stl == OR_ST_UNPHYSICAL || str == OR_ST_UNPHYSICAL) cnt->face_bad = 1;
          cnt->iters += itl + itr;
          double *F = fx[(d * 64 + a * 8 + b) * 9 + c];
          if (riemann == OR_HLLE) sc_hlle(scheme, d, wl, wr, F);
          else sc_hllc(scheme, d, wl, wr, F);
        }
  /* Full update: U^{n+1} = U^n - (dt/dh) sum_d (F_{+1/2} - F_{-1/2}). */
  double full = dt / dh;
  for (int k = 0; k < PS; k++)
    for (int j = 0; j < PS; j++)
      for (int i = 0; i < PS; i++) {
        int ci[3] = {i, j, k};
        for (int f = 0; f < 5; f++) {
          double acc = 0.0;
          for (int d = 0; d < 3; d++) {
            int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
            int a = ci[t1], b = ci[t0], c = ci[d];
            const double *Fm = fx[(d * 64 + a * 8 + b) * 9 + c];
            const double *Fp = fx[(d * 64 + a * 8 + b) * 9 + c + 1];
            acc += Fp[f] - Fm[f];
          }
          out[f * 512 + (k * PS + j) * PS + i] = or_get(P, f, i, j, k) - full * acc;
        }
      }
  or_boundary_fluxes((const double (*)[5])fx, bflux);
  int nbad = 0;
  for (int c = 0; c < 512; c++) {
    double u[5];
    for (int f = 0; f < 5; f++) u[f] = out[f * 512 + c];
    nbad += !sc_is_physical(scheme, u);
  }
  free(fx);
  free(hf);
  free(C);
  return nbad;
}

/* ===================================================================================== */
/* VL predictor-corrector step on one padded patch                                       */
/* ===================================================================================== */

/* Box [-3, 11)^3: the predictor reads the neighbours of cells up to two layers outside. */
#define VB 14
#define VIDX(i, j, k) ((((k) + 3) * VB + ((j) + 3)) * VB + ((i) + 3))

/* Cells whose half-step primitives the corrector reads: along each axis d the cells with
 * coordinate d in [-2, 10) and the other two coordinates inside the patch. */
static int or_in_vl_half(int i, int j, int k)
{
  int c[3] = {i, j, k};
  int out = 0;
  for (int d = 0; d < 3; d++) {
    if (c[d] >= 0 && c[d] < PS) continue;
    if (c[d] >= -2 && c[d] < PS + 2) out++;
    else return 0;
  }
  return out <= 1;
}

typedef struct {
  double w[VB * VB * VB][5];
  unsigned char have[VB * VB * VB];
  const or_patch *P;
  or_counts *cnt;
  int scheme;
} or_vl_cache;

static const double *or_vl_prim(or_vl_cache *C, int i, int j, int k)
{
  int id = VIDX(i, j, k);
  if (!C->have[id]) {
    double u[5];
    int it = 0;
    for (int f = 0; f < 5; f++) u[f] = or_get(C->P, f, i, j, k);
    int st = sc_cons2prim(C->scheme, u, C->w[id], &it);
    if (st == OR_ST_UNPHYSICAL) { C->cnt->unphys++; C->cnt->centre_bad = 1; }
    C->cnt->iters += it;
    C->have[id] = 1;
  }
  return C->w[id];
}

static void sc_riemann(int scheme, int riemann, int d, const double wl[5], const double wr[5],
                       double F[5])
{
  if (riemann == OR_HLLE) sc_hlle(scheme, d, wl, wr, F);
  else sc_hllc(scheme, d, wl, wr, F);
}

/* One VL step of one patch with limiter coefficient theta (the corrector's PLM):
 *   predictor  U*(c) = U^n(c) - (dt / 2dh) sum_d [F_d(W_c, W_{c+d}) - F_d(W_{c-d}, W_c)] with
 *              the cell-centre primitives as the face states, then W*(c) = cons -> prim of U*;
 *   corrector  the interface flux from PLM face states of W* (W* -/+ slope/2 on either side),
 *              U^{n+1} = U^n - (dt/dh) sum_d (F_{+1/2} - F_{-1/2}).
 * A predictor state that fails the inversion (no limiter acts on it) is replaced by the cell's
 * state at t^n, W* = W^n: the half step is dropped for that cell.  With theta = 0 (piecewise-
 * constant reconstruction, the retry's last resort) the half step is dropped everywhere, W* = W^n:
 * the first-order Godunov step, as MUSCL-Hancock is with theta = 0.  Returns the number of
 * output cells failing Eq. 30. */
static int or_vl_step_patch(const or_patch *P, double dt, double dh, double theta, int riemann,
                            int scheme, double *out, or_counts *cnt, double *bflux)
{
  or_vl_cache *C = (or_vl_cache *)calloc(1, sizeof(or_vl_cache));
  C->P = P;
  C->cnt = cnt;
  C->scheme = scheme;
  double (*wh)[5] = (double (*)[5])calloc(VB * VB * VB, sizeof(*wh));
  double half = 0.5 * dt / dh;
  for (int k = -2; k < PS + 2; k++)
    for (int j = -2; j < PS + 2; j++)
      for (int i = -2; i < PS + 2; i++) {
        if (!or_in_vl_half(i, j, k)) continue;
        const double *wc = or_vl_prim(C, i, j, k);
        if (theta == 0.0) {
          for (int f = 0; f < 5; f++) wh[VIDX(i, j, k)][f] = wc[f];
          continue;
        }
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int d = 0; d < 3; d++) {
          int di = (d == 0), dj = (d == 1), dk = (d == 2);
          const double *wm = or_vl_prim(C, i - di, j - dj, k - dk);
          const double *wp = or_vl_prim(C, i + di, j + dj, k + dk);
          double Fm[5], Fp[5];
          sc_riemann(scheme, riemann, d, wm, wc, Fm);
          sc_riemann(scheme, riemann, d, wc, wp, Fp);
          for (int f = 0; f < 5; f++) acc[f] += Fp[f] - Fm[f];
        }
        double u[5];
        for (int f = 0; f < 5; f++) u[f] = or_get(P, f, i, j, k) - half * acc[f];
        int it = 0;
        int st = sc_cons2prim(scheme, u, wh[VIDX(i, j, k)], &it);
        cnt->iters += it;
        if (st == OR_ST_UNPHYSICAL) {
          for (int f = 0; f < 5; f++) wh[VIDX(i, j, k)][f] = wc[f];
          cnt->pred_fallback++;
        }
      }
  double (*fx)[5] = (double (*)[5])calloc(3 * 9 * 64, sizeof(*fx));
  for (int d = 0; d < 3; d++)
    for (int a = 0; a < PS; a++)
      for (int b = 0; b < PS; b++)
        for (int c = 0; c <= PS; c++) {
          int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
          int cr[3];
          cr[d] = c; cr[t0] = b; cr[t1] = a;
          int e[3] = {d == 0, d == 1, d == 2};
          /* cells c-2, c-1 (left side) and c, c+1 (right side) along d */
          const double *w[4];
          for (int q = 0; q < 4; q++)
            w[q] = wh[VIDX(cr[0] + (q - 2) * e[0], cr[1] + (q - 2) * e[1], cr[2] + (q - 2) * e[2])];
          double wl[5], wr[5];
          for (int f = 0; f < 5; f++) {
            wl[f] = w[1][f] + 0.5 * or_slope(w[0][f], w[1][f], w[2][f], theta);
            wr[f] = w[2][f] - 0.5 * or_slope(w[1][f], w[2][f], w[3][f], theta);
          }
          sc_riemann(scheme, riemann, d, wl, wr, fx[(d * 64 + a * 8 + b) * 9 + c]);
        }
  double full = dt / dh;
  for (int k = 0; k < PS; k++)
    for (int j = 0; j < PS; j++)
      for (int i = 0; i < PS; i++) {
        int ci[3] = {i, j, k};
        for (int f = 0; f < 5; f++) {
          double acc = 0.0;
          for (int d = 0; d < 3; d++) {
            int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
            int a = ci[t1], b = ci[t0], c = ci[d];
            acc += fx[(d * 64 + a * 8 + b) * 9 + c + 1][f] - fx[(d * 64 + a * 8 + b) * 9 + c][f];
          }
          out[f * 512 + (k * PS + j) * PS + i] = or_get(P, f, i, j, k) - full * acc;
        }
      }
  or_boundary_fluxes((const double (*)[5])fx, bflux);
  int nbad = 0;
  for (int c = 0; c < 512; c++) {
    double u[5];
    for (int f = 0; f < 5; f++) u[f] = out[f * 512 + c];
    nbad += !sc_is_physical(scheme, u);
  }
  free(fx);
  free(wh);
  free(C);
  return nbad;
}

/* Step of every patch.  When a patch's step meets an unphysical state -- a half-step face
 * state that fails the inversion, or an updated cell that fails Eq. 30 -- the patch is redone
 * with the limiter coefficient reduced by 0.75 (Sec. 3.4, "SRHD solver"), at most max_retry
 * times, and finally once with a zero coefficient (piecewise-constant reconstruction).  An
 * unphysical input cell cannot be cured by reconstruction and ends the attempts.
 * integrator 0: MUSCL-Hancock (ghost >= 2); 1: VL (ghost >= 3; only updated cells trigger
 * the retry; a predictor state that fails is replaced by the cell's state at t^n).  bflux (or NULL): [P][6][5][64]
 * fluxes through the six faces of each patch in its final attempt (layout of
 * or_boundary_fluxes).
 * counts = {unphysical inversions + failed output cells of the final attempt, non-converged
 *           inversions, solver iterations, retried attempts, VL predictor fallbacks of the final
 *           attempt}. */
int or_fluid_step(int64_t n_patch, int ghost, const double *padded, const int8_t *level,
                  const double *dh_lev, const double *dt_lev, double theta, int riemann,
                  int max_retry, int scheme, int integrator, double *out, int64_t *counts,
                  double *bflux)
{
  if (ghost < (integrator ? 3 : 2)) return -1;
  int N = PS + 2 * ghost;
  int64_t per = (int64_t)NF * N * N * N;
  int64_t unphys = 0, noconv = 0, iters = 0, retries = 0, pfb = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : unphys, noconv, iters, retries, pfb)
  for (int64_t p = 0; p < n_patch; p++) {
    or_patch P = {ghost, N, padded + p * per};
    int lv = level ? level[p] : 0;
    double th = theta;
    for (int attempt = 0;; attempt++) {
      or_counts c = {0, 0, 0, 0, 0, 0};
      double *bf = bflux ? bflux + p * 6 * NF * 64 : NULL;
      int nbad = integrator
                     ? or_vl_step_patch(&P, dt_lev[lv], dh_lev[lv], th, riemann, scheme, out + p * NF * 512, &c, bf)
                     : or_step_patch(&P, dt_lev[lv], dh_lev[lv], th, riemann, scheme, out + p * NF * 512, &c, bf);
      iters += c.iters;
      int fail = c.face_bad || nbad > 0;
      if (!fail || c.centre_bad || th == 0.0) {
        unphys += c.unphys + nbad;
        noconv += c.noconv;
        pfb += c.pred_fallback;
        break;
      }
      retries++;
      th = (attempt < max_retry) ? 0.75 * th : 0.0;
    }
  }
  if (counts) {
    counts[0] = unphys; counts[1] = noconv; counts[2] = iters; counts[3] = retries; counts[4] = pfb;
  }
  return 0;
}

/* ===================================================================================== */
/* Ghost fill                                                                            */
/* ===================================================================================== */

/* Neighbour table: neighbor[p][n] with n = (oz+1)*9 + (oy+1)*3 + (ox+1) for the offset
 * (ox, oy, oz) in {-1,0,1}^3; entry 13 (offset 0) is the patch's own index in `interior`, so a
 * table of a subset of patches fills just those patches.  -1 in a face entry
 * marks a domain boundary in that direction: there the ghost cells copy the nearest cell
 * inside the domain (outflow, zero gradient).  Periodic domains list wrapped neighbours. */
int or_fill_ghosts(int64_t n_patch, int ghost, int64_t n_src, const double *interior,
                   const int32_t *neighbor, double *padded)
{
  int N = PS + 2 * ghost;
  int64_t per = (int64_t)NF * N * N * N;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t p = 0; p < n_patch; p++) {
    const int32_t *nb = neighbor + p * 27;
    for (int z = 0; z < N; z++)
      for (int y = 0; y < N; y++)
        for (int x = 0; x < N; x++) {
          int c[3] = {x - ghost, y - ghost, z - ghost};
          /* clamp toward the domain where a face neighbour is the domain boundary (-1) */
          for (int d = 0; d < 3; d++) {
            int o = (c[d] < 0) ? -1 : (c[d] >= PS ? 1 : 0);
            if (o == 0) continue;
            int face = 13 + o * (d == 0 ? 1 : (d == 1 ? 3 : 9));
            if (nb[face] == -1) c[d] = (o < 0) ? 0 : PS - 1;
          }
          int o[3];
          for (int d = 0; d < 3; d++) o[d] = (c[d] < 0) ? -1 : (c[d] >= PS ? 1 : 0);
          int slot = (o[2] + 1) * 9 + (o[1] + 1) * 3 + (o[0] + 1);
          int64_t src = nb[slot];
          if (src == OR_NB_COARSE) continue;      /* filled from the coarser level */
          if (src < 0 || src >= n_src) { bad = 1; continue; }
          int si = c[0] - PS * o[0], sj = c[1] - PS * o[1], sk = c[2] - PS * o[2];
          for (int f = 0; f < NF; f++)
            padded[p * per + (((int64_t)f * N + z) * N + y) * N + x] =
                interior[(src * NF + f) * 512 + (sk * PS + sj) * PS + si];
        }
  }
  return bad ? -1 : 0;
}

/* ===================================================================================== */
/* AMR neighbour operations (Sec. 3.4 items 3 and 4; refinement ratio 2)                 */
/* ===================================================================================== */

/* The neighbour slot that a padded cell's value comes from, after the outflow clamp; writes the
 * (possibly clamped) interior coordinates to c. */
static int or_ghost_slot(const int32_t *nb, int c[3])
{
  for (int d = 0; d < 3; d++) {
    int o = (c[d] < 0) ? -1 : (c[d] >= PS ? 1 : 0);
    if (o == 0) continue;
    int face = 13 + o * (d == 0 ? 1 : (d == 1 ? 3 : 9));
    if (nb[face] == -1) c[d] = (o < 0) ? 0 : PS - 1;
  }
  int o[3];
  for (int d = 0; d < 3; d++) o[d] = (c[d] < 0) ? -1 : (c[d] >= PS ? 1 : 0);
  return (o[2] + 1) * 9 + (o[1] + 1) * 3 + (o[0] + 1);
}

/* Coarse-to-fine ghost fill.  A ghost cell of fine patch p whose neighbour slot is
 * OR_NB_COARSE lies on the parent level: with I = 8 b + c the cell's fine index relative to the
 * parent (b the patch's octant bit along that axis, c its coordinate in the patch), the coarse
 * cell is C = floor(I / 2) and the fine cell's centre sits at -1/4 or +1/4 of a coarse cell from
 * C's centre.  The value is the coarse state (time-interpolated, (1 - alpha) old + alpha new)
 * plus the limited coarse slope along each axis times that offset -- a linear interpolation
 * whose eight children average back to the coarse value.  The conserved variables are
 * interpolated; if the result fails Eq. 30 the primitive variables of the same coarse cells are
 * interpolated instead and converted back (Sec. 3.4, ghost-zone interpolation).
 * coarse_*: padded parents [n_coarse][5][Nc^3] with ghost_c >= ghost / 2 + 2 layers. */
static void or_coarse_state(const double *co, const double *cn, double alpha, int Nc, int gc,
                            int ci, int cj, int ck, double u[5])
{
  int64_t N3 = (int64_t)Nc * Nc * Nc;
  int64_t off = ((int64_t)(ck + gc) * Nc + (cj + gc)) * Nc + (ci + gc);
  for (int f = 0; f < 5; f++) {
    double a = co[f * N3 + off];
    u[f] = cn ? (1.0 - alpha) * a + alpha * cn[f * N3 + off] : a;
  }
}

int or_fill_ghosts_coarse(int64_t n_fine, int ghost, const int32_t *neighbor, const int32_t *parent,
                          const int8_t *octant, int64_t n_coarse, int ghost_c,
                          const double *coarse_old, const double *coarse_new, double alpha,
                          double theta, double *fine_padded, int64_t *counts)
{
  if (ghost_c < ghost / 2 + 2) return -1;
  int N = PS + 2 * ghost, Nc = PS + 2 * ghost_c;
  int64_t per = (int64_t)NF * N * N * N, perc = (int64_t)NF * Nc * Nc * Nc;
  int64_t n_interp = 0, n_fallback = 0;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_interp, n_fallback) reduction(| : bad)
  for (int64_t p = 0; p < n_fine; p++) {
    const int32_t *nb = neighbor + p * 27;
    int64_t par = parent[p];
    if (par < 0 || par >= n_coarse) { bad = 1; continue; }
    const double *co = coarse_old + par * perc;
    const double *cn = coarse_new ? coarse_new + par * perc : NULL;
    int bit[3] = {octant[p] & 1, (octant[p] >> 1) & 1, (octant[p] >> 2) & 1};
    for (int z = 0; z < N; z++)
      for (int y = 0; y < N; y++)
        for (int x = 0; x < N; x++) {
          int c[3] = {x - ghost, y - ghost, z - ghost};
          if (c[0] >= 0 && c[0] < PS && c[1] >= 0 && c[1] < PS && c[2] >= 0 && c[2] < PS) continue;
          int cc[3] = {c[0], c[1], c[2]};
          if (nb[or_ghost_slot(nb, cc)] != OR_NB_COARSE) continue;
          int C[3];
          double sgn[3];
          for (int d = 0; d < 3; d++) {
            int I = 8 * bit[d] + c[d];
            C[d] = (I >= 0) ? I / 2 : -((1 - I) / 2);       /* floor(I / 2) */
            sgn[d] = (I - 2 * C[d]) ? 0.25 : -0.25;
          }
          double u0[5], um[3][5], up[3][5];
          or_coarse_state(co, cn, alpha, Nc, ghost_c, C[0], C[1], C[2], u0);
          for (int d = 0; d < 3; d++) {
            int e[3] = {d == 0, d == 1, d == 2};
            or_coarse_state(co, cn, alpha, Nc, ghost_c, C[0] - e[0], C[1] - e[1], C[2] - e[2], um[d]);
            or_coarse_state(co, cn, alpha, Nc, ghost_c, C[0] + e[0], C[1] + e[1], C[2] + e[2], up[d]);
          }
          double u[5];
          for (int f = 0; f < 5; f++) {
            u[f] = u0[f];
            for (int d = 0; d < 3; d++) u[f] += sgn[d] * or_slope(um[d][f], u0[f], up[d][f], theta);
          }
          n_interp++;
          if (!or_is_physical(u)) {
            double w0[5], wm[3][5], wp[3][5], w[5];
            int it;
            or_cons2prim_one(u0, w0, NULL, &it);
            for (int d = 0; d < 3; d++) {
              or_cons2prim_one(um[d], wm[d], NULL, &it);
              or_cons2prim_one(up[d], wp[d], NULL, &it);
            }
            for (int f = 0; f < 5; f++) {
              w[f] = w0[f];
              for (int d = 0; d < 3; d++) w[f] += sgn[d] * or_slope(wm[d][f], w0[f], wp[d][f], theta);
            }
            or_prim2cons_one(w, u);
            n_fallback++;
          }
          for (int f = 0; f < NF; f++)
            fine_padded[p * per + (((int64_t)f * N + z) * N + y) * N + x] = u[f];
        }
  }
  if (counts) { counts[0] = n_interp; counts[1] = n_fallback; }
  return bad ? -1 : 0;
}

/* Restriction: each parent cell becomes the average of its eight children (the volume-weighted
 * average of Sec. 3.4, exact conservation).  child[p][o] (o = octant bits x | y << 1 | z << 2)
 * lists the children of coarse patch parent_of[p]; coarse[parent_of[p]] is overwritten. */
void or_restrict(int64_t n, const int32_t *parent_of, const int32_t *child, const double *fine,
                 double *coarse)
{
  for (int64_t p = 0; p < n; p++) {
    double *cp = coarse + (int64_t)parent_of[p] * NF * 512;
    for (int k = 0; k < PS; k++)
      for (int j = 0; j < PS; j++)
        for (int i = 0; i < PS; i++) {
          int o = (i >= 4) | ((j >= 4) << 1) | ((k >= 4) << 2);
          const double *fp = fine + (int64_t)child[p * 8 + o] * NF * 512;
          int fi = 2 * (i & 3), fj = 2 * (j & 3), fk = 2 * (k & 3);
          for (int f = 0; f < NF; f++) {
            double s = 0.0;
            for (int dz = 0; dz < 2; dz++)
              for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++)
                  s += fp[f * 512 + ((fk + dz) * PS + (fj + dy)) * PS + (fi + dx)];
            cp[f * 512 + (k * PS + j) * PS + i] = 0.125 * s;
          }
        }
  }
}

/* Coarse-fine flux correction (Sec. 3.4 item 4).  Face record q: coarse patch faces[q].coarse,
 * side s = 2 d + u (axis d, u = 1 upper), and the four fine patches across that face, fine[t]
 * for the quadrant t = (a >= 4) + 2 (b >= 4) of the face cell (a, b) (transverse coordinates in
 * increasing axis order).  Fluxes are per face cell, [patch][6][5][64], time-integrated by the
 * caller: coarse_flux = dt_c F_c, fine_flux = sum over the fine steps of dt_f F_f.  The coarse
 * cell at the face gets dU = (u ? -1 : +1) (<fine> - coarse) / dh_c, <fine> the mean of the four
 * fine face cells covering it; a cell whose corrected state fails Eq. 30 keeps its state.  The
 * records are applied side by side (s = 0 .. 5): a corner cell on faces of several sides gets
 * each correction in that order. */
int64_t or_flux_correct(int64_t n_face, const int32_t *faces /* [n][6]: coarse, side, fine[4] */,
                        double *coarse, const double *coarse_flux, const double *fine_flux,
                        double dh_c)
{
  int64_t skipped = 0;
  for (int side = 0; side < 6; side++)
  for (int64_t q = 0; q < n_face; q++) {
    const int32_t *r = faces + q * 6;
    if (r[1] != side) continue;
    int64_t P = r[0];
    int s = r[1], d = s >> 1, up = s & 1;
    int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
    for (int b = 0; b < PS; b++)
      for (int a = 0; a < PS; a++) {
        int child = r[2 + (a >= 4) + 2 * (b >= 4)];
        int ci[3];
        ci[d] = up ? PS - 1 : 0;
        ci[t0] = a;
        ci[t1] = b;
        int64_t cell = (int64_t)(ci[2] * PS + ci[1]) * PS + ci[0];
        double u[5];
        for (int f = 0; f < NF; f++) {
          double fc = coarse_flux[((P * 6 + s) * NF + f) * 64 + b * 8 + a];
          double ff = 0.0;
          for (int db = 0; db < 2; db++)
            for (int da = 0; da < 2; da++) {
              int fa = 2 * (a & 3) + da, fb = 2 * (b & 3) + db;
              ff += fine_flux[(((int64_t)child * 6 + (s ^ 1)) * NF + f) * 64 + fb * 8 + fa];
            }
          ff *= 0.25;
          u[f] = coarse[(P * NF + f) * 512 + cell] + (up ? -1.0 : 1.0) * (ff - fc) / dh_c;
        }
        if (!or_is_physical(u)) { skipped++; continue; }
        for (int f = 0; f < NF; f++) coarse[(P * NF + f) * 512 + cell] = u[f];
      }
  }
  return skipped;
}

/* Copy the interior of padded patches into a compact [P][5][8^3] array. */
void or_extract_interior(int64_t n_patch, int ghost, const double *padded, double *interior)
{
  int N = PS + 2 * ghost;
  int64_t per = (int64_t)NF * N * N * N;
  for (int64_t p = 0; p < n_patch; p++)
    for (int f = 0; f < NF; f++)
      for (int k = 0; k < PS; k++)
        for (int j = 0; j < PS; j++)
          for (int i = 0; i < PS; i++)
            interior[(p * NF + f) * 512 + (k * PS + j) * PS + i] =
                padded[p * per + (((int64_t)f * N + k + ghost) * N + j + ghost) * N + i + ghost];
}

int or_num_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
