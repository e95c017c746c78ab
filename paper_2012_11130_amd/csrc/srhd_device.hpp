// srhd_device.hpp -- device math of the SRHD step for gfx950 (arXiv:2012.11130).
//
// Everything here is __device__ code shared by the conversion and step kernels:
//   * error-free transformations and a K = 3 compensated sum for the left-hand side
//     L = x^2 + 2x - m^2 of Eq. 15 (its cancellation is the (1 + Mach^2) eps of Eq. 20);
//   * the TM EoS: Eq. 22 (ht of Theta), Eq. 16 (Theta of ht), Eq. 14 (sound speed);
//   * the Newton iteration for f(ht) = L (Eqs. 15, A1, A2) and the analytic guess (Eqs. A3-A7,
//     with A4 taken as the positive root of A3);
//   * prim -> cons (Eqs. 8, 5a, 5b, 22, 15, 23) and the recovery after the root (Eqs. 17, 8,
//     5a, 16, 18);
//   * fluxes (Eqs. 4a, 4b, 7), signal speeds and the HLLE / HLLC Riemann solvers adapted to
//     the TM sound speed and to the reduced energy (Sec. 3.2);
//   * the original scheme's total-energy variables, flux and naive L (Sec. 4, Eqs. 5c, 21);
//   * the polytropic EoS of Sec. 2.2 as an alternative EoS type (EosPoly).
// Templates take the bulk arithmetic type T (double or float) and the inversion type.
#pragma once
#include <float.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace srhd {

// ------------------------------------------------------------------------------ arithmetic
// Division and square root: IEEE in double; hardware reciprocal / square root (about 1 ulp)
// in float, where the bulk of the mixed-precision path tolerates FP32 rounding anyway.
__device__ __forceinline__ double dv(double a, double b) { return a / b; }
__device__ __forceinline__ float dv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// Reciprocal to about 1 ulp where no correctly rounded quotient is needed: the hardware estimate
// refined by two Newton-Raphson steps (6 instructions in FP64 against 11 for a division).  For
// normal, finite arguments of moderate exponent only (no scaling of extreme exponents).  The
// inversions use it with FAST: in every FP64 step kernel (both layouts alike, so that they give
// the same bits) and in the FP32-bulk gather-layout and VL kernels, where it measures faster (in
// the FP32-bulk padded kernels the compiler's schedule around it costs registers and occupancy).
// The FP64 bulk uses it through dvx below.
__device__ __forceinline__ double rcp_nr(double b)
{
  double r = __builtin_amdgcn_rcp(b);
  r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
}
__device__ __forceinline__ float rcp_nr(float b) { return __builtin_amdgcn_rcpf(b); }
// Square root to about 1 ulp on the same terms: the hardware reciprocal square root refined by
// one Newton-Raphson step on it and one on the root (Markstein's coupled iteration).
__device__ __forceinline__ double sqrt_nr(double x)
{
  double y = __builtin_amdgcn_rsq(x);           // ~ 1 / sqrt(x)
  double g = x * y, hh = 0.5 * y;               // g ~ sqrt(x), hh ~ 1 / (2 sqrt(x))
  double r = __builtin_fma(-g, hh, 0.5);
  g = __builtin_fma(g, r, g);
  hh = __builtin_fma(hh, r, hh);
  const double d = __builtin_fma(-g, g, x);
  return __builtin_fma(d, hh, g);
}
__device__ __forceinline__ float sqrt_nr(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sq(double a) { return __builtin_sqrt(a); }
__device__ __forceinline__ float sq(float a) { return __builtin_amdgcn_sqrtf(a); }
// Division in the step's bulk: with FX (the FP64 step kernels) a times the refined reciprocal
// (about 1 ulp) in FP64; otherwise dv.  In limited_slope with FX a zero dl + dr yields NaN for
// the harmonic mean, which the sign test then discards, as it discards the infinity of the IEEE
// division.
template <bool FX, class T> __device__ __forceinline__ T dvx(T a, T b)
{
  if constexpr (FX && sizeof(T) == 8) return a * rcp_nr(b);
  else return dv(a, b);
}
// Square root likewise (FX: the refined square root, for positive x only).
template <bool FX, class T> __device__ __forceinline__ T sqx(T x)
{
  if constexpr (FX && sizeof(T) == 8) return sqrt_nr(x);
  else return sq(x);
}
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <class T> __device__ __forceinline__ T absT(T a) { return a < T(0) ? -a : a; }
template <class T> __device__ __forceinline__ T minT(T a, T b) { return b < a ? b : a; }
template <class T> __device__ __forceinline__ T maxT(T a, T b) { return b > a ? b : a; }
template <class T> __device__ __forceinline__ bool finiteT(T a) { return a - a == T(0); }

// The error-free transformations below must see every product rounded exactly once, so FMA
// contraction (on by default in HIP) is switched off inside them: fusing a rounded product
// into the following sum would silently break the exactness.

// Knuth's branch-free two-sum: s + e == a + b exactly.
template <class T>
__device__ __forceinline__ void two_sum(T a, T b, T &s, T &e)
{
#pragma clang fp contract(off)
  s = a + b;
  T bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Ogita-Rump-Oishi SumK with K = 3: two error-free cascades, then the plain sum.  The result
// is as accurate as if summed in triple precision and rounded once.
template <class T, int N>
__device__ __forceinline__ T sum_k3(T (&t)[N])
{
#pragma clang fp contract(off)
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int i = 1; i < N; ++i) {
      T s, e;
      two_sum(t[i], t[i - 1], s, e);
      t[i] = s;
      t[i - 1] = e;
    }
  }
  T r = t[0];
#pragma unroll
  for (int i = 1; i < N - 1; ++i) r += t[i];
  return r + t[N - 1];
}

// L = (Et^2 + 2 Et D - |M|^2) / D^2 with the numerator summed from error-free products
// (a*b = p + fma(a, b, -p)).
template <class T>
__device__ __forceinline__ T lhs_L(T D, T Mx, T My, T Mz, T Et)
{
#pragma clang fp contract(off)
  T t[10];
  t[0] = Et * Et;       t[1] = fmaT(Et, Et, -t[0]);
  T e2 = T(2) * Et;
  t[2] = e2 * D;        t[3] = fmaT(e2, D, -t[2]);
  t[4] = -(Mx * Mx);    t[5] = -fmaT(Mx, Mx, t[4]);
  t[6] = -(My * My);    t[7] = -fmaT(My, My, t[6]);
  t[8] = -(Mz * Mz);    t[9] = -fmaT(Mz, Mz, t[8]);
  T N = sum_k3(t);
  if constexpr (sizeof(T) == 8) return N / (D * D);      // one division (D^2 stays in range)
  else return dv(dv(N, D), D);
}

// The same in double from FP32 conserved variables: products of floats are exact in double.
__device__ __forceinline__ double lhs_L_from_f32(float D, float Mx, float My, float Mz, float Et)
{
#pragma clang fp contract(off)
  double d = D, e = Et, x = Mx, y = My, z = Mz;
  double t[5];
  t[0] = e * e;
  t[1] = 2.0 * e * d;
  t[2] = -(x * x);
  t[3] = -(y * y);
  t[4] = -(z * z);
  double N = sum_k3(t);
  return N / (d * d);
}

// The same for a wavefront of face states whose results are consumed in FP32: the five exact
// products summed plainly, with relative error at most 4 u cond (u = 2^-53, cond = sum |t_i| /
// |sum t_i|), where every lane has cond <= 2^10 (so below 5e-13: under the FP32 resolution of
// what the inversion returns); the compensated sum otherwise.  A gas at rest has cond = 1; a
// cold, fast gas has cond ~ U^2 / Theta and takes the compensated sum.  All lanes must call it.
template <bool FAST = false>
__device__ __forceinline__ double lhs_L_from_f32_adaptive(float D, float Mx, float My, float Mz, float Et)
{
#pragma clang fp contract(off)
  double d = D, e = Et, x = Mx, y = My, z = Mz;
  double t[5];
  t[0] = e * e;
  t[1] = 2.0 * e * d;
  t[2] = -(x * x);
  t[3] = -(y * y);
  t[4] = -(z * z);
  const double pos = t[0] + t[1], neg = (t[2] + t[3]) + t[4];
  double N = pos + neg;
  const bool cheap = __builtin_fabs(pos) + __builtin_fabs(neg) <= 1024.0 * __builtin_fabs(N);
  if (__any(!cheap)) {
    const double Nk = sum_k3(t);
    N = cheap ? N : Nk;
  }
  return FAST ? N * rcp_nr(d * d) : N / (d * d);
}

// The same for FP64 conserved variables whose inversion feeds one step of the FP64 bulk: the
// plain sum of the five rounded products (relative error at most 5 u cond) where every lane of
// the wavefront has cond <= 2^10, so below 6e-13 -- three orders under the step's 1e-10 parity --
// and the exact lhs_L otherwise.  The choice is made per lane (the wavefront only decides whether
// the exact sum is formed at all), so a state's L does not depend on its wavefront neighbours.
template <bool FAST = false>
__device__ __forceinline__ double lhs_L_adaptive(double D, double Mx, double My, double Mz, double Et)
{
  const double pos = Et * Et + 2.0 * Et * D;
  const double neg = -(Mx * Mx + My * My + Mz * Mz);
  const double N = pos + neg;
  const bool cheap = __builtin_fabs(pos) + __builtin_fabs(neg) <= 1024.0 * __builtin_fabs(N);
  double l = FAST ? N * rcp_nr(D * D) : N / (D * D);
  if (__any(!cheap)) {
    const double le = lhs_L(D, Mx, My, Mz, Et);
    l = cheap ? l : le;
  }
  return l;
}

// ------------------------------------------------------------------------------ EoS
// Eq. 22: reduced enthalpy from Theta, free of the subtraction h - 1.
template <bool FX = false, class T>
__device__ __forceinline__ T htilde_of_theta(T th)
{
  T a = T(2.25) * th * th;
  return T(2.5) * th + dvx<FX>(a, T(1) + sqx<FX>(a + T(1)));
}

// Eq. 16: Theta from the reduced enthalpy, with 9 ht^2 + 18 ht + 25 = 9 h^2 + 16.
template <class T>
__device__ __forceinline__ T theta_of_htilde(T ht)
{
  T h = ht + T(1);
  return dv(T(2) * ht * (ht + T(2)), T(5) * h + sq(T(9) * h * h + T(16)));
}

// Eq. 14: squared sound speed.
template <bool FX = false, class T>
__device__ __forceinline__ T sound_speed2(T th)
{
  T h = T(2.5) * th + sqx<FX>(T(2.25) * th * th + T(1));
  return dvx<FX>(th * (T(5) * h - T(8) * th), T(3) * h * (h - th));
}

// The polytropic EoS of Sec. 2.2, h = 1 + Theta / k with k = (Gamma - 1) / Gamma, as an
// alternative to the TM EoS above (EosTm, the default of every function taking an EoS).
struct EosTm {};
struct EosPoly {
  double k;      // (Gamma - 1) / Gamma
};

template <bool FX = false, class T> __device__ __forceinline__ T htilde_of_theta(T th, EosTm) { return htilde_of_theta<FX>(th); }
template <bool FX = false, class T> __device__ __forceinline__ T htilde_of_theta(T th, const EosPoly &e) { return dvx<FX>(th, T(e.k)); }
template <class T> __device__ __forceinline__ T theta_of_htilde(T ht, EosTm) { return theta_of_htilde(ht); }
template <class T> __device__ __forceinline__ T theta_of_htilde(T ht, const EosPoly &e) { return T(e.k) * ht; }
template <bool FX = false, class T> __device__ __forceinline__ T sound_speed2(T th, EosTm) { return sound_speed2<FX>(th); }
// c_s^2 = Gamma Theta / h = k Theta / ((1 - k)(k + Theta))
template <bool FX = false, class T> __device__ __forceinline__ T sound_speed2(T th, const EosPoly &e)
{
  const T k = T(e.k);
  return dvx<FX>(k * th, (T(1) - k) * (k + th));
}

// ------------------------------------------------------------------------------ inversion
// App. A: analytic guess -- hot (Eq. A6) above the threshold of Eq. A7, else the positive root
// of the quadratic Eq. A3 (the corrected Eq. A4).
template <class T>
__device__ __forceinline__ T guess_analytic(T L, T m2)
{
  T a = T(1) + m2;
  bool hot;
  if constexpr (sizeof(T) == 8) {
    // L > (1800 a / c)^2 with c = 437 m^2 + 117, without the division (no overflow in double)
    T c = T(437) * m2 + T(117), u = T(1800) * a;
    hot = L * c * c > u * u;
  } else {
    // sqrt(L) c > 1800 a: the hot branch's square root, and no division (nothing overflows)
    const T sl = sq(L);
    hot = sl * (T(437) * m2 + T(117)) > T(1800) * a;
    if (hot) return T(4.0 / 3.0) * sl;
  }
  // a starting point only: in FP64 the refined reciprocal and square root (about 1 ulp) will do
  if (hot) return T(4.0 / 3.0) * sqrt_nr(L);
  T b = T(43) * m2 + T(63);
  return T(125) * a * L * rcp_nr(T(75) * a + sqrt_nr(T(125) * a * b * L + T(5625) * a * a));
}

// Newton iteration for f(ht) = L from x.  With h = ht + 1, s = sqrt(9 h^2 + 16),
// den = 5 h + s, q = h^2 + m^2 and r = h^2 / q:
//   Theta  = 2 ht (ht + 2) / den                            (Eq. 16)
//   Theta' = (4 h - Theta (5 + 9 h / s)) / den              (Eq. A2)
//   f      = ht (ht + 2) - 2 Theta h + Theta^2 r            (Eq. 15)
//   f'     = 2 h - 2 Theta - 2 h Theta' + 2 Theta Theta' r + 2 Theta^2 r (m^2/q) / h   (Eq. A1)
// f is increasing and convex, so from any positive start the iterates stay positive and
// converge quadratically; the loop stops once the applied step is below tol * ht, which
// leaves an error of order tol^2.  Returns false on a non-finite iterate or after max_iter.
template <class T, bool FAST = false>
__device__ __forceinline__ bool newton_htilde(T L, T m2, T x, T tol, int max_iter, T &ht,
                                              int &iters)
{
  for (int it = 1; it <= max_iter; ++it) {
    T h = x + T(1);
    T h2 = h * h;
    T s2 = T(9) * h2 + T(16);
    T s = FAST ? sqrt_nr(s2) : sq(s2);
    T iden, iq, is;
    if constexpr (sizeof(T) == 8) {
      // one division for 1/den, 1/q and 1/s: the product den q s^2 stays far inside the double
      // range for any iterate that can still converge (an overflow ends in a non-finite step)
      T den = T(5) * h + s, q = h2 + m2;
      T inv = FAST ? rcp_nr(den * q * s2) : dv(T(1), den * q * s2);
      iden = q * s2 * inv;
      iq = den * s2 * inv;
      is = s * den * q * inv;
    } else {
      iden = dv(T(1), T(5) * h + s);
      iq = dv(T(1), h2 + m2);
      is = dv(T(1), s);
    }
    T th = T(2) * x * (x + T(2)) * iden;
    T dth = (T(4) * h - th * (T(5) + T(9) * h * is)) * iden;
    T r = h2 * iq;
    T f = x * (x + T(2)) - T(2) * th * h + th * th * r;
    // the last term of Eq. A1, Theta^2 r (m^2/q) / h: in double as Theta^2 h m^2 / q^2 (no
    // division); in float as written, whose products stay inside the FP32 range
    T last;
    if constexpr (sizeof(T) == 8) last = th * th * h * m2 * iq * iq;
    else last = dv(th * th * r * (m2 * iq), h);
    T fp = T(2) * (h - th - h * dth + th * dth * r + last);
    T dx = FAST ? (f - L) * rcp_nr(fp) : dv(f - L, fp);
    x -= dx;
    if (!(x > T(0)) || !finiteT(x)) { iters = it; ht = x; return false; }
    if (absT(dx) <= tol * x) { iters = it; ht = x; return true; }
  }
  iters = max_iter;
  ht = x;
  return false;
}

enum { ST_OK = 0, ST_UNPHYSICAL = 1, ST_FALLBACK = 2, ST_NOCONV = 3 };

template <class T>
struct InvOut {
  T rho, ux, uy, uz, p;        // primitive variables
  T ht;                        // reduced enthalpy (the root)
  T gam, igam, cs2;            // gamma, 1 / gamma and c_s^2 (Eq. 14) of the result: FP32 TM recovery only
  int status;                  // SRHD_ST_*
  int iters;                   // Newton iterations (both guesses)
};

// Recovery after the root: Eqs. 17, 8, 5a, 16, 18.  FAST (FP64): the refined reciprocal and
// square root (about 1 ulp) in place of IEEE division and square root.
template <class T, bool FAST = false>
__device__ __forceinline__ void recover(T D, T Mx, T My, T Mz, T ht, InvOut<T> &o)
{
  T iDh = FAST ? rcp_nr(D * (T(1) + ht)) : dv(T(1), D * (T(1) + ht));
  o.ux = Mx * iDh;
  o.uy = My * iDh;
  o.uz = Mz * iDh;
  const T g2 = T(1) + o.ux * o.ux + o.uy * o.uy + o.uz * o.uz;
  T gam = FAST ? sqrt_nr(g2) : sq(g2);
  if constexpr (sizeof(T) == 8) {
    // rho = D / gamma and Theta of Eq. 16 share one division
    T h = ht + T(1);
    const T s2 = T(9) * h * h + T(16);
    T den = T(5) * h + (FAST ? sqrt_nr(s2) : sq(s2));
    T inv = FAST ? rcp_nr(gam * den) : dv(T(1), gam * den);
    o.rho = D * den * inv;
    o.p = o.rho * (T(2) * ht * (ht + T(2)) * gam * inv);
  } else {
    // FP32: also keep gamma, 1 / gamma and c_s^2 (Eq. 14 from Theta and h = 1 + ht), which the
    // Riemann solver of a face state needs
    const T igam = dv(T(1), gam);
    const T th = theta_of_htilde(ht);
    const T h = T(1) + ht;
    o.rho = D * igam;
    o.p = o.rho * th;
    o.gam = gam;
    o.igam = igam;
    o.cs2 = dv(th * (T(5) * h - T(8) * th), T(3) * h * (h - th));
  }
  o.ht = ht;
}

template <class T>
__device__ __forceinline__ void set_unphysical(InvOut<T> &o)
{
  const T nan = T(__builtin_nan(""));
  o.rho = o.ux = o.uy = o.uz = o.p = o.ht = nan;
  o.gam = o.igam = o.cs2 = nan;
  o.status = ST_UNPHYSICAL;
  o.iters = 0;
}

// The physical check shared by the inversion and the step's output test (Eq. 30, strict).
template <class T>
__device__ __forceinline__ bool admissible(T D, T Mx, T My, T Mz, T Et, T eps, T &L)
{
  if (!(finiteT(D) && finiteT(Mx) && finiteT(My) && finiteT(Mz) && finiteT(Et)) ||
      !(D > T(0)) || !(Et > T(0))) {
    L = T(0);
    return false;
  }
  L = lhs_L(D, Mx, My, Mz, Et);
  return L > eps;
}

// The same check for a wavefront of FP64 states whose inversion results are consumed in FP32:
// L from the plain sum of the five rounded products (relative error at most 5 u cond, under
// 6e-13) where every lane has cond = sum |t_i| / |sum t_i| <= 2^10, else the exact lhs_L.  Near
// the threshold eps the condition number is above 10^15, so the decision is the exact one's.
// All lanes must call it.
template <bool FAST = false>
__device__ __forceinline__ bool admissible_adaptive(double D, double Mx, double My, double Mz, double Et,
                                                    double eps, double &L)
{
  const bool basic = finiteT(D) && finiteT(Mx) && finiteT(My) && finiteT(Mz) && finiteT(Et) &&
                     D > 0.0 && Et > 0.0;
  const double pos = Et * Et + 2.0 * Et * D;
  const double neg = -(Mx * Mx + My * My + Mz * Mz);
  double N = pos + neg;
  const bool cheap = basic && __builtin_fabs(pos) + __builtin_fabs(neg) <= 1024.0 * __builtin_fabs(N);
  double l = FAST ? N * rcp_nr(D * D) : N / (D * D);
  if (__any(basic && !cheap)) {
    const double le = basic ? lhs_L(D, Mx, My, Mz, Et) : 0.0;
    l = cheap ? l : le;
  }
  L = basic ? l : 0.0;
  return basic && L > eps;
}

// The polytropic EoS: a starting point with the small-ht slope f ~ 2 (1 - k) ht and the
// large-ht growth f ~ (1 - k)^2 ht^2 (App. A's guess belongs to the TM EoS), the Newton
// iteration of Eqs. 15 and A1 with Theta = k ht and Theta' = k, and the recovery.
template <class T>
__device__ __forceinline__ T guess_poly(T L, T k)
{
  return dv(L, (T(1) - k) * (T(2) + sq(L)));
}

template <class T>
__device__ __forceinline__ bool newton_htilde_poly(T L, T m2, T x, T k, T tol, int max_iter, T &ht,
                                                   int &iters)
{
  for (int it = 1; it <= max_iter; ++it) {
    T h = x + T(1);
    T h2 = h * h;
    T iq = dv(T(1), h2 + m2);
    T th = k * x;
    T r = h2 * iq;
    T f = x * (x + T(2)) - T(2) * th * h + th * th * r;
    T fp = T(2) * (h - th - h * k + th * k * r + dv(th * th * r * (m2 * iq), h));
    T dx = dv(f - L, fp);
    x -= dx;
    if (!(x > T(0)) || !finiteT(x)) { iters = it; ht = x; return false; }
    if (absT(dx) <= tol * x) { iters = it; ht = x; return true; }
  }
  iters = max_iter;
  ht = x;
  return false;
}

template <class T>
__device__ __forceinline__ void recover_poly(T D, T Mx, T My, T Mz, T ht, T k, InvOut<T> &o)
{
  T iDh = dv(T(1), D * (T(1) + ht));
  o.ux = Mx * iDh;
  o.uy = My * iDh;
  o.uz = Mz * iDh;
  T gam = sq(T(1) + o.ux * o.ux + o.uy * o.uy + o.uz * o.uz);
  o.rho = dv(D, gam);
  o.p = o.rho * (k * ht);
  o.ht = ht;
}

// The analytic starting point of the EoS (App. A for TM), formed in G.
template <class T, class G, class E>
__device__ __forceinline__ T start_guess(T L, T m2, T k)
{
  if constexpr (std::is_same<E, EosPoly>::value) return guess_poly(L, k);
  else return T(guess_analytic<G>(G(L), G(m2)));
}

// Inversion from a known, admissible L.  With `have_guess` the supplied guess is tried first
// and the analytic guess is the fallback (status FALLBACK when the supplied guess is not a
// positive finite number or its Newton iteration fails and the analytic one converges);
// otherwise the analytic guess is used directly.  The analytic guess is formed in G (a starting
// point only: FP32 suffices where the result is consumed in FP32); one Newton loop serves both
// starts.  The recovery of the primitives from the root (Eqs. 17, 8, 5a, 16, 18: no cancellation,
// each a few correctly rounded or 1-ulp operations) runs in R, FP32 where the primitives are
// consumed in FP32; L and the Newton iteration keep T.
template <class T, class G = T, class R = T, bool FAST = false, class E = EosTm>
__device__ __forceinline__ void invert_with_L(T D, T Mx, T My, T Mz, T L, T guess, bool have_guess,
                                              T tol, int max_iter, InvOut<T> &o, const E &eos = E())
{
  constexpr bool poly = std::is_same<E, EosPoly>::value;
  // (the polytropic build keeps the division: the reciprocal's registers cost it occupancy)
  T iD = (FAST && !poly) ? rcp_nr(D) : dv(T(1), D);
  T mx = Mx * iD, my = My * iD, mz = Mz * iD;
  T m2 = mx * mx + my * my + mz * mz;
  T ht;
  T k = T(0);
  if constexpr (poly) k = T(eos.k);
  const bool supplied = have_guess && guess > T(0) && finiteT(guess);
  bool fell_back = have_guess && !supplied;
  T x0 = supplied ? guess : start_guess<T, G, E>(L, m2, k);
  bool ok = false;
  int its = 0;
#pragma unroll 1
  for (int a = 0; a < 2; ++a) {
    int it = 0;
    if constexpr (poly) ok = newton_htilde_poly(L, m2, x0, k, tol, max_iter, ht, it);
    else ok = newton_htilde<T, FAST>(L, m2, x0, tol, max_iter, ht, it);
    its += it;
    if (ok || fell_back || !have_guess) break;
    fell_back = true;                       // the supplied guess failed: restart from App. A
    x0 = start_guess<T, G, E>(L, m2, k);
  }
  o.status = ok ? (fell_back ? ST_FALLBACK : ST_OK) : ST_NOCONV;
  o.iters = its;
  if constexpr (std::is_same<R, T>::value) {
    if constexpr (poly) recover_poly(D, Mx, My, Mz, ht, k, o);
    else recover<T, FAST && !poly>(D, Mx, My, Mz, ht, o);
  } else {
    InvOut<R> r;
    if constexpr (poly) recover_poly((R)D, (R)Mx, (R)My, (R)Mz, (R)ht, (R)k, r);
    else recover((R)D, (R)Mx, (R)My, (R)Mz, (R)ht, r);
    o.rho = r.rho;
    o.ux = r.ux;
    o.uy = r.uy;
    o.uz = r.uz;
    o.p = r.p;
    o.ht = ht;
    o.gam = r.gam;
    o.igam = r.igam;
    o.cs2 = r.cs2;
  }
}

// ------------------------------------------------------------------------------ prim -> cons
template <class T>
struct Prim { T rho, u[3], p; };
template <class T>
struct Cons { T D, m[3], E; };   // E is the reduced energy Et

// Eqs. 8, 5a, 22, 5b, 15 (with Theta = p / rho known), 23.
template <bool FX = false, class T, class E = EosTm>
__device__ __forceinline__ Cons<T> prim2cons(const Prim<T> &w, const E &eos = E())
{
  T U2 = w.u[0] * w.u[0] + w.u[1] * w.u[1] + w.u[2] * w.u[2];
  T gam = sqx<FX>(T(1) + U2);
  T D = w.rho * gam;
  T th = dvx<FX>(w.p, w.rho);
  T ht = htilde_of_theta<FX>(th, eos);
  T h = T(1) + ht;
  T Dh = D * h;
  T h2 = h * h;
  T m2 = h2 * U2;
  T f = ht * (ht + T(2)) - T(2) * th * h + dvx<FX>(th * th * h2, h2 + m2);
  T a = m2 + f;
  Cons<T> u;
  u.D = D;
  u.m[0] = Dh * w.u[0];
  u.m[1] = Dh * w.u[1];
  u.m[2] = Dh * w.u[2];
  u.E = dvx<FX>(D * a, T(1) + sqx<FX>(T(1) + a));
  return u;
}

// Eq. 15's left-hand side L of a primitive state: f of Eq. 15 at the state's own reduced enthalpy
// (what prim -> cons forms on its way to Et), in the arithmetic of T.
template <class T, class E = EosTm>
__device__ __forceinline__ T lhs_L_of_prim(T rho, T ux, T uy, T uz, T p, const E &eos = E())
{
  const T U2 = ux * ux + uy * uy + uz * uz;
  const T th = dv(p, rho);
  const T ht = htilde_of_theta(th, eos);
  const T h = T(1) + ht;
  const T h2 = h * h;
  return ht * (ht + T(2)) - T(2) * th * h + dv(th * th * h2, h2 + h2 * U2);
}

// The original scheme's conserved variables (Sec. 4): D and M as above and, in the energy slot,
// the total energy E = D h gamma - p of Eq. 5c (h = 1 + ht, Eq. 10) instead of Et.
template <class T>
__device__ __forceinline__ Cons<T> prim2cons_total(const Prim<T> &w)
{
  T U2 = w.u[0] * w.u[0] + w.u[1] * w.u[1] + w.u[2] * w.u[2];
  T gam = sq(T(1) + U2);
  T D = w.rho * gam;
  T h = T(1) + htilde_of_theta(dv(w.p, w.rho));
  T Dh = D * h;
  Cons<T> u;
  u.D = D;
  u.m[0] = Dh * w.u[0];
  u.m[1] = Dh * w.u[1];
  u.m[2] = Dh * w.u[2];
  u.E = Dh * gam - w.p;
  return u;
}

template <bool TOT, bool FX = false, class T, class E = EosTm>
__device__ __forceinline__ Cons<T> prim2cons_s(const Prim<T> &w, const E &eos = E())
{
  if constexpr (TOT) return prim2cons_total(w);
  else return prim2cons<FX>(w, eos);
}

// The original scheme's physical check and left-hand side of Eq. 15: L = (E/D)^2 - (|M|/D)^2 - 1
// formed from the divided variables in the arithmetic of type I (Eq. 21), with correctly rounded
// divisions and no fused multiply-adds, so that its cancellation is that of the plain formula.
// Returns whether the state is finite with D > 0, E > 0 and L > DBL_EPSILON; L = 0 otherwise.
template <class I>
__device__ __forceinline__ bool admissible_total(I D, I Mx, I My, I Mz, I E, double &L)
{
#pragma clang fp contract(off)
  L = 0.0;
  if (!(finiteT(D) && finiteT(Mx) && finiteT(My) && finiteT(Mz) && finiteT(E)) ||
      !(D > I(0)) || !(E > I(0)))
    return false;
  const I e = E / D, mx = Mx / D, my = My / D, mz = Mz / D;
  const I l = e * e - (mx * mx + my * my + mz * mz) - I(1);
  const bool ok = (double)l > DBL_EPSILON;
  if (ok) L = (double)l;
  return ok;
}

// ------------------------------------------------------------------------------ fluxes
// The direction d is a template parameter so that every component index is a constant.

// What the Riemann solvers need of each side besides the primitives: gamma, 1 / gamma and c_s^2.
template <class T>
struct FaceAux { T gam, igam, cs2; };

template <bool FX = false, class T, class E = EosTm>
__device__ __forceinline__ FaceAux<T> face_aux(const Prim<T> &w, const E &eos = E())
{
  FaceAux<T> x;
  x.gam = sqx<FX>(T(1) + w.u[0] * w.u[0] + w.u[1] * w.u[1] + w.u[2] * w.u[2]);
  x.igam = dvx<FX>(T(1), x.gam);
  x.cs2 = sound_speed2<FX>(dvx<FX>(w.p, w.rho), eos);
  return x;
}

// Physical flux along d (Eqs. 4a, 4b, 7) with v_d = U_d / gamma.  TOT: the original scheme, whose
// energy variable E has the flux (E + p) v_d = M_d.
template <int d, bool TOT = false, class T>
__device__ __forceinline__ Cons<T> phys_flux(const Prim<T> &w, const Cons<T> &u, T igam)
{
  T v = w.u[d] * igam;
  Cons<T> F;
  F.D = u.D * v;
  F.m[0] = u.m[0] * v;
  F.m[1] = u.m[1] * v;
  F.m[2] = u.m[2] * v;
  F.m[d] += w.p;
  if constexpr (TOT) F.E = u.m[d];
  else F.E = (u.E + w.p) * v;
  return F;
}
template <int d, bool TOT = false, class T>
__device__ __forceinline__ Cons<T> phys_flux(const Prim<T> &w, const Cons<T> &u)
{
  return phys_flux<d, TOT>(w, u, dv(T(1), sq(T(1) + w.u[0] * w.u[0] + w.u[1] * w.u[1] + w.u[2] * w.u[2])));
}

// Signal speeds along d in four-velocity form:
// lambda_pm = [gamma U_d (1 - cs^2) +- cs sqrt(1 + U_perp^2 (1 - cs^2))] / (1 + U^2 (1 - cs^2)).
template <int d, bool FX = false, class T>
__device__ __forceinline__ void signal_speeds(const Prim<T> &w, const FaceAux<T> &x, T &lm, T &lp)
{
  constexpr int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
  const T cs2 = x.cs2, gam = x.gam;
  T Ud = w.u[d];
  T Up2 = w.u[a1] * w.u[a1] + w.u[a2] * w.u[a2];
  T U2 = Ud * Ud + Up2;
  T a = T(1) - cs2;
  T iden = dvx<FX>(T(1), T(1) + U2 * a);
  // cs sqrt(1 + Up^2 a) as one square root in FP32
  T s = sizeof(T) == 4 ? sq(cs2 * (T(1) + Up2 * a)) : sqx<FX>(cs2) * sqx<FX>(T(1) + Up2 * a);
  T c = gam * Ud * a;
  lm = (c - s) * iden;
  lp = (c + s) * iden;
}
template <int d, class T, class E = EosTm>
__device__ __forceinline__ void signal_speeds(const Prim<T> &w, T &lm, T &lp, const E &eos = E())
{
  signal_speeds<d>(w, face_aux(w, eos), lm, lp);
}

// HLLE: HLL flux with S_L^- = min(S_L, 0), S_R^+ = max(S_R, 0).  ul, ur are the conserved
// variables of wl, wr (the states the primitives were inverted from, where the caller has them).
// TOT: the original scheme's variables (total energy E).
// xl, xr: gamma, 1 / gamma and c_s^2 of the two sides.
template <int d, bool TOT = false, bool FX = false, class T>
__device__ __forceinline__ Cons<T> hlle(const Prim<T> &wl, const Prim<T> &wr, const Cons<T> &ul,
                                        const Cons<T> &ur, const FaceAux<T> &xl, const FaceAux<T> &xr)
{
  Cons<T> fl = phys_flux<d, TOT>(wl, ul, xl.igam), fr = phys_flux<d, TOT>(wr, ur, xr.igam);
  T lmL, lpL, lmR, lpR;
  signal_speeds<d, FX>(wl, xl, lmL, lpL);
  signal_speeds<d, FX>(wr, xr, lmR, lpR);
  T sl = minT(minT(lmL, lmR), T(0));
  T sr = maxT(maxT(lpL, lpR), T(0));
  T inv = dvx<FX>(T(1), sr - sl);
  T srl = sr * sl;
  Cons<T> F;
  F.D = (sr * fl.D - sl * fr.D + srl * (ur.D - ul.D)) * inv;
#pragma unroll
  for (int k = 0; k < 3; ++k) F.m[k] = (sr * fl.m[k] - sl * fr.m[k] + srl * (ur.m[k] - ul.m[k])) * inv;
  F.E = (sr * fl.E - sl * fr.E + srl * (ur.E - ul.E)) * inv;
  return F;
}
template <int d, bool TOT = false, class T, class E = EosTm>
__device__ __forceinline__ Cons<T> hlle(const Prim<T> &wl, const Prim<T> &wr, const Cons<T> &ul,
                                        const Cons<T> &ur, const E &eos = E())
{
  return hlle<d, TOT>(wl, wr, ul, ur, face_aux(wl, eos), face_aux(wr, eos));
}

template <class T>
__device__ __forceinline__ Cons<T> sel(bool c, const Cons<T> &a, const Cons<T> &b)
{
  Cons<T> r;
  r.D = c ? a.D : b.D;
  r.m[0] = c ? a.m[0] : b.m[0];
  r.m[1] = c ? a.m[1] : b.m[1];
  r.m[2] = c ? a.m[2] : b.m[2];
  r.E = c ? a.E : b.E;
  return r;
}

// HLLC (Mignone & Bodo 2005) with the total energy E = Et + D in the contact-speed quadratic
// F^E l^2 - (E + F^m) l + m = 0 (root 2 m / (B + sqrt(B^2 - 4 F^E m)), B = E + F^m), the star
// pressure p* = F^m - l* F^E, and the reduced-energy star state
// Et* = [Et (S - v) + p* l* - p v] / (S - l*), which carries no rest-mass cancellation.
// TOT: the original scheme, whose energy slot already holds E (and its flux M_d); its star state
// E* takes the same form.
template <int d, bool TOT = false, bool FX = false, class T>
__device__ __forceinline__ Cons<T> hllc(const Prim<T> &wl, const Prim<T> &wr, const Cons<T> &ul,
                                        const Cons<T> &ur, const FaceAux<T> &xl, const FaceAux<T> &xr)
{
  Cons<T> fl = phys_flux<d, TOT>(wl, ul, xl.igam), fr = phys_flux<d, TOT>(wr, ur, xr.igam);
  T lmL, lpL, lmR, lpR;
  signal_speeds<d, FX>(wl, xl, lmL, lpL);
  signal_speeds<d, FX>(wr, xr, lmR, lpR);
  T sl = minT(lmL, lmR);
  T sr = maxT(lpL, lpR);
  T inv = dvx<FX>(T(1), sr - sl);
  T srl = sl * sr;
  // HLL averages of the quantities the contact speed needs
  T Dh = (sr * ur.D - sl * ul.D + fl.D - fr.D) * inv;
  T Eh = (sr * ur.E - sl * ul.E + fl.E - fr.E) * inv + (TOT ? T(0) : Dh);
  T mh = (sr * ur.m[d] - sl * ul.m[d] + fl.m[d] - fr.m[d]) * inv;
  T FDh = (srl * (ur.D - ul.D) + sr * fl.D - sl * fr.D) * inv;
  T FEh = (srl * (ur.E - ul.E) + sr * fl.E - sl * fr.E) * inv + (TOT ? T(0) : FDh);
  T Fmh = (srl * (ur.m[d] - ul.m[d]) + sr * fl.m[d] - sl * fr.m[d]) * inv;
  T B = Eh + Fmh;
  T disc = maxT(B * B - T(4) * FEh * mh, T(0));
  // (IEEE square root here: the refined one would push the 768-thread FP64 step into spills)
  T ls = dvx<FX>(T(2) * mh, B + sq(disc));
  T ps = Fmh - ls * FEh;
  bool left = ls >= T(0);
  Cons<T> u = sel(left, ul, ur);
  Cons<T> f = sel(left, fl, fr);
  T S = left ? sl : sr;
  T wp = left ? wl.p : wr.p;
  T v = (left ? wl.u[d] : wr.u[d]) * (left ? xl.igam : xr.igam);
  T a = S - v;
  T iS = dvx<FX>(T(1), S - ls);
  Cons<T> us;
  us.D = u.D * a * iS;
#pragma unroll
  for (int k = 0; k < 3; ++k) us.m[k] = u.m[k] * a * iS;
  us.m[d] = (u.m[d] * a + ps - wp) * iS;
  us.E = (u.E * a + ps * ls - wp * v) * iS;
  Cons<T> F;
  F.D = f.D + S * (us.D - u.D);
#pragma unroll
  for (int k = 0; k < 3; ++k) F.m[k] = f.m[k] + S * (us.m[k] - u.m[k]);
  F.E = f.E + S * (us.E - u.E);
  // supersonic cases: the upwind physical flux
  F = sel(sl >= T(0), fl, F);
  F = sel(sr <= T(0), fr, F);
  return F;
}
template <int d, bool TOT = false, class T, class E = EosTm>
__device__ __forceinline__ Cons<T> hllc(const Prim<T> &wl, const Prim<T> &wr, const Cons<T> &ul,
                                        const Cons<T> &ur, const E &eos = E())
{
  return hllc<d, TOT>(wl, wr, ul, ur, face_aux(wl, eos), face_aux(wr, eos));
}

// ------------------------------------------------------------------------------ CFL
// Eqs. 26-27 for one cell (the sum over |Ux| + |Uy| + |Uz|): U_max = gamma_s sum |U_i| +
// 3 gamma U_s, S_max = U_max / sqrt(1 + U_max^2).  Always in double.
template <class E = EosTm>
__device__ __forceinline__ double signal_smax(double rho, double ux, double uy, double uz, double p,
                                              const E &eos = E())
{
  double cs2 = sound_speed2(p / rho, eos);
  double gs = 1.0 / sqrt(1.0 - cs2);                  // gamma_s
  double Us = sqrt(cs2) * gs;                         // U_s = c_s / sqrt(1 - c_s^2)
  double gam = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
  double Umax = gs * (fabs(ux) + fabs(uy) + fabs(uz)) + 3.0 * gam * Us;
  return Umax / sqrt(1.0 + Umax * Umax);
}

// The same in the arithmetic of T, for primitives stored in FP32: the FP32-bulk gather steps hand
// the next step its S_max from their FP32 output primitives (a time step needs no more than FP32
// accuracy; the maximum over cells stays exact and order independent).
template <class T, class E = EosTm>
__device__ __forceinline__ T signal_smax_t(T rho, T ux, T uy, T uz, T p, const E &eos = E())
{
  T cs2 = sound_speed2(dv(p, rho), eos);
  T gs = dv(T(1), sq(T(1) - cs2));
  T Us = sq(cs2) * gs;
  T gam = sq(T(1) + ux * ux + uy * uy + uz * uz);
  T Umax = gs * (absT(ux) + absT(uy) + absT(uz)) + T(3) * gam * Us;
  return dv(Umax, sq(T(1) + Umax * Umax));
}

// Eq. 20's conversion condition number kappa = 1 + M^2 of a primitive state against a threshold:
// M = U / U_s is the Mach number in four-velocities, U_s^2 = c_s^2 / (1 - c_s^2), so kappa > kmax
// is U^2 (1 - c_s^2) > (kmax - 1) c_s^2 (no division by a vanishing sound speed).  A threshold
// only: formed in the arithmetic of T (FX: with dvx / sqx); false for non-finite input.
template <class T, class E = EosTm, bool FX = false>
__device__ __forceinline__ bool kappa_above(T rho, T ux, T uy, T uz, T p, T kmax_m1, const E &eos = E())
{
  const T cs2 = sound_speed2<FX>(dvx<FX>(p, rho), eos);
  const T u2 = ux * ux + uy * uy + uz * uz;
  return u2 * (T(1) - cs2) > kmax_m1 * cs2;
}

// ------------------------------------------------------------------------------ PLM
// Hybrid van Leer / generalized minmod slope (zero at extrema).  One-sided differences below
// the smallest normal number count as zero: in FP32 the harmonic mean's division is a hardware
// reciprocal, which flushes a denormal denominator to zero, and 0 * inf would make the slope NaN
// (for any theta, 0 included).  In FP64 such differences give a zero slope either way.
//
// In FP32 the same slope is formed as |s| = m min(theta, 2 M / (m + M)) with m, M the smaller and
// larger of |dl|, |dr| (equal to min(2 |dl dr| / |dl + dr|, theta |dl|, theta |dr|) for
// differences of one sign): the ratio is bounded by 2, so nothing overflows, and it takes about
// half the instructions.
template <bool FX = false, class T>
__device__ __forceinline__ T limited_slope(T wl, T wc, T wr, T theta)
{
  T dl = wc - wl, dr = wr - wc;
  if constexpr (sizeof(T) == 4) {
    const float a = __builtin_fabsf(dl), b = __builtin_fabsf(dr);
    const float m = __builtin_fminf(a, b), M = __builtin_fmaxf(a, b);
    const bool mono = ((__float_as_int(dl) ^ __float_as_int(dr)) >= 0) && m >= FLT_MIN;
    const float q = (M + M) * __builtin_amdgcn_rcpf(m + M);
    const float s = __builtin_copysignf(m * __builtin_fminf(theta, q), dl);
    return mono ? s : 0.0f;
  } else {
    constexpr T tiny = T(DBL_MIN);
    bool mono = (dl >= tiny && dr >= tiny) || (dl <= -tiny && dr <= -tiny);
    T vl = absT(dvx<FX>(T(2) * dl * dr, dl + dr));
    T s = minT(vl, minT(theta * absT(dl), theta * absT(dr)));
    s = dl > T(0) ? s : -s;
    return mono ? s : T(0);
  }
}

// The Riemann fluxes from primitives alone.
template <int d, class T>
__device__ __forceinline__ Cons<T> hlle(const Prim<T> &wl, const Prim<T> &wr)
{
  return hlle<d>(wl, wr, prim2cons(wl), prim2cons(wr));
}
template <int d, class T>
__device__ __forceinline__ Cons<T> hllc(const Prim<T> &wl, const Prim<T> &wr)
{
  return hllc<d>(wl, wr, prim2cons(wl), prim2cons(wr));
}

}  // namespace srhd
