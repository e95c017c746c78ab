// srhd_kernels.hip -- batch conversions (Sec. 2.3), ghost fill (Sec. 3.1) and the CFL time
// step (Sec. 3.3) for gfx950.  All arrays are structure-of-arrays so that each field is read
// and written with unit stride across a wavefront.
#include <float.h>

#include "srhd_device.hpp"
#include "srhd_internal.hpp"

namespace srhd {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n, int per_thread = 1)
{
  int64_t b = (n + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
  if (b < 1) b = 1;
  if (b > 256 * 64) b = 256 * 64;       // grid-stride beyond 64 workgroups per CU
  return (int)b;
}

// Newton stopping thresholds (see newton_htilde): the step that falls below tol * ht leaves an
// error of order tol^2 relative, i.e. below the unit round-off of the arithmetic type.
template <class T> struct Tol;
template <> struct Tol<double> { static constexpr double v = 0x1p-27; static constexpr double eps = DBL_EPSILON; };
template <> struct Tol<float> { static constexpr float v = 0x1p-12f; static constexpr float eps = FLT_EPSILON; };

// ------------------------------------------------------------------------------ conversions
template <class T, class E>
__global__ void __launch_bounds__(kBlock) k_prim2cons(int64_t n, const T *__restrict__ prim,
                                                      T *__restrict__ cons, E eos)
{
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    Prim<T> w;
    w.rho = prim[i];
    w.u[0] = prim[n + i];
    w.u[1] = prim[2 * n + i];
    w.u[2] = prim[3 * n + i];
    w.p = prim[4 * n + i];
    Cons<T> u = prim2cons(w, eos);
    cons[i] = u.D;
    cons[n + i] = u.m[0];
    cons[2 * n + i] = u.m[1];
    cons[3 * n + i] = u.m[2];
    cons[4 * n + i] = u.E;
  }
}

// With MLP, the learned guess is tried first and the analytic guess is the fallback.  The loop
// runs the same number of times in every lane of a wavefront (the network's matrix instructions
// need all lanes); lanes past the end work on a dummy state and store nothing.  Each iteration
// loads the next state of the grid-stride loop before inverting the current one, so that the
// loads' latency overlaps the Newton iteration.
template <class T, bool MLP, class E>
__global__ void __launch_bounds__(kBlock) k_cons2prim(int64_t n, const T *__restrict__ cons,
                                                      T *__restrict__ prim,
                                                      int8_t *__restrict__ status,
                                                      uint8_t *__restrict__ iters, int max_iter,
                                                      MlpDev mlp, E eos)
{
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t base = (int64_t)blockIdx.x * blockDim.x;
  T nD = T(0), nMx = T(0), nMy = T(0), nMz = T(0), nEt = T(0);
  if (base < n) {
    const int64_t i = base + threadIdx.x, j = i < n ? i : 0;
    nD = cons[j]; nMx = cons[n + j]; nMy = cons[2 * n + j]; nMz = cons[3 * n + j]; nEt = cons[4 * n + j];
  }
  for (; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool in = i < n;
    T D = nD, Mx = nMx, My = nMy, Mz = nMz, Et = nEt;
    if (base + stride < n) {                         // uniform across the workgroup
      const int64_t i2 = base + stride + threadIdx.x, j2 = i2 < n ? i2 : 0;
      nD = cons[j2]; nMx = cons[n + j2]; nMy = cons[2 * n + j2]; nMz = cons[3 * n + j2];
      nEt = cons[4 * n + j2];
    }
    T L;
    const bool adm = admissible(D, Mx, My, Mz, Et, T(Tol<T>::eps), L);
    bool consulted = false;
    unsigned int evals = 0;
    T guess = T(-1);
    if (MLP) guess = (T)mlp_guess(mlp, D, Mx, My, Mz, Et, (in && adm) ? (double)L : 0.0, consulted, evals);
    if (!in) continue;
    InvOut<T> o;
    // FP64: the guess, the Newton iteration and the recovery through the refined reciprocal and
    // square root (about 1 ulp); L stays correctly rounded
    if (adm)
      invert_with_L<T, T, T, sizeof(T) == 8>(D, Mx, My, Mz, L, guess, consulted, T(Tol<T>::v), max_iter, o, eos);
    else
      set_unphysical(o);
    prim[i] = o.rho;
    prim[n + i] = o.ux;
    prim[2 * n + i] = o.uy;
    prim[3 * n + i] = o.uz;
    prim[4 * n + i] = o.p;
    if (status) status[i] = (int8_t)o.status;
    if (iters) iters[i] = (uint8_t)(o.iters > 255 ? 255 : o.iters);
  }
}

// ------------------------------------------------------------------------------ ghost fill
// One thread per padded cell: the cell's offset class selects a neighbour slot; directions
// whose face slot is -1 are clamped to the patch edge first (outflow), which also resolves
// edges and corners that touch the domain boundary.
template <class T>
__global__ void __launch_bounds__(kBlock) k_fill_ghosts(int64_t n_patch, int g, int64_t n_src,
                                                        const T *__restrict__ interior,
                                                        const int32_t *__restrict__ nb,
                                                        T *__restrict__ padded)
{
  const int N = 8 + 2 * g;
  const int N3 = N * N * N;
  const int64_t total = n_patch * N3;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    int64_t p = t / N3;
    int c = (int)(t - p * N3);
    int x = c % N, y = (c / N) % N, z = c / (N * N);
    int ci[3] = {x - g, y - g, z - g};
    const int32_t *np = nb + p * 27;
    const int fstride[3] = {1, 3, 9};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int o = ci[d] < 0 ? -1 : (ci[d] >= 8 ? 1 : 0);
      if (o != 0 && np[13 + o * fstride[d]] == -1) ci[d] = o < 0 ? 0 : 7;
    }
    int o0 = ci[0] < 0 ? -1 : (ci[0] >= 8 ? 1 : 0);
    int o1 = ci[1] < 0 ? -1 : (ci[1] >= 8 ? 1 : 0);
    int o2 = ci[2] < 0 ? -1 : (ci[2] >= 8 ? 1 : 0);
    int slot = (o2 + 1) * 9 + (o1 + 1) * 3 + (o0 + 1);
    int64_t src = np[slot];
    T *dst = padded + p * 5 * N3 + c;
    if (src == SRHD_NB_COARSE) continue;             // filled from the coarser level
    if (src < 0 || src >= n_src) {
#pragma unroll
      for (int f = 0; f < 5; ++f) dst[(int64_t)f * N3] = T(__builtin_nan(""));
      continue;
    }
    int s = ((ci[2] - 8 * o2) * 8 + (ci[1] - 8 * o1)) * 8 + (ci[0] - 8 * o0);
    const T *srcp = interior + src * 5 * 512 + s;
#pragma unroll
    for (int f = 0; f < 5; ++f) dst[(int64_t)f * N3] = srcp[f * 512];
  }
}

// ------------------------------------------------------------------------------ CFL
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Eqs. 26-27 per interior cell, maximum over the workgroup, then an integer atomic maximum on
// the bit pattern (order preserving for non-negative doubles) -- exact and order independent.
template <class T, class E>
__global__ void __launch_bounds__(kBlock) k_cfl_smax(int64_t n_patch,
                                                     const T *__restrict__ interior,
                                                     unsigned long long *__restrict__ smax_bits,
                                                     E eos)
{
  __shared__ double red[kBlock / 64];
  const int64_t total = n_patch * 512;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double vmax = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    int64_t p = t >> 9;
    int c = (int)(t & 511);
    const T *q = interior + p * 5 * 512 + c;
    T D = q[0], Mx = q[512], My = q[1024], Mz = q[1536], Et = q[2048];
    T L;
    // FP64: the L and inversion arithmetic of the FP64 step's own output inversion, so that the
    // step's S_max of its output and this kernel's agree bit for bit
    bool adm;
    if constexpr (sizeof(T) == 8) adm = admissible_adaptive<true>(D, Mx, My, Mz, Et, T(Tol<T>::eps), L);
    else adm = admissible(D, Mx, My, Mz, Et, T(Tol<T>::eps), L);
    if (!adm) continue;
    InvOut<T> o;
    invert_with_L<T, T, T, sizeof(T) == 8>(D, Mx, My, Mz, L, T(-1), false, T(Tol<T>::v), 30, o, eos);
    double S = signal_smax(o.rho, o.ux, o.uy, o.uz, o.p, eos);
    if (S > vmax) vmax = S;
  }
  vmax = wave_max(vmax);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = vmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, red[w]);
    atomicMax(smax_bits, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
  int i = threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void k_cfl_finish(const unsigned long long *__restrict__ smax_bits, LevelArgs lv,
                             double c_cfl, double *__restrict__ dt_lev)
{
  int l = threadIdx.x;
  if (l >= lv.n_level) return;
  double smax = __longlong_as_double((long long)smax_bits[0]);
  dt_lev[l] = c_cfl * lv.dh[l] / smax;
}

}  // namespace

// ------------------------------------------------------------------------------ launchers
template <class T, class E>
void prim2cons_e(int64_t n, const void *prim, void *cons, E eos, hipStream_t s)
{
  hipLaunchKernelGGL((k_prim2cons<T, E>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, (const T *)prim,
                     (T *)cons, eos);
}

hipError_t launch_prim2cons(int dtype, int64_t n, const void *prim, void *cons, double eos_k,
                            hipStream_t s)
{
  if (n == 0) return hipSuccess;
  if (eos_k > 0.0) {
    if (dtype == SRHD_F64) prim2cons_e<double>(n, prim, cons, EosPoly{eos_k}, s);
    else prim2cons_e<float>(n, prim, cons, EosPoly{eos_k}, s);
  } else {
    if (dtype == SRHD_F64) prim2cons_e<double>(n, prim, cons, EosTm{}, s);
    else prim2cons_e<float>(n, prim, cons, EosTm{}, s);
  }
  return hipGetLastError();
}

template <class T, bool MLP, class E>
void cons2prim_e(int64_t n, const void *cons, void *prim, int8_t *status, uint8_t *iters, int mi,
                 const MlpDev &m, E eos, hipStream_t s)
{
  hipLaunchKernelGGL((k_cons2prim<T, MLP, E>), dim3(grid_for(n)), dim3(kBlock), 0, s, n,
                     (const T *)cons, (T *)prim, status, iters, mi, m, eos);
}

// The learned guess exists for the TM EoS only (the caller rejects it with eos_k > 0).
hipError_t launch_cons2prim(int dtype, int64_t n, const void *cons, void *prim, int8_t *status,
                            uint8_t *iters, const GuessArgs &g, double eos_k, hipStream_t s)
{
  if (n == 0) return hipSuccess;
  int mi = g.max_iter > 0 ? g.max_iter : 30;
  MlpDev m = g.dev();
  const bool mlp = g.kind == SRHD_GUESS_MLP;
  const bool f64 = dtype == SRHD_F64;
  if (eos_k > 0.0) {
    if (mlp) return hipErrorInvalidValue;
    if (f64) cons2prim_e<double, false>(n, cons, prim, status, iters, mi, m, EosPoly{eos_k}, s);
    else cons2prim_e<float, false>(n, cons, prim, status, iters, mi, m, EosPoly{eos_k}, s);
  } else if (mlp) {
    if (f64) cons2prim_e<double, true>(n, cons, prim, status, iters, mi, m, EosTm{}, s);
    else cons2prim_e<float, true>(n, cons, prim, status, iters, mi, m, EosTm{}, s);
  } else {
    if (f64) cons2prim_e<double, false>(n, cons, prim, status, iters, mi, m, EosTm{}, s);
    else cons2prim_e<float, false>(n, cons, prim, status, iters, mi, m, EosTm{}, s);
  }
  return hipGetLastError();
}

hipError_t launch_fill_ghosts(int dtype, int64_t n_patch, int ghost, int64_t n_src, const void *interior,
                              const int32_t *neighbor, void *padded, hipStream_t s)
{
  if (n_patch == 0) return hipSuccess;
  int N = 8 + 2 * ghost;
  int64_t total = n_patch * N * N * N;
  if (dtype == SRHD_F64)
    hipLaunchKernelGGL(k_fill_ghosts<double>, dim3(grid_for(total, 4)), dim3(kBlock), 0, s,
                       n_patch, ghost, n_src, (const double *)interior, neighbor, (double *)padded);
  else
    hipLaunchKernelGGL(k_fill_ghosts<float>, dim3(grid_for(total, 4)), dim3(kBlock), 0, s,
                       n_patch, ghost, n_src, (const float *)interior, neighbor, (float *)padded);
  return hipGetLastError();
}

template <class T, class E>
void cfl_e(int64_t n_patch, const void *interior, unsigned long long *bits, E eos, hipStream_t s)
{
  const int64_t total = n_patch * 512;
  hipLaunchKernelGGL((k_cfl_smax<T, E>), dim3(grid_for(total, 2)), dim3(kBlock), 0, s, n_patch,
                     (const T *)interior, bits, eos);
}

hipError_t launch_cfl(int dtype, int64_t n_patch, const void *interior, const LevelArgs &lv,
                      double c_cfl, double *dt_lev, void *work, double eos_k, hipStream_t s)
{
  unsigned long long *bits = (unsigned long long *)work;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, bits, 1);
  if (n_patch > 0) {
    const bool f64 = dtype == SRHD_F64;
    if (eos_k > 0.0) {
      if (f64) cfl_e<double>(n_patch, interior, bits, EosPoly{eos_k}, s);
      else cfl_e<float>(n_patch, interior, bits, EosPoly{eos_k}, s);
    } else {
      if (f64) cfl_e<double>(n_patch, interior, bits, EosTm{}, s);
      else cfl_e<float>(n_patch, interior, bits, EosTm{}, s);
    }
  }
  hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(64), 0, s, (const unsigned long long *)bits,
                     lv, c_cfl, dt_lev);
  return hipGetLastError();
}

hipError_t launch_stats_reset(srhd_step_stats *st, hipStream_t s)
{
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)st,
                     (int)(sizeof(srhd_step_stats) / 8));
  return hipGetLastError();
}

}  // namespace srhd
