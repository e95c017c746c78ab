// srhd_amr.hip -- the AMR neighbours of the patch step on gfx950 (Sec. 3.4 items 3 and 4,
// refinement ratio 2): coarse-to-fine ghost-zone interpolation with the primitive-variable
// fallback, restriction of children to their parent, time integration of boundary fluxes and
// the coarse-fine flux correction.  All arrays are FP64 structure-of-arrays patches.
#include <float.h>

#include "srhd_device.hpp"
#include "srhd_internal.hpp"

namespace srhd {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void count_wave(unsigned long long *ctr, bool flag)
{
  // one atomic per wavefront: the number of lanes with the flag set
  const unsigned long long m = __ballot(flag);
  if (ctr && m && (threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// Coarse state at padded coordinates (ci, cj, ck) of one parent, time-interpolated.
__device__ __forceinline__ void coarse_state(const double *co, const double *cn, double alpha, int Nc,
                                             int gc, int ci, int cj, int ck, double u[5])
{
  const int64_t N3 = (int64_t)Nc * Nc * Nc;
  const int64_t off = ((int64_t)(ck + gc) * Nc + (cj + gc)) * Nc + (ci + gc);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const double v = co[f * N3 + off];
    u[f] = cn ? (1.0 - alpha) * v + alpha * cn[f * N3 + off] : v;
  }
}

__device__ __forceinline__ void to_prim(const double u[5], double w[5])
{
  double L;
  InvOut<double> o;
  if (admissible(u[0], u[1], u[2], u[3], u[4], DBL_EPSILON, L))
    invert_with_L<double>(u[0], u[1], u[2], u[3], L, -1.0, false, 0x1p-27, 30, o);
  else set_unphysical(o);
  w[0] = o.rho;
  w[1] = o.ux;
  w[2] = o.uy;
  w[3] = o.uz;
  w[4] = o.p;
}

// One thread per padded cell of the fine patches; only ghost cells whose source slot is
// SRHD_NB_COARSE are written.
__global__ void __launch_bounds__(kBlock) k_fill_ghosts_coarse(
    int64_t n_fine, int g, const int32_t *__restrict__ nb, const int32_t *__restrict__ parent,
    const int8_t *__restrict__ octant, int64_t n_coarse, int gc, const double *__restrict__ coarse_old,
    const double *__restrict__ coarse_new, double alpha, double theta, double *__restrict__ fine,
    unsigned long long *counts)
{
  const int N = 8 + 2 * g, N3 = N * N * N, Nc = 8 + 2 * gc;
  const int64_t perc = 5 * (int64_t)Nc * Nc * Nc;
  const int64_t total = n_fine * N3;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // the loop runs the same number of rounds in every lane of a wavefront (the wave-level
  // counters need whole wavefronts): lanes past the end do no work
  const int64_t rounds = (total + stride - 1) / stride;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t it = 0; it < rounds; ++it) {
    const int64_t t = t0 + it * stride;
    bool interp = false, fallback = false;
    if (t < total) {
      const int64_t p = t / N3;
      const int c = (int)(t - p * N3);
      int ci[3] = {c % N - g, (c / N) % N - g, c / (N * N) - g};
      const bool inside = ci[0] >= 0 && ci[0] < 8 && ci[1] >= 0 && ci[1] < 8 && ci[2] >= 0 && ci[2] < 8;
      const int32_t *np = nb + p * 27;
      int cc[3] = {ci[0], ci[1], ci[2]};
      const int fstride[3] = {1, 3, 9};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int o = cc[d] < 0 ? -1 : (cc[d] >= 8 ? 1 : 0);
        if (o != 0 && np[13 + o * fstride[d]] == -1) cc[d] = o < 0 ? 0 : 7;
      }
      const int o0 = cc[0] < 0 ? -1 : (cc[0] >= 8 ? 1 : 0);
      const int o1 = cc[1] < 0 ? -1 : (cc[1] >= 8 ? 1 : 0);
      const int o2 = cc[2] < 0 ? -1 : (cc[2] >= 8 ? 1 : 0);
      const int64_t par = parent[p];
      if (!inside && np[(o2 + 1) * 9 + (o1 + 1) * 3 + (o0 + 1)] == SRHD_NB_COARSE && par >= 0 &&
          par < n_coarse) {
        interp = true;
        const int oc = octant[p];
        int C[3];
        double sgn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int I = 8 * ((oc >> d) & 1) + ci[d];
          C[d] = I >= 0 ? I / 2 : -((1 - I) / 2);          // floor(I / 2)
          sgn[d] = (I - 2 * C[d]) ? 0.25 : -0.25;
        }
        const double *co = coarse_old + par * perc;
        const double *cn = coarse_new ? coarse_new + par * perc : nullptr;
        double u0[5], um[3][5], up[3][5];
        coarse_state(co, cn, alpha, Nc, gc, C[0], C[1], C[2], u0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          coarse_state(co, cn, alpha, Nc, gc, C[0] - (d == 0), C[1] - (d == 1), C[2] - (d == 2), um[d]);
          coarse_state(co, cn, alpha, Nc, gc, C[0] + (d == 0), C[1] + (d == 1), C[2] + (d == 2), up[d]);
        }
        double u[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          u[f] = u0[f];
#pragma unroll
          for (int d = 0; d < 3; ++d) u[f] += sgn[d] * limited_slope(um[d][f], u0[f], up[d][f], theta);
        }
        double L;
        if (!admissible(u[0], u[1], u[2], u[3], u[4], DBL_EPSILON, L)) {
          fallback = true;
          double w0[5], wm[3][5], wp[3][5];
          to_prim(u0, w0);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            to_prim(um[d], wm[d]);
            to_prim(up[d], wp[d]);
          }
          double w[5];
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            w[f] = w0[f];
#pragma unroll
            for (int d = 0; d < 3; ++d) w[f] += sgn[d] * limited_slope(wm[d][f], w0[f], wp[d][f], theta);
          }
          Prim<double> pw;
          pw.rho = w[0];
          pw.u[0] = w[1];
          pw.u[1] = w[2];
          pw.u[2] = w[3];
          pw.p = w[4];
          const Cons<double> cu = prim2cons(pw);
          u[0] = cu.D;
          u[1] = cu.m[0];
          u[2] = cu.m[1];
          u[3] = cu.m[2];
          u[4] = cu.E;
        }
        double *dst = fine + p * 5 * (int64_t)N3 + c;
#pragma unroll
        for (int f = 0; f < 5; ++f) dst[(int64_t)f * N3] = u[f];
      }
    }
    count_wave(counts, interp);
    count_wave(counts ? counts + 1 : nullptr, fallback);
  }
}

// One workgroup of 512 threads per parent: each thread averages the 8 children of one cell.
__global__ void __launch_bounds__(512) k_restrict(int64_t n, const int32_t *__restrict__ parent_of,
                                                  const int32_t *__restrict__ child, int64_t n_fine,
                                                  const double *__restrict__ fine, int64_t n_coarse,
                                                  double *__restrict__ coarse)
{
  const int64_t q = blockIdx.x;
  if (q >= n) return;
  const int c = threadIdx.x, i = c & 7, j = (c >> 3) & 7, k = c >> 6;
  const int o = (i >= 4) | ((j >= 4) << 1) | ((k >= 4) << 2);
  const int64_t ch = child[q * 8 + o], pa = parent_of[q];
  if (ch < 0 || ch >= n_fine || pa < 0 || pa >= n_coarse) return;     // invalid record: skipped
  const double *fp = fine + ch * 5 * 512;
  double *cp = coarse + pa * 5 * 512;
  const int fi = 2 * (i & 3), fj = 2 * (j & 3), fk = 2 * (k & 3);
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double s = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) s += fp[f * 512 + ((fk + dz) * 8 + (fj + dy)) * 8 + (fi + dx)];
    cp[f * 512 + c] = 0.125 * s;
  }
}

__global__ void __launch_bounds__(kBlock) k_flux_accumulate(int64_t n, double *__restrict__ acc,
                                                            const double *__restrict__ flux,
                                                            double beta, double weight)
{
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    acc[i] = (beta == 0.0 ? 0.0 : beta * acc[i]) + weight * flux[i];
}

// The face records of one side: one thread per (record, face cell).
__global__ void __launch_bounds__(kBlock) k_flux_correct(int64_t n_face, int side,
                                                         const int32_t *__restrict__ faces,
                                                         int64_t n_coarse, double *__restrict__ coarse,
                                                         const double *__restrict__ coarse_flux,
                                                         int64_t n_fine,
                                                         const double *__restrict__ fine_flux,
                                                         double dh_c, unsigned long long *skipped)
{
  const int64_t total = n_face * 64;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t rounds = (total + stride - 1) / stride;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t it = 0; it < rounds; ++it) {
    const int64_t t = t0 + it * stride;
    bool skip = false;
    if (t < total) {
      const int64_t q = t >> 6;
      const int32_t *r = faces + q * 6;
      const int cellf = (int)(t & 63), a = cellf & 7, b = cellf >> 3;
      const int64_t P = r[0];
      const int64_t child = r[2 + (a >= 4) + 2 * (b >= 4)];
      // records of other sides wait for their launch; invalid indices are skipped
      if (r[1] == side && P >= 0 && P < n_coarse && child >= 0 && child < n_fine) {
        const int s = r[1], d = s >> 1, up = s & 1;
        const int t0a = d == 0 ? 1 : 0, t1a = d == 2 ? 1 : 2;
        int ci[3];
        ci[d] = up ? 7 : 0;
        ci[t0a] = a;
        ci[t1a] = b;
        const int cell = (ci[2] * 8 + ci[1]) * 8 + ci[0];
        double u[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const double fc = coarse_flux[((P * 6 + s) * 5 + f) * 64 + b * 8 + a];
          double ff = 0.0;
#pragma unroll
          for (int db = 0; db < 2; ++db)
#pragma unroll
            for (int da = 0; da < 2; ++da)
              ff += fine_flux[((child * 6 + (s ^ 1)) * 5 + f) * 64 + (2 * (b & 3) + db) * 8 + 2 * (a & 3) + da];
          ff *= 0.25;
          u[f] = coarse[(P * 5 + f) * 512 + cell] + (up ? -1.0 : 1.0) * ((ff - fc) / dh_c);
        }
        double L;
        if (admissible(u[0], u[1], u[2], u[3], u[4], DBL_EPSILON, L)) {
#pragma unroll
          for (int f = 0; f < 5; ++f) coarse[(P * 5 + f) * 512 + cell] = u[f];
        } else {
          skip = true;
        }
      }
    }
    count_wave(skipped, skip);
  }
}

int grid_blocks(int64_t total)
{
  int64_t b = (total + kBlock - 1) / kBlock;
  return (int)(b < 1 ? 1 : (b > 256 * 64 ? 256 * 64 : b));
}

}  // namespace

hipError_t launch_fill_ghosts_coarse(int64_t n_fine, int ghost, const int32_t *neighbor,
                                     const int32_t *parent, const int8_t *octant, int64_t n_coarse,
                                     int ghost_c, const double *coarse_old, const double *coarse_new,
                                     double alpha, double theta, double *fine_padded,
                                     unsigned long long *counts, hipStream_t s)
{
  if (n_fine == 0) return hipSuccess;
  const int N = 8 + 2 * ghost;
  const int64_t total = n_fine * (int64_t)N * N * N;
  hipLaunchKernelGGL(k_fill_ghosts_coarse, dim3(grid_blocks(total)), dim3(kBlock), 0, s, n_fine,
                     ghost, neighbor, parent, octant, n_coarse, ghost_c, coarse_old, coarse_new,
                     alpha, theta, fine_padded, counts);
  return hipGetLastError();
}

hipError_t launch_restrict(int64_t n_parent, const int32_t *parent_of, const int32_t *child,
                           int64_t n_fine, const double *fine, int64_t n_coarse, double *coarse,
                           hipStream_t s)
{
  if (n_parent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict, dim3((unsigned)n_parent), dim3(512), 0, s, n_parent, parent_of,
                     child, n_fine, fine, n_coarse, coarse);
  return hipGetLastError();
}

hipError_t launch_flux_accumulate(int64_t n, double *acc, const double *flux, double beta,
                                  double weight, hipStream_t s)
{
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flux_accumulate, dim3(grid_blocks(n)), dim3(kBlock), 0, s, n, acc, flux,
                     beta, weight);
  return hipGetLastError();
}

hipError_t launch_flux_correct(int64_t n_face, const int32_t *faces, int64_t n_coarse,
                               double *coarse, const double *coarse_flux, int64_t n_fine,
                               const double *fine_flux, double dh_c, unsigned long long *skipped,
                               hipStream_t s)
{
  if (n_face == 0) return hipSuccess;
  for (int side = 0; side < 6; ++side) {
    hipLaunchKernelGGL(k_flux_correct, dim3(grid_blocks(n_face * 64)), dim3(kBlock), 0, s, n_face,
                       side, faces, n_coarse, coarse, coarse_flux, n_fine, fine_flux, dh_c, skipped);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace srhd
