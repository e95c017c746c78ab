// srhd_mlp.hip -- the learned Newton guess: batch inference on the matrix cores, and the
// training kernels (per-sample forward/backward, a deterministic gradient reduction, Adam).
//
// Network, inputs and BF16 rounding points are those of srhd_mlp.hpp.  Training minimises the
// mean squared error of the standardised output against the standardised log ht.  The backward
// treats the BF16 rounding of the first layer's activations as the identity.  Gradients are
// summed over the minibatch by one thread per parameter in sample order, so they are
// bit-reproducible.
#include <float.h>

#include "srhd_device.hpp"
#include "srhd_internal.hpp"
#include "srhd_mlp.hpp"

namespace srhd {
namespace {

constexpr int kBlk = 256;

// ------------------------------------------------------------------------------ features
// L of Eq. 15 as the inversion computes it (0 when the state is not admissible, Eq. 30).
__device__ __forceinline__ double feature_L(double D, double Mx, double My, double Mz, double Et)
{
  double L;
  return admissible(D, Mx, My, Mz, Et, DBL_EPSILON, L) ? L : 0.0;
}
__device__ __forceinline__ double feature_L(float D, float Mx, float My, float Mz, float Et)
{
  if (!(finiteT(D) && finiteT(Mx) && finiteT(My) && finiteT(Mz) && finiteT(Et)) ||
      !(D > 0.0f) || !(Et > 0.0f))
    return 0.0;
  const double L = lhs_L_from_f32(D, Mx, My, Mz, Et);
  return L > DBL_EPSILON ? L : 0.0;
}

// Features of each state and, when its primitives are given, the training target log ht with
// ht from Eq. 22 at Theta = p / rho.
template <class T>
__global__ void __launch_bounds__(kBlk) k_mlp_features(int set, int64_t n, const T *__restrict__ cons,
                                                       const T *__restrict__ prim,
                                                       float *__restrict__ feat,
                                                       float *__restrict__ target)
{
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float f0, f1, f2;
    const T D = cons[i], Mx = cons[n + i], My = cons[2 * n + i], Mz = cons[3 * n + i],
            Et = cons[4 * n + i];
    const double L = set ? feature_L(D, Mx, My, Mz, Et) : 0.0;
    mlp_features(set, D, Mx, My, Mz, Et, L, f0, f1, f2);
    feat[i] = f0;
    feat[n + i] = f1;
    feat[2 * n + i] = f2;
    if (prim && target) {
      double th = (double)prim[4 * n + i] / (double)prim[i];
      target[i] = (float)log(htilde_of_theta(th));
    }
  }
}

// ------------------------------------------------------------------------------ inference
// y = mean_out + std_out * z for each feature vector.  Every wavefront runs the same number of
// iterations with all lanes active (the matrix instructions need the whole wavefront); lanes past
// the end evaluate a dummy input and store nothing.
__global__ void __launch_bounds__(kBlk) k_mlp_forward(MlpDev m, int64_t n, const float *__restrict__ feat,
                                                      float *__restrict__ y)
{
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    int64_t i = base + threadIdx.x;
    bool ok = i < n;
    float f0 = ok ? feat[i] : 0.0f, f1 = ok ? feat[n + i] : 0.0f, f2 = ok ? feat[2 * n + i] : 0.0f;
    float z = mlp_eval(m, f0, f1, f2);
    if (ok) y[i] = m.norm[6] + m.norm[7] * z;
  }
}

// ------------------------------------------------------------------------------ training
// Per-sample forward and backward in FP32, lane-local, with the inference's rounding points.
// Workspace per sample s (column-major by sample, n = batch):
//   x[3][n] standardised inputs, h1[64][n] (BF16-rounded), h2[64][n], da2[64][n], da1[64][n],
//   dz[n] (= 2 (z - t) / n), r2[n] (= (z - t)^2).
struct TrainWs {
  float *x, *h1, *h2, *da2, *da1, *dz, *r2;
};

__device__ __forceinline__ float dsilu_f(float a)
{
  float s = __builtin_amdgcn_rcpf(1.0f + __expf(-a));
  return s * (1.0f + a * (1.0f - s));
}

__global__ void __launch_bounds__(kBlk) k_mlp_sample_grads(MlpDev m, int64_t n, const float *__restrict__ feat,
                                                           const float *__restrict__ target, TrainWs ws)
{
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[3];
  for (int i = 0; i < 3; ++i) x[i] = (feat[i * n + s] - m.norm[i]) / m.norm[3 + i];
  float a1[64], h1[64];
  for (int k = 0; k < 64; ++k) {
    float a = m.bias[MLP_B1 + k];
    for (int i = 0; i < 3; ++i) a = __builtin_fmaf(bf16_to_f(m.w[MLP_W1 + 3 * k + i]), x[i], a);
    a1[k] = a;
    h1[k] = (float)(__bf16)silu_f(a);                    // the matrix cores' operand precision
  }
  float a2[64];
  float z = m.bias[MLP_B3];
  for (int h = 0; h < 64; ++h) {
    float a = 0.0f;
    for (int k = 0; k < 64; ++k) a = __builtin_fmaf(bf16_to_f(m.w[MLP_W2 + 64 * h + k]), h1[k], a);
    a += m.bias[MLP_B2 + h];
    a2[h] = a;
    float h2 = silu_f(a);
    ws.h2[h * n + s] = h2;
    z = __builtin_fmaf(bf16_to_f(m.w[MLP_W3 + h]), h2, z);
  }
  float t = (target[s] - m.norm[6]) / m.norm[7];
  float r = z - t;
  float dz = 2.0f * r / (float)n;
  ws.dz[s] = dz;
  ws.r2[s] = r * r;
  float da2[64];
  for (int h = 0; h < 64; ++h) {
    da2[h] = bf16_to_f(m.w[MLP_W3 + h]) * dz * dsilu_f(a2[h]);
    ws.da2[h * n + s] = da2[h];
  }
  for (int k = 0; k < 64; ++k) {
    float d = 0.0f;
    for (int h = 0; h < 64; ++h) d = __builtin_fmaf(bf16_to_f(m.w[MLP_W2 + 64 * h + k]), da2[h], d);
    ws.da1[k * n + s] = d * dsilu_f(a1[k]);
    ws.h1[k * n + s] = h1[k];
  }
  for (int i = 0; i < 3; ++i) ws.x[i * n + s] = x[i];
}

// One thread per parameter (and one for the loss): the sum over the minibatch in sample order.
__global__ void __launch_bounds__(kBlk) k_mlp_reduce(int64_t n, TrainWs ws, float *__restrict__ grad,
                                                     float *__restrict__ loss)
{
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > MLP_NPARAM) return;
  const float *a = nullptr, *b = nullptr;
  if (p < 192) { a = ws.da1 + (p / 3) * n; b = ws.x + (p % 3) * n; }                 // W1[h][i]
  else if (p < 256) { a = ws.da1 + (p - 192) * n; }                                   // b1[h]
  else if (p < 4352) { int q = p - 256; a = ws.da2 + (q / 64) * n; b = ws.h1 + (q % 64) * n; }  // W2[h][k]
  else if (p < 4416) { a = ws.da2 + (p - 4352) * n; }                                 // b2[h]
  else if (p < 4480) { a = ws.dz; b = ws.h2 + (p - 4416) * n; }                       // W3[h]
  else if (p == 4480) { a = ws.dz; }                                                  // b3
  else { a = ws.r2; }                                                                 // loss
  double acc = 0.0;
  for (int64_t s = 0; s < n; ++s) acc += b ? (double)a[s] * (double)b[s] : (double)a[s];
  if (p < MLP_NPARAM) grad[p] = (float)acc;
  else loss[0] = (float)(acc / (double)n);
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters; refreshes the BF16 weights and the
// FP32 biases that inference reads.
__global__ void __launch_bounds__(kBlk) k_mlp_adam(float *__restrict__ master, float *__restrict__ m1,
                                                   float *__restrict__ m2, const float *__restrict__ grad,
                                                   int step, float lr, uint16_t *__restrict__ w,
                                                   float *__restrict__ bias)
{
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float g = grad[p];
  float mm = b1 * m1[p] + (1.0f - b1) * g;
  float vv = b2 * m2[p] + (1.0f - b2) * g * g;
  m1[p] = mm;
  m2[p] = vv;
  float mh = mm / (1.0f - powf(b1, (float)step));
  float vh = vv / (1.0f - powf(b2, (float)step));
  float th = master[p] - lr * mh / (sqrtf(vh) + eps);
  master[p] = th;
  uint16_t bf = __builtin_bit_cast(uint16_t, (__bf16)th);
  if (p < 192) w[MLP_W1 + p] = bf;
  else if (p < 256) bias[MLP_B1 + p - 192] = th;
  else if (p < 4352) w[MLP_W2 + p - 256] = bf;
  else if (p < 4416) bias[MLP_B2 + p - 4352] = th;
  else if (p < 4480) w[MLP_W3 + p - 4416] = bf;
  else bias[MLP_B3] = th;
}

inline int grid_of(int64_t n)
{
  int64_t b = (n + kBlk - 1) / kBlk;
  if (b < 1) b = 1;
  if (b > 256 * 64) b = 256 * 64;
  return (int)b;
}

}  // namespace

size_t mlp_workspace_bytes(int64_t batch) { return (size_t)batch * (3 + 4 * 64 + 2) * 4 + 256; }

hipError_t launch_mlp_features(int dtype, int features, int64_t n, const void *cons, const void *prim,
                               float *feat, float *target, hipStream_t s)
{
  if (n == 0) return hipSuccess;
  if (dtype == SRHD_F64)
    hipLaunchKernelGGL(k_mlp_features<double>, dim3(grid_of(n)), dim3(kBlk), 0, s, features, n,
                       (const double *)cons, (const double *)prim, feat, target);
  else
    hipLaunchKernelGGL(k_mlp_features<float>, dim3(grid_of(n)), dim3(kBlk), 0, s, features, n,
                       (const float *)cons, (const float *)prim, feat, target);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev &m, int64_t n, const float *feat, float *y, hipStream_t s)
{
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid_of(n)), dim3(kBlk), 0, s, m, n, feat, y);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDev &m, int64_t n, const float *feat, const float *target,
                           float *grad, float *loss, void *ws, hipStream_t s)
{
  TrainWs w;
  float *f = (float *)ws;
  w.x = f;
  w.h1 = w.x + 3 * n;
  w.h2 = w.h1 + 64 * n;
  w.da2 = w.h2 + 64 * n;
  w.da1 = w.da2 + 64 * n;
  w.dz = w.da1 + 64 * n;
  w.r2 = w.dz + n;
  hipLaunchKernelGGL(k_mlp_sample_grads, dim3((unsigned)((n + kBlk - 1) / kBlk)), dim3(kBlk), 0, s,
                     m, n, feat, target, w);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + kBlk - 1) / kBlk), dim3(kBlk), 0, s,
                     n, w, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float *master, float *m1, float *m2, const float *grad, int step,
                           float lr, uint16_t *w, float *bias, hipStream_t s)
{
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + kBlk - 1) / kBlk), dim3(kBlk), 0, s, master,
                     m1, m2, grad, step, lr, w, bias);
  return hipGetLastError();
}

}  // namespace srhd
