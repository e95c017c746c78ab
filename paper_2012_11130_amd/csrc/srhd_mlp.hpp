// srhd_mlp.hpp -- learned initial guess for the Newton inversion: inference of a 3-64-64-1
// perceptron with SiLU activations on the matrix cores of gfx950.
//
// Inputs are three log-scaled invariants of the conserved state, standardised with the training
// set's mean and deviation: f = (log D, log max(|M|/D, 1e-300), log(Et/D)) (feature set 0), or
// f = (log L, log max(|M|/D, 1e-300), log(Et/D)) with L the left-hand side of Eq. 15 as the
// inversion computes it (feature set 1).  The output is the standardised log of the reduced
// enthalpy ht, the unknown of Eq. 15.  The network is consulted only for states with L above a
// gate; the others keep the analytic guess.
//
// One call evaluates the network for the 64 states held by the 64 lanes of a wavefront (every
// lane must be active).  Layer 1 (3 -> 64) is FP32 on the vector units.  Layer 2 (64 -> 64)
// runs on v_mfma_f32_16x16x32_bf16 with the states as the N dimension: D[h][s] =
// sum_k W2[h][k] H1[k][s] with BF16 operands and FP32 accumulation, over four 16-state tiles.
// For that instruction lane l supplies A[i][k] and B[k][n] for i, n = l % 16 and
// k = 8 (l / 16) + 0..7, and receives D[i][n] for n = l % 16, i = 4 (l / 16) + 0..3; so for
// state tile nt each lane forms the 8 layer-1 activations of its K rows for the state in column
// l % 16 (whose inputs it reads from lane 16 nt + l % 16).  Layer 3 (64 -> 1) sums each lane's
// rows of D and then the four lanes that share a column.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srhd {

constexpr int MLP_H = 64;
constexpr int MLP_W1 = 0, MLP_W2 = 192, MLP_W3 = 192 + 4096, MLP_NW = 192 + 4096 + 64;
constexpr int MLP_B1 = 0, MLP_B2 = 64, MLP_B3 = 128, MLP_NB = 129;
constexpr int MLP_NPARAM = 4481;   // W1 b1 W2 b2 W3 b3

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

struct MlpDev {
  const uint16_t *w;    // BF16 weights: W1[64][3], W2[64][64] (row = output unit), W3[64]
  const float *bias;    // b1[64], b2[64], b3
  const float *norm;    // mean_in[3], std_in[3], mean_out, std_out
  int features;         // 0: log D first; 1: log L first
  double gate;          // consulted for L > gate only
};

// SiLU(a) = a sigmoid(a) with the hardware exponential and reciprocal.
__device__ __forceinline__ float silu_f(float a)
{
  return a * __builtin_amdgcn_rcpf(1.0f + __expf(-a));
}

__device__ __forceinline__ float bf16_to_f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Two floats rounded to BF16 (nearest even), lo in the low half: one packed conversion.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
  const f32x2_t v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

union Frag8 {
  bf16x8_t v;
  uint32_t u[4];
};

// Standardised network output z for this lane's features (f0, f1, f2).
// For each 16-state tile the lane forms the B operands of both 32-unit K-slabs (8 registers), then
// accumulates the four 16-row tiles of the hidden layer one at a time (4 accumulator registers)
// and folds each into the layer-3 sum: every layer-1 activation is formed once, and only a small
// working set is live (the step kernels call the network from code that needs its registers).
__device__ __forceinline__ float mlp_eval(const MlpDev &m, float f0, float f1, float f2)
{
  const int lane = threadIdx.x & 63;
  const int grp = lane >> 4, col = lane & 15;
  const float x0 = (f0 - m.norm[0]) / m.norm[3];
  const float x1 = (f1 - m.norm[1]) / m.norm[4];
  const float x2 = (f2 - m.norm[2]) / m.norm[5];
  float out = 0.0f;
#pragma unroll 1
  for (int nt = 0; nt < 4; ++nt) {
    // the weights are the same for every state tile: reload them per tile (from cache) rather
    // than let them be hoisted out of the loop into some 40 registers
    const uint16_t *wgt = m.w;
    const float *bia = m.bias;
    asm volatile("" : "+s"(wgt), "+s"(bia));
    // inputs of the state in column col of tile nt
    const int src = 16 * nt + col;
    const float y0 = __shfl(x0, src, 64), y1 = __shfl(x1, src, 64), y2 = __shfl(x2, src, 64);
    Frag8 b[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      // this lane's units k0 .. k0 + 7: 24 W1 weights (48 bytes at a 16-byte aligned offset of
      // the 16-byte aligned weights) and 8 biases
      const int k0 = 32 * ks + 8 * grp;
      const uint4 *wp = reinterpret_cast<const uint4 *>(wgt + MLP_W1 + 3 * k0);
      const uint4 q0 = wp[0], q1 = wp[1], q2 = wp[2];
      const uint32_t wd[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float h[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int i = 2 * j + e;
          float w3[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int q = 3 * i + c;                  // BF16 element q of the 24
            w3[c] = __uint_as_float(q & 1 ? wd[q >> 1] & 0xffff0000u : wd[q >> 1] << 16);
          }
          float a = __builtin_fmaf(w3[0], y0, bia[MLP_B1 + k0 + i]);
          a = __builtin_fmaf(w3[1], y1, a);
          a = __builtin_fmaf(w3[2], y2, a);
          h[e] = silu_f(a);
        }
        b[ks].u[j] = pack_bf16(h[0], h[1]);
      }
    }
    float pt = 0.0f;       // layer-3 sum over this lane's rows, for the state in column col
#pragma unroll 1
    for (int mt = 0; mt < 4; ++mt) {
      f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        // A[i][k] = W2[16 mt + col][32 ks + 8 grp + 0..7]: 16 contiguous bytes
        const uint4 wv = *reinterpret_cast<const uint4 *>(wgt + MLP_W2 + (16 * mt + col) * 64 + 32 * ks + 8 * grp);
        Frag8 a;
        a.u[0] = wv.x;
        a.u[1] = wv.y;
        a.u[2] = wv.z;
        a.u[3] = wv.w;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b[ks].v, acc, 0, 0, 0);
      }
      // acc[v] = D[16 mt + 4 grp + v][state 16 nt + col]
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int hrow = 16 * mt + 4 * grp + v;
        pt = __builtin_fmaf(bf16_to_f(wgt[MLP_W3 + hrow]), silu_f(acc[v] + bia[MLP_B2 + hrow]), pt);
      }
    }
    // the four lanes of column col hold the sums over rows 4 grp + 16 mt + 0..3: add them (the
    // same two sums, in the same order, in every lane of the column)
    pt += __shfl_xor(pt, 16, 64);
    pt += __shfl_xor(pt, 32, 64);
    if (grp == nt) out = pt;                  // lane 16 nt + col holds the state of that column
  }
  return out + m.bias[MLP_B3];
}

// Natural logarithm of a positive double, in FP32 arithmetic over the whole double range: the
// binary exponent is taken exactly and the log of the mantissa by the hardware log2.
__device__ __forceinline__ float log_wide(double v)
{
  int e;
  const double mnt = frexp(v, &e);          // v = mnt 2^e, mnt in [0.5, 1)
  return ((float)e + __log2f((float)mnt)) * 0.693147180559945309f;
}

// Features of a conserved state, the network's input before standardisation; L is the
// left-hand side of Eq. 15 (used by feature set 1).
__device__ __forceinline__ void mlp_features(int set, double D, double Mx, double My, double Mz,
                                             double Et, double L, float &f0, float &f1, float &f2)
{
  const double iD = 1.0 / D;
  const double m = sqrt(Mx * Mx + My * My + Mz * Mz) * iD;
  f0 = log_wide(set ? L : D);
  f1 = m > 1e-300 ? log_wide(m) : -690.77552789821368f;     // log(1e-300): states at rest
  f2 = log_wide(Et * iD);
}

// Guess of ht for this lane's state from the network (exp of the de-standardised output), or -1
// where the network is not consulted (L at or below the gate, or L not admissible: pass L = 0).
// The whole wavefront must call it; the network runs only if some lane needs it, and then
// `evals` is incremented (per lane: the count of network evaluations performed).
__device__ __forceinline__ double mlp_guess(const MlpDev &m, double D, double Mx, double My,
                                            double Mz, double Et, double L, bool &consulted,
                                            unsigned int &evals)
{
  consulted = L > m.gate;
  if (!__any(consulted)) return -1.0;
  ++evals;
  float f0, f1, f2;
  mlp_features(m.features, D, Mx, My, Mz, Et, L, f0, f1, f2);
  const float z = mlp_eval(m, f0, f1, f2);
  return consulted ? (double)__expf(m.norm[6] + m.norm[7] * z) : -1.0;
}

// The same from features already formed (the caller decided `consulted`, L > gate).
__device__ __forceinline__ double mlp_guess_f(const MlpDev &m, float f0, float f1, float f2,
                                              bool consulted, unsigned int &evals)
{
  if (!__any(consulted)) return -1.0;
  ++evals;
  const float z = mlp_eval(m, f0, f1, f2);
  return consulted ? (double)__expf(m.norm[6] + m.norm[7] * z) : -1.0;
}

}  // namespace srhd
