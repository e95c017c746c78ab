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
// lane must be active).  Layer 1 (3 -> 64) is lane-local FP32.  Layer 2 (64 -> 64) runs on
// v_mfma_f32_32x32x16_bf16 with the states as the N dimension: D[h][s] = sum_k W2[h][k] H1[k][s]
// with BF16 operands and FP32 accumulation.  For that instruction lane l supplies B[k][n] for
// n = l % 32 and k = 8 (l / 32) + 0..7; every lane holds all 64 hidden values of its own state,
// so one v_permlane32_swap per register builds the operands of both 32-state tiles at once.
// Layer 3 (64 -> 1) sums each lane's 32 rows of D and adds the partner lane's half.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srhd {

constexpr int MLP_H = 64;
constexpr int MLP_W1 = 0, MLP_W2 = 192, MLP_W3 = 192 + 4096, MLP_NW = 192 + 4096 + 64;
constexpr int MLP_B1 = 0, MLP_B2 = 64, MLP_B3 = 128, MLP_NB = 129;
constexpr int MLP_NPARAM = 4481;   // W1 b1 W2 b2 W3 b3

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

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
// The two 32-row halves of the hidden layer are produced one after the other, each from four
// K-slabs of 16 layer-1 units (the K extent of one matrix instruction): a slab is packed to
// BF16, lane-swapped into the two state tiles' B operands and accumulated into the half's two
// 32x32 output tiles [state tile].  Layer 1 is evaluated once per half, so only 32 accumulator
// registers and one slab of activations are live at a time (the step kernels run this inside
// code that needs its registers).
__device__ __forceinline__ float mlp_eval(const MlpDev &m, float f0, float f1, float f2)
{
  const int lane = threadIdx.x & 63;
  const float x0 = (f0 - m.norm[0]) / m.norm[3];
  const float x1 = (f1 - m.norm[1]) / m.norm[4];
  const float x2 = (f2 - m.norm[2]) / m.norm[5];

  float part0 = 0.0f, part1 = 0.0f;     // layer-3 partial sums of state tiles 0 and 1
#pragma unroll 1
  for (int mt = 0; mt < 2; ++mt) {
    f32x16_t acc0 = {}, acc1 = {};      // rows 32 mt .. 32 mt + 31, state tiles 0 and 1
#pragma unroll 1
    for (int ks = 0; ks < 4; ++ks) {
      Frag8 lo, hi;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        // hidden units k0 and k0 + 1 of this slab; j < 4 fills the low half, j >= 4 the high half
        const int k0 = 16 * ks + 2 * j;
        float h[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int k = k0 + e;
          float a = m.bias[MLP_B1 + k];
          a = __builtin_fmaf(bf16_to_f(m.w[MLP_W1 + 3 * k + 0]), x0, a);
          a = __builtin_fmaf(bf16_to_f(m.w[MLP_W1 + 3 * k + 1]), x1, a);
          a = __builtin_fmaf(bf16_to_f(m.w[MLP_W1 + 3 * k + 2]), x2, a);
          h[e] = silu_f(a);
        }
        if (j < 4) lo.u[j] = pack_bf16(h[0], h[1]);
        else hi.u[j - 4] = pack_bf16(h[0], h[1]);
      }
      // lanes < 32 keep their own low half and receive the low half of lane + 32 (second
      // tile); lanes >= 32 receive the high half of lane - 32 (first tile), keep their own high
      Frag8 t0, t1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        auto r = __builtin_amdgcn_permlane32_swap(lo.u[j], hi.u[j], false, false);
        t0.u[j] = r[0];
        t1.u[j] = r[1];
      }
      // A[h][k] = W2[32 mt + lane % 32][16 ks + 8 (lane / 32) + 0..7]: 16 contiguous bytes
      const uint4 wv = *reinterpret_cast<const uint4 *>(
          m.w + MLP_W2 + (32 * mt + (lane & 31)) * 64 + 16 * ks + 8 * (lane >> 5));
      Frag8 a;
      a.u[0] = wv.x;
      a.u[1] = wv.y;
      a.u[2] = wv.z;
      a.u[3] = wv.w;
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, t0.v, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, t1.v, acc1, 0, 0, 0);
    }
    // layer 3 on this half: acc_nt[v] = D[32 mt + 8 (v / 4) + 4 (lane / 32) + v % 4][32 nt + lane % 32]
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int hrow = 32 * mt + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const float w3 = bf16_to_f(m.w[MLP_W3 + hrow]);
      const float b2 = m.bias[MLP_B2 + hrow];
      part0 = __builtin_fmaf(w3, silu_f(acc0[v] + b2), part0);
      part1 = __builtin_fmaf(w3, silu_f(acc1[v] + b2), part1);
    }
  }
  // the other half of the 64 rows of a state's column sits in lane ^ 32; the state of this lane
  // is column lane % 32 of tile lane / 32
  const float part = lane < 32 ? part0 : part1;
  const float give = lane < 32 ? part1 : part0;     // what the partner lane needs
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(give), __float_as_uint(give), false, false);
  const float other = __uint_as_float(lane < 32 ? r[1] : r[0]);
  return part + other + m.bias[MLP_B3];
}

// The same network with one 32x32 accumulator tile live at a time.  The B operand of state tile
// nt holds, in lane l, hidden units 16 ks + 8 (l / 32) + 0..7 of the state in column l % 32 of
// that tile, so each lane forms just those 8 activations per slab, from that state's inputs (one
// lane swap per tile), for each (tile, half of the hidden layer) pass: the same layer-1 work as
// mlp_eval, no swaps per slab, and only 16 accumulator registers and one B operand live (the
// step kernels call the network from code that needs its registers).  The activations, the
// MFMA operands, their order and the layer-3 sums are those of mlp_eval, so the result is the
// same bit for bit.
__device__ __forceinline__ float mlp_eval_lean(const MlpDev &m, float f0, float f1, float f2)
{
  const int lane = threadIdx.x & 63;
  const float x0 = (f0 - m.norm[0]) / m.norm[3];
  const float x1 = (f1 - m.norm[1]) / m.norm[4];
  const float x2 = (f2 - m.norm[2]) / m.norm[5];
  float part0 = 0.0f, part1 = 0.0f;
#pragma unroll 1
  for (int nt = 0; nt < 2; ++nt) {
    // inputs of the state in column lane % 32 of tile nt (lane % 32 + 32 nt)
    float y0, y1, y2;
    {
      auto r0 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x0), __float_as_uint(x0), false, false);
      auto r1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x1), __float_as_uint(x1), false, false);
      auto r2 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x2), __float_as_uint(x2), false, false);
      y0 = __uint_as_float(nt ? r0[1] : r0[0]);
      y1 = __uint_as_float(nt ? r1[1] : r1[0]);
      y2 = __uint_as_float(nt ? r2[1] : r2[0]);
    }
    float pt = 0.0f;
#pragma unroll 1
    for (int mt = 0; mt < 2; ++mt) {
      f32x16_t acc = {};
#pragma unroll 1
      for (int ks = 0; ks < 4; ++ks) {
        // this lane's units k0 .. k0 + 7: their 24 W1 weights (48 bytes at a 16-byte aligned
        // offset of the 16-byte aligned weights) and their biases
        const int k0 = 16 * ks + 8 * (lane >> 5);
        const uint4 *wp = reinterpret_cast<const uint4 *>(m.w + MLP_W1 + 3 * k0);
        const uint4 q0 = wp[0], q1 = wp[1], q2 = wp[2];
        const uint32_t wd[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
        float b1[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) b1[i] = m.bias[MLP_B1 + k0 + i];
        Frag8 t;
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
            float a = __builtin_fmaf(w3[0], y0, b1[i]);
            a = __builtin_fmaf(w3[1], y1, a);
            a = __builtin_fmaf(w3[2], y2, a);
            h[e] = silu_f(a);
          }
          t.u[j] = pack_bf16(h[0], h[1]);
        }
        const uint4 wv = *reinterpret_cast<const uint4 *>(
            m.w + MLP_W2 + (32 * mt + (lane & 31)) * 64 + 16 * ks + 8 * (lane >> 5));
        Frag8 a;
        a.u[0] = wv.x;
        a.u[1] = wv.y;
        a.u[2] = wv.z;
        a.u[3] = wv.w;
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, t.v, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int hrow = 32 * mt + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        pt = __builtin_fmaf(bf16_to_f(m.w[MLP_W3 + hrow]), silu_f(acc[v] + m.bias[MLP_B2 + hrow]), pt);
      }
    }
    if (nt == 0) part0 = pt;
    else part1 = pt;
  }
  const float part = lane < 32 ? part0 : part1;
  const float give = lane < 32 ? part1 : part0;
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(give), __float_as_uint(give), false, false);
  const float other = __uint_as_float(lane < 32 ? r[1] : r[0]);
  return part + other + m.bias[MLP_B3];
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
// LEAN selects mlp_eval_lean (inside the step kernels) or mlp_eval (throughput kernels); both
// give the same result.
// The whole wavefront must call it; the network runs only if some lane needs it, and then
// `evals` is incremented (per lane: the count of network evaluations performed).
template <bool LEAN = true>
__device__ __forceinline__ double mlp_guess(const MlpDev &m, double D, double Mx, double My,
                                            double Mz, double Et, double L, bool &consulted,
                                            unsigned int &evals)
{
  consulted = L > m.gate;
  if (!__any(consulted)) return -1.0;
  ++evals;
  float f0, f1, f2;
  mlp_features(m.features, D, Mx, My, Mz, Et, L, f0, f1, f2);
  const float z = LEAN ? mlp_eval_lean(m, f0, f1, f2) : mlp_eval(m, f0, f1, f2);
  return consulted ? (double)__expf(m.norm[6] + m.norm[7] * z) : -1.0;
}

// The same from features already formed (the caller decided `consulted`, L > gate).
__device__ __forceinline__ double mlp_guess_f(const MlpDev &m, float f0, float f1, float f2,
                                              bool consulted, unsigned int &evals)
{
  if (!__any(consulted)) return -1.0;
  ++evals;
  const float z = mlp_eval_lean(m, f0, f1, f2);
  return consulted ? (double)__expf(m.norm[6] + m.norm[7] * z) : -1.0;
}

}  // namespace srhd
