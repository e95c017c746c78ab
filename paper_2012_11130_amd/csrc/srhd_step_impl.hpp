// srhd_step_impl.hpp -- one unsplit MUSCL-Hancock step (Sec. 3.2) of a batch of padded 8^3 patches
// on gfx950: one workgroup of 512 threads (8 wavefronts) per patch, with the patch's
// primitive tile, half-step corrections and interface fluxes staged in LDS.
//
// Work per patch (interior coordinates i in [0, 8); ghosts at -1, -2, 8, 9 are used):
//   A. cell-centre inversions of the 1376 cells the stencil touches       -> LDS W (12^3 box)
//   B. for the 896 cells whose face states the full step needs (the interior and the first
//      ghost layer across each face): PLM slopes in x, y, z, the six face states, their
//      conserved variables and physical fluxes, and the half-step correction
//      C = -(dt / 2dh) sum_d [F_d(W_{d,+}) - F_d(W_{d,-})]                  -> LDS C (10^3 box)
//   C. for the 3 x 576 interfaces: the two half-step face states U(W_face) + C, their
//      inversions, and the HLLC / HLLE flux                                  -> LDS F (ring)
//   D. the full update U^{n+1} = U^n - (dt/dh) sum_d (F_{+1/2} - F_{-1/2}) with the Eq. 30
//      check of every output cell.
// Phase C runs over the flat list of 1728 interfaces in rounds of 512; a two-direction ring
// buffer of fluxes lets each thread fold a direction's flux differences into its own cell as
// soon as that direction is complete (x after round 1, y after round 2, z after round 3).
// If any half-step face state or output cell is unphysical, the whole patch repeats B-D with
// theta *= 0.75 (max_retry times), then theta = 0 (Sec. 3.4); A is not repeated.
//
// Kernel variants K: the analytic guess of App. A, the learned guess, the original scheme of
// Sec. 4 (the total energy E of Eq. 5c in the energy slot, evolved with the flux M_d, and every
// inversion from the naive L = (E/D)^2 - (|M|/D)^2 - 1 of Eq. 21 in the inversion type; analytic
// guess, padded layout, equal bulk and inversion types only), and the polytropic EoS of Sec. 2.2
// (padded layout).
#pragma once
#include <float.h>
#include <type_traits>

#include "srhd_device.hpp"
#include "srhd_internal.hpp"

namespace srhd {
namespace {

constexpr int NT = 512;          // interior cells per patch (threads of an FP32-bulk workgroup)

// Threads per workgroup: one per interior cell.  The phases are written for any multiple of 512
// (threads 512.. would take part in the tile phases only); 1024 for the FP64 bulk, whose 155 KB
// tile admits one workgroup per CU, doubles the wavefronts per SIMD but caps the registers at 128
// and spills 170-250 bytes per lane, and measured no faster, so every kernel runs 512.
template <class T> constexpr int threads_of() { return sizeof(T) == 8 ? 768 : 512; }
constexpr int NT_MAX = 1024;
constexpr int BX = 12;           // primitive box [-2, 10)^3
constexpr int NB = BX * BX * BX;
constexpr int HX = 10;           // half-step box [-1, 9)^3
constexpr int NHB = HX * HX * HX;
constexpr int NPC = 1376;        // centre inversions per patch
constexpr int NHC = 896;         // half-step cells per patch
constexpr int NIF = 576;         // interfaces per direction (9 x 8 x 8)

constexpr bool in_half(int i, int j, int k)
{
  int c[3] = {i, j, k};
  int out = 0;
  for (int d = 0; d < 3; ++d) {
    if (c[d] >= 0 && c[d] < 8) continue;
    if (c[d] == -1 || c[d] == 8) ++out;
    else return false;
  }
  return out <= 1;
}

constexpr bool in_prim(int i, int j, int k)
{
  return in_half(i, j, k) || in_half(i - 1, j, k) || in_half(i + 1, j, k) ||
         in_half(i, j - 1, k) || in_half(i, j + 1, k) || in_half(i, j, k - 1) ||
         in_half(i, j, k + 1);
}

struct Tables {
  uint16_t pcell[NPC];   // 12-box index of each centre cell, increasing (x fastest)
  uint16_t hcell[NHC];   // 10-box index of each half-step cell, increasing
};

constexpr Tables make_tables()
{
  Tables t{};
  int np = 0, nh = 0;
  for (int k = -2; k < 10; ++k)
    for (int j = -2; j < 10; ++j)
      for (int i = -2; i < 10; ++i) {
        if (in_prim(i, j, k)) t.pcell[np++] = (uint16_t)(((k + 2) * BX + (j + 2)) * BX + (i + 2));
        if (in_half(i, j, k)) t.hcell[nh++] = (uint16_t)(((k + 1) * HX + (j + 1)) * HX + (i + 1));
      }
  return t;
}

constexpr Tables kTabInit = make_tables();
static_assert(kTabInit.pcell[NPC - 1] != 0 && kTabInit.hcell[NHC - 1] != 0, "cell tables");
__constant__ Tables kTab = kTabInit;

enum : int { KV_ANALYTIC = 0, KV_MLP = 1, KV_TOTAL = 2, KV_POLY = 3 };

// The EoS of a variant: the polytropic EoS (Sec. 2.2) for KV_POLY (analytic-type guess, padded
// layout), TM otherwise.
template <int K> struct KEos { using type = EosTm; };
template <> struct KEos<KV_POLY> { using type = EosPoly; };
template <int K>
__device__ __forceinline__ typename KEos<K>::type make_eos(const StepArgs &a)
{
  if constexpr (K == KV_POLY) return EosPoly{a.eos_k};
  else return EosTm{};
}

// The analytic guess's type and the recovery's: FP32 whenever the bulk is FP32 (a starting point,
// and primitives consumed in FP32), else I.
template <class T, class I>
using GuessT = typename std::conditional<sizeof(T) == 4, float, I>::type;

// Refined hardware reciprocals and square roots (about 1 ulp) in the inversions and L: every FP64
// step kernel and entry inversion (the padded and gather layouts and the CFL kernel therefore
// give the same bits), and the FP32-bulk gather kernels (in the FP32-bulk padded kernels they
// cost registers and occupancy).
template <class T, bool GATHER> constexpr bool fast_of() { return sizeof(T) == 8 || GATHER; }
// Downstream of the face inversions (the face states' gamma, 1 / gamma and c_s^2, the Riemann
// solver) the FP64 bulk divides through the refined reciprocal (about 1 ulp).  Upstream of them
// (slopes, prim -> cons, the half-step corrections) it does so only in patches whose tile holds
// no cell with kappa = 1 + M^2 above KAPPA_FAST: an inversion turns a changed rounding of its
// input into a change of the face state of up to kappa times it (Eq. 20), under 1e-12 there but
// about 1e-9 where kappa ~ 1e6, beyond the step's 1e-10 parity against the oracle; those patches
// keep IEEE division.  The FP32 bulk keeps its own arithmetic.
template <class T> constexpr bool fx_of() { return sizeof(T) == 8; }
constexpr double KAPPA_FAST = 1000.0;

// Newton tolerance by (bulk type T, inversion type I): FP64 to ~2^-54; an FP64 inversion whose
// result is consumed in FP32 to ~2^-28; an FP32 inversion to FP32 accuracy.
template <class T, class I> struct StepTol;
template <> struct StepTol<double, double> { static constexpr double v = 0x1p-27; };
template <> struct StepTol<float, double> { static constexpr double v = 0x1p-14; };
template <> struct StepTol<float, float> { static constexpr double v = 0x1p-12; };

// LDS tile.  Field-major so that neighbouring lanes touch neighbouring words.
template <class T>
struct Tile {
  T W[5][NB];            // centre primitives (rho, Ux, Uy, Uz, p), 12^3 box
  T C[5][NHB];           // half-step corrections, 10^3 box
  T F[2][5][NIF];        // interface fluxes of two directions (ring)
  double red[NT_MAX / 64];   // per-wavefront maxima
  unsigned int cnt[8];   // workgroup counters
  int nb[32];            // neighbour table row (gather mode)
  unsigned long long claim;  // queue position claimed by the workgroup (persistent schedule)
  unsigned int orf[2][4];    // workgroup OR (wg_or): one byte per wavefront, two buffers
};

// the updated state of the final inversion (5 doubles per thread) is parked in the primitive tile
static_assert(sizeof(float) * 5 * NB >= sizeof(double) * 5 * NT, "parking space in the tile");

// Workgroup-wide OR of a per-thread bit set (8 bits) with one barrier: lane 0 of each wavefront
// stores its wavefront's OR (a ballot per bit) into its byte of buffer `par`, and every thread
// reads the buffer after the barrier.  The two buffers alternate, so a buffer is written again
// only after a further barrier -- after every thread has read it; bytes of absent wavefronts are
// zeroed at the patch's start.  (The runtime's __syncthreads_or costs three barriers and a static
// LDS block, which moves the dynamic tile to a link-time offset and the tile's addresses into
// spilled scalar registers.)  Every thread of the workgroup must call it.  S: a tile with the
// member orf[2][4].
template <class S>
__device__ __forceinline__ unsigned int wg_or(S &s, unsigned int v, int &par)
{
  unsigned int m = 0u;
#pragma unroll
  for (int i = 0; i < 8; ++i) m |= (__ballot((v >> i) & 1u) != 0ull ? 1u : 0u) << i;
  if ((threadIdx.x & 63) == 0) reinterpret_cast<unsigned char *>(s.orf[par])[threadIdx.x >> 6] = (unsigned char)m;
  __syncthreads();
  const uint4 q = *reinterpret_cast<const uint4 *>(s.orf[par]);
  par ^= 1;
  unsigned int r = q.x | q.y | q.z | q.w;
  r |= r >> 16;
  r |= r >> 8;
  return r & 0xffu;
}

__device__ __forceinline__ int bidx(int i, int j, int k) { return ((k + 2) * BX + (j + 2)) * BX + (i + 2); }
__device__ __forceinline__ int hidx(int i, int j, int k) { return ((k + 1) * HX + (j + 1)) * HX + (i + 1); }

template <class T>
__device__ __forceinline__ Prim<T> load_prim(const Tile<T> &s, int b)
{
  Prim<T> w;
  w.rho = s.W[0][b];
  w.u[0] = s.W[1][b];
  w.u[1] = s.W[2][b];
  w.u[2] = s.W[3][b];
  w.p = s.W[4][b];
  return w;
}

// Double inversion of bulk-type conserved variables (FP64 path: the adaptive sum of the rounded
// products; mixed path: the float values' products are exact in double).
template <bool FAST>
__device__ __forceinline__ double L_of(const Cons<double> &u) { return lhs_L_adaptive<FAST>(u.D, u.m[0], u.m[1], u.m[2], u.E); }
template <bool FAST>
__device__ __forceinline__ double L_of(const Cons<float> &u) { return lhs_L_from_f32_adaptive<FAST>(u.D, u.m[0], u.m[1], u.m[2], u.E); }

// Admissibility (Eq. 30) of a face state and its L (0 when not admissible).
template <bool FAST, class T>
__device__ __forceinline__ bool face_L(const Cons<T> &u, double &L)
{
  bool ok = finiteT(u.D) && finiteT(u.m[0]) && finiteT(u.m[1]) && finiteT(u.m[2]) &&
            finiteT(u.E) && u.D > T(0) && u.E > T(0);
  L = ok ? L_of<FAST>(u) : 0.0;
  ok = ok && L > DBL_EPSILON;
  if (!ok) L = 0.0;
  return ok;
}

// Inversion of a face state in the inversion type I from its (exact, FP64) L.  With a learned
// guess (MLP) the wavefront takes the guess-free inversion unless one of its lanes has a guess:
// that inversion is the analytic-guess build's code, with the supplied-guess start and its
// fallback attempt compiled out.
// x receives gamma, 1 / gamma and c_s^2 of the face state for the Riemann solver: from the FP32
// TM recovery, which has them, else formed from w.
template <class I, bool MLP, bool FAST, class T, class E>
__device__ __forceinline__ bool invert_face(const Cons<T> &u, bool ok, double L, Prim<T> &w,
                                            FaceAux<T> &x, int &iters, int &status, double guess,
                                            bool have_guess, const E &eos)
{
  I D = u.D, Mx = u.m[0], My = u.m[1], Mz = u.m[2];
  InvOut<I> o;
  const bool any_guess = MLP && __any(have_guess);
  if (ok) {
    if (any_guess)
      invert_with_L<I, GuessT<T, I>, GuessT<T, I>, FAST>(D, Mx, My, Mz, (I)L, (I)guess, have_guess, (I)StepTol<T, I>::v, 30, o, eos);
    else
      invert_with_L<I, GuessT<T, I>, GuessT<T, I>, FAST>(D, Mx, My, Mz, (I)L, (I)-1.0, false, (I)StepTol<T, I>::v, 30, o, eos);
  } else set_unphysical(o);
  w.rho = (T)o.rho;
  w.u[0] = (T)o.ux;
  w.u[1] = (T)o.uy;
  w.u[2] = (T)o.uz;
  w.p = (T)o.p;
  if constexpr (sizeof(T) == 4 && std::is_same<E, EosTm>::value) {
    x.gam = (T)o.gam;
    x.igam = (T)o.igam;
    x.cs2 = (T)o.cs2;
  } else {
    x = face_aux<fx_of<T>()>(w, eos);
  }
  iters = o.iters;
  status = o.status;
  return ok;
}

// Face state of cell (i, j, k) on side `side` (0: minus, 1: plus) of direction d: PLM along d,
// prim -> cons, plus the cell's half-step correction, then the inversion.
template <int d, int K, class I, bool FAST, bool FXU, class T>
__device__ __forceinline__ bool face_state(const Tile<T> &s, int side, int i, int j, int k,
                                           T theta, const MlpDev &mlp, Prim<T> &w, Cons<T> &u,
                                           FaceAux<T> &x, int &iters, int &status, unsigned int &evals,
                                           const typename KEos<K>::type &eos)
{
  constexpr int sd = d == 0 ? 1 : (d == 1 ? BX : BX * BX);
  int b = bidx(i, j, k);
  int hb = hidx(i, j, k);
  T half = side ? T(0.5) : T(-0.5);
  Prim<T> wf;
  T v[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    T wc = s.W[f][b];
    v[f] = wc + half * limited_slope<FXU>(s.W[f][b - sd], wc, s.W[f][b + sd], theta);
  }
  wf.rho = v[0];
  wf.u[0] = v[1];
  wf.u[1] = v[2];
  wf.u[2] = v[3];
  wf.p = v[4];
  constexpr bool MLP = K == KV_MLP;
  u = prim2cons_s<K == KV_TOTAL, FXU>(wf, eos);
  u.D += s.C[0][hb];
  u.m[0] += s.C[1][hb];
  u.m[1] += s.C[2][hb];
  u.m[2] += s.C[3][hb];
  u.E += s.C[4][hb];
  // the learned guess is evaluated by every lane of the wavefront (a wavefront handles one
  // direction and all its lanes are active here)
  double L;
  bool ok;
  if constexpr (K == KV_TOTAL) ok = admissible_total<I>(u.D, u.m[0], u.m[1], u.m[2], u.E, L);
  else ok = face_L<FAST>(u, L);
  bool consulted = false;
  double guess = MLP ? mlp_guess(mlp, u.D, u.m[0], u.m[1], u.m[2], u.E, L, consulted, evals) : -1.0;
  return invert_face<I, MLP, FAST>(u, ok, L, w, x, iters, status, guess, consulted, eos);
}

// Physical flux along d of a face state given by its primitives, with 1 / gamma = rho / D from
// the conserved variables just formed (one reciprocal instead of a square root and a reciprocal).
// The original scheme (TOT) keeps its own arithmetic: it is the comparison baseline.
template <int d, bool TOT, bool FXU, class T, class E>
__device__ __forceinline__ Cons<T> state_flux(const Prim<T> &w, const E &eos)
{
  const Cons<T> u = prim2cons_s<TOT, FXU>(w, eos);
  if constexpr (TOT) return phys_flux<d, TOT>(w, u);
  else return phys_flux<d, TOT>(w, u, w.rho * dvx<FXU>(T(1), u.D));
}

struct IfaceCount {
  unsigned int iters, inv, fb, nc, unphys, mlp;
};

// Flux through interface r of direction d (between cells c-1 and c along d, interfaces numbered
// with x fastest, then y, then z), written to the ring slot of d.
template <int d, int K, class I, bool FAST, bool FXU, class T>
__device__ __forceinline__ bool interface_flux(Tile<T> &s, int r, T theta, int solver,
                                               const MlpDev &mlp, IfaceCount &cnt,
                                               const typename KEos<K>::type &eos)
{
  // x is the fastest index in every direction, so the lanes of a wavefront read neighbouring
  // LDS words (a y- or z-fastest order would put them 12 or 144 words apart, on few banks)
  int cr[3];
  if (d == 0) { cr[0] = r % 9; cr[1] = (r / 9) & 7; cr[2] = r / 72; }         // x in [0, 9)
  else if (d == 1) { cr[0] = r & 7; cr[1] = (r >> 3) % 9; cr[2] = r / 72; }   // y in [0, 9)
  else { cr[0] = r & 7; cr[1] = (r >> 3) & 7; cr[2] = r >> 6; }               // z in [0, 9)
  int cl[3] = {cr[0], cr[1], cr[2]};
  cl[d] -= 1;
  Prim<T> wl, wr;
  Cons<T> ul, ur;
  FaceAux<T> xl, xr;
  int itl, itr, stl, str;
  bool okl = face_state<d, K, I, FAST, FXU>(s, 1, cl[0], cl[1], cl[2], theta, mlp, wl, ul, xl, itl, stl, cnt.mlp, eos);
  bool okr = face_state<d, K, I, FAST, FXU>(s, 0, cr[0], cr[1], cr[2], theta, mlp, wr, ur, xr, itr, str, cnt.mlp, eos);
  cnt.iters += itl + itr;
  cnt.inv += 2;
  cnt.fb += (stl == ST_FALLBACK) + (str == ST_FALLBACK);
  cnt.nc += (stl == ST_NOCONV) + (str == ST_NOCONV);
  cnt.unphys += !okl + !okr;
  // the face states' conserved variables are the ones just inverted: no round trip through
  // prim -> cons
  constexpr bool TOT = K == KV_TOTAL;
  constexpr bool FX = fx_of<T>();
  Cons<T> F = solver == SRHD_HLLE ? hlle<d, TOT, FX>(wl, wr, ul, ur, xl, xr)
                                  : hllc<d, TOT, FX>(wl, wr, ul, ur, xl, xr);
  constexpr int slot = d & 1;
  s.F[slot][0][r] = F.D;
  s.F[slot][1][r] = F.m[0];
  s.F[slot][2][r] = F.m[1];
  s.F[slot][3][r] = F.m[2];
  s.F[slot][4][r] = F.E;
  return okl && okr;
}

// Reductions over a wavefront into its last lane (lane 63; the other lanes keep partial
// results), on the cross-lane DPP paths of the VALU rather than LDS permutes: an inclusive scan
// within each row of 16 lanes (row_shr 1, 2, 4, 8), then the row totals carried into rows 1 and 3
// (row_bcast:15) and from lane 31 into rows 2 and 3 (row_bcast:31).  A lane whose DPP source lies
// outside its row, or whose row the row mask leaves out, receives `old`: the operation's neutral
// value (0 for a sum or an OR, the lane's own value for a maximum).  Every lane must be active.
// Counters are summed this way before one lane per wavefront adds them to the workgroup's (an
// atomic add from all 64 lanes to one address is compiled to a loop over the lanes, which cost the
// whole step ~15 %); the six dependent LDS permutes per value of a butterfly cost the patch's tail
// ~3 % of the FP64 step.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned int dpp_u32(unsigned int old, unsigned int v)
{
  return (unsigned int)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double old, double v)
{
  const unsigned long long o = (unsigned long long)__double_as_longlong(old),
                           x = (unsigned long long)__double_as_longlong(v);
  const unsigned int lo = dpp_u32<CTRL, ROWS>((unsigned int)o, (unsigned int)x);
  const unsigned int hi = dpp_u32<CTRL, ROWS>((unsigned int)(o >> 32), (unsigned int)(x >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ unsigned int wave_sum_hi(unsigned int v)
{
  v += dpp_u32<0x111, 0xf>(0u, v);
  v += dpp_u32<0x112, 0xf>(0u, v);
  v += dpp_u32<0x114, 0xf>(0u, v);
  v += dpp_u32<0x118, 0xf>(0u, v);
  v += dpp_u32<0x142, 0xa>(0u, v);
  v += dpp_u32<0x143, 0xc>(0u, v);
  return v;
}

__device__ __forceinline__ unsigned int wave_or_hi(unsigned int v)
{
  v |= dpp_u32<0x111, 0xf>(0u, v);
  v |= dpp_u32<0x112, 0xf>(0u, v);
  v |= dpp_u32<0x114, 0xf>(0u, v);
  v |= dpp_u32<0x118, 0xf>(0u, v);
  v |= dpp_u32<0x142, 0xa>(0u, v);
  v |= dpp_u32<0x143, 0xc>(0u, v);
  return v;
}

__device__ __forceinline__ double wave_max_hi(double v)
{
  v = fmax(v, dpp_f64<0x111, 0xf>(v, v));
  v = fmax(v, dpp_f64<0x112, 0xf>(v, v));
  v = fmax(v, dpp_f64<0x114, 0xf>(v, v));
  v = fmax(v, dpp_f64<0x118, 0xf>(v, v));
  v = fmax(v, dpp_f64<0x142, 0xa>(v, v));
  v = fmax(v, dpp_f64<0x143, 0xc>(v, v));
  return v;
}

// Network-mask regions of interior cell (i, j, k): bit (rz + 1) 9 + (ry + 1) 3 + (rx + 1) for
// every region it lies in, along each axis r = 0 (every cell), r = -1 (the two lowest layers),
// r = +1 (the two highest).
__device__ __forceinline__ unsigned int region_mask(int i, int j, int k)
{
  const unsigned int ax = 2u | (i < 2 ? 1u : 0u) | (i >= 6 ? 4u : 0u);
  const unsigned int ay = 2u | (j < 2 ? 1u : 0u) | (j >= 6 ? 4u : 0u);
  const unsigned int az = 2u | (k < 2 ? 1u : 0u) | (k >= 6 ? 4u : 0u);
  unsigned int m = 0u;
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int x = 0; x < 3; ++x)
        if (((az >> z) & (ay >> y) & (ax >> x)) & 1u) m |= 1u << (z * 9 + y * 3 + x);
  return m;
}

// Whether the 12^3 tile of a patch with neighbours nb[27] (index (dz + 1) 9 + (dy + 1) 3 +
// (dx + 1) for the neighbour at offset (dx, dy, dz); -1 where there is none) holds a cell that
// set a network mask: neighbour n contributes the region next to the patch, (-dx, -dy, -dz), whose
// bit is 26 - n.  (Where a face neighbour is missing, the tile's outflow copies come from cells
// in regions with r = 0 along that axis, which the other entries cover.)
__device__ __forceinline__ bool tile_hits_mask(int n, int64_t q, int64_t n_patch, const unsigned int *mask)
{
  return q >= 0 && q < n_patch && ((mask[q] >> (26 - n)) & 1u);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2); this mapping
// hands each XCD a contiguous range of patches so that neighbouring patches, whose cells the
// gather reads, are processed under the same L2.
__device__ __forceinline__ int64_t patch_of_block(int64_t n_patch, int remap)
{
  if (!remap) return blockIdx.x;
  int64_t chunk = (n_patch + 7) / 8;
  return (int64_t)(blockIdx.x % 8) * chunk + blockIdx.x / 8;
}

// GATHER = false: padded conserved patches, cell-centre inversions in phase A.
// GATHER = true : the 1,376 tile cells' primitives are read from the interiors of the patch and
//                 its 26 neighbours (outflow clamping where a face neighbour is -1), and every
//                 updated cell is inverted at the end -- its primitives and the workgroup's
//                 maximum signal speed (Eqs. 26-27) feed the next step.  PS is the storage type
//                 of those primitives (T, or float for the FP64 step of a guarded FP32 chain).
// With an FP32 bulk and the precision guard on (a.defer), a patch whose tile holds a cell with
// 1 + M^2 > kappa_max (Eq. 20) is listed in a.defer after phase A and left to the FP64 kernel.
// That kernel (T = double, PS = float in the gather layout) inverts the gathered FP64 conserved
// variables of its tile: FP32-rounded primitives would put rounding-sized errors into the
// fluxes, which the update turns into (1 + M^2) eps_32 pressure errors of the next state.
template <class T, class I, bool GATHER, int K, class PS = T>
__device__ __forceinline__ void step_patch(const StepArgs &a, Tile<T> &s, const MlpDev &mlp, const int64_t p)
{
  constexpr bool GCONS = GATHER && sizeof(T) != sizeof(PS);
  constexpr int NTT = threads_of<T>();
  constexpr bool MLP = K == KV_MLP;
  constexpr bool TOT = K == KV_TOTAL;
  static_assert(!TOT || (!GATHER && sizeof(T) == sizeof(I)), "original scheme: padded, one type");
  static_assert(K != KV_POLY || !GATHER, "polytropic EoS: padded layout");
  const auto eos = make_eos<K>(a);
  const int tid = threadIdx.x;
  const int g = a.ghost;
  const int N = 8 + 2 * g;
  const int N3 = N * N * N;
  const double *__restrict__ q = GATHER ? nullptr : a.padded + p * 5 * N3;
  int lv = a.level ? (int)a.level[p] : 0;
  lv = lv < 0 ? 0 : (lv >= a.n_level ? a.n_level - 1 : lv);     // never index past dt_lev
  const double dh = a.dh[lv];
  double dt;
  if (a.dt_lev) dt = a.dt_lev[lv];
  else dt = a.c_cfl * dh / __longlong_as_double((long long)a.smax_in[0]);
  if (GATHER && a.dt_out && p == 0 && tid < a.n_level)
    a.dt_out[tid] = a.dt_lev ? a.dt_lev[tid]
                             : a.c_cfl * a.dh[tid] / __longlong_as_double((long long)a.smax_in[0]);

  if (tid < 8) s.cnt[tid] = 0u;
  if (tid < 8) s.orf[tid >> 2][tid & 3] = 0u;
  int par = 0;
  if (GATHER && tid < 27) s.nb[tid] = a.neighbor[p * 27 + tid];
  unsigned int my_iters = 0, my_inv = 0, my_fb = 0, my_nc = 0, my_mlp = 0;
  __syncthreads();
  // learned-guess split with the input's network masks: a patch whose tile holds a cell above
  // the gate is on the list that the learned kernel steps (k_net_list applies the same rule).
  // The masks are read here and tested after phase A, so that their latency overlaps it.
  const bool prelisted = GATHER && K == KV_ANALYTIC && a.net_list && a.net_in;
  bool hit = false;
  if (prelisted && tid < 27) hit = tile_hits_mask(tid, s.nb[tid], a.n_patch, a.net_in);

  // ---------------------------------------------------------------- A: centre primitives
  bool centre_bad = false, hot = false, net = false, steep = false;
  const T kf1 = T(KAPPA_FAST - 1.0);
  unsigned int centre_unphys = 0;
  const T km1 = T(a.kappa_max - 1.0);
  // the learned-guess split's first launch (the kernel without the network) lists the patches
  // whose tile holds a cell with L above the network's gate
  const bool split = K == KV_ANALYTIC && a.net_list != nullptr && !(GATHER && a.net_in);
  for (int r0 = 0; r0 < NPC; r0 += NTT) {
    // every lane runs every round (the learned guess needs whole wavefronts); lanes past the
    // end of the list work on the first cell again and store nothing
    const int r = r0 + tid;
    const bool valid = r < NPC;
    int b = kTab.pcell[valid ? r : 0];
    int bi = b % BX, bj = (b / BX) % BX, bk = b / (BX * BX);
    // gather layout: the source patch and cell of this tile cell (outflow clamping where a
    // face neighbour is -1)
    int64_t src = 0;
    int sc = 0;
    bool okc = true;
    if (GATHER) {
      if (!valid) continue;
      int c[3] = {bi - 2, bj - 2, bk - 2};
      const int fs[3] = {1, 3, 9};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int o = c[d] < 0 ? -1 : (c[d] >= 8 ? 1 : 0);
        if (o != 0 && s.nb[13 + o * fs[d]] < 0) c[d] = o < 0 ? 0 : 7;     // outflow
      }
      int o0 = c[0] < 0 ? -1 : (c[0] >= 8 ? 1 : 0);
      int o1 = c[1] < 0 ? -1 : (c[1] >= 8 ? 1 : 0);
      int o2 = c[2] < 0 ? -1 : (c[2] >= 8 ? 1 : 0);
      src = s.nb[(o2 + 1) * 9 + (o1 + 1) * 3 + (o0 + 1)];
      okc = src >= 0 && src < a.n_patch;
      sc = ((c[2] - 8 * o2) * 8 + (c[1] - 8 * o1)) * 8 + (c[0] - 8 * o0);
    }
    if (GATHER && !GCONS) {
      const PS *__restrict__ pr = (const PS *)a.prims;
      const T nan = T(__builtin_nan(""));
      const PS *w = pr + (okc ? src : 0) * 5 * 512 + sc;
      T v0 = okc ? (T)w[0] : nan, v1 = okc ? (T)w[512] : nan, v2 = okc ? (T)w[1024] : nan,
        v3 = okc ? (T)w[1536] : nan, v4 = okc ? (T)w[2048] : nan;
      bool bad = !(v0 > T(0)) || !(v4 > T(0)) || !finiteT(v1) || !finiteT(v2) || !finiteT(v3);
      if constexpr (sizeof(T) == 4) {
        if (a.defer) hot |= kappa_above<T>(v0, v1, v2, v3, v4, km1, eos);
      } else {
        steep |= bad || kappa_above<T, typename KEos<K>::type, true>(v0, v1, v2, v3, v4, kf1, eos);
      }
      if (split) net |= !bad && (double)lhs_L_of_prim<T>(v0, v1, v2, v3, v4) > a.guess.gate;
      centre_bad |= bad;
      centre_unphys += bad;
      s.W[0][b] = v0;
      s.W[1][b] = v1;
      s.W[2][b] = v2;
      s.W[3][b] = v3;
      s.W[4][b] = v4;
    } else {
      double D, Mx, My, Mz, Et;
      if (GCONS) {
        const double nan = __builtin_nan("");
        const double *u = a.cons + (okc ? src : 0) * 5 * 512 + sc;
        D = okc ? u[0] : nan;
        Mx = okc ? u[512] : nan;
        My = okc ? u[1024] : nan;
        Mz = okc ? u[1536] : nan;
        Et = okc ? u[2048] : nan;
      } else {
        int off = ((bk + g - 2) * N + (bj + g - 2)) * N + (bi + g - 2);
        D = q[off];
        Mx = q[N3 + off];
        My = q[2 * N3 + off];
        Mz = q[3 * N3 + off];
        Et = q[4 * N3 + off];
      }
      double L;
      InvOut<I> o;
      bool adm;
      if constexpr (TOT) adm = admissible_total<I>((I)D, (I)Mx, (I)My, (I)Mz, (I)Et, L);
      else adm = admissible_adaptive<sizeof(T) == 8>(D, Mx, My, Mz, Et, DBL_EPSILON, L);
      bool consulted = false;
      unsigned int ev = 0;
      double guess = MLP ? mlp_guess(mlp, D, Mx, My, Mz, Et, (valid && adm) ? L : 0.0, consulted, ev) : -1.0;
      my_mlp += valid ? ev : 0u;
      if (!valid) continue;
      if (adm) invert_with_L<I, GuessT<T, I>, GuessT<T, I>, sizeof(T) == 8>((I)D, (I)Mx, (I)My, (I)Mz, (I)L, (I)guess, consulted, (I)StepTol<T, I>::v, 30, o, eos);
      else set_unphysical(o);
      centre_bad |= o.status == ST_UNPHYSICAL;
      centre_unphys += o.status == ST_UNPHYSICAL;
      my_iters += o.iters;
      my_inv += 1;
      my_nc += o.status == ST_NOCONV;
      s.W[0][b] = (T)o.rho;
      s.W[1][b] = (T)o.ux;
      s.W[2][b] = (T)o.uy;
      s.W[3][b] = (T)o.uz;
      s.W[4][b] = (T)o.p;
      if constexpr (sizeof(T) == 4) {
        if (a.defer) hot |= kappa_above<T>((T)o.rho, (T)o.ux, (T)o.uy, (T)o.uz, (T)o.p, km1, eos);
      } else {
        steep |= o.status == ST_UNPHYSICAL ||
                 kappa_above<T, typename KEos<K>::type, true>((T)o.rho, (T)o.ux, (T)o.uy, (T)o.uz,
                                                             (T)o.p, kf1, eos);
      }
      if (split) net |= adm && L > a.guess.gate;
    }
  }
  // the tile's flags, OR-ed over the workgroup in one pass
  const unsigned int tf = wg_or(s, (centre_bad ? 1u : 0u) | (hit ? 2u : 0u) | (steep ? 4u : 0u) |
                                       (hot ? 8u : 0u) | (net ? 16u : 0u), par);
  centre_bad = tf & 1u;
  if (prelisted && (tf & 2u)) return;    // before the guard: the learned pass guards the patch
  // FP64 bulk: the refined division upstream of the face inversions in patches whose tile holds
  // no cell with kappa > KAPPA_FAST (nor an unphysical one)
  const bool fast64 = sizeof(T) == 8 && !(tf & 4u);

  // precision guard: a patch holding a cell beyond kappa_max goes to the FP64 kernel (its
  // unphysical centre cells are counted there)
  bool deferred = false;
  if constexpr (sizeof(T) == 4) {
    if (a.defer) {
      deferred = tf & 8u;
      if (deferred) {
        centre_unphys = 0;
        if (tid == 0) a.defer[2 + atomicAdd(&a.defer[0], 1ull)] = (unsigned long long)p;
      }
    }
  }
  if (split && !deferred) {
    deferred = tf & 16u;
    if (deferred) {
      centre_unphys = 0;
      if (tid == 0) a.net_list[2 + atomicAdd(&a.net_list[0], 1ull)] = (unsigned long long)p;
    }
  }

  // this thread's interior cell for phase D (threads 512.. own none)
  const bool owner = NTT == NT || tid < NT;
  const int ci = tid & 7, cj = (tid >> 3) & 7, ck = (tid >> 6) & 7;
  const int cq = ((ck + g) * N + (cj + g)) * N + (ci + g);

  T theta = (T)a.theta;
  unsigned int retries = 0, unphys = 0;
  // the attempts, with the FP64 bulk's refined division upstream of the face inversions (FXU)
  // where the tile allows it
  auto attempts = [&](auto fx_tag) {
  constexpr bool FXU = decltype(fx_tag)::value;
  for (int attempt = 0; !deferred; ++attempt) {
    // -------------------------------------------------------------- B: half-step corrections
    const T half = T(0.5 * dt / dh);
    for (int r = tid; r < NHC; r += NTT) {
      int hb = kTab.hcell[r];
      int i = hb % HX - 1, j = (hb / HX) % HX - 1, k = hb / (HX * HX) - 1;
      int b = bidx(i, j, k);
      Prim<T> wc = load_prim(s, b);
      T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int sd = d == 0 ? 1 : (d == 1 ? BX : BX * BX);
        Prim<T> wm = load_prim(s, b - sd), wp = load_prim(s, b + sd);
        T sl[5];
        sl[0] = limited_slope<FXU>(wm.rho, wc.rho, wp.rho, theta);
        sl[1] = limited_slope<FXU>(wm.u[0], wc.u[0], wp.u[0], theta);
        sl[2] = limited_slope<FXU>(wm.u[1], wc.u[1], wp.u[1], theta);
        sl[3] = limited_slope<FXU>(wm.u[2], wc.u[2], wp.u[2], theta);
        sl[4] = limited_slope<FXU>(wm.p, wc.p, wp.p, theta);
        Prim<T> fm, fp;
        fm.rho = wc.rho - T(0.5) * sl[0];  fp.rho = wc.rho + T(0.5) * sl[0];
        fm.u[0] = wc.u[0] - T(0.5) * sl[1]; fp.u[0] = wc.u[0] + T(0.5) * sl[1];
        fm.u[1] = wc.u[1] - T(0.5) * sl[2]; fp.u[1] = wc.u[1] + T(0.5) * sl[2];
        fm.u[2] = wc.u[2] - T(0.5) * sl[3]; fp.u[2] = wc.u[2] + T(0.5) * sl[3];
        fm.p = wc.p - T(0.5) * sl[4];      fp.p = wc.p + T(0.5) * sl[4];
        Cons<T> Fm, Fp;
        if (d == 0) { Fm = state_flux<0, TOT, FXU>(fm, eos); Fp = state_flux<0, TOT, FXU>(fp, eos); }
        else if (d == 1) { Fm = state_flux<1, TOT, FXU>(fm, eos); Fp = state_flux<1, TOT, FXU>(fp, eos); }
        else { Fm = state_flux<2, TOT, FXU>(fm, eos); Fp = state_flux<2, TOT, FXU>(fp, eos); }
        acc[0] += Fp.D - Fm.D;
        acc[1] += Fp.m[0] - Fm.m[0];
        acc[2] += Fp.m[1] - Fm.m[1];
        acc[3] += Fp.m[2] - Fm.m[2];
        acc[4] += Fp.E - Fm.E;
      }
#pragma unroll
      for (int f = 0; f < 5; ++f) s.C[f][hb] = -half * acc[f];
    }
    __syncthreads();

    // -------------------------------------------------------------- C + D: fluxes, update
    bool fail = false;
    T dU[5] = {T(0), T(0), T(0), T(0), T(0)};
    constexpr int NROUND = (3 * NIF + NTT - 1) / NTT;
    int folded = 0;
#pragma unroll 1
    for (int round = 0; round < NROUND; ++round) {
      int qi = round * NTT + tid;
      if (qi < 3 * NIF) {
        // 576 = 9 x 64: the direction is uniform across each wavefront
        int d = qi / NIF;
        int r = qi - d * NIF;
        IfaceCount ic = {0, 0, 0, 0, 0, 0};
        bool ok;
        if (d == 0) ok = interface_flux<0, K, I, fast_of<T, GATHER>(), FXU>(s, r, theta, a.riemann, mlp, ic, eos);
        else if (d == 1) ok = interface_flux<1, K, I, fast_of<T, GATHER>(), FXU>(s, r, theta, a.riemann, mlp, ic, eos);
        else ok = interface_flux<2, K, I, fast_of<T, GATHER>(), FXU>(s, r, theta, a.riemann, mlp, ic, eos);
        fail |= !ok;
        my_iters += ic.iters;
        my_mlp += ic.mlp;
        my_inv += ic.inv;
        my_fb += ic.fb;
        my_nc += ic.nc;
        unphys += ic.unphys;
      }
      __syncthreads();
      // every direction this round completed: fold F_{+1/2} - F_{-1/2} into this thread's cell
      // (directions d and d + 2 share a ring slot: d is folded before d + 2 is written)
      const int done = (round + 1) * NTT / NIF < 3 ? (round + 1) * NTT / NIF : 3;
      for (; folded < done; ++folded) {
        const int d = folded;
        const int slot = d & 1;
        if (owner) {
          // this cell's lower face along d, and the step to its upper face, in the order above
          int r = d == 0 ? (ck * 8 + cj) * 9 + ci : (d == 1 ? (ck * 9 + cj) * 8 + ci : (ck * 8 + cj) * 8 + ci);
          int up = d == 0 ? 1 : (d == 1 ? 8 : 64);
#pragma unroll
          for (int f = 0; f < 5; ++f) dU[f] += s.F[slot][f][r + up] - s.F[slot][f][r];
        }
        if constexpr (!GATHER) {
          if (a.flux_out && tid < 128) write_boundary_fluxes(a.flux_out, p, d, &s.F[slot][0][0], NIF, tid);
        }
        __syncthreads();
      }
    }
    const double full = dt / dh;
    // this thread's offsets into the interior arrays, formed here: hoisted out of the retry
    // loop they would hold fifteen 64-bit per-lane addresses across the whole patch
    int lt = tid, lq = cq;
    asm volatile("" : "+v"(lt), "+v"(lq));
    double un[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double Lo = 0.0;
    bool ok_out = true;
    if (owner) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        double u0 = GATHER ? a.cons[(p * 5 + f) * 512 + lt] : q[f * N3 + lq];
        un[f] = u0 - full * (double)dU[f];
      }
      if constexpr (TOT) ok_out = admissible_total<I>((I)un[0], (I)un[1], (I)un[2], (I)un[3], (I)un[4], Lo);
      else ok_out = admissible_adaptive<fast_of<T, GATHER>()>(un[0], un[1], un[2], un[3], un[4], DBL_EPSILON, Lo);
    }
    fail |= !ok_out;
    fail = wg_or(s, fail ? 1u : 0u, par) != 0u;
    bool last = !fail || centre_bad || theta == T(0);
    if (last) {
      if (owner) {
        double *o = a.out + p * 5 * 512 + lt;
#pragma unroll
        for (int f = 0; f < 5; ++f) o[f * 512] = un[f];
        unphys += !ok_out;
      }
      if (GATHER) {
       double sm = 0.0;
       if (owner) {                  // whole wavefronts: the network evaluates 64 lanes at once
        // the updated cell's primitives and signal speed, for the next step
        InvOut<I> w;
        bool consulted = false;
        double guess = -1.0;
        if (MLP) {
          // the network needs most of the registers: park the updated state in the (now unused)
          // primitive tile while it runs instead of spilling it
          consulted = ok_out && Lo > mlp.gate;
          float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
          if (__any(consulted)) mlp_features(mlp.features, un[0], un[1], un[2], un[3], un[4], Lo, f0, f1, f2);
          double *park = reinterpret_cast<double *>(&s.W[0][0]) + tid;
#pragma unroll
          for (int f = 0; f < 5; ++f) park[f * NT] = un[f];
          asm volatile("" ::: "memory");
          guess = mlp_guess_f(mlp, f0, f1, f2, consulted, my_mlp);
          asm volatile("" ::: "memory");
#pragma unroll
          for (int f = 0; f < 5; ++f) un[f] = park[f * NT];
        }
        // as in invert_face: the guess-free inversion unless a lane of the wavefront has a guess
        const bool any_guess = MLP && __any(consulted);
        if (ok_out) {
          if (any_guess)
            invert_with_L<I, GuessT<T, I>, GuessT<T, I>, fast_of<T, GATHER>()>((I)un[0], (I)un[1], (I)un[2], (I)un[3], (I)Lo, (I)guess,
                                                         consulted, (I)StepTol<T, I>::v, 30, w);
          else
            invert_with_L<I, GuessT<T, I>, GuessT<T, I>, fast_of<T, GATHER>()>((I)un[0], (I)un[1], (I)un[2], (I)un[3], (I)Lo, (I)-1.0,
                                                         false, (I)StepTol<T, I>::v, 30, w);
        } else set_unphysical(w);
        my_iters += w.iters;
        my_inv += 1;
        my_nc += w.status == ST_NOCONV;
        PS *po = (PS *)a.prims_out + p * 5 * 512 + lt;
        po[0] = (PS)(T)w.rho;
        po[512] = (PS)(T)w.ux;
        po[1024] = (PS)(T)w.uy;
        po[1536] = (PS)(T)w.uz;
        po[2048] = (PS)(T)w.p;
        if constexpr (sizeof(PS) == 4) {
          if (ok_out) sm = (double)signal_smax_t<float>((float)(T)w.rho, (float)(T)w.ux, (float)(T)w.uy, (float)(T)w.uz, (float)(T)w.p);
        } else {
          if (ok_out) sm = signal_smax((double)w.rho, (double)w.ux, (double)w.uy, (double)w.uz, (double)w.p);
        }
       }
        if (a.net_out) {
          // the updated state's network mask: L of the output check against the gate
          const unsigned int m = wave_or_hi(owner && ok_out && Lo > a.net_gate ? region_mask(ci, cj, ck) : 0u);
          if ((tid & 63) == 63 && m) atomicOr(&s.cnt[7], m);
          __syncthreads();
          if (tid == 0) a.net_out[p] = s.cnt[7];
        }
        sm = wave_max_hi(sm);
        if ((tid & 63) == 63) s.red[tid >> 6] = sm;
        __syncthreads();
        if (tid == 0) {
          double m = s.red[0];
#pragma unroll
          for (int w8 = 1; w8 < NTT / 64; ++w8) m = fmax(m, s.red[w8]);
          atomicMax(a.smax_out, (unsigned long long)__double_as_longlong(m));
        }
      }
      break;
    }
    ++retries;
    unphys = 0;
    theta = attempt < a.max_retry ? theta * T(0.75) : T(0);
  }
  };
  if constexpr (sizeof(T) == 8) {
    if (fast64) attempts(std::true_type{});
    else attempts(std::false_type{});
  } else {
    attempts(std::false_type{});
  }

  // ---------------------------------------------------------------- counters
  if (a.stats) {
    const unsigned int c0 = wave_sum_hi(unphys + centre_unphys), c1 = wave_sum_hi(my_fb),
                       c2 = wave_sum_hi(my_nc), c3 = wave_sum_hi(my_iters), c4 = wave_sum_hi(my_inv),
                       c5 = MLP ? wave_sum_hi(my_mlp) : 0u;
    if ((tid & 63) == 63) {
      atomicAdd(&s.cnt[0], c0);
      atomicAdd(&s.cnt[1], c1);
      atomicAdd(&s.cnt[2], c2);
      atomicAdd(&s.cnt[3], c3);
      atomicAdd(&s.cnt[4], c4);
      if (MLP) atomicAdd(&s.cnt[5], c5);
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long *st = (unsigned long long *)a.stats;
      if (s.cnt[0]) atomicAdd(&st[0], (unsigned long long)s.cnt[0]);
      if (s.cnt[1]) atomicAdd(&st[1], (unsigned long long)s.cnt[1]);
      if (s.cnt[2]) atomicAdd(&st[2], (unsigned long long)s.cnt[2]);
      atomicAdd(&st[3], (unsigned long long)s.cnt[3]);
      atomicAdd(&st[4], (unsigned long long)s.cnt[4]);
      if (MLP && s.cnt[5]) atomicAdd(&st[6], (unsigned long long)s.cnt[5]);
      if (retries) atomicAdd(&st[5], (unsigned long long)retries);
    }
  }
}

// One patch per workgroup (a.queue == NULL), or a persistent grid of a.groups workgroups that
// claim a.chunk patches at a time.  The persistent schedule keeps one queue counter per XCD over
// that XCD's contiguous range of patches (the same ranges as the one-per-patch mapping); a
// workgroup drains its own XCD's range first and then helps the others in turn, so every
// workgroup leaves the loop once all eight ranges are exhausted.
template <class T, class I, bool GATHER, int K>
__device__ __forceinline__ void step_body(const StepArgs &a)
{
  const MlpDev mlp = a.guess.dev();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Tile<T> &s = *reinterpret_cast<Tile<T> *>(smem_raw);
  if (!a.queue) {
    const int64_t p = patch_of_block(a.n_patch, a.xcd_remap);
    if (p < a.n_patch) step_patch<T, I, GATHER, K>(a, s, mlp, p);     // uniform per workgroup
    return;
  }
  const int64_t range = (a.n_patch + 7) / 8;
  const int home = blockIdx.x % 8;
  for (int k = 0; k < 8; ++k) {
    const int x = (home + k) % 8;
    const int64_t lo = x * range;
    const int64_t hi = lo + range < a.n_patch ? lo + range : a.n_patch;
    for (;;) {
      __syncthreads();                               // the tile and s.claim are free again
      if (threadIdx.x == 0) s.claim = atomicAdd(&a.queue[x], (unsigned long long)a.chunk);
      __syncthreads();
      // every thread read the same claim: make that visible to the compiler (scalar registers)
      const int64_t p0 = lo + (int64_t)__builtin_amdgcn_readfirstlane((int)s.claim);
      if (p0 >= hi) break;                           // uniform: every thread read the same claim
      const int64_t p1 = p0 + a.chunk < hi ? p0 + a.chunk : hi;
      for (int64_t p = p0; p < p1; ++p) {
        step_patch<T, I, GATHER, K>(a, s, mlp, p);
        __syncthreads();
      }
    }
  }
}

template <class T, class I, bool GATHER, int K>
__global__ void __launch_bounds__(threads_of<T>()) k_step(StepArgs a)
{
  step_body<T, I, GATHER, K>(a);
}

// The same kernel compiled for at most 128 VGPRs (four waves per SIMD), so that two 512-thread
// workgroups share a CU when their LDS tiles fit (the mixed-precision tile takes 78 KB); the
// compiler then keeps a few values of the per-patch setup in scratch instead of registers.
template <class T, class I, bool GATHER, int K>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) k_step_occ2(StepArgs a)
{
  step_body<T, I, GATHER, K>(a);
}

// A launch over a list of patches written by a previous launch on the stream (a.list: [0] count,
// [1] claim counter, [2..] indices): a persistent grid claims them one at a time; every workgroup
// leaves once the list is exhausted.  Each listed patch adds 1 to word a.list_counter of the
// step counters.  Serves the precision guard's FP64 pass (T = I = double; PS, the storage type
// of the gather layout's primitives, float) and the learned-guess split's network pass.
template <class T, class I, bool GATHER, int K, class PS>
__device__ __forceinline__ void listed_body(const StepArgs &a)
{
  const MlpDev mlp = a.guess.dev();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Tile<T> &s = *reinterpret_cast<Tile<T> *>(smem_raw);
  const unsigned long long n = a.list[0];
  for (;;) {
    __syncthreads();                                 // the tile and s.claim are free again
    if (threadIdx.x == 0) s.claim = atomicAdd(&a.list[1], 1ull);
    __syncthreads();
    const unsigned long long i = s.claim;
    if (i >= n) break;                               // uniform: every thread read the same claim
    step_patch<T, I, GATHER, K, PS>(a, s, mlp, (int64_t)a.list[2 + i]);
    if (a.stats && threadIdx.x == 0)
      atomicAdd((unsigned long long *)a.stats + a.list_counter, 1ull);
  }
}

template <class T, class I, bool GATHER, int K, class PS>
__global__ void __launch_bounds__(threads_of<T>()) k_step_listed(StepArgs a)
{
  listed_body<T, I, GATHER, K, PS>(a);
}

// The same within the two-workgroup register budget (FP32 bulk): run beside the kernel without the
// network, a workgroup then fits into the slot one of that kernel's workgroups leaves, instead of
// waiting for a CU whose workgroups have all left -- which, while that kernel still has patches to
// hand out, does not happen.
template <class T, class I, bool GATHER, int K, class PS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) k_step_listed_occ2(StepArgs a)
{
  listed_body<T, I, GATHER, K, PS>(a);
}

// The counters a step starts from: the two lists' count and claim words, the output S_max and
// the n_mask output network masks (NULL pointers skipped).
__global__ void k_step_prologue(unsigned long long *defer, unsigned long long *net_list,
                                unsigned long long *smax_out, unsigned int *net_out,
                                int64_t n_mask)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (net_out && i < n_mask) net_out[i] = 0u;
  if (i < 2) {
    if (defer) defer[i] = 0ull;
    if (net_list) net_list[i] = 0ull;
  }
  if (i == 0 && smax_out) smax_out[0] = 0ull;
}

// The learned-guess split's list from the input's network masks: every patch whose tile holds a
// cell above the gate, in no particular order.
__global__ void __launch_bounds__(256) k_net_list(int64_t n_patch, const int32_t *__restrict__ neighbor,
                                                  const unsigned int *__restrict__ mask,
                                                  unsigned long long *list)
{
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_patch) return;
  bool hit = false;
  for (int k = 0; k < 27; ++k) hit |= tile_hits_mask(k, neighbor[p * 27 + k], n_patch, mask);
  if (hit) list[2 + atomicAdd(&list[0], 1ull)] = (unsigned long long)p;
}

// Inversion of every interior cell into the bulk type, with the maximum signal speed (the
// entry state of the gather-mode step).  Same inversion and tolerance as the step's own output
// inversion, so a chain of steps sees identically computed primitives throughout.
template <class T, class I, bool MLP>
__global__ void __launch_bounds__(256) k_grid_prims(int64_t n_patch, const double *__restrict__ cons,
                                                    T *__restrict__ prims,
                                                    unsigned long long *__restrict__ smax_bits,
                                                    unsigned int *__restrict__ net_mask,
                                                    double net_gate, MlpDev mlp)
{
  __shared__ double red[4];
  const int64_t total = n_patch * 512;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double vmax = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += stride) {
    const int64_t t = base + threadIdx.x;       // total is a multiple of 512: always in range
    int64_t pp = t >> 9;
    int c = (int)(t & 511);
    const double *u = cons + pp * 5 * 512 + c;
    double L;
    InvOut<I> w;
    // the step's output check and L (adaptive with an FP32 bulk), so that both give the same bits
    bool ok;
    ok = admissible_adaptive<true>(u[0], u[512], u[1024], u[1536], u[2048], DBL_EPSILON, L);
    bool consulted = false;
    unsigned int evals = 0;
    double guess = MLP ? mlp_guess(mlp, u[0], u[512], u[1024], u[1536], u[2048], ok ? L : 0.0, consulted, evals) : -1.0;
    if (ok)
      invert_with_L<I, GuessT<T, I>, GuessT<T, I>, true>((I)u[0], (I)u[512], (I)u[1024], (I)u[1536], (I)L, (I)guess, consulted,
                       (I)StepTol<T, I>::v, 30, w);
    else set_unphysical(w);
    // the state's network mask (every wavefront's cells lie in one patch)
    if (net_mask) {
      const unsigned int m = wave_or_hi(ok && L > net_gate ? region_mask(c & 7, (c >> 3) & 7, c >> 6) : 0u);
      if ((threadIdx.x & 63) == 63 && m) atomicOr(&net_mask[pp], m);
    }
    T *po = prims + pp * 5 * 512 + c;
    po[0] = (T)w.rho;
    po[512] = (T)w.ux;
    po[1024] = (T)w.uy;
    po[1536] = (T)w.uz;
    po[2048] = (T)w.p;
    // S_max as the step's own output does it (FP32 from the stored primitives with an FP32 bulk)
    if constexpr (sizeof(T) == 4) {
      if (ok) vmax = fmax(vmax, (double)signal_smax_t<T>((T)w.rho, (T)w.ux, (T)w.uy, (T)w.uz, (T)w.p));
    } else {
      if (ok) vmax = fmax(vmax, signal_smax((double)w.rho, (double)w.ux, (double)w.uy, (double)w.uz, (double)w.p));
    }
  }
  vmax = wave_max_hi(vmax);
  if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = vmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(smax_bits, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void k_zero_queue(unsigned long long *q)
{
  if (threadIdx.x < SRHD_QUEUE_WORDS) q[threadIdx.x] = 0ull;
}

// Kernel of a (precision, layout, guess, register budget) combination.  The two-workgroup
// variant exists for the FP32-bulk kernels only: the FP64 tile fills the LDS of a CU by itself.
// With the learned guess it spills around the network's evaluation, which runs only in
// wavefronts that consult it.
template <class T, class I, bool GATHER, int K>
const void *step_kernel(bool occ2)
{
  if constexpr (sizeof(T) == 4)
    if (occ2) return (const void *)k_step_occ2<T, I, GATHER, K>;
  return (const void *)k_step<T, I, GATHER, K>;
}

template <class T, class I, bool GATHER, int K>
int occupancy_k(bool occ2)
{
  int n = 0;
  const size_t bytes = sizeof(Tile<T>);
  const void *fn = step_kernel<T, I, GATHER, K>(occ2);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads_of<T>(), bytes) != hipSuccess) return 0;
  return n;
}

// A persistent launch over a list of patches (k_step_listed): as many workgroups as fit on the
// device at once (the FP64 tile fills a CU's LDS; two FP32-bulk tiles fit), at most the patches.
// occ2 (FP32 bulk only): the kernel of the two-workgroup register budget.
template <class T, class I, bool GATHER, int K, class PS>
hipError_t launch_listed(const StepArgs &a, unsigned long long *list, int counter, hipStream_t st,
                         bool occ2 = false)
{
  const size_t bytes = sizeof(Tile<T>);
  const void *fn = (const void *)k_step_listed<T, I, GATHER, K, PS>;
  if constexpr (sizeof(T) == 4) {
    if (occ2) fn = (const void *)k_step_listed_occ2<T, I, GATHER, K, PS>;
  } else {
    occ2 = false;
  }
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  int dev = 0, cus = 0, per_cu = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads_of<T>(), bytes);
  if (e != hipSuccess) return e;
  int64_t groups = (int64_t)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  if (groups > a.n_patch) groups = a.n_patch;
  StepArgs b = a;
  b.list = list;
  b.list_counter = counter;
  b.queue = nullptr;
  b.net_list = nullptr;
  if constexpr (sizeof(T) == 4) {
    if (occ2) {
      hipLaunchKernelGGL((k_step_listed_occ2<T, I, GATHER, K, PS>), dim3((unsigned)groups), dim3(NT), bytes, st, b);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_step_listed<T, I, GATHER, K, PS>), dim3((unsigned)groups), dim3(threads_of<T>()), bytes, st, b);
  return hipGetLastError();
}

// The FP64 step of the patches a guarded FP32-bulk step listed.
template <bool GATHER, int K>
hipError_t launch_step_listed(const StepArgs &a, hipStream_t st)
{
  constexpr int KD = K == KV_MLP ? KV_ANALYTIC : K;
  StepArgs b = a;
  b.defer = nullptr;
  return launch_listed<double, double, GATHER, KD, float>(b, a.defer, 8, st);
}

// Zeroes, in one launch, what the step's kernels count from: the guard's and the split's list
// words, and in the gather layout the output S_max and network bits.
template <class T, bool GATHER>
hipError_t launch_prologue(const StepArgs &a, hipStream_t st)
{
  const bool guard = sizeof(T) == 4 && a.defer != nullptr;
  const int64_t nw = GATHER && a.net_out ? a.n_patch : 0;
  const int64_t n = nw > 2 ? nw : 2;
  hipLaunchKernelGGL(k_step_prologue, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     guard ? a.defer : nullptr, a.net_list, GATHER ? a.smax_out : nullptr,
                     GATHER ? a.net_out : nullptr, nw);
  return hipGetLastError();
}

// The step kernel over every patch (one workgroup per patch, or the persistent grid).
template <class T, class I, bool GATHER, int K>
hipError_t launch_main(const StepArgs &a, hipStream_t st)
{
  const size_t bytes = sizeof(Tile<T>);
  const bool occ2 = a.occ2 && sizeof(T) == 4;
  hipError_t e = hipFuncSetAttribute(step_kernel<T, I, GATHER, K>(occ2),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  int64_t blocks;
  if (a.queue) {
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, st, a.queue);
    blocks = a.groups;
  } else {
    blocks = a.xcd_remap ? 8 * ((a.n_patch + 7) / 8) : a.n_patch;
  }
  if constexpr (sizeof(T) == 4) {
    if (occ2) hipLaunchKernelGGL((k_step_occ2<T, I, GATHER, K>), dim3((unsigned)blocks), dim3(NT), bytes, st, a);
    else hipLaunchKernelGGL((k_step<T, I, GATHER, K>), dim3((unsigned)blocks), dim3(NT), bytes, st, a);
  } else {
    hipLaunchKernelGGL((k_step<T, I, GATHER, K>), dim3((unsigned)blocks), dim3(threads_of<T>()), bytes, st, a);
  }
  return hipGetLastError();
}

template <class T, class I, bool GATHER, int K>
hipError_t launch_step_k(const StepArgs &a, hipStream_t st)
{
  hipError_t e = launch_prologue<T, GATHER>(a, st);
  if (e == hipSuccess) e = launch_main<T, I, GATHER, K>(a, st);
  if (e != hipSuccess || !(sizeof(T) == 4 && a.defer)) return e;
  return launch_step_listed<GATHER, K>(a, st);
}

// The learned-guess split with the input's network masks (gather layout): the list is formed
// before the step, and the learned kernel steps the listed patches on the side stream while the
// kernel without the network steps the others on `st`; the guard's FP64 pass, over the patches
// either of them deferred, follows the join.
template <class T, class I>
hipError_t launch_split_concurrent(const StepArgs &a, hipStream_t st)
{
  hipError_t e = launch_prologue<T, true>(a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_net_list, dim3((unsigned)((a.n_patch + 255) / 256)), dim3(256), 0, st,
                     a.n_patch, a.neighbor, a.net_in, a.net_list);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  SideStream side;
  if ((e = side_stream(side)) != hipSuccess) return e;
  std::lock_guard<std::mutex> hold(*side.lock);
  if ((e = hipEventRecord(side.fork, st)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(side.stream, side.fork, 0)) != hipSuccess) return e;
  // the learned kernel applies the precision guard to its own patches (a.defer kept)
  hipError_t el = launch_listed<T, I, true, KV_MLP, T>(a, a.net_list, 9, side.stream, true);
  hipError_t ej = hipEventRecord(side.join, side.stream);
  hipError_t em = el == hipSuccess ? launch_main<T, I, true, KV_ANALYTIC>(a, st) : hipSuccess;
  if (ej == hipSuccess) ej = hipStreamWaitEvent(st, side.join, 0);
  if (el != hipSuccess) return el;
  if (ej != hipSuccess) return ej;
  if (em != hipSuccess) return em;
  if (sizeof(T) == 4 && a.defer) return launch_step_listed<true, KV_ANALYTIC>(a, st);
  return hipSuccess;
}

// The original scheme exists where it can run: padded layout, bulk type = inversion type; the
// polytropic EoS for the padded layout.
template <class T, class I, bool GATHER>
constexpr bool has_total() { return !GATHER && sizeof(T) == sizeof(I); }

template <class T, class I, bool GATHER>
hipError_t launch_step_t(const StepArgs &a, hipStream_t st)
{
  if (a.energy == SRHD_ENERGY_TOTAL) {
    if constexpr (has_total<T, I, GATHER>()) return launch_step_k<T, I, GATHER, KV_TOTAL>(a, st);
    else return hipErrorInvalidValue;
  }
  if (a.eos_k > 0.0) {
    if constexpr (!GATHER) return launch_step_k<T, I, GATHER, KV_POLY>(a, st);
    else return hipErrorInvalidValue;
  }
  if (a.guess.kind != SRHD_GUESS_MLP) {
    StepArgs b = a;
    b.net_list = nullptr;
    return launch_step_k<T, I, GATHER, KV_ANALYTIC>(b, st);
  }
  if (!a.net_list) return launch_step_k<T, I, GATHER, KV_MLP>(a, st);
  if constexpr (GATHER) {
    if (a.net_in) return launch_split_concurrent<T, I>(a, st);
  }
  // learned-guess split: the kernel without the network steps every patch and lists those whose
  // tile consults the network; then the learned kernel steps the listed ones
  hipError_t e = launch_step_k<T, I, GATHER, KV_ANALYTIC>(a, st);
  if (e != hipSuccess) return e;
  StepArgs b = a;
  b.defer = nullptr;
  return launch_listed<T, I, GATHER, KV_MLP, T>(b, a.net_list, 9, st);
}

template <class T, class I, bool GATHER>
int occupancy_g(int kind, bool occ2)
{
  if (kind == KV_TOTAL) {
    if constexpr (has_total<T, I, GATHER>()) return occupancy_k<T, I, GATHER, KV_TOTAL>(occ2);
    else return 0;
  }
  if (kind == KV_POLY) {
    if constexpr (!GATHER) return occupancy_k<T, I, GATHER, KV_POLY>(occ2);
    else return 0;
  }
  return kind == KV_MLP ? occupancy_k<T, I, GATHER, KV_MLP>(occ2) : occupancy_k<T, I, GATHER, KV_ANALYTIC>(occ2);
}

// kind: 0 analytic guess, 1 learned guess, 2 original scheme, 3 polytropic EoS
template <class T, class I>
int occupancy_ti(bool gather, int kind, bool occ2)
{
  return gather ? occupancy_g<T, I, true>(kind, occ2) : occupancy_g<T, I, false>(kind, occ2);
}

template <class T, class I>
void launch_grid_prims_ti(int64_t n_patch, const double *cons, void *prims,
                          unsigned long long *smax_bits, unsigned int *net_mask,
                          double net_gate, const MlpDev &m, bool mlp, int blocks, hipStream_t st)
{
  if (mlp)
    hipLaunchKernelGGL((k_grid_prims<T, I, true>), dim3(blocks), dim3(256), 0, st, n_patch, cons,
                       (T *)prims, smax_bits, net_mask, net_gate, m);
  else
    hipLaunchKernelGGL((k_grid_prims<T, I, false>), dim3(blocks), dim3(256), 0, st, n_patch, cons,
                       (T *)prims, smax_bits, net_mask, net_gate, m);
}

// Entry points of one precision mode (bulk type T, inversion type I); each mode is compiled in
// a translation unit of its own.
template <class T, class I>
hipError_t step_launch_ti(const StepArgs &a, bool gather, hipStream_t st)
{
  if (gather) {
    if (a.n_patch == 0) return launch_prologue<T, true>(a, st);
    return launch_step_t<T, I, true>(a, st);
  }
  if (a.n_patch == 0) return hipSuccess;
  return launch_step_t<T, I, false>(a, st);
}

// net_mask (may be NULL): the state's network masks, from the cells with L > gate of a learned
// guess (all zero with the analytic guess).
template <class T, class I>
hipError_t grid_prims_ti(int64_t n_patch, const double *cons, void *prims,
                         unsigned long long *smax_bits, unsigned int *net_mask,
                         const GuessArgs &g, hipStream_t st)
{
  const int64_t nw = net_mask ? n_patch : 0;
  const int64_t n = nw > 2 ? nw : 2;
  hipLaunchKernelGGL(k_step_prologue, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (unsigned long long *)nullptr, (unsigned long long *)nullptr, smax_bits,
                     net_mask, nw);
  if (n_patch > 0) {
    const int64_t total = n_patch * 512;
    int blocks = (int)((total + 511) / 512);
    if (blocks > 256 * 64) blocks = 256 * 64;
    const bool mlp = g.kind == SRHD_GUESS_MLP;
    launch_grid_prims_ti<T, I>(n_patch, cons, prims, smax_bits, net_mask,
                               mlp ? g.gate : __builtin_huge_val(), g.dev(), mlp, blocks, st);
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace srhd
