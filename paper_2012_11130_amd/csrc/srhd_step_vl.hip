// srhd_step_vl.hip -- the VL predictor-corrector step (the paper's second integrator, Sec. 3.1;
// Falle 1991, van Leer 2006) on 8^3 patches, one 512-thread workgroup per patch:
//
//   A. centre primitives of the 2,112 cells the predictor reads: the 12^3 box [-2, 10)^3 (as far
//      as it is needed) and the six 8x8 slabs one layer further out (coordinate -3 or 10 along
//      one axis) -- inverted from padded conserved patches, or, in the gather layout, read from
//      the primitives of the patch and its 26 neighbours that the previous step (or
//      srhd_grid_prims) stored                                                -> LDS W
//   P. predictor, one direction at a time: first-order fluxes F_d(W_left, W_right) with the
//      cell-centre primitives as face states on the 1,408 faces the half-step cells need
//      -> LDS buffer; each of the 1,280 half-step cells (coordinate d in [-2, 10), the other
//      two inside the patch, for some d) adds its two face differences to registers.  Then
//      U* = U^n - (dt / 2dh) sum_d dF, inverted to W*, written over W^n at those cells.
//   C. corrector: for the 3 x 576 interfaces, PLM face states of W* (W* -/+ slope/2 on the two
//      sides), their conserved variables and the HLLC / HLLE flux -> LDS ring, folded into
//      each interior cell as in the MUSCL-Hancock kernel.
//   D. U^{n+1} = U^n - (dt/dh) sum_d (F_{+1/2} - F_{-1/2}) with the Eq. 30 check; in the gather
//      layout each updated cell is then inverted, and its primitives and the workgroup's maximum
//      signal speed (Eqs. 26-27) feed the next step.
// The face states of C are primitives (no inversion); the limiter keeps rho and p between
// neighbouring values, so only an output cell can fail: then C-D are redone with
// theta *= 0.75 (max_retry times) and theta = 0 (Sec. 3.4).  A predictor state that fails the
// inversion (no limiter acts on it) is replaced by the cell's state at t^n.  With theta = 0 the
// half step is dropped everywhere (W* = W^n): the first-order Godunov step, as MUSCL-Hancock is
// with theta = 0 -- so the retry's last attempt restores W^n at the half-step cells.
#include "srhd_step_impl.hpp"

namespace srhd {
namespace {

constexpr int NVH = 1280;                // half-step (predictor) cells
constexpr int NVF = 1408;                // predictor faces per direction
constexpr int NVS = 384;                 // slab cells (six 8 x 8 slabs)
constexpr int NVW = NB + NVS;            // LDS primitive slots: 12^3 box + slabs

constexpr bool in_range(int v, int lo, int hi) { return v >= lo && v < hi; }

// Threads of a workgroup: 512 with an FP32 bulk (one per interior cell); 768 with the FP64 bulk,
// whose 141 KB tile leaves one workgroup per CU -- three wavefronts per SIMD instead of two to
// hide the FP64 latency (threads 512.. own no interior cell).
template <class T> constexpr int vl_threads() { return sizeof(T) == 8 ? 768 : 512; }

// Cells whose half-step primitives the corrector reads.
constexpr bool vl_half(int i, int j, int k)
{
  int c[3] = {i, j, k};
  int out = 0;
  for (int d = 0; d < 3; ++d) {
    if (in_range(c[d], 0, 8)) continue;
    if (in_range(c[d], -2, 10)) ++out;
    else return false;
  }
  return out <= 1;
}

// Cells whose centre primitives the predictor reads: the half-step cells and their neighbours.
constexpr bool vl_prim(int i, int j, int k)
{
  return vl_half(i, j, k) || vl_half(i - 1, j, k) || vl_half(i + 1, j, k) || vl_half(i, j - 1, k) ||
         vl_half(i, j + 1, k) || vl_half(i, j, k - 1) || vl_half(i, j, k + 1);
}

// Predictor face along d whose right cell is (i, j, k): needed when either side is a half-step cell.
constexpr bool vl_face(int d, int i, int j, int k)
{
  return vl_half(i, j, k) || vl_half(i - (d == 0), j - (d == 1), k - (d == 2));
}

// LDS slot of a cell the predictor reads: the 12^3 box, or a slab (coordinate -3 or 10 along one
// axis, the other two in [0, 8)).
constexpr int vslot(int i, int j, int k)
{
  if (in_range(i, -2, 10) && in_range(j, -2, 10) && in_range(k, -2, 10))
    return ((k + 2) * BX + (j + 2)) * BX + (i + 2);
  const int c[3] = {i, j, k};
  int d = in_range(i, -2, 10) ? (in_range(j, -2, 10) ? 2 : 1) : 0;
  const int side = c[d] < 0 ? 0 : 1;
  const int a = d == 0 ? j : i, b = d == 2 ? j : k;
  return NB + (2 * d + side) * 64 + b * 8 + a;
}

// Packed cell coordinates: 5 bits per axis, offset by 3.
constexpr uint16_t pack(int i, int j, int k) { return (uint16_t)((i + 3) | ((j + 3) << 5) | ((k + 3) << 10)); }
__device__ __forceinline__ void unpack(uint32_t v, int &i, int &j, int &k)
{
  i = (int)(v & 31) - 3;
  j = (int)((v >> 5) & 31) - 3;
  k = (int)((v >> 10) & 31) - 3;
}

struct VlTables {
  uint16_t pcell[NVW];           // cells inverted in A (packed), count np
  uint16_t hcell[NVH];           // half-step cells (packed)
  uint16_t face[3][NVF];         // predictor faces per direction: right cell (packed)
  uint16_t hface[3][NVH][2];     // per half-step cell and direction: its minus and plus face
  int np;
};

constexpr VlTables make_vl_tables()
{
  VlTables t{};
  int16_t fidx[3][14][14][14] = {};        // face index by direction and right cell
  int np = 0, nh = 0, nf[3] = {0, 0, 0};
  for (int k = -3; k < 11; ++k)
    for (int j = -3; j < 11; ++j)
      for (int i = -3; i < 11; ++i) {
        if (vl_prim(i, j, k)) t.pcell[np++] = pack(i, j, k);
        if (vl_half(i, j, k)) t.hcell[nh++] = pack(i, j, k);
        for (int d = 0; d < 3; ++d) {
          fidx[d][k + 3][j + 3][i + 3] = -1;
          if (vl_face(d, i, j, k)) {
            fidx[d][k + 3][j + 3][i + 3] = (int16_t)nf[d];
            t.face[d][nf[d]++] = pack(i, j, k);
          }
        }
      }
  t.np = np;
  for (int h = 0; h < nh; ++h) {
    const int i = (t.hcell[h] & 31) - 3, j = ((t.hcell[h] >> 5) & 31) - 3, k = ((t.hcell[h] >> 10) & 31) - 3;
    for (int d = 0; d < 3; ++d) {
      // the minus face's right cell is the cell itself, the plus face's the next cell along d
      t.hface[d][h][0] = (uint16_t)fidx[d][k + 3][j + 3][i + 3];
      t.hface[d][h][1] = (uint16_t)fidx[d][k + 3 + (d == 2)][j + 3 + (d == 1)][i + 3 + (d == 0)];
    }
  }
  return t;
}

constexpr VlTables kVlInit = make_vl_tables();

constexpr bool vl_tables_ok(const VlTables &t)
{
  int nh = 0, nf = 0;
  for (int k = -3; k < 11; ++k)
    for (int j = -3; j < 11; ++j)
      for (int i = -3; i < 11; ++i) {
        nh += vl_half(i, j, k);
        nf += vl_face(0, i, j, k);
        if (vl_prim(i, j, k) && (vslot(i, j, k) < 0 || vslot(i, j, k) >= NVW)) return false;
        // every cell the predictor reads outside the box lies in a slab
        if (vl_prim(i, j, k) && !(in_range(i, -2, 10) && in_range(j, -2, 10) && in_range(k, -2, 10))) {
          int out = !in_range(i, 0, 8) + !in_range(j, 0, 8) + !in_range(k, 0, 8);
          if (out != 1) return false;
        }
      }
  if (nh != NVH || nf != NVF || t.np > NVW) return false;
  for (int d = 0; d < 3; ++d)
    for (int h = 0; h < NVH; ++h)
      if (t.hface[d][h][0] >= NVF || t.hface[d][h][1] >= NVF) return false;
  return true;
}
static_assert(vl_tables_ok(kVlInit), "VL cell and face tables");

__constant__ VlTables kVl = kVlInit;

template <class T>
struct VlTile {
  T W[5][NVW];                   // centre primitives, then W* at the half-step cells
  T B[5 * NVF];                  // predictor fluxes of one direction / corrector flux ring
  double red[16];                // per-wavefront maxima
  unsigned int cnt[8];
  unsigned long long claim;
  unsigned int orf[2][4];        // workgroup OR (wg_or)
  int nb[28];                    // neighbour table row (gather layout)
};
static_assert(5 * NVF >= 2 * 5 * NIF, "the corrector's ring fits in the predictor buffer");

template <class T>
__device__ __forceinline__ Prim<T> vload(const VlTile<T> &s, int b)
{
  Prim<T> w;
  w.rho = s.W[0][b];
  w.u[0] = s.W[1][b];
  w.u[1] = s.W[2][b];
  w.u[2] = s.W[3][b];
  w.p = s.W[4][b];
  return w;
}

// FX: the refined division and square roots of the FP64 bulk (dvx, sqx).  The corrector's fluxes
// are not inverted again and always take them; the predictor's are (U* -> W*), and an inversion
// turns a changed rounding of its input into up to kappa (Eq. 20) times that change, so the
// predictor takes them only in a patch whose tile has kappa <= KAPPA_FAST everywhere (as the
// MUSCL-Hancock FP64 step gates its upstream arithmetic).
template <int d, bool FX, class T>
__device__ __forceinline__ Cons<T> riemann(int solver, const Prim<T> &wl, const Prim<T> &wr)
{
  const Cons<T> ul = prim2cons<FX>(wl), ur = prim2cons<FX>(wr);
  const FaceAux<T> xl = face_aux<FX>(wl), xr = face_aux<FX>(wr);
  return solver == SRHD_HLLE ? hlle<d, false, FX>(wl, wr, ul, ur, xl, xr)
                             : hllc<d, false, FX>(wl, wr, ul, ur, xl, xr);
}

// Eq. 30 and L of an FP64 state: the adaptive sum of the exact products (every caller runs whole
// wavefronts), as in the MUSCL-Hancock step.
template <class T>
__device__ __forceinline__ bool vl_admissible(double D, double Mx, double My, double Mz, double Et, double &L)
{
  return admissible_adaptive<true>(D, Mx, My, Mz, Et, DBL_EPSILON, L);
}

// Gather layout: the patch and cell holding tile cell (i, j, k), coordinates in [-3, 11).  Along
// an axis whose face neighbour is missing (< 0) the coordinate is clamped to the patch's own
// boundary layer: the outflow (zero-gradient) copy of the padded ghost fill.  False when the
// neighbour holding the cell is missing or out of range.
__device__ __forceinline__ bool gather_cell(const int *nb, int64_t n_patch, int i, int j, int k,
                                            int64_t &src, int &sc)
{
  int c[3] = {i, j, k};
  const int fs[3] = {1, 3, 9};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int o = c[d] < 0 ? -1 : (c[d] >= 8 ? 1 : 0);
    if (o != 0 && nb[13 + o * fs[d]] < 0) c[d] = o < 0 ? 0 : 7;
  }
  const int o0 = c[0] < 0 ? -1 : (c[0] >= 8 ? 1 : 0);
  const int o1 = c[1] < 0 ? -1 : (c[1] >= 8 ? 1 : 0);
  const int o2 = c[2] < 0 ? -1 : (c[2] >= 8 ? 1 : 0);
  src = nb[(o2 + 1) * 9 + (o1 + 1) * 3 + (o0 + 1)];
  sc = ((c[2] - 8 * o2) * 8 + (c[1] - 8 * o1)) * 8 + (c[0] - 8 * o0);
  const bool ok = src >= 0 && src < n_patch;
  if (!ok) src = 0;
  return ok;
}

// Gather layout: the stored primitives of tile cell (i, j, k) into v and slot b of the tile (NaN
// where the cell's patch is missing); true for a physical state.
template <class T>
__device__ __forceinline__ bool gather_prim(VlTile<T> &s, const StepArgs &a, int i, int j, int k, int b,
                                            T (&v)[5])
{
  int64_t src;
  int sc;
  const bool okc = gather_cell(s.nb, a.n_patch, i, j, k, src, sc);
  const T *w = (const T *)a.prims + src * 5 * 512 + sc;
  const T nan = T(__builtin_nan(""));
#pragma unroll
  for (int f = 0; f < 5; ++f) v[f] = okc ? w[f * 512] : nan;
#pragma unroll
  for (int f = 0; f < 5; ++f) s.W[f][b] = v[f];
  return v[0] > T(0) && v[4] > T(0) && finiteT(v[1]) && finiteT(v[2]) && finiteT(v[3]);
}

// First-order flux of predictor face r along d into the buffer (FX: see riemann).
template <int d, bool FX, class T>
__device__ __forceinline__ void predictor_face(VlTile<T> &s, int r, int solver)
{
  int i, j, k;
  unpack(kVl.face[d][r], i, j, k);
  const Prim<T> wr = vload(s, vslot(i, j, k));
  const Prim<T> wl = vload(s, vslot(i - (d == 0), j - (d == 1), k - (d == 2)));
  const Cons<T> F = riemann<d, FX>(solver, wl, wr);
  s.B[0 * NVF + r] = F.D;
  s.B[1 * NVF + r] = F.m[0];
  s.B[2 * NVF + r] = F.m[1];
  s.B[3 * NVF + r] = F.m[2];
  s.B[4 * NVF + r] = F.E;
}

// Corrector flux through interface r of direction d (numbered as in the MUSCL-Hancock kernel:
// x fastest, the coordinate along d in [0, 9)), into ring slot d & 1.
template <int d, class T>
__device__ __forceinline__ void corrector_face(VlTile<T> &s, int r, T theta, int solver)
{
  int cr[3];
  if (d == 0) { cr[0] = r % 9; cr[1] = (r / 9) & 7; cr[2] = r / 72; }
  else if (d == 1) { cr[0] = r & 7; cr[1] = (r >> 3) % 9; cr[2] = r / 72; }
  else { cr[0] = r & 7; cr[1] = (r >> 3) & 7; cr[2] = r >> 6; }
  constexpr int sd = d == 0 ? 1 : (d == 1 ? BX : BX * BX);
  const int b = bidx(cr[0], cr[1], cr[2]);       // right cell; left cell b - sd
  T vl[5], vr[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const T a0 = s.W[f][b - 2 * sd], a1 = s.W[f][b - sd], a2 = s.W[f][b], a3 = s.W[f][b + sd];
    vl[f] = a1 + T(0.5) * limited_slope<sizeof(T) == 8>(a0, a1, a2, theta);
    vr[f] = a2 - T(0.5) * limited_slope<sizeof(T) == 8>(a1, a2, a3, theta);
  }
  Prim<T> wl, wr;
  wl.rho = vl[0]; wl.u[0] = vl[1]; wl.u[1] = vl[2]; wl.u[2] = vl[3]; wl.p = vl[4];
  wr.rho = vr[0]; wr.u[0] = vr[1]; wr.u[1] = vr[2]; wr.u[2] = vr[3]; wr.p = vr[4];
  const Cons<T> F = riemann<d, sizeof(T) == 8>(solver, wl, wr);
  constexpr int slot = d & 1;
  s.B[(slot * 5 + 0) * NIF + r] = F.D;
  s.B[(slot * 5 + 1) * NIF + r] = F.m[0];
  s.B[(slot * 5 + 2) * NIF + r] = F.m[1];
  s.B[(slot * 5 + 3) * NIF + r] = F.m[2];
  s.B[(slot * 5 + 4) * NIF + r] = F.E;
}

// GATHER = false: padded conserved patches (ghost >= 3), centre inversions in phase A.
// GATHER = true : the tile's primitives are gathered from the stored primitives of the patch and
//                 its neighbours, U^n of the half-step cells from their conserved interiors; the
//                 updated cells are inverted at the end.  The stored primitives come from the
//                 same inversion as phase A's (srhd_grid_prims and this kernel's output), so for
//                 equal dt both layouts give the same bits.
template <class T, class I, bool GATHER>
__device__ __forceinline__ void vl_patch(const StepArgs &a, VlTile<T> &s, const int64_t p)
{
  constexpr int NTV = vl_threads<T>();
  constexpr int HPT = (NVH + NTV - 1) / NTV;     // half-step cells per thread
  const int tid = threadIdx.x;
  const bool owner = tid < NT;                   // owns interior cell tid in D
  const int g = a.ghost;
  const int N = 8 + 2 * g;
  const int N3 = N * N * N;
  const double *__restrict__ q = GATHER ? nullptr : a.padded + p * 5 * N3;
  int lv = a.level ? (int)a.level[p] : 0;
  lv = lv < 0 ? 0 : (lv >= a.n_level ? a.n_level - 1 : lv);
  const double dh = a.dh[lv];
  double dt;
  if (!GATHER || a.dt_lev) dt = a.dt_lev[lv];
  else dt = a.c_cfl * dh / __longlong_as_double((long long)a.smax_in[0]);
  if (GATHER && a.dt_out && p == 0 && tid < a.n_level)
    a.dt_out[tid] = a.dt_lev ? a.dt_lev[tid]
                             : a.c_cfl * a.dh[tid] / __longlong_as_double((long long)a.smax_in[0]);

  if (tid < 8) s.cnt[tid] = 0u;
  if (tid < 8) s.orf[tid >> 2][tid & 3] = 0u;
  if (GATHER && tid < 27) s.nb[tid] = a.neighbor[p * 27 + tid];
  int par = 0;
  unsigned int my_iters = 0, my_inv = 0, my_nc = 0, bad_in = 0, my_pfb = 0;
  __syncthreads();

  // ---------------------------------------------------------------- A: centre primitives
  // steep: a tile cell with kappa > KAPPA_FAST or an unphysical one (FP64 bulk)
  bool steep = false;
  const T kf1 = T(KAPPA_FAST - 1.0);
  for (int r = tid; r < kVl.np; r += NTV) {
    int i, j, k;
    unpack(kVl.pcell[r], i, j, k);
    const int b = vslot(i, j, k);
    if constexpr (GATHER) {
      T v[5];
      const bool ok = gather_prim(s, a, i, j, k, b, v);
      bad_in += !ok;
      if constexpr (sizeof(T) == 8) steep |= !ok || kappa_above<T, EosTm, true>(v[0], v[1], v[2], v[3], v[4], kf1);
    } else {
      const int off = ((k + g) * N + (j + g)) * N + (i + g);
      const double D = q[off], Mx = q[N3 + off], My = q[2 * N3 + off], Mz = q[3 * N3 + off],
                   Et = q[4 * N3 + off];
      double L;
      InvOut<I> o;
      if (vl_admissible<T>(D, Mx, My, Mz, Et, L))
        invert_with_L<I, GuessT<T, I>, GuessT<T, I>, true>((I)D, (I)Mx, (I)My, (I)Mz, (I)L, (I)-1.0, false,
                                       (I)StepTol<T, I>::v, 30, o);
      else set_unphysical(o);
      bad_in += o.status == ST_UNPHYSICAL;
      my_iters += o.iters;
      my_inv += 1;
      my_nc += o.status == ST_NOCONV;
      s.W[0][b] = (T)o.rho;
      s.W[1][b] = (T)o.ux;
      s.W[2][b] = (T)o.uy;
      s.W[3][b] = (T)o.uz;
      s.W[4][b] = (T)o.p;
      if constexpr (sizeof(T) == 8)
        steep |= o.status == ST_UNPHYSICAL || kappa_above<T, EosTm, true>((T)o.rho, (T)o.ux, (T)o.uy, (T)o.uz, (T)o.p, kf1);
    }
  }
  // the predictor's arithmetic (the OR's barrier also ends phase A)
  bool fast = false;
  if constexpr (sizeof(T) == 8) fast = wg_or(s, steep ? 1u : 0u, par) == 0u;
  else __syncthreads();

  // ---------------------------------------------------------------- P: predictor
  // this thread's half-step cells: tid + h NTV for h < HPT (below NVH)
  // With theta = 0 (piecewise-constant reconstruction) the half step is dropped everywhere: the
  // step is the first-order Godunov step, W* = W^n.
  const bool predicted = a.theta > 0.0;        // uniform across the workgroup
  if (predicted) {
    T acc[HPT][5];
#pragma unroll
    for (int h = 0; h < HPT; ++h)
#pragma unroll
      for (int f = 0; f < 5; ++f) acc[h][f] = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      for (int r = tid; r < NVF; r += NTV) {
        if (fast) {                                  // uniform across the workgroup
          if (d == 0) predictor_face<0, true>(s, r, a.riemann);
          else if (d == 1) predictor_face<1, true>(s, r, a.riemann);
          else predictor_face<2, true>(s, r, a.riemann);
        } else {
          if (d == 0) predictor_face<0, false>(s, r, a.riemann);
          else if (d == 1) predictor_face<1, false>(s, r, a.riemann);
          else predictor_face<2, false>(s, r, a.riemann);
        }
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < HPT; ++h) {
        const int hc = tid + h * NTV;
        if (hc < NVH) {
          const int fm = kVl.hface[d][hc][0], fp = kVl.hface[d][hc][1];
#pragma unroll
          for (int f = 0; f < 5; ++f) acc[h][f] += s.B[f * NVF + fp] - s.B[f * NVF + fm];
        }
      }
      __syncthreads();
    }
    const double half = 0.5 * dt / dh;
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
      const int hc = tid + h * NTV;
      if (hc < NVH) {
        int i, j, k;
        unpack(kVl.hcell[hc], i, j, k);
        double u[5];
        if constexpr (GATHER) {
          int64_t src;
          int sc;
          const bool okc = gather_cell(s.nb, a.n_patch, i, j, k, src, sc);
          const double *c = a.cons + src * 5 * 512 + sc;
#pragma unroll
          for (int f = 0; f < 5; ++f) u[f] = (okc ? c[f * 512] : __builtin_nan("")) - half * (double)acc[h][f];
        } else {
          const int off = ((k + g) * N + (j + g)) * N + (i + g);
#pragma unroll
          for (int f = 0; f < 5; ++f) u[f] = q[f * N3 + off] - half * (double)acc[h][f];
        }
        double L;
        InvOut<I> o;
        if (vl_admissible<T>(u[0], u[1], u[2], u[3], u[4], L))
          invert_with_L<I, GuessT<T, I>, GuessT<T, I>, true>((I)u[0], (I)u[1], (I)u[2], (I)u[3], (I)L, (I)-1.0, false,
                                         (I)StepTol<T, I>::v, 30, o);
        else set_unphysical(o);
        my_iters += o.iters;
        my_inv += 1;
        my_nc += o.status == ST_NOCONV;
        if (o.status == ST_UNPHYSICAL) {
          // the half step is dropped for this cell: W* = W^n (still in the tile)
          const int b = bidx(i, j, k);
#pragma unroll
          for (int f = 0; f < 5; ++f) acc[h][f] = s.W[f][b];
          ++my_pfb;
        } else {
          acc[h][0] = (T)o.rho;
          acc[h][1] = (T)o.ux;
          acc[h][2] = (T)o.uy;
          acc[h][3] = (T)o.uz;
          acc[h][4] = (T)o.p;
        }
      }
    }
    // every read of the centre primitives ended at the last barrier above: overwrite with W*
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
      const int hc = tid + h * NTV;
      if (hc < NVH) {
        int i, j, k;
        unpack(kVl.hcell[hc], i, j, k);
        const int b = bidx(i, j, k);
#pragma unroll
        for (int f = 0; f < 5; ++f) s.W[f][b] = acc[h][f];
      }
    }
  }
  const bool input_bad = wg_or(s, bad_in != 0 ? 1u : 0u, par) != 0u;

  // this thread's interior cell for D
  const int ci = tid & 7, cj = (tid >> 3) & 7, ck = (tid >> 6) & 7;
  const int cq = GATHER ? tid : ((ck + g) * N + (cj + g)) * N + (ci + g);
  T theta = (T)a.theta;
  unsigned int retries = 0, unphys = 0;
  bool have_pred = predicted;
  for (int attempt = 0;; ++attempt) {
    if (theta == T(0) && have_pred) {
      // the last resort of the retry (theta = 0) is the Godunov step: put W^n back at the
      // half-step cells, inverted again from the padded input (gathered again from the stored
      // primitives)
#pragma unroll
      for (int h = 0; h < HPT; ++h) {
        const int hc = tid + h * NTV;
        if (GATHER && hc < NVH) {
          int i, j, k;
          unpack(kVl.hcell[hc], i, j, k);
          T v[5];
          gather_prim(s, a, i, j, k, bidx(i, j, k), v);
        } else if (hc < NVH) {
          int i, j, k;
          unpack(kVl.hcell[hc], i, j, k);
          const int off = ((k + g) * N + (j + g)) * N + (i + g);
          const double D = q[off], Mx = q[N3 + off], My = q[2 * N3 + off], Mz = q[3 * N3 + off],
                       Et = q[4 * N3 + off];
          double L;
          InvOut<I> o;
          if (vl_admissible<T>(D, Mx, My, Mz, Et, L))
            invert_with_L<I, GuessT<T, I>, GuessT<T, I>, true>((I)D, (I)Mx, (I)My, (I)Mz, (I)L, (I)-1.0, false,
                                           (I)StepTol<T, I>::v, 30, o);
          else set_unphysical(o);
          my_iters += o.iters;
          my_inv += 1;
          my_nc += o.status == ST_NOCONV;
          const int b = bidx(i, j, k);
          s.W[0][b] = (T)o.rho;
          s.W[1][b] = (T)o.ux;
          s.W[2][b] = (T)o.uy;
          s.W[3][b] = (T)o.uz;
          s.W[4][b] = (T)o.p;
        }
      }
      have_pred = false;
      __syncthreads();
    }
    // -------------------------------------------------------------- C + D: corrector, update
    T dU[5] = {T(0), T(0), T(0), T(0), T(0)};
    constexpr int NROUND = (3 * NIF + NTV - 1) / NTV;
    int folded = 0;
#pragma unroll 1
    for (int round = 0; round < NROUND; ++round) {
      const int qi = round * NTV + tid;
      if (qi < 3 * NIF) {
        const int d = qi / NIF;                      // uniform across each wavefront
        const int r = qi - d * NIF;
        if (d == 0) corrector_face<0>(s, r, theta, a.riemann);
        else if (d == 1) corrector_face<1>(s, r, theta, a.riemann);
        else corrector_face<2>(s, r, theta, a.riemann);
      }
      __syncthreads();
      // every direction this round completed: fold it into this thread's cell before the ring
      // slot it shares with direction d + 2 is written again
      const int done = (round + 1) * NTV / NIF < 3 ? (round + 1) * NTV / NIF : 3;
      for (; folded < done; ++folded) {
        const int d = folded;
        const int slot = d & 1;
        if (owner) {
          const int r = d == 0 ? (ck * 8 + cj) * 9 + ci : (d == 1 ? (ck * 9 + cj) * 8 + ci : (ck * 8 + cj) * 8 + ci);
          const int up = d == 0 ? 1 : (d == 1 ? 8 : 64);
#pragma unroll
          for (int f = 0; f < 5; ++f) dU[f] += s.B[(slot * 5 + f) * NIF + r + up] - s.B[(slot * 5 + f) * NIF + r];
        }
        if constexpr (!GATHER) {
          if (a.flux_out && tid < 128) write_boundary_fluxes(a.flux_out, p, d, &s.B[slot * 5 * NIF], NIF, tid);
        }
        __syncthreads();
      }
    }
    const double full = dt / dh;
    int lt = tid, lq = cq;
    asm volatile("" : "+v"(lt), "+v"(lq));
    double un[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double Lo = 0.0;
    bool ok_out = true;
    if (owner) {
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const double u0 = GATHER ? a.cons[(p * 5 + f) * 512 + lt] : q[f * N3 + lq];
        un[f] = u0 - full * (double)dU[f];
      }
      ok_out = vl_admissible<T>(un[0], un[1], un[2], un[3], un[4], Lo);
    }
    const bool fail = wg_or(s, ok_out ? 0u : 1u, par) != 0u;
    if (!fail || input_bad || theta == T(0)) {
      if (owner) {
        double *o = a.out + p * 5 * 512 + lt;
#pragma unroll
        for (int f = 0; f < 5; ++f) o[f * 512] = un[f];
        unphys += !ok_out;
      }
      if constexpr (GATHER) {
        // the updated cell's primitives (the inversion of srhd_grid_prims) and signal speed
        double sm = 0.0;
        if (owner) {
          InvOut<I> w;
          if (ok_out)
            invert_with_L<I, GuessT<T, I>, GuessT<T, I>, true>((I)un[0], (I)un[1], (I)un[2], (I)un[3], (I)Lo, (I)-1.0,
                                                               false, (I)StepTol<T, I>::v, 30, w);
          else set_unphysical(w);
          my_iters += w.iters;
          my_inv += 1;
          my_nc += w.status == ST_NOCONV;
          T *po = (T *)a.prims_out + p * 5 * 512 + lt;
          po[0] = (T)w.rho;
          po[512] = (T)w.ux;
          po[1024] = (T)w.uy;
          po[1536] = (T)w.uz;
          po[2048] = (T)w.p;
          if constexpr (sizeof(T) == 4) {
            if (ok_out) sm = (double)signal_smax_t<float>((T)w.rho, (T)w.ux, (T)w.uy, (T)w.uz, (T)w.p);
          } else {
            if (ok_out) sm = signal_smax((double)w.rho, (double)w.ux, (double)w.uy, (double)w.uz, (double)w.p);
          }
        }
        sm = wave_max_hi(sm);
        if ((tid & 63) == 63) s.red[tid >> 6] = sm;
        __syncthreads();
        if (tid == 0) {
          double m = s.red[0];
#pragma unroll
          for (int w8 = 1; w8 < NTV / 64; ++w8) m = fmax(m, s.red[w8]);
          atomicMax(a.smax_out, (unsigned long long)__double_as_longlong(m));
        }
      }
      break;
    }
    ++retries;
    theta = attempt < a.max_retry ? theta * T(0.75) : T(0);
  }

  // ---------------------------------------------------------------- counters
  if (a.stats) {
    const unsigned int c0 = wave_sum_hi(unphys + bad_in), c2 = wave_sum_hi(my_nc),
                       c3 = wave_sum_hi(my_iters), c4 = wave_sum_hi(my_inv), c7 = wave_sum_hi(my_pfb);
    if ((tid & 63) == 63) {
      atomicAdd(&s.cnt[0], c0);
      atomicAdd(&s.cnt[2], c2);
      atomicAdd(&s.cnt[3], c3);
      atomicAdd(&s.cnt[4], c4);
      atomicAdd(&s.cnt[7], c7);
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long *st = (unsigned long long *)a.stats;
      if (s.cnt[0]) atomicAdd(&st[0], (unsigned long long)s.cnt[0]);
      if (s.cnt[2]) atomicAdd(&st[2], (unsigned long long)s.cnt[2]);
      if (s.cnt[7]) atomicAdd(&st[7], (unsigned long long)s.cnt[7]);
      atomicAdd(&st[3], (unsigned long long)s.cnt[3]);
      atomicAdd(&st[4], (unsigned long long)s.cnt[4]);
      if (retries) atomicAdd(&st[5], (unsigned long long)retries);
    }
  }
}

// One patch per workgroup, or the persistent per-XCD queues, exactly as the MUSCL-Hancock
// kernel's step_body distributes patches (the loop is repeated here rather than shared through a
// callable: a call left out of line in the middle of these kernels costs them their registers).
template <class T, class I, bool GATHER>
__device__ __forceinline__ void vl_body(const StepArgs &a)
{
  extern __shared__ __align__(16) unsigned char smem_raw[];
  VlTile<T> &s = *reinterpret_cast<VlTile<T> *>(smem_raw);
  if (!a.queue) {
    const int64_t p = patch_of_block(a.n_patch, a.xcd_remap);
    if (p < a.n_patch) vl_patch<T, I, GATHER>(a, s, p);       // uniform per workgroup
    return;
  }
  const int64_t range = (a.n_patch + 7) / 8;
  const int home = blockIdx.x % 8;
  for (int k = 0; k < 8; ++k) {
    const int x = (home + k) % 8;
    const int64_t lo = x * range;
    const int64_t hi = lo + range < a.n_patch ? lo + range : a.n_patch;
    for (;;) {
      __syncthreads();
      if (threadIdx.x == 0) s.claim = atomicAdd(&a.queue[x], (unsigned long long)a.chunk);
      __syncthreads();
      const int64_t p0 = lo + (int64_t)__builtin_amdgcn_readfirstlane((int)s.claim);
      if (p0 >= hi) break;
      const int64_t p1 = p0 + a.chunk < hi ? p0 + a.chunk : hi;
      for (int64_t p = p0; p < p1; ++p) {
        vl_patch<T, I, GATHER>(a, s, p);
        __syncthreads();
      }
    }
  }
}

template <class T, class I, bool GATHER>
__global__ void __launch_bounds__(vl_threads<T>()) k_vl(StepArgs a)
{
  vl_body<T, I, GATHER>(a);
}

// Two workgroups per CU (FP32 bulk): at most 128 VGPRs.
template <class T, class I, bool GATHER>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4))) k_vl_occ2(StepArgs a)
{
  vl_body<T, I, GATHER>(a);
}

template <class T, class I, bool GATHER>
const void *vl_kernel(bool occ2)
{
  if constexpr (sizeof(T) == 4)
    if (occ2) return (const void *)k_vl_occ2<T, I, GATHER>;
  return (const void *)k_vl<T, I, GATHER>;
}

template <class T, class I, bool GATHER>
int vl_occupancy_ti(bool occ2)
{
  int n = 0;
  const size_t bytes = sizeof(VlTile<T>);
  const void *fn = vl_kernel<T, I, GATHER>(occ2);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, vl_threads<T>(), bytes) != hipSuccess) return 0;
  return n;
}

// The gather layout's prologue zeroes the output's S_max (and network masks, which stay zero:
// the VL step takes the analytic guess) before the kernel takes maxima into it.
template <class T, class I, bool GATHER>
hipError_t vl_launch_ti(const StepArgs &a, hipStream_t st)
{
  if (GATHER) {
    hipError_t e = launch_prologue<T, true>(a, st);
    if (e != hipSuccess) return e;
  }
  if (a.n_patch == 0) return hipSuccess;
  const size_t bytes = sizeof(VlTile<T>);
  const bool occ2 = a.occ2 && sizeof(T) == 4;
  hipError_t e = hipFuncSetAttribute(vl_kernel<T, I, GATHER>(occ2), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  int64_t blocks;
  if (a.queue) {
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, st, a.queue);
    blocks = a.groups;
  } else {
    blocks = a.xcd_remap ? 8 * ((a.n_patch + 7) / 8) : a.n_patch;
  }
  if constexpr (sizeof(T) == 4) {
    if (occ2) {
      hipLaunchKernelGGL((k_vl_occ2<T, I, GATHER>), dim3((unsigned)blocks), dim3(NT), bytes, st, a);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_vl<T, I, GATHER>), dim3((unsigned)blocks), dim3(vl_threads<T>()), bytes, st, a);
  return hipGetLastError();
}

template <bool GATHER>
hipError_t launch_vl(int prec, const StepArgs &a, hipStream_t st)
{
  if (prec == SRHD_PREC_MIXED) return vl_launch_ti<float, double, GATHER>(a, st);
  if (prec == SRHD_PREC_FP32) return vl_launch_ti<float, float, GATHER>(a, st);
  return vl_launch_ti<double, double, GATHER>(a, st);
}

template <bool GATHER>
int occupancy_vl(int prec, bool occ2)
{
  if (prec == SRHD_PREC_MIXED) return vl_occupancy_ti<float, double, GATHER>(occ2);
  if (prec == SRHD_PREC_FP32) return vl_occupancy_ti<float, float, GATHER>(occ2);
  return vl_occupancy_ti<double, double, GATHER>(occ2);
}

}  // namespace

hipError_t launch_step_vl(int prec, const StepArgs &a, hipStream_t st)
{
  return launch_vl<false>(prec, a, st);
}

hipError_t launch_step_vl_grid(int prec, const StepArgs &a, hipStream_t st)
{
  return launch_vl<true>(prec, a, st);
}

int step_occupancy_vl(int prec, bool gather, bool occ2)
{
  return gather ? occupancy_vl<true>(prec, occ2) : occupancy_vl<false>(prec, occ2);
}

}  // namespace srhd
