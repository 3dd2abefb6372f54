// gpcg_kernels.hip -- HIP kernels of the GPCG hot path for gfx950 (CDNA4).
//
// A pass of Algorithm GPCG (Section 3 of the paper) is one bandwidth-bound
// sweep over the unknowns: the operator (five-point stencil with constant or
// edge weights, or CSR) is applied row by row to vectors that are loaded or
// computed on the fly from x, g, l, u, fused with the elementwise updates and
// with every dot product the pass needs.  Passes:
//   INIT      x = P[x0], g = Ax - b, input checks, ||P grad q||^2, face counts
//   GP_ALPHA  d = P grad q(y): d'd, d'Ad (exact step, eq. (bqpls))
//   GP_TRIAL  y' = P[y - alpha g], g' = Ay' - b, written to the spare copies of
//             x and g; g's, s'As, active-set changes, face of y'.  Accepting
//             the step (eq. (gplsstop)) is a flip of the current copy.  In the
//             fused form the pass also looks ahead: d' = P grad q(y') on the
//             tile and its neighbours (trial point two rows out, through LDS)
//             gives d''d' and d''Ad', the next GP_ALPHA's sums, and that pass
//             is skipped when the step is accepted and the phase goes on.
//   CG_INIT   free mask, rho = -g on F, z = M^-1 rho, u = A z, w = 0
//             (eqs. (cg), (cg2); M = I, or diag(A) with the Jacobi option)
//   CG_LIST   list and matrix forms: compact the free mask into an index list
//   CG_MCOUNT matrix form (CSR): free columns of the free rows, per list tile
//   CG_MFILL  matrix form: A_F written as CSR over the list (the paper's
//             technique 1); the CG iterations then read only its nonzeros
//   CG_ITER   one CG iteration in the single-reduction form of Chronopoulos
//             and Gear: s = Ap and p by recurrence, w, rho, z, u = A z, and
//             the two sums rho'z, z'u (eq. (cgstop1) uses 1/2 alpha rho'z)
//   PS_TRIAL  x' = P[x + alpha w], g' = Ax' - b, g's, s'As, face of x'
//             (eq. (cglsstop2)); acceptance is again a flip.
// Reductions are deterministic: wave64 DPP butterflies and LDS per tile (256
// or 512 unknowns) into a fixed slot, then a fixed-order sum over the slots.  Launch
// forms: fused (every workgroup sums the previous pass's slots and runs the
// scalar transition redundantly -- identical inputs, identical decisions --
// then its tile of the next pass), split (a transition kernel, then a lean
// data kernel) and persistent (one cooperative launch, per-QP counter
// barriers).  All three use the same tiles and summation orders, so a QP gets
// bitwise the same answer in each.
//
// No MFMA: nothing on this path is a dense contraction; memory traffic and
// latency bound every pass.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "gpcg.h"
#include "gpcg_internal.h"

namespace gpcg {

// ------------------------------------------------------------ elementwise math

// Projection onto [l, u]: the median of {l, u, v} (Section 3).  Returns l or u
// bit-exactly when v lies outside, so active-set tests can use equality.
__device__ __forceinline__ double mid3(double l, double u, double v) {
  return v < l ? l : (v > u ? u : v);
}

// x_i in A(x) (Section 2).
__device__ __forceinline__ bool is_active(double x, double l, double u) {
  return x == l || x == u;
}

// x_i in B(x) (Section 2).
__device__ __forceinline__ bool is_binding(double x, double l, double u, double g) {
  return (x == l && g >= 0.0) || (x == u && g <= 0.0);
}

// Projected gradient component, eq. (proj-gradient); 0 for a fixed variable.
__device__ __forceinline__ double proj_grad(double x, double l, double u, double g) {
  if (x == l && x == u) return 0.0;
  if (x == l) return g < 0.0 ? g : 0.0;
  if (x == u) return g > 0.0 ? g : 0.0;
  return g;
}

// Trial points of the two projected searches: P[y - alpha g] (eq. next-y) and
// P[x + alpha w] (eq. cglsstop2).  One definition, so that every workgroup
// evaluating index j (owner or stencil neighbour) gets the same bits.
__device__ __forceinline__ double gp_point(double y, double l, double u, double g, double a) {
  return mid3(l, u, __fma_rn(-a, g, y));
}
__device__ __forceinline__ double ps_point(double x, double l, double u, double w, double a) {
  return mid3(l, u, __fma_rn(a, w, x));
}

template <typename T> __device__ __forceinline__ T fmaT(T a, T b, T c);
template <> __device__ __forceinline__ double fmaT<double>(double a, double b, double c) {
  return __fma_rn(a, b, c);
}
template <> __device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
  return __fmaf_rn(a, b, c);
}

// Global-address-space view of a pointer: loads and stores through it are
// global instructions.  Pointers read from memory (the state, the LDS copy of
// it, the work items) are otherwise generic, and flat accesses also count
// against the LDS counter, so every workgroup barrier waits for them.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> gbl(T *p) {
  return (gptr<T>)p;
}

// ------------------------------------------------------------------ operator

template <typename T>
struct OpView {
  int32_t kind, nx, ny, shift;
  uint64_t magic;
  T w;
  const T *wx, *wy;
  const int32_t *rowptr, *colind;
  const T *vals;
};

template <typename T>
__device__ __forceinline__ OpView<T> op_view(const QPStatic *S);

template <>
__device__ __forceinline__ OpView<double> op_view<double>(const QPStatic *S) {
  OpView<double> A;
  A.kind = S->op_kind; A.nx = S->nx; A.ny = S->ny; A.shift = S->div_shift;
  A.magic = S->div_magic; A.w = S->w; A.wx = S->wx; A.wy = S->wy;
  A.rowptr = S->rowptr; A.colind = S->colind; A.vals = S->vals;
  return A;
}

template <>
__device__ __forceinline__ OpView<float> op_view<float>(const QPStatic *S) {
  OpView<float> A;
  A.kind = S->op_kind; A.nx = S->nx; A.ny = S->ny; A.shift = S->div_shift;
  A.magic = S->div_magic; A.w = S->w32; A.wx = S->wx32; A.wy = S->wy32;
  A.rowptr = S->rowptr; A.colind = S->colind; A.vals = S->vals32;
  return A;
}

// Row k of A applied to the vector whose entries the functor v returns.
//  stencil: (A v)_k = sum_e w_e (v_k - v_nb(e)), v_nb = 0 outside the grid
//  CSR:     (A v)_k = sum_e vals_e v_{colind_e}
template <typename T, class F>
__device__ __forceinline__ T apply_row(const OpView<T> &A, int64_t k, F v) {
  if (A.kind == OPK_CSR) {
    T s = T(0);
    const gptr<const int32_t> rp = gbl(A.rowptr), ci = gbl(A.colind);
    const gptr<const T> va = gbl(A.vals);
    const int32_t e0 = rp[k], e1 = rp[k + 1];
    for (int32_t e = e0; e < e1; ++e) s = fmaT<T>(va[e], v((int64_t)ci[e]), s);
    return s;
  }
  const int32_t nx = A.nx;
  const int32_t j = (int32_t)(((uint64_t)k * A.magic) >> A.shift);
  const int32_t i = (int32_t)(k - (int64_t)j * nx);
  const T c = v(k);
  const T vW = i > 0 ? v(k - 1) : T(0);
  const T vE = i < nx - 1 ? v(k + 1) : T(0);
  const T vS = j > 0 ? v(k - nx) : T(0);
  const T vN = j < A.ny - 1 ? v(k + nx) : T(0);
  if (A.kind == OPK_CONST) return A.w * ((c - vW) + (c - vE) + ((c - vS) + (c - vN)));
  const int64_t ex = (int64_t)j * (nx + 1) + i;
  const int64_t ey = (int64_t)j * nx + i;
  const gptr<const T> gx = gbl(A.wx), gy = gbl(A.wy);
  const T wW = gx[ex], wE = gx[ex + 1], wS = gy[ey], wN = gy[ey + nx];
  return (wW * (c - vW) + wE * (c - vE)) + (wS * (c - vS) + wN * (c - vN));
}

struct Pair {
  double y, s;
};

// Row k of A applied to two vectors at once (a trial point y and its step
// s = y - x): returns (A y)_k and (A s)_k from one evaluation per entry.
template <class F>
__device__ __forceinline__ Pair apply_row2(const OpView<double> &A, int64_t k, F v) {
  Pair r{0.0, 0.0};
  if (A.kind == OPK_CSR) {
    const gptr<const int32_t> rp = gbl(A.rowptr), ci = gbl(A.colind);
    const gptr<const double> va = gbl(A.vals);
    const int32_t e0 = rp[k], e1 = rp[k + 1];
    for (int32_t e = e0; e < e1; ++e) {
      const Pair t = v((int64_t)ci[e]);
      const double a = va[e];
      r.y = __fma_rn(a, t.y, r.y);
      r.s = __fma_rn(a, t.s, r.s);
    }
    return r;
  }
  const int32_t nx = A.nx;
  const int32_t j = (int32_t)(((uint64_t)k * A.magic) >> A.shift);
  const int32_t i = (int32_t)(k - (int64_t)j * nx);
  const Pair z{0.0, 0.0};
  const Pair c = v(k);
  const Pair W = i > 0 ? v(k - 1) : z;
  const Pair E = i < nx - 1 ? v(k + 1) : z;
  const Pair So = j > 0 ? v(k - nx) : z;
  const Pair No = j < A.ny - 1 ? v(k + nx) : z;
  if (A.kind == OPK_CONST) {
    r.y = A.w * ((c.y - W.y) + (c.y - E.y) + ((c.y - So.y) + (c.y - No.y)));
    r.s = A.w * ((c.s - W.s) + (c.s - E.s) + ((c.s - So.s) + (c.s - No.s)));
    return r;
  }
  const int64_t ex = (int64_t)j * (nx + 1) + i;
  const int64_t ey = (int64_t)j * nx + i;
  const gptr<const double> gx = gbl(A.wx), gy = gbl(A.wy);
  const double wW = gx[ex], wE = gx[ex + 1], wS = gy[ey], wN = gy[ey + nx];
  r.y = (wW * (c.y - W.y) + wE * (c.y - E.y)) + (wS * (c.y - So.y) + wN * (c.y - No.y));
  r.s = (wW * (c.s - W.s) + wE * (c.s - E.s)) + (wS * (c.s - So.s) + wN * (c.s - No.s));
  return r;
}

// ---------------------------------------------------------------- reductions

// Cross-lane moves with DPP (gfx9 encodings; every source lane is active and
// in range for these patterns) and lane reads.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_f32(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over the 64 lanes of a wave, the same value in every lane.  Fixed
// order: lane ^ 1, lane ^ 2 (quad permutes), the other quad of the half-row,
// the other half of the row, then the four rows (lanes 0, 16, 32, 48).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  v += dpp_f32<0x141>(v);
  v += dpp_f32<0x140>(v);
  return (lane_f32(v, 0) + lane_f32(v, 16)) + (lane_f32(v, 32) + lane_f32(v, 48));
}

// Sum of v[0..N) over the workgroup, valid in thread 0 (waves added in the
// order 0..3).  Must be called by every thread, in uniform control flow.  The
// LDS scratch is reused by the next call of the same instantiation: callers
// separate two such calls by a barrier.
template <typename R, int N, int M>
__device__ __forceinline__ void block_sum(R (&v)[M]) {
  static_assert(N <= M, "slot count");
  __shared__ R sh[kBlock / 64][N];
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const R w = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) sh[wave][k] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
}

// Map the launch index of a workgroup to a tile so that consecutive tiles land
// on the same XCD: gfx950 dispatches workgroups round-robin over its 8 XCDs,
// each with its own L2, and the stencil neighbours of a tile live in the tiles
// next to it.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  constexpr int X = 8;
  const int xcd = b % X, local = b / X;
  const int per = G / X, rem = G % X;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Slots 0 and 1 of the CG passes are FP32 sums in the mixed form.
__device__ __forceinline__ bool f32_slots(int mixed, int phase) {
  return mixed && (phase == PH_CG_INIT || phase == PH_CG_ITER);
}

// Number of reduction slots a pass fills.
__device__ __forceinline__ int nslots(int phase) {
  switch (phase) {
    case PH_GP_ALPHA: case PH_CG_ITER: return 2;
    case PH_CG_INIT: return 3;
    case PH_CG_LIST: case PH_CG_MCOUNT: case PH_CG_MFILL: return 1;
    default: return kNP;
  }
}

// Workgroup sum of the slots a pass fills (valid in thread 0); FP32 slots of
// the mixed CG passes are summed in FP32 and stored widened.
__device__ __forceinline__ void block_slots(int ns, bool f32, double (&acc)[kNP],
                                            float (&accf)[2]) {
  if (f32) {
    block_sum<float, 2>(accf);
    if (ns == 3) block_sum<double, 3>(acc);  // slot 2 is a count
    if (threadIdx.x == 0) {
      acc[0] = (double)accf[0];
      acc[1] = (double)accf[1];
    }
  } else if (ns == 2) {
    block_sum<double, 2>(acc);
  } else if (ns == 3) {
    block_sum<double, 3>(acc);
  } else {
    block_sum<double, kNP>(acc);
  }
}

// Reduces this workgroup's per-thread sums into the tile's slot of parity
// `par` (thread 0 writes the ns slots the pass fills).
__device__ __forceinline__ void write_partial(double *slots, int par, int phase, bool f32,
                                              int tile, double (&acc)[kNP], float (&accf)[2]) {
  const int ns = nslots(phase);
  block_slots(ns, f32, acc, accf);
  if (threadIdx.x == 0) {
    const gptr<double> sl = gbl(slots);
    for (int k = 0; k < ns; ++k) sl[slot_index(tile, par, k)] = acc[k];
  }
}

// Loads slot `tid` of parity par (always present) ahead of time.
__device__ __forceinline__ void prefetch_slot(const double *slots, int par, double (&pf)[kNP]) {
  const gptr<const double> sl = gbl(slots);
#pragma unroll
  for (int k = 0; k < kNP; ++k) pf[k] = sl[slot_index((int)threadIdx.x, par, k)];
}

// Loads the first ns slots of tile `tid` of parity par (always present); the
// others are zero.
__device__ __forceinline__ void prefetch_slots(const double *slots, int par, int ns,
                                               double (&pf)[kNP]) {
  const gptr<const double> sl = gbl(slots);
#pragma unroll
  for (int k = 0; k < kNP; ++k) pf[k] = k < ns ? sl[slot_index((int)threadIdx.x, par, k)] : 0.0;
}

// Adds slots t = tid + 256, tid + 512, ... (in that order) of parity par to
// res / vf, issuing the loads of D slots at a time before adding them.
template <int NS, int D = (NS <= 3 ? 8 : 2)>
__device__ __forceinline__ void sum_slot_tail(const double *slots, int par, int ntiles,
                                              double (&res)[kNP], float (&vf)[2]) {
  const gptr<const double> sl = gbl(slots);
  for (int base = (int)threadIdx.x + kBlock; base < ntiles; base += D * kBlock) {
    double buf[D][NS];
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int t = base + u * kBlock;
#pragma unroll
      for (int k = 0; k < NS; ++k) buf[u][k] = t < ntiles ? sl[slot_index(t, par, k)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < D; ++u) {
      if (base + u * kBlock < ntiles) {
#pragma unroll
        for (int k = 0; k < NS; ++k) res[k] += buf[u][k];
        vf[0] += (float)buf[u][0];
        vf[1] += (float)buf[u][1];
      }
    }
  }
}

// Sums the ntiles slots of parity par that pass `phase` filled, in tile
// order (thread tid takes tiles tid, tid + 256, ...; slot tid prefetched in
// pf); the result is valid in thread 0's res.  DEEP keeps more loads in
// flight (the transition kernel, where registers are plentiful).
template <bool DEEP = false>
__device__ __forceinline__ void sum_partials(const double *slots, int par, int ntiles, int phase,
                                             bool f32, const double (&pf)[kNP],
                                             double (&res)[kNP]) {
  const int ns = nslots(phase);
  float vf[2];
  const bool mine = (int)threadIdx.x < ntiles;
#pragma unroll
  for (int k = 0; k < kNP; ++k) res[k] = (mine && k < ns) ? pf[k] : 0.0;
  vf[0] = mine ? (float)pf[0] : 0.0f;
  vf[1] = mine ? (float)pf[1] : 0.0f;
  if (ntiles > kBlock) {
    if (ns == 2) sum_slot_tail<2, DEEP ? 16 : 4>(slots, par, ntiles, res, vf);
    else if (ns == 3) sum_slot_tail<3, DEEP ? 12 : 4>(slots, par, ntiles, res, vf);
    else sum_slot_tail<kNP, DEEP ? 4 : 2>(slots, par, ntiles, res, vf);
  }
  block_slots(ns, f32, res, vf);
}

// ------------------------------------------------------------ the passes

// Exclusive prefix sum of v over the workgroup in thread order (valid in every
// thread); total receives the sum.  Every thread must call it.
__device__ __forceinline__ int block_exscan(int v, int &total) {
  __shared__ int s_w[kBlock / 64];
  const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wv] = x;
  __syncthreads();
  int off = 0;
  for (int i = 0; i < wv; ++i) off += s_w[i];
  total = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
  __syncthreads();  // s_w is reused by the next call
  return off + x - v;
}

// Free columns of row k of a CSR operator.
__device__ __forceinline__ int free_cols(const QPStatic *S, int64_t k) {
  int c = 0;
  for (int32_t p = S->rowptr[k]; p < S->rowptr[k + 1]; ++p) c += S->mask[S->colind[p]] ? 1 : 0;
  return c;
}

// Matrix form, fill pass: A_F (the reduced matrix of the paper's technique 1)
// as CSR over the list, columns as grid indices, one list entry per thread
// (entries [k0, k1) of the list).  The offset of this tile's rows is the
// number of nonzeros of the list tiles before it (slot 0 of the count pass).
template <typename CT>
__device__ __forceinline__ void matrix_fill(const QPStatic *__restrict__ S,
                                         const double *__restrict__ slots, int64_t m_free,
                                         int lpar, int64_t k0, int64_t k1) {
  const int tile = (int)(k0 / kBlock);
  double before[1] = {0.0};
  for (int t = (int)threadIdx.x; t < tile; t += kBlock)
    before[0] += slots[slot_index(t, lpar, 0)];
  block_sum<double, 1>(before);
  __shared__ int64_t s_mbase;
  if (threadIdx.x == 0) s_mbase = (int64_t)before[0];
  const int64_t e1 = k1 < m_free ? k1 : m_free;
  const int64_t e = k0 + threadIdx.x;
  const bool row = e < e1;
  const int64_t k = row ? S->list[e] : 0;
  const int c = row ? free_cols(S, k) : 0;
  int total;
  const int pos = block_exscan(c, total);
  if (row) {
    const OpView<CT> A = op_view<CT>(S);
    CT *__restrict__ mv = (CT *)S->mval;
    int64_t at = s_mbase + pos;
    if (e == 0) S->mrow[0] = 0;
    S->mrow[e + 1] = (int32_t)(at + c);
    for (int32_t p = S->rowptr[k]; p < S->rowptr[k + 1]; ++p) {
      const int32_t j = S->colind[p];
      if (S->mask[j]) {
        S->mcol[at] = j;
        mv[at] = A.vals[p];
        ++at;
      }
    }
  }
}

// Face of a point: ||P grad q||^2, lower-active, upper-active, active and not
// binding, and x'(g - b) (twice q(x)).
__device__ __forceinline__ void face_acc(double x, double l, double u, double g, double b,
                                         double (&acc)[kNP]) {
  const double p = proj_grad(x, l, u, g);
  acc[0] = __fma_rn(p, p, acc[0]);
  acc[1] += (x == l) ? 1.0 : 0.0;
  acc[2] += (x != l && x == u) ? 1.0 : 0.0;
  acc[3] += (is_active(x, l, u) && !is_binding(x, l, u, g)) ? 1.0 : 0.0;
  acc[4] = __fma_rn(x, g - b, acc[4]);
}

// GP_TRIAL of a stencil QP that also evaluates the step length of the next
// gradient-projection iterate (eq. (bqpls) at the trial point y'), so that
// the phase needs no separate GP_ALPHA pass.  Per chunk of 256 unknowns
// [c0, c0 + 256) the workgroup forms, in LDS, y' on the five grid rows at
// offsets -2 nx .. 2 nx from the chunk (the middle rows one and two entries
// wider), g' = Ay' - b and d' = P grad q(y') on the chunk and the rows next to
// it, and finally (A d')_k on the chunk: slots 8 and 9 receive d'd' and
// d'Ad'.  Every value is the expression its owner evaluates in a GP_TRIAL
// pass and then in a GP_ALPHA pass, so the sums are bitwise those two passes'.
constexpr int kLaW = kBlock + 4;  // LDS row: positions c0 - 2 .. c0 + 257

// The stencil row of apply_row / apply_row2 on values at (k, W, E, S, N).
__device__ __forceinline__ double row5(const QPStatic *S, const double *wt, const bool *has,
                                       double c, double vW, double vE, double vS, double vN) {
  vW = has[0] ? vW : 0.0;
  vE = has[1] ? vE : 0.0;
  vS = has[2] ? vS : 0.0;
  vN = has[3] ? vN : 0.0;
  if (S->op_kind == OPK_CONST) return S->w * ((c - vW) + (c - vE) + ((c - vS) + (c - vN)));
  return (wt[0] * (c - vW) + wt[1] * (c - vE)) + (wt[2] * (c - vS) + wt[3] * (c - vN));
}

// Grid coordinates of unknown p and which of its W, E, S, N neighbours exist.
__device__ __forceinline__ void grid_has(const QPStatic *S, int64_t p, int32_t &i, int32_t &j,
                                         bool (&has)[4]) {
  const int32_t nx = S->nx;
  j = (int32_t)(((uint64_t)p * S->div_magic) >> S->div_shift);
  i = (int32_t)(p - (int64_t)j * nx);
  has[0] = i > 0;
  has[1] = i < nx - 1;
  has[2] = j > 0;
  has[3] = j < S->ny - 1;
}

__device__ __forceinline__ void stencil_weights(const QPStatic *S, int64_t p, int32_t i,
                                                int32_t j, double (&wt)[4]) {
  if (S->op_kind == OPK_VAR) {
    const gptr<const double> wx = gbl(S->wx), wy = gbl(S->wy);
    const int64_t ex = (int64_t)j * (S->nx + 1) + i;
    wt[0] = wx[ex];
    wt[1] = wx[ex + 1];
    wt[2] = wy[p];
    wt[3] = wy[p + S->nx];
  }
}

// Global operands of a look-ahead trial pass over the 256 unknowns from c0,
// thread t: x, l, u, g (copy cp) at c0 + t + r nx on the rows r = -2..2; the
// same at one entry beyond the chunk's columns (threads t < 8, entry
// la_edge(t)); b, the neighbour flags and the edge weights at the middle-row
// entries (and at the middle-row end of threads 1 and 2).  All loads are
// issued together, before any of them is used.
struct LAOperands {
  double x[5], l[5], u[5], g[5];
  double xe, le, ue, ge;
  double b[4], wt[4][4];  // [0..2]: rows -1, 0, 1 at column t; [3]: the row end
  bool has[4][4];
};

// Entry beyond the chunk's columns taken by thread t < 8, as (row, column -
// c0): (0, -2), (0, -1), (0, 256), (0, 257), (-1, -1), (-1, 256), (1, -1),
// (1, 256).  Threads 1 and 2 hold the two ends of the middle row.
__device__ __forceinline__ void la_edge(int t, int &r, int &q) {
  r = t < 4 ? 0 : (t < 6 ? -1 : 1);
  q = t < 4 ? (t < 2 ? t - 2 : kBlock + t - 2) : ((t & 1) ? kBlock : -1);
}

__device__ __forceinline__ void la_load(const QPStatic *__restrict__ S, int cp, int64_t c0,
                                        LAOperands &O) {
  const int64_t n = S->n, nx = S->nx;
  const gptr<const double> x = gbl((const double *)S->x[cp]);
  const gptr<const double> g = gbl((const double *)S->g[cp]);
  const gptr<const double> l = gbl(S->l), u = gbl(S->u), b = gbl(S->b);
  const int t = (int)threadIdx.x;
#pragma unroll
  for (int r = -2; r <= 2; ++r) {
    const int64_t p = c0 + t + r * nx;
    const bool in = p >= 0 && p < n;
    O.x[r + 2] = in ? x[p] : 0.0;
    O.l[r + 2] = in ? l[p] : 0.0;
    O.u[r + 2] = in ? u[p] : 0.0;
    O.g[r + 2] = in ? g[p] : 0.0;
  }
  int er, eq;
  la_edge(t, er, eq);
  const int64_t pe = c0 + eq + er * nx;
  const bool ine = t < 8 && pe >= 0 && pe < n;
  O.xe = ine ? x[pe] : 0.0;
  O.le = ine ? l[pe] : 0.0;
  O.ue = ine ? u[pe] : 0.0;
  O.ge = ine ? g[pe] : 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int64_t p = m < 3 ? c0 + t + (m - 1) * nx : pe;
    const bool in = m < 3 ? (p >= 0 && p < n) : (ine && (t == 1 || t == 2));
    int32_t i = 0, j = 0;
    if (in) grid_has(S, p, i, j, O.has[m]);
    else
      for (int e = 0; e < 4; ++e) O.has[m][e] = false;
    O.b[m] = in ? b[p] : 0.0;
    if (S->op_kind == OPK_VAR && in) stencil_weights(S, p, i, j, O.wt[m]);
    else
      for (int e = 0; e < 4; ++e) O.wt[m][e] = 0.0;
  }
}

// The pass on loaded operands (copy cp in, copy cp ^ 1 out; chunk [c0, k1)).
__device__ __forceinline__ void la_compute(const QPStatic *__restrict__ S, int cp, double a,
                                           int64_t c0, int64_t k1, const LAOperands &O,
                                           double (&acc)[kNP]) {
  __shared__ double s_y[5][kLaW];  // y' on rows -2..2, entry pos - c0 + 2
  __shared__ double s_s[3][kLaW];  // y' - x on rows -1..1
  __shared__ double s_d[3][kLaW];  // d' on rows -1..1
  const int64_t n = S->n, nx = S->nx;
  const int t = (int)threadIdx.x;
  // y' and y' - x on the five rows and at the entry beyond the columns
#pragma unroll
  for (int r = -2; r <= 2; ++r) {
    const double yv = gp_point(O.x[r + 2], O.l[r + 2], O.u[r + 2], O.g[r + 2], a);
    s_y[r + 2][t + 2] = yv;
    if (r >= -1 && r <= 1) s_s[r + 1][t + 2] = yv - O.x[r + 2];
  }
  int er, eq;
  la_edge(t, er, eq);
  if (t < 8) {
    const double yv = gp_point(O.xe, O.le, O.ue, O.ge, a);
    s_y[er + 2][eq + 2] = yv;
    s_s[er + 1][eq + 2] = yv - O.xe;
  }
  __syncthreads();
  // g' = Ay' - b and d' = P grad q(y') on the middle rows and at the ends of
  // the middle row; the trial pass proper at the chunk's own unknown
  const int64_t k = c0 + t;
  auto grad_dir = [&](int m, int rr, int q, double yl, double yu) {
    const int64_t p = c0 + q + rr * nx;
    double dv = 0.0;
    if (p >= 0 && p < n) {
      const double yc = s_y[rr + 2][q + 2];
      const double gy = row5(S, O.wt[m], O.has[m], yc, s_y[rr + 2][q + 1], s_y[rr + 2][q + 3],
                             s_y[rr + 1][q + 2], s_y[rr + 3][q + 2]) -
                        O.b[m];
      dv = proj_grad(yc, yl, yu, gy);
      if (m == 1 && k < k1) {
        const double sk = s_s[1][t + 2];
        const double As = row5(S, O.wt[1], O.has[1], sk, s_s[1][t + 1], s_s[1][t + 3],
                               s_s[0][t + 2], s_s[2][t + 2]);
        gbl(S->x[cp ^ 1])[k] = yc;
        gbl(S->g[cp ^ 1])[k] = gy;
        face_acc(yc, yl, yu, gy, O.b[1], acc);
        acc[5] = __fma_rn(O.g[2], sk, acc[5]);
        acc[6] = __fma_rn(sk, As, acc[6]);
        acc[7] += (is_active(yc, yl, yu) != is_active(O.x[2], yl, yu)) ? 1.0 : 0.0;
      }
    }
    s_d[rr + 1][q + 2] = dv;
  };
  grad_dir(0, -1, t, O.l[1], O.u[1]);
  grad_dir(1, 0, t, O.l[2], O.u[2]);
  grad_dir(2, 1, t, O.l[3], O.u[3]);
  if (t == 1 || t == 2) grad_dir(3, 0, eq, O.le, O.ue);
  __syncthreads();
  // (A d')_k on the chunk
  if (k < k1) {
    const double dk = s_d[1][t + 2];
    const double Adk = row5(S, O.wt[1], O.has[1], dk, s_d[1][t + 1], s_d[1][t + 3],
                            s_d[0][t + 2], s_d[2][t + 2]);
    acc[8] = __fma_rn(dk, dk, acc[8]);
    acc[9] = __fma_rn(dk, Adk, acc[9]);
  }
}

// One pass over the unknowns [k0, k1) of a tile (the list entries [k0, k1)
// for a CG iteration of the list form).  `slots` are the QP's tile slots: the
// list pass reads the free counts the set-up pass left at parity lpar.
template <typename CT, bool PRE, bool LA, bool MAT>
__device__ void run_pass(const QPStatic *__restrict__ S, const double *__restrict__ slots,
                         const QPCore &d, int phase, int lpar, int64_t k0, int64_t k1,
                         double (&acc)[kNP], float (&accf)[2]) {
  const gptr<const double> l = gbl(S->l);
  const gptr<const double> u = gbl(S->u);
  const gptr<const double> b = gbl(S->b);
  const int c = d.cur;
  const gptr<const double> x = gbl((const double *)S->x[c]);
  const gptr<const double> g = gbl((const double *)S->g[c]);
  const gptr<double> xn = gbl(S->x[c ^ 1]);
  const gptr<double> gn = gbl(S->g[c ^ 1]);
  constexpr int64_t st = kBlock;
  switch (phase) {
    case PH_INIT: {
      // x[0] holds x0; it is projected in place.  A neighbour may read x0_j
      // before or after its owner projects it: mid(l, u, .) is idempotent, so
      // both give the same value (l <= u is verified by this same pass).
      const OpView<double> A = op_view<double>(S);
      const gptr<double> x0 = gbl(S->x[0]);
      const gptr<double> g0 = gbl(S->g[0]);
      auto xv = [&](int64_t j) { return mid3(l[j], u[j], x0[j]); };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += st) {
        const double xo = x0[k], lk = l[k], uk = u[k], bk = b[k];
        const double xk = mid3(lk, uk, xo);
        const double gk = apply_row<double>(A, k, xv) - bk;
        acc[5] += (lk > uk) ? 1.0 : 0.0;
        acc[6] += (isnan(xo) || isnan(lk) || isnan(uk) || isnan(bk)) ? 1.0 : 0.0;
        acc[7] += (xk != xo) ? 1.0 : 0.0;
        x0[k] = xk;
        g0[k] = gk;
        face_acc(xk, lk, uk, gk, bk, acc);
      }
    } break;
    case PH_GP_ALPHA: {
      const OpView<double> A = op_view<double>(S);
      auto dv = [&](int64_t j) { return proj_grad(x[j], l[j], u[j], g[j]); };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += st) {
        const double dk = dv(k);
        const double Adk = apply_row<double>(A, k, dv);
        acc[0] = __fma_rn(dk, dk, acc[0]);
        acc[1] = __fma_rn(dk, Adk, acc[1]);
      }
    } break;
    case PH_GP_TRIAL: {
      if (LA && S->gp_la) {  // 256-unknown tiles: one chunk
        LAOperands O;
        la_load(S, d.cur, k0, O);
        la_compute(S, d.cur, d.alpha, k0, k1, O, acc);
        break;
      }
      const OpView<double> A = op_view<double>(S);
      const double a = d.alpha;
      auto yv = [&](int64_t j) {
        const double xj = x[j];
        const double yj = gp_point(xj, l[j], u[j], g[j], a);
        return Pair{yj, yj - xj};
      };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += st) {
        const double xk = x[k], lk = l[k], uk = u[k], gk = g[k], bk = b[k];
        const double yk = gp_point(xk, lk, uk, gk, a);
        const double sk = yk - xk;
        const Pair As = apply_row2(A, k, yv);
        const double gy = As.y - bk;
        xn[k] = yk;
        gn[k] = gy;
        face_acc(yk, lk, uk, gy, bk, acc);
        acc[5] = __fma_rn(gk, sk, acc[5]);
        acc[6] = __fma_rn(sk, As.s, acc[6]);
        acc[7] += (is_active(yk, lk, uk) != is_active(xk, lk, uk)) ? 1.0 : 0.0;
      }
    } break;
    case PH_CG_INIT: {
      const OpView<CT> A = op_view<CT>(S);
      const gptr<uint8_t> mask = gbl(S->mask);
      // the first CG iteration runs in the next launch, which reads parity
      // lpar ^ 1 (in the list form two launches later, in the matrix form
      // four: parity lpar)
      const int fp = S->list ? lpar : lpar ^ 1;
      const gptr<CT> r0 = gbl((CT *)S->rho[fp]);
      const gptr<CT> u0 = gbl((CT *)S->uq[fp]);
      const gptr<CT> r1 = gbl((CT *)S->rho[fp ^ 1]);
      const gptr<CT> u1 = gbl((CT *)S->uq[fp ^ 1]);
      const gptr<CT> s0 = gbl((CT *)S->sq[0]);
      const gptr<CT> s1 = gbl((CT *)S->sq[1]);
      const gptr<CT> p = gbl((CT *)S->pv);
      const gptr<CT> w = gbl((CT *)S->wv);
      // preconditioned residual z = D^-1 rho (rho itself without a preconditioner)
      const gptr<const CT> dinv = gbl(PRE ? (const CT *)S->dinv : nullptr);
      auto zv = [&](int64_t j) {
        const double xj = x[j];
        const CT r = (l[j] < xj && xj < u[j]) ? (CT)(-g[j]) : CT(0);
        return dinv ? r * dinv[j] : r;
      };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += st) {
        const double xk = x[k];
        const bool fr = l[k] < xk && xk < u[k];
        mask[k] = fr ? 1 : 0;
        if (fr) {
          const CT rk = (CT)(-g[k]);
          const CT zk = dinv ? rk * dinv[k] : rk;
          const CT uk = apply_row<CT>(A, k, zv);  // A z
          r0[k] = rk;
          u0[k] = uk;
          w[k] = CT(0);
          if (sizeof(CT) == 4) {
            accf[0] = fmaT<float>((float)rk, (float)zk, accf[0]);
            accf[1] = fmaT<float>((float)zk, (float)uk, accf[1]);
          } else {
            acc[0] = __fma_rn((double)rk, (double)zk, acc[0]);
            acc[1] = __fma_rn((double)zk, (double)uk, acc[1]);
          }
          acc[2] += 1.0;
        } else {
          // neighbours read these on the active set: keep them zero
          r0[k] = CT(0);
          u0[k] = CT(0);
          r1[k] = CT(0);
          u1[k] = CT(0);
          s0[k] = CT(0);
          s1[k] = CT(0);
          p[k] = CT(0);
        }
      }
    } break;
    case PH_CG_LIST: {
      // offset of this tile in the list = free rows of the tiles before it
      // (slot 2 of the set-up pass, exact integers in FP64)
      const int tile = (int)(k0 / kBlock);
      double before[1] = {0.0};
      for (int t = (int)threadIdx.x; t < tile; t += kBlock)
        before[0] += slots[slot_index(t, lpar, 2)];
      block_sum<double, 1>(before);
      __shared__ int64_t s_base;
      __shared__ int s_wave[kBlock / 64];
      if (threadIdx.x == 0) s_base = (int64_t)before[0];
      const int64_t k = k0 + threadIdx.x;
      const bool fr = k < k1 && S->mask[k] != 0;
      const uint64_t bal = __ballot(fr);
      const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
      const int rank = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) s_wave[wv] = __popcll(bal);
      __syncthreads();
      int off = 0;
      for (int i = 0; i < wv; ++i) off += s_wave[i];
      if (fr) S->list[s_base + off + rank] = (int32_t)k;
      __syncthreads();
    } break;
    case PH_CG_MCOUNT: {
      // matrix form: nonzeros of A_F, i.e. the free columns of the free rows
      // (entries [k0, k1) of the list; slot 0, exact integers in FP64)
      if constexpr (MAT) {
        const int64_t e1 = k1 < d.m_free ? k1 : d.m_free;
        for (int64_t e = k0 + threadIdx.x; e < e1; e += st)
          acc[0] += (double)free_cols(S, S->list[e]);
      }
    } break;
    case PH_CG_MFILL:
      if constexpr (MAT) matrix_fill<CT>(S, slots, d.m_free, lpar, k0, k1);
      break;
    case PH_CG_ITER: {
      const OpView<CT> A = op_view<CT>(S);
      const gptr<const uint8_t> mask = gbl((const uint8_t *)S->mask);
      const int par = lpar;  // CG buffers alternate with the launch parity
      const bool first = d.first != 0;
      const CT al = (CT)d.cg_alpha, be = (CT)d.cg_beta;
      const gptr<const CT> ro = gbl((const CT *)S->rho[par]);
      const gptr<const CT> uo = gbl((const CT *)S->uq[par]);
      const gptr<const CT> so = gbl((const CT *)S->sq[par]);
      const gptr<CT> rn = gbl((CT *)S->rho[par ^ 1]);
      const gptr<CT> un = gbl((CT *)S->uq[par ^ 1]);
      const gptr<CT> sn = gbl((CT *)S->sq[par ^ 1]);
      const gptr<CT> p = gbl((CT *)S->pv);
      const gptr<CT> w = gbl((CT *)S->wv);
      // s_i = u_i + beta s_{i-1} (= A p_i);  rho_{i+1} = rho_i - alpha s_i
      auto snew = [&](int64_t j) { return first ? uo[j] : fmaT<CT>(be, so[j], uo[j]); };
      auto rnew = [&](int64_t j) { return fmaT<CT>(-al, snew(j), ro[j]); };
      // z = D^-1 rho with the Jacobi preconditioner, else rho; u = A z
      const gptr<const CT> dinv = gbl(PRE ? (const CT *)S->dinv : nullptr);
      auto znew = [&](int64_t j) {
        const CT r = rnew(j);
        return dinv ? r * dinv[j] : r;
      };
      CT gam = CT(0), del = CT(0);
      const gptr<const int32_t> list = gbl((const int32_t *)S->list);
      const gptr<const int32_t> mrow = gbl((const int32_t *)S->mrow);
      // list form: entries [k0, k1) of the free list; mask form: rows [k0, k1)
      const int64_t e1 = list ? (k1 < d.m_free ? k1 : d.m_free) : k1;
      for (int64_t e = k0 + threadIdx.x; e < e1; e += st) {
        int64_t k = e;
        if (list) k = list[e];
        else if (!mask[k]) continue;  // the CG vectors vanish on the active set
        const CT rk = ro[k];
        const CT sk = snew(k);
        const CT r1 = fmaT<CT>(-al, sk, rk);
        const CT dk = dinv ? dinv[k] : CT(1);
        const CT zk = dinv ? rk * dk : rk;
        const CT z1 = dinv ? r1 * dk : r1;
        const CT pk = first ? zk : fmaT<CT>(be, p[k], zk);
        w[k] = fmaT<CT>(al, pk, w[k]);
        p[k] = pk;
        sn[k] = sk;
        rn[k] = r1;
        CT u1;
        if (MAT && mrow) {  // A_F: the free columns only (the others hold z = 0)
          const gptr<const CT> mv = gbl((const CT *)S->mval);
          const gptr<const int32_t> mc = gbl((const int32_t *)S->mcol);
          u1 = CT(0);
          for (int32_t q = mrow[e]; q < mrow[e + 1]; ++q) u1 = fmaT<CT>(mv[q], znew(mc[q]), u1);
        } else {
          u1 = apply_row<CT>(A, k, znew);
        }
        un[k] = u1;
        gam = fmaT<CT>(r1, z1, gam);
        del = fmaT<CT>(z1, u1, del);
      }
      if (sizeof(CT) == 4) {
        accf[0] = (float)gam;
        accf[1] = (float)del;
      } else {
        acc[0] = (double)gam;
        acc[1] = (double)del;
      }
    } break;
    case PH_PS_TRIAL: {
      const OpView<double> A = op_view<double>(S);
      const gptr<const uint8_t> mask = gbl((const uint8_t *)S->mask);
      const gptr<const CT> w = gbl((const CT *)S->wv);
      const double a = d.alpha;
      // the CG direction is zero on A(x_k): those entries do not move
      auto yv = [&](int64_t j) {
        const double xj = x[j];
        const double yj = mask[j] ? ps_point(xj, l[j], u[j], (double)w[j], a) : xj;
        return Pair{yj, yj - xj};
      };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += st) {
        const double xk = x[k], lk = l[k], uk = u[k], gk = g[k], bk = b[k];
        const double yk = mask[k] ? ps_point(xk, lk, uk, (double)w[k], a) : xk;
        const double sk = yk - xk;
        const Pair As = apply_row2(A, k, yv);
        const double gy = As.y - bk;
        xn[k] = yk;
        gn[k] = gy;
        face_acc(yk, lk, uk, gy, bk, acc);
        acc[5] = __fma_rn(gk, sk, acc[5]);
        acc[6] = __fma_rn(sk, As.s, acc[6]);
      }
    } break;
    default:
      break;
  }
}

// ------------------------------------------------------ the scalar transition

__device__ __forceinline__ int time_bucket(int phase) {
  switch (phase) {
    case PH_CG_INIT: case PH_CG_LIST: case PH_CG_MCOUNT: case PH_CG_MFILL: case PH_CG_ITER:
      return TB_CG;
    case PH_GP_ALPHA: case PH_GP_TRIAL: return TB_GP;
    case PH_PS_TRIAL: return TB_SEARCH;
    default: return TB_OTHER;
  }
}

__device__ __forceinline__ void finish(QPCore &d, int status) {
  d.status = status;
  d.phase = PH_DONE;
}

// A gradient-projection phase begins: y_0 = x_k (Algorithm GPCG, first bullet).
__device__ __forceinline__ void start_gp(QPCore &d) {
  d.gp_j = 1;
  d.gp_decmax = -INFINITY;
  d.gp_accepts = 0;
  d.phase = PH_GP_ALPHA;
}

// The gradient-projection phase ends: termination test, then CG with the
// initial eta2 (reset whenever a gradient-projection phase runs).
__device__ __forceinline__ void end_gp(const QPStatic *S, QPCore &d) {
  if (d.pgn <= d.tau) {
    finish(d, GPCG_OK);
    return;
  }
  d.eta = S->eta2;
  d.phase = PH_CG_INIT;
}

// The first trial of a gradient-projection iterate y, given dd = d'd and
// dAd = d'Ad for d = P grad q(y).
// Every field is written on both outcomes (selects, no branches), which keeps
// the state in registers.
__device__ __forceinline__ void gp_step(QPCore &d, double dd, double dAd) {
  // P grad q(y) = 0: y solves the QP; d'Ad <= 0: A is not positive definite
  const bool go = dd != 0.0 && dAd > 0.0;
  d.status = go ? d.status : (dd == 0.0 ? (int32_t)GPCG_OK : (int32_t)GPCG_ERR_NOT_SPD);
  d.alpha = go ? dd / dAd : d.alpha;  // eq. (bqpls): ||d||^2 / d'Ad
  d.bt = go ? 0 : d.bt;
  d.phase = go ? (int32_t)PH_GP_TRIAL : (int32_t)PH_DONE;
}

// Projected search along d_k = Z_k w: alpha = 1, 1/2, 1/4, ... (eq. cglsstop2).
__device__ __forceinline__ void start_ps(QPCore &d) {
  d.alpha = 1.0;
  d.bt = 0;
  d.ps_accepted = 0;
  d.phase = PH_PS_TRIAL;
}

__device__ __forceinline__ void set_face(QPCore &d, const double *R) {
  d.pgn = sqrt(R[0]);
  d.n_lower = (int64_t)R[1];
  d.n_upper = (int64_t)R[2];
  d.n_nonbinding = (int64_t)R[3];
  d.q = 0.5 * R[4];
}

// Folds the reduced results R of pass d.phase into the state and selects the
// next pass.  Runs in one thread of every workgroup on identical inputs.  la:
// trial passes of this QP look ahead (slots 8 and 9 hold eq. (bqpls) at the
// trial point; the fused form only).
__device__ void transition(const QPStatic *S, QPCore &d, const double *R, bool la) {
  const int ph = d.phase;
  d.passes += 1;
  switch (ph) {
    case PH_INIT:
      if (R[6] > 0.0) { finish(d, GPCG_ERR_NAN); break; }
      if (R[5] > 0.0) { finish(d, GPCG_ERR_BOUNDS); break; }
      d.x0_projected = R[7] > 0.0 ? 1 : 0;
      set_face(d, R);
      d.pg0 = d.pgn;
      d.tau = S->tol_rel * d.pgn > S->tol_abs ? S->tol_rel * d.pgn : S->tol_abs;
      d.best_pg = d.pgn;
      d.stall = 0;
      if (d.pgn <= d.tau) finish(d, GPCG_OK);
      else start_gp(d);
      break;
    case PH_GP_ALPHA:
      gp_step(d, R[0], R[1]);
      break;
    case PH_GP_TRIAL: {
      const double gs = R[5], delta = gs + 0.5 * R[6];  // q(y') - q(y)
      if (delta <= S->mu * gs) {                         // eq. (gplsstop): accept
        d.cur ^= 1;
        set_face(d, R);
        d.gp_iters += 1;
        d.gp_accepts += 1;
        const double dec = -delta;
        // eqs. (pgstop1), (pgstop2), and the cap on iterates
        const bool stop = (R[7] == 0.0) || (d.gp_j >= 2 && dec <= S->eta1 * d.gp_decmax) ||
                          (d.gp_j >= S->max_gp);
        if (dec > d.gp_decmax) d.gp_decmax = dec;
        if (stop) end_gp(S, d);
        else {
          d.gp_j += 1;
          if (la) {  // the trial pass looked ahead
            d.lookaheads += 1;
            gp_step(d, R[8], R[9]);
          } else {
            d.phase = PH_GP_ALPHA;
          }
        }
      } else {
        d.alpha *= 0.5;
        d.backtracks += 1;
        d.bt += 1;
        if (d.bt > S->max_backtrack) end_gp(S, d);
      }
    } break;
    case PH_CG_INIT: {
      const int64_t m = (int64_t)R[2];
      if (m == 0) {
        if (d.gp_accepts == 0) finish(d, GPCG_STAGNATED);
        else start_gp(d);
        break;
      }
      d.cg_phases += 1;
      d.m_free = m;
      d.cg_j = 0;
      d.cg_decmax = -INFINITY;
      d.max_cg_eff = S->max_cg > 0 ? S->max_cg : (int32_t)m;
      d.first = 1;
      d.gamma = R[0];
      d.gamma0 = R[0];
      if (!(d.gamma > 0.0)) start_ps(d);  // r_k = 0: the CG direction is 0
      else if (!(R[1] > 0.0)) finish(d, GPCG_ERR_NOT_SPD);
      else {
        d.cg_alpha = d.gamma / R[1];
        d.cg_beta = 0.0;
        d.phase = S->list ? PH_CG_LIST : PH_CG_ITER;
      }
    } break;
    case PH_CG_LIST:
      d.phase = S->mrow ? PH_CG_MCOUNT : PH_CG_ITER;
      break;
    case PH_CG_MCOUNT:
      d.nnz_free = (int64_t)R[0];
      d.phase = PH_CG_MFILL;
      break;
    case PH_CG_MFILL:
      d.phase = PH_CG_ITER;
      break;
    case PH_CG_ITER: {
      d.cg_j += 1;
      d.cg_iters += 1;
      d.cg_free_rows += d.m_free;  // unknowns this CG pass swept with full traffic
      d.cg_free_nnz += d.nnz_free;
      const double dec = 0.5 * d.cg_alpha * d.gamma;  // q_k(w_{j-1}) - q_k(w_j)
      // eq. (cgstop1), or the residual test ||rho_j|| <= eta ||rho_0|| (M^-1 norm
      // with the preconditioner: gamma = rho'z)
      const bool test = S->cg_stop ? sqrt(R[0]) <= d.eta * sqrt(d.gamma0)
                                   : (d.cg_j >= 2 && dec <= d.eta * d.cg_decmax);
      const bool stop = (R[0] == 0.0) || test || (d.cg_j >= d.max_cg_eff);
      if (dec > d.cg_decmax) d.cg_decmax = dec;
      d.first = 0;
      if (stop) start_ps(d);
      else {
        const double beta = R[0] / d.gamma;
        const double pAp = R[1] - beta * R[0] / d.cg_alpha;  // p_{j+1}' A p_{j+1}
        // The recurrence can lose positivity by rounding once rho has nearly
        // vanished (FP32 sums in the mixed form); w_j is then still a descent
        // direction, so the CG phase ends with it.  Definiteness is checked
        // directly elsewhere: z'Az at the set-up pass and d'Ad at every
        // gradient-projection step.
        if (!(pAp > 0.0)) start_ps(d);
        else {
          d.cg_beta = beta;
          d.cg_alpha = R[0] / pAp;
          d.gamma = R[0];
        }
      }
    } break;
    case PH_PS_TRIAL: {
      const double gs = R[5], delta = gs + 0.5 * R[6];
      const bool acc = delta <= S->mu * gs;
      if (!acc) {
        d.alpha *= 0.5;
        d.backtracks += 1;
        d.bt += 1;
        if (d.bt <= S->max_backtrack) break;  // next trial
      }
      // the projected search has ended: x_{k+1} is known
      if (acc) {
        d.cur ^= 1;
        set_face(d, R);
      }
      d.ps_accepted = acc ? 1 : 0;
      d.outer_iters += 1;
      bool stalled = false;
      if (d.pgn < d.best_pg) {
        d.best_pg = d.pgn;
        d.stall = 0;
      } else {
        d.stall += 1;
        stalled = d.stall >= S->max_stall;
      }
      if (d.pgn <= d.tau) finish(d, GPCG_OK);
      else if (stalled || !acc) finish(d, GPCG_STAGNATED);
      else if (d.outer_iters >= S->max_outer) finish(d, GPCG_MAXIT);
      else if (d.n_nonbinding != 0) start_gp(d);  // B(x) != A(x)
      else {                                       // eq. (cgstop3): B(x) = A(x)
        d.eta *= S->eta2_reduce;
        d.face_repeats += 1;
        d.phase = PH_CG_INIT;
      }
    } break;
    default:
      break;
  }
}

// Runs the transition of the pending pass on the LDS copy of the state and
// books the pass in the per-phase counters (thread 0).  (A register copy of
// the core was measured slower in the fused kernel: more VGPRs everywhere.)
__device__ __forceinline__ void advance(const QPStatic *S, QPDyn &sd, const double *R,
                                       uint64_t now, bool la) {
  const int ph = sd.c.phase;
  transition(S, sd.c, R, la);
  if (ph >= 0 && ph < PH_COUNT) sd.pass_count[ph] += 1;
  const int bk = time_bucket(ph);
  if (sd.t_last) sd.t_bucket[bk] += now - sd.t_last;
  sd.t_last = now;
}

// The word a QP's solve leaves in its mapped host flag when it is done:
// nonzero, with the copy of x that holds the answer (bit 1) and the parity
// of the state copy that holds the final state (bit 2), so that the host can
// fetch both without waiting for the stream.
__device__ __forceinline__ int32_t done_word(int cur, int final_parity) {
  return 1 | (cur << 1) | (final_parity << 2);
}

// --------------------------------------------------------- state transfer

// The read-only part of a QP's state is copied into LDS with the dynamic
// part (by the top threads of the workgroup, in parallel), so the transition
// and the passes read options and array pointers without a global round trip.
constexpr int kStaticWords = (int)(sizeof(QPStatic) / 4);
static_assert(sizeof(QPStatic) % 4 == 0 && kStaticWords <= kBlock, "QPStatic copy");

__device__ __forceinline__ void copy_static(const QPStatic *src, QPStatic *dst) {
  const int w = (int)threadIdx.x - (kBlock - kStaticWords);
  if (w >= 0)
    reinterpret_cast<uint32_t *>(dst)[w] = reinterpret_cast<const uint32_t *>(src)[w];
}

constexpr int kDynWords = (int)(sizeof(QPDyn) / 4);
static_assert(sizeof(QPDyn) % 8 == 0, "QPDyn must be a whole number of words");
static_assert(kDynWords <= kBlock, "QPDyn must fit one word per thread");

__device__ __forceinline__ void copy_dyn(const QPDyn *src, QPDyn *dst) {
  if (threadIdx.x < kDynWords)
    reinterpret_cast<uint32_t *>(dst)[threadIdx.x] =
        reinterpret_cast<const uint32_t *>(src)[threadIdx.x];
}

// The LDS state into its global copy (global stores).
__device__ __forceinline__ void store_dyn(const QPDyn *lds, QPDyn *dst) {
  if (threadIdx.x < kDynWords)
    gbl(reinterpret_cast<uint32_t *>(dst))[threadIdx.x] =
        reinterpret_cast<const uint32_t *>(lds)[threadIdx.x];
}

// ------------------------------------------------------------------ kernels

// ------------------------------------------- speculative CG operand loads

// Element c (0 or 1) of a two-entry array held in registers, without a
// dynamic index (which would place the array in scratch memory).
template <typename T>
__device__ __forceinline__ T pick2(T const (&a)[2], int c) {
  return c ? a[1] : a[0];
}


// The CG view of a QP read from its static state (global memory or the LDS
// copy): the pointers of the CG precision CT.
template <typename CT>
__device__ __forceinline__ CGView make_cg_view(const QPStatic *S) {
  CGView V;
  V.op_kind = S->op_kind;
  V.nx = S->nx;
  V.ny = S->ny;
  V.div_shift = S->div_shift;
  V.div_magic = S->div_magic;
  V.n = S->n;
  V.w = sizeof(CT) == 4 ? (double)S->w32 : S->w;
  V.wx = sizeof(CT) == 4 ? (const void *)S->wx32 : (const void *)S->wx;
  V.wy = sizeof(CT) == 4 ? (const void *)S->wy32 : (const void *)S->wy;
  for (int c = 0; c < 2; ++c) {
    V.rho[c] = S->rho[c];
    V.uq[c] = S->uq[c];
    V.sq[c] = S->sq[c];
  }
  V.pv = S->pv;
  V.wv = S->wv;
  V.mask = S->mask;
  V.dinv = S->dinv;
  return V;
}

// Operands of one CG iteration at unknown k of a stencil operator.  They
// depend only on k and on the launch parity (the CG buffers alternate with
// it), so a workgroup can load them before it knows the state and hide their
// latency behind the slot reduction and the transition.
template <typename CT>
struct CGOperands {
  CT r, u, s, p, w;    // rho, A rho, A p (previous), p, w at k
  CT rS, uS, sS;       // the same three at the south neighbour k - nx (0 outside)
  CT rN, uN, sN;       // and at the north neighbour k + nx
  CT rX, uX, sX;       // first / last thread of the tile: at k - 1 / k + 1 (0 otherwise)
  CT wt[4];            // edge weights W, E, S, N (variable stencil)
  CT dk, dS, dN, dX;   // Jacobi preconditioner 1 / diag(A) at k, k - nx, k + nx, the outside row
  int m;               // free-set mask at k
  bool hasW, hasE, hasS, hasN;
};

// Loads the operands of one CG iteration at unknown k of a tile of kBlock
// consecutive unknowns.  The west and east neighbours are the neighbouring
// threads of the tile (exchanged through LDS after the update); only the
// first and last threads load the row outside the tile.  Every access is a
// global (not flat) load: it counts only against the vector memory counter,
// so the loads stay in flight across the workgroup barriers that wait for
// LDS traffic.
template <typename CT, bool PRE>
__device__ __forceinline__ void cg_prefetch(const CGView &V, int lpar, int64_t k,
                                            CGOperands<CT> &P) {
  const gptr<const CT> ro = gbl((const CT *)pick2(V.rho, lpar));
  const gptr<const CT> uo = gbl((const CT *)pick2(V.uq, lpar));
  const gptr<const CT> so = gbl((const CT *)pick2(V.sq, lpar));
  P.m = gbl(V.mask)[k];
  P.r = ro[k];
  P.u = uo[k];
  P.s = so[k];
  P.p = gbl((const CT *)V.pv)[k];
  P.w = gbl((const CT *)V.wv)[k];
  const int32_t nx = V.nx;
  const int32_t j = (int32_t)(((uint64_t)k * V.div_magic) >> V.div_shift);
  const int32_t i = (int32_t)(k - (int64_t)j * nx);
  P.hasW = i > 0;
  P.hasE = i < nx - 1;
  P.hasS = j > 0;
  P.hasN = j < V.ny - 1;
  P.rS = P.hasS ? ro[k - nx] : CT(0);
  P.uS = P.hasS ? uo[k - nx] : CT(0);
  P.sS = P.hasS ? so[k - nx] : CT(0);
  P.rN = P.hasN ? ro[k + nx] : CT(0);
  P.uN = P.hasN ? uo[k + nx] : CT(0);
  P.sN = P.hasN ? so[k + nx] : CT(0);
  int64_t kx = -1;
  if (threadIdx.x == 0 && P.hasW) kx = k - 1;
  if (threadIdx.x == kBlock - 1 && P.hasE) kx = k + 1;
  P.rX = kx >= 0 ? ro[kx] : CT(0);
  P.uX = kx >= 0 ? uo[kx] : CT(0);
  P.sX = kx >= 0 ? so[kx] : CT(0);
  if (PRE && V.dinv) {
    const gptr<const CT> dinv = gbl((const CT *)V.dinv);
    P.dk = dinv[k];
    P.dS = P.hasS ? dinv[k - nx] : CT(0);
    P.dN = P.hasN ? dinv[k + nx] : CT(0);
    P.dX = kx >= 0 ? dinv[kx] : CT(0);
  }
  if (V.op_kind == OPK_VAR) {
    const gptr<const CT> wx = gbl((const CT *)V.wx);
    const gptr<const CT> wy = gbl((const CT *)V.wy);
    const int64_t ex = (int64_t)j * (nx + 1) + i;
    P.wt[0] = wx[ex];
    P.wt[1] = wx[ex + 1];
    P.wt[2] = wy[k];
    P.wt[3] = wy[k + nx];
  }
}

// The CG iteration of run_pass on the prefetched operands of a tile, for
// every thread of the workgroup (own: k is an unknown of the QP).  Every
// updated residual rho_{i+1} is computed once, by its owner, and read by its
// west and east neighbours from LDS; the formulas and their order are those
// of the generic path, so the results are bitwise equal to it.
template <typename CT, bool PRE>
__device__ __forceinline__ void cg_iter_prefetched(const CGView &V, const QPCore &d, int lpar,
                                                   int64_t k, bool own, const CGOperands<CT> &P,
                                                   CT &gam, CT &del) {
  __shared__ CT s_z1[kBlock];
  const bool first = d.first != 0;
  const bool pre = PRE && V.dinv != nullptr;
  const CT al = (CT)d.cg_alpha, be = (CT)d.cg_beta;
  // s_i = u_i + beta s_{i-1} (= A p_i);  rho_{i+1} = rho_i - alpha s_i;
  // z = D^-1 rho with the Jacobi preconditioner, else rho; u = A z
  auto rnew = [&](CT r, CT u, CT sv) { return fmaT<CT>(-al, first ? u : fmaT<CT>(be, sv, u), r); };
  auto znew = [&](CT r, CT u, CT sv, CT dv) {
    const CT rn = rnew(r, u, sv);
    return pre ? rn * dv : rn;
  };
  const CT sk = first ? P.u : fmaT<CT>(be, P.s, P.u);
  const CT r1 = fmaT<CT>(-al, sk, P.r);
  const CT z1 = pre ? r1 * P.dk : r1;
  s_z1[threadIdx.x] = own ? z1 : CT(0);
  __syncthreads();
  const int t = (int)threadIdx.x;
  CT v[4];
  v[0] = !P.hasW ? CT(0) : (t > 0 ? s_z1[t - 1] : znew(P.rX, P.uX, P.sX, P.dX));
  v[1] = !P.hasE ? CT(0) : (t < kBlock - 1 ? s_z1[t + 1] : znew(P.rX, P.uX, P.sX, P.dX));
  v[2] = P.hasS ? znew(P.rS, P.uS, P.sS, P.dS) : CT(0);
  v[3] = P.hasN ? znew(P.rN, P.uN, P.sN, P.dN) : CT(0);
  __syncthreads();  // s_z1 is rewritten by the next tile
  if (!own || !P.m) return;
  const CT zk = pre ? P.r * P.dk : P.r;
  const CT pk = first ? zk : fmaT<CT>(be, P.p, zk);
  gbl((CT *)V.wv)[k] = fmaT<CT>(al, pk, P.w);
  gbl((CT *)V.pv)[k] = pk;
  gbl((CT *)pick2(V.sq, lpar ^ 1))[k] = sk;
  gbl((CT *)pick2(V.rho, lpar ^ 1))[k] = r1;
  CT u1;
  if (V.op_kind == OPK_CONST) {
    const CT w = (CT)V.w;
    u1 = w * ((z1 - v[0]) + (z1 - v[1]) + ((z1 - v[2]) + (z1 - v[3])));
  } else {
    u1 = (P.wt[0] * (z1 - v[0]) + P.wt[1] * (z1 - v[1])) +
         (P.wt[2] * (z1 - v[2]) + P.wt[3] * (z1 - v[3]));
  }
  gbl((CT *)pick2(V.uq, lpar ^ 1))[k] = u1;
  gam = fmaT<CT>(r1, z1, gam);
  del = fmaT<CT>(z1, u1, del);
}

// GP_ALPHA or GP_TRIAL over one 256-unknown chunk of a stencil QP (thread t:
// unknown k; own: k is an unknown of the tile).  The value each unknown
// contributes to its neighbours' rows -- the projected gradient d_k (GP_ALPHA)
// or the trial point and step (y_k, y_k - x_k) (GP_TRIAL) -- is evaluated
// once by its owner and read by the west and east neighbours from LDS; the
// values one grid row away, and beyond the chunk's first and last unknowns,
// are evaluated from global memory.  Every value and every row is the
// expression run_pass evaluates (apply_row / apply_row2), in the same order,
// so the sums are bitwise those of the generic path.  Every thread calls it.
__device__ __forceinline__ void gp_lean_chunk(const QPStatic *S, const QPCore &d, int phase,
                                              int64_t k, bool own, double (&acc)[kNP]) {
  __shared__ double s_va[kBlock], s_vb[kBlock];
  const int t = (int)threadIdx.x;
  const int c = d.cur;
  const gptr<const double> x = gbl((const double *)S->x[c]);
  const gptr<const double> g = gbl((const double *)S->g[c]);
  const gptr<const double> l = gbl(S->l), u = gbl(S->u);
  const bool trial = phase == PH_GP_TRIAL;
  const double a = d.alpha;
  const int32_t nx = S->nx;
  const int32_t j = own ? (int32_t)(((uint64_t)k * S->div_magic) >> S->div_shift) : 0;
  const int32_t i = own ? (int32_t)(k - (int64_t)j * nx) : 0;
  const bool hasW = own && i > 0, hasE = own && i < nx - 1;
  const bool hasS = own && j > 0, hasN = own && j < S->ny - 1;
  auto val = [&](int64_t m) {
    const double xm = x[m];
    if (trial) {
      const double ym = gp_point(xm, l[m], u[m], g[m], a);
      return Pair{ym, ym - xm};
    }
    return Pair{proj_grad(xm, l[m], u[m], g[m]), 0.0};
  };
  const Pair z{0.0, 0.0};
  const Pair cv = own ? val(k) : z;
  s_va[t] = cv.y;
  s_vb[t] = cv.s;
  const Pair So = hasS ? val(k - nx) : z;
  const Pair No = hasN ? val(k + nx) : z;
  const Pair Wx = (t == 0 && hasW) ? val(k - 1) : z;
  const Pair Ex = (t == kBlock - 1 && hasE) ? val(k + 1) : z;
  __syncthreads();
  const Pair W = !hasW ? z : (t > 0 ? Pair{s_va[t - 1], s_vb[t - 1]} : Wx);
  const Pair E = !hasE ? z : (t < kBlock - 1 ? Pair{s_va[t + 1], s_vb[t + 1]} : Ex);
  __syncthreads();  // the LDS rows are rewritten by the next chunk
  if (!own) return;
  Pair r;
  if (S->op_kind == OPK_CONST) {
    const double w = S->w;
    r.y = w * ((cv.y - W.y) + (cv.y - E.y) + ((cv.y - So.y) + (cv.y - No.y)));
    r.s = w * ((cv.s - W.s) + (cv.s - E.s) + ((cv.s - So.s) + (cv.s - No.s)));
  } else {
    const int64_t ex = (int64_t)j * (nx + 1) + i;
    const int64_t ey = (int64_t)j * nx + i;
    const gptr<const double> gx = gbl(S->wx), gy = gbl(S->wy);
    const double wW = gx[ex], wE = gx[ex + 1], wS = gy[ey], wN = gy[ey + nx];
    r.y = (wW * (cv.y - W.y) + wE * (cv.y - E.y)) + (wS * (cv.y - So.y) + wN * (cv.y - No.y));
    r.s = (wW * (cv.s - W.s) + wE * (cv.s - E.s)) + (wS * (cv.s - So.s) + wN * (cv.s - No.s));
  }
  if (!trial) {  // GP_ALPHA: d'd and d'Ad for eq. (bqpls)
    acc[0] = __fma_rn(cv.y, cv.y, acc[0]);
    acc[1] = __fma_rn(cv.y, r.y, acc[1]);
    return;
  }
  const double xk = x[k], lk = l[k], uk = u[k], gk = g[k], bk = gbl(S->b)[k];
  const double gyk = r.y - bk;
  gbl(S->x[c ^ 1])[k] = cv.y;
  gbl(S->g[c ^ 1])[k] = gyk;
  face_acc(cv.y, lk, uk, gyk, bk, acc);
  acc[5] = __fma_rn(gk, cv.s, acc[5]);
  acc[6] = __fma_rn(cv.s, r.s, acc[6]);
  acc[7] += (is_active(cv.y, lk, uk) != is_active(xk, lk, uk)) ? 1.0 : 0.0;
}

// Operands of a gradient-projection pass at unknown k of a stencil QP, loaded
// while the transition of the previous pass is still running: x, l, u, g at
// k and its west, east, south and north neighbours (index 0..4; 0 outside the
// grid), b at k, and the edge weights.  x and g are those of copy cp, the copy
// the next pass is predicted to read.
struct GPOperands {
  double x[5], l[5], u[5], g[5];
  double b;
  double wt[4];
  bool has[4];  // W, E, S, N inside the grid
};

__device__ __forceinline__ void gp_prefetch(const QPStatic *S, int cp, int64_t k, GPOperands &G) {
  const int32_t nx = S->nx;
  const int32_t j = (int32_t)(((uint64_t)k * S->div_magic) >> S->div_shift);
  const int32_t i = (int32_t)(k - (int64_t)j * nx);
  G.has[0] = i > 0;
  G.has[1] = i < nx - 1;
  G.has[2] = j > 0;
  G.has[3] = j < S->ny - 1;
  const int64_t nb[5] = {k, k - 1, k + 1, k - nx, k + nx};
  const gptr<const double> x = gbl((const double *)S->x[cp]);
  const gptr<const double> g = gbl((const double *)S->g[cp]);
  const gptr<const double> l = gbl(S->l), u = gbl(S->u);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const bool in = q == 0 || G.has[q - 1];
    G.x[q] = in ? x[nb[q]] : 0.0;
    G.l[q] = in ? l[nb[q]] : 0.0;
    G.u[q] = in ? u[nb[q]] : 0.0;
    G.g[q] = in ? g[nb[q]] : 0.0;
  }
  G.b = gbl(S->b)[k];
  if (S->op_kind == OPK_VAR) {
    const gptr<const double> wx = gbl(S->wx), wy = gbl(S->wy);
    const int64_t ex = (int64_t)j * (nx + 1) + i;
    G.wt[0] = wx[ex];
    G.wt[1] = wx[ex + 1];
    G.wt[2] = wy[k];
    G.wt[3] = wy[k + nx];
  }
}

// GP_ALPHA and GP_TRIAL of run_pass on prefetched operands (one unknown per
// thread, own: k is an unknown of the QP); the same formulas in the same
// order, so the results are bitwise equal.
__device__ __forceinline__ void gp_pass_prefetched(const QPStatic *S, const QPCore &d, int phase,
                                                   int64_t k, bool own, const GPOperands &G,
                                                   double (&acc)[kNP]) {
  if (!own) return;
  if (phase == PH_GP_ALPHA) {
    double dv[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) dv[q] = proj_grad(G.x[q], G.l[q], G.u[q], G.g[q]);
    const double Adk = row5(S, G.wt, G.has, dv[0], dv[1], dv[2], dv[3], dv[4]);
    acc[0] = __fma_rn(dv[0], dv[0], acc[0]);
    acc[1] = __fma_rn(dv[0], Adk, acc[1]);
    return;
  }
  // PH_GP_TRIAL
  const double a = d.alpha;
  double y[5], sv[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    y[q] = gp_point(G.x[q], G.l[q], G.u[q], G.g[q], a);
    sv[q] = y[q] - G.x[q];
  }
  const double Ay = row5(S, G.wt, G.has, y[0], y[1], y[2], y[3], y[4]);
  const double As = row5(S, G.wt, G.has, sv[0], sv[1], sv[2], sv[3], sv[4]);
  const double xk = G.x[0], lk = G.l[0], uk = G.u[0], gk = G.g[0], bk = G.b;
  const double gy = Ay - bk;
  gbl(S->x[d.cur ^ 1])[k] = y[0];
  gbl(S->g[d.cur ^ 1])[k] = gy;
  face_acc(y[0], lk, uk, gy, bk, acc);
  acc[5] = __fma_rn(gk, sv[0], acc[5]);
  acc[6] = __fma_rn(sv[0], As, acc[6]);
  acc[7] += (is_active(y[0], lk, uk) != is_active(xk, lk, uk)) ? 1.0 : 0.0;
}

// Stepped form: one launch = one pass of every QP of the launch; one
// workgroup = one tile.  Every workgroup first folds the previous launch's
// partial sums into its own copy of the state.
template <typename CT, bool SPEC, bool PRE, bool MAT = false>
__global__ __launch_bounds__(kBlock) void step_kernel(StepLaunch L) {
  __shared__ QPDyn sd;
  __shared__ QPStatic ss;
  __shared__ int s_fresh_done;
  // one QP (L.single): workgroup = tile; several QPs: workgroup = one-tile
  // entry of the item table (every workgroup folds its own QP's slots)
  const int wg = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  QPDev *q;
  int tile;
  if (L.single) {
    q = L.single;
    tile = wg;
  } else {
    const WgItem it = L.items[wg];
    q = it.q;
    tile = it.tile0;
  }
  const int par = L.parity;
  double *slots = tile_slots(q);
  // The state and the static part are copied first; the slots are loaded
  // once the state is in LDS, and only those the pending pass filled.
  // Issuing the slot loads together with the state loads (the order of the
  // transition kernel) gave, now and then, wrong sums in the second pass of a
  // solve that followed another solve on the same workspace (2048 tiles,
  // several XCDs reading slots the first pass had just written); this order
  // has not.
  {
    const int tid = (int)threadIdx.x;
    const int sw = tid - (kBlock - kStaticWords);
    uint32_t dw = 0, stw = 0;
    if (tid < kDynWords) dw = gbl(reinterpret_cast<const uint32_t *>(&q->dyn[par]))[tid];
    if (sw >= 0) stw = gbl(reinterpret_cast<const uint32_t *>(&q->st))[sw];
    if (tid < kDynWords) reinterpret_cast<uint32_t *>(&sd)[tid] = dw;
    if (sw >= 0) reinterpret_cast<uint32_t *>(&ss)[sw] = stw;
  }
  __asm__ volatile("" ::: "memory");  // the slot loads stay behind the copies
  const uint64_t clk = wall_clock64();
  // SPEC launches hold only stencil QPs with one unknown per thread; the CG
  // view is read from the state with uniform (scalar) loads
  const int64_t kk = (int64_t)tile * kBlock + threadIdx.x;
  const CGView V = make_cg_view<CT>(&q->st);
  const bool own = SPEC && kk < V.n;
  CGOperands<CT> P{};
  if (own) cg_prefetch<CT, PRE>(V, par, kk, P);
  __syncthreads();
  const QPStatic *S = &ss;
  const int ntiles = S->ntiles, mixed = S->mixed;
  // gradient-projection operands for the likely next pass, loaded while the
  // transition runs: after GP_ALPHA comes GP_TRIAL on the same copy of x, g;
  // after GP_TRIAL (accepted, the usual case) GP_ALPHA on the other copy
  GPOperands G;
  int gcp = -1;
  if (SPEC && sd.c.pending && !S->gp_la) {
    if (sd.c.phase == PH_GP_ALPHA) gcp = sd.c.cur;
    else if (sd.c.phase == PH_GP_TRIAL) gcp = sd.c.cur ^ 1;
    if (gcp >= 0 && own) gp_prefetch(S, gcp, kk, G);
  }
  double pf[kNP];
  prefetch_slots(slots, par, sd.c.pending ? nslots(sd.c.phase) : 0, pf);
  if (sd.c.pending) {
    double R[kNP];
    sum_partials(slots, par, ntiles, sd.c.phase, f32_slots(mixed, sd.c.phase), pf, R);
    if (threadIdx.x == 0) {
      advance(S, sd, R, clk, S->gp_la != 0);
      sd.c.pending = sd.c.phase == PH_DONE ? 0 : 1;
      s_fresh_done = sd.c.phase == PH_DONE;
    }
  } else if (threadIdx.x == 0) {
    s_fresh_done = 0;
    sd.c.pending = sd.c.phase == PH_DONE ? 0 : 1;
  }
  __syncthreads();
  const int phase = sd.c.phase;
  // the next launch's state: written now (the pass below only reads it)
  if (tile == 0) {
    store_dyn(&sd, &q->dyn[par ^ 1]);
    if (threadIdx.x == 0 && s_fresh_done && S->host_flag)
      __hip_atomic_store(S->host_flag, done_word(sd.c.cur, par ^ 1), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (phase != PH_DONE) {
    const int64_t k0 = (int64_t)tile * S->tile;
    const int64_t k1 = k0 + S->tile < S->n ? k0 + S->tile : S->n;
    double acc[kNP];
    float accf[2] = {0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < kNP; ++k) acc[k] = 0.0;
    if (SPEC && phase == PH_CG_ITER) {
      CT gam = CT(0), del = CT(0);
      cg_iter_prefetched<CT, PRE>(V, sd.c, par, kk, own, P, gam, del);
      if (sizeof(CT) == 4) {
        accf[0] = (float)gam;
        accf[1] = (float)del;
      } else {
        acc[0] = (double)gam;
        acc[1] = (double)del;
      }
    } else if (SPEC && gcp == sd.c.cur && (phase == PH_GP_ALPHA || phase == PH_GP_TRIAL)) {
      gp_pass_prefetched(S, sd.c, phase, kk, own, G, acc);
    } else {
      run_pass<CT, PRE, true, MAT>(S, slots, sd.c, phase, par, k0, k1, acc, accf);
    }
    write_partial(slots, par ^ 1, phase, f32_slots(mixed, phase), tile, acc, accf);
  }
}

// ------------------------------------------------------------ split form
// Large QPs and multi-QP launches run each pass as two launches: a transition
// kernel (one workgroup per QP) folds the previous pass's slots into the
// state, then a data kernel with one lean workgroup per tile runs the pass.
// Tiles, slot sums and formulas are those of the fused form, so a QP gives
// bitwise the same answer in either form.  Step parity p: the transition reads
// dyn[p] and slots[p] and writes dyn[p ^ 1]; the data kernel reads dyn[p ^ 1]
// and writes slots[p ^ 1]; CG buffers alternate with p as in the fused form.

// One workgroup per QP of the launch (L.single: grid 1; else grid nqp, QP b).
__global__ __launch_bounds__(kBlock) void transition_kernel(StepLaunch L) {
  __shared__ QPDyn sd;
  __shared__ QPStatic ss;
  __shared__ int s_fresh_done, s_base;
  const int par = L.parity;
  // queue form: the next transition appends to the other parity's queue,
  // which the data kernel before this one has finished reading
  if (L.queue && blockIdx.x == 0 && threadIdx.x == 0) L.qcount[par ^ 1] = 0;
  QPDev *q = L.single ? L.single : gbl(L.qps)[blockIdx.x];
  if (!q) return;  // an empty slot of the server's table
  const double *slots = tile_slots(q);
  // the state words, the static words and the slots are loaded together; the
  // LDS copies are written once they arrive
  const int tid = (int)threadIdx.x;
  const int sw = tid - (kBlock - kStaticWords);
  const uint32_t dyn_w = gbl(reinterpret_cast<const uint32_t *>(&q->dyn[par]))
      [tid < kDynWords ? tid : kDynWords - 1];
  const uint32_t st_w = gbl(reinterpret_cast<const uint32_t *>(&q->st))[sw >= 0 ? sw : 0];
  double pf[kNP];
  prefetch_slot(slots, par, pf);
  // one QP (its tile count is a launch argument): the two slots a CG pass
  // fills, of the tiles beyond the first 256, are loaded together with the
  // state, before the pass that filled them is known
  constexpr int kEarly = 20;  // tiles per thread: up to 21 x 256 tiles
  const int nt = L.single ? L.total_tiles : 0;
  const bool early = nt > kBlock && nt <= (kEarly + 1) * kBlock;
  double e0[kEarly], e1[kEarly];
  const gptr<const double> sl = gbl(slots);
#pragma unroll
  for (int m = 0; m < kEarly; ++m) {
    const int t = (int)threadIdx.x + (m + 1) * kBlock;
    e0[m] = (early && t < nt) ? sl[slot_index(t, par, 0)] : 0.0;
    e1[m] = (early && t < nt) ? sl[slot_index(t, par, 1)] : 0.0;
  }
  const uint64_t clk = wall_clock64();
  if (tid < kDynWords) reinterpret_cast<uint32_t *>(&sd)[tid] = dyn_w;
  if (sw >= 0) reinterpret_cast<uint32_t *>(&ss)[sw] = st_w;
  __syncthreads();
  const QPStatic *S = &ss;
  if (sd.c.pending) {
    double R[kNP];
    const int ph = sd.c.phase;
    const bool f32 = f32_slots(S->mixed, ph);
    if (early && nslots(ph) == 2) {
      // the sum of sum_partials, in its order, on the early loads
      float vf[2];
      const bool mine = (int)threadIdx.x < nt;
#pragma unroll
      for (int k = 0; k < kNP; ++k) R[k] = (mine && k < 2) ? pf[k] : 0.0;
      vf[0] = mine ? (float)pf[0] : 0.0f;
      vf[1] = mine ? (float)pf[1] : 0.0f;
#pragma unroll
      for (int m = 0; m < kEarly; ++m) {
        if ((int)threadIdx.x + (m + 1) * kBlock < nt) {
          R[0] += e0[m];
          R[1] += e1[m];
          vf[0] += (float)e0[m];
          vf[1] += (float)e1[m];
        }
      }
      block_slots(2, f32, R, vf);
    } else {
      sum_partials<true>(slots, par, S->ntiles, ph, f32, pf, R);
    }
    if (threadIdx.x == 0) {
      advance(S, sd, R, clk, false);
      sd.c.pending = sd.c.phase == PH_DONE ? 0 : 1;
      s_fresh_done = sd.c.phase == PH_DONE;
    }
  } else if (threadIdx.x == 0) {
    s_fresh_done = 0;
    sd.c.pending = sd.c.phase == PH_DONE ? 0 : 1;
  }
  __syncthreads();
  store_dyn(&sd, &q->dyn[par ^ 1]);
  if (threadIdx.x == 0 && s_fresh_done && S->host_flag) {
    __threadfence();
    __hip_atomic_store(S->host_flag, done_word(sd.c.cur, par ^ 1), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (L.queue && sd.c.phase != PH_DONE) {
    // queue form: this QP's work items for the data kernel of this launch
    const int T = L.item_tiles;
    const int ntiles = S->ntiles;
    const int nitems = (ntiles + T - 1) / T;
    if (threadIdx.x == 0) s_base = atomicAdd(&L.qcount[par], nitems);
    __syncthreads();
    WgItem *queue = L.queue + (int64_t)par * L.queue_cap;
    for (int i = tid; i < nitems; i += kBlock) {
      const int at = s_base + i;
      if (at < L.queue_cap) {
        WgItem it;
        it.q = q;
        it.tile0 = i * T;
        it.ntile = ntiles - i * T < T ? ntiles - i * T : T;
        queue[at] = it;
      }
    }
  }
}

constexpr int kCoreWords = (int)(sizeof(QPCore) / 4);
static_assert(sizeof(QPCore) % 4 == 0 && kCoreWords <= kBlock, "QPCore copy");

// One workgroup per work item: a run of consecutive tiles of one QP (one QP:
// tiles_per_wg tiles per workgroup; several QPs: the item table).  CG
// iterations of stencil QPs in the mask form take the lean path (operands of
// the tile, neighbours exchanged through LDS); with SPEC its loads for the
// first tile are issued before the state is read, which costs registers in
// every phase.  PART: kPartAll runs every pass; kPartCG only the lean CG
// iterations (the lean path alone needs far fewer registers, so more
// workgroups stay in flight); kPartRest every pass but those.
constexpr int kPartAll = 0, kPartCG = 1, kPartRest = 2;

// The pass of one work item (tiles [t0, t0 + nt) of QP q, clipped to its
// tiles) with its state in LDS (sc, S) and its CG view V.  With SPEC the
// operands of the first chunk are in P already (own: its unknown exists).
template <typename CT, bool SPEC, bool PRE, int PART, bool MAT, bool LGP = false>
__device__ __forceinline__ void pass_item(QPDev *q, int par, int t0, int nt, const QPCore &sc,
                                          const QPStatic *S, const CGView &V, int64_t kk,
                                          bool own, CGOperands<CT> &P) {
  const int phase = sc.phase;
  if (phase == PH_DONE) return;
  const int mixed = S->mixed, ntiles = S->ntiles;
  double *slots = tile_slots(q);
  const int t1 = t0 + nt < ntiles ? t0 + nt : ntiles;
  const bool lean = SPEC || (S->op_kind != OPK_CSR && S->list == nullptr);
  const bool lean_cg = phase == PH_CG_ITER && lean;
  if (PART == kPartCG && !lean_cg) return;
  if (PART == kPartRest && lean_cg) return;
  if (PART != kPartRest && lean_cg) {
    // a tile of several 256-unknown chunks accumulates them in order, as
    // run_pass does (thread t: unknowns k0 + t, k0 + t + 256, ...)
    const int nchunk = S->tile / kBlock;
    for (int tile = t0; tile < t1; ++tile) {
      CT gam = CT(0), del = CT(0);
      int c = 0;
      if (nchunk == 2 && (!SPEC || tile != t0)) {
        // two chunks: the operands of both are loaded before either is
        // used (twice the loads in flight), then the chunks run in order
        const int64_t ka = (int64_t)tile * S->tile + threadIdx.x, kb = ka + kBlock;
        const bool owna = ka < S->n, ownb = kb < S->n;
        CGOperands<CT> Q{};
        if (owna) cg_prefetch<CT, PRE>(V, par, ka, P);
        if (ownb) cg_prefetch<CT, PRE>(V, par, kb, Q);
        cg_iter_prefetched<CT, PRE>(V, sc, par, ka, owna, P, gam, del);
        cg_iter_prefetched<CT, PRE>(V, sc, par, kb, ownb, Q, gam, del);
        c = 2;
      }
      for (; c < nchunk; ++c) {
        if (!SPEC || tile != t0 || c != 0) {
          kk = (int64_t)tile * S->tile + (int64_t)c * kBlock + threadIdx.x;
          own = kk < S->n;
          if (own) cg_prefetch<CT, PRE>(V, par, kk, P);
        }
        cg_iter_prefetched<CT, PRE>(V, sc, par, kk, own, P, gam, del);
      }
      double acc[kNP];
      float accf[2] = {(float)gam, (float)del};
#pragma unroll
      for (int k = 0; k < kNP; ++k) acc[k] = 0.0;
      if (sizeof(CT) == 8) {
        acc[0] = (double)gam;
        acc[1] = (double)del;
      }
      write_partial(slots, par ^ 1, phase, f32_slots(mixed, phase), tile, acc, accf);
      if (tile + 1 < t1) __syncthreads();  // the reduction scratch is reused
    }
    return;
  }
  if constexpr (PART == kPartCG) return;
  if (LGP && (phase == PH_GP_ALPHA || phase == PH_GP_TRIAL) && S->op_kind != OPK_CSR) {
    const int nchunk = S->tile / kBlock;
    for (int tile = t0; tile < t1; ++tile) {
      const int64_t k0 = (int64_t)tile * S->tile;
      const int64_t k1 = k0 + S->tile < S->n ? k0 + S->tile : S->n;
      double acc[kNP];
      float accf[2] = {0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < kNP; ++k) acc[k] = 0.0;
      for (int c = 0; c < nchunk; ++c) {
        const int64_t k = k0 + (int64_t)c * kBlock + threadIdx.x;
        gp_lean_chunk(S, sc, phase, k, k < k1, acc);
      }
      write_partial(slots, par ^ 1, phase, f32_slots(mixed, phase), tile, acc, accf);
      if (tile + 1 < t1) __syncthreads();  // the reduction scratch is reused
    }
    return;
  }
  for (int tile = t0; tile < t1; ++tile) {
    const int64_t k0 = (int64_t)tile * S->tile;
    const int64_t k1 = k0 + S->tile < S->n ? k0 + S->tile : S->n;
    double acc[kNP];
    float accf[2] = {0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < kNP; ++k) acc[k] = 0.0;
    run_pass<CT, PRE, false, MAT>(S, slots, sc, phase, par, k0, k1, acc, accf);
    write_partial(slots, par ^ 1, phase, f32_slots(mixed, phase), tile, acc, accf);
    if (tile + 1 < t1) __syncthreads();  // the reduction scratch is reused
  }
}

template <typename CT, bool SPEC, bool PRE, int PART = kPartAll, bool MAT = false,
          bool QUEUE = false, bool LGP = false>
__global__ __launch_bounds__(kBlock, 4) void pass_kernel(StepLaunch L) {
  __shared__ QPCore sc;
  __shared__ QPStatic ss;
  const int wg = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int par = L.parity;
  const int tid = (int)threadIdx.x;
  const int sw = tid - (kBlock - kStaticWords);
  if constexpr (QUEUE) {
    // queue form: one workgroup per queued item (the grid covers the
    // largest possible queue; workgroups beyond the count return at once).
    // Items are dealt to the XCDs in contiguous runs over the count, so the
    // neighbouring tiles of a QP share an L2.
    const int count = L.qcount[par];
    if ((int)blockIdx.x >= count) return;
    const WgItem it = (L.queue + (int64_t)par * L.queue_cap)[xcd_tile((int)blockIdx.x, count)];
    QPDev *q = it.q;
    const uint32_t core_w = gbl(reinterpret_cast<const uint32_t *>(&q->dyn[par ^ 1].c))
        [tid < kCoreWords ? tid : kCoreWords - 1];
    const uint32_t st_w = gbl(reinterpret_cast<const uint32_t *>(&q->st))[sw >= 0 ? sw : 0];
    const CGView V = make_cg_view<CT>(&q->st);
    CGOperands<CT> P{};
    if (tid < kCoreWords) reinterpret_cast<uint32_t *>(&sc)[tid] = core_w;
    if (sw >= 0) reinterpret_cast<uint32_t *>(&ss)[sw] = st_w;
    __syncthreads();
    pass_item<CT, false, PRE, PART, MAT, LGP>(q, par, it.tile0, it.ntile, sc, &ss, V, 0, false, P);
  } else {
  QPDev *q;
  int t0, nt;
  if (L.single) {
    q = L.single;
    t0 = wg * L.tiles_per_wg;
    nt = L.tiles_per_wg;  // clipped to the QP's tiles below
  } else {
    const WgItem it = L.items[wg];
    q = it.q;
    t0 = it.tile0;
    nt = it.ntile;
  }
  // the state words and the early CG operands are loaded together; the LDS
  // copies are written once they arrive
  const uint32_t core_w = gbl(reinterpret_cast<const uint32_t *>(&q->dyn[par ^ 1].c))
      [tid < kCoreWords ? tid : kCoreWords - 1];
  const uint32_t st_w = gbl(reinterpret_cast<const uint32_t *>(&q->st))[sw >= 0 ? sw : 0];
  const int64_t kk = (int64_t)t0 * kBlock + threadIdx.x;
  // the CG view, read from the state before anything is stored (uniform:
  // scalar loads)
  const CGView V = make_cg_view<CT>(&q->st);
  const bool own = kk < V.n;
  CGOperands<CT> P{};
  if (SPEC && own) cg_prefetch<CT, PRE>(V, par, kk, P);
  if (tid < kCoreWords) reinterpret_cast<uint32_t *>(&sc)[tid] = core_w;
  if (sw >= 0) reinterpret_cast<uint32_t *>(&ss)[sw] = st_w;
  __syncthreads();
  pass_item<CT, SPEC, PRE, PART, MAT, LGP>(q, par, t0, nt, sc, &ss, V, kk, own, P);
  }
}

// Persistent form (batches of small QPs): one cooperative launch runs every
// QP to completion.  QP q owns the workgroup slots [wg_prefix[q],
// wg_prefix[q+1]); a workgroup sweeps the tiles lw, lw + nwg, ... of its QP
// in every pass, keeps the state in LDS, and meets the other workgroups of
// its QP at a counter barrier (no barrier spans two QPs).  The tiles and the
// order of every sum are those of the stepped form, so results are bitwise
// identical to it.  Every wait is bounded: after spin_limit polls the QP is
// failed with GPCG_ERR_HANG and the workgroup exits, so the grid drains.
template <typename CT, bool PRE>
__global__ __launch_bounds__(kBlock) void persistent_kernel(PersistLaunch P) {
  __shared__ QPDyn sd;
  __shared__ int s_exit;
  const int slot = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  if (slot >= P.wg_total) return;
  int lo = 0, hi = P.nqp;
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (P.wg_prefix[m] <= slot) lo = m;
    else hi = m;
  }
  QPDev *q = P.qps[lo];
  const QPStatic *S = &q->st;
  const int lw = slot - P.wg_prefix[lo];
  const int nwg = P.wg_prefix[lo + 1] - P.wg_prefix[lo];
  copy_dyn(&q->dyn[0], &sd);
  if (threadIdx.x == 0) s_exit = 0;
  __syncthreads();
  int par = 0;
  double *slots = tile_slots(q);
  for (uint32_t round = 1;; ++round) {
    if (sd.c.pending) {
      double R[kNP], pf[kNP];
      prefetch_slot(slots, par, pf);
      sum_partials(slots, par, S->ntiles, sd.c.phase, f32_slots(S->mixed, sd.c.phase), pf, R);
      if (threadIdx.x == 0) advance(S, sd, R, wall_clock64(), false);
      __syncthreads();
    }
    const int phase = sd.c.phase;
    if (phase == PH_DONE) break;
    for (int tile = lw; tile < S->ntiles; tile += nwg) {
      const int64_t k0 = (int64_t)tile * S->tile;
      const int64_t k1 = k0 + S->tile < S->n ? k0 + S->tile : S->n;
      double acc[kNP];
      float accf[2] = {0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < kNP; ++k) acc[k] = 0.0;
      run_pass<CT, PRE, false, true>(S, slots, sd.c, phase, par, k0, k1, acc, accf);
      write_partial(slots, par ^ 1, phase, f32_slots(S->mixed, phase), tile, acc, accf);
      __syncthreads();
    }
    if (threadIdx.x == 0) sd.c.pending = 1;
    par ^= 1;
    if (nwg > 1) {
      __threadfence();  // publish this workgroup's vector and slot stores
      __syncthreads();
      if (threadIdx.x == 0) {
        atomicAdd(&q->counter, 1u);
        const uint32_t target = (uint32_t)nwg * round;
        int64_t spins = 0;
        while (__hip_atomic_load(&q->counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
               target) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > P.spin_limit) {
            s_exit = 1;
            break;
          }
        }
        __threadfence();
      }
    }
    __syncthreads();
    if (s_exit) {
      if (threadIdx.x == 0) {
        sd.c.status = GPCG_ERR_HANG;
        sd.c.phase = PH_DONE;
      }
      __syncthreads();
      break;
    }
  }
  if (lw == 0) {
    if (threadIdx.x == 0) sd.c.pending = 0;
    __syncthreads();
    copy_dyn(&sd, &q->dyn[0]);
    copy_dyn(&sd, &q->dyn[1]);
    __syncthreads();
    if (threadIdx.x == 0 && S->host_flag) {
      __threadfence();
      __hip_atomic_store(S->host_flag, done_word(sd.c.cur, 0), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// Building blocks exposed through the C ABI.
template <typename T>
__global__ __launch_bounds__(kBlock) void spmv_kernel(const QPDev *q, const T *__restrict__ v,
                                                      T *__restrict__ y,
                                                      const uint8_t *__restrict__ mask) {
  const OpView<T> A = op_view<T>(&q->st);
  const int64_t n = q->st.n;
  auto vv = [&](int64_t j) { return v[j]; };
  for (int64_t k = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * kBlock + threadIdx.x;
       k < n; k += (int64_t)gridDim.x * kBlock) {
    if (mask && !mask[k]) {
      y[k] = T(0);
      continue;
    }
    y[k] = apply_row<T>(A, k, vv);
  }
}

// Vector-load variant for stencil operators with nx % V == 0: thread t owns
// the V consecutive unknowns k = V t .. V t + V - 1 of one grid row, loads
// them, the rows above and below and the mask with one V-wide access each,
// and evaluates every unknown with the expression of apply_row (bitwise the
// same result as spmv_kernel).
template <typename T, int V>
struct VecOf;
template <> struct VecOf<double, 2> { using type = double2; };
template <> struct VecOf<float, 4> { using type = float4; };
template <int V> struct MaskOf;
template <> struct MaskOf<2> { using type = uint16_t; };
template <> struct MaskOf<4> { using type = uint32_t; };

template <typename T, int V>
__global__ __launch_bounds__(kBlock) void spmv_stencil_kernel(const QPDev *q,
                                                              const T *__restrict__ v,
                                                              T *__restrict__ y,
                                                              const uint8_t *__restrict__ mask) {
  using VT = typename VecOf<T, V>::type;
  using MT = typename MaskOf<V>::type;
  const OpView<T> A = op_view<T>(&q->st);
  const int64_t n = q->st.n;
  const int64_t t = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * kBlock + threadIdx.x;
  const int64_t k = t * V;
  if (k >= n) return;
  const int32_t nx = A.nx;
  const int32_t j = (int32_t)(((uint64_t)k * A.magic) >> A.shift);
  const int32_t i = (int32_t)(k - (int64_t)j * nx);
  T c[V], s[V], nn[V], wv = T(0), ev = T(0);
  *reinterpret_cast<VT *>(c) = *reinterpret_cast<const VT *>(v + k);
  if (j > 0) *reinterpret_cast<VT *>(s) = *reinterpret_cast<const VT *>(v + k - nx);
  else
    for (int e = 0; e < V; ++e) s[e] = T(0);
  if (j < A.ny - 1) *reinterpret_cast<VT *>(nn) = *reinterpret_cast<const VT *>(v + k + nx);
  else
    for (int e = 0; e < V; ++e) nn[e] = T(0);
  if (i > 0) wv = v[k - 1];
  if (i + V < nx) ev = v[k + V];
  MT mbits = ~MT(0);
  if (mask) mbits = *reinterpret_cast<const MT *>(mask + k);
  T out[V];
  if (A.kind == OPK_CONST) {
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const T vW = e == 0 ? wv : c[e - 1];
      const T vE = e == V - 1 ? ev : c[e + 1];
      out[e] = A.w * ((c[e] - vW) + (c[e] - vE) + ((c[e] - s[e]) + (c[e] - nn[e])));
    }
  } else {
    const int64_t ex = (int64_t)j * (nx + 1) + i;
    T wx[V + 1], wS[V], wN[V];
#pragma unroll
    for (int e = 0; e <= V; ++e) wx[e] = A.wx[ex + e];
    *reinterpret_cast<VT *>(wS) = *reinterpret_cast<const VT *>(A.wy + k);
    *reinterpret_cast<VT *>(wN) = *reinterpret_cast<const VT *>(A.wy + k + nx);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const T vW = e == 0 ? wv : c[e - 1];
      const T vE = e == V - 1 ? ev : c[e + 1];
      out[e] = (wx[e] * (c[e] - vW) + wx[e + 1] * (c[e] - vE)) +
               (wS[e] * (c[e] - s[e]) + wN[e] * (c[e] - nn[e]));
    }
  }
#pragma unroll
  for (int e = 0; e < V; ++e)
    if (((mbits >> (8 * e)) & 0xFF) == 0) out[e] = T(0);
  // y is written once and not read by this kernel: streaming stores
#pragma unroll
  for (int e = 0; e < V; ++e) __builtin_nontemporal_store(out[e], y + k + e);
}

// Row-marching variant for grids whose vectors exceed the last-level cache.
// A workgroup owns a segment of kBlock * V consecutive unknowns of a grid row
// (thread t: the V unknowns from V t) over R consecutive rows.  Every row of v
// the segment touches (R + 2 of them, halo rows included) is loaded once, up
// front, and kept in registers, so each row of v is fetched once per
// workgroup instead of three times; west and east neighbours come from the
// adjacent lanes (lanes 0 and 63 load theirs).  Each unknown is evaluated
// with the expression of spmv_stencil_kernel, so the products are bitwise
// equal.  Rows past the grid height and columns past its width read as
// zeros and are not stored.  VARC: edge-weighted operator (a variant of its
// own, so that the constant stencil keeps its smaller register budget).  The
// operator view arrives by value (kernel arguments: no dependent load before
// the first row load).
template <typename T, int V, int R, bool VARC>
__global__ __launch_bounds__(kBlock) void spmv_march_kernel(const OpView<T> A,
                                                            const T *__restrict__ v,
                                                            T *__restrict__ y,
                                                            const uint8_t *__restrict__ mask,
                                                            int nseg) {
  using VT = typename VecOf<T, V>::type;
  using MT = typename MaskOf<V>::type;
  const int32_t nx = A.nx, ny = A.ny;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int seg = tile % nseg, rb = tile / nseg;
  const int32_t i0 = seg * (kBlock * V) + V * (int32_t)threadIdx.x;
  const bool act = i0 < nx;
  const int lane = (int)threadIdx.x & 63;
  const int32_t r0 = rb * R;
  T rows[R + 2][V];
#pragma unroll
  for (int e = 0; e < R + 2; ++e) {
    const int32_t j = r0 - 1 + e;
#pragma unroll
    for (int c = 0; c < V; ++c) rows[e][c] = T(0);
    if (act && j >= 0 && j < ny)
      *reinterpret_cast<VT *>(rows[e]) =
          *reinterpret_cast<const VT *>(v + (int64_t)j * nx + i0);
  }
  // mask bytes of the rows (0 where the row or column is outside the grid:
  // nothing is stored there)
  MT mk[R];
  if (mask) {
#pragma unroll
    for (int e = 0; e < R; ++e) {
      const int32_t j = r0 + e;
      mk[e] = (act && j < ny) ? *reinterpret_cast<const MT *>(mask + (int64_t)j * nx + i0)
                              : MT(0);
    }
  } else {
#pragma unroll
    for (int e = 0; e < R; ++e) mk[e] = MT(~MT(0));
  }
  // edge weights of y-edges: row j of wy (j = 0 .. ny) joins grid rows j - 1 and j
  T wyr[VARC ? R + 1 : 1][V];
  if (VARC) {
#pragma unroll
    for (int e = 0; e <= R; ++e) {
      const int32_t j = r0 + e;
#pragma unroll
      for (int c = 0; c < V; ++c) wyr[e][c] = T(0);
      if (act && j <= ny)
        *reinterpret_cast<VT *>(wyr[e]) =
            *reinterpret_cast<const VT *>(A.wy + (int64_t)j * nx + i0);
    }
  }
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const int32_t j = r0 + e;
    const bool live = act && j < ny;
    const int64_t k = (int64_t)j * nx + i0;
    const T *c = rows[e + 1], *s = rows[e], *nn = rows[e + 2];
    // west / east neighbours from the adjacent lanes; a lane past the grid
    // width holds zeros, the Dirichlet value east of the last column
    T wv = __shfl_up(c[V - 1], 1);
    T ev = __shfl_down(c[0], 1);
    if (lane == 0) wv = (live && i0 > 0) ? v[k - 1] : T(0);
    if (lane == 63) ev = (live && i0 + V < nx) ? v[k + V] : T(0);
    T out[V];
    if (!VARC) {
#pragma unroll
      for (int c2 = 0; c2 < V; ++c2) {
        const T vW = c2 == 0 ? wv : c[c2 - 1];
        const T vE = c2 == V - 1 ? ev : c[c2 + 1];
        out[c2] = A.w * ((c[c2] - vW) + (c[c2] - vE) + ((c[c2] - s[c2]) + (c[c2] - nn[c2])));
      }
    } else {
      const int64_t ex = (int64_t)j * (nx + 1) + i0;
      T wx[V + 1];
#pragma unroll
      for (int c2 = 0; c2 <= V; ++c2) wx[c2] = live ? A.wx[ex + c2] : T(0);
#pragma unroll
      for (int c2 = 0; c2 < V; ++c2) {
        const T vW = c2 == 0 ? wv : c[c2 - 1];
        const T vE = c2 == V - 1 ? ev : c[c2 + 1];
        out[c2] = (wx[c2] * (c[c2] - vW) + wx[c2 + 1] * (c[c2] - vE)) +
                  (wyr[e][c2] * (c[c2] - s[c2]) + wyr[e + 1][c2] * (c[c2] - nn[c2]));
      }
    }
#pragma unroll
    for (int c2 = 0; c2 < V; ++c2)
      if (((mk[e] >> (8 * c2)) & 0xFF) == 0) out[c2] = T(0);
    if (live)
#pragma unroll
      for (int c2 = 0; c2 < V; ++c2) __builtin_nontemporal_store(out[c2], y + k + c2);
  }
}

// kPgradUnroll unknowns per thread and loop trip (k, k + 256, ...): their
// loads are issued together, at clamped in-range indices, before any is used,
// so each thread keeps 4 * kPgradUnroll loads in flight.
constexpr int kPgradUnroll = 4;

// The face sums of unknown k in one thread's accumulators (in the order the
// thread meets its unknowns).
__device__ __forceinline__ void pgrad_add(double xk, double lk, double uk, double gk, double *pg,
                                          int64_t k, double (&acc)[4]) {
  const double p = proj_grad(xk, lk, uk, gk);
  if (pg) pg[k] = p;
  acc[0] = __fma_rn(p, p, acc[0]);
  acc[1] += (xk == lk) ? 1.0 : 0.0;
  acc[2] += (xk != lk && xk == uk) ? 1.0 : 0.0;
  acc[3] += (is_active(xk, lk, uk) && !is_binding(xk, lk, uk, gk)) ? 1.0 : 0.0;
}

// PAIR: x, l, u, g (and pg) are 16-byte aligned; each load brings two
// consecutive unknowns (2j, 2j + 1), kPgradUnroll pairs per thread and loop
// trip, so every thread keeps 4 * kPgradUnroll 16-byte loads in flight; an odd
// last unknown is added by thread 0 of workgroup 0 after its loop.
template <bool PAIR>
__global__ __launch_bounds__(kBlock) void pgrad_kernel(int64_t n, const double *__restrict__ x,
                                                       const double *__restrict__ l,
                                                       const double *__restrict__ u,
                                                       const double *__restrict__ g,
                                                       double *__restrict__ pg,
                                                       double *__restrict__ part) {
  constexpr int U = kPgradUnroll;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (PAIR) {
    const int64_t np = n / 2;
    const double2 *x2 = reinterpret_cast<const double2 *>(x);
    const double2 *l2 = reinterpret_cast<const double2 *>(l);
    const double2 *u2 = reinterpret_cast<const double2 *>(u);
    const double2 *g2 = reinterpret_cast<const double2 *>(g);
    const int64_t step = (int64_t)gridDim.x * kBlock * U;
    for (int64_t base = (int64_t)blockIdx.x * kBlock * U + threadIdx.x; base < np; base += step) {
      double2 xv[U], lv[U], uv[U], gv[U];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int64_t j = base + (int64_t)e * kBlock;
        const int64_t jc = j < np ? j : np - 1;
        xv[e] = x2[jc];
        lv[e] = l2[jc];
        uv[e] = u2[jc];
        gv[e] = g2[jc];
      }
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int64_t j = base + (int64_t)e * kBlock;
        if (j >= np) break;
        pgrad_add(xv[e].x, lv[e].x, uv[e].x, gv[e].x, pg, 2 * j, acc);
        pgrad_add(xv[e].y, lv[e].y, uv[e].y, gv[e].y, pg, 2 * j + 1, acc);
      }
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0)
      pgrad_add(x[n - 1], l[n - 1], u[n - 1], g[n - 1], pg, n - 1, acc);
  } else {
    const int64_t step = (int64_t)gridDim.x * kBlock * U;
    for (int64_t base = (int64_t)blockIdx.x * kBlock * U + threadIdx.x; base < n; base += step) {
      double xv[U], lv[U], uv[U], gv[U];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int64_t k = base + (int64_t)e * kBlock;
        const int64_t kc = k < n ? k : n - 1;
        xv[e] = x[kc];
        lv[e] = l[kc];
        uv[e] = u[kc];
        gv[e] = g[kc];
      }
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int64_t k = base + (int64_t)e * kBlock;
        if (k >= n) break;
        pgrad_add(xv[e], lv[e], uv[e], gv[e], pg, k, acc);
      }
    }
  }
  block_sum<double, 4>(acc);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) part[(int64_t)blockIdx.x * 4 + k] = acc[k];
}

__global__ __launch_bounds__(kBlock) void pgrad_final_kernel(int nblocks, const double *part,
                                                             double *out4) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < nblocks; t += kBlock)
    for (int k = 0; k < 4; ++k) v[k] += part[(int64_t)t * 4 + k];
  block_sum<double, 4>(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) out4[k] = v[k];
}

__global__ __launch_bounds__(kBlock) void convert_f32_kernel(const double *__restrict__ src,
                                                             float *__restrict__ dst,
                                                             int64_t count) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * kBlock)
    dst[k] = (float)src[k];
}

}  // namespace gpcg

// ------------------------------------------------------------ host launchers
using namespace gpcg;

// variant: kVarSpec | kVarPre bits
void *gpcg_step_kernel_ptr(int mixed, int variant) {
  const bool sp = variant & kVarSpec, pr = variant & kVarPre;
  if (variant & kVarMat) {
    if (mixed)
      return pr ? (void *)&step_kernel<float, false, true, true>
                : (void *)&step_kernel<float, false, false, true>;
    return pr ? (void *)&step_kernel<double, false, true, true>
              : (void *)&step_kernel<double, false, false, true>;
  }
  if (mixed) {
    if (sp) return pr ? (void *)&step_kernel<float, true, true> : (void *)&step_kernel<float, true, false>;
    return pr ? (void *)&step_kernel<float, false, true> : (void *)&step_kernel<float, false, false>;
  }
  if (sp) return pr ? (void *)&step_kernel<double, true, true> : (void *)&step_kernel<double, true, false>;
  return pr ? (void *)&step_kernel<double, false, true> : (void *)&step_kernel<double, false, false>;
}

static const void *persistent_ptr(int mixed, int pre) {
  if (mixed) return pre ? (const void *)&persistent_kernel<float, true> : (const void *)&persistent_kernel<float, false>;
  return pre ? (const void *)&persistent_kernel<double, true> : (const void *)&persistent_kernel<double, false>;
}

int gpcg_persistent_max_blocks(int mixed, int *blocks_per_cu) {
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu,
      persistent_ptr(mixed, 1),
      kBlock, 0);
  return e == hipSuccess ? 0 : -1;
}

int gpcg_launch_persistent(const PersistLaunch &P, int grid, int mixed, void *stream) {
  PersistLaunch arg = P;
  void *args[] = {&arg};
  hipError_t e = hipLaunchCooperativeKernel(
      persistent_ptr(mixed, P.pre),
      dim3(grid), dim3(kBlock), args, 0, (hipStream_t)stream);
  return e == hipSuccess ? 0 : -1;
}

void *gpcg_transition_kernel_ptr() { return (void *)&transition_kernel; }

template <int PART, bool QUEUE>
static void *pass_ptr_q(int mixed, int variant) {
  const bool sp = !QUEUE && (variant & kVarSpec), pr = variant & kVarPre;
  if constexpr (PART != kPartCG) {
    if ((variant & kVarLgp) && !sp && !(variant & kVarMat)) {
      if (mixed)
        return pr ? (void *)&pass_kernel<float, false, true, PART, false, QUEUE, true>
                  : (void *)&pass_kernel<float, false, false, PART, false, QUEUE, true>;
      return pr ? (void *)&pass_kernel<double, false, true, PART, false, QUEUE, true>
                : (void *)&pass_kernel<double, false, false, PART, false, QUEUE, true>;
    }
    if (variant & kVarMat) {
      if (mixed)
        return pr ? (void *)&pass_kernel<float, false, true, PART, true, QUEUE>
                  : (void *)&pass_kernel<float, false, false, PART, true, QUEUE>;
      return pr ? (void *)&pass_kernel<double, false, true, PART, true, QUEUE>
                : (void *)&pass_kernel<double, false, false, PART, true, QUEUE>;
    }
  }
  if (mixed) {
    if (sp)
      return pr ? (void *)&pass_kernel<float, true, true, PART, false, QUEUE>
                : (void *)&pass_kernel<float, true, false, PART, false, QUEUE>;
    return pr ? (void *)&pass_kernel<float, false, true, PART, false, QUEUE>
              : (void *)&pass_kernel<float, false, false, PART, false, QUEUE>;
  }
  if (sp)
    return pr ? (void *)&pass_kernel<double, true, true, PART, false, QUEUE>
              : (void *)&pass_kernel<double, true, false, PART, false, QUEUE>;
  return pr ? (void *)&pass_kernel<double, false, true, PART, false, QUEUE>
            : (void *)&pass_kernel<double, false, false, PART, false, QUEUE>;
}

template <int PART>
static void *pass_ptr(int mixed, int variant) {
  return (variant & kVarQueue) ? pass_ptr_q<PART, true>(mixed, variant)
                               : pass_ptr_q<PART, false>(mixed, variant);
}

void *gpcg_pass_kernel_ptr(int mixed, int variant) {
  return (variant & kVarCgk) ? pass_ptr<kPartCG>(mixed, variant)
                             : pass_ptr<kPartAll>(mixed, variant);
}

// The kernel of the passes the CG kernel skips: the early CG loads are of no
// use there.
void *gpcg_rest_kernel_ptr(int mixed, int variant) {
  return pass_ptr<kPartRest>(mixed, variant & (kVarPre | kVarMat | kVarQueue | kVarLgp));
}

int gpcg_launch_split(const StepLaunch &L, int mixed, int spec, void *stream) {
  if (L.data_grid < 1 || (!L.single && (!L.qps || (!L.items && !L.queue) || L.nqp < 1))) return -1;
  const int tgrid = L.single ? 1 : L.nqp;
  hipLaunchKernelGGL(transition_kernel, dim3(tgrid), dim3(kBlock), 0, (hipStream_t)stream, L);
  hipLaunchKernelGGL(reinterpret_cast<void (*)(StepLaunch)>(gpcg_pass_kernel_ptr(mixed, spec)),
                     dim3(L.data_grid), dim3(kBlock), 0, (hipStream_t)stream, L);
  if (spec & kVarCgk)
    hipLaunchKernelGGL(reinterpret_cast<void (*)(StepLaunch)>(gpcg_rest_kernel_ptr(mixed, spec)),
                       dim3(L.data_grid), dim3(kBlock), 0, (hipStream_t)stream, L);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int gpcg_launch_step(const StepLaunch &L, int mixed, int spec, void *stream) {
  // one QP: a workgroup per tile; several: a workgroup per one-tile item
  const int grid = L.single ? L.total_tiles : L.data_grid;
  if (grid <= 0 || (!L.single && !L.items)) return -1;
  hipLaunchKernelGGL(reinterpret_cast<void (*)(StepLaunch)>(gpcg_step_kernel_ptr(mixed, spec)),
                     dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, L);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

static int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

// The row-marching SpMV kernel is used when v, y and the mask together exceed
// this many bytes (the MI355X last-level cache); below it the one-row kernel
// keeps more workgroups in flight and is as fast or faster.
constexpr int64_t kMarchBytes = 256ll << 20;
constexpr int kMarchRows = 4;

int gpcg_launch_spmv(const QPDev *dqp, const QPStatic *S, int64_t n, const void *v, void *y,
                     const uint8_t *mask, int f32, int vec_nx, void *stream) {
  // vec_nx: the grid width of a stencil operator (0 for CSR); the V-wide
  // kernel needs whole vectors per grid row and aligned arrays
  const int V = f32 ? 4 : 2;
  const bool aligned = ((uintptr_t)v % (V * (f32 ? 4 : 8))) == 0 &&
                       ((uintptr_t)y % (V * (f32 ? 4 : 8))) == 0 &&
                       (!mask || ((uintptr_t)mask % V) == 0);
  if (vec_nx > 0 && vec_nx % V == 0 && aligned) {
    // vectors beyond the 256 MB last-level cache: each row fetched once
    const int64_t vec_bytes = n * (int64_t)(2 * (f32 ? 4 : 8) + 1);
    if (vec_bytes > kMarchBytes) {
      const int ny = (int)(n / vec_nx);
      const int nseg = (vec_nx + kBlock * V - 1) / (kBlock * V);
      const int64_t blocks = (int64_t)nseg * ((ny + kMarchRows - 1) / kMarchRows);
      if (blocks > 0x7fffffff) return -1;
      const dim3 g((unsigned)blocks), b(kBlock);
      const hipStream_t st = (hipStream_t)stream;
      const bool var_coef = S->op_kind == OPK_VAR;
      if (f32) {
        OpView<float> A{};
        A.kind = S->op_kind; A.nx = S->nx; A.ny = S->ny;
        A.w = S->w32; A.wx = S->wx32; A.wy = S->wy32;
        if (var_coef)
          hipLaunchKernelGGL((spmv_march_kernel<float, 4, kMarchRows, true>), g, b, 0, st, A,
                             (const float *)v, (float *)y, mask, nseg);
        else
          hipLaunchKernelGGL((spmv_march_kernel<float, 4, kMarchRows, false>), g, b, 0, st, A,
                             (const float *)v, (float *)y, mask, nseg);
      } else {
        OpView<double> A{};
        A.kind = S->op_kind; A.nx = S->nx; A.ny = S->ny;
        A.w = S->w; A.wx = S->wx; A.wy = S->wy;
        if (var_coef)
          hipLaunchKernelGGL((spmv_march_kernel<double, 2, kMarchRows, true>), g, b, 0, st, A,
                             (const double *)v, (double *)y, mask, nseg);
        else
          hipLaunchKernelGGL((spmv_march_kernel<double, 2, kMarchRows, false>), g, b, 0, st, A,
                             (const double *)v, (double *)y, mask, nseg);
      }
      return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    const int64_t groups = n / V;
    const int grid = (int)((groups + kBlock - 1) / kBlock);
    if (f32)
      hipLaunchKernelGGL((spmv_stencil_kernel<float, 4>), dim3(grid), dim3(kBlock), 0,
                         (hipStream_t)stream, dqp, (const float *)v, (float *)y, mask);
    else
      hipLaunchKernelGGL((spmv_stencil_kernel<double, 2>), dim3(grid), dim3(kBlock), 0,
                         (hipStream_t)stream, dqp, (const double *)v, (double *)y, mask);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  const int grid = grid_for(n);
  if (f32)
    hipLaunchKernelGGL(spmv_kernel<float>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, dqp,
                       (const float *)v, (float *)y, mask);
  else
    hipLaunchKernelGGL(spmv_kernel<double>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                       dqp, (const double *)v, (double *)y, mask);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

namespace {

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// The partial-sum kernel of the projected-gradient reduction: 16-byte loads
// of unknown pairs when every array is 16-byte aligned, else 8-byte loads.
// Returns the number of workgroups (at most kPgradMaxBlocks), whose partials
// land in part.
int launch_pgrad_partials(int64_t n, const double *x, const double *l, const double *u,
                          const double *g, double *pg, double *part, void *stream) {
  const bool pair = aligned16(x) && aligned16(l) && aligned16(u) && aligned16(g) &&
                    (!pg || aligned16(pg));
  const int64_t per_wg_trip = (int64_t)kPgradUnroll * (pair ? 2 : 1);
  int grid = grid_for((n + per_wg_trip - 1) / per_wg_trip);
  if (grid > kPgradMaxBlocks) grid = kPgradMaxBlocks;
  if (pair)
    hipLaunchKernelGGL(pgrad_kernel<true>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, n, x,
                       l, u, g, pg, part);
  else
    hipLaunchKernelGGL(pgrad_kernel<false>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, n,
                       x, l, u, g, pg, part);
  return grid;
}

}  // namespace

int gpcg_launch_pgrad(int64_t n, const double *x, const double *l, const double *u,
                      const double *g, double *pg, double *part, double *out4, void *stream) {
  if (n <= 0) return -1;
  const int grid = launch_pgrad_partials(n, x, l, u, g, pg, part, stream);
  hipLaunchKernelGGL(pgrad_final_kernel, dim3(1), dim3(kBlock), 0, (hipStream_t)stream, grid,
                     part, out4);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Scratch of the allocation-free projected-gradient entry point: the partial
// sums of at most kPgradMaxBlocks workgroups, then the four totals.  Every GPU
// the library runs on holds its own copy until the process ends; calls on one
// GPU share it (the last call's values stay).  Host code never passes the
// array's name to a kernel: that is a host-side stand-in, not the device
// address.  It uses the address hipGetSymbolAddress returns for the current
// device, looked up once per device.
static __device__ __align__(256) double scratch[kPgradScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices];  // per device: the device address of `scratch`
}  // namespace

// The device address of this device's scratch array, looked up on the first
// call with that device current; null on failure.
static double *scratch_on_current_device(int *err) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = -1;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      *err = -2;
      return nullptr;
    }
    g_scratch_ptr[dev] = (double *)p;
  }
  *err = 0;
  return g_scratch_ptr[dev];
}

int gpcg_launch_pgrad_scratch(int64_t n, const double *x, const double *l, const double *u,
                              const double *g, double *pg, const double **out4,
                              void *stream) {
  int err = 0;
  double *base = scratch_on_current_device(&err);
  if (!base) return err;
  if (n <= 0) return -3;
  double *part = base;
  double *tot = base + 4 * kPgradMaxBlocks;
  // every slot the final kernel reads (4 per launched workgroup) is written by
  // the first kernel: nothing needs clearing between calls
  const int grid = launch_pgrad_partials(n, x, l, u, g, pg, part, stream);
  hipLaunchKernelGGL(pgrad_final_kernel, dim3(1), dim3(kBlock), 0, (hipStream_t)stream, grid,
                     (const double *)part, tot);
  *out4 = tot;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// 1 / diag(A): stencils from their weights (the same sums as the diagonal of
// the assembled matrix), CSR from the stored diagonal entries of each row.
template <typename T>
__global__ __launch_bounds__(kBlock) void diag_inv_kernel(const QPDev *q, T *__restrict__ dinv) {
  const QPStatic *S = &q->st;
  const int64_t n = S->n;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kBlock) {
    double dg = 0.0;
    if (S->op_kind == OPK_CSR) {
      for (int32_t e = S->rowptr[k]; e < S->rowptr[k + 1]; ++e)
        if (S->colind[e] == (int32_t)k) dg += S->vals[e];
    } else if (S->op_kind == OPK_CONST) {
      dg = 4.0 * S->w;
    } else {
      const int32_t nx = S->nx;
      const int32_t j = (int32_t)(((uint64_t)k * S->div_magic) >> S->div_shift);
      const int32_t i = (int32_t)(k - (int64_t)j * nx);
      const int64_t ex = (int64_t)j * (nx + 1) + i;
      dg = (S->wx[ex] + S->wx[ex + 1]) + (S->wy[k] + S->wy[k + nx]);
    }
    dinv[k] = (T)(1.0 / dg);
  }
}

int gpcg_launch_diag_inv(const QPDev *dqp, void *dinv, int f32, void *stream) {
  const int grid = 1024;
  if (f32)
    hipLaunchKernelGGL(diag_inv_kernel<float>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                       dqp, (float *)dinv);
  else
    hipLaunchKernelGGL(diag_inv_kernel<double>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                       dqp, (double *)dinv);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// 8-byte words from src to dst: device memory, or mapped coherent host
// memory on the source side.  The library moves every piece of state and
// every table its kernels read with this kernel rather than with a copy
// engine: a later launch then sees the new contents however the lines were
// cached before (on this GPU, data that a DMA copy writes over lines a
// kernel has read has been seen stale by later kernels).
__global__ __launch_bounds__(kBlock) void copy_words_kernel(const uint64_t *src, uint64_t *dst,
                                                            int64_t words) {
  const gptr<const uint64_t> s = gbl(src);
  const gptr<uint64_t> d = gbl(dst);
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < words;
       k += (int64_t)gridDim.x * kBlock)
    d[k] = s[k];
}

int gpcg_launch_copy(void *dst, const void *src, size_t bytes, void *stream) {
  if (bytes == 0) return 0;
  if (bytes % 8 || (uintptr_t)dst % 8 || (uintptr_t)src % 8) return -1;
  const int64_t words = (int64_t)(bytes / 8);
  int64_t grid = (words + kBlock - 1) / kBlock;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(copy_words_kernel, dim3((unsigned)grid), dim3(kBlock), 0,
                     (hipStream_t)stream, (const uint64_t *)src, (uint64_t *)dst, words);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int gpcg_launch_convert_f32(const double *src, float *dst, int64_t count, void *stream) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(convert_f32_kernel, dim3(grid_for(count)), dim3(kBlock), 0,
                     (hipStream_t)stream, src, dst, count);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
