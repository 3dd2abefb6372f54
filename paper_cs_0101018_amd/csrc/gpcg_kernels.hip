// gpcg_kernels.hip -- HIP kernels of the GPCG hot path for gfx950 (CDNA4).
//
// One kernel, `step_kernel`, executes one *pass* of Algorithm GPCG (Section 3
// of the paper) for every QP of a launch.  A pass is a bandwidth-bound sweep
// over the unknowns: the operator (five-point stencil with constant or edge
// weights, or CSR) is applied row by row to a vector that is either loaded or
// computed on the fly from x, g, l, u (a projected-gradient direction or a
// trial step), fused with the elementwise updates and with the dot products
// the pass needs.  Reductions are deterministic: each workgroup reduces its
// tile with wave64 shuffles and LDS into a fixed slot, and the last workgroup
// to arrive sums the slots in tile order.  That workgroup then runs the
// scalar transition of the GPCG state machine (which pass comes next, the
// step lengths, the stop tests eqs. (pgstop1), (pgstop2), (cgstop1),
// (cgstop3) and the termination test (bqp_approximate_sol)).
//
// No MFMA: nothing on this path is a dense contraction.  Memory traffic is the
// bound; see the per-pass byte counts in the runtime.
#include <hip/hip_runtime.h>
#include <math.h>

#include "gpcg_internal.h"
#include "../../include/gpcg.h"

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
// P[x + alpha w] (eq. cglsstop2).  Written once so that every workgroup that
// needs the value at index j (owner or stencil neighbour) gets the same bits.
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

// ------------------------------------------------------------------ operator

template <typename T>
struct OpView {
  int32_t kind, nx, ny;
  int32_t shift;
  uint64_t magic;
  T w;
  const T *wx, *wy;
  const int32_t *rowptr, *colind;
  const T *vals;
};

template <typename T>
__device__ __forceinline__ OpView<T> op_view(const QPState *q);

template <>
__device__ __forceinline__ OpView<double> op_view<double>(const QPState *q) {
  OpView<double> A;
  A.kind = q->op_kind; A.nx = q->nx; A.ny = q->ny; A.shift = q->div_shift; A.magic = q->div_magic;
  A.w = q->w; A.wx = q->wx; A.wy = q->wy; A.rowptr = q->rowptr; A.colind = q->colind;
  A.vals = q->vals;
  return A;
}

template <>
__device__ __forceinline__ OpView<float> op_view<float>(const QPState *q) {
  OpView<float> A;
  A.kind = q->op_kind; A.nx = q->nx; A.ny = q->ny; A.shift = q->div_shift; A.magic = q->div_magic;
  A.w = q->w32; A.wx = q->wx32; A.wy = q->wy32; A.rowptr = q->rowptr; A.colind = q->colind;
  A.vals = q->vals32;
  return A;
}

// Row k of A applied to the vector whose entries the functor v returns.
//  stencil: (A v)_k = sum_e w_e (v_k - v_nb(e)), v_nb = 0 outside the grid
//  CSR:     (A v)_k = sum_e vals_e v_{colind_e}
template <typename T, class F>
__device__ __forceinline__ T apply_row(const OpView<T> &A, int64_t k, F v) {
  if (A.kind == OPK_CSR) {
    T s = T(0);
    const int32_t e0 = A.rowptr[k], e1 = A.rowptr[k + 1];
    for (int32_t e = e0; e < e1; ++e) s = fmaT<T>(A.vals[e], v((int64_t)A.colind[e]), s);
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
  const T wW = A.wx[ex], wE = A.wx[ex + 1], wS = A.wy[ey], wN = A.wy[ey + nx];
  return (wW * (c - vW) + wE * (c - vE)) + (wS * (c - vS) + wN * (c - vN));
}

// ---------------------------------------------------------------- reductions

// Sum of N values over the workgroup; the result is valid in thread 0.  The
// order of additions is fixed (butterfly in each wave64, then waves 0..3).
template <typename R, int N>
__device__ __forceinline__ void block_sum(R (&v)[N]) {
  __shared__ R sh[kBlock / 64][N];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) sh[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
  __syncthreads();
}

// Map the launch index of a workgroup to a tile so that consecutive tiles land
// on the same XCD: gfx950 dispatches workgroups round-robin over its 8 XCDs,
// each with its own L2, and stencil neighbours of a tile live in the tiles
// next to it.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  constexpr int X = 8;
  const int xcd = b % X, local = b / X;
  const int per = G / X, rem = G % X;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Which reduction type a pass uses: FP32 for the CG passes of the mixed form.
__device__ __forceinline__ bool f32_pass(int mixed, int phase) {
  return mixed && (phase == PH_CG_INIT || phase == PH_CG_A || phase == PH_CG_B);
}

// ------------------------------------------------------------------- passes

template <typename CT>
struct Vecs {
  CT *w, *r, *pold, *pnew;
};

template <typename CT>
__device__ __forceinline__ Vecs<CT> cg_vecs(const QPState *q) {
  Vecs<CT> V;
  V.w = (CT *)q->vw;
  V.r = (CT *)q->vr;
  CT *p0 = (CT *)q->vp0, *p1 = (CT *)q->vp1;
  V.pold = q->pcur ? p1 : p0;
  V.pnew = q->pcur ? p0 : p1;
  return V;
}

// One pass over the unknowns [k0, k1) of QP q; fills acc (this thread's part).
template <typename CT>
__device__ void run_pass(const QPState *__restrict__ q, int phase, int64_t k0, int64_t k1,
                         double (&acc)[kNP], float (&accf)[kNP]) {
  const double *__restrict__ l = q->l;
  const double *__restrict__ u = q->u;
  const double *__restrict__ b = q->b;
  double *__restrict__ x = q->x;
  double *__restrict__ g = q->g;
  const int64_t s = kBlock;
  switch (phase) {
    case PH_PROJECT: {
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) {
        const double x0 = x[k], lk = l[k], uk = u[k], bk = b[k];
        acc[1] += (isnan(x0) || isnan(lk) || isnan(uk) || isnan(bk)) ? 1.0 : 0.0;
        acc[0] += (lk > uk) ? 1.0 : 0.0;
        const double xn = mid3(lk, uk, x0);
        acc[2] += (xn != x0) ? 1.0 : 0.0;
        x[k] = xn;
      }
    } break;
    case PH_GRAD: {
      const OpView<double> A = op_view<double>(q);
      auto xv = [&](int64_t j) { return x[j]; };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) {
        const double xk = x[k], lk = l[k], uk = u[k], bk = b[k];
        const double gk = apply_row<double>(A, k, xv) - bk;
        g[k] = gk;
        const double pg = proj_grad(xk, lk, uk, gk);
        acc[0] = __fma_rn(pg, pg, acc[0]);
        acc[1] += (xk == lk) ? 1.0 : 0.0;
        acc[2] += (xk != lk && xk == uk) ? 1.0 : 0.0;
        acc[3] += (is_active(xk, lk, uk) && !is_binding(xk, lk, uk, gk)) ? 1.0 : 0.0;
        acc[4] = __fma_rn(xk, gk - bk, acc[4]);
      }
    } break;
    case PH_GP_ALPHA: {
      const OpView<double> A = op_view<double>(q);
      auto dv = [&](int64_t j) { return proj_grad(x[j], l[j], u[j], g[j]); };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) {
        const double dk = dv(k);
        const double Adk = apply_row<double>(A, k, dv);
        acc[0] = __fma_rn(dk, dk, acc[0]);
        acc[1] = __fma_rn(dk, Adk, acc[1]);
      }
    } break;
    case PH_GP_TRIAL: {
      const OpView<double> A = op_view<double>(q);
      const double a = q->alpha;
      auto sv = [&](int64_t j) {
        const double yj = x[j];
        return gp_point(yj, l[j], u[j], g[j], a) - yj;
      };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) {
        const double yk = x[k], lk = l[k], uk = u[k], gk = g[k];
        const double yn = gp_point(yk, lk, uk, gk, a);
        const double sk = yn - yk;
        const double Ask = apply_row<double>(A, k, sv);
        acc[0] = __fma_rn(gk, sk, acc[0]);
        acc[1] = __fma_rn(sk, Ask, acc[1]);
        acc[2] += (is_active(yn, lk, uk) != is_active(yk, lk, uk)) ? 1.0 : 0.0;
      }
    } break;
    case PH_GP_ACCEPT: {
      const double a = q->alpha;
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) x[k] = gp_point(x[k], l[k], u[k], g[k], a);
    } break;
    case PH_CG_INIT: {
      const Vecs<CT> V = cg_vecs<CT>(q);
      CT *p0 = (CT *)q->vp0, *p1 = (CT *)q->vp1;
      uint8_t *mask = q->mask;
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) {
        const double xk = x[k];
        const bool fr = l[k] < xk && xk < u[k];
        const CT rk = fr ? (CT)(-g[k]) : CT(0);
        mask[k] = fr ? 1 : 0;
        V.r[k] = rk;
        V.w[k] = CT(0);
        if (!fr) {
          p0[k] = CT(0);
          p1[k] = CT(0);
        }
        if (sizeof(CT) == 4) accf[0] = fmaT<float>((float)rk, (float)rk, accf[0]);
        else acc[0] = __fma_rn((double)rk, (double)rk, acc[0]);
        acc[1] += fr ? 1.0 : 0.0;
      }
    } break;
    case PH_CG_A: {
      const OpView<CT> A = op_view<CT>(q);
      const Vecs<CT> V = cg_vecs<CT>(q);
      const uint8_t *mask = q->mask;
      const bool first = q->first_cg != 0;
      const CT beta = (CT)q->beta;
      auto pn = [&](int64_t j) { return first ? V.r[j] : fmaT<CT>(beta, V.pold[j], V.r[j]); };
      CT sum = CT(0);
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) {
        if (!mask[k]) continue;  // r, w, p are zero on the active set
        const CT pk = pn(k);
        V.pnew[k] = pk;
        const CT Apk = apply_row<CT>(A, k, pn);
        sum = fmaT<CT>(pk, Apk, sum);
      }
      if (sizeof(CT) == 4) accf[0] = (float)sum;
      else acc[0] = (double)sum;
    } break;
    case PH_CG_B: {
      const OpView<CT> A = op_view<CT>(q);
      const Vecs<CT> V = cg_vecs<CT>(q);
      const uint8_t *mask = q->mask;
      const CT a = (CT)q->cg_alpha;
      const CT *__restrict__ p = V.pnew;
      auto pv = [&](int64_t j) { return p[j]; };
      CT sum = CT(0);
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) {
        if (!mask[k]) continue;
        const CT pk = p[k];
        const CT Apk = apply_row<CT>(A, k, pv);
        V.w[k] = fmaT<CT>(a, pk, V.w[k]);
        const CT rk = fmaT<CT>(-a, Apk, V.r[k]);
        V.r[k] = rk;
        sum = fmaT<CT>(rk, rk, sum);
      }
      if (sizeof(CT) == 4) accf[0] = (float)sum;
      else acc[0] = (double)sum;
    } break;
    case PH_PS_TRIAL: {
      const OpView<double> A = op_view<double>(q);
      const CT *__restrict__ w = (const CT *)q->vw;
      const uint8_t *mask = q->mask;
      const double a = q->alpha;
      auto sv = [&](int64_t j) {
        if (!mask[j]) return 0.0;  // the CG direction is zero on A(x_k)
        const double xj = x[j];
        return ps_point(xj, l[j], u[j], (double)w[j], a) - xj;
      };
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s) {
        if (!mask[k]) continue;
        const double sk = sv(k);
        const double Ask = apply_row<double>(A, k, sv);
        acc[0] = __fma_rn(g[k], sk, acc[0]);
        acc[1] = __fma_rn(sk, Ask, acc[1]);
      }
    } break;
    case PH_PS_ACCEPT: {
      const CT *__restrict__ w = (const CT *)q->vw;
      const uint8_t *mask = q->mask;
      const double a = q->alpha;
      for (int64_t k = k0 + threadIdx.x; k < k1; k += s)
        if (mask[k]) x[k] = ps_point(x[k], l[k], u[k], (double)w[k], a);
    } break;
    default:
      break;
  }
}

// ------------------------------------------------------ the scalar transition

__device__ __forceinline__ int time_bucket(int phase, int ctx) {
  switch (phase) {
    case PH_CG_INIT: case PH_CG_A: case PH_CG_B: return TB_CG;
    case PH_GP_ALPHA: case PH_GP_TRIAL: case PH_GP_ACCEPT: return TB_GP;
    case PH_PS_TRIAL: case PH_PS_ACCEPT: return TB_SEARCH;
    case PH_GRAD: return ctx == CTX_GP ? TB_GP : (ctx == CTX_PS ? TB_SEARCH : TB_OTHER);
    default: return TB_OTHER;
  }
}

__device__ void finish(QPState *q, int status) {
  q->status = status;
  q->phase = PH_DONE;
  if (q->host_flag)
    __hip_atomic_store(q->host_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A gradient-projection phase begins: y_0 = x_k (Algorithm GPCG, first bullet).
__device__ void start_gp(QPState *q) {
  q->gp_j = 1;
  q->gp_decmax = -INFINITY;
  q->gp_accepts = 0;
  q->phase = PH_GP_ALPHA;
}

// The gradient-projection phase ends: termination test, then CG with the
// initial eta2 (it is reset whenever a gradient-projection phase runs).
__device__ void end_gp(QPState *q) {
  if (q->pgn <= q->tau) {
    finish(q, GPCG_OK);
    return;
  }
  q->eta = q->eta2;
  q->phase = PH_CG_INIT;
}

// Projected search along d_k = Z_k w: alpha = 1, 1/2, 1/4, ... (eq. cglsstop2).
__device__ void start_ps(QPState *q) {
  q->alpha = 1.0;
  q->bt = 0;
  q->ps_accepted = 0;
  q->phase = PH_PS_TRIAL;
}

// Runs in one thread after the pass `phase` of QP q has been reduced into r.
__device__ void transition(QPState *q, int phase, const double *r) {
  const uint64_t now = wall_clock64();
  if (q->t_last) q->t_bucket[time_bucket(phase, q->ctx)] += now - q->t_last;
  q->t_last = now;
  q->passes += 1;
  q->pass_count[phase] += 1;
  switch (phase) {
    case PH_PROJECT:
      if (r[1] > 0.0) { finish(q, GPCG_ERR_NAN); break; }
      if (r[0] > 0.0) { finish(q, GPCG_ERR_BOUNDS); break; }
      q->x0_projected = r[2] > 0.0 ? 1 : 0;
      q->phase = PH_GRAD;
      q->ctx = CTX_INIT;
      break;
    case PH_GRAD: {
      q->pgn = sqrt(r[0]);
      q->n_lower = (int64_t)r[1];
      q->n_upper = (int64_t)r[2];
      q->n_nonbinding = (int64_t)r[3];
      q->q = 0.5 * r[4];
      if (q->ctx == CTX_INIT) {
        q->pg0 = q->pgn;
        double tau = q->tol_abs;
        if (q->tol_rel * q->pgn > tau) tau = q->tol_rel * q->pgn;
        q->tau = tau;
        q->best_pg = q->pgn;
        q->stall = 0;
        if (q->pgn <= tau) finish(q, GPCG_OK);
        else start_gp(q);
      } else if (q->ctx == CTX_GP) {
        // y_j accepted and its gradient known: eqs. (pgstop1), (pgstop2)
        q->gp_iters += 1;
        q->gp_accepts += 1;
        const double dec = q->pend_dec;
        const bool stop = (q->pend_nchg == 0) ||
                          (q->gp_j >= 2 && dec <= q->eta1 * q->gp_decmax) ||
                          (q->gp_j >= q->max_gp);
        if (dec > q->gp_decmax) q->gp_decmax = dec;
        if (stop) end_gp(q);
        else {
          q->gp_j += 1;
          q->phase = PH_GP_ALPHA;
        }
      } else {
        // x_{k+1} known: termination test, then eq. (cgstop3)
        q->outer_iters += 1;
        bool stalled = false;
        if (q->pgn < q->best_pg) {
          q->best_pg = q->pgn;
          q->stall = 0;
        } else {
          q->stall += 1;
          stalled = q->stall >= q->max_stall;
        }
        if (q->pgn <= q->tau) finish(q, GPCG_OK);
        else if (stalled) finish(q, GPCG_STAGNATED);
        else if (!q->ps_accepted) finish(q, GPCG_STAGNATED);
        else if (q->outer_iters >= q->max_outer) finish(q, GPCG_MAXIT);
        else if (q->n_nonbinding != 0) start_gp(q);
        else {
          q->eta *= q->eta2_reduce;
          q->face_repeats += 1;
          q->phase = PH_CG_INIT;
        }
      }
    } break;
    case PH_GP_ALPHA:
      if (r[0] == 0.0) finish(q, GPCG_OK);  // P grad q(y) = 0: y solves the QP
      else if (!(r[1] > 0.0)) finish(q, GPCG_ERR_NOT_SPD);
      else {
        q->alpha = r[0] / r[1];  // eq. (bqpls): ||d||^2 / d'Ad
        q->bt = 0;
        q->phase = PH_GP_TRIAL;
      }
      break;
    case PH_GP_TRIAL: {
      const double delta = r[0] + 0.5 * r[1];  // q(y') - q(y)
      if (delta <= q->mu * r[0]) {             // eq. (gplsstop)
        q->pend_dec = -delta;
        q->pend_nchg = (int64_t)r[2];
        q->phase = PH_GP_ACCEPT;
      } else {
        q->alpha *= 0.5;
        q->backtracks += 1;
        q->bt += 1;
        if (q->bt > q->max_backtrack) end_gp(q);
      }
    } break;
    case PH_GP_ACCEPT:
      q->phase = PH_GRAD;
      q->ctx = CTX_GP;
      break;
    case PH_CG_INIT: {
      q->m_free = (int64_t)r[1];
      if (q->m_free == 0) {
        if (q->gp_accepts == 0) finish(q, GPCG_STAGNATED);
        else start_gp(q);
        break;
      }
      q->cg_phases += 1;
      q->rr = r[0];
      q->cg_j = 0;
      q->cg_decmax = -INFINITY;
      q->max_cg_eff = q->max_cg > 0 ? q->max_cg : (int32_t)q->m_free;
      q->first_cg = 1;
      if (q->rr > 0.0) q->phase = PH_CG_A;
      else start_ps(q);
    } break;
    case PH_CG_A:
      if (!(r[0] > 0.0)) finish(q, GPCG_ERR_NOT_SPD);
      else {
        q->cg_alpha = q->rr / r[0];
        q->phase = PH_CG_B;
      }
      q->cg_free_rows += q->m_free;
      break;
    case PH_CG_B: {
      q->cg_j += 1;
      q->cg_iters += 1;
      q->cg_free_rows += q->m_free;
      const double dec = 0.5 * q->cg_alpha * q->rr;  // q_k(w_{j-1}) - q_k(w_j)
      const bool stop = (r[0] == 0.0) || (q->cg_j >= 2 && dec <= q->eta * q->cg_decmax) ||
                        (q->cg_j >= q->max_cg_eff);  // eq. (cgstop1)
      if (dec > q->cg_decmax) q->cg_decmax = dec;
      q->pcur ^= 1;
      if (stop) start_ps(q);
      else {
        q->beta = r[0] / q->rr;
        q->rr = r[0];
        q->first_cg = 0;
        q->phase = PH_CG_A;
      }
    } break;
    case PH_PS_TRIAL: {
      q->cg_free_rows += q->m_free;
      const double delta = r[0] + 0.5 * r[1];
      if (delta <= q->mu * r[0]) {
        q->ps_accepted = 1;
        q->phase = PH_PS_ACCEPT;
      } else {
        q->alpha *= 0.5;
        q->backtracks += 1;
        q->bt += 1;
        if (q->bt > q->max_backtrack) {
          q->ps_accepted = 0;  // x stays; the gradient pass decides
          q->phase = PH_GRAD;
          q->ctx = CTX_PS;
        }
      }
    } break;
    case PH_PS_ACCEPT:
      q->cg_free_rows += q->m_free;
      q->phase = PH_GRAD;
      q->ctx = CTX_PS;
      break;
    default:
      break;
  }
}

// ------------------------------------------------------------ one workgroup

// Reduces this workgroup's share of a tile into partials[tile] (thread 0
// writes the slot).  The per-tile value does not depend on which workgroup
// or which launch form computed it.
__device__ __forceinline__ void tile_partial(QPState *q, bool f32, int tile, double (&acc)[kNP],
                                             float (&accf)[kNP]) {
  if (f32) {
    block_sum<float, kNP>(accf);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < kNP; ++k) acc[k] = (double)accf[k];
  } else {
    block_sum<double, kNP>(acc);
  }
  if (threadIdx.x == 0) {
    double *slot = q->partials + (int64_t)tile * kNP;
#pragma unroll
    for (int k = 0; k < kNP; ++k) slot[k] = acc[k];
  }
}

// Arrives at the QP's ticket; if this is the last of `expected` arrivals,
// sums the ntiles slots in tile order and runs the transition.
// `release_all`: every thread's stores must be visible to other workgroups
// after the arrival (persistent form); in the stepped form only the slot
// must be, the kernel boundary publishes the rest.
__device__ bool arrive(QPState *q, int phase, bool f32, int ntiles, uint32_t expected,
                       bool release_all) {
  __shared__ int s_last;
  if (release_all) __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(&q->ticket, 1u);
    s_last = (prev == expected - 1) ? 1 : 0;
    if (s_last) __threadfence();
  }
  __syncthreads();
  if (!s_last) return false;
  double res[kNP];
  if (f32) {
    float v[kNP];
#pragma unroll
    for (int k = 0; k < kNP; ++k) v[k] = 0.0f;
    for (int t = threadIdx.x; t < ntiles; t += kBlock) {
      const double *slot = q->partials + (int64_t)t * kNP;
#pragma unroll
      for (int k = 0; k < kNP; ++k) v[k] += (float)slot[k];
    }
    block_sum<float, kNP>(v);
#pragma unroll
    for (int k = 0; k < kNP; ++k) res[k] = (double)v[k];
  } else {
    double v[kNP];
#pragma unroll
    for (int k = 0; k < kNP; ++k) v[k] = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += kBlock) {
      const double *slot = q->partials + (int64_t)t * kNP;
#pragma unroll
      for (int k = 0; k < kNP; ++k) v[k] += slot[k];
    }
    block_sum<double, kNP>(v);
#pragma unroll
    for (int k = 0; k < kNP; ++k) res[k] = v[k];
  }
  if (threadIdx.x == 0) {
    q->ticket = 0;
    transition(q, phase, res);
  }
  return true;
}

// ------------------------------------------------------------------ kernels

// Stepped form: one launch = one pass of every QP; workgroup = one tile.
template <typename CT>
__global__ __launch_bounds__(kBlock) void step_kernel(StepLaunch L) {
  const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  int lo = 0, hi = L.nqp;
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (L.prefix[m] <= t) lo = m;
    else hi = m;
  }
  QPState *q = L.qps[lo];
  const int tile = t - L.prefix[lo];
  const int phase = q->phase;
  if (phase == PH_DONE) return;
  const int ntiles = q->ntiles;
  const int64_t k0 = (int64_t)tile * q->tile;
  int64_t k1 = k0 + q->tile;
  if (k1 > q->n) k1 = q->n;
  double acc[kNP];
  float accf[kNP];
#pragma unroll
  for (int k = 0; k < kNP; ++k) {
    acc[k] = 0.0;
    accf[k] = 0.0f;
  }
  run_pass<CT>(q, phase, k0, k1, acc, accf);
  const bool f32 = f32_pass(q->mixed, phase);
  tile_partial(q, f32, tile, acc, accf);
  arrive(q, phase, f32, ntiles, (uint32_t)ntiles, false);
}

// Persistent form: one cooperative launch runs every QP to completion.  QP q
// owns the workgroup slots [wg_prefix[q], wg_prefix[q+1]); in each pass a
// workgroup sweeps the tiles lw, lw + nwg, ... of its QP, then arrives at
// the QP's ticket.  The last arrival runs the transition and bumps the QP's
// generation counter, which the other workgroups of that QP wait for.  No
// barrier spans two QPs, so every QP advances at its own pace.  Every wait
// is bounded: after spin_limit polls the QP is failed with GPCG_ERR_HANG
// and the workgroup exits, so the grid always drains.
template <typename CT>
__global__ __launch_bounds__(kBlock) void persistent_kernel(PersistLaunch P) {
  const int slot = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  if (slot >= P.wg_total) return;
  int lo = 0, hi = P.nqp;
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (P.wg_prefix[m] <= slot) lo = m;
    else hi = m;
  }
  QPState *q = P.qps[lo];
  const int lw = slot - P.wg_prefix[lo];
  const int nwg = P.wg_prefix[lo + 1] - P.wg_prefix[lo];
  __shared__ int s_exit;
  for (;;) {
    const int phase = __hip_atomic_load(&q->phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (phase == PH_DONE) break;
    const uint32_t gen =
        __hip_atomic_load(&q->generation, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int ntiles = q->ntiles;
    const bool f32 = f32_pass(q->mixed, phase);
    for (int tile = lw; tile < ntiles; tile += nwg) {
      const int64_t k0 = (int64_t)tile * q->tile;
      int64_t k1 = k0 + q->tile;
      if (k1 > q->n) k1 = q->n;
      double acc[kNP];
      float accf[kNP];
#pragma unroll
      for (int k = 0; k < kNP; ++k) {
        acc[k] = 0.0;
        accf[k] = 0.0f;
      }
      run_pass<CT>(q, phase, k0, k1, acc, accf);
      tile_partial(q, f32, tile, acc, accf);
    }
    const bool last = arrive(q, phase, f32, ntiles, (uint32_t)nwg, true);
    if (threadIdx.x == 0) {
      s_exit = 0;
      if (last) {
        __threadfence();
        __hip_atomic_store(&q->generation, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        int64_t spins = 0;
        while (__hip_atomic_load(&q->generation, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) ==
               gen) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > P.spin_limit) {
            q->status = GPCG_ERR_HANG;
            __hip_atomic_store(&q->phase, (int32_t)PH_DONE, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (q->host_flag)
              __hip_atomic_store(q->host_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            s_exit = 1;
            break;
          }
        }
      }
      __threadfence();
    }
    __syncthreads();
    if (s_exit) break;
  }
}

// Building blocks exposed through the C ABI.
template <typename T>
__global__ __launch_bounds__(kBlock) void spmv_kernel(const QPState *q, const T *__restrict__ v,
                                                      T *__restrict__ y,
                                                      const uint8_t *__restrict__ mask) {
  const OpView<T> A = op_view<T>(q);
  const int64_t n = q->n;
  auto vv = [&](int64_t j) { return v[j]; };
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kBlock) {
    if (mask && !mask[k]) {
      y[k] = T(0);
      continue;
    }
    y[k] = apply_row<T>(A, k, vv);
  }
}

__global__ __launch_bounds__(kBlock) void pgrad_kernel(int64_t n, const double *__restrict__ x,
                                                       const double *__restrict__ l,
                                                       const double *__restrict__ u,
                                                       const double *__restrict__ g,
                                                       double *__restrict__ pg,
                                                       double *__restrict__ part) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kBlock) {
    const double xk = x[k], lk = l[k], uk = u[k], gk = g[k];
    const double p = proj_grad(xk, lk, uk, gk);
    if (pg) pg[k] = p;
    acc[0] = __fma_rn(p, p, acc[0]);
    acc[1] += (xk == lk) ? 1.0 : 0.0;
    acc[2] += (xk != lk && xk == uk) ? 1.0 : 0.0;
    acc[3] += (is_active(xk, lk, uk) && !is_binding(xk, lk, uk, gk)) ? 1.0 : 0.0;
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

void *gpcg_step_kernel_ptr(int mixed) {
  return mixed ? (void *)&step_kernel<float> : (void *)&step_kernel<double>;
}

void *gpcg_persistent_kernel_ptr(int mixed) {
  return mixed ? (void *)&persistent_kernel<float> : (void *)&persistent_kernel<double>;
}

int gpcg_persistent_max_blocks(int mixed, int *blocks_per_cu) {
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, mixed ? (const void *)&persistent_kernel<float>
                           : (const void *)&persistent_kernel<double>,
      kBlock, 0);
  return e == hipSuccess ? 0 : -1;
}

int gpcg_launch_persistent(const PersistLaunch &P, int grid, int mixed, void *stream) {
  PersistLaunch arg = P;
  void *args[] = {&arg};
  hipError_t e = hipLaunchCooperativeKernel(
      mixed ? (const void *)&persistent_kernel<float> : (const void *)&persistent_kernel<double>,
      dim3(grid), dim3(kBlock), args, 0, (hipStream_t)stream);
  return e == hipSuccess ? 0 : -1;
}

int gpcg_launch_step(const StepLaunch &L, int mixed, void *stream) {
  if (L.total_tiles <= 0) return 0;
  if (mixed)
    hipLaunchKernelGGL(step_kernel<float>, dim3(L.total_tiles), dim3(kBlock), 0,
                       (hipStream_t)stream, L);
  else
    hipLaunchKernelGGL(step_kernel<double>, dim3(L.total_tiles), dim3(kBlock), 0,
                       (hipStream_t)stream, L);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

static int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

int gpcg_launch_spmv(const QPState *dqp, const QPState &hqp, const void *v, void *y,
                     const uint8_t *mask, int f32, void *stream) {
  const int grid = grid_for(hqp.n);
  if (f32)
    hipLaunchKernelGGL(spmv_kernel<float>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, dqp,
                       (const float *)v, (float *)y, mask);
  else
    hipLaunchKernelGGL(spmv_kernel<double>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                       dqp, (const double *)v, (double *)y, mask);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int gpcg_launch_pgrad(const QPState *dqp, const QPState &hqp, const double *x, const double *l,
                      const double *u, const double *g, double *pg, double *out4, void *stream) {
  (void)dqp;
  // partial slots live in the handle's partial area, which holds >= 2048 tiles
  int grid = grid_for(hqp.n);
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(pgrad_kernel, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, hqp.n, x, l,
                     u, g, pg, hqp.partials);
  hipLaunchKernelGGL(pgrad_final_kernel, dim3(1), dim3(kBlock), 0, (hipStream_t)stream, grid,
                     hqp.partials, out4);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int gpcg_launch_convert_f32(const double *src, float *dst, int64_t count, void *stream) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(convert_f32_kernel, dim3(grid_for(count)), dim3(kBlock), 0,
                     (hipStream_t)stream, src, dst, count);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
