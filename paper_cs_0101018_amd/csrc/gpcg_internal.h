// gpcg_internal.h -- device-resident state of one GPCG solve and the launch
// interface between the host runtime and the HIP kernels.
//
// Every QP being solved owns one QPState in device memory (inside its
// workspace).  The whole control flow of Algorithm GPCG (Section 3 of the
// paper) lives on the device as a state machine over *passes*: one pass is
// one data-parallel sweep over the QP's unknowns (a projection, a gradient,
// a trial point of a projected search, one half of a CG iteration, ...).
// Every workgroup of a pass reduces its tile into a fixed slot of
// `partials`; the last workgroup to arrive (atomic ticket) sums the slots in
// a fixed order and runs the scalar transition that picks the next pass.
// The host only replays launches and waits for the DONE flag.
#pragma once

#include <stdint.h>

namespace gpcg {

constexpr int kBlock = 256;   // threads per workgroup (four wave64s)
constexpr int kNP = 6;        // reduction slots per tile and pass

enum Phase : int32_t {
  PH_PROJECT = 0,  // x <- mid(l, u, x0); validate inputs
  PH_GRAD,         // g <- Ax - b; projected gradient norm; face counts
  PH_GP_ALPHA,     // d = P grad q(y): d'd and d'Ad for alpha_0 (eq. bqpls)
  PH_GP_TRIAL,     // trial y' = P[y - alpha g]: g's, s'As, active changes
  PH_GP_ACCEPT,    // y <- y'
  PH_CG_INIT,      // free mask, r = -g on F, w = 0, p = r
  PH_CG_A,         // p <- r + beta p ; q = M.(A p) ; p'q
  PH_CG_B,         // w += alpha p ; r -= alpha q ; r'r
  PH_PS_TRIAL,     // trial x' = P[x + alpha w]: g's, s'As
  PH_PS_ACCEPT,    // x <- x'
  PH_DONE,
  PH_COUNT
};

enum Ctx : int32_t { CTX_INIT = 0, CTX_GP = 1, CTX_PS = 2 };

enum OpKind : int32_t { OPK_CONST = 1, OPK_VAR = 2, OPK_CSR = 3 };

enum PhaseBucket : int32_t { TB_CG = 0, TB_GP = 1, TB_SEARCH = 2, TB_OTHER = 3 };

struct QPState {
  // ---------------- static description (written by the host per solve)
  int32_t op_kind, nx, ny, tile;
  int32_t ntiles, mixed, pad0, pad1;
  int64_t n;
  uint64_t div_magic;  // k / nx == (k * div_magic) >> div_shift for k < 2^31
  int32_t div_shift, pad2;
  double w;            // constant stencil weight
  float w32, pad3;
  const double *wx, *wy;        // variable stencil weights (FP64)
  const float *wx32, *wy32;     // FP32 copies (mixed precision)
  const int32_t *rowptr, *colind;
  const double *vals;
  const float *vals32;
  const double *b, *l, *u;
  double *x, *g;
  void *vw, *vr, *vp0, *vp1;    // CG vectors, FP64 or FP32
  uint8_t *mask;
  double *partials;             // [ntiles][kNP]
  int32_t *host_flag;           // device view of a mapped host word, or null
  double tol_rel, tol_abs, eta1, eta2, eta2_reduce, mu;
  int32_t max_outer, max_gp, max_backtrack, max_cg;
  int32_t max_stall, pad8;

  // ---------------- dynamic state (reset by the host, then device-owned)
  uint32_t ticket, generation;
  int32_t phase, ctx, status, x0_projected;
  int32_t gp_j, bt, gp_accepts, cg_j;
  int32_t pcur, first_cg, ps_accepted, max_cg_eff;
  int32_t stall, pad5;
  double tau, pg0, pgn, q, best_pg;
  double alpha, gp_decmax, pend_dec;
  int64_t pend_nchg;
  double eta, rr, cg_alpha, beta, cg_decmax;
  int64_t m_free, n_lower, n_upper, n_nonbinding;

  // ---------------- statistics
  int32_t outer_iters, gp_iters, cg_iters, backtracks;
  int32_t face_repeats, cg_phases, pad6, pad7;
  int64_t passes;
  int64_t pass_count[PH_COUNT];
  int64_t cg_free_rows;          // sum of m over CG_A/CG_B/PS passes
  uint64_t t_last;
  uint64_t t_bucket[4];          // wall-clock ticks per phase bucket
};

// Host-callable launchers implemented in gpcg_kernels.hip.
struct StepLaunch {
  QPState *const *qps;  // device array of nqp state pointers
  const int32_t *prefix;  // device array, nqp+1 tile offsets
  int32_t nqp;
  int32_t total_tiles;
};

struct PersistLaunch {
  QPState *const *qps;     // device array of nqp state pointers
  const int32_t *wg_prefix;  // device array, nqp+1 workgroup-slot offsets
  int32_t nqp;
  int32_t wg_total;
  int64_t spin_limit;      // polls before a wait is declared hung
};

}  // namespace gpcg

extern "C++" {
// Kernel entry symbols, exposed so the runtime can build graph nodes.
void *gpcg_step_kernel_ptr(int mixed);
void *gpcg_persistent_kernel_ptr(int mixed);
int gpcg_launch_step(const gpcg::StepLaunch &L, int mixed, void *stream);
int gpcg_launch_spmv(const gpcg::QPState *dqp, const gpcg::QPState &hqp, const void *v, void *y,
                     const uint8_t *mask, int f32, void *stream);
int gpcg_launch_pgrad(const gpcg::QPState *dqp, const gpcg::QPState &hqp, const double *x,
                      const double *l, const double *u, const double *g, double *pg,
                      double *out4, void *stream);
int gpcg_launch_convert_f32(const double *src, float *dst, int64_t count, void *stream);
int gpcg_persistent_max_blocks(int mixed, int *blocks_per_cu);
int gpcg_launch_persistent(const gpcg::PersistLaunch &P, int grid, int mixed, void *stream);
}
