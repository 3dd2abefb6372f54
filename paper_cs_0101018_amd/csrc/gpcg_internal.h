// gpcg_internal.h -- device-resident state of one GPCG solve and the launch
// interface between the host runtime and the HIP kernels.
//
// The control flow of Algorithm GPCG (Section 3 of the paper) runs on the
// device as a state machine over *passes*.  A pass is one data-parallel sweep
// over the unknowns of a QP (the initial projection and gradient, the exact
// step length of a gradient-projection iterate, a trial point of a projected
// search fused with the gradient at that point, the set-up of a reduced CG
// solve, one CG iteration).  The unknowns are cut into tiles of 256 or 512;
// each tile's partial sums go to fixed slots of that tile.  Before the next pass the slots are summed in tile order
// and the scalar transition picks the next pass: in every workgroup of the
// next launch (fused form) or in a transition kernel (split form).  The
// kernel boundary is the barrier; the state and the slots are double-buffered
// by launch parity.
#pragma once

#include <stdint.h>

namespace gpcg {

constexpr int kBlock = 256;   // threads per workgroup (four wave64s)
constexpr int kNP = 10;       // reduction slots per tile and pass
// Projected-gradient building block: at most this many workgroups, each
// leaving four partial sums, then the four totals.
constexpr int kPgradMaxBlocks = 2048;
constexpr int kPgradScratchDoubles = 4 * kPgradMaxBlocks + 4;

enum Phase : int32_t {
  PH_INIT = 0,    // x <- mid(l, u, x0); g <- Ax - b; checks; P grad q norm; face counts
  PH_GP_ALPHA,    // d = P grad q(y): d'd and d'Ad for alpha_0 (eq. bqpls)
  PH_GP_TRIAL,    // y' = P[y - alpha g] and g' = Ay' - b: decrease and face of y'
  PH_CG_INIT,     // free mask, rho = -g on F, u = A rho, w = 0
  PH_CG_ITER,     // one single-reduction CG iteration on the free set
  PH_PS_TRIAL,    // x' = P[x + alpha w] and g' = Ax' - b: decrease and face of x'
  PH_CG_LIST,     // list form: compact the free mask into an ascending index list
  PH_CG_MCOUNT,   // matrix form: free columns of every free row (nonzeros of A_F)
  PH_CG_MFILL,    // matrix form: write A_F (rows of the list, free columns only)
  PH_DONE,
  PH_COUNT
};

enum Ctx : int32_t { CTX_INIT = 0, CTX_GP = 1, CTX_PS = 2 };

enum OpKind : int32_t { OPK_CONST = 1, OPK_VAR = 2, OPK_CSR = 3 };

enum PhaseBucket : int32_t { TB_CG = 0, TB_GP = 1, TB_SEARCH = 2, TB_OTHER = 3 };

// Read-only during a solve.
struct QPStatic {
  int32_t op_kind, nx, ny, tile;  // tile: unknowns per workgroup and pass
  int32_t ntiles, mixed, max_outer, max_gp;
  int32_t max_backtrack, max_cg, max_stall, cg_stop;  // cg_stop: 0 eq. (cgstop1), 1 residual
  int64_t n;
  uint64_t div_magic;  // k / nx == (k * div_magic) >> div_shift for k < 2^30
  int32_t div_shift;
  int32_t gp_la;  // fused form: GP_TRIAL also sums eq. (bqpls) at the trial point
  double w;  // constant stencil weight
  float w32, pad2;
  const double *wx, *wy;     // edge weights (FP64)
  const float *wx32, *wy32;  // FP32 copies (mixed precision)
  const int32_t *rowptr, *colind;
  const double *vals;
  const float *vals32;
  const double *b, *l, *u;
  double *x[2], *g[2];           // x[0] is the caller's x; current copy: dyn.cur
  void *rho[2], *uq[2], *sq[2];  // CG residual, A*residual, A*direction (FP64/FP32)
  void *pv, *wv;                 // CG direction and iterate
  uint8_t *mask;                 // free set of the current CG phase
  int32_t *list;                 // list form: free indices in ascending order (else null)
  int32_t *mrow, *mcol;          // matrix form: A_F as CSR over the list (row pointers,
  void *mval;                    //   grid column indices, values FP64/FP32), or null
  const void *dinv;              // Jacobi preconditioner: 1 / diag(A) (FP64/FP32), or null
  int32_t *host_flag;            // device view of a mapped host word, or null
  double tol_rel, tol_abs, eta1, eta2, eta2_reduce, mu;
};

// The scalar state machine: the part the transition reads and writes.
struct QPCore {
  int32_t phase, ctx, status, pending;  // pending: partials of `phase` await reduction
  int32_t cur, first, ps_accepted, gp_j;
  int32_t bt, gp_accepts, cg_j, max_cg_eff;
  int32_t stall, x0_projected, outer_iters, gp_iters;
  int32_t cg_iters, backtracks, face_repeats, cg_phases;
  double tau, pg0, pgn, q, best_pg;
  double alpha, gp_decmax;
  double eta, cg_alpha, cg_beta, gamma, cg_decmax, gamma0;
  int64_t m_free, n_lower, n_upper, n_nonbinding;
  int64_t passes, cg_free_rows;
  int64_t lookaheads;  // eq. (bqpls) evaluated inside a trial pass
  int64_t nnz_free, cg_free_nnz;  // matrix form: nonzeros of A_F; summed over CG passes
};

// One copy of the state per launch parity: the core plus per-pass counters.
struct QPDyn {
  QPCore c;
  int64_t pass_count[PH_COUNT];
  uint64_t t_last;
  uint64_t t_bucket[4];
};

struct QPDev {
  QPStatic st;
  QPDyn dyn[2];
  uint32_t counter;  // persistent form: arrivals (monotonic)
  uint32_t pad[63];
};

// The tile slots of a QP follow its QPDev at a fixed offset.  They are laid
// out in blocks of kBlock tiles, [tile / kBlock][2 parities][kNP][tile %
// kBlock] doubles, so the threads of a workgroup that read the slots of
// consecutive tiles read consecutive words, and at least one block exists.
constexpr size_t kQPDevBytes = (sizeof(QPDev) + 255) / 256 * 256;

__host__ __device__ inline double *tile_slots(QPDev *q) {
  return reinterpret_cast<double *>(reinterpret_cast<char *>(q) + kQPDevBytes);
}
__host__ __device__ inline const double *tile_slots(const QPDev *q) {
  return reinterpret_cast<const double *>(reinterpret_cast<const char *>(q) + kQPDevBytes);
}
__host__ __device__ inline int64_t slot_index(int tile, int par, int k) {
  return (((int64_t)(tile / kBlock) * 2 + par) * kNP + k) * kBlock + (tile % kBlock);
}
__host__ __device__ inline size_t tile_slot_bytes(int ntiles) {
  const size_t blocks = ntiles > kBlock ? ((size_t)ntiles + kBlock - 1) / kBlock : 1;
  return sizeof(double) * 2 * kNP * kBlock * blocks;
}

struct WgItem {
  QPDev *q;
  int32_t tile0, ntile;
};

// What a CG iteration of a stencil QP reads besides the scalar state: the
// operator and the CG vectors of one QP.  The kernels read it from the QP's
// static state with uniform (scalar) loads before anything else, and issue
// the CG operand loads from it before the state is known.  wx, wy and w are
// those of the CG precision (FP32 copies in the mixed form).
struct CGView {
  int32_t op_kind, nx, ny, div_shift;
  uint64_t div_magic;
  int64_t n;
  double w;
  const void *wx, *wy;
  void *rho[2], *uq[2], *sq[2];
  void *pv, *wv;
  const uint8_t *mask;
  const void *dinv;  // Jacobi preconditioner or null
};

struct StepLaunch {
  QPDev *single;           // one QP: its state (tables unused)
  QPDev *const *qps;       // several QPs: device array of nqp pointers (transition kernel)
  const WgItem *items;     // several QPs: device array of data_grid work items
  int32_t nqp;
  int32_t total_tiles;     // one QP: its tile count (grid of the fused kernel)
  int32_t parity;          // this launch reads dyn/partials[parity]
  int32_t tiles_per_wg;    // one QP, split form: consecutive tiles per data workgroup
  int32_t data_grid;       // split form: workgroups of the data kernel
  int32_t item_tiles;      // queue form: tiles per queued work item
  // Queue form (several QPs, split form): the transition kernel of launch
  // parity p appends the work items of every QP that is not done to
  // queue[p * queue_cap ...], counting them in qcount[p] (and zeroes the
  // other parity's count); the data kernel runs the qcount[p] queued items
  // with a fixed grid.  No work item exists for a finished QP.
  int32_t queue_cap;       // items per parity
  int32_t pad2;
  WgItem *queue;           // 2 * queue_cap items, or null (item table / one QP)
  int32_t *qcount;         // 2 counters
};

struct PersistLaunch {
  QPDev *const *qps;         // device array of nqp state pointers
  const int32_t *wg_prefix;  // device array, nqp+1 workgroup-slot offsets
  int32_t nqp;
  int32_t wg_total;
  int64_t spin_limit;        // polls before a wait is declared hung
  int32_t pre;               // some QP has the Jacobi preconditioner
  int32_t pad;
};

// Kernel variants (the `spec` argument of the launchers below is a set of
// these bits).  kVarSpec: the launch holds only stencil QPs with 256-unknown
// tiles, which may load CG operands before the state is known.  kVarPre: some
// QP of the launch has the Jacobi preconditioner.  kVarCgk: split form, the
// lean CG iterations run in a data kernel of their own (fewer registers, more
// workgroups in flight) and the data kernel of the other passes skips them.
constexpr int kVarSpec = 1;
constexpr int kVarPre = 2;
constexpr int kVarCgk = 4;
// kVarMat: some QP of the launch has the matrix free set (the kernels that
// carry its count and fill passes; never with kVarSpec).
constexpr int kVarMat = 8;
// kVarQueue: the data kernels of the queue form (a fixed grid running the
// items the transition kernel queued; never with kVarSpec).
constexpr int kVarQueue = 16;
// kVarLgp: the gradient-projection passes of stencil QPs take the lean path
// (values shared through LDS; bitwise the generic path).  Set by batches and
// the server; not with kVarSpec or kVarMat.  The kernel of one large QP keeps
// the generic path: there the extra code slowed its CG passes by 2 %, and
// gradient-projection passes are 1-2 % of its passes.
constexpr int kVarLgp = 32;

}  // namespace gpcg

extern "C++" {
void *gpcg_step_kernel_ptr(int mixed, int spec);
int gpcg_launch_step(const gpcg::StepLaunch &L, int mixed, int spec, void *stream);
// Split form: a transition kernel (grid = QPs) then a data kernel (grid = tiles);
// with kVarCgk two data kernels, the CG kernel (gpcg_pass_kernel_ptr) and the
// kernel of the other passes (gpcg_rest_kernel_ptr), on the same grid.
void *gpcg_transition_kernel_ptr();
void *gpcg_pass_kernel_ptr(int mixed, int spec);
void *gpcg_rest_kernel_ptr(int mixed, int spec);
int gpcg_launch_split(const gpcg::StepLaunch &L, int mixed, int spec, void *stream);
// dqp: the QP's device state; S: the host copy of its static part (the same
// operator); vec_nx: grid width of a stencil operator whose arrays allow
// 16-byte loads (0: the scalar kernel).
int gpcg_launch_spmv(const gpcg::QPDev *dqp, const gpcg::QPStatic *S, int64_t n, const void *v,
                     void *y, const uint8_t *mask, int f32, int vec_nx, void *stream);
int gpcg_launch_pgrad(int64_t n, const double *x, const double *l, const double *u,
                      const double *g, double *pg, double *part, double *out4, void *stream);
// The same on the library's own per-device scratch array (no workspace): *out4
// receives the device address of the four totals.  0 on success; -1 no
// current device, -2 the scratch address lookup failed, -3 a bad size or a
// launch error.
int gpcg_launch_pgrad_scratch(int64_t n, const double *x, const double *l, const double *u,
                              const double *g, double *pg, const double **out4, void *stream);
// Copies `bytes` (a multiple of 8, both ends 8-byte aligned) from src
// (device memory or mapped coherent host memory) to dst with a kernel.
// Returns -1 on a bad argument or launch error.
int gpcg_launch_copy(void *dst, const void *src, size_t bytes, void *stream);
int gpcg_launch_convert_f32(const double *src, float *dst, int64_t count, void *stream);
// 1 / diag(A) of the QP's operator into dinv (FP64 or FP32); the device state
// must hold the operator.  Returns -1 on a launch error.
int gpcg_launch_diag_inv(const gpcg::QPDev *dqp, void *dinv, int f32, void *stream);
int gpcg_persistent_max_blocks(int mixed, int *blocks_per_cu);
int gpcg_launch_persistent(const gpcg::PersistLaunch &P, int grid, int mixed, void *stream);
}
