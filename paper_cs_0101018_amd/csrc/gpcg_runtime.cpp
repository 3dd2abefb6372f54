// gpcg_runtime.cpp -- host side of the C ABI declared in include/gpcg.h.
//
// The runtime validates descriptors, carves the caller's workspace, writes the
// device-resident state of each solve (QPDev) and then only replays launches
// of the pass kernel -- as chunks of a HIP graph -- until the device raises
// the DONE flag in mapped host memory.  Every GPCG decision is taken on the
// device.  Launch i reads state and partial sums of parity i & 1 and writes
// the other parity; chunks hold an even number of launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "gpcg.h"
#include "gpcg_internal.h"

using namespace gpcg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HIP_OK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(GPCG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int64_t op_n(const gpcg_operator *op) {
  if (op->kind == GPCG_OP_CSR) return op->n;
  return (int64_t)op->nx * (int64_t)op->ny;
}

int validate_op(const gpcg_operator *op) {
  if (!op) return fail(GPCG_ERR_ARG, "operator is NULL");
  switch (op->kind) {
    case GPCG_OP_STENCIL5_CONST:
      if (!(op->w > 0.0) || !std::isfinite(op->w))
        return fail(GPCG_ERR_ARG, "constant stencil weight must be positive and finite");
      [[fallthrough]];
    case GPCG_OP_STENCIL5_VAR:
      if (op->nx < 1 || op->ny < 1) return fail(GPCG_ERR_ARG, "stencil grid must be >= 1 x 1");
      if (op->kind == GPCG_OP_STENCIL5_VAR && (!op->wx || !op->wy))
        return fail(GPCG_ERR_ARG, "variable stencil needs wx and wy");
      break;
    case GPCG_OP_CSR:
      if (op->n < 1) return fail(GPCG_ERR_ARG, "CSR order must be >= 1");
      if (op->nnz < 1 || op->nnz >= (int64_t)1 << 31)
        return fail(GPCG_ERR_ARG, "CSR nnz out of range");
      if (!op->rowptr || !op->colind || !op->vals) return fail(GPCG_ERR_ARG, "CSR arrays missing");
      break;
    default:
      return fail(GPCG_ERR_ARG, "unknown operator kind");
  }
  if (op_n(op) > ((int64_t)1 << 30)) return fail(GPCG_ERR_ARG, "n > 2^30 not supported");
  return GPCG_OK;
}

int validate_opt(const gpcg_options *o) {
  if (!(o->tol_rel >= 0.0) || !(o->tol_abs >= 0.0)) return fail(GPCG_ERR_ARG, "tolerances < 0");
  if (!(o->eta1 > 0.0) || !(o->eta2 > 0.0)) return fail(GPCG_ERR_ARG, "eta1, eta2 must be > 0");
  if (!(o->eta2_reduce > 0.0 && o->eta2_reduce <= 1.0))
    return fail(GPCG_ERR_ARG, "eta2_reduce must be in (0, 1]");
  if (!(o->mu > 0.0 && o->mu < 0.5)) return fail(GPCG_ERR_ARG, "mu must be in (0, 1/2)");
  if (o->max_outer < 1 || o->max_gp < 1 || o->max_backtrack < 0)
    return fail(GPCG_ERR_ARG, "iteration caps must be positive");
  if (o->precision != GPCG_PREC_FP64 && o->precision != GPCG_PREC_MIXED)
    return fail(GPCG_ERR_ARG, "unknown precision");
  if (o->free_set != GPCG_FREESET_MASK && o->tile != 0 && o->tile != kBlock)
    return fail(GPCG_ERR_ARG, "the list and matrix free sets need 256-unknown tiles");
  if (o->free_set != GPCG_FREESET_MASK && o->free_set != GPCG_FREESET_LIST &&
      o->free_set != GPCG_FREESET_MATRIX)
    return fail(GPCG_ERR_ARG, "unknown free-set mode");
  if (o->tile < 0 || o->tile % kBlock != 0 || o->tile > (1 << 16))
    return fail(GPCG_ERR_ARG, "tile must be a multiple of 256 in [256, 65536]");
  if (o->chunk < 0 || o->chunk > 4096 || (o->chunk & 1))
    return fail(GPCG_ERR_ARG, "chunk must be even and at most 4096");
  if (o->max_stall < 1) return fail(GPCG_ERR_ARG, "max_stall must be >= 1");
  if (o->form < GPCG_FORM_AUTO || o->form > GPCG_FORM_SPLIT)
    return fail(GPCG_ERR_ARG, "unknown launch form");
  if (o->tiles_per_wg < 0 || o->tiles_per_wg > 64)
    return fail(GPCG_ERR_ARG, "tiles_per_wg must be in [0, 64]");
  if (o->prefetch < GPCG_PREFETCH_AUTO || o->prefetch > GPCG_PREFETCH_OFF)
    return fail(GPCG_ERR_ARG, "unknown prefetch mode");
  if (o->precond != GPCG_PRECOND_NONE && o->precond != GPCG_PRECOND_JACOBI)
    return fail(GPCG_ERR_ARG, "unknown preconditioner");
  if (o->cg_stop != GPCG_CGSTOP_DECREASE && o->cg_stop != GPCG_CGSTOP_RESIDUAL)
    return fail(GPCG_ERR_ARG, "unknown CG stopping test");
  if (o->lookahead < GPCG_LOOKAHEAD_AUTO || o->lookahead > GPCG_LOOKAHEAD_OFF)
    return fail(GPCG_ERR_ARG, "unknown lookahead mode");
  if (o->cg_kernel < GPCG_CGK_AUTO || o->cg_kernel > GPCG_CGK_OFF)
    return fail(GPCG_ERR_ARG, "unknown cg_kernel mode");
  return GPCG_OK;
}

// Options that depend on the operator.
int validate_pair(const gpcg_operator *op, const gpcg_options &o) {
  if (o.free_set == GPCG_FREESET_MATRIX && op->kind != GPCG_OP_CSR)
    return fail(GPCG_ERR_ARG, "the matrix free set needs a CSR operator");
  return GPCG_OK;
}

// The fused form sums every tile slot of the previous pass in every
// workgroup; beyond this many 256-unknown tiles the split form is cheaper.
constexpr int kFusedMaxTiles = 1024;

// Unknowns per tile (one reduction slot per tile and pass): 256, one per
// thread, up to 1024 x 256 unknowns; beyond that 512, which halves the slots
// the transition of the split form sums.  Wider tiles save more slots but a
// data workgroup sweeps the 256-unknown chunks of its tile one after the
// other: at 1600^2 in FP64 (5000 tiles of 512) 1024-unknown tiles lose more
// there than they gain (43.0 against 38.4 us per pass).  Once the grid holds
// kWideTiles tiles even of 1024 or 2048 unknowns, the per-tile costs weigh
// more: at 4096^2 in FP64, beyond the last-level cache, a pass takes 351 us
// with 512-unknown tiles, 334 with 1024 and 321 with 2048 (the transition's
// slot sum 21.6 -> 8.5 us, the data kernel 329 -> 312 us).  The mixed form
// moves half the CG bytes per unknown, so the per-tile costs weigh more
// there: 1024-unknown tiles from 1024 such tiles on (1024^2: 15.15 -> 13.65
// us per pass; 1600^2: 26.86 -> 26.13, where 2048 takes 29.58), 2048 from
// the same size as in FP64 (4096^2: 197.6 us with 512, 174.1 with 1024,
// 171.8 with 2048).  A function of n and the precision alone: a QP has the
// same tiles, hence the same summation order and answer, alone, in a batch,
// in the server and in every launch form.
constexpr int64_t kWideTiles = 8192;
constexpr int64_t kWideTilesMixed = 1024;
int tuned_tile(int64_t n, bool mixed) {
  if (n <= (int64_t)kFusedMaxTiles * kBlock) return kBlock;
  if (n >= kWideTiles * 8 * kBlock) return 8 * kBlock;
  if (n >= (mixed ? kWideTilesMixed : kWideTiles) * 4 * kBlock) return 4 * kBlock;
  return 2 * kBlock;
}

struct Layout {
  size_t qp, slots, pgpart, x1, g0, g1, rho0, rho1, uq0, uq1, sq0, sq1, p, w, mask;
  size_t wx32, wy32, vals32, list, mrow, mcol, mval, dinv, total;
  int tile, ntiles;
};

static_assert(kQPDevBytes % 256 == 0, "the slots follow the state at an aligned offset");

Layout layout_for(const gpcg_operator *op, int precision, int tile_opt, int free_set,
                  int precond) {
  Layout L{};
  const int64_t n = op_n(op);
  const bool mixed = precision == GPCG_PREC_MIXED;
  const size_t ct = mixed ? 4 : 8;
  // the list and matrix forms compact the free set tile by tile with one
  // unknown per thread: they keep 256-unknown tiles at every size
  L.tile = tile_opt > 0 ? tile_opt
                        : (free_set != GPCG_FREESET_MASK ? kBlock : tuned_tile(n, mixed));
  L.ntiles = (int)((n + L.tile - 1) / L.tile);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  L.qp = take(sizeof(QPDev));
  L.slots = take(tile_slot_bytes(L.ntiles));  // at L.qp + kQPDevBytes
  L.pgpart = take(sizeof(double) * kPgradScratchDoubles + 64);
  L.x1 = take(8 * (size_t)n);
  L.g0 = take(8 * (size_t)n);
  L.g1 = take(8 * (size_t)n);
  L.rho0 = take(ct * (size_t)n);
  L.rho1 = take(ct * (size_t)n);
  L.uq0 = take(ct * (size_t)n);
  L.uq1 = take(ct * (size_t)n);
  L.sq0 = take(ct * (size_t)n);
  L.sq1 = take(ct * (size_t)n);
  L.p = take(ct * (size_t)n);
  L.w = take(ct * (size_t)n);
  L.mask = take((size_t)n);
  L.wx32 = L.wy32 = L.vals32 = 0;
  if (mixed && op->kind == GPCG_OP_STENCIL5_VAR) {
    L.wx32 = take(4 * (size_t)op->ny * (op->nx + 1));
    L.wy32 = take(4 * (size_t)(op->ny + 1) * op->nx);
  }
  if (mixed && op->kind == GPCG_OP_CSR) L.vals32 = take(4 * (size_t)op->nnz);
  const bool matrix = free_set == GPCG_FREESET_MATRIX && op->kind == GPCG_OP_CSR;
  L.list = free_set != GPCG_FREESET_MASK ? take(4 * (size_t)n) : 0;
  // matrix form: A_F as CSR (row pointers over the list, at most nnz entries)
  L.mrow = matrix ? take(4 * ((size_t)n + 1)) : 0;
  L.mcol = matrix ? take(4 * (size_t)op->nnz) : 0;
  L.mval = matrix ? take(ct * (size_t)op->nnz) : 0;
  // the constant stencil has a constant diagonal: Jacobi scaling leaves the
  // CG iterates unchanged there, so it is not applied
  L.dinv = precond == GPCG_PRECOND_JACOBI && op->kind != GPCG_OP_STENCIL5_CONST
               ? take(ct * (size_t)n)
               : 0;
  L.total = off;
  return L;
}

void magic_for(int32_t d, uint64_t *magic, int32_t *shift) {
  int L = 0;
  while (((int64_t)1 << L) < d) ++L;
  *shift = 32 + L;
  *magic = ((uint64_t)1 << *shift) / (uint64_t)d + 1;
}

struct PinnedWords {
  int32_t *host = nullptr;  // mapped, coherent host memory
  int32_t *dev = nullptr;   // its device address
};

int alloc_flag(PinnedWords *f, size_t words) {
  void *h = nullptr;
  HIP_OK(hipHostMalloc(&h, sizeof(int32_t) * words, hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(h, 0, sizeof(int32_t) * words);
  void *d = nullptr;
  HIP_OK(hipHostGetDevicePointer(&d, h, 0));
  f->host = (int32_t *)h;
  f->dev = (int32_t *)d;
  return GPCG_OK;
}

// Pinned host memory that kernels read directly (mapped, coherent): the
// staging of state and tables, moved to the device by gpcg_launch_copy.
int alloc_pinned(void **host, void **dev, size_t bytes) {
  *host = nullptr;
  *dev = nullptr;
  HIP_OK(hipHostMalloc(host, bytes, hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(*host, 0, bytes);
  HIP_OK(hipHostGetDevicePointer(dev, *host, 0));
  return GPCG_OK;
}

// A device copy by kernel (see gpcg_launch_copy).
#define COPY_OK(dst, src, bytes, stream)                                         \
  do {                                                                           \
    if (gpcg_launch_copy((dst), (src), (bytes), (stream)) != 0)                  \
      return fail(GPCG_ERR_HIP, "device copy failed (" #dst ")");               \
  } while (0)

double wall_clock_hz() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1e8;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return 1e8;
  return khz * 1e3;
}

// Options copied into the static state.
void put_options(QPStatic &s, const gpcg_options &o) {
  s.tol_rel = o.tol_rel;
  s.tol_abs = o.tol_abs;
  s.eta1 = o.eta1;
  s.eta2 = o.eta2;
  s.eta2_reduce = o.eta2_reduce;
  s.mu = o.mu;
  s.max_outer = o.max_outer;
  s.max_gp = o.max_gp;
  s.max_backtrack = o.max_backtrack;
  s.max_cg = o.max_cg;
  s.max_stall = o.max_stall;
  s.cg_stop = o.cg_stop;
}

// The initial state of a solve (phase INIT, nothing pending).
void initial_dyn(QPDyn &d) {
  std::memset(&d, 0, sizeof(d));
  d.c.phase = PH_INIT;
  d.c.ctx = CTX_INIT;
  d.c.status = GPCG_OK;
  d.c.gp_decmax = -INFINITY;
  d.c.cg_decmax = -INFINITY;
}

// Algorithmic HBM bytes of a finished solve: every array a pass touches is
// counted once per pass (stencil neighbours are assumed reused on chip).
// Passes that sweep only the free set (CG iterations) count the mask byte for
// every unknown and the vector traffic for the free unknowns.
double solve_bytes(const QPStatic &s, const QPDyn &dy) {
  const QPCore &d = dy.c;
  const bool mixed = s.mixed != 0;
  const double c = mixed ? 4.0 : 8.0;
  double coef64 = 0.0, coefc = 0.0;
  if (s.op_kind == OPK_VAR) {
    coef64 = 16.0;
    coefc = mixed ? 8.0 : 16.0;
  } else if (s.op_kind == OPK_CSR) {
    coef64 = 4.0 + 5.0 * 12.0;  // rowptr + ~5 (colind, value) per row
    coefc = 4.0 + 5.0 * (mixed ? 8.0 : 12.0);
  }
  const double n = (double)s.n;
  const double it = (double)dy.pass_count[PH_CG_ITER];
  const double mean_m = it > 0 ? (double)d.cg_free_rows / it : 0.5 * n;
  double B = 0.0;
  B += dy.pass_count[PH_INIT] * n * (48.0 + coef64);      // x0, l, u, b in; x, g out
  B += dy.pass_count[PH_GP_ALPHA] * n * (32.0 + coef64);  // x, l, u, g
  B += dy.pass_count[PH_GP_TRIAL] * n * (56.0 + coef64);  // x, l, u, g, b in; x', g' out
  B += dy.pass_count[PH_CG_INIT] * (n * 33.0 + mean_m * (3 * c + coefc) + (n - mean_m) * 7 * c);
  if (s.dinv) {  // the preconditioner is read once per free row and pass
    B += (double)d.cg_free_rows * c;
    B += dy.pass_count[PH_CG_INIT] * mean_m * c;
  }
  if (s.mrow) {
    // matrix form: per free row the vectors, its list index and row pointer;
    // per nonzero of A_F a column index and a value; the count and fill passes
    // read the list, the CSR row pointers and (about five per row) the column
    // indices and mask bytes, and the fill pass writes A_F
    const double nnz_f = it > 0 ? (double)d.cg_free_nnz / it : 0.0;
    B += (double)d.cg_free_rows * (10 * c + 8.0) + (double)d.cg_free_nnz * (4.0 + c);
    B += dy.pass_count[PH_CG_LIST] * (n * 1.0 + mean_m * 4.0);
    B += dy.pass_count[PH_CG_MCOUNT] * mean_m * (12.0 + 5.0 * 5.0);
    B += dy.pass_count[PH_CG_MFILL] * (mean_m * (16.0 + 5.0 * 17.0) + nnz_f * (4.0 + c));
  } else if (s.list) {
    // list form: the index of each free row instead of the mask of every row;
    // the list pass reads the mask and writes the list
    B += (double)d.cg_free_rows * (10 * c + coefc + 4.0);
    B += dy.pass_count[PH_CG_LIST] * (n * 1.0 + mean_m * 4.0);
  } else {
    B += (double)d.cg_free_rows * (10 * c + coefc) + it * n * 1.0;  // rho,u,s,p,w in+out; mask
  }
  B += dy.pass_count[PH_PS_TRIAL] * (n * (57.0 + coef64) + mean_m * c);
  return B;
}

void fill_stats(const QPStatic &s, const QPDyn &dy, double tick_hz, gpcg_stats *st) {
  if (!st) return;
  const QPCore &d = dy.c;
  std::memset(st, 0, sizeof(*st));
  st->status = d.status;
  st->outer_iters = d.outer_iters;
  st->gp_iters = d.gp_iters;
  st->cg_iters = d.cg_iters;
  st->backtracks = d.backtracks;
  st->face_repeats = d.face_repeats;
  st->cg_phases = d.cg_phases;
  st->x0_projected = d.x0_projected;
  st->pg0 = d.pg0;
  st->pg = d.pgn;
  st->tau = d.tau;
  st->q = d.q;
  st->n_lower = d.n_lower;
  st->n_upper = d.n_upper;
  st->n_free = s.n - d.n_lower - d.n_upper;
  st->passes = d.passes;
  st->lookaheads = d.lookaheads;
  st->bytes = solve_bytes(s, dy);
  const double ms = 1e3 / tick_hz;
  st->ms_cg = dy.t_bucket[TB_CG] * ms;
  st->ms_gp = dy.t_bucket[TB_GP] * ms;
  st->ms_search = dy.t_bucket[TB_SEARCH] * ms;
  st->ms_other = dy.t_bucket[TB_OTHER] * ms;
}

// A graph of `count` chained steps with alternating parity (count is even, so
// replays continue the parity sequence).  A fused step is one launch of the
// pass kernel; a split step is the transition kernel then the data kernel.
int build_chain_graph(const StepLaunch &L, int mixed, int spec, int split, int count,
                      hipGraphExec_t *out) {
  hipGraph_t g = nullptr;
  HIP_OK(hipGraphCreate(&g, 0));
  hipGraphNode_t prev = nullptr;
  auto add = [&](void *func, unsigned grid, const StepLaunch &arg0) -> int {
    hipKernelNodeParams p{};
    p.func = func;
    p.gridDim = dim3(grid);
    p.blockDim = dim3(kBlock);
    p.sharedMemBytes = 0;
    StepLaunch arg = arg0;
    void *args[] = {&arg};
    p.kernelParams = args;
    p.extra = nullptr;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
    if (e != hipSuccess)
      return fail(GPCG_ERR_HIP, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
    prev = node;
    return GPCG_OK;
  };
  for (int i = 0; i < count; ++i) {
    StepLaunch arg = L;
    arg.parity = i & 1;
    int rc;
    if (split) {
      rc = add(gpcg_transition_kernel_ptr(), L.single ? 1u : (unsigned)L.nqp, arg);
      if (!rc) rc = add(gpcg_pass_kernel_ptr(mixed, spec), (unsigned)L.data_grid, arg);
      if (!rc && (spec & kVarCgk))
        rc = add(gpcg_rest_kernel_ptr(mixed, spec), (unsigned)L.data_grid, arg);
    } else {  // one QP: a workgroup per tile; several: one per one-tile item
      rc = add(gpcg_step_kernel_ptr(mixed, spec),
               (unsigned)(L.single ? L.total_tiles : L.data_grid), arg);
    }
    if (rc) {
      (void)hipGraphDestroy(g);
      return rc;
    }
  }
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess)
    return fail(GPCG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return GPCG_OK;
}

// Launches one chunk: the graph, or `chunk` plain steps of alternating parity
// starting at 0.
int launch_chunk(hipStream_t stream, StepLaunch L, int mixed, int spec, int split, int chunk,
                 hipGraphExec_t graph) {
  if (graph) {
    HIP_OK(hipGraphLaunch(graph, stream));
    return GPCG_OK;
  }
  for (int i = 0; i < chunk; ++i) {
    L.parity = i & 1;
    const int rc = split ? gpcg_launch_split(L, mixed, spec, stream)
                         : gpcg_launch_step(L, mixed, spec, stream);
    if (rc != 0) return fail(GPCG_ERR_HIP, "pass kernel launch failed");
  }
  return GPCG_OK;
}

// Replays chunks until `done()` holds.  The next chunk is queued while the
// running one still has a lead time left (its expected duration is that of
// the chunk before it), so the GPU does not idle between chunks; queuing it
// later than that would idle the GPU, queuing it earlier adds launches past
// the last pass (they find the state done and return).  The lead is a fifth
// of a chunk and at least four times what queuing a chunk costs the host.
template <class Done>
int run_until(hipStream_t stream, const StepLaunch &L, int mixed, int spec, int split, int chunk,
              hipGraphExec_t graph,
              hipEvent_t *ev, Done done, int64_t max_launches, int64_t *launches,
              int64_t *checks) {
  double t_q = now_s();
  int rc = launch_chunk(stream, L, mixed, spec, split, chunk, graph);
  if (rc) return rc;
  double t_start = now_s();  // the running chunk started no earlier than this
  double submit = t_start - t_q;
  double dur = 0.0;  // duration of the last finished chunk; 0 = not known yet
  *launches += chunk;
  HIP_OK(hipEventRecord(ev[0], stream));
  for (int64_t i = 1;; ++i) {
    if (*launches >= max_launches)
      return fail(GPCG_ERR_HANG, "device did not finish within the launch budget");
    hipEvent_t prev = ev[(i - 1) & 1];
    if (dur > 0.0) {  // hold the next chunk until the running one nears its end
      const double lead = std::max(0.2 * dur, 4.0 * submit);
      const double t_go = t_start + dur - lead;
      while (now_s() < t_go && !done()) {
        hipError_t e = hipEventQuery(prev);
        if (e == hipSuccess) break;  // ended sooner than expected
        if (e != hipErrorNotReady)
          return fail(GPCG_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
        std::this_thread::yield();
      }
      if (done()) break;
    }
    t_q = now_s();
    rc = launch_chunk(stream, L, mixed, spec, split, chunk, graph);
    if (rc) return rc;
    submit = 0.5 * submit + 0.5 * (now_s() - t_q);
    *launches += chunk;
    HIP_OK(hipEventRecord(ev[i & 1], stream));
    for (;;) {
      if (done()) break;
      hipError_t e = hipEventQuery(prev);
      if (e == hipSuccess) break;
      if (e != hipErrorNotReady)
        return fail(GPCG_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
      std::this_thread::yield();
    }
    *checks += 1;
    if (done()) break;
    // chunk i - 1 ended now; chunk i, queued before, starts now
    const double t = now_s();
    dur = t - t_start;
    t_start = t;
  }
  HIP_OK(hipStreamSynchronize(stream));
  return GPCG_OK;
}

int default_chunk(const gpcg_options &o) { return o.chunk > 0 ? o.chunk : 32; }

// Whether a QP may run in the launch variant with speculative CG operand
// loads (stencil operator, one unknown per thread).
bool spec_ok(const QPStatic &s) {
  return s.tile == kBlock && s.op_kind != OPK_CSR && s.list == nullptr;
}

}  // namespace

// ------------------------------------------------------------------ handle

// How a QP's passes are launched.  Every configuration gives bitwise the
// same answer (same tiles, same summation orders); only the speed differs.
struct LaunchCfg {
  int split;         // 0: fused form, 1: split form
  int tiles_per_wg;  // split form: consecutive tiles per data workgroup
  int spec;          // CG operands loaded before the state is known (stencils)
  int chunk;         // passes per graph replay / host check (even)
  int shrink = 3;    // stepped batch: re-form the launch once 1/shrink of its tiles are done;
                     // 0: the queue form (never re-formed; a device queue holds the
                     // work items of the QPs that are not done)
  int cgk = 0;       // split form: CG iterations in a data kernel of their own
  bool operator==(const LaunchCfg &o) const {
    return split == o.split && tiles_per_wg == o.tiles_per_wg && spec == o.spec &&
           chunk == o.chunk && shrink == o.shrink && cgk == o.cgk;
  }
  bool operator!=(const LaunchCfg &o) const { return !(*this == o); }
};

namespace {

// Tuned configurations by operator shape and precision, shared by the handles
// of the process (handles created with automatic options start from them).
struct TuneKey {
  int kind, nx, ny, mixed, list, precond, tile;
  int64_t n, nnz;
  bool operator<(const TuneKey &o) const {
    return std::tie(kind, nx, ny, mixed, list, precond, tile, n, nnz) <
           std::tie(o.kind, o.nx, o.ny, o.mixed, o.list, o.precond, o.tile, o.n, o.nnz);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, LaunchCfg> g_tuned;

}  // namespace

struct gpcg_handle_s {
  gpcg_operator op;
  gpcg_options opt;
  hipStream_t stream;
  char *ws;
  size_t ws_bytes;
  Layout L;
  QPStatic st;          // static part (x[0] filled per solve)
  QPDev *dqp;           // device state
  QPDev *stage;         // pinned host staging for uploads / downloads
  QPDev *stage_dev;     // its device address
  PinnedWords flag;     // DONE flag written by the device
  hipGraphExec_t graph = nullptr;
  LaunchCfg graph_cfg{};  // configuration the graph was built for
  hipEvent_t ev[2] = {nullptr, nullptr};
  double tick_hz;
  LaunchCfg cfg{};        // launch configuration of this handle's solves
};

namespace {

TuneKey tune_key(const gpcg_handle_s *h) {
  return TuneKey{h->op.kind, h->st.nx, h->st.ny, h->st.mixed, h->st.mrow ? 2 : h->st.list ? 1 : 0,
                 h->st.dinv ? 1 : 0, h->st.tile, h->st.n,
                 h->op.kind == GPCG_OP_CSR ? h->op.nnz : 0};
}

void fill_static(gpcg_handle_s *h) {
  QPStatic &q = h->st;
  std::memset(&q, 0, sizeof(q));
  const gpcg_operator &op = h->op;
  char *ws = h->ws;
  const Layout &L = h->L;
  const bool mixed = h->opt.precision == GPCG_PREC_MIXED;
  q.op_kind = op.kind == GPCG_OP_STENCIL5_CONST ? OPK_CONST
              : op.kind == GPCG_OP_STENCIL5_VAR ? OPK_VAR
                                                : OPK_CSR;
  q.nx = op.kind == GPCG_OP_CSR ? 1 : op.nx;
  q.ny = op.kind == GPCG_OP_CSR ? 1 : op.ny;
  q.n = op_n(&op);
  q.tile = L.tile;
  q.ntiles = L.ntiles;
  q.mixed = mixed ? 1 : 0;
  magic_for(q.nx, &q.div_magic, &q.div_shift);
  q.w = op.w;
  q.w32 = (float)op.w;
  q.wx = op.wx;
  q.wy = op.wy;
  q.wx32 = L.wx32 ? (const float *)(ws + L.wx32) : nullptr;
  q.wy32 = L.wy32 ? (const float *)(ws + L.wy32) : nullptr;
  q.rowptr = op.rowptr;
  q.colind = op.colind;
  q.vals = op.vals;
  q.vals32 = L.vals32 ? (const float *)(ws + L.vals32) : nullptr;
  q.x[1] = (double *)(ws + L.x1);
  q.g[0] = (double *)(ws + L.g0);
  q.g[1] = (double *)(ws + L.g1);
  q.rho[0] = ws + L.rho0;
  q.rho[1] = ws + L.rho1;
  q.uq[0] = ws + L.uq0;
  q.uq[1] = ws + L.uq1;
  q.sq[0] = ws + L.sq0;
  q.sq[1] = ws + L.sq1;
  q.pv = ws + L.p;
  q.wv = ws + L.w;
  q.mask = (uint8_t *)(ws + L.mask);
  q.list = L.list ? (int32_t *)(ws + L.list) : nullptr;
  q.mrow = L.mrow ? (int32_t *)(ws + L.mrow) : nullptr;
  q.mcol = L.mcol ? (int32_t *)(ws + L.mcol) : nullptr;
  q.mval = L.mval ? (void *)(ws + L.mval) : nullptr;
  q.dinv = L.dinv ? (const void *)(ws + L.dinv) : nullptr;
  q.host_flag = h->flag.dev;
  put_options(q, h->opt);
}

// Uploads the state of a new solve of handle h (not yet started).
int upload_solve(gpcg_handle_s *h, const double *b, const double *l, const double *u, double *x,
                 int32_t *flag_dev, bool fused, hipStream_t stream) {
  QPDev &q = *h->stage;
  std::memset(&q, 0, sizeof(q));
  q.st = h->st;
  q.st.b = b;
  q.st.l = l;
  q.st.u = u;
  q.st.x[0] = x;
  q.st.host_flag = flag_dev;
  // trial passes look ahead in the fused form only (its kernel carries the
  // code; the split form's lean data kernel keeps its register budget)
  q.st.gp_la = (fused && h->st.op_kind != OPK_CSR && h->st.tile == kBlock &&
                h->opt.lookahead != GPCG_LOOKAHEAD_OFF)
                   ? 1
                   : 0;
  initial_dyn(q.dyn[0]);
  initial_dyn(q.dyn[1]);
  COPY_OK(h->dqp, h->stage_dev, sizeof(QPDev), stream);
  return GPCG_OK;
}

// After the solve: the answer into the caller's x when it sits in the spare
// copy, the gradient into g_out; the final state into the staging copy.
int finish_solve(gpcg_handle_s *h, int final_parity, double *g_out, hipStream_t stream) {
  HIP_OK(hipMemcpyAsync(h->stage, h->dqp, sizeof(QPDev), hipMemcpyDeviceToHost, stream));
  HIP_OK(hipStreamSynchronize(stream));
  const QPCore &d = h->stage->dyn[final_parity].c;
  const QPStatic &s = h->stage->st;
  const size_t bytes = sizeof(double) * (size_t)s.n;
  if (d.cur == 1) COPY_OK(s.x[0], s.x[1], bytes, stream);
  if (g_out) COPY_OK(g_out, s.g[d.cur], bytes, stream);
  HIP_OK(hipStreamSynchronize(stream));
  return GPCG_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

void gpcg_options_default(gpcg_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol_rel = 1e-8;
  o->tol_abs = 0.0;
  o->eta1 = 0.1;
  o->eta2 = 0.05;
  o->eta2_reduce = 0.1;
  o->mu = 0.01;
  o->max_outer = 100000;
  o->max_gp = 50;
  o->max_backtrack = 60;
  o->max_cg = 0;
  o->precision = GPCG_PREC_FP64;
  o->free_set = GPCG_FREESET_MASK;
  o->tile = 0;
  o->chunk = 0;
  o->use_graph = 1;
  o->max_stall = 100;
  o->form = GPCG_FORM_AUTO;
  o->tiles_per_wg = 0;
  o->prefetch = GPCG_PREFETCH_AUTO;
  o->precond = GPCG_PRECOND_NONE;
  o->cg_stop = GPCG_CGSTOP_DECREASE;
  o->lookahead = GPCG_LOOKAHEAD_AUTO;
  o->cg_kernel = GPCG_CGK_AUTO;
}

int gpcg_workspace_bytes(const gpcg_operator *op, const gpcg_options *opt, size_t *bytes) {
  if (!bytes) return fail(GPCG_ERR_ARG, "bytes is NULL");
  int rc = validate_op(op);
  if (rc) return rc;
  gpcg_options o;
  if (opt) o = *opt;
  else gpcg_options_default(&o);
  rc = validate_opt(&o);
  if (rc) return rc;
  rc = validate_pair(op, o);
  if (rc) return rc;
  *bytes = layout_for(op, o.precision, o.tile, o.free_set, o.precond).total;
  return GPCG_OK;
}

int gpcg_create(const gpcg_operator *op, const gpcg_options *opt, void *workspace,
                size_t ws_bytes, void *stream, gpcg_handle *out) {
  if (!out) return fail(GPCG_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate_op(op);
  if (rc) return rc;
  gpcg_options o;
  if (opt) o = *opt;
  else gpcg_options_default(&o);
  rc = validate_opt(&o);
  if (rc) return rc;
  rc = validate_pair(op, o);
  if (rc) return rc;
  Layout L = layout_for(op, o.precision, o.tile, o.free_set, o.precond);
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0)
    return fail(GPCG_ERR_WORKSPACE, "workspace missing or not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(GPCG_ERR_WORKSPACE, "workspace smaller than gpcg_workspace_bytes()");
  auto *h = new gpcg_handle_s();
  h->op = *op;
  h->opt = o;
  h->stream = (hipStream_t)stream;
  h->ws = (char *)workspace;
  h->ws_bytes = ws_bytes;
  h->L = L;
  h->dqp = (QPDev *)(h->ws + L.qp);
  h->tick_hz = wall_clock_hz();
  auto cleanup = [&](int code) {
    gpcg_destroy(h);
    return code;
  };
  rc = alloc_flag(&h->flag, 16);
  if (rc) return cleanup(rc);
  void *st = nullptr, *st_dev = nullptr;
  rc = alloc_pinned(&st, &st_dev, sizeof(QPDev));
  if (rc) return cleanup(rc);
  h->stage = (QPDev *)st;
  h->stage_dev = (QPDev *)st_dev;
  fill_static(h);
  h->cfg.split = o.form == GPCG_FORM_SPLIT ||
                 (o.form == GPCG_FORM_AUTO && h->st.n > (int64_t)kFusedMaxTiles * kBlock);
  h->cfg.tiles_per_wg = o.tiles_per_wg > 0 ? o.tiles_per_wg : 1;
  h->cfg.spec = spec_ok(h->st) && o.prefetch != GPCG_PREFETCH_OFF ? 1 : 0;
  h->cfg.chunk = default_chunk(o);
  h->cfg.cgk = o.cg_kernel == GPCG_CGK_ON ? 1 : 0;
  if (o.form == GPCG_FORM_AUTO && o.tiles_per_wg == 0 && o.chunk == 0 &&
      o.prefetch == GPCG_PREFETCH_AUTO && o.cg_kernel == GPCG_CGK_AUTO) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(h));
    if (it != g_tuned.end()) h->cfg = it->second;
  }
  // early operand loads need a stencil QP with one unknown per thread
  if (!spec_ok(h->st)) h->cfg.spec = 0;
  if (hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(GPCG_ERR_HIP, "hipEventCreate failed"));
  // FP32 copy of the operator for the mixed form
  if (L.wx32) {
    if (gpcg_launch_convert_f32(op->wx, (float *)(h->ws + L.wx32),
                                (int64_t)op->ny * (op->nx + 1), stream) ||
        gpcg_launch_convert_f32(op->wy, (float *)(h->ws + L.wy32),
                                (int64_t)(op->ny + 1) * op->nx, stream))
      return cleanup(fail(GPCG_ERR_HIP, "FP32 weight conversion failed"));
  }
  if (L.vals32 &&
      gpcg_launch_convert_f32(op->vals, (float *)(h->ws + L.vals32), op->nnz, stream))
    return cleanup(fail(GPCG_ERR_HIP, "FP32 value conversion failed"));
  // the operator part of the device state is valid from here on (the
  // building-block kernels read it; solves rewrite only the vector pointers)
  h->stage->st = h->st;
  if (gpcg_launch_copy(&h->dqp->st, &h->stage_dev->st, sizeof(QPStatic), h->stream) != 0)
    return cleanup(fail(GPCG_ERR_HIP, "state upload failed in create"));
  // Jacobi preconditioner: 1 / diag(A) from the operator in the device state
  if (L.dinv && gpcg_launch_diag_inv(h->dqp, h->ws + L.dinv, h->st.mixed, h->stream) != 0)
    return cleanup(fail(GPCG_ERR_HIP, "preconditioner set-up failed"));
  if (hipStreamSynchronize(h->stream) != hipSuccess)
    return cleanup(fail(GPCG_ERR_HIP, "stream synchronize failed in create"));
  *out = h;
  return GPCG_OK;
}

int gpcg_destroy(gpcg_handle h) {
  if (!h) return GPCG_OK;
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  for (auto &e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->stage) (void)hipHostFree(h->stage);
  if (h->flag.host) (void)hipHostFree(h->flag.host);
  delete h;
  return GPCG_OK;
}

int gpcg_solve(gpcg_handle h, const double *b, const double *l, const double *u, double *x,
               double *g_out, gpcg_stats *stats) {
  if (!h) return fail(GPCG_ERR_ARG, "handle is NULL");
  if (!b || !l || !u || !x) return fail(GPCG_ERR_ARG, "b, l, u and x are required");
  const double t0 = now_s();
  HIP_OK(hipStreamSynchronize(h->stream));  // the staging buffer may still be in flight
  h->flag.host[0] = 0;
  int rc = upload_solve(h, b, l, u, x, h->flag.dev, !h->cfg.split, h->stream);
  if (rc) return rc;
  StepLaunch SL{};
  SL.single = h->dqp;
  SL.nqp = 1;
  SL.total_tiles = h->L.ntiles;
  const LaunchCfg c = h->cfg;
  const int variant = (c.spec ? kVarSpec : 0) | (h->st.dinv ? kVarPre : 0) |
                      (c.split && c.cgk ? kVarCgk : 0) | (h->st.mrow ? kVarMat : 0);
  SL.tiles_per_wg = c.tiles_per_wg;
  SL.data_grid = (h->L.ntiles + c.tiles_per_wg - 1) / c.tiles_per_wg;
  const int chunk = c.chunk;
  if (h->opt.use_graph && (!h->graph || h->graph_cfg != c)) {
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    rc = build_chain_graph(SL, h->st.mixed, variant, c.split, chunk, &h->graph);
    if (rc) return rc;
    h->graph_cfg = c;
  }
  int64_t launches = 0, checks = 0;
  volatile int32_t *flag = h->flag.host;
  rc = run_until(h->stream, SL, h->st.mixed, variant, c.split, chunk,
                 h->opt.use_graph ? h->graph : nullptr, h->ev,
                 [&] { return *flag != 0; }, (int64_t)1 << 26, &launches, &checks);
  if (rc) return rc;
  rc = finish_solve(h, (int)(launches & 1), g_out, h->stream);
  if (rc) return rc;
  const QPDyn &dy = h->stage->dyn[launches & 1];
  const QPCore &d = dy.c;
  if (stats) {
    fill_stats(h->stage->st, dy, h->tick_hz, stats);
    stats->launches = launches;
    stats->host_checks = checks;
    stats->ms_total = (now_s() - t0) * 1e3;
  }
  if (d.status < 0) g_last_error = gpcg_status_string(d.status);
  return d.status;
}

namespace {

// Times one solve of the problem under configuration c (the first solve under
// a configuration builds its graph and is not timed).
int timed_solve(gpcg_handle h, const LaunchCfg &c, const double *b, const double *l,
                const double *u, const double *x0, double *x, double *ms) {
  const LaunchCfg keep = h->cfg;
  h->cfg = c;
  double best = 1e300;
  int rc = GPCG_OK;
  for (int rep = 0; rep < 2 && rc >= 0; ++rep) {
    if (gpcg_launch_copy(x, x0, sizeof(double) * (size_t)h->st.n, h->stream) != 0 ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      rc = fail(GPCG_ERR_HIP, "copy of x0 failed in autotune");
      break;
    }
    const double t0 = now_s();
    rc = gpcg_solve(h, b, l, u, x, nullptr, nullptr);
    const double t = (now_s() - t0) * 1e3;
    if (rep == 1) best = t;
  }
  h->cfg = keep;
  *ms = best;
  return rc;
}

void note(gpcg_tune_report *r, const LaunchCfg &c, double ms) {
  if (!r || r->count >= GPCG_TUNE_MAX) return;
  gpcg_tune_entry &e = r->cand[r->count++];
  e.form = c.split ? GPCG_FORM_SPLIT : GPCG_FORM_FUSED;
  e.tiles_per_wg = c.tiles_per_wg;
  e.prefetch = c.spec;
  e.chunk = c.chunk;
  e.shrink = c.shrink;
  e.cg_kernel = c.cgk;
  e.ms = ms;
}

}  // namespace

int gpcg_autotune(gpcg_handle h, const double *b, const double *l, const double *u,
                  const double *x0, double *x_work, gpcg_tune_report *report) {
  if (!h || !b || !l || !u || !x0 || !x_work)
    return fail(GPCG_ERR_ARG, "handle, b, l, u, x0 and x_work are required");
  if (report) std::memset(report, 0, sizeof(*report));
  const size_t n = (size_t)h->st.n;
  std::vector<double> first(n), other(n);
  LaunchCfg best = h->cfg;
  double best_ms = 0.0;
  int rc = timed_solve(h, best, b, l, u, x0, x_work, &best_ms);
  if (rc < 0) return rc;
  note(report, best, best_ms);
  HIP_OK(hipMemcpy(first.data(), x_work, sizeof(double) * n, hipMemcpyDeviceToHost));
  int mismatches = 0;
  auto consider = [&](LaunchCfg c) -> int {
    if (c == best) return GPCG_OK;
    double ms = 0.0;
    const int r = timed_solve(h, c, b, l, u, x0, x_work, &ms);
    if (r < 0) return r;
    note(report, c, ms);
    HIP_OK(hipMemcpy(other.data(), x_work, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (std::memcmp(first.data(), other.data(), sizeof(double) * n) != 0) {
      ++mismatches;  // configurations must agree bitwise: never keep one that does not
      return GPCG_OK;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    return GPCG_OK;
  };
  // one dimension at a time: launch form, tiles per data workgroup, operand
  // prefetch, chunk length
  if (h->st.n <= (int64_t)4 * kFusedMaxTiles * kBlock) {
    LaunchCfg c = best;
    c.split = best.split ? 0 : 1;
    c.tiles_per_wg = 1;
    if ((rc = consider(c)) < 0) return rc;
  }
  if (best.split)
    for (int t : {1, 2, 4})
      if (t <= h->L.ntiles) {
        LaunchCfg c = best;
        c.tiles_per_wg = t;
        if ((rc = consider(c)) < 0) return rc;
      }
  if (best.split) {
    LaunchCfg c = best;
    c.cgk = best.cgk ? 0 : 1;
    if ((rc = consider(c)) < 0) return rc;
  }
  if (spec_ok(h->st)) {
    LaunchCfg c = best;
    c.spec = best.spec ? 0 : 1;
    if ((rc = consider(c)) < 0) return rc;
  }
  for (int ch : {16, 32, 64}) {
    LaunchCfg c = best;
    c.chunk = ch;
    if ((rc = consider(c)) < 0) return rc;
  }
  h->cfg = best;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[tune_key(h)] = best;
  }
  if (report) {
    report->mismatches = mismatches;
    report->chosen.form = best.split ? GPCG_FORM_SPLIT : GPCG_FORM_FUSED;
    report->chosen.tiles_per_wg = best.tiles_per_wg;
    report->chosen.prefetch = best.spec;
    report->chosen.chunk = best.chunk;
    report->chosen.cg_kernel = best.cgk;
    report->chosen.ms = best_ms;
  }
  if (mismatches) return fail(GPCG_ERR_HIP, "autotune: launch configurations disagreed");
  return GPCG_OK;
}

// Grid width for the vector-load SpMV kernel, or 0 to use the scalar one
// (CSR, or edge weights not aligned to the vector width).
static int spmv_vec_nx(const gpcg_handle_s *h, int f32) {
  if (h->st.op_kind == OPK_CSR) return 0;
  const void *wy = f32 ? (const void *)h->st.wy32 : (const void *)h->st.wy;
  if (h->st.op_kind == OPK_VAR && ((uintptr_t)wy % 16) != 0) return 0;
  return h->st.nx;
}

int gpcg_spmv(gpcg_handle h, const double *v, double *y, const uint8_t *mask) {
  if (!h || !v || !y) return fail(GPCG_ERR_ARG, "handle, v and y are required");
  // the kernel reads the operator from the device state uploaded at create
  if (gpcg_launch_spmv(h->dqp, &h->st, h->st.n, v, y, mask, 0, spmv_vec_nx(h, 0),
                       h->stream))
    return fail(GPCG_ERR_HIP, "spmv launch failed");
  return GPCG_OK;
}

int gpcg_spmv_f32(gpcg_handle h, const float *v, float *y, const uint8_t *mask) {
  if (!h || !v || !y) return fail(GPCG_ERR_ARG, "handle, v and y are required");
  if (!h->st.mixed) return fail(GPCG_ERR_ARG, "handle was not created with GPCG_PREC_MIXED");
  if (gpcg_launch_spmv(h->dqp, &h->st, h->st.n, v, y, mask, 1, spmv_vec_nx(h, 1),
                       h->stream))
    return fail(GPCG_ERR_HIP, "spmv launch failed");
  return GPCG_OK;
}

int gpcg_projected_gradient(gpcg_handle h, const double *x, const double *l, const double *u,
                            const double *g, double *pg, double *norm2, int64_t *n_lower,
                            int64_t *n_upper, int64_t *n_nonbinding) {
  if (!h || !x || !l || !u || !g) return fail(GPCG_ERR_ARG, "handle, x, l, u, g required");
  double *part = (double *)(h->ws + h->L.pgpart);
  double *out4 = part + 4 * kPgradMaxBlocks;
  if (gpcg_launch_pgrad(h->st.n, x, l, u, g, pg, part, out4, h->stream))
    return fail(GPCG_ERR_HIP, "projected-gradient launch failed");
  double r[4];
  HIP_OK(hipMemcpyAsync(r, out4, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  if (norm2) *norm2 = r[0];
  if (n_lower) *n_lower = (int64_t)r[1];
  if (n_upper) *n_upper = (int64_t)r[2];
  if (n_nonbinding) *n_nonbinding = (int64_t)r[3];
  return GPCG_OK;
}

int gpcg_projected_gradient_noalloc(int64_t n, const double *x, const double *l,
                                    const double *u, const double *g, double *pg,
                                    double *norm2, int64_t *n_lower, int64_t *n_upper,
                                    int64_t *n_nonbinding, void *stream) {
  if (!x || !l || !u || !g) return fail(GPCG_ERR_ARG, "x, l, u, g required");
  if (n < 1 || n > GPCG_NOALLOC_MAX_N)
    return fail(GPCG_ERR_ARG, "gpcg_projected_gradient_noalloc: n must be in [1, " +
                                  std::to_string((long long)GPCG_NOALLOC_MAX_N) + "], got " +
                                  std::to_string((long long)n));
  const hipStream_t st = (hipStream_t)stream;
  const double *tot = nullptr;
  const int rc = gpcg_launch_pgrad_scratch(n, x, l, u, g, pg, &tot, st);
  if (rc == -1) return fail(GPCG_ERR_HIP, "no current HIP device");
  if (rc == -2) return fail(GPCG_ERR_HIP, "hipGetSymbolAddress of the scratch array failed");
  if (rc) return fail(GPCG_ERR_HIP, "projected-gradient launch failed");
  double r[4];
  HIP_OK(hipMemcpyAsync(r, tot, sizeof(r), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (norm2) *norm2 = r[0];
  if (n_lower) *n_lower = (int64_t)r[1];
  if (n_upper) *n_upper = (int64_t)r[2];
  if (n_nonbinding) *n_nonbinding = (int64_t)r[3];
  return GPCG_OK;
}

const char *gpcg_status_string(int s) {
  switch (s) {
    case GPCG_OK: return "converged";
    case GPCG_MAXIT: return "iteration limit reached";
    case GPCG_STAGNATED: return "stagnated: no sufficient decrease above rounding level";
    case GPCG_ERR_ARG: return "invalid argument";
    case GPCG_ERR_BOUNDS: return "lower bound above upper bound";
    case GPCG_ERR_NAN: return "NaN in the input";
    case GPCG_ERR_NOT_SPD: return "operator is not positive definite";
    case GPCG_ERR_WORKSPACE: return "workspace missing or too small";
    case GPCG_ERR_HIP: return "HIP runtime error";
    case GPCG_ERR_NOSPACE: return "request does not fit the arena";
    case GPCG_ERR_HANG: return "device did not make progress";
    default: return "unknown status";
  }
}

const char *gpcg_last_error(void) { return g_last_error.c_str(); }

const char *gpcg_build_info(void) {
  return "gpcg-mi355x 0.2 (HIP, offload gfx950, wave64, FP64 + mixed FP32 reduced CG)";
}

}  // extern "C"

// ================================================================== batches

namespace {

// Launch tables of a batch or the server: QP pointers, tile prefix sums (the
// persistent form's workgroup offsets) and the work items of the data kernel.
size_t tables_bytes(int count, size_t items) {
  return align_up(sizeof(void *) * (size_t)count) + align_up(sizeof(int32_t) * (count + 1)) +
         align_up(sizeof(WgItem) * items);
}

size_t items_offset(int count) {
  return align_up(sizeof(void *) * (size_t)count) + align_up(sizeof(int32_t) * (count + 1));
}

// The device work queue of the queue form, after the tables: two counters,
// then two arrays (one per launch parity) of `items` work items.
size_t queue_bytes(size_t items) { return kAlign + align_up(sizeof(WgItem) * 2 * items); }


// Work items of a split data kernel over the QPs qp[0..cnt): runs of at most
// T consecutive tiles, QP by QP.  Returns the number of items.
int fill_items(WgItem *out, QPDev *const *qp, const int32_t *ntiles, int cnt, int T) {
  int m = 0;
  for (int a = 0; a < cnt; ++a)
    for (int t = 0; t < ntiles[a]; t += T) {
      out[m].q = qp[a];
      out[m].tile0 = t;
      out[m].ntile = std::min(T, ntiles[a] - t);
      ++m;
    }
  return m;
}

// Workgroup slots per QP for the persistent form: proportional to the QP's
// share of all unknowns, at least one, at most eight (the per-QP barrier stays
// cheap) and at most its tile count; the total fits the co-resident
// workgroups.
std::vector<int32_t> persistent_slots(const std::vector<const QPStatic *> &qs, int capacity) {
  const int cnt = (int)qs.size();
  std::vector<int32_t> w(cnt, 1);
  if (cnt == 0 || capacity < cnt) return {};
  double total = 0.0;
  for (auto *q : qs) total += (double)q->n;
  int used = 0;
  for (int i = 0; i < cnt; ++i) {
    int want = (int)std::floor(capacity * (double)qs[i]->n / total);
    want = std::max(1, std::min({want, qs[i]->ntiles, 8}));
    w[i] = want;
    used += want;
  }
  while (used > capacity) {
    int arg = (int)(std::max_element(w.begin(), w.end()) - w.begin());
    if (w[arg] <= 1) break;
    --w[arg];
    --used;
  }
  return w;
}

int persistent_capacity(int mixed, int *cap) {
  int per_cu = 0;
  if (gpcg_persistent_max_blocks(mixed, &per_cu) != 0 || per_cu < 1)
    return fail(GPCG_ERR_HIP, "occupancy query for the persistent kernel failed");
  int dev = 0, cus = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  *cap = per_cu * cus;
  return GPCG_OK;
}

}  // namespace

struct gpcg_batch_s {
  std::vector<gpcg_handle> hs;
  hipStream_t stream;
  char *ws;
  size_t ws_bytes;
  QPDev **qptrs;       // device
  int32_t *prefix;     // device
  WgItem *items;       // device
  size_t tbytes;
  char *stage_dev;     // device address of the pinned tables (kBlock more: zeros)
  int32_t *qcount;     // device: the queue form's two counters
  WgItem *queue;       // device: 2 x queue_cap items
  size_t queue_cap;
  char *stage;         // pinned copy of the tables
  PinnedWords flags;   // one DONE word per QP
  hipEvent_t ev[2] = {nullptr, nullptr};
  int mixed;
  LaunchCfg cfg{};     // stepped form: always split; tiles, prefetch, chunk tunable
};

extern "C" {

namespace {
size_t batch_items(int count, const gpcg_handle *handles) {
  size_t items = 0;
  for (int i = 0; i < count; ++i) items += (size_t)handles[i]->L.ntiles;
  return items;
}
}  // namespace

int gpcg_batch_workspace_bytes(int count, const gpcg_handle *handles, size_t *bytes) {
  if (count < 1 || !bytes || !handles) return fail(GPCG_ERR_ARG, "count >= 1 and handles required");
  for (int i = 0; i < count; ++i)
    if (!handles[i]) return fail(GPCG_ERR_ARG, "NULL handle in batch");
  const size_t items = batch_items(count, handles);
  *bytes = tables_bytes(count, items) + queue_bytes(items);
  return GPCG_OK;
}

int gpcg_batch_create(int count, const gpcg_handle *handles, void *workspace, size_t ws_bytes,
                      void *stream, gpcg_batch *out) {
  if (!out || count < 1 || !handles) return fail(GPCG_ERR_ARG, "bad batch arguments");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    if (!handles[i]) return fail(GPCG_ERR_ARG, "NULL handle in batch");
    if (handles[i]->st.mixed != handles[0]->st.mixed)
      return fail(GPCG_ERR_ARG, "all handles of a batch must share the precision");
  }
  const size_t nitems = batch_items(count, handles);
  const size_t need = tables_bytes(count, nitems);
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 ||
      ws_bytes < need + queue_bytes(nitems))
    return fail(GPCG_ERR_WORKSPACE, "batch workspace missing, misaligned or too small");
  auto *b = new gpcg_batch_s();
  b->hs.assign(handles, handles + count);
  b->stream = (hipStream_t)stream;
  b->ws = (char *)workspace;
  b->ws_bytes = ws_bytes;
  b->qptrs = (QPDev **)b->ws;
  b->prefix = (int32_t *)(b->ws + align_up(sizeof(void *) * (size_t)count));
  b->items = (WgItem *)(b->ws + items_offset(count));
  b->tbytes = need;
  b->qcount = (int32_t *)(b->ws + align_up(need));
  b->queue = (WgItem *)(b->ws + align_up(need) + kAlign);
  b->queue_cap = nitems;
  b->mixed = handles[0]->st.mixed;
  // stepped batches: the split form unless the members ask for the fused one
  // (one launch per pass, every workgroup folding its own QP's slots: cheaper
  // for few small QPs, dearer for many large ones; the autotuner decides)
  b->cfg = LaunchCfg{handles[0]->opt.form == GPCG_FORM_FUSED ? 0 : 1, 1, 1,
                     default_chunk(handles[0]->opt), 0};
  if (handles[0]->opt.tiles_per_wg > 0) b->cfg.tiles_per_wg = handles[0]->opt.tiles_per_wg;
  b->cfg.cgk = handles[0]->opt.cg_kernel == GPCG_CGK_ON ? 1 : 0;
  b->cfg.spec = handles[0]->opt.prefetch == GPCG_PREFETCH_OFF ? 0 : 1;
  int rc = alloc_flag(&b->flags, (size_t)count);
  if (rc) {
    delete b;
    return rc;
  }
  void *st = nullptr, *st_dev = nullptr;
  rc = alloc_pinned(&st, &st_dev, b->tbytes + kAlign);
  if (rc) {
    gpcg_batch_destroy(b);
    return rc;
  }
  b->stage = (char *)st;
  b->stage_dev = (char *)st_dev;
  if (hipEventCreateWithFlags(&b->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev[1], hipEventDisableTiming) != hipSuccess) {
    gpcg_batch_destroy(b);
    return fail(GPCG_ERR_HIP, "hipEventCreate failed");
  }
  *out = b;
  return GPCG_OK;
}

int gpcg_batch_destroy(gpcg_batch b) {
  if (!b) return GPCG_OK;
  for (auto &e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->stage) (void)hipHostFree(b->stage);
  if (b->flags.host) (void)hipHostFree(b->flags.host);
  delete b;
  return GPCG_OK;
}

int gpcg_batch_solve(gpcg_batch b, const gpcg_problem *probs, int mode, gpcg_stats *stats) {
  if (!b || !probs) return fail(GPCG_ERR_ARG, "batch and problems are required");
  if (mode != GPCG_BATCH_STEPPED && mode != GPCG_BATCH_PERSISTENT)
    return fail(GPCG_ERR_ARG, "unknown batch mode");
  const int cnt = (int)b->hs.size();
  const double t0 = now_s();
  HIP_OK(hipStreamSynchronize(b->stream));
  for (int i = 0; i < cnt; ++i) {
    const gpcg_problem &p = probs[i];
    if (!p.b || !p.l || !p.u || !p.x) return fail(GPCG_ERR_ARG, "problem arrays missing");
    gpcg_handle h = b->hs[i];
    HIP_OK(hipStreamSynchronize(h->stream));
    b->flags.host[i] = 0;
    int rc = upload_solve(h, p.b, p.l, p.u, p.x, b->flags.dev + i, false, b->stream);
    if (rc) return rc;
  }
  auto **qp = (QPDev **)b->stage;
  auto *pre = (int32_t *)(b->stage + align_up(sizeof(void *) * (size_t)cnt));
  int64_t launches = 0, checks = 0;
  int final_parity = 0;
  if (mode == GPCG_BATCH_PERSISTENT) {
    int cap = 0;
    int rc = persistent_capacity(b->mixed, &cap);
    if (rc) return rc;
    std::vector<const QPStatic *> qs(cnt);
    for (int i = 0; i < cnt; ++i) qs[i] = &b->hs[i]->st;
    std::vector<int32_t> w = persistent_slots(qs, cap);
    if (w.empty()) return fail(GPCG_ERR_ARG, "more QPs than co-resident workgroups");
    pre[0] = 0;
    for (int i = 0; i < cnt; ++i) {
      qp[i] = b->hs[i]->dqp;
      pre[i + 1] = pre[i] + w[i];
    }
    const int grid = pre[cnt];
    COPY_OK(b->ws, b->stage_dev, b->tbytes, b->stream);
    int pre = 0;
    for (int i = 0; i < cnt; ++i) pre |= b->hs[i]->st.dinv ? 1 : 0;
    PersistLaunch P{b->qptrs, b->prefix, cnt, grid, (int64_t)1 << 22, pre, 0};
    if (gpcg_launch_persistent(P, grid, b->mixed, b->stream) != 0)
      return fail(GPCG_ERR_HIP, std::string("cooperative launch failed: ") +
                                    hipGetErrorString(hipGetLastError()));
    launches = 1;
    HIP_OK(hipStreamSynchronize(b->stream));
  } else {
    // stepped: replay chunks; shrink the launch to the unfinished QPs as they
    // complete (results do not depend on the launch composition)
    std::vector<int> active(cnt);
    for (int i = 0; i < cnt; ++i) active[i] = i;
    const int chunk = b->cfg.chunk;
    // the fused form (one launch per pass; every workgroup folds its own QP's
    // slots) unless chosen otherwise or some QP has too many tiles for it
    bool split = b->cfg.split != 0;
    for (int i = 0; i < cnt; ++i) split = split || b->hs[i]->st.ntiles > kFusedMaxTiles;
    const int T = split ? b->cfg.tiles_per_wg : 1;
    if (split && b->cfg.shrink == 0) {
      // queue form: one launch table for the whole solve; every transition
      // queues the work items of the QPs that are not done, and the data
      // kernel (a fixed grid) runs them, so finished QPs cost nothing and
      // the launch is never re-formed on the host
      bool pre = false, mat = false;
      for (int i = 0; i < cnt; ++i) {
        qp[i] = b->hs[i]->dqp;
        pre = pre || b->hs[i]->st.dinv != nullptr;
        mat = mat || b->hs[i]->st.mrow != nullptr;
      }
      COPY_OK(b->ws, b->stage_dev, b->tbytes, b->stream);
      COPY_OK(b->qcount, b->stage_dev + b->tbytes, 2 * sizeof(int32_t), b->stream);
      const int spec = kVarQueue | kVarLgp | (pre ? kVarPre : 0) | (b->cfg.cgk ? kVarCgk : 0) |
                       (mat ? kVarMat : 0);
      StepLaunch SL{};
      SL.qps = b->qptrs;
      SL.nqp = cnt;
      SL.tiles_per_wg = T;
      SL.item_tiles = T;
      SL.queue = b->queue;
      SL.qcount = b->qcount;
      SL.queue_cap = (int32_t)b->queue_cap;
      // one workgroup per item of the largest possible queue
      SL.data_grid = 0;
      for (int i = 0; i < cnt; ++i) SL.data_grid += (b->hs[i]->st.ntiles + T - 1) / T;
      hipGraphExec_t graph = nullptr;
      int rc = build_chain_graph(SL, b->mixed, spec, 1, chunk, &graph);
      if (rc) return rc;
      auto all_done = [&]() {
        for (int i = 0; i < cnt; ++i)
          if (!b->flags.host[i]) return false;
        return true;
      };
      rc = run_until(b->stream, SL, b->mixed, spec, 1, chunk, graph, b->ev, all_done,
                     (int64_t)1 << 26, &launches, &checks);
      (void)hipGraphExecDestroy(graph);
      if (rc) return rc;
      active.clear();
    }
    while (!active.empty()) {
      HIP_OK(hipStreamSynchronize(b->stream));  // the staged tables may still be in flight
      pre[0] = 0;
      std::vector<int32_t> nt(active.size());
      for (size_t a = 0; a < active.size(); ++a) {
        qp[a] = b->hs[active[a]]->dqp;
        nt[a] = b->hs[active[a]]->st.ntiles;
        pre[a + 1] = pre[a] + nt[a];
      }
      const int total = pre[active.size()];
      auto *items = (WgItem *)(b->stage + items_offset(cnt));
      const int nitems = fill_items(items, qp, nt.data(), (int)active.size(), T);
      COPY_OK(b->ws, b->stage_dev, b->tbytes, b->stream);
      StepLaunch SL{};
      SL.qps = b->qptrs;
      SL.items = b->items;
      SL.nqp = (int32_t)active.size();
      SL.total_tiles = total;
      SL.tiles_per_wg = T;
      SL.data_grid = nitems;
      bool sp = b->cfg.spec != 0, pre = false, mat = false;
      for (int i : active) {
        sp = sp && spec_ok(b->hs[i]->st);
        pre = pre || b->hs[i]->st.dinv != nullptr;
        mat = mat || b->hs[i]->st.mrow != nullptr;
      }
      const int spec = (sp ? kVarSpec : 0) | (pre ? kVarPre : 0) |
                       (split && b->cfg.cgk ? kVarCgk : 0) | (mat ? kVarMat : 0) |
                       (split ? kVarLgp : 0);
      hipGraphExec_t graph = nullptr;
      int rc = build_chain_graph(SL, b->mixed, spec, split ? 1 : 0, chunk, &graph);
      if (rc) return rc;
      // run until 1/shrink of this launch's tiles belong to finished QPs
      // (shrink 0, the queue form's setting, in the fused form: until all are)
      auto enough = [&]() {
        int done_tiles = 0;
        for (int i : active)
          if (b->flags.host[i]) done_tiles += b->hs[i]->st.ntiles;
        return b->cfg.shrink > 0 ? (int64_t)b->cfg.shrink * done_tiles >= total
                                 : done_tiles >= total;
      };
      rc = run_until(b->stream, SL, b->mixed, spec, split ? 1 : 0, chunk, graph, b->ev, enough,
                     (int64_t)1 << 26, &launches, &checks);
      (void)hipGraphExecDestroy(graph);
      if (rc) return rc;
      std::vector<int> still;
      for (int i : active)
        if (!b->flags.host[i]) still.push_back(i);
      active.swap(still);
    }
    final_parity = (int)(launches & 1);
  }
  int first_err = GPCG_OK;
  const double ms = (now_s() - t0) * 1e3;
  for (int i = 0; i < cnt; ++i) {
    gpcg_handle h = b->hs[i];
    int rc = finish_solve(h, final_parity, probs[i].g_out, b->stream);
    if (rc) return rc;
    const QPDyn &dy = h->stage->dyn[final_parity];
    if (dy.c.status < 0 && first_err == GPCG_OK) first_err = dy.c.status;
    if (stats) {
      fill_stats(h->stage->st, dy, h->tick_hz, &stats[i]);
      stats[i].launches = launches;
      stats[i].host_checks = checks;
      stats[i].ms_total = ms;
    }
  }
  if (first_err < 0) g_last_error = gpcg_status_string(first_err);
  return first_err;
}

int gpcg_batch_autotune(gpcg_batch b, const gpcg_problem *probs, const double *const *x0s,
                        gpcg_tune_report *report) {
  if (!b || !probs || !x0s) return fail(GPCG_ERR_ARG, "batch, problems and x0s are required");
  if (report) std::memset(report, 0, sizeof(*report));
  const int cnt = (int)b->hs.size();
  size_t total = 0;
  for (int i = 0; i < cnt; ++i) {
    if (!x0s[i] || !probs[i].x) return fail(GPCG_ERR_ARG, "x0s[i] and probs[i].x are required");
    total += (size_t)b->hs[i]->st.n;
  }
  std::vector<double> first(total), other(total);
  // two solves per configuration, the faster one counts (the first of a
  // configuration also builds its graphs)
  auto run = [&](const LaunchCfg &c, double *ms, std::vector<double> &out) -> int {
    const LaunchCfg keep = b->cfg;
    b->cfg = c;
    *ms = 1e300;
    int rc = GPCG_OK;
    for (int rep = 0; rep < 2 && rc >= 0; ++rep) {
      for (int i = 0; i < cnt; ++i)
        COPY_OK(probs[i].x, x0s[i], sizeof(double) * (size_t)b->hs[i]->st.n, b->stream);
      HIP_OK(hipStreamSynchronize(b->stream));
      const double t0 = now_s();
      rc = gpcg_batch_solve(b, probs, GPCG_BATCH_STEPPED, nullptr);
      const double t = (now_s() - t0) * 1e3;
      if (t < *ms) *ms = t;
    }
    b->cfg = keep;
    if (rc < 0) return rc;
    size_t off = 0;
    for (int i = 0; i < cnt; ++i) {
      const size_t n = (size_t)b->hs[i]->st.n;
      HIP_OK(hipMemcpy(out.data() + off, probs[i].x, sizeof(double) * n, hipMemcpyDeviceToHost));
      off += n;
    }
    return GPCG_OK;
  };
  LaunchCfg best = b->cfg;
  double best_ms = 0.0;
  int rc = run(best, &best_ms, first);
  if (rc < 0) return rc;
  note(report, best, best_ms);
  int mismatches = 0;
  auto consider = [&](LaunchCfg c) -> int {
    if (c == best) return GPCG_OK;
    double ms = 0.0;
    const int r = run(c, &ms, other);
    if (r < 0) return r;
    note(report, c, ms);
    if (std::memcmp(first.data(), other.data(), sizeof(double) * total) != 0) {
      ++mismatches;
      return GPCG_OK;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    return GPCG_OK;
  };
  {  // launch form: fused (one launch per pass) or split
    LaunchCfg c = best;
    c.split = best.split ? 0 : 1;
    if ((rc = consider(c)) < 0) return rc;
  }
  if (best.split)
    for (int t : {1, 2, 4}) {
      LaunchCfg c = best;
      c.tiles_per_wg = t;
      if ((rc = consider(c)) < 0) return rc;
    }
  {
    LaunchCfg c = best;
    c.spec = best.spec ? 0 : 1;
    if ((rc = consider(c)) < 0) return rc;
  }
  for (int ch : {16, 32, 64}) {
    LaunchCfg c = best;
    c.chunk = ch;
    if ((rc = consider(c)) < 0) return rc;
  }
  for (int sh : {0, 3, 6, 12}) {
    LaunchCfg c = best;
    c.shrink = sh;
    if ((rc = consider(c)) < 0) return rc;
  }
  // the CG kernel of its own last, and the schedule again if it is taken
  if (best.split) {
    LaunchCfg c = best;
    c.cgk = best.cgk ? 0 : 1;
    if ((rc = consider(c)) < 0) return rc;
  }
  if (best.split && best.cgk)
    for (int sh : {0, 3, 6, 12}) {
      LaunchCfg c = best;
      c.shrink = sh;
      if ((rc = consider(c)) < 0) return rc;
    }
  b->cfg = best;
  if (report) {
    report->mismatches = mismatches;
    report->chosen.form = best.split ? GPCG_FORM_SPLIT : GPCG_FORM_FUSED;
    report->chosen.tiles_per_wg = best.tiles_per_wg;
    report->chosen.prefetch = best.spec;
    report->chosen.chunk = best.chunk;
    report->chosen.shrink = best.shrink;
    report->chosen.cg_kernel = best.cgk;
    report->chosen.ms = best_ms;
  }
  if (mismatches) return fail(GPCG_ERR_HIP, "batch autotune: launch configurations disagreed");
  return GPCG_OK;
}

}  // extern "C"

// ================================================================== serving

namespace {

// Arena bytes of one request: its QPDev, the workspace layout of a handle for
// its operator, resident copies of b, l, u and the start, and for
// edge-weighted stencils the weights.
struct ReqLayout {
  Layout L;
  size_t b, l, u, x0, wx, wy, total;
};

// Served requests always run in the split form, whose data kernel keeps the
// loads of two 256-unknown chunks in flight per workgroup with 512-unknown
// tiles; the fused form's reasons for 256-unknown tiles on small QPs (early
// operand loads, look-ahead) do not apply.
ReqLayout req_layout(const gpcg_operator *op, int precision) {
  static_assert(GPCG_SERVER_TILE % kBlock == 0, "server tile");
  ReqLayout R{};
  R.L = layout_for(op, precision, GPCG_SERVER_TILE, GPCG_FREESET_MASK, GPCG_PRECOND_NONE);
  const int64_t n = op_n(op);
  size_t off = R.L.total;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  R.b = take(8 * (size_t)n);
  R.l = take(8 * (size_t)n);
  R.u = take(8 * (size_t)n);
  R.x0 = take(8 * (size_t)n);
  R.wx = R.wy = 0;
  if (op->kind == GPCG_OP_STENCIL5_VAR) {
    R.wx = take(8 * (size_t)op->ny * (op->nx + 1));
    R.wy = take(8 * (size_t)(op->ny + 1) * op->nx);
  }
  R.total = off;
  return R;
}

struct SrvSlot {
  bool used = false;
  bool retiring = false;  // done on the device; its answer is being copied out
  size_t off = 0, bytes = 0;
  gpcg_request req{};
  double t_submit = 0, t_admit = 0;
  int ntiles = 0;
  int final_parity = 0;
};

struct SrvPending {
  gpcg_request req;
  double t_submit;
  size_t bytes;
};

// Copies of finished requests' answers and states in flight on the stream,
// completed when `ev` has passed.
struct SrvRetire {
  hipEvent_t ev;
  std::vector<int> slots;
};

}  // namespace

// The server runs the queue form of the split launch over a fixed device
// table of max_slots QP pointers (null: an empty slot): every pass, the
// transition kernel queues the work items of the resident requests that are
// not done and the data kernel runs them, so a request that finishes costs
// nothing for the rest of the chunk.  Chunks of `quantum` passes are queued as plain
// launches (the data grid covers the running requests' tiles), at most two
// chunks in flight; between them the host admits requests
// (uploads queued on the stream, table entry set), notices finished ones
// from their mapped done words, queues the copies of their answers and
// states, and completes them once those copies have passed: nothing waits
// for the whole stream.
struct gpcg_server_s {
  gpcg_server_options opt;
  hipStream_t stream;
  char *arena;
  size_t header;        // device table and work queue at the start of the arena
  QPDev **qptrs;        // device table, max_slots entries
  int32_t *qcount;      // device: the queue's two counters
  WgItem *queue;        // device: 2 x item_cap items
  size_t item_cap;
  QPDev **tab_host;     // host copy of the table
  QPDev **tab_stage[2]; // pinned staging of table uploads
  QPDev **tab_stage_dev[2];
  hipEvent_t tab_ev[2] = {nullptr, nullptr};
  int tab_next = 0;
  bool tab_dirty = false;
  QPDev *stage;         // pinned, one per slot
  QPDev *stage_dev;     // its device address
  char *zeros_dev;      // device address of a pinned zero block
  PinnedWords flags;    // one done word per slot
  std::vector<SrvSlot> slots;
  std::deque<SrvPending> queue_in;
  std::deque<gpcg_completion> done;
  std::deque<SrvRetire> retiring;
  std::vector<hipEvent_t> ev_pool;
  std::map<size_t, size_t> free_list;  // offset -> bytes, coalesced
  int resident = 0;     // admitted and not yet completed (retiring included)
  int running = 0;      // admitted and not yet noticed done
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};
  int64_t chunks = 0;   // chunks issued
  int64_t chunks_seen = 0;  // chunks known complete
  double tick_hz;
  gpcg_options solve_opt;

  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_list.begin(); it != free_list.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_list.erase(it);
        if (rest) free_list[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_list.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_list.erase(nx);
    }
    if (it != free_list.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_list.erase(it);
      }
    }
  }
  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
};

namespace {

int srv_admit(gpcg_server_s *s, int slot_id, const SrvPending &p, size_t off) {
  SrvSlot &sl = s->slots[slot_id];
  const gpcg_request &rq = p.req;
  const gpcg_operator &op = rq.op;
  const ReqLayout R = req_layout(&op, s->opt.precision);
  const Layout &L = R.L;
  char *base = s->arena + off;
  const int64_t n = op_n(&op);
  hipStream_t st = s->stream;
  const size_t vb = 8 * (size_t)n;
  COPY_OK(base + R.b, rq.b, vb, st);
  COPY_OK(base + R.l, rq.l, vb, st);
  COPY_OK(base + R.u, rq.u, vb, st);
  COPY_OK(base + R.x0, rq.x0, vb, st);
  const size_t ex = (size_t)op.ny * (op.nx + 1), ey = (size_t)(op.ny + 1) * op.nx;
  if (op.kind == GPCG_OP_STENCIL5_VAR) {
    COPY_OK(base + R.wx, op.wx, 8 * ex, st);
    COPY_OK(base + R.wy, op.wy, 8 * ey, st);
    if (L.wx32 &&
        (gpcg_launch_convert_f32((const double *)(base + R.wx), (float *)(base + L.wx32),
                                 (int64_t)ex, st) ||
         gpcg_launch_convert_f32((const double *)(base + R.wy), (float *)(base + L.wy32),
                                 (int64_t)ey, st)))
      return fail(GPCG_ERR_HIP, "FP32 weight conversion failed");
  }
  // the slot's staging copy is free: its last use (the retirement of the
  // request before) completed before the slot was released
  QPDev &q = s->stage[slot_id];
  std::memset(&q, 0, sizeof(q));
  QPStatic &S = q.st;
  S.op_kind = op.kind == GPCG_OP_STENCIL5_CONST ? OPK_CONST : OPK_VAR;
  S.nx = op.nx;
  S.ny = op.ny;
  S.n = n;
  S.tile = L.tile;
  S.ntiles = L.ntiles;
  S.mixed = s->opt.precision == GPCG_PREC_MIXED ? 1 : 0;
  magic_for(S.nx, &S.div_magic, &S.div_shift);
  S.w = op.w;
  S.w32 = (float)op.w;
  S.wx = R.wx ? (const double *)(base + R.wx) : nullptr;
  S.wy = R.wy ? (const double *)(base + R.wy) : nullptr;
  S.wx32 = L.wx32 ? (const float *)(base + L.wx32) : nullptr;
  S.wy32 = L.wy32 ? (const float *)(base + L.wy32) : nullptr;
  S.b = (const double *)(base + R.b);
  S.l = (const double *)(base + R.l);
  S.u = (const double *)(base + R.u);
  S.x[0] = (double *)(base + R.x0);
  S.x[1] = (double *)(base + L.x1);
  S.g[0] = (double *)(base + L.g0);
  S.g[1] = (double *)(base + L.g1);
  S.rho[0] = base + L.rho0;
  S.rho[1] = base + L.rho1;
  S.uq[0] = base + L.uq0;
  S.uq[1] = base + L.uq1;
  S.sq[0] = base + L.sq0;
  S.sq[1] = base + L.sq1;
  S.pv = base + L.p;
  S.wv = base + L.w;
  S.mask = (uint8_t *)(base + L.mask);
  S.host_flag = s->flags.dev + slot_id;
  put_options(S, s->solve_opt);
  initial_dyn(q.dyn[0]);
  initial_dyn(q.dyn[1]);
  s->flags.host[slot_id] = 0;
  COPY_OK(base + L.qp, &s->stage_dev[slot_id], sizeof(QPDev), st);
  sl.used = true;
  sl.retiring = false;
  sl.off = off;
  sl.bytes = p.bytes;
  sl.req = rq;
  sl.t_submit = p.t_submit;
  sl.t_admit = now_s();
  sl.ntiles = L.ntiles;
  s->tab_host[slot_id] = (QPDev *)(base + L.qp);
  s->tab_dirty = true;
  s->resident += 1;
  s->running += 1;
  return GPCG_OK;
}

// Requests whose done word is set: their answers and final states are copied
// out behind the chunks already queued (the device never writes a finished
// request's x again), and they leave the device table.
int srv_notice_done(gpcg_server_s *s) {
  SrvRetire r{};
  for (int i = 0; i < (int)s->slots.size(); ++i) {
    SrvSlot &sl = s->slots[i];
    if (!sl.used || sl.retiring) continue;
    const int32_t w = s->flags.host[i];
    if (!w) continue;
    const int cur = (w >> 1) & 1;
    sl.final_parity = (w >> 2) & 1;
    const ReqLayout R = req_layout(&sl.req.op, s->opt.precision);
    char *base = s->arena + sl.off;
    if (sl.req.x_out)
      COPY_OK(sl.req.x_out, base + (cur ? R.L.x1 : R.x0), 8 * (size_t)op_n(&sl.req.op),
              s->stream);
    HIP_OK(hipMemcpyAsync(&s->stage[i], base + R.L.qp, sizeof(QPDev), hipMemcpyDeviceToHost,
                          s->stream));
    sl.retiring = true;
    s->tab_host[i] = nullptr;
    s->tab_dirty = true;
    s->running -= 1;
    r.slots.push_back(i);
  }
  if (r.slots.empty()) return GPCG_OK;
  r.ev = s->take_event();
  if (!r.ev) return fail(GPCG_ERR_HIP, "hipEventCreate failed");
  HIP_OK(hipEventRecord(r.ev, s->stream));
  s->retiring.push_back(std::move(r));
  return GPCG_OK;
}

// Completes the requests whose copies have passed; their slots and arena
// space are free again.
int srv_complete(gpcg_server_s *s) {
  while (!s->retiring.empty()) {
    SrvRetire &r = s->retiring.front();
    const hipError_t e = hipEventQuery(r.ev);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) return fail(GPCG_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
    const double t = now_s();
    for (int i : r.slots) {
      SrvSlot &sl = s->slots[i];
      const QPDyn &dy = s->stage[i].dyn[sl.final_parity];
      gpcg_completion c{};
      c.tag = sl.req.tag;
      fill_stats(s->stage[i].st, dy, s->tick_hz, &c.stats);
      c.status = dy.c.status;
      c.t_submit = sl.t_submit;
      c.t_admit = sl.t_admit;
      c.t_done = t;
      c.stats.ms_total = (t - sl.t_admit) * 1e3;
      s->done.push_back(c);
      s->release(sl.off, sl.bytes);
      sl.used = false;
      sl.retiring = false;
      s->flags.host[i] = 0;
      s->resident -= 1;
    }
    s->ev_pool.push_back(r.ev);
    s->retiring.pop_front();
  }
  return GPCG_OK;
}

// Queues the upload of the device table when it changed (double-buffered
// pinned staging: a staging copy is rewritten only after its last upload).
int srv_upload_table(gpcg_server_s *s) {
  if (!s->tab_dirty) return GPCG_OK;
  const int k = s->tab_next;
  HIP_OK(hipEventSynchronize(s->tab_ev[k]));
  const size_t bytes = sizeof(QPDev *) * s->slots.size();
  std::memcpy(s->tab_stage[k], s->tab_host, bytes);
  COPY_OK(s->qptrs, s->tab_stage_dev[k], bytes, s->stream);
  HIP_OK(hipEventRecord(s->tab_ev[k], s->stream));
  s->tab_next ^= 1;
  s->tab_dirty = false;
  return GPCG_OK;
}

}  // namespace

extern "C" {

int gpcg_server_footprint(const gpcg_operator *op, int precision, size_t *bytes) {
  if (!bytes) return fail(GPCG_ERR_ARG, "bytes is NULL");
  int rc = validate_op(op);
  if (rc) return rc;
  if (op->kind == GPCG_OP_CSR) return fail(GPCG_ERR_ARG, "the server takes stencil operators");
  if (precision != GPCG_PREC_FP64 && precision != GPCG_PREC_MIXED)
    return fail(GPCG_ERR_ARG, "unknown precision");
  *bytes = req_layout(op, precision).total;
  return GPCG_OK;
}

int gpcg_server_create(const gpcg_server_options *opt, void *stream, gpcg_server *out) {
  if (!opt || !out) return fail(GPCG_ERR_ARG, "options and out are required");
  *out = nullptr;
  if (opt->max_slots < 1 || opt->max_slots > 65536) return fail(GPCG_ERR_ARG, "max_slots");
  if (opt->precision != GPCG_PREC_FP64 && opt->precision != GPCG_PREC_MIXED)
    return fail(GPCG_ERR_ARG, "unknown precision");
  if (!(opt->tol_rel >= 0.0)) return fail(GPCG_ERR_ARG, "tol_rel < 0");
  if (opt->quantum < 0 || (opt->quantum & 1)) return fail(GPCG_ERR_ARG, "quantum must be even");
  if (!opt->arena || ((uintptr_t)opt->arena % kAlign) != 0)
    return fail(GPCG_ERR_WORKSPACE, "arena missing or not 256-byte aligned");
  // a resident request holds at least 24 bytes per unknown (x1, g0, g1), so
  // the arena holds at most arena / (24 * 256) tiles plus one partial tile per slot
  const size_t item_cap = (size_t)opt->max_slots + opt->arena_bytes / (24 * (size_t)kBlock);
  const size_t tab = align_up(sizeof(void *) * (size_t)opt->max_slots);
  const size_t header = tab + queue_bytes(item_cap);
  if (opt->arena_bytes <= header) return fail(GPCG_ERR_WORKSPACE, "arena too small");
  if (item_cap > (size_t)INT32_MAX) return fail(GPCG_ERR_ARG, "arena too large for the work queue");
  auto *s = new gpcg_server_s();
  s->opt = *opt;
  if (s->opt.quantum <= 0) s->opt.quantum = 64;
  s->stream = (hipStream_t)stream;
  s->arena = (char *)opt->arena;
  s->header = header;
  s->qptrs = (QPDev **)s->arena;
  s->qcount = (int32_t *)(s->arena + tab);
  s->queue = (WgItem *)(s->arena + tab + kAlign);
  s->item_cap = item_cap;
  s->slots.resize(opt->max_slots);
  s->free_list[header] = opt->arena_bytes - header;
  s->tick_hz = wall_clock_hz();
  gpcg_options_default(&s->solve_opt);
  s->solve_opt.tol_rel = opt->tol_rel;
  s->solve_opt.precision = opt->precision;
  s->tab_host = new QPDev *[opt->max_slots]();
  int rc = alloc_flag(&s->flags, (size_t)opt->max_slots);
  void *st = nullptr, *st_dev = nullptr;
  const size_t tbytes = sizeof(QPDev *) * (size_t)opt->max_slots;
  if (!rc) rc = alloc_pinned(&st, &st_dev, sizeof(QPDev) * opt->max_slots);
  s->stage = (QPDev *)st;
  s->stage_dev = (QPDev *)st_dev;
  for (int k = 0; !rc && k < 2; ++k) {
    void *t = nullptr, *td = nullptr;
    rc = alloc_pinned(&t, &td, tbytes + kAlign);  // the extra block stays zero
    s->tab_stage[k] = (QPDev **)t;
    s->tab_stage_dev[k] = (QPDev **)td;
  }
  if (!rc) s->zeros_dev = (char *)s->tab_stage_dev[1] + tbytes;
  for (int k = 0; !rc && k < 2; ++k)
    if (hipEventCreateWithFlags(&s->tab_ev[k], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->chunk_ev[k], hipEventDisableTiming) != hipSuccess)
      rc = fail(GPCG_ERR_HIP, "hipEventCreate failed");
  if (!rc) {
    // an empty table and a zero queue count, then the chunk graph over them
    std::memset(s->tab_stage[0], 0, tbytes);
    if (gpcg_launch_copy(s->qptrs, s->tab_stage_dev[0], tbytes, s->stream) != 0 ||
        gpcg_launch_copy(s->qcount, s->zeros_dev, 2 * sizeof(int32_t), s->stream) != 0 ||
        hipEventRecord(s->tab_ev[0], s->stream) != hipSuccess)
      rc = fail(GPCG_ERR_HIP, "server table initialisation failed");
  }
  if (rc) {
    gpcg_server_destroy(s);
    return rc;
  }
  *out = s;
  return GPCG_OK;
}

int gpcg_server_submit(gpcg_server s, const gpcg_request *req) {
  if (!s || !req) return fail(GPCG_ERR_ARG, "server and request are required");
  size_t bytes = 0;
  int rc = gpcg_server_footprint(&req->op, s->opt.precision, &bytes);
  if (rc) return rc;
  if (!req->b || !req->l || !req->u || !req->x0) return fail(GPCG_ERR_ARG, "request arrays");
  if (bytes > s->opt.arena_bytes - s->header)
    return fail(GPCG_ERR_NOSPACE, "request footprint exceeds the arena");
  s->queue_in.push_back(SrvPending{*req, now_s(), bytes});
  return GPCG_OK;
}

int gpcg_server_step(gpcg_server s, int *active) {
  if (!s) return fail(GPCG_ERR_ARG, "server is NULL");
  int rc = srv_notice_done(s);
  if (!rc) rc = srv_complete(s);
  if (rc) return rc;
  // admission: FIFO, by free slot and arena space; a new request starts at
  // the next chunk, whose first launch has parity 0 (chunks are even)
  while (!s->queue_in.empty()) {
    int slot = -1;
    for (int i = 0; i < (int)s->slots.size(); ++i)
      if (!s->slots[i].used) {
        slot = i;
        break;
      }
    if (slot < 0) break;
    size_t off = 0;
    if (!s->alloc(s->queue_in.front().bytes, &off)) break;
    rc = srv_admit(s, slot, s->queue_in.front(), off);
    if (rc) return rc;
    s->queue_in.pop_front();
  }
  rc = srv_upload_table(s);
  if (rc) return rc;
  if (s->running > 0) {
    // at most two chunks in flight: wait for the older one before queuing
    if (s->chunks - s->chunks_seen >= 2) {
      HIP_OK(hipEventSynchronize(s->chunk_ev[s->chunks_seen & 1]));
      s->chunks_seen += 1;
    }
    // the data kernel's grid covers the work items of every request still
    // running (one workgroup each); the queue can only shrink within a chunk
    int64_t tiles = 0;
    for (int i = 0; i < (int)s->slots.size(); ++i)
      if (s->tab_host[i]) tiles += s->slots[i].ntiles;
    StepLaunch SL{};
    SL.qps = s->qptrs;
    SL.nqp = (int32_t)s->slots.size();
    SL.tiles_per_wg = 1;
    SL.item_tiles = 1;
    SL.queue = s->queue;
    SL.qcount = s->qcount;
    SL.queue_cap = (int32_t)s->item_cap;
    SL.data_grid = (int32_t)std::max<int64_t>(1, tiles);
    const int mixed = s->opt.precision == GPCG_PREC_MIXED ? 1 : 0;
    for (int k = 0; k < s->opt.quantum; ++k) {
      SL.parity = k & 1;
      if (gpcg_launch_split(SL, mixed, kVarQueue | kVarLgp, s->stream) != 0)
        return fail(GPCG_ERR_HIP, "pass kernel launch failed");
    }
    HIP_OK(hipEventRecord(s->chunk_ev[s->chunks & 1], s->stream));
    s->chunks += 1;
  } else if (!s->retiring.empty() && s->queue_in.empty()) {
    // nothing left to run: wait for the copies of the last answers
    HIP_OK(hipEventSynchronize(s->retiring.back().ev));
    rc = srv_complete(s);
    if (rc) return rc;
  }
  if (active) *active = (int)s->queue_in.size() + s->resident;
  return GPCG_OK;
}

int gpcg_server_poll(gpcg_server s, gpcg_completion *out, int max, int *got) {
  if (!s || !got) return fail(GPCG_ERR_ARG, "server and got are required");
  int k = 0;
  while (k < max && !s->done.empty() && out) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *got = k;
  return GPCG_OK;
}

int gpcg_server_destroy(gpcg_server s) {
  if (!s) return GPCG_OK;
  (void)hipStreamSynchronize(s->stream);
  for (auto &r : s->retiring) (void)hipEventDestroy(r.ev);
  for (auto e : s->ev_pool) (void)hipEventDestroy(e);
  for (int k = 0; k < 2; ++k) {
    if (s->tab_ev[k]) (void)hipEventDestroy(s->tab_ev[k]);
    if (s->chunk_ev[k]) (void)hipEventDestroy(s->chunk_ev[k]);
    if (s->tab_stage[k]) (void)hipHostFree(s->tab_stage[k]);
  }
  delete[] s->tab_host;
  if (s->stage) (void)hipHostFree(s->stage);
  if (s->flags.host) (void)hipHostFree(s->flags.host);
  delete s;
  return GPCG_OK;
}

}  // extern "C"
