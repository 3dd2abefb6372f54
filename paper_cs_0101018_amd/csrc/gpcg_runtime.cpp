// gpcg_runtime.cpp -- host side of the C ABI declared in include/gpcg.h.
//
// The runtime validates descriptors, carves the caller's workspace, fills the
// device-resident QPState of every solve and then only replays launches of
// the pass kernel (as chunks of a HIP graph) until the device raises the DONE
// flag in mapped host memory.  All GPCG decisions are taken on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gpcg.h"
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
  if (o->free_set != GPCG_FREESET_MASK && o->free_set != GPCG_FREESET_LIST)
    return fail(GPCG_ERR_ARG, "unknown free-set mode");
  if (o->tile < 0 || o->tile % kBlock != 0 || o->tile > (1 << 16))
    return fail(GPCG_ERR_ARG, "tile must be a multiple of 256 in [256, 65536]");
  if (o->chunk < 0 || o->chunk > 4096) return fail(GPCG_ERR_ARG, "chunk out of range");
  if (o->max_stall < 1) return fail(GPCG_ERR_ARG, "max_stall must be >= 1");
  return GPCG_OK;
}

// Unknowns per workgroup and pass, chosen from the size alone so that a QP
// reduces in the same order whether it is solved alone or inside a batch.
// Small grids use many small tiles (latency: more workgroups in flight);
// large grids use larger tiles (fewer partial slots, longer streams per
// workgroup).  Tuned on MI355X; overridable with gpcg_options.tile.
int tuned_tile(int64_t n) {
  if (n <= (int64_t)1 << 17) return 256;
  if (n <= (int64_t)1 << 20) return 512;
  return 1024;
}

struct Layout {
  size_t state, partials, g, w, r, p0, p1, mask, wx32, wy32, vals32, scratch, total;
  int tile, ntiles;
};

Layout layout_for(const gpcg_operator *op, const gpcg_options *o) {
  Layout L{};
  const int64_t n = op_n(op);
  const bool mixed = o->precision == GPCG_PREC_MIXED;
  const size_t ct = mixed ? 4 : 8;
  L.tile = o->tile > 0 ? o->tile : tuned_tile(n);
  L.ntiles = (int)((n + L.tile - 1) / L.tile);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  L.state = take(sizeof(QPState));
  L.partials = take(sizeof(double) * kNP * (size_t)std::max(L.ntiles, 2048));
  L.scratch = take(sizeof(double) * 8);
  L.g = take(8 * (size_t)n);
  L.w = take(ct * (size_t)n);
  L.r = take(ct * (size_t)n);
  L.p0 = take(ct * (size_t)n);
  L.p1 = take(ct * (size_t)n);
  L.mask = take((size_t)n);
  L.wx32 = L.wy32 = L.vals32 = 0;
  if (mixed && op->kind == GPCG_OP_STENCIL5_VAR) {
    L.wx32 = take(4 * (size_t)op->ny * (op->nx + 1));
    L.wy32 = take(4 * (size_t)(op->ny + 1) * op->nx);
  }
  if (mixed && op->kind == GPCG_OP_CSR) L.vals32 = take(4 * (size_t)op->nnz);
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
  int32_t *host = nullptr;   // mapped, coherent host memory
  int32_t *dev = nullptr;    // its device address
};

}  // namespace

// ------------------------------------------------------------------ handle

struct gpcg_handle_s {
  gpcg_operator op;
  gpcg_options opt;
  hipStream_t stream;
  char *ws;
  size_t ws_bytes;
  Layout L;
  QPState tmpl;         // static part, filled at create
  QPState *dqp;         // device state
  QPState *stage;       // pinned host staging for uploads / downloads
  PinnedWords flag;     // DONE flag written by the device
  // single-QP launch tables (device): pointer array + prefix
  QPState **dqptrs;
  int32_t *dprefix;
  hipGraphExec_t graph = nullptr;
  int graph_chunk = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  double tick_hz;
};

namespace {

// Algorithmic HBM bytes of one pass (each array touched once; stencil
// neighbours assumed reused on chip).  `rows` is the unknowns a pass sweeps
// with full traffic: n for passes over all unknowns, m (the free count) for
// CG and projected-search passes, which skip the active set after reading
// its mask byte.
struct PassBytes {
  double per_var[PH_COUNT];   // bytes per unknown, every unknown
  double per_free[PH_COUNT];  // extra bytes per free unknown (masked passes)
};

PassBytes pass_bytes(const QPState &q) {
  PassBytes B{};
  const bool mixed = q.mixed != 0;
  const double c = mixed ? 4.0 : 8.0;  // CG vector element
  double coef64 = 0.0, coefc = 0.0;    // operator bytes per row
  if (q.op_kind == OPK_VAR) {
    coef64 = 16.0;
    coefc = mixed ? 8.0 : 16.0;
  } else if (q.op_kind == OPK_CSR) {
    // rowptr + (colind + value) per stored entry; ~5 entries per row
    const double nnz_row = q.n > 0 ? 5.0 : 0.0;
    coef64 = 4.0 + nnz_row * 12.0;
    coefc = 4.0 + nnz_row * (mixed ? 8.0 : 12.0);
  }
  B.per_var[PH_PROJECT] = 40;                  // x, l, u, b in; x out
  B.per_var[PH_GRAD] = 40 + coef64;            // x, l, u, b in; g out
  B.per_var[PH_GP_ALPHA] = 32 + coef64;        // x, l, u, g
  B.per_var[PH_GP_TRIAL] = 32 + coef64;        // x, l, u, g
  B.per_var[PH_GP_ACCEPT] = 40;                // x, l, u, g in; x out
  B.per_var[PH_CG_INIT] = 32 + 1 + 2 * c;      // x, l, u, g in; mask, r, w out
  B.per_var[PH_CG_A] = 1;                      // mask
  B.per_free[PH_CG_A] = 3 * c + coefc;         // r, p_old in; p out
  B.per_var[PH_CG_B] = 1;
  B.per_free[PH_CG_B] = 5 * c + coefc;         // p, w, r in; w, r out
  B.per_var[PH_PS_TRIAL] = 1;
  B.per_free[PH_PS_TRIAL] = 32 + c + coef64;   // x, l, u, g, w
  B.per_var[PH_PS_ACCEPT] = 1;
  B.per_free[PH_PS_ACCEPT] = 32 + c;           // x, l, u, w in; x out
  return B;
}

double solve_bytes(const QPState &q) {
  PassBytes B = pass_bytes(q);
  double total = 0.0;
  for (int p = 0; p < PH_DONE; ++p) total += B.per_var[p] * (double)q.pass_count[p] * (double)q.n;
  // free-row traffic: cg_free_rows sums m over CG_A, CG_B, PS_TRIAL, PS_ACCEPT
  const int64_t nA = q.pass_count[PH_CG_A], nB = q.pass_count[PH_CG_B];
  const int64_t nT = q.pass_count[PH_PS_TRIAL], nS = q.pass_count[PH_PS_ACCEPT];
  const int64_t cnt = nA + nB + nT + nS;
  if (cnt > 0) {
    const double mean_m = (double)q.cg_free_rows / (double)cnt;
    total += mean_m * (B.per_free[PH_CG_A] * nA + B.per_free[PH_CG_B] * nB +
                       B.per_free[PH_PS_TRIAL] * nT + B.per_free[PH_PS_ACCEPT] * nS);
  }
  return total;
}

void fill_stats(const QPState &q, double tick_hz, gpcg_stats *st) {
  if (!st) return;
  std::memset(st, 0, sizeof(*st));
  st->status = q.status;
  st->outer_iters = q.outer_iters;
  st->gp_iters = q.gp_iters;
  st->cg_iters = q.cg_iters;
  st->backtracks = q.backtracks;
  st->face_repeats = q.face_repeats;
  st->cg_phases = q.cg_phases;
  st->x0_projected = q.x0_projected;
  st->pg0 = q.pg0;
  st->pg = q.pgn;
  st->tau = q.tau;
  st->q = q.q;
  st->n_lower = q.n_lower;
  st->n_upper = q.n_upper;
  st->n_free = q.n - q.n_lower - q.n_upper;
  st->passes = q.passes;
  st->bytes = solve_bytes(q);
  const double ms = 1e3 / tick_hz;
  st->ms_cg = q.t_bucket[TB_CG] * ms;
  st->ms_gp = q.t_bucket[TB_GP] * ms;
  st->ms_search = q.t_bucket[TB_SEARCH] * ms;
  st->ms_other = q.t_bucket[TB_OTHER] * ms;
}

// Resets the dynamic part of a state for a new solve.
void reset_dynamic(QPState &q) {
  const size_t off = offsetof(QPState, ticket);
  std::memset(reinterpret_cast<char *>(&q) + off, 0, sizeof(QPState) - off);
  q.phase = PH_PROJECT;
  q.ctx = CTX_INIT;
  q.status = GPCG_OK;
  q.gp_decmax = -INFINITY;
  q.cg_decmax = -INFINITY;
}

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

double wall_clock_hz() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1e8;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return 1e8;
  return khz * 1e3;
}

// Builds a graph of `count` chained launches of the pass kernel.
int build_chain_graph(const StepLaunch &L, int mixed, int count, hipGraphExec_t *out) {
  hipGraph_t g = nullptr;
  HIP_OK(hipGraphCreate(&g, 0));
  hipKernelNodeParams p{};
  p.func = gpcg_step_kernel_ptr(mixed);
  p.gridDim = dim3((unsigned)L.total_tiles);
  p.blockDim = dim3(kBlock);
  p.sharedMemBytes = 0;
  StepLaunch arg = L;
  void *args[] = {&arg};
  p.kernelParams = args;
  p.extra = nullptr;
  hipGraphNode_t prev = nullptr;
  for (int i = 0; i < count; ++i) {
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(GPCG_ERR_HIP, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
    }
    prev = node;
  }
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess)
    return fail(GPCG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return GPCG_OK;
}

// Replays chunks of `chunk` passes until every flag in `flags` is set.
// Keeps one chunk queued behind the one the host waits on, so the GPU never
// idles while the host checks.  Returns launches issued via *launches.
int run_until_done(hipStream_t stream, const StepLaunch &L, int mixed, int chunk,
                   hipGraphExec_t graph, hipEvent_t *ev, volatile int32_t *flags, int nflags,
                   int64_t max_launches, int64_t *launches, int64_t *checks) {
  auto all_done = [&]() {
    for (int i = 0; i < nflags; ++i)
      if (!flags[i]) return false;
    return true;
  };
  auto launch_chunk = [&]() -> int {
    if (graph) {
      HIP_OK(hipGraphLaunch(graph, stream));
    } else {
      for (int i = 0; i < chunk; ++i)
        if (gpcg_launch_step(L, mixed, stream) != 0)
          return fail(GPCG_ERR_HIP, "pass kernel launch failed");
    }
    *launches += chunk;
    return GPCG_OK;
  };
  int rc = launch_chunk();
  if (rc) return rc;
  HIP_OK(hipEventRecord(ev[0], stream));
  for (int64_t i = 1;; ++i) {
    if (*launches >= max_launches)
      return fail(GPCG_ERR_HANG, "device did not finish within the launch budget");
    rc = launch_chunk();
    if (rc) return rc;
    HIP_OK(hipEventRecord(ev[i & 1], stream));
    hipEvent_t prev = ev[(i - 1) & 1];
    for (;;) {
      if (all_done()) break;
      hipError_t e = hipEventQuery(prev);
      if (e == hipSuccess) break;
      if (e != hipErrorNotReady)
        return fail(GPCG_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
      std::this_thread::yield();
    }
    *checks += 1;
    if (all_done()) break;
  }
  HIP_OK(hipStreamSynchronize(stream));
  return GPCG_OK;
}

int default_chunk(const gpcg_options &o) { return o.chunk > 0 ? o.chunk : 32; }

void fill_static(gpcg_handle_s *h) {
  QPState &q = h->tmpl;
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
  q.g = (double *)(ws + L.g);
  q.vw = ws + L.w;
  q.vr = ws + L.r;
  q.vp0 = ws + L.p0;
  q.vp1 = ws + L.p1;
  q.mask = (uint8_t *)(ws + L.mask);
  q.partials = (double *)(ws + L.partials);
  q.host_flag = h->flag.dev;
  q.tol_rel = h->opt.tol_rel;
  q.tol_abs = h->opt.tol_abs;
  q.eta1 = h->opt.eta1;
  q.eta2 = h->opt.eta2;
  q.eta2_reduce = h->opt.eta2_reduce;
  q.mu = h->opt.mu;
  q.max_outer = h->opt.max_outer;
  q.max_gp = h->opt.max_gp;
  q.max_backtrack = h->opt.max_backtrack;
  q.max_cg = h->opt.max_cg;
  q.max_stall = h->opt.max_stall;
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
  o->max_stall = 25;
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
  *bytes = layout_for(op, &o).total;
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
  Layout L = layout_for(op, &o);
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
  h->dqp = (QPState *)(h->ws + L.state);
  h->tick_hz = wall_clock_hz();
  auto cleanup = [&](int code) {
    gpcg_destroy(h);
    return code;
  };
  rc = alloc_flag(&h->flag, 16);
  if (rc) return cleanup(rc);
  void *st = nullptr;
  if (hipHostMalloc(&st, sizeof(QPState) + 2 * sizeof(void *) + 64, hipHostMallocDefault) !=
      hipSuccess)
    return cleanup(fail(GPCG_ERR_HIP, "hipHostMalloc of the staging state failed"));
  h->stage = (QPState *)st;
  // single-QP launch tables live in the scratch slot of the workspace
  h->dqptrs = (QPState **)(h->ws + L.scratch);
  h->dprefix = (int32_t *)(h->ws + L.scratch + 2 * sizeof(void *));
  fill_static(h);
  if (hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(GPCG_ERR_HIP, "hipEventCreate failed"));
  // the launch tables: {dqp} and {0, ntiles}
  struct {
    QPState *p[2];
    int32_t pre[4];
  } tables{};
  tables.p[0] = h->dqp;
  tables.pre[0] = 0;
  tables.pre[1] = L.ntiles;
  if (hipMemcpyAsync(h->ws + L.scratch, &tables, sizeof(tables), hipMemcpyHostToDevice,
                     h->stream) != hipSuccess)
    return cleanup(fail(GPCG_ERR_HIP, "upload of the launch tables failed"));
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
  QPState &q = *h->stage;
  q = h->tmpl;
  q.b = b;
  q.l = l;
  q.u = u;
  q.x = x;
  reset_dynamic(q);
  h->flag.host[0] = 0;
  HIP_OK(hipMemcpyAsync(h->dqp, &q, sizeof(QPState), hipMemcpyHostToDevice, h->stream));
  StepLaunch SL{h->dqptrs, h->dprefix, 1, h->L.ntiles};
  const int chunk = default_chunk(h->opt);
  if (h->opt.use_graph && (!h->graph || h->graph_chunk != chunk)) {
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    int rc = build_chain_graph(SL, h->tmpl.mixed, chunk, &h->graph);
    if (rc) return rc;
    h->graph_chunk = chunk;
  }
  int64_t launches = 0, checks = 0;
  int rc = run_until_done(h->stream, SL, h->tmpl.mixed, chunk,
                          h->opt.use_graph ? h->graph : nullptr, h->ev, h->flag.host, 1,
                          (int64_t)1 << 26, &launches, &checks);
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(h->stage, h->dqp, sizeof(QPState), hipMemcpyDeviceToHost, h->stream));
  if (g_out)
    HIP_OK(hipMemcpyAsync(g_out, h->tmpl.g, sizeof(double) * (size_t)h->tmpl.n,
                          hipMemcpyDeviceToDevice, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  const QPState &res = *h->stage;
  if (stats) {
    fill_stats(res, h->tick_hz, stats);
    stats->launches = launches;
    stats->host_checks = checks;
    stats->ms_total = (now_s() - t0) * 1e3;
  }
  if (res.status < 0) g_last_error = gpcg_status_string(res.status);
  return res.status;
}

int gpcg_spmv(gpcg_handle h, const double *v, double *y, const uint8_t *mask) {
  if (!h || !v || !y) return fail(GPCG_ERR_ARG, "handle, v and y are required");
  // the kernel reads the operator from the device state: refresh it
  QPState &q = *h->stage;
  HIP_OK(hipStreamSynchronize(h->stream));
  q = h->tmpl;
  HIP_OK(hipMemcpyAsync(h->dqp, &q, sizeof(QPState), hipMemcpyHostToDevice, h->stream));
  if (gpcg_launch_spmv(h->dqp, h->tmpl, v, y, mask, 0, h->stream))
    return fail(GPCG_ERR_HIP, "spmv launch failed");
  return GPCG_OK;
}

int gpcg_spmv_f32(gpcg_handle h, const float *v, float *y, const uint8_t *mask) {
  if (!h || !v || !y) return fail(GPCG_ERR_ARG, "handle, v and y are required");
  if (!h->tmpl.mixed) return fail(GPCG_ERR_ARG, "handle was not created with GPCG_PREC_MIXED");
  QPState &q = *h->stage;
  HIP_OK(hipStreamSynchronize(h->stream));
  q = h->tmpl;
  HIP_OK(hipMemcpyAsync(h->dqp, &q, sizeof(QPState), hipMemcpyHostToDevice, h->stream));
  if (gpcg_launch_spmv(h->dqp, h->tmpl, v, y, mask, 1, h->stream))
    return fail(GPCG_ERR_HIP, "spmv launch failed");
  return GPCG_OK;
}

int gpcg_projected_gradient(gpcg_handle h, const double *x, const double *l, const double *u,
                            const double *g, double *pg, double *norm2, int64_t *n_lower,
                            int64_t *n_upper, int64_t *n_nonbinding) {
  if (!h || !x || !l || !u || !g) return fail(GPCG_ERR_ARG, "handle, x, l, u, g required");
  double *out4 = (double *)(h->ws + h->L.scratch + 64);
  if (gpcg_launch_pgrad(h->dqp, h->tmpl, x, l, u, g, pg, out4, h->stream))
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
  return "gpcg-mi355x 0.1 (HIP, offload gfx950, wave64, FP64 + mixed FP32 reduced CG)";
}

}  // extern "C"

// ================================================================== batches

namespace {

// Launch tables for a set of QPs: pointer array + tile prefix (stepped form)
// or workgroup-slot prefix (persistent form).  Lives at the start of a
// workspace; `stage` is pinned host memory of the same layout.
struct Tables {
  QPState **qptrs;   // device
  int32_t *prefix;   // device
  size_t bytes;
};

size_t tables_bytes(int count) {
  return align_up(sizeof(void *) * (size_t)count) + align_up(sizeof(int32_t) * (count + 1));
}

// Workgroup slots per QP for the persistent form: proportional to the QP's
// share of all unknowns, at least one, at most its tile count; the total
// fits the number of co-resident workgroups.
std::vector<int32_t> persistent_slots(const std::vector<const QPState *> &qs, int capacity) {
  const int cnt = (int)qs.size();
  std::vector<int32_t> w(cnt, 1);
  if (cnt == 0 || capacity < cnt) return {};
  double total = 0.0;
  for (auto *q : qs) total += (double)q->n;
  int used = 0;
  for (int i = 0; i < cnt; ++i) {
    int want = (int)std::floor(capacity * (double)qs[i]->n / total);
    want = std::max(1, std::min(want, qs[i]->ntiles));
    w[i] = want;
    used += want;
  }
  while (used > capacity) {  // rounding overflow: trim the largest shares
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
  Tables T;
  char *stage;          // pinned copy of the tables
  PinnedWords flags;    // one DONE word per QP
  hipEvent_t ev[2] = {nullptr, nullptr};
  int mixed;
};

extern "C" {

int gpcg_batch_workspace_bytes(int count, size_t *bytes) {
  if (count < 1 || !bytes) return fail(GPCG_ERR_ARG, "count must be >= 1");
  *bytes = tables_bytes(count);
  return GPCG_OK;
}

int gpcg_batch_create(int count, const gpcg_handle *handles, void *workspace, size_t ws_bytes,
                      void *stream, gpcg_batch *out) {
  if (!out || count < 1 || !handles) return fail(GPCG_ERR_ARG, "bad batch arguments");
  *out = nullptr;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || ws_bytes < tables_bytes(count))
    return fail(GPCG_ERR_WORKSPACE, "batch workspace missing, misaligned or too small");
  for (int i = 0; i < count; ++i) {
    if (!handles[i]) return fail(GPCG_ERR_ARG, "NULL handle in batch");
    if (handles[i]->tmpl.mixed != handles[0]->tmpl.mixed)
      return fail(GPCG_ERR_ARG, "all handles of a batch must share the precision");
  }
  auto *b = new gpcg_batch_s();
  b->hs.assign(handles, handles + count);
  b->stream = (hipStream_t)stream;
  b->ws = (char *)workspace;
  b->ws_bytes = ws_bytes;
  b->T.qptrs = (QPState **)b->ws;
  b->T.prefix = (int32_t *)(b->ws + align_up(sizeof(void *) * (size_t)count));
  b->T.bytes = tables_bytes(count);
  b->mixed = handles[0]->tmpl.mixed;
  int rc = alloc_flag(&b->flags, (size_t)count);
  if (rc) {
    delete b;
    return rc;
  }
  void *st = nullptr;
  if (hipHostMalloc(&st, b->T.bytes, hipHostMallocDefault) != hipSuccess) {
    gpcg_batch_destroy(b);
    return fail(GPCG_ERR_HIP, "hipHostMalloc of batch tables failed");
  }
  b->stage = (char *)st;
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
    QPState &q = *h->stage;
    q = h->tmpl;
    q.b = p.b;
    q.l = p.l;
    q.u = p.u;
    q.x = p.x;
    q.host_flag = b->flags.dev + i;
    reset_dynamic(q);
    b->flags.host[i] = 0;
    HIP_OK(hipMemcpyAsync(h->dqp, &q, sizeof(QPState), hipMemcpyHostToDevice, b->stream));
  }
  // tables over all QPs
  std::vector<const QPState *> qs(cnt);
  for (int i = 0; i < cnt; ++i) qs[i] = &b->hs[i]->tmpl;
  auto **qp = (QPState **)b->stage;
  auto *pre = (int32_t *)(b->stage + align_up(sizeof(void *) * (size_t)cnt));
  int64_t launches = 0, checks = 0;
  int grid = 0;
  if (mode == GPCG_BATCH_PERSISTENT) {
    int cap = 0;
    int rc = persistent_capacity(b->mixed, &cap);
    if (rc) return rc;
    std::vector<int32_t> w = persistent_slots(qs, cap);
    if (w.empty()) return fail(GPCG_ERR_ARG, "more QPs than co-resident workgroups");
    pre[0] = 0;
    for (int i = 0; i < cnt; ++i) {
      qp[i] = b->hs[i]->dqp;
      pre[i + 1] = pre[i] + w[i];
    }
    grid = pre[cnt];
    HIP_OK(hipMemcpyAsync(b->ws, b->stage, b->T.bytes, hipMemcpyHostToDevice, b->stream));
    PersistLaunch P{b->T.qptrs, b->T.prefix, cnt, grid, (int64_t)1 << 22};
    if (gpcg_launch_persistent(P, grid, b->mixed, b->stream) != 0)
      return fail(GPCG_ERR_HIP, std::string("cooperative launch failed: ") +
                                    hipGetErrorString(hipGetLastError()));
    launches = 1;
    HIP_OK(hipStreamSynchronize(b->stream));
  } else {
    // stepped: replay chunks; shrink the launch to the unfinished QPs as
    // they complete (results do not depend on the launch composition)
    std::vector<int> active(cnt);
    for (int i = 0; i < cnt; ++i) active[i] = i;
    const int chunk = default_chunk(b->hs[0]->opt);
    while (!active.empty()) {
      int total = 0;
      pre[0] = 0;
      for (size_t a = 0; a < active.size(); ++a) {
        qp[a] = b->hs[active[a]]->dqp;
        pre[a + 1] = pre[a] + b->hs[active[a]]->tmpl.ntiles;
      }
      total = pre[active.size()];
      HIP_OK(hipStreamSynchronize(b->stream));
      HIP_OK(hipMemcpyAsync(b->ws, b->stage, b->T.bytes, hipMemcpyHostToDevice, b->stream));
      StepLaunch SL{b->T.qptrs, b->T.prefix, (int32_t)active.size(), total};
      hipGraphExec_t graph = nullptr;
      int rc = build_chain_graph(SL, b->mixed, chunk, &graph);
      if (rc) return rc;
      // run until at least a third of the launch's tiles belong to finished QPs
      const int64_t before = launches;
      (void)before;
      bool shrink = false;
      launches += chunk;
      HIP_OK(hipGraphLaunch(graph, b->stream));
      HIP_OK(hipEventRecord(b->ev[0], b->stream));
      for (int64_t i = 1; !shrink; ++i) {
        if (launches >= ((int64_t)1 << 26)) {
          (void)hipGraphExecDestroy(graph);
          return fail(GPCG_ERR_HANG, "batch did not finish within the launch budget");
        }
        HIP_OK(hipGraphLaunch(graph, b->stream));
        launches += chunk;
        HIP_OK(hipEventRecord(b->ev[i & 1], b->stream));
        hipEvent_t prev = b->ev[(i - 1) & 1];
        for (;;) {
          hipError_t e = hipEventQuery(prev);
          if (e == hipSuccess) break;
          if (e != hipErrorNotReady) {
            (void)hipGraphExecDestroy(graph);
            return fail(GPCG_ERR_HIP, "hipEventQuery failed");
          }
          std::this_thread::yield();
        }
        ++checks;
        int done_tiles = 0;
        for (size_t a = 0; a < active.size(); ++a)
          if (b->flags.host[active[a]]) done_tiles += b->hs[active[a]]->tmpl.ntiles;
        if (3 * done_tiles >= total) shrink = true;
      }
      HIP_OK(hipStreamSynchronize(b->stream));
      (void)hipGraphExecDestroy(graph);
      std::vector<int> still;
      for (int i : active)
        if (!b->flags.host[i]) still.push_back(i);
      active.swap(still);
    }
  }
  int first_err = GPCG_OK;
  for (int i = 0; i < cnt; ++i) {
    gpcg_handle h = b->hs[i];
    HIP_OK(hipMemcpyAsync(h->stage, h->dqp, sizeof(QPState), hipMemcpyDeviceToHost, b->stream));
    if (probs[i].g_out)
      HIP_OK(hipMemcpyAsync(probs[i].g_out, h->tmpl.g, sizeof(double) * (size_t)h->tmpl.n,
                            hipMemcpyDeviceToDevice, b->stream));
  }
  HIP_OK(hipStreamSynchronize(b->stream));
  const double ms = (now_s() - t0) * 1e3;
  for (int i = 0; i < cnt; ++i) {
    gpcg_handle h = b->hs[i];
    const QPState &res = *h->stage;
    if (res.status < 0 && first_err == GPCG_OK) first_err = res.status;
    if (stats) {
      fill_stats(res, h->tick_hz, &stats[i]);
      stats[i].launches = launches;
      stats[i].host_checks = checks;
      stats[i].ms_total = ms;
    }
  }
  if (first_err < 0) g_last_error = gpcg_status_string(first_err);
  return first_err;
}

}  // extern "C"

// ================================================================== serving

namespace {

// Arena bytes of one request: its QPState, reduction slots, resident copies
// of b, l, u, the iterate x and gradient g, the CG vectors, the free mask
// and, for edge-weighted stencils, the weights (plus FP32 copies in the
// mixed form).
struct ReqLayout {
  size_t state, partials, b, l, u, x, g, w, r, p0, p1, mask, wx, wy, wx32, wy32, total;
  int tile, ntiles;
};

ReqLayout req_layout(const gpcg_operator *op, int precision) {
  ReqLayout R{};
  const int64_t n = op_n(op);
  const size_t ct = precision == GPCG_PREC_MIXED ? 4 : 8;
  R.tile = tuned_tile(n);
  R.ntiles = (int)((n + R.tile - 1) / R.tile);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  R.state = take(sizeof(QPState));
  R.partials = take(sizeof(double) * kNP * (size_t)R.ntiles);
  R.b = take(8 * (size_t)n);
  R.l = take(8 * (size_t)n);
  R.u = take(8 * (size_t)n);
  R.x = take(8 * (size_t)n);
  R.g = take(8 * (size_t)n);
  R.w = take(ct * (size_t)n);
  R.r = take(ct * (size_t)n);
  R.p0 = take(ct * (size_t)n);
  R.p1 = take(ct * (size_t)n);
  R.mask = take((size_t)n);
  R.wx = R.wy = R.wx32 = R.wy32 = 0;
  if (op->kind == GPCG_OP_STENCIL5_VAR) {
    const size_t ex = (size_t)op->ny * (op->nx + 1), ey = (size_t)(op->ny + 1) * op->nx;
    R.wx = take(8 * ex);
    R.wy = take(8 * ey);
    if (precision == GPCG_PREC_MIXED) {
      R.wx32 = take(4 * ex);
      R.wy32 = take(4 * ey);
    }
  }
  R.total = off;
  return R;
}

struct SrvSlot {
  bool used = false;
  size_t off = 0, bytes = 0;
  gpcg_request req{};
  double t_submit = 0, t_admit = 0;
  int ntiles = 0;
};

struct SrvPending {
  gpcg_request req;
  double t_submit;
  size_t bytes;
};

}  // namespace

struct gpcg_server_s {
  gpcg_server_options opt;
  hipStream_t stream;
  char *arena;
  size_t header;        // launch tables at the start of the arena
  Tables T;
  char *stage_tables;   // pinned
  QPState *stage;       // pinned, one per slot
  PinnedWords flags;    // one DONE word per slot
  std::vector<SrvSlot> slots;
  std::deque<SrvPending> queue;
  std::vector<gpcg_completion> done;
  std::map<size_t, size_t> free_list;  // offset -> bytes, coalesced
  bool dirty = true;
  int resident = 0;
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
};

namespace {

int srv_admit(gpcg_server_s *s, int slot_id, const SrvPending &p, size_t off) {
  SrvSlot &sl = s->slots[slot_id];
  const gpcg_request &rq = p.req;
  const gpcg_operator &op = rq.op;
  const ReqLayout R = req_layout(&op, s->opt.precision);
  char *base = s->arena + off;
  const int64_t n = op_n(&op);
  hipStream_t st = s->stream;
  HIP_OK(hipMemcpyAsync(base + R.b, rq.b, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
  HIP_OK(hipMemcpyAsync(base + R.l, rq.l, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
  HIP_OK(hipMemcpyAsync(base + R.u, rq.u, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
  HIP_OK(hipMemcpyAsync(base + R.x, rq.x0, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
  const size_t ex = (size_t)op.ny * (op.nx + 1), ey = (size_t)(op.ny + 1) * op.nx;
  if (op.kind == GPCG_OP_STENCIL5_VAR) {
    HIP_OK(hipMemcpyAsync(base + R.wx, op.wx, 8 * ex, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(base + R.wy, op.wy, 8 * ey, hipMemcpyDeviceToDevice, st));
    if (R.wx32) {
      if (gpcg_launch_convert_f32((const double *)(base + R.wx), (float *)(base + R.wx32),
                                  (int64_t)ex, st) ||
          gpcg_launch_convert_f32((const double *)(base + R.wy), (float *)(base + R.wy32),
                                  (int64_t)ey, st))
        return fail(GPCG_ERR_HIP, "FP32 weight conversion failed");
    }
  }
  QPState &q = s->stage[slot_id];
  std::memset(&q, 0, sizeof(q));
  q.op_kind = op.kind == GPCG_OP_STENCIL5_CONST ? OPK_CONST : OPK_VAR;
  q.nx = op.nx;
  q.ny = op.ny;
  q.n = n;
  q.tile = R.tile;
  q.ntiles = R.ntiles;
  q.mixed = s->opt.precision == GPCG_PREC_MIXED ? 1 : 0;
  magic_for(q.nx, &q.div_magic, &q.div_shift);
  q.w = op.w;
  q.w32 = (float)op.w;
  q.wx = R.wx ? (const double *)(base + R.wx) : nullptr;
  q.wy = R.wy ? (const double *)(base + R.wy) : nullptr;
  q.wx32 = R.wx32 ? (const float *)(base + R.wx32) : nullptr;
  q.wy32 = R.wy32 ? (const float *)(base + R.wy32) : nullptr;
  q.b = (const double *)(base + R.b);
  q.l = (const double *)(base + R.l);
  q.u = (const double *)(base + R.u);
  q.x = (double *)(base + R.x);
  q.g = (double *)(base + R.g);
  q.vw = base + R.w;
  q.vr = base + R.r;
  q.vp0 = base + R.p0;
  q.vp1 = base + R.p1;
  q.mask = (uint8_t *)(base + R.mask);
  q.partials = (double *)(base + R.partials);
  q.host_flag = s->flags.dev + slot_id;
  const gpcg_options &o = s->solve_opt;
  q.tol_rel = o.tol_rel;
  q.tol_abs = o.tol_abs;
  q.eta1 = o.eta1;
  q.eta2 = o.eta2;
  q.eta2_reduce = o.eta2_reduce;
  q.mu = o.mu;
  q.max_outer = o.max_outer;
  q.max_gp = o.max_gp;
  q.max_backtrack = o.max_backtrack;
  q.max_cg = o.max_cg;
  q.max_stall = o.max_stall;
  reset_dynamic(q);
  s->flags.host[slot_id] = 0;
  HIP_OK(hipMemcpyAsync(base + R.state, &q, sizeof(QPState), hipMemcpyHostToDevice, st));
  sl.used = true;
  sl.off = off;
  sl.bytes = p.bytes;
  sl.req = rq;
  sl.t_submit = p.t_submit;
  sl.t_admit = now_s();
  sl.ntiles = R.ntiles;
  s->resident += 1;
  s->dirty = true;
  return GPCG_OK;
}

// Moves finished requests to the completion list (after the stream is idle).
int srv_retire(gpcg_server_s *s) {
  std::vector<int> fin;
  for (int i = 0; i < (int)s->slots.size(); ++i)
    if (s->slots[i].used && s->flags.host[i]) fin.push_back(i);
  if (fin.empty()) return GPCG_OK;
  for (int i : fin) {
    SrvSlot &sl = s->slots[i];
    const ReqLayout R = req_layout(&sl.req.op, s->opt.precision);
    char *base = s->arena + sl.off;
    HIP_OK(hipMemcpyAsync(&s->stage[i], base + R.state, sizeof(QPState), hipMemcpyDeviceToHost,
                          s->stream));
    if (sl.req.x_out)
      HIP_OK(hipMemcpyAsync(sl.req.x_out, base + R.x, 8 * (size_t)op_n(&sl.req.op),
                            hipMemcpyDeviceToDevice, s->stream));
  }
  HIP_OK(hipStreamSynchronize(s->stream));
  const double t = now_s();
  for (int i : fin) {
    SrvSlot &sl = s->slots[i];
    gpcg_completion c{};
    c.tag = sl.req.tag;
    fill_stats(s->stage[i], s->tick_hz, &c.stats);
    c.status = s->stage[i].status;
    c.t_submit = sl.t_submit;
    c.t_admit = sl.t_admit;
    c.t_done = t;
    c.stats.ms_total = (t - sl.t_admit) * 1e3;
    s->done.push_back(c);
    s->release(sl.off, sl.bytes);
    sl.used = false;
    s->flags.host[i] = 0;
    s->resident -= 1;
    s->dirty = true;
  }
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
  if (!opt->arena || ((uintptr_t)opt->arena % kAlign) != 0)
    return fail(GPCG_ERR_WORKSPACE, "arena missing or not 256-byte aligned");
  const size_t header = tables_bytes(opt->max_slots);
  if (opt->arena_bytes <= header) return fail(GPCG_ERR_WORKSPACE, "arena too small");
  auto *s = new gpcg_server_s();
  s->opt = *opt;
  if (s->opt.quantum <= 0) s->opt.quantum = 64;
  s->stream = (hipStream_t)stream;
  s->arena = (char *)opt->arena;
  s->header = header;
  s->T.qptrs = (QPState **)s->arena;
  s->T.prefix = (int32_t *)(s->arena + align_up(sizeof(void *) * (size_t)opt->max_slots));
  s->T.bytes = header;
  s->slots.resize(opt->max_slots);
  s->free_list[header] = opt->arena_bytes - header;
  s->tick_hz = wall_clock_hz();
  gpcg_options_default(&s->solve_opt);
  s->solve_opt.tol_rel = opt->tol_rel;
  s->solve_opt.precision = opt->precision;
  int rc = alloc_flag(&s->flags, (size_t)opt->max_slots);
  void *st = nullptr, *tb = nullptr;
  if (!rc && (hipHostMalloc(&st, sizeof(QPState) * opt->max_slots, hipHostMallocDefault) !=
                  hipSuccess ||
              hipHostMalloc(&tb, header, hipHostMallocDefault) != hipSuccess))
    rc = fail(GPCG_ERR_HIP, "hipHostMalloc for the server failed");
  s->stage = (QPState *)st;
  s->stage_tables = (char *)tb;
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
  s->queue.push_back(SrvPending{*req, now_s(), bytes});
  return GPCG_OK;
}

int gpcg_server_step(gpcg_server s, int *active) {
  if (!s) return fail(GPCG_ERR_ARG, "server is NULL");
  int rc = GPCG_OK;
  // admission: FIFO, by free slot and arena space
  while (!s->queue.empty() && s->resident < s->opt.max_slots) {
    size_t off = 0;
    if (!s->alloc(s->queue.front().bytes, &off)) break;
    int slot = -1;
    for (int i = 0; i < (int)s->slots.size(); ++i)
      if (!s->slots[i].used) {
        slot = i;
        break;
      }
    rc = srv_admit(s, slot, s->queue.front(), off);
    if (rc) return rc;
    s->queue.pop_front();
  }
  if (s->resident > 0) {
    auto **qp = (QPState **)s->stage_tables;
    auto *pre = (int32_t *)(s->stage_tables + align_up(sizeof(void *) * s->slots.size()));
    int cnt = 0;
    pre[0] = 0;
    for (int i = 0; i < (int)s->slots.size(); ++i) {
      if (!s->slots[i].used) continue;
      const ReqLayout R = req_layout(&s->slots[i].req.op, s->opt.precision);
      qp[cnt] = (QPState *)(s->arena + s->slots[i].off + R.state);
      pre[cnt + 1] = pre[cnt] + s->slots[i].ntiles;
      ++cnt;
    }
    HIP_OK(hipMemcpyAsync(s->arena, s->stage_tables, s->header, hipMemcpyHostToDevice,
                          s->stream));
    StepLaunch SL{s->T.qptrs, s->T.prefix, cnt, pre[cnt]};
    for (int k = 0; k < s->opt.quantum; ++k)
      if (gpcg_launch_step(SL, s->opt.precision == GPCG_PREC_MIXED, s->stream) != 0)
        return fail(GPCG_ERR_HIP, "pass kernel launch failed");
    HIP_OK(hipStreamSynchronize(s->stream));
    s->dirty = false;
    rc = srv_retire(s);
    if (rc) return rc;
  }
  if (active) *active = (int)s->queue.size() + s->resident;
  return GPCG_OK;
}

int gpcg_server_poll(gpcg_server s, gpcg_completion *out, int max, int *got) {
  if (!s || !got) return fail(GPCG_ERR_ARG, "server and got are required");
  int k = 0;
  while (k < max && !s->done.empty() && out) {
    out[k++] = s->done.front();
    s->done.erase(s->done.begin());
  }
  *got = k;
  return GPCG_OK;
}

int gpcg_server_destroy(gpcg_server s) {
  if (!s) return GPCG_OK;
  (void)hipStreamSynchronize(s->stream);
  if (s->stage) (void)hipHostFree(s->stage);
  if (s->stage_tables) (void)hipHostFree(s->stage_tables);
  if (s->flags.host) (void)hipHostFree(s->flags.host);
  delete s;
  return GPCG_OK;
}

}  // extern "C"
