/*
 * gpcg.h -- C ABI of the MI355X (gfx950) GPCG library.
 *
 * GPCG (Benson, McInnes & More, arXiv cs/0101018, Section 3; method of
 * More & Toraldo) solves the bound-constrained convex quadratic program
 *
 *     minimise  q(x) = 1/2 x'Ax - b'x   subject to  l <= x <= u        (1)
 *
 * with A sparse symmetric positive definite (Section 2, eqs. (def_bqp),
 * (def_bounds), (def-quadratic); the paper writes +b'x, here g = Ax - b).
 * Components of l may be -inf and of u +inf.
 *
 * The interface follows the five-call solver context of Section 4 (figure
 * "TAO interface for GPCG": create, set the quadratic, set the bounds, solve,
 * destroy) with a data-structure-neutral operator (Section 4, last
 * paragraph; Section 6 on structured storage): A is a five-point stencil on a
 * grid (constant or edge-varying weights) or a general CSR matrix.
 *
 * Conventions for every entry point
 *  - All array arguments are DEVICE pointers (e.g. from torch tensors) unless
 *    stated otherwise; scalars and structs are host values.  The caller owns
 *    every array; the library never frees caller memory.
 *  - `stream` arguments are hipStream_t values passed as void* (NULL is the
 *    default stream).  Work is stream-ordered on that stream.
 *  - Every function returns an int status: GPCG_OK (0), a warning (> 0) or an
 *    error (< 0).  No C++ exception crosses this boundary.
 *    gpcg_last_error() returns a thread-local message for the last error.
 *  - The library does not call hipMalloc during a solve.  The caller
 *    allocates the workspace whose size gpcg_workspace_bytes() reports; the
 *    only library-side allocations are a few pinned host words per handle,
 *    made in gpcg_create / gpcg_batch_create.
 *  - A handle is used by one host thread at a time.  Solves on different
 *    handles may run concurrently on different streams.
 *
 * Grid convention for the stencil operators: nx x ny interior unknowns,
 * index k = j*nx + i (i fastest), homogeneous Dirichlet data outside:
 *   (A x)_k = sum over the four edges e of k of  w_e (x_k - x_nb(e)),
 * x_nb = 0 outside the grid.  wx has ny*(nx+1) entries, wx[j*(nx+1)+e] is the
 * edge between columns e-1 and e of row j; wy has (ny+1)*nx entries,
 * wy[e*nx+i] is the edge between rows e-1 and e of column i.  The constant
 * operator uses one weight w on every edge (w = 1/h^2 for the Laplacian).
 */
#ifndef GPCG_H
#define GPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define GPCG_OK 0
#define GPCG_MAXIT 1          /* max_outer GPCG iterations reached           */
#define GPCG_STAGNATED 2      /* no sufficient decrease above rounding level */
#define GPCG_ERR_ARG (-1)     /* bad argument / descriptor / option          */
#define GPCG_ERR_BOUNDS (-2)  /* some l_i > u_i                              */
#define GPCG_ERR_NAN (-3)     /* NaN in b, l, u or x0                        */
#define GPCG_ERR_NOT_SPD (-4) /* d'Ad <= 0 or p'Ap <= 0 met: A not SPD       */
#define GPCG_ERR_WORKSPACE (-5) /* workspace missing, too small or misaligned */
#define GPCG_ERR_HIP (-6)     /* a HIP runtime call failed                   */
#define GPCG_ERR_NOSPACE (-7) /* server: request does not fit the arena     */
#define GPCG_ERR_HANG (-8)    /* persistent kernel: a bounded wait expired   */

/* --------------------------------------------------------------- operators */
#define GPCG_OP_STENCIL5_CONST 1
#define GPCG_OP_STENCIL5_VAR 2
#define GPCG_OP_CSR 3

typedef struct {
  int32_t kind;          /* GPCG_OP_*                                        */
  int32_t nx, ny;        /* stencil grid (n = nx*ny); ignored for CSR        */
  double w;              /* STENCIL5_CONST: the edge weight                  */
  const double *wx;      /* STENCIL5_VAR: device, ny*(nx+1) edge weights     */
  const double *wy;      /* STENCIL5_VAR: device, (ny+1)*nx edge weights     */
  int64_t n;             /* CSR: order of A                                  */
  int64_t nnz;           /* CSR: number of stored entries                    */
  const int32_t *rowptr; /* CSR: device, n+1 row offsets (rowptr[0] = 0)     */
  const int32_t *colind; /* CSR: device, nnz column indices                  */
  const double *vals;    /* CSR: device, nnz values; A must be symmetric     */
} gpcg_operator;

/* ----------------------------------------------------------------- options */
#define GPCG_PREC_FP64 0  /* everything in FP64                              */
#define GPCG_PREC_MIXED 1 /* reduced CG (SpMV, axpy, dots) in FP32 with FP32
                             accumulation; g = Ax - b, projections, the
                             projected-gradient test, the active / binding
                             decisions and the q differences stay FP64       */

#define GPCG_FREESET_MASK 0 /* CG vectors full length, zero on the active set */
#define GPCG_FREESET_LIST 1 /* CG loops over a compacted list of free indices */
#define GPCG_FREESET_MATRIX 2 /* CSR operators: the list form plus the reduced
                               matrix A_F (rows and columns of the free set;
                               the paper's technique 1) written out once per
                               CG phase; CG iterations read only its nonzeros */

typedef struct {
  double tol_rel;      /* stop when ||P grad q(x)||_2 <= tau,                 */
  double tol_abs;      /*   tau = max(tol_abs, tol_rel*||P grad q(x0)||_2)    */
  double eta1;         /* eq. (pgstop2); Section 5 uses 0.1                   */
  double eta2;         /* eq. (cgstop1); Section 5 uses 0.05                  */
  double eta2_reduce;  /* factor applied to eta2 when eq. (cgstop3) holds     */
  double mu;           /* sufficient decrease, eqs. (gplsstop), (cglsstop2)   */
  int32_t max_outer;   /* cap on GPCG iterations (projected searches)         */
  int32_t max_gp;      /* cap on gradient-projection iterates per phase       */
  int32_t max_backtrack; /* cap on halvings in one projected search           */
  int32_t max_cg;      /* cap on CG iterations per phase; <= 0: m_k           */
  int32_t precision;   /* GPCG_PREC_*                                         */
  int32_t free_set;    /* GPCG_FREESET_*                                      */
  int32_t tile;        /* unknowns per tile, the unit of one reduction slot
                          per pass (multiple of 256); 0 = library choice, a
                          function of n and the precision only: 256 up to
                          262,144 unknowns, 512 beyond, 1024 from 8,388,608
                          (FP64) or 1,048,576 (mixed), 2048 from 16,777,216
                          (8192 tiles of 2048) on; the list and matrix free
                          sets keep 256.  The tile fixes the summation order:
                          the answer depends on it, and on nothing else of
                          the launch set-up                                   */
  int32_t chunk;       /* device passes per host check; 0 = library choice    */
  int32_t use_graph;   /* 1 = replay chunks as HIP graphs (default), 0 = launch */
  int32_t max_stall;   /* stop as GPCG_STAGNATED when ||P grad q|| after a
                          projected search has not improved on its best value
                          for this many consecutive GPCG iterations (the
                          rounding floor of FP64 has been reached)            */
  int32_t form;        /* launch form: GPCG_FORM_AUTO (fused when the grid
                          has at most 1024 tiles of 256 unknowns, else split),
                          GPCG_FORM_FUSED or GPCG_FORM_SPLIT; the answer is
                          bitwise the same in every form                     */
  int32_t tiles_per_wg; /* split form: consecutive tiles (of `tile` unknowns)
                          per data workgroup, 1..64; 0 = 1.  The answer does
                          not depend on it                                    */
  int32_t prefetch;     /* CG operands of stencil QPs loaded before the state
                          is read: GPCG_PREFETCH_AUTO (on), _ON or _OFF.  The
                          answer does not depend on it                        */
  int32_t precond;      /* preconditioner of the reduced CG: GPCG_PRECOND_NONE
                          or GPCG_PRECOND_JACOBI (the diagonal of the reduced
                          Hessian A_k, i.e. of A on the free set; Section
                          "Preconditioners" of the paper).  x* is the same;
                          the CG iterates and counts are not.  The constant
                          stencil has a constant diagonal, which leaves the
                          iterates unchanged: there it is not applied      */
  int32_t cg_stop;      /* GPCG_CGSTOP_DECREASE (default) or _RESIDUAL       */
  int32_t cg_kernel;    /* split form: GPCG_CGK_ON runs the CG iterations of
                          stencil QPs (mask free set) in a data kernel of
                          their own, which needs far fewer registers than the
                          kernel of every pass and so keeps more workgroups
                          in flight, at the price of a third launch per pass;
                          GPCG_CGK_OFF one data kernel; GPCG_CGK_AUTO the
                          library's choice.  The answer does not depend on it */
  int32_t lookahead;    /* fused form, stencil operators, 256-unknown tiles:
                          the pass that evaluates a trial point of the
                          gradient-projection search also evaluates eq.
                          (bqpls) at it, the step length of the next iterate,
                          which then needs no pass of its own:
                          GPCG_LOOKAHEAD_AUTO (on), _ON (the same) or _OFF.
                          x and every count but the passes are bitwise the
                          same either way                                    */
} gpcg_options;

#define GPCG_PRECOND_NONE 0
#define GPCG_PRECOND_JACOBI 1
#define GPCG_CGSTOP_DECREASE 0 /* eq. (cgstop1): relative decrease of q_k         */
#define GPCG_CGSTOP_RESIDUAL 1 /* ||r_k + A_k w_j|| <= eta_2 ||r_k||, the standard
                                  test the paper contrasts with eq. (cgstop1)
                                  (M^-1 norm when preconditioned)               */

#define GPCG_CGK_AUTO 0
#define GPCG_CGK_ON 1
#define GPCG_CGK_OFF 2

#define GPCG_LOOKAHEAD_AUTO 0
#define GPCG_LOOKAHEAD_ON 1
#define GPCG_LOOKAHEAD_OFF 2

#define GPCG_PREFETCH_AUTO 0
#define GPCG_PREFETCH_ON 1
#define GPCG_PREFETCH_OFF 2

#define GPCG_FORM_AUTO 0
#define GPCG_FORM_FUSED 1 /* one launch per pass; every workgroup folds the
                             previous pass's sums into the state itself       */
#define GPCG_FORM_SPLIT 2 /* two launches per pass: a transition kernel (one
                             workgroup per QP), then a data kernel            */

/* Fills the defaults: tol_rel 1e-8, tol_abs 0, eta1 0.1, eta2 0.05,
 * eta2_reduce 0.1, mu 0.01, max_outer 100000, max_gp 50, max_backtrack 60,
 * max_cg 0, FP64, mask free set, tile 0, chunk 0, use_graph 1, max_stall 100,
 * form GPCG_FORM_AUTO, tiles_per_wg 0, prefetch GPCG_PREFETCH_AUTO,
 * precond GPCG_PRECOND_NONE, cg_stop GPCG_CGSTOP_DECREASE,
 * cg_kernel GPCG_CGK_AUTO, lookahead GPCG_LOOKAHEAD_AUTO. */
void gpcg_options_default(gpcg_options *opt);

/* ------------------------------------------------------------------- stats */
typedef struct {
  int32_t status;        /* final status (as returned by gpcg_solve)          */
  int32_t outer_iters;   /* GPCG iterations (projected searches)              */
  int32_t gp_iters;      /* accepted gradient-projection iterates ("n_GP")    */
  int32_t cg_iters;      /* CG iterations, all phases                         */
  int32_t backtracks;    /* rejected trial steps, both searches               */
  int32_t face_repeats;  /* times eq. (cgstop3) held                          */
  int32_t cg_phases;     /* reduced CG solves                                 */
  int32_t x0_projected;  /* 1 if x0 was outside [l, u] and was projected      */
  double pg0, pg, tau;   /* ||P grad q|| at x0 and at the answer; tau         */
  double q;              /* q(x) at the answer                                */
  int64_t n_free, n_lower, n_upper; /* face of the answer (fixed vars: lower) */
  int64_t passes;        /* device passes executed                            */
  int64_t lookaheads;    /* gradient-projection step lengths evaluated by the
                            trial pass before them (no pass of their own):
                            passes + lookaheads is the same in every form    */
  int64_t launches;      /* kernel launches issued (including no-op tails)    */
  int64_t host_checks;   /* host waits on device progress                     */
  double bytes;          /* algorithmic HBM bytes of all passes               */
  double ms_total;       /* wall time of the solve on the host                */
  double ms_cg, ms_gp, ms_search, ms_other; /* device time per phase          */
} gpcg_stats;

/* ----------------------------------------------------------- single solves */
typedef struct gpcg_handle_s *gpcg_handle;

/* Bytes of device workspace a handle for this operator and these options
 * needs (256-byte aligned base required). */
int gpcg_workspace_bytes(const gpcg_operator *op, const gpcg_options *opt, size_t *bytes);

/* Creates a solver context.  `workspace` is a device buffer of at least
 * gpcg_workspace_bytes() bytes that the handle uses until gpcg_destroy; the
 * operator arrays must stay valid as long as the handle.  For the mixed
 * precision an FP32 copy of the operator is made into the workspace here.
 * opt may be NULL (defaults). */
int gpcg_create(const gpcg_operator *op, const gpcg_options *opt, void *workspace,
                size_t ws_bytes, void *stream, gpcg_handle *out);

/* Solves (1) (Algorithm GPCG, Section 3).  b, l, u: device FP64 arrays of
 * length n.  x: device FP64 array of length n, the start x0 on entry (a start
 * outside [l, u] is projected and stats->x0_projected is set), the answer on
 * return.  g_out: NULL or a device FP64 array receiving g = Ax - b at the
 * answer.  stats: NULL or a host struct.  Returns after the solve has
 * completed on the handle's stream. */
int gpcg_solve(gpcg_handle h, const double *b, const double *l, const double *u, double *x,
               double *g_out, gpcg_stats *stats);

/* Releases the host state of the handle (not the workspace). */
int gpcg_destroy(gpcg_handle h);

/* -------------------------------------------------------- building blocks */
/* y = A v on the handle's operator (the "Mat-Vec Multiply" of Section 6),
 * FP64.  mask: NULL or a device byte array; where mask[k] == 0 the result is
 * 0 (the reduced product Z Z' A Z Z' v used by the CG phase).  v and y are
 * device arrays of length n that must not overlap.  Stream-ordered on the
 * handle's stream; does not wait.  The library picks the kernel by layout and
 * size (stencils: 16-byte loads when the grid width and the arrays allow it;
 * v, y and mask above 256 MB: rows kept in registers); every choice gives
 * bitwise the same product. */
int gpcg_spmv(gpcg_handle h, const double *v, double *y, const uint8_t *mask);

/* Same in FP32 for a handle created with GPCG_PREC_MIXED (the FP32 copy of
 * the operator made by gpcg_create). */
int gpcg_spmv_f32(gpcg_handle h, const float *v, float *y, const uint8_t *mask);

/* Projected gradient of Section 2 (eq. (proj-gradient)) and the face of x:
 * writes pg (device, length n, may be NULL), and returns on the host
 * ||pg||_2^2 and the counts of lower-active (x = l), upper-active (x = u != l)
 * and active-but-not-binding variables (zero exactly when B(x) = A(x)).
 * Waits for completion. */
int gpcg_projected_gradient(gpcg_handle h, const double *x, const double *l, const double *u,
                            const double *g, double *pg, double *norm2, int64_t *n_lower,
                            int64_t *n_upper, int64_t *n_nonbinding);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the result
 * of gpcg_projected_gradient without a handle or workspace.  x, l, u, g: device
 * FP64 arrays of length n; pg: NULL or a device FP64 array of length n;
 * norm2 and the three counts: host outputs as in gpcg_projected_gradient (each
 * may be NULL).  stream: hipStream_t as void* (NULL: default stream); the call
 * waits for completion on it.  Its partial sums live in a fixed scratch array
 * of the library, one per GPU (64 KiB + 32 B: four sums for each of at most
 * 2048 workgroups, then the totals), held until the process ends; the call
 * makes no device or host allocation.  n must be in [1, GPCG_NOALLOC_MAX_N]
 * (GPCG_ERR_ARG otherwise).  The results are bitwise those of
 * gpcg_projected_gradient.  Calls that overlap in time on one GPU (other
 * threads, other streams) share that scratch array and race: serialise them. */
#define GPCG_NOALLOC_MAX_N ((int64_t)1 << 34)
int gpcg_projected_gradient_noalloc(int64_t n, const double *x, const double *l,
                                    const double *u, const double *g, double *pg,
                                    double *norm2, int64_t *n_lower, int64_t *n_upper,
                                    int64_t *n_nonbinding, void *stream);

/* --------------------------------------------------------------- autotuner
 * Picks the launch configuration of a handle by timing it: the launch form
 * (fused, split), the consecutive tiles per data workgroup of the split form
 * (1, 2, 4), the early loading of CG operands (stencil operators) and the
 * number of passes per graph replay (16, 32, 64), one dimension at a time,
 * each candidate timed on a full solve of the given problem (after one
 * untimed solve that builds its graph).  Every configuration gives bitwise
 * the same answer; a candidate whose answer differs is never kept and makes
 * the call return GPCG_ERR_HIP.  The winner is kept by the handle and in a
 * process-wide table keyed by operator shape, precision and free-set form:
 * handles created later with GPCG_FORM_AUTO, tiles_per_wg 0, chunk 0 and
 * GPCG_PREFETCH_AUTO start from it.  x0 is read only; x_work (device, n doubles) receives the answer.
 * report: NULL or filled with every candidate timed and the choice. */
#define GPCG_TUNE_MAX 32

typedef struct {
  int32_t form;         /* GPCG_FORM_FUSED or GPCG_FORM_SPLIT                 */
  int32_t tiles_per_wg; /* split form: tiles per data workgroup              */
  int32_t prefetch;     /* 1: CG operands loaded before the state is read    */
  int32_t chunk;        /* passes per graph replay                           */
  int32_t shrink;       /* stepped batch: the launch is re-formed over the
                           unfinished QPs once 1/shrink of its tiles are done;
                           0: the queue form (one launch table for the whole
                           solve; every pass, a device-side queue holds the
                           work items of the QPs that are not done) */
  int32_t cg_kernel;    /* split form, 1: CG iterations in a data kernel of
                           their own (see gpcg_options.cg_kernel)            */
  double ms;            /* wall time of one solve                            */
} gpcg_tune_entry;

typedef struct {
  int32_t count;        /* candidates timed (entries of cand)                */
  int32_t mismatches;   /* candidates whose answer differed (0 expected)     */
  gpcg_tune_entry chosen;
  gpcg_tune_entry cand[GPCG_TUNE_MAX];
} gpcg_tune_report;

int gpcg_autotune(gpcg_handle h, const double *b, const double *l, const double *u,
                  const double *x0, double *x_work, gpcg_tune_report *report);

/* -------------------------------------------------------------- batches */
/* A batch advances many QPs (each with its own handle and workspace; all of
 * one precision) through one sequence of launches on one stream.  Results
 * are bitwise identical to solving each QP alone with the same handle. */
typedef struct {
  const double *b, *l, *u; /* device, length n of the QP's handle */
  double *x;               /* device, in: x0, out: answer         */
  double *g_out;           /* device or NULL                      */
} gpcg_problem;

typedef struct gpcg_batch_s *gpcg_batch;

#define GPCG_BATCH_STEPPED 0    /* one pass per launch, chunks replayed as graphs */
#define GPCG_BATCH_PERSISTENT 1 /* one cooperative launch; each QP advances on its
                                   own workgroups with a per-QP barrier            */

/* Device workspace for a batch of the `count` handles (tables of the launch:
 * QP pointers and one work item per tile of every QP). */
int gpcg_batch_workspace_bytes(int count, const gpcg_handle *handles, size_t *bytes);

/* Groups `count` handles (created with the same precision) into a batch.
 * The handles must outlive the batch. */
int gpcg_batch_create(int count, const gpcg_handle *handles, void *workspace,
                      size_t ws_bytes, void *stream, gpcg_batch *out);

/* Solves problem i with handle i for every i.  stats: NULL or `count`
 * structs.  Returns the first error status met, else GPCG_OK. */
int gpcg_batch_solve(gpcg_batch bt, const gpcg_problem *probs, int mode, gpcg_stats *stats);

/* Autotuner of the stepped batch form (see gpcg_autotune): tiles per data
 * workgroup (1, 2, 4), early CG operand loads, passes per graph replay and
 * the schedule (the launch is re-formed over the unfinished QPs once 1/3,
 * 1/6 or 1/12 of its tiles are done), each candidate timed on a full stepped
 * solve of the batch.  x0s[i] (device,
 * read only) is copied into probs[i].x before every candidate; probs[i].x
 * receives the answer.  The choice is kept by the batch. */
int gpcg_batch_autotune(gpcg_batch bt, const gpcg_problem *probs, const double *const *x0s,
                        gpcg_tune_report *report);

int gpcg_batch_destroy(gpcg_batch bt);

/* ------------------------------------------------------------ serving */
/* Continuous batching: requests are admitted while others run, as slots and
 * arena memory free up; every request's state stays resident in the arena
 * until it completes.  The caller drives the loop with gpcg_server_step.
 * Requests are laid out with 512-unknown tiles (GPCG_SERVER_TILE) whatever
 * their size, so a served answer is bitwise that of a solo solve with
 * options.tile = GPCG_SERVER_TILE. */
#define GPCG_SERVER_TILE 512
typedef struct gpcg_server_s *gpcg_server;

typedef struct {
  void *arena;          /* device buffer for all request state            */
  size_t arena_bytes;
  int32_t max_slots;    /* most requests resident at once                  */
  int32_t precision;    /* GPCG_PREC_*                                     */
  double tol_rel;       /* per-request projected-gradient tolerance        */
  int32_t quantum;      /* device passes per step (0 = library choice)     */
} gpcg_server_options;

typedef struct {
  gpcg_operator op;     /* stencil operator; weight arrays are device      */
  const double *b, *l, *u, *x0; /* device, length n; copied at admission */
  double *x_out;        /* device, length n: receives the answer            */
  uint64_t tag;         /* caller's id, echoed in the completion            */
} gpcg_request;

typedef struct {
  uint64_t tag;
  int32_t status;
  gpcg_stats stats;
  double t_submit, t_admit, t_done; /* host clock, seconds; t_done: when the
                                       answer was seen copied to x_out     */
} gpcg_completion;

/* Arena bytes one request of this operator needs at this precision. */
int gpcg_server_footprint(const gpcg_operator *op, int precision, size_t *bytes);
int gpcg_server_create(const gpcg_server_options *opt, void *stream, gpcg_server *out);
/* Queues a request (arrays must stay valid until it is admitted; x_out until
 * it completes).  GPCG_ERR_NOSPACE if it can never fit the arena. */
int gpcg_server_submit(gpcg_server s, const gpcg_request *req);
/* One turn of the serving loop, without waiting for the stream except to
 * keep at most two quanta in flight: requests whose device done word is set
 * have the copies of their answers (to x_out) and final states queued;
 * requests whose copies have passed complete (their slot and arena space are
 * free again); queued requests are admitted while a slot and arena space are
 * free; one quantum of device passes over every running request is queued.
 * *active receives the number of requests queued, running or completing. */
int gpcg_server_step(gpcg_server s, int *active);
/* Moves up to max finished completions into out; *got receives the count. */
int gpcg_server_poll(gpcg_server s, gpcg_completion *out, int max, int *got);
int gpcg_server_destroy(gpcg_server s);

/* ------------------------------------------------------------------ misc */
const char *gpcg_status_string(int status);
const char *gpcg_last_error(void);
/* Library version and the offload target it was built for. */
const char *gpcg_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* GPCG_H */
