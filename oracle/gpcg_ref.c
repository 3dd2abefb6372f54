/*
 * gpcg_ref.c -- plain FP64 CPU reference ("oracle") for GPCG.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or constant table with the
 * HIP implementation.
 *
 * What it computes (Benson, McInnes & More, "GPCG: a case study in the
 * performance and scalability of optimization algorithms", arXiv cs/0101018):
 *
 *   minimise q(x) = 1/2 x'Ax - b'x  subject to  l <= x <= u,  A sparse SPD
 *
 * (the paper's Section 2 writes +b'x; this file uses g = Ax - b throughout).
 * The method is Algorithm GPCG of Section 3: gradient-projection iterates
 * with a projected backtracking search from the exact 1-D minimiser along the
 * projected gradient, stopped by the active-set test (pgstop1) or the
 * relative-decrease test (pgstop2); conjugate gradients on the reduced system
 * of the free variables, stopped by the relative-decrease test (cgstop1); a
 * projected search along the CG direction; and, when the binding set equals
 * the active set (cgstop3), a further CG pass on the same face with a smaller
 * eta2.  Like the paper's own implementation (Section 4, "technique 1"), the
 * reduced matrix A_k = Z_k' A Z_k is extracted explicitly for each CG phase.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - the stopping norm is the Euclidean norm of the projected gradient and
 *    tau = max(tol_abs, tol_rel * ||P grad q(x0)||);
 *  - mu, the sufficient-decrease constant, is an option (default 0.01);
 *  - alpha_0 of the gradient-projection search is recomputed at every
 *    iterate y_j along -P grad q(y_j);
 *  - the ratio tests (pgstop2, cgstop1) take the max over an empty set as
 *    -infinity, so they can only fire from the second iterate on;
 *  - a failed backtracking (more than max_backtrack halvings) ends the
 *    gradient-projection phase; max_gp caps its iterates;
 *  - cgstop3 multiplies eta2 by eta2_reduce and restarts CG from w = 0 on the
 *    face of the new iterate, skipping the gradient-projection phase; eta2 is
 *    reset to its initial value whenever a gradient-projection phase runs;
 *  - a fixed variable (l_i = u_i) is always active and binding and its
 *    projected-gradient component is 0;
 *  - the termination test is applied after each gradient-projection phase and
 *    after each projected search;
 *  - below the rounding floor of FP64 the tests above can no longer fire, so
 *    the solve stops as stagnated when ||P grad q|| after a projected search
 *    has not improved on its best value for max_stall consecutive searches;
 *  - decreases of q are evaluated as g's + 1/2 s'As (equal to q(x+s)-q(x)) and
 *    the CG decrease as 1/2 alpha_j rho'z, z = M^{-1} rho (equal to
 *    q_k(w_{j-1})-q_k(w_j));
 *  - the reduced CG may be preconditioned by the diagonal of A_k (the point
 *    Jacobi preconditioner of the paper's Section "Preconditioners"); the
 *    default is no preconditioner;
 *  - the CG may instead stop by the residual test that the paper contrasts
 *    with eq. (cgstop1), ||r_k + A_k w_j|| <= eta_2 ||r_k||, measured in the
 *    M^{-1} norm when preconditioned; the default is eq. (cgstop1).
 *
 * Build: gcc -O3 -ffp-contract=off -fPIC -shared (no FMA contraction, IEEE
 * round-to-nearest, sequential sums in index order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORA_MUTANT
#define ORA_MUTANT 0 /* >0 plants a deliberate mistake (tests of the pins) */
#endif

enum {
  ORA_OK = 0,
  ORA_MAXIT = 1,
  ORA_STAGNATED = 2,
  ORA_ERR_ARG = -1,
  ORA_ERR_BOUNDS = -2,
  ORA_ERR_NAN = -3,
  ORA_ERR_NOT_SPD = -4,
};

typedef struct {
  int64_t n;
  const int32_t *rowptr; /* n+1 */
  const int32_t *colind; /* nnz */
  const double *vals;    /* nnz */
} ora_csr;

typedef struct {
  double tol_rel, tol_abs, eta1, eta2, eta2_reduce, mu;
  int32_t max_outer, max_gp, max_backtrack, max_cg; /* max_cg <= 0: m_k */
  int32_t max_stall; /* outer iterations without a new best ||P grad q|| */
  int32_t precond;   /* reduced CG: 0 none, 1 diagonal (Jacobi) of A_k */
  int32_t cg_stop;   /* reduced CG: 0 relative decrease (cgstop1), 1 residual */
} ora_options;

typedef struct {
  int32_t status, outer_iters, gp_iters, cg_iters;
  int32_t backtracks, face_repeats, cg_phases, x0_projected;
  double pg0, pg, tau, q;
  int64_t n_free, n_lower, n_upper;
  double *trace_q;    /* optional: q after every projected search */
  int64_t *trace_act; /* optional: |A(x)| before each CG phase and after
                         the projected search that follows it (2 per entry) */
  int32_t trace_cap, trace_len;
  /* optional trace of the CG phases, one entry per phase: the eta its
   * stopping test used, its CG iterations, 1 when it repeats CG on the face
   * of the previous phase (eq. (cgstop3)) and 0 when a gradient-projection
   * phase ran before it, and its CG decreases (the first trace_dec_per of
   * each phase, at trace_cg_dec[phase * trace_dec_per]) */
  double *trace_cg_eta;
  int32_t *trace_cg_iters, *trace_cg_repeat;
  double *trace_cg_dec;
  int32_t trace_cg_cap, trace_cg_len, trace_dec_per;
} ora_stats;

void ora_default_options(ora_options *o) {
  o->tol_rel = 1e-8;
  o->tol_abs = 0.0;
  o->eta1 = 0.1;   /* Section 5: eta_1 = 0.1 */
  o->eta2 = 0.05;  /* Section 5: eta_2 = 0.05 */
  o->eta2_reduce = 0.1;
  o->mu = 0.01;
  o->max_outer = 100000;
  o->max_gp = 50;
  o->max_backtrack = 60;
  o->max_cg = 0;
  o->max_stall = 100;
  o->precond = 0;
  o->cg_stop = 0;
}

/* ----------------------------------------------------------- building blocks */

/* y = A x (CSR, row by row, entries in stored order). */
void ora_matvec(const ora_csr *A, const double *x, double *y) {
  for (int64_t i = 0; i < A->n; ++i) {
    double s = 0.0;
    for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
      s += A->vals[k] * x[A->colind[k]];
    y[i] = s;
  }
}

double ora_dot(int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Gradient of q: g = A x - b. */
void ora_gradient(const ora_csr *A, const double *x, const double *b, double *g) {
  ora_matvec(A, x, g);
  for (int64_t i = 0; i < A->n; ++i) {
#if ORA_MUTANT == 7
    g[i] = b[i] - g[i];
#else
    g[i] = g[i] - b[i];
#endif
  }
}

/* q(x) = 1/2 x'Ax - b'x (Section 2, with the sign of b as above). */
double ora_objective(const ora_csr *A, const double *b, const double *x) {
  double *Ax = (double *)malloc(sizeof(double) * (size_t)(A->n > 0 ? A->n : 1));
  ora_matvec(A, x, Ax);
#if ORA_MUTANT == 17
  double q = ora_dot(A->n, x, Ax) - ora_dot(A->n, b, x);
#else
  double q = 0.5 * ora_dot(A->n, x, Ax) - ora_dot(A->n, b, x);
#endif
  free(Ax);
  return q;
}

/* Projection onto the box: the median of {l_i, u_i, v_i} (Section 3). */
static double mid3(double l, double u, double v) {
  if (v < l) return l;
#if ORA_MUTANT == 8
  if (v > u) return l;
#else
  if (v > u) return u;
#endif
  return v;
}

void ora_project(int64_t n, const double *l, const double *u, const double *v, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = mid3(l[i], u[i], v[i]);
}

/* Active set A(x): x_i at one of its bounds (Section 2). */
static int is_active(double x, double l, double u) { return x == l || x == u; }

/* Binding set B(x): at l with d_i q >= 0, or at u with d_i q <= 0 (Section 2). */
static int is_binding(double x, double l, double u, double g) {
#if ORA_MUTANT == 9
  return (x == l && g <= 0.0) || (x == u && g >= 0.0);
#else
  return (x == l && g >= 0.0) || (x == u && g <= 0.0);
#endif
}

/* Projected gradient, eq. (proj-gradient) of Section 2; a fixed variable
 * (l_i = u_i) gets 0. */
static double proj_grad_1(double x, double l, double u, double g) {
  if (x == l && x == u) return 0.0;
  if (x == l) return g < 0.0 ? g : 0.0;
#if ORA_MUTANT == 1
  if (x == u) return g < 0.0 ? g : 0.0;
#else
  if (x == u) return g > 0.0 ? g : 0.0;
#endif
  return g;
}

void ora_proj_gradient(int64_t n, const double *x, const double *l, const double *u,
                       const double *g, double *pg) {
  for (int64_t i = 0; i < n; ++i) pg[i] = proj_grad_1(x[i], l[i], u[i], g[i]);
}

double ora_proj_gradient_norm(int64_t n, const double *x, const double *l, const double *u,
                              const double *g) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double p = proj_grad_1(x[i], l[i], u[i], g[i]);
    s += p * p;
  }
  return sqrt(s);
}

/* Counts of the face of x: lower-active (x = l, including fixed), upper-active
 * (x = u != l), and active-but-not-binding variables.  The last is zero exactly
 * when B(x) = A(x). */
void ora_classify(int64_t n, const double *x, const double *l, const double *u,
                  const double *g, int64_t *n_lower, int64_t *n_upper,
                  int64_t *n_nonbinding) {
  int64_t lo = 0, up = 0, nb = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (x[i] == l[i]) ++lo;
    else if (x[i] == u[i]) ++up;
    if (is_active(x[i], l[i], u[i]) && !is_binding(x[i], l[i], u[i], g[i])) ++nb;
  }
  *n_lower = lo;
  *n_upper = up;
  *n_nonbinding = nb;
}

/* Initial step of the gradient-projection search, eq. (bqpls): along
 * d = -P grad q(y) the model is a 1-D quadratic in alpha whose minimiser is
 * ||d||^2 / d'Ad (g'P grad q = ||P grad q||^2).  Returns d'd and d'Ad. */
void ora_gp_alpha0(const ora_csr *A, const double *y, const double *l, const double *u,
                   const double *g, double *dd, double *dAd) {
  int64_t n = A->n;
  double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *Ad = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  ora_proj_gradient(n, y, l, u, g, d);
  ora_matvec(A, d, Ad);
  *dd = ora_dot(n, d, d);
  *dAd = ora_dot(n, d, Ad);
  free(d);
  free(Ad);
}

/* One trial point of a projected search: ynew = P[y + alpha dir], s = ynew - y,
 * the decrease pieces g's and s'As (q(ynew) - q(y) = g's + 1/2 s'As), and the
 * number of variables whose membership in the active set changes. */
void ora_trial(const ora_csr *A, const double *y, const double *dir, double alpha,
               const double *l, const double *u, const double *g, double *ynew,
               double *gs, double *sAs, int64_t *nchg) {
  int64_t n = A->n;
  double *s = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *As = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  int64_t c = 0;
  for (int64_t i = 0; i < n; ++i) {
    double t = y[i] + alpha * dir[i];
    ynew[i] = mid3(l[i], u[i], t);
    s[i] = ynew[i] - y[i];
    if (is_active(ynew[i], l[i], u[i]) != is_active(y[i], l[i], u[i])) ++c;
  }
  ora_matvec(A, s, As);
  *gs = ora_dot(n, g, s);
  *sAs = ora_dot(n, s, As);
  *nchg = c;
  free(s);
  free(As);
}

/* q(y + s) - q(y) = g's + 1/2 s'As, exactly, for the quadratic q. */
double ora_decrease(double gs, double sAs) {
#if ORA_MUTANT == 2
  return gs + sAs;
#else
  return gs + 0.5 * sAs;
#endif
}

/* Reduced matrix A_k = Z_k' A Z_k for the index set F (the free variables,
 * listed in increasing order): rows and columns of A whose index is in F. */
static void extract_submatrix(const ora_csr *A, const int64_t *F, int64_t m, const int64_t *pos,
                              int32_t **rp, int32_t **ci, double **va) {
  int64_t nnz = 0;
  for (int64_t a = 0; a < m; ++a) {
    int64_t i = F[a];
    for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
      if (pos[A->colind[k]] >= 0) ++nnz;
  }
  *rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  *va = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t t = 0;
  (*rp)[0] = 0;
  for (int64_t a = 0; a < m; ++a) {
    int64_t i = F[a];
    for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
      int64_t p = pos[A->colind[k]];
      if (p >= 0) {
        (*ci)[t] = (int32_t)p;
        (*va)[t] = A->vals[k];
        ++t;
      }
    }
    (*rp)[a + 1] = (int32_t)t;
  }
}

/* Conjugate gradients on the reduced problem min 1/2 w'A_k w + r_k'w from
 * w_0 = 0 (Section 3, eq. (cg2)), stopped by the relative-decrease test
 * (cgstop1) with tolerance eta, when the residual vanishes, or after max_cg
 * iterations.  `free_mask[i]` != 0 marks the free variables; the result is
 * d = Z_k w written into d (zero on the active set).  Returns ORA_OK or
 * ORA_ERR_NOT_SPD; *iters gets the number of CG iterations; decs (optional,
 * capacity dec_cap) receives q_k(w_{j-1}) - q_k(w_j) for each iteration. */
int ora_reduced_cg(const ora_csr *A, const unsigned char *free_mask, const double *g,
                   double eta, int32_t max_cg, int32_t precond, int32_t cg_stop, double *d,
                   int32_t *iters, double *decs, int32_t dec_cap) {
  int64_t n = A->n;
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (free_mask[i]) {
      pos[i] = m;
      F[m++] = i;
    } else {
      pos[i] = -1;
    }
  }
  for (int64_t i = 0; i < n; ++i) d[i] = 0.0;
  *iters = 0;
  if (m == 0) {
    free(pos);
    free(F);
    return ORA_OK;
  }
  int32_t *rp, *ci;
  double *va;
  extract_submatrix(A, F, m, pos, &rp, &ci, &va);
  ora_csr Ak = {m, rp, ci, va};

  double *w = (double *)calloc((size_t)m, sizeof(double));
  double *rho = (double *)malloc(sizeof(double) * (size_t)m);
  double *z = (double *)malloc(sizeof(double) * (size_t)m);
  double *p = (double *)malloc(sizeof(double) * (size_t)m);
  double *q = (double *)malloc(sizeof(double) * (size_t)m);
  double *dinv = (double *)malloc(sizeof(double) * (size_t)m);
  int status = ORA_OK;
  /* Preconditioner M: the identity, or the diagonal of A_k (the paper's
   * diagonal Jacobi preconditioner, Section "Preconditioners"). */
  for (int64_t a = 0; a < m; ++a) {
    dinv[a] = 1.0;
    if (precond == 1) {
      double diag = 0.0;
      for (int32_t e = rp[a]; e < rp[a + 1]; ++e)
        if (ci[e] == a) diag += va[e];
      if (!(diag > 0.0)) status = ORA_ERR_NOT_SPD;
      dinv[a] = 1.0 / diag;
    }
  }
  /* r_k = Z_k' grad q(x_k); the residual of A_k w + r_k = 0 at w = 0 is -r_k */
  for (int64_t a = 0; a < m; ++a) {
#if ORA_MUTANT == 6
    rho[a] = g[F[a]];
#else
    rho[a] = -g[F[a]];
#endif
    z[a] = precond == 1 ? dinv[a] * rho[a] : rho[a];
    p[a] = z[a];
  }
  double rz = ora_dot(m, rho, z);
  const double rz0 = rz;
  int64_t cap = max_cg > 0 ? max_cg : m;
  double decmax = -INFINITY;
  int32_t j = 0;
  if (status == ORA_OK && rz > 0.0) {
    for (;;) {
      ora_matvec(&Ak, p, q);
      double pq = ora_dot(m, p, q);
      if (!(pq > 0.0)) {
        status = ORA_ERR_NOT_SPD;
        break;
      }
      double alpha = rz / pq;
      for (int64_t a = 0; a < m; ++a) w[a] += alpha * p[a];
      for (int64_t a = 0; a < m; ++a) rho[a] -= alpha * q[a];
      for (int64_t a = 0; a < m; ++a) z[a] = precond == 1 ? dinv[a] * rho[a] : rho[a];
      double rz_new = ora_dot(m, rho, z);
      ++j;
      /* q_k(w_{j-1}) - q_k(w_j) = alpha rho'z - 1/2 alpha^2 p'A_k p = 1/2 alpha rho'z,
       * since rho'p = rho'z for (preconditioned) conjugate gradients */
#if ORA_MUTANT == 10
      double dec = alpha * rz;
#else
      double dec = 0.5 * alpha * rz;
#endif
      if (decs && j <= dec_cap) decs[j - 1] = dec;
      /* eq. (cgstop1); or the standard residual test the paper sets it
       * against, ||r_k + A_k w_j|| <= eta ||r_k|| (in the M^{-1} norm when
       * preconditioned: rho'z) */
      int stop = (rz_new == 0.0) || (j >= cap);
#if ORA_MUTANT == 12
      if (cg_stop == 1) stop = stop || (rz_new <= eta * rz0);
#else
      if (cg_stop == 1) stop = stop || (sqrt(rz_new) <= eta * sqrt(rz0));
#endif
      else stop = stop || (j >= 2 && dec <= eta * decmax);
#if ORA_MUTANT == 13
      if (j == 1) decmax = dec;
#else
      if (dec > decmax) decmax = dec;
#endif
      if (stop) break;
#if ORA_MUTANT == 5
      double beta = rz / rz_new;
#else
      double beta = rz_new / rz;
#endif
#if ORA_MUTANT == 11
      for (int64_t a = 0; a < m; ++a) p[a] = rho[a] + beta * p[a];
#else
      for (int64_t a = 0; a < m; ++a) p[a] = z[a] + beta * p[a];
#endif
      rz = rz_new;
    }
  }
  for (int64_t a = 0; a < m; ++a) d[F[a]] = w[a];
  *iters = j;
  free(w);
  free(rho);
  free(z);
  free(p);
  free(q);
  free(dinv);
  free(rp);
  free(ci);
  free(va);
  free(pos);
  free(F);
  return status;
}

/* ----------------------------------------------------------- Algorithm GPCG */

static int has_nan(int64_t n, const double *v) {
  for (int64_t i = 0; i < n; ++i)
    if (v[i] != v[i]) return 1;
  return 0;
}

static int finish(ora_stats *st, int status, const ora_csr *A, const double *b,
                  const double *l, const double *u, const double *x, const double *g) {
  int64_t lo, up, nb;
  st->status = status;
  st->pg = ora_proj_gradient_norm(A->n, x, l, u, g);
  ora_classify(A->n, x, l, u, g, &lo, &up, &nb);
  st->n_lower = lo;
  st->n_upper = up;
  st->n_free = A->n - lo - up;
  st->q = ora_objective(A, b, x);
  return status;
}

/* Solve the QP from x0; x receives the answer, g (nullable) its gradient. */
int ora_gpcg(const ora_csr *A, const double *b, const double *l, const double *u,
             const double *x0, const ora_options *opt_in, double *x, double *g_out,
             ora_stats *st) {
  ora_options opt;
  if (opt_in) opt = *opt_in;
  else ora_default_options(&opt);
  int64_t n = A->n;
  ora_stats keep = *st; /* the caller's trace buffers survive the reset */
  memset(st, 0, sizeof(*st));
  st->trace_q = keep.trace_q;
  st->trace_act = keep.trace_act;
  st->trace_cap = keep.trace_cap;
  st->trace_cg_eta = keep.trace_cg_eta;
  st->trace_cg_iters = keep.trace_cg_iters;
  st->trace_cg_repeat = keep.trace_cg_repeat;
  st->trace_cg_dec = keep.trace_cg_dec;
  st->trace_cg_cap = keep.trace_cg_cap;
  st->trace_dec_per = keep.trace_dec_per;
  if (n <= 0) return st->status = ORA_ERR_ARG;
  if (has_nan(n, b) || has_nan(n, l) || has_nan(n, u) || has_nan(n, x0))
    return st->status = ORA_ERR_NAN;
  for (int64_t i = 0; i < n; ++i)
    if (l[i] > u[i]) return st->status = ORA_ERR_BOUNDS;

  size_t bytes = sizeof(double) * (size_t)n;
  double *g = (double *)malloc(bytes);
  double *y = (double *)malloc(bytes);
  double *dir = (double *)malloc(bytes);
  double *d = (double *)malloc(bytes);
  unsigned char *fm = (unsigned char *)malloc((size_t)n);
  int status = ORA_OK;

  /* x_0 must lie in the feasible set; an outside start is projected. */
  ora_project(n, l, u, x0, x);
  for (int64_t i = 0; i < n; ++i)
    if (x[i] != x0[i]) {
      st->x0_projected = 1;
      break;
    }
  ora_gradient(A, x, b, g);
  double pgn = ora_proj_gradient_norm(n, x, l, u, g);
  st->pg0 = pgn;
  double tau = opt.tol_abs;
  if (opt.tol_rel * pgn > tau) tau = opt.tol_rel * pgn;
  st->tau = tau;
  if (pgn <= tau) goto done;
  double best_pg = pgn;
  int32_t stall = 0;
#if ORA_MUTANT == 14
  const double eta_gp = opt.eta2, eta_cg0 = opt.eta1;
#else
  const double eta_gp = opt.eta1, eta_cg0 = opt.eta2;
#endif
  double eta = eta_cg0;

  for (;;) {
    /* ---- gradient-projection phase, eqs. (next-y)-(pgstop2) ---- */
    int32_t gp_accepts = 0;
    {
      double decmax = -INFINITY;
      for (int32_t j = 1;; ++j) {
        double dd, dAd;
        ora_gp_alpha0(A, x, l, u, g, &dd, &dAd);
        if (dd == 0.0) goto done; /* P grad q = 0: x is optimal */
        if (!(dAd > 0.0)) {
          status = ORA_ERR_NOT_SPD;
          goto done;
        }
#if ORA_MUTANT == 4
        double alpha = dAd / dd;
#else
        double alpha = dd / dAd;
#endif
        for (int64_t i = 0; i < n; ++i) dir[i] = -g[i];
        int accepted = 0;
        double gs = 0, sAs = 0, delta = 0;
        int64_t nchg = 0;
        for (int32_t bt = 0; bt <= opt.max_backtrack; ++bt) {
          ora_trial(A, x, dir, alpha, l, u, g, y, &gs, &sAs, &nchg);
          delta = ora_decrease(gs, sAs);
          if (delta <= opt.mu * gs) {
            accepted = 1;
            break;
          }
          alpha *= 0.5;
          ++st->backtracks;
        }
        if (!accepted) break; /* no sufficient decrease above rounding level */
        memcpy(x, y, bytes);
        ora_gradient(A, x, b, g);
        ++st->gp_iters;
        ++gp_accepts;
        double dec = -delta;
        int stop = (nchg == 0) || (j >= 2 && dec <= eta_gp * decmax) || (j >= opt.max_gp);
        if (dec > decmax) decmax = dec;
        if (stop) break;
      }
      pgn = ora_proj_gradient_norm(n, x, l, u, g);
      if (pgn <= tau) goto done;
    }

    /* ---- CG on the face, then projected search; repeat while B = A ---- */
#if ORA_MUTANT != 16
    eta = eta_cg0; /* a gradient-projection phase ran: eta2 starts afresh */
#endif
    int repeat = 0;
    for (;;) {
      int64_t m = 0;
      for (int64_t i = 0; i < n; ++i) {
#if ORA_MUTANT == 3
        fm[i] = !is_binding(x[i], l[i], u[i], g[i]);
#else
        fm[i] = !is_active(x[i], l[i], u[i]);
#endif
        m += fm[i];
      }
      int64_t act_before = n - m;
      if (m == 0) {
        /* no free variable: back to gradient projection, unless that phase
         * could not move at all (nothing left above rounding level) */
        if (gp_accepts == 0) {
          status = ORA_STAGNATED;
          goto done;
        }
        break;
      }
      int32_t it = 0;
      const int traced = st->trace_cg_len < st->trace_cg_cap;
      double *dec_out = NULL;
      if (traced) {
        if (st->trace_cg_eta) st->trace_cg_eta[st->trace_cg_len] = eta;
        if (st->trace_cg_repeat) st->trace_cg_repeat[st->trace_cg_len] = repeat;
        if (st->trace_cg_dec && st->trace_dec_per > 0)
          dec_out = st->trace_cg_dec + (int64_t)st->trace_cg_len * st->trace_dec_per;
      }
      int cgs = ora_reduced_cg(A, fm, g, eta, opt.max_cg, opt.precond, opt.cg_stop, d, &it,
                               dec_out, dec_out ? st->trace_dec_per : 0);
      if (traced) {
        if (st->trace_cg_iters) st->trace_cg_iters[st->trace_cg_len] = it;
        ++st->trace_cg_len;
      }
      st->cg_iters += it;
      ++st->cg_phases;
      if (cgs != ORA_OK) {
        status = cgs;
        goto done;
      }
      /* projected search along d_k, eq. (cglsstop2), alpha = 1, 1/2, ... */
      double alpha = 1.0;
      int accepted = 0;
      double gs = 0, sAs = 0, delta = 0;
      int64_t nchg = 0;
      for (int32_t bt = 0; bt <= opt.max_backtrack; ++bt) {
        ora_trial(A, x, d, alpha, l, u, g, y, &gs, &sAs, &nchg);
        delta = ora_decrease(gs, sAs);
        if (delta <= opt.mu * gs) {
          accepted = 1;
          break;
        }
        alpha *= 0.5;
        ++st->backtracks;
      }
      if (accepted) memcpy(x, y, bytes);
      ora_gradient(A, x, b, g);
      ++st->outer_iters;
      if (st->trace_len < st->trace_cap) {
        if (st->trace_q) st->trace_q[st->trace_len] = ora_objective(A, b, x);
        if (st->trace_act) {
          int64_t act_after = 0;
          for (int64_t i = 0; i < n; ++i) act_after += is_active(x[i], l[i], u[i]);
          st->trace_act[2 * st->trace_len] = act_before;
          st->trace_act[2 * st->trace_len + 1] = act_after;
        }
        ++st->trace_len;
      }
      pgn = ora_proj_gradient_norm(n, x, l, u, g);
      if (pgn <= tau) goto done;
      if (pgn < best_pg) {
        best_pg = pgn;
        stall = 0;
      } else if (++stall >= opt.max_stall) {
        status = ORA_STAGNATED;
        goto done;
      }
      if (!accepted) {
        status = ORA_STAGNATED;
        goto done;
      }
      if (st->outer_iters >= opt.max_outer) {
        status = ORA_MAXIT;
        goto done;
      }
      int64_t lo, up, nb;
      ora_classify(n, x, l, u, g, &lo, &up, &nb);
      if (nb != 0) break; /* B(x) != A(x): next GPCG iteration starts with GP */
#if ORA_MUTANT != 15
      eta *= opt.eta2_reduce; /* cgstop3: same face, more accurate CG */
#endif
      repeat = 1;
      ++st->face_repeats;
    }
  }

done:
  finish(st, status, A, b, l, u, x, g);
  if (g_out) memcpy(g_out, g, bytes);
  free(g);
  free(y);
  free(dir);
  free(d);
  free(fm);
  return st->status;
}
