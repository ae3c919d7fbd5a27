/*
 * zeus_oracle.h -- plain CPU oracle for the batched multistart method of
 * "Zeus: An Efficient GPU Optimization Method Integrating PSO, BFGS, and
 * Automatic Differentiation" (Soos, Paterno, Ranjan, Zubair).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, constant table or helper with the GPU library: everything
 * here (Philox, dual numbers, objectives, PSO, BFGS) is written separately.
 *
 * Everything is IEEE double, built with -O2 -ffp-contract=off and without
 * -ffast-math: a multiply-add is fused only where the code calls fma().
 *
 * The file builds twice.  The default build fixes the order of every
 * rounding by readings stated in the source (balanced pairwise sums, blocked
 * fused row products, sin/cos/exp by Cody-Waite reduction and Taylor series).
 * The plain build (-DZO_PLAIN, libzeus_oracle_plain.so) takes the textbook
 * order: every sum left to right, row products and the rank-2 update
 * unfused, the C library's sin, cos, exp and log.
 *
 * Readings of the paper that this oracle fixes (the paper is silent or
 * ambiguous there) are listed next to the code that applies them.
 */
#ifndef ZEUS_ORACLE_H
#define ZEUS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Objective identifiers (values are this library's own). */
enum {
  ZO_ROSENBROCK = 0,      /* Sec. V-B, Rosenbrock                         */
  ZO_RASTRIGIN = 1,       /* Sec. V-B, Rastrigin, A = 10                  */
  ZO_ACKLEY = 2,          /* Sec. V-B, Ackley                             */
  ZO_STYBLINSKI_TANG = 3, /* standard Styblinski-Tang test function       */
  ZO_GOLDSTEIN_PRICE = 4, /* Sec. V-B, Goldstein-Price (dim = 2)          */
  ZO_SPHERE = 5,          /* test-only: 0.5 * sum x_i^2                    */
  ZO_QUARTIC = 6,         /* test-only: sum x_i^4                          */
  ZO_USER = 7             /* user source, see zo_set_user                  */
};

/* Relative decision margin below which a branch counts as a near-tie. */
#define ZO_TIE_MARGIN 1e-9

/* Per-start termination status. */
enum { ZO_MAXITER = 0, ZO_CONVERGED = 1, ZO_STOPPED = 2, ZO_NONFINITE = 3 };

/* Random-stream tags (fourth Philox counter word). */
enum { ZO_TAG_X0 = 0, ZO_TAG_V0 = 1, ZO_TAG_R1 = 2, ZO_TAG_R2 = 3 };

typedef struct {
  int32_t objective;
  int32_t dim;
  int64_t n;            /* particles == BFGS starts                          */
  double lower, upper;  /* sampling box, same on every axis                  */
  int32_t iter_pso;     /* number of synchronous swarm updates               */
  double w, c1, c2;     /* inertia, cognitive, social coefficients           */
  double v_half;        /* initial velocity drawn in [-v_half, v_half];
                           <= 0 means (upper - lower) as in Alg. 2            */
  int32_t iter_bfgs;    /* BFGS iteration budget                              */
  int32_t iter_ls;      /* Armijo trials per line search                      */
  double armijo_c;      /* sufficient-decrease constant                       */
  double ls_shrink;     /* backtracking factor                                */
  double grad_tol;      /* Theta: converged when ||g||_2 < Theta               */
  uint64_t seed;        /* Philox key word 0                                  */
  uint64_t request_id;  /* Philox key word 1                                  */
  int32_t lbfgs_m;      /* 0: BFGS with the full inverse Hessian; m > 0:
                           L-BFGS keeping the m most recent (s, y) pairs       */
} zo_problem;

/* Swarm state after PSO.  Arrays are caller-owned, row-major [n][dim]. */
typedef struct {
  double *x;     /* current positions (BFGS starts)   */
  double *v;     /* velocities                        */
  double *px;    /* personal-best positions           */
  double *pf;    /* personal-best values   [n]        */
  double *gx;    /* global-best position   [dim]      */
  double gf;     /* global-best value                 */
  int64_t gidx;  /* particle that supplied gx         */
  int64_t near_ties; /* best-comparisons whose operands were within a relative
                        1e-12 of each other (possible flips under ulp noise)  */
} zo_swarm;

/* Per-start BFGS outcome.  Caller-owned arrays indexed by position in the
 * list of starts handed to zo_bfgs. */
typedef struct {
  double *x;          /* [m][dim] final iterate                         */
  double *f;          /* [m] final objective value                      */
  int32_t *iters;     /* [m] BFGS steps taken                           */
  int32_t *status;    /* [m] ZO_MAXITER / ZO_CONVERGED / ZO_NONFINITE   */
  int32_t *ls_trials; /* [m] objective evaluations in line searches     */
  int32_t *ls_fail;   /* [m] line searches with no accepted trial        */
  int32_t *skips;     /* [m] updates skipped because y's <= 0            */
  int32_t *resets;    /* [m] H reset to I because g'p was not < 0        */
  double *min_margin; /* [m] smallest relative margin of any discrete
                         decision taken (Armijo, y's > 0, g'p < 0,
                         ||g|| < Theta); nullable                         */
  int32_t *tie_iter;  /* [m] first iteration with a decision margin below
                         ZO_TIE_MARGIN, -1 if none; nullable              */
  double *trace;      /* [m][trace_len][dim] iterates x_0..; nullable    */
  int32_t trace_len;
} zo_bfgs_out;

/* ---- pieces, exposed for pinning tests ---------------------------------- */

/* Philox4x64 with 10 rounds (Salmon et al., SC'11). */
void zo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                      uint64_t out[4]);

/* The uniform in [0,1) used for draw j of stream (start i, iteration t, tag):
 * counter (j/4, i, t, tag), key (seed, request_id), word j%4, mapped by
 * (w >> 11) * 2^-53. */
double zo_uniform(uint64_t seed, uint64_t request_id, uint64_t i, uint64_t t,
                  uint64_t tag, uint64_t j);

/* sin, cos, exp and log used by the objectives: Cody-Waite reduction and
 * Taylor series with fused multiply-adds (about one ulp; sin and cos are NaN
 * from |x| = 2^48 on); the C library's in the plain build. */
double zo_sin(double x);
double zo_cos(double x);
double zo_exp(double x);
double zo_log(double x);

/* User objective (ZO_USER): `value` returns f(x) evaluated in double,
 * `dual_eval` evaluates f once on the dual numbers xv[i] + xt[i] eps and
 * returns the value part, storing the tangent part in *t.  Both come from
 * the user's source compiled for the CPU (oracle/user.py) and must be safe
 * to call from several threads.  Process-wide; NULL clears it. */
typedef double (*zo_user_value_fn)(const double *x, int d);
typedef double (*zo_user_dual_fn)(const double *xv, const double *xt, int d, double *t);
void zo_set_user(zo_user_value_fn value, zo_user_dual_fn dual_eval);

/* Objective value (primal evaluation). */
double zo_f(int objective, const double *x, int dim);

/* Forward-mode AD gradient, Alg. 5: dim passes of the objective evaluated on
 * dual numbers, pass j seeded with tangent e_j.  *f receives the value part
 * of the last pass (all passes have the same value part). */
void zo_grad(int objective, const double *x, int dim, double *f, double *g);

/* Row of the inverse Hessian times a vector, sum_c hrow[c] v[c] over
 * c < dim: fused multiply-add chains over blocks of 16 consecutive columns,
 * the block sums added pairwise (the order used for u = H y and p = -H g);
 * plain build: unfused, columns ascending. */
double zo_hrow_dot(const double *hrow, const double *v, int dim);

/* One rank-2 inverse-Hessian update (Alg. 4), in place on H [dim][dim].
 * Returns 1 if applied, 0 if skipped because y's <= 0 (or NaN). */
int zo_bfgs_update(double *H, const double *s, const double *y, int dim);

/* Armijo backtracking line search (Alg. 6).  Returns the step length; *trials
 * receives the number of objective evaluations, *accepted 1/0. */
double zo_line_search(const zo_problem *pb, const double *x, double f0,
                      const double *p, double ddir, double *xt_scratch,
                      int32_t *trials, int32_t *accepted);

/* ---- the method --------------------------------------------------------- */

/* L-BFGS search direction p = -H g by the two-loop recursion (Nocedal and
 * Wright, "Numerical Optimization", 2nd ed., Alg. 7.4): H is the inverse-
 * Hessian approximation built from the `count` pairs in the rows of S and Y
 * (oldest first, rho_i = 1 / y_i's_i) on H0 = gamma I, gamma = s'y / y'y of
 * the newest pair (their eq. 7.20); with no pairs, p = -g. */
void zo_lbfgs_direction(const double *S, const double *Y, const double *rho, int count,
                        const double *g, int dim, double *p);

/* The L-BFGS pair window: S and Y hold the *count <= m newest pairs in their
 * rows, oldest first, with rho_i = 1 / (y_i's_i).  Appends (s, y) when
 * y's > 0, first dropping the oldest pair when m are held, and returns 1;
 * returns 0 and leaves the window unchanged otherwise.  A restart from H = I
 * empties the window (*count = 0). */
int zo_lbfgs_push(double *S, double *Y, double *rho, int *count, int m, const double *s,
                  const double *y, int dim);

/* 0 if the problem is acceptable, -1 otherwise. */
int zo_validate(const zo_problem *pb);

/* Alg. 2 then iter_pso synchronous applications of Alg. 3. */
int zo_pso(const zo_problem *pb, zo_swarm *sw);

/* BFGS (Alg. 4 with Alg. 5 and Alg. 6) from starts x0[idx[k]], k < m.
 * x0 is [n][dim].  Parallel over starts with OpenMP when nthreads > 1. */
int zo_bfgs(const zo_problem *pb, const double *x0, const int64_t *idx,
            int64_t m, zo_bfgs_out *out, int nthreads);

/* Best-of-N (Alg. 7's final reduction): lowest finite f, lowest index on
 * ties; returns -1 when no f is finite.  *n_conv gets the CONVERGED count. */
int64_t zo_best(const double *f, const int32_t *status, int64_t m,
                int64_t *n_conv);

/* Number of OpenMP threads this build would use. */
int zo_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
