/*
 * zeus.h -- C ABI of libzeus.so: batched multistart minimisation on AMD
 * Instinct MI355X (gfx950) following "Zeus: An Efficient GPU Optimization
 * Method Integrating PSO, BFGS, and Automatic Differentiation".
 *
 * The problem statement follows the paper's driver (Alg. 7, and Alg. 1 for
 * the sequential form): minimise f over the box [lower, upper]^dim from N
 * starts.  A swarm of N particles is initialised uniformly in the box
 * (Alg. 2 / Alg. 8) and moved by iter_pso synchronous PSO updates (Alg. 3 /
 * Alg. 9); then one BFGS run starts from every particle's position (Alg. 4 /
 * Alg. 10) with forward-mode dual-number gradients (Alg. 5) and an Armijo
 * backtracking line search (Alg. 6); finally the best start is reduced
 * (Alg. 7).  Each start reports its minimum, argmin, iteration count and
 * status.
 *
 * Conventions for every entry point:
 *  - Every call returns a zeus_err; no C++ exception crosses this boundary.
 *    On an error, zeus_last_error() returns a message (thread-local, valid
 *    until the next call on the same thread) and no output has been written
 *    (asynchronous calls: nothing has been enqueued).
 *  - The caller owns every struct and array passed in.  The library copies
 *    the problem at call time.
 *  - Results are a pure function of the problem: they do not depend on the
 *    device's occupancy, on work-queue order or on other calls.
 *  - A context serialises its own calls; different contexts may be used from
 *    different threads.
 */
#ifndef ZEUS_H
#define ZEUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ZEUS_ABI_VERSION 2u

typedef enum zeus_err {
  ZEUS_OK = 0,
  ZEUS_NOT_READY = 1,
  ZEUS_EINVAL = -1,       /* invalid argument or problem                     */
  ZEUS_ENOMEM = -2,       /* device or host allocation failed                 */
  ZEUS_EHIP = -3,         /* a HIP runtime call failed (message has details)  */
  ZEUS_EUNSUPPORTED = -4, /* valid problem this build cannot run              */
  ZEUS_ECANCELLED = -5,
  ZEUS_ETIMEOUT = -6
} zeus_err;

/* Objectives.  Rosenbrock, Rastrigin, Ackley and Goldstein-Price are the test
 * functions of Sec. V-B; Styblinski-Tang is the standard test function
 * 0.5 * sum (x^4 - 16 x^2 + 5 x); SPHERE (0.5 ||x||^2) and QUARTIC (sum x^4)
 * are small test objectives with exactly representable line searches. */
typedef enum zeus_objective {
  ZEUS_ROSENBROCK = 0,      /* dim >= 2 */
  ZEUS_RASTRIGIN = 1,
  ZEUS_ACKLEY = 2,
  ZEUS_STYBLINSKI_TANG = 3,
  ZEUS_GOLDSTEIN_PRICE = 4, /* dim == 2 */
  ZEUS_SPHERE = 5,
  ZEUS_QUARTIC = 6,
  ZEUS_USER = 7             /* user code, see zeus_objective_compile */
} zeus_objective;

/* ZEUS_FP64: everything in IEEE double.
 * ZEUS_MIXED: objective and dual numbers in float; inverse Hessian, search
 *             direction, g'p, the Armijo comparison, s, y and y's in double. */
typedef enum zeus_precision { ZEUS_FP64 = 0, ZEUS_MIXED = 1 } zeus_precision;

/* Per-start termination status (Alg. 4: status 1 when ||grad|| < Theta,
 * status 0 when the iteration budget runs out). */
typedef enum zeus_start_status {
  ZEUS_ST_MAXITER = 0,
  ZEUS_ST_CONVERGED = 1,
  ZEUS_ST_STOPPED = 2,   /* stopped early at required_converged                 */
  ZEUS_ST_NONFINITE = 3  /* f or a gradient component became inf/NaN          */
} zeus_start_status;

/* The problem, after Alg. 7's argument list
 * Zeus(f, N, range, iter_bfgs, iter_pso, iter_ls, required_c, Theta, w, c1, c2).
 * Field meanings and the defaults the paper uses: */
typedef struct zeus_problem {
  uint32_t abi_version;  /* must be ZEUS_ABI_VERSION                             */
  int32_t objective;     /* zeus_objective                                       */
  int32_t dim;           /* 1 <= dim <= 256 in this build                         */
  int32_t precision;     /* zeus_precision                                       */
  int64_t n_starts;      /* N particles == N BFGS starts, >= 1                    */
  double lower, upper;   /* sampling box, same on every axis (Alg. 2 'range');
                            the search itself is unconstrained                    */
  int32_t iter_pso;      /* synchronous PSO updates, >= 0                          */
  int32_t iter_bfgs;     /* BFGS iteration budget per start, >= 0                  */
  int32_t iter_ls;       /* Armijo trials per line search, >= 1 (paper: 20)         */
  int32_t lbfgs_m;       /* 0: BFGS with the full inverse Hessian (Alg. 4).  1..8:
                            limited-memory BFGS keeping the lbfgs_m newest (s, y)
                            pairs with y's > 0, direction by the two-loop
                            recursion on H0 = (s'y / y'y) I of the newest pair
                            (Nocedal and Wright, Alg. 7.4 and eq. 7.20), the
                            remedy Sec. VII names for the d^2 update; no d x d
                            matrix is kept.  > 8: ZEUS_EUNSUPPORTED            */
  double w, c1, c2;      /* PSO inertia, cognitive, social (paper: 0.5, 1.2, 1.5)  */
  double v_half;         /* initial velocity in [-v_half, v_half]; <= 0 selects
                            upper - lower as in Alg. 2                             */
  double armijo_c;       /* sufficient-decrease constant in (0,1) (paper: 0.3)      */
  double ls_shrink;      /* backtracking factor in (0,1) (paper: 0.5)               */
  double grad_tol;       /* Theta > 0: a start converges when ||grad||_2 < Theta     */
  int64_t required_converged; /* 0: off.  c > 0: stop when c starts have converged
                            (Alg. 10), read iteration-synchronously: K* is the
                            iteration at which the c-th start converges, and
                            every start still running at K* ends there with
                            status ZEUS_ST_STOPPED (its K*-th iterate).  Decided
                            on the device, with no host round trip, at every
                            entry point; the workspace grows by
                            4 (iter_bfgs + 5) bytes                           */
  uint64_t seed;         /* Philox key word 0                                      */
  uint64_t request_id;   /* Philox key word 1                                      */
} zeus_problem;

/* Reductions over all starts (Alg. 7's final ParallelReduction and counts). */
typedef struct zeus_summary {
  int64_t best_index;     /* start with the lowest finite f (lowest index on
                             ties); -1 if no f is finite                          */
  double best_f;
  int64_t n_converged;    /* starts with status CONVERGED                         */
  int64_t n_nonfinite;    /* starts with status NONFINITE                         */
  int64_t total_iters;    /* sum of BFGS iterations over starts                   */
  int64_t total_ls_trials;/* sum of line-search objective evaluations, counted as
                             the sequential Alg. 6 would evaluate them            */
  int64_t pso_best_index; /* particle holding the PSO global best                 */
  double pso_best_f;
} zeus_summary;

/* Where results go.  For zeus_minimize every pointer is host memory; for
 * zeus_minimize_async every pointer is device memory.  Required: f, x,
 * iters, status, summary.  Optional (NULL to skip): everything else. */
typedef struct zeus_result {
  double *f;            /* [N] final objective value per start                 */
  double *x;            /* [N][dim] final iterate per start (row-major)        */
  int32_t *iters;       /* [N] BFGS iterations taken                           */
  int32_t *status;      /* [N] zeus_start_status                               */
  int32_t *ls_trials;   /* [N] line-search evaluations (sequential count)      */
  double *seeds;        /* [N][dim] particle positions after PSO = BFGS starts */
  double *pso_v;        /* [N][dim] velocities after PSO                        */
  double *pso_px;       /* [N][dim] personal-best positions after PSO           */
  double *pso_pf;       /* [N] personal-best values after PSO                   */
  double *pso_best_x;   /* [dim] PSO global-best position                       */
  double *trace;        /* [N][trace_len][dim] iterates x_0, x_1, ...; entries
                           after a start's last iterate are NaN                 */
  int32_t trace_len;    /* 0 disables the trace                                 */
  int32_t reserved0;
  zeus_summary *summary;/* one zeus_summary                                     */
  int32_t *skips;       /* [N] steps whose rank-2 update was skipped because
                           y's <= 0 (Alg. 4's curvature condition; L-BFGS: the
                           pair was not kept)                                    */
  int32_t *resets;      /* [N] search directions that were not descent
                           directions, so H was reset to I and p = -g (L-BFGS:
                           the kept pairs were dropped).  In mixed precision a
                           direction formed again after an escalation to FP64
                           counts again                                          */
} zeus_result;

typedef struct zeus_context zeus_context;

/* Per-kernel device time accumulated by a context while profiling is on,
 * measured with HIP events on the stream the kernels run on. */
typedef struct zeus_profile {
  double pso_ms;        /* swarm initialisation + updates                        */
  double bfgs_ms;       /* the BFGS kernel                                        */
  double reduce_ms;     /* final best-of-N reduction                              */
  int64_t pso_launches, bfgs_launches, reduce_launches;
} zeus_profile;

/* Library and ABI version. */
uint32_t zeus_abi_version(void);
const char *zeus_version(void);

/* Message for the last error on this thread ("" if none). */
const char *zeus_last_error(void);

/* Checks a problem against the rules above.  ZEUS_OK, ZEUS_EINVAL (invalid) or
 * ZEUS_EUNSUPPORTED (valid but outside this build, e.g. dim > 256). */
zeus_err zeus_validate(const zeus_problem *problem);

/* Device workspace that zeus_minimize_async needs for this problem, in bytes.
 * Swarm state x, v, px ([N][dim] doubles each) and pf [N], plus reduction
 * scratch.  Up to 208 dimensions the inverse Hessians never leave the chip
 * (registers, and above 128 dimensions registers and LDS); BFGS above 208
 * dimensions adds one inverse-Hessian slot per resident block (at most 2048
 * slots) of dim x (dim rounded up to 64) doubles. */
zeus_err zeus_workspace_bytes(const zeus_problem *problem, size_t *bytes);

/* Creates a context on HIP device `device` with its own stream (default
 * priority).  *out receives the handle. */
zeus_err zeus_context_create(int device, zeus_context **out);
zeus_err zeus_context_destroy(zeus_context *ctx);

/* Turns per-kernel event timing on or off and clears the accumulators. */
zeus_err zeus_context_set_profiling(zeus_context *ctx, int enabled);
zeus_err zeus_context_get_profile(zeus_context *ctx, zeus_profile *out);

/* Blocking solve.  Allocates (and caches in the context) device memory,
 * runs PSO, BFGS and the reduction on the context's stream, copies every
 * requested output to the host arrays of *out and returns when done. */
zeus_err zeus_minimize(zeus_context *ctx, const zeus_problem *problem,
                       const zeus_result *out);

/* Blocking solve of n independent problems (a batch of uneven requests:
 * objectives, dimensions, start counts and budgets may all differ).  outs[r]
 * receives problem r's results (host memory, as for zeus_minimize).  Requests
 * that share objective, precision and lane count run as one launch group:
 * one swarm launch per sweep and one persistent BFGS launch over all their
 * starts; different groups run concurrently on up to four streams.  Every
 * problem is validated first; if any is invalid nothing runs and the message
 * names it.  Each request's results are bit-identical to solving it alone. */
zeus_err zeus_minimize_batch(zeus_context *ctx, const zeus_problem *problems, int32_t n,
                             const zeus_result *outs);

/* Asynchronous solve on `stream` (a hipStream_t; NULL = the context's stream)
 * with caller-owned device memory: `workspace` of at least
 * zeus_workspace_bytes() bytes (256-byte aligned) and device result arrays in
 * *out.  Only enqueues work; the caller synchronises the stream.  The
 * workspace and outputs must not be used by other work until the stream has
 * passed this call. */
zeus_err zeus_minimize_async(zeus_context *ctx, const zeus_problem *problem,
                             void *workspace, size_t workspace_bytes,
                             const zeus_result *out, void *stream);

/* Largest device workspace that zeus_minimize_async_static can serve: 64 MiB
 * (zeus_workspace_bytes() grows as 24 N dim bytes of swarm state, so for
 * example N = 65,536 starts up to dim 40, or N = 131,072 up to dim 20). */
#define ZEUS_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/* zeus_minimize_async with no device allocation at all, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  The workspace is a fixed device
 * array of ZEUS_STATIC_WORKSPACE_BYTES inside the library, one per GPU, held
 * from the first zeus_context_create on that GPU until the process ends; the
 * caller passes the device result arrays in *out as for
 * zeus_minimize_async, and the results are the same.  Only enqueues work on
 * `stream` (NULL = the context's stream).  ZEUS_ENOMEM, with nothing
 * enqueued, when zeus_workspace_bytes() of the problem exceeds
 * ZEUS_STATIC_WORKSPACE_BYTES.  Every call on one GPU uses that GPU's one
 * array, which keeps the last call's contents: calls whose device work
 * overlaps (different streams, or different contexts on the same GPU,
 * without ordering between them) race and give wrong results; calls on one
 * stream run in order and are safe.  The kernels initialise everything they
 * read from the array (a kernel clears the work counter), so no call depends
 * on what an earlier call left there. */
zeus_err zeus_minimize_async_static(zeus_context *ctx, const zeus_problem *problem,
                                    const zeus_result *out, void *stream);

/* ------------------------------------------------------------------------ */
/* Plans: a batch captured once into a HIP graph and replayed.              */
/*                                                                          */
/* zeus_plan_create lays a batch out in a caller-owned device workspace      */
/* (zeus_plan_workspace_bytes bytes, 256-byte aligned), uploads its request */
/* tables, and captures the kernels of every launch group (counter reset,   */
/* each PSO sweep, the swarm best, the persistent BFGS kernel and the       */
/* best-of-N reduction) into one graph; launch groups become parallel       */
/* branches.  zeus_plan_launch replays the whole solve with one graph       */
/* launch on `stream` (a hipStream_t; NULL = the null stream).  Every       */
/* replay recomputes the same results from the problems' seeds, written to  */
/* the device arrays of outs.  The swarm-state outputs (seeds, pso_*) are   */
/* not available in a plan (ZEUS_EINVAL).  The workspace and outputs must   */
/* not be used by other work while a replay runs, and must outlive the     */
/* plan; replays on one plan must not overlap.                              */
/* ------------------------------------------------------------------------ */
typedef struct zeus_plan zeus_plan;

zeus_err zeus_plan_workspace_bytes(const zeus_problem *problems, int32_t n, size_t *bytes);
zeus_err zeus_plan_create(zeus_context *ctx, const zeus_problem *problems, int32_t n,
                          void *workspace, size_t workspace_bytes, const zeus_result *outs,
                          zeus_plan **out);
zeus_err zeus_plan_launch(zeus_plan *plan, void *stream);
zeus_err zeus_plan_destroy(zeus_plan *plan);

/* ------------------------------------------------------------------------ */
/* Serving: a request loop with continuous batching of starts.              */
/*                                                                          */
/* The paper solves one problem per call (Alg. 7).  A server takes such     */
/* problems from any number of callers and runs them together while more   */
/* arrive, sharing the GPU at the level of starts:                          */
/*  - zeus_server_create allocates the server's device-memory budget once   */
/*    and starts one scheduling thread;                                     */
/*  - requests wait in arrival order and are admitted, oldest first, as     */
/*    soon as their own device memory (result arrays, swarm state, early-   */
/*    stop state, a one-request table) fits in the free budget; there is no */
/*    limit on the number of requests in flight but memory.  An admitted    */
/*    request runs its swarm (Alg. 2 / 3) at once;                          */
/*  - BFGS runs in steps: one persistent kernel launch over slices of the   */
/*    starts of every swarm-finished request of one kernel class (objective,*/
/*    precision, method, lanes), each request taking an equal share, so a   */
/*    short request is not queued behind a long one.  Inside a step a      */
/*    group of lanes takes the next start of any slice when its start       */
/*    retires.  A step runs about four starts per resident group, and two   */
/*    steps run at a time, so requests join within a step's time;          */
/*  - when all starts of a request have run, its best-of-N (Alg. 7) and the */
/*    copies into the caller's arrays finish it and its memory returns to   */
/*    the budget at once.                                                   */
/* A request with required_converged > 0 runs whole in one step of its own */
/* (its stop depends on all its starts).  A request's results are bit-      */
/* identical to solving it alone with zeus_minimize.  A quarter of the      */
/* budget (at most 2 GiB) is kept for the two steps' request tables and the */
/* H slots of problems above 208 dimensions.                                */
/* All server calls are thread-safe.                                        */
/* ------------------------------------------------------------------------ */
typedef struct zeus_server zeus_server;

/* Host steady-clock times (nanoseconds, arbitrary origin) of one request. */
typedef struct zeus_request_times {
  uint64_t t_submit_ns;  /* zeus_server_submit accepted it                  */
  uint64_t t_admit_ns;   /* its memory was allocated and its swarm launched */
  uint64_t t_done_ns;    /* its results were in the host arrays             */
} zeus_request_times;

/* Creates a server on the device of ctx with hbm_budget_bytes of device
 * memory (>= 1 MiB).  min(budget / 4, 2 GiB) of it holds the two steps'
 * tables and H slots; the rest is for requests.  The context must outlive
 * the server. */
zeus_err zeus_server_create(zeus_context *ctx, size_t hbm_budget_bytes, zeus_server **out);

/* Device bytes a request holds from admission until its results are in
 * host_out: its result arrays (the outputs host_out asks for), swarm state,
 * early-stop state and one-request table.  ZEUS_EINVAL as zeus_server_submit. */
zeus_err zeus_server_request_bytes(const zeus_problem *problem, const zeus_result *host_out,
                                   size_t *bytes);

/* Queues one problem.  host_out is as for zeus_minimize (host memory) and,
 * with the problem it points to, must stay valid until the ticket has been
 * waited for (the problem is copied at submission).  *ticket identifies the
 * request.  ZEUS_EINVAL / ZEUS_EUNSUPPORTED as zeus_validate; ZEUS_ENOMEM if
 * the request alone needs more device memory than the budget;
 * ZEUS_ECANCELLED once the server is being destroyed. */
zeus_err zeus_server_submit(zeus_server *srv, const zeus_problem *problem,
                            const zeus_result *host_out, uint64_t *ticket);

/* Waits for a ticket: timeout_ns < 0 waits without limit, 0 only polls.
 * Returns ZEUS_OK (results written; times filled if not NULL),
 * ZEUS_NOT_READY (poll, still queued or running), ZEUS_ETIMEOUT,
 * ZEUS_ECANCELLED (cancelled before it ran), or the error that stopped its
 * batch.  Every outcome but NOT_READY / ETIMEOUT releases the ticket;
 * waiting on a released or unknown ticket is ZEUS_EINVAL. */
zeus_err zeus_server_wait(zeus_server *srv, uint64_t ticket, int64_t timeout_ns,
                          zeus_request_times *times);

/* Cancels a queued request (its wait then returns ZEUS_ECANCELLED).  A
 * request already launched cannot be stopped: ZEUS_NOT_READY, wait for it. */
zeus_err zeus_server_cancel(zeus_server *srv, uint64_t ticket);

/* Cancels every queued request, waits for the admitted ones, stops the
 * scheduling thread and frees the budget. */
zeus_err zeus_server_destroy(zeus_server *srv);

/* The scheduling of a server without a GPU, for testing admission, queueing,
 * cancellation and the sharing of steps on the host.  Nothing runs on a
 * device and no device memory is touched: the budget is only accounted.  An
 * admitted request's swarm takes swarm_ns of host time, a step takes
 * step_ns plus start_ns for every resident_starts starts it runs (rounded
 * up), and finishing a request takes finish_ns; the results written into the
 * caller's arrays are placeholders (f = request_id, x = 0, iters = 0, status
 * ZEUS_ST_MAXITER; summary best_index 0, best_f = request_id, counts 0). */
typedef struct zeus_emulation {
  uint64_t swarm_ns, step_ns, start_ns, finish_ns;
  int64_t resident_starts;  /* starts a step runs at once (> 0)              */
} zeus_emulation;

/* A server as zeus_server_create, on the emulated device of *emu (copied);
 * use it with zeus_server_submit / wait / cancel / destroy.  ZEUS_EINVAL
 * for a NULL argument, resident_starts < 1 or a budget below 1 MiB. */
zeus_err zeus_server_create_emulated(size_t hbm_budget_bytes, const zeus_emulation *emu,
                                     zeus_server **out);

/* ------------------------------------------------------------------------ */
/* User-defined objectives.                                                 */
/*                                                                          */
/* The paper's f is user code: a function of the point written once over a  */
/* number type, so that it gives values and, on dual numbers, directional   */
/* derivatives (Sec. III-C, Alg. 5).  Here it is C++ source compiled at run */
/* time (hipRTC) together with the library's kernel templates.  The source  */
/* defines                                                                  */
/*     template <class T, class X> ZEUS_FN T objective(const X &x, int d);  */
/* where x[i], i < d, is the point's coordinate i as a T; T is double or    */
/* zeus::Dual, and for the float evaluations of ZEUS_MIXED zeus::F32 or     */
/* zeus::DualF (the coordinate rounded to float; every operation in float,  */
/* a double operand rounded to float first); +, -, *, / work between Ts and */
/* doubles, and zsin, zcos, zexp, zlog and zsqrt are provided for all four. */
/* All four are compiled, so the source is generic over T; helpers are      */
/* ZEUS_FN too and data may sit in namespace-scope constexpr arrays.        */
/* Without a term structure the kernels evaluate the whole function: a      */
/* value is one call, lane j of a start computes df/dx_j by one call on     */
/* dual numbers seeded with e_j (Alg. 5 as written), and a line-search      */
/* round tries one step length per lane (one block per start above dim 64:  */
/* a trial per lane).  Built in FP64 and in mixed precision: BFGS up to dim */
/* 208 (H in registers, and above dim 128 in registers and LDS), L-BFGS     */
/* (lbfgs_m > 0, a lane then owns up to four coordinates) up to dim 256.    */
/* ------------------------------------------------------------------------ */
typedef struct zeus_user_objective zeus_user_objective;

/* Compiles `source` (NUL-terminated) for the context's device and loads its
 * kernels.  *out receives the handle (owned by the caller, released with
 * zeus_objective_destroy; valid while the context lives).  ZEUS_EINVAL with
 * the compiler's messages in zeus_last_error() when the source does not
 * compile; ZEUS_EHIP when loading fails. */
zeus_err zeus_objective_compile(zeus_context *ctx, const char *source, zeus_user_objective **out);

/* Compiles `source` for gfx950 without loading it (no device needed): the
 * same checks as zeus_objective_compile, for validating a source. */
zeus_err zeus_objective_check(const char *source);

zeus_err zeus_objective_destroy(zeus_user_objective *obj);

/* Blocking solve of n >= 1 problems of the user objective `obj`, as
 * zeus_minimize_batch: every problem has objective ZEUS_USER (else
 * ZEUS_EINVAL), precision ZEUS_FP64 or ZEUS_MIXED, and dim <= 208 with
 * lbfgs_m 0 or dim <= 256 with lbfgs_m 1..8 (else ZEUS_EUNSUPPORTED);
 * required_converged works as for zeus_minimize.  The other entry points
 * refuse ZEUS_USER. */
zeus_err zeus_minimize_user(zeus_context *ctx, const zeus_user_objective *obj,
                            const zeus_problem *problems, int32_t n, const zeus_result *outs);

#ifdef __cplusplus
}
#endif
#endif /* ZEUS_H */
