// zeus_bfgs_common.h -- pieces shared by the two BFGS kernels (one group of
// lanes per start, and one block per start for wide problems).
#pragma once

#include "zeus_device.h"
#include "zeus_group.h"
#include "zeus_internal.h"

namespace zeus {

// The scalars of a start's request that every iteration reads, kept in LDS
// (registers hold only the request index; output pointers are read from the
// request table when a start retires).
struct ReqHot {
  int d, m;                  // dimension, number of terms
  int iter_bfgs, iter_ls, trace_len, ri;
  int stop_status;           // status at the iteration budget
  int m_hist;                // L-BFGS pairs kept
  double armijo_c, tol, shrink;
  int32_t *es;               // early-stop state while a start may stop at its bound
  int64_t es_c;              // converged starts that stop the request
};
constexpr int kHotDoubles = (sizeof(ReqHot) + 7) / 8;

// Term sums an objective's outer function combines (Ackley has two).
constexpr int kMaxSums = 2;

// Per-start counts of two decisions of Alg. 4, kept in LDS and touched only
// by the start's first lane (no registers): steps whose rank-2 update was
// skipped because y's <= 0, and search directions reset to -g because g'p
// was not negative.
struct StartCounts {
  int32_t skips, resets;
};

// Step lengths alpha_t = shrink^t of the first kTabTrials trials, each the
// product of the previous one and shrink, as Alg. 6 forms them.
constexpr int kTabTrials = 32;

__device__ __forceinline__ double step_length(const double *al, double shrink, int t) {
  if (t < kTabTrials) return al[t];
  double alpha = al[kTabTrials - 1];
  for (int e = kTabTrials - 1; e < t; ++e) alpha = alpha * shrink;
  return alpha;
}

// Lanes lane0, lane0 + stride, ... below kTabTrials fill the table.
__device__ __forceinline__ void fill_step_lengths(double *al, double shrink, int lane0, int stride) {
  for (int t = lane0; t < kTabTrials; t += stride) {
    double a = 1.0;
    for (int e = 0; e < t; ++e) a = a * shrink;
    al[t] = a;
  }
}

// In the second early-stop pass almost every claimed start keeps its
// first-pass result, so a claim is mostly a skip and the agent-scope work
// counter would serialise the pass (one same-address atomic per start).
// There a worker (group or block) `self` of `workers` takes the starts
// self, self + workers, self + 2 workers, ... instead: the reruns are short
// and alike, so a static split balances them.  Returns the worker's n-th
// start (n >= 1) in that split.
__device__ __forceinline__ unsigned long long strided_claim(unsigned long long self,
                                                            unsigned long long workers, int n) {
  return self + (unsigned long long)n * workers;
}

// The request of a launch group that holds global start `got` (the start
// offsets of the table ascend from 0).
__device__ __forceinline__ int request_of(const ReqDev *reqs, int nreq, int64_t got) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (reqs[mid].start_offset <= got) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// sqrt(gg) < bound, the norm test of a start (gg = g'g), decided exactly as
// written but without the square root when gg >= 4 bound^2: there the root
// is at least twice the bound up to a few roundings, so the test fails.
__device__ __forceinline__ bool norm_below(double gg, double bound) {
  if (!(gg < (4.0 * bound) * bound)) return false;
  return sqrt(gg) < bound;
}

// Relaxed agent-scope access to the early-stop state: its values are only
// ever bounds (a stale bound is a larger one), so no ordering is needed.
__device__ __forceinline__ int es_load(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Smallest iteration k at which the counts of the Fenwick tree (nodes
// 1 .. n, node i for iteration i - 1) reach c convergences at iterations
// <= k, or -1 when they do not.  With counts read while they still grow the
// answer can only be too large, never too small.
__device__ __forceinline__ int es_search(const int32_t *es, int n, int64_t c) {
  const int32_t *tree = es + kEsTree;
  int step = 1;
  while (2 * step <= n) step *= 2;
  int pos = 0;
  int64_t rem = c;
  for (; step > 0; step >>= 1)
    if (pos + step <= n) {
      const int64_t t = (uint32_t)es_load(tree + pos + step);
      if (t < rem) {
        pos += step;
        rem -= t;
      }
    }
  return pos < n ? pos : -1;
}

// A start of a request with early stop has converged at iteration k (one
// lane per start): count it, and lower the stopping bound to the c-th
// smallest convergence iteration counted so far.
__device__ __forceinline__ void es_converged(int32_t *es, int k, int iter_bfgs, int64_t c) {
  const int n = iter_bfgs + 1;
  for (int i = k + 1; i <= n; i += i & -i)
    __hip_atomic_fetch_add(es + kEsTree + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int64_t cnt =
      (int64_t)(uint32_t)__hip_atomic_fetch_add(es + kEsCount, 1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT) + 1;
  if (cnt < c || k >= es_load(es + kEsBound)) return;
  const int kc = es_search(es, n, c);
  if (kc >= 0) __hip_atomic_fetch_min(es + kEsBound, kc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Early-stop pass of a launch group (BatchDev::es_pass), read once per kernel.
__device__ __forceinline__ int es_pass_of(const BatchDev *hdr) {
  return (int)__hip_atomic_load(&hdr->es_pass, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// In the second pass a claimed start reruns only if its request stops early
// and the start went past K* in the first pass; every other start keeps the
// results of the first pass.
__device__ __forceinline__ bool es_rerun(const ReqDev &rq, int64_t idx) {
  if (!rq.ws.es) return false;
  const int ks = es_load(rq.ws.es + kEsKstar);
  return ks >= 0 && rq.out_iters[idx] > ks;
}

// The request's scalars for the start a group claimed; in the second
// early-stop pass the start reruns with K* as its budget and ends STOPPED.
template <int OBJ>
__device__ __forceinline__ void load_hot(ReqHot &w, const ReqDev &rq, int ri, int es_pass) {
  w.d = rq.d;
  w.m = Elem<OBJ>::terms(rq.d);
  w.iter_bfgs = rq.iter_bfgs;
  w.stop_status = rq.stop_status;
  w.m_hist = rq.lbfgs_m;
  w.iter_ls = rq.iter_ls;
  w.trace_len = rq.trace ? rq.trace_len : 0;
  w.ri = ri;
  w.armijo_c = rq.armijo_c;
  w.tol = rq.tol;
  w.shrink = rq.shrink;
  w.es = es_pass == 1 ? rq.ws.es : nullptr;
  w.es_c = rq.required_c;
  if (es_pass == 2) {
    w.iter_bfgs = es_load(rq.ws.es + kEsKstar);
    w.stop_status = ZEUS_ST_STOPPED;
  }
}

// Status of a start at iteration k that is neither non-finite nor converged:
// the budget, else (first early-stop pass) the stopping bound read at the top
// of the iteration, else still running (-1).
__device__ __forceinline__ int budget_status(const ReqHot &q, int k, int bound) {
  if (k == q.iter_bfgs) return q.stop_status;  // MAXITER, or STOPPED in the rerun
  if (k >= bound) return ZEUS_ST_STOPPED;
  return -1;
}

// Stopping bound of the start's request for this iteration (no bound without
// early stop).
__device__ __forceinline__ int es_bound(const ReqHot &q) {
  return q.es ? es_load(q.es + kEsBound) : 0x7fffffff;
}

// Line-search trials per round: R trials of G / R lanes each.  64-lane
// groups take two (d = 50 BFGS 3-7% faster than with four, d = 200 L-BFGS
// 23%; one was slower): at 1.4 to 2.8 trials per iteration wider rounds
// mostly evaluate trials past the accepted one.  Smaller groups take four:
// two made Rastrigin at d <= 3 (many trials per iteration) up to 1.5 times
// slower at every lane count from 4 to 32, and was even at d = 10.
template <int G>
constexpr int kRound = G == 64 ? 2 : (G < 4 ? G : 4);

// One Armijo search (Alg. 6) with the objective evaluated in number type U,
// by a group of G lanes covering SLOTS term slots (SLOTS a multiple of G; the
// point is xs + alpha ps, both in LDS and zero past the dimension).  A round
// evaluates R consecutive trials of the sequence at once, each spread over
// TP = G / R lanes holding B = SLOTS / TP consecutive term slots (zero past
// the last term): a lane adds its slots pairwise and the trial's lanes finish
// the pairwise sum with a butterfly.  The first trial that passes is the step
// Alg. 6 returns.  Returns its index, or -1 when none of the iter_ls trials
// passes.  When acc (the group's LDS) is given and a trial passes, the
// trial's first lane writes its k-th term sum to acc[k] (objectives with a
// term structure); the group sees it after its next wave_sync.
template <int OBJ, int G, int SLOTS, class U>
__device__ __forceinline__ int armijo_search(const GroupLanes<G> &L, const double *xs,
                                             const double *ps, const double *al, const ReqHot &q,
                                             double f, double ddir, double *acc = nullptr) {
  using E = Elem<OBJ>;
  constexpr int R = kRound<G>, TP = G / R, B = SLOTS / TP;
  constexpr uint64_t leaders = [] {  // bit r * TP for every trial r of a round
    uint64_t b = 0;
    for (int r = 0; r < R; ++r) b |= 1ull << (r * TP);
    return b;
  }();
  if constexpr (whole_form<E>::value) {
    // one trial per lane: trials base .. base + G - 1 in a round
    for (int base = 0; base < q.iter_ls; base += G) {
      const int t = base + L.j;
      const double alpha = step_length(al, q.shrink, t);
      const double ft = E::template trial<U>(xs, ps, alpha, q.d);
      const bool ok = t < q.iter_ls && ft <= f + (q.armijo_c * alpha) * ddir;
      const uint64_t hit = L.ballot(ok);
      if (hit != 0ull) return base + (__ffsll((unsigned long long)hit) - 1);
    }
    return -1;
  } else {
  const int trial_slot = L.j / TP, c = L.j % TP;
  const int d = q.d, m = q.m;
  for (int base = 0; base < q.iter_ls; base += R) {
    const int t = base + trial_slot;
    const double alpha = step_length(al, q.shrink, t);
    // Every slot is evaluated (indices clamped into the vectors) and the
    // slots past the last term are replaced by zero afterwards: no branch
    // per slot, so the loads of a chunk of CB slots are in flight together.
    // A lane's B slots are taken CB at a time (a memory clobber between
    // chunks keeps the next chunk's loads from being hoisted, which bounds
    // the live registers); the pairwise tree over B is the tree over the
    // chunk sums.
    constexpr int CB = B < 4 ? B : 4;
    U csum[E::K][B / CB];
#pragma unroll
    for (int cb = 0; cb < B / CB; ++cb) {
      if (cb > 0) asm volatile("" ::: "memory");
      U tv[E::K][CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int i = c * B + cb * CB + b;
        U w[E::W], out[E::K];
#pragma unroll
        for (int e = 0; e < E::W; ++e) {
          const int ie = i + e < SLOTS ? i + e : SLOTS - 1;
          w[e] = (U)(xs[ie] + alpha * ps[ie]);
        }
        E::template term<U>(w, out);
#pragma unroll
        for (int kk = 0; kk < E::K; ++kk) tv[kk][b] = i < m ? out[kk] : U(0);
      }
#pragma unroll
      for (int kk = 0; kk < E::K; ++kk) csum[kk][cb] = reg_tree_sum<CB, U>(tv[kk]);
    }
    U sums[E::K];
#pragma unroll
    for (int kk = 0; kk < E::K; ++kk)
      sums[kk] = lane_tree_sum<TP, U>(reg_tree_sum<B / CB, U>(csum[kk]));
    const double ft = (double)E::template outer<U>(d, sums);
    const bool ok = t < q.iter_ls && ft <= f + (q.armijo_c * alpha) * ddir;
    const uint64_t hit = L.ballot(ok) & leaders;
    if (hit != 0ull) {
      const int r = (__ffsll((unsigned long long)hit) - 1) / TP;  // the passing trial's slot
      static_assert(E::K <= kMaxSums, "more term sums than the slots kept for them");
      if (acc && L.j == r * TP)
#pragma unroll
        for (int kk = 0; kk < E::K; ++kk) acc[kk] = (double)sums[kk];
      return base + r;
    }
  }
  return -1;
  }
}

}  // namespace zeus

