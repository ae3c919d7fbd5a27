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
};
constexpr int kHotDoubles = (sizeof(ReqHot) + 7) / 8;

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

template <int OBJ>
__device__ __forceinline__ void load_hot(ReqHot &w, const ReqDev &rq, int ri) {
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
// passes.
template <int OBJ, int G, int SLOTS, class U>
__device__ __forceinline__ int armijo_search(const GroupLanes<G> &L, const double *xs,
                                             const double *ps, const double *al, const ReqHot &q,
                                             double f, double ddir) {
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
      const double ft = E::trial(xs, ps, alpha, q.d);
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
    if (hit != 0ull) return base + (__ffsll((unsigned long long)hit) - 1) / TP;
  }
  return -1;
  }
}

}  // namespace zeus

