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
  w.iter_ls = rq.iter_ls;
  w.trace_len = rq.trace ? rq.trace_len : 0;
  w.ri = ri;
  w.armijo_c = rq.armijo_c;
  w.tol = rq.tol;
  w.shrink = rq.shrink;
}

}  // namespace zeus
