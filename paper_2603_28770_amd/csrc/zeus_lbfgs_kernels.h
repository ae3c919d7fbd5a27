// zeus_lbfgs_kernels.h -- limited-memory BFGS kernel template for gfx950: the BFGS run of Alg. 4 /
// Alg. 10 with the dual-number gradient of Alg. 5 and the Armijo search of
// Alg. 6, but the search direction comes from the m most recent (s, y) pairs
// by the two-loop recursion (Nocedal and Wright, "Numerical Optimization",
// 2nd ed., Alg. 7.4; H0 = gamma I with gamma = s'y / y'y of the newest pair,
// their eq. 7.20), the remedy the paper names for the O(d^2) update.
//
// Mapping: one group of G lanes per start (G a power of two <= 64, so a group
// never spans two wavefronts); lane j owns coordinates j, j + G, ..., j +
// (CPL-1) G, so a single wavefront covers up to 256 coordinates.  Each lane
// keeps its coordinates of the stored pairs in registers (2 m CPL doubles);
// there is no d x d matrix anywhere.  Sums over coordinates are the pairwise
// trees used everywhere (a lane butterfly per block of G slots, then the CPL
// block sums pairwise).  The claim loop, termination, mixed precision and
// retirement follow the BFGS kernel.
#pragma once

#include "zeus_bfgs_common.h"

namespace zeus {
namespace {

constexpr int kHist = kLbfgsMaxHistory;  // pairs kept in registers (m <= kHist)

// Per-group LDS slice: the point under evaluation and the search direction
// (the line search reads both in full), the step lengths, the accepted
// trial's term sums, the start's counts and the request.
__device__ __host__ __forceinline__ constexpr int lbfgs_stride(int slots) {
  return 2 * slots + kTabTrials + kMaxSums + 1 + kHotDoubles;
}

// sum over the group's G * CPL coordinate slots of a[c] b[c] (pairwise).
//
// With 64 lanes and several blocks the blocks' butterflies share their two
// lane-swap levels: after the levels within 16 lanes, the 16-lane swap leaves
// block 0's 32-lane partial in the lower half of each 32 lanes and block 1's
// in the upper half (blocks 2 and 3 likewise), and the 32-lane swap finishes
// one block per 16 lanes (four blocks) or per half (two).  Two (or one) more
// swaps then add the block sums as (S0 + S1) + (S2 + S3).  Every addition has
// the operands it has in the separate butterflies followed by the register
// tree, so the bits agree; each lane pays one swap level per value instead of
// one per block.
template <int G, int CPL>
__device__ __forceinline__ double slot_dot(const double (&a)[CPL], const double (&b)[CPL]) {
  if constexpr (G == 64 && CPL == 4) {
    double v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = lane_tree_sum<16, double>(a[c] * b[c]);
    const double q0 = half_pair_sum<16>(v[0], v[1]);
    const double q1 = half_pair_sum<16>(v[2], v[3]);
    const double s = half_pair_sum<32>(q0, q1);  // S0, S1, S2, S3 by 16 lanes
    const double p = half_pair_sum<16>(s, s);    // S0 + S1 in lanes 0-31, S2 + S3 above
    return half_pair_sum<32>(p, p);
  } else if constexpr (G == 64 && CPL == 2) {
    const double v0 = lane_tree_sum<16, double>(a[0] * b[0]);
    const double v1 = lane_tree_sum<16, double>(a[1] * b[1]);
    const double q = half_pair_sum<16>(v0, v1);
    const double s = half_pair_sum<32>(q, q);  // S0 in lanes 0-15 and 32-47, S1 in the others
    return half_pair_sum<16>(s, s);
  } else {
    double blk[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) blk[c] = lane_tree_sum<G, double>(a[c] * b[c]);
    return reg_tree_sum<CPL, double>(blk);
  }
}

// Value and gradient at xs in number type T for coordinates j + G c (see
// group_value_grad: the same per-coordinate dual terms, the value summed over
// all G * CPL term slots).
//
// known, when given (the same pointer on every lane of the group), holds in
// the group's LDS the term sums of the line-search trial that produced xs
// (armijo_search): the same terms at the same point in the same number type
// over the same pairwise tree of G * CPL slots, so they are the sums this
// evaluation would form, and the value's butterflies are skipped (d = 200,
// m = 8: 40.6 -> 39.5 ms).  In the BFGS lane-group kernel the same reuse saved
// no time: there the value's butterfly overlaps other work.
template <int OBJ, int G, int CPL, class T>
__device__ __forceinline__ double value_grad_slots(const GroupLanes<G> &L, int d, const double *xs,
                                                   double (&gj)[CPL], const double *known = nullptr) {
  using E = Elem<OBJ>;
  if constexpr (whole_form<E>::value) {
    // Alg. 5 as written: for each of its coordinates the lane evaluates the
    // function once on dual numbers seeded with that coordinate's e_j
    double fv = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int jj = L.j + G * c;
      double g;
      fv = E::template value_grad<T>(xs, d, jj < d ? jj : -1, &g);
      gj[c] = jj < d ? g : 0.0;
    }
    return fv;
  } else {
  static_assert(E::W <= 2, "the tangent sum assumes at most two terms per coordinate");
  const int m = E::terms(d);
  T val[E::K][CPL], tan[E::K][CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int jj = L.j + G * c;
#pragma unroll
    for (int k = 0; k < E::K; ++k) {
      tan[k][c] = T(0);
      val[k][c] = T(0);
    }
    // evaluated on every lane (indices clamped), a missing term contributing
    // an exact zero, so the loads are not behind branches
#pragma unroll
    for (int back = E::W - 1; back >= 0; --back) {
      const int i = jj - back;
      const bool valid = jj < d && i >= 0 && i < m;
      dual<T> w[E::W], out[E::K];
#pragma unroll
      for (int q = 0; q < E::W; ++q) {
        int iq = i + q < 0 ? 0 : i + q;
        iq = iq < G * CPL ? iq : G * CPL - 1;
        w[q] = dual<T>{(T)xs[iq], q == back ? T(1) : T(0)};
      }
      E::template term<dual<T>>(w, out);
#pragma unroll
      for (int k = 0; k < E::K; ++k) tan[k][c] = tan[k][c] + (valid ? out[k].t : T(0));
      if (back == 0)
#pragma unroll
        for (int k = 0; k < E::K; ++k) val[k][c] = valid ? out[k].v : T(0);
    }
  }
  T sv[E::K];
  if (known) {
#pragma unroll
    for (int k = 0; k < E::K; ++k) sv[k] = (T)known[k];
  } else {
#pragma unroll
    for (int k = 0; k < E::K; ++k) {
      T blk[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) blk[c] = lane_tree_sum<G, T>(val[k][c]);
      sv[k] = reg_tree_sum<CPL, T>(blk);
    }
  }
  double fv = 0.0;
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    dual<T> sd[E::K];
#pragma unroll
    for (int k = 0; k < E::K; ++k) sd[k] = dual<T>{sv[k], tan[k][c]};
    const dual<T> r = E::template outer<dual<T>>(d, sd);
    gj[c] = (L.j + G * c < d) ? (double)r.t : 0.0;
    fv = (double)r.v;
  }
  return fv;
  }
}

template <int OBJ, int G, int CPL, class T>
__device__ __forceinline__ double value_slots(const GroupLanes<G> &L, int d, const double *xs) {
  return group_value_slots<OBJ, G, CPL, T>(L, d, xs);
}

// Two waves per SIMD for the 4-coordinate kernels of the polynomial
// objectives, which then fit 256 registers without spilling (the
// transcendental ones would spill over a hundred and stay at one wave, and
// user code is of unknown size).
template <int OBJ, int CPL>
constexpr int kLbfgsWaves =
    CPL == 4 && OBJ != kRastrigin && OBJ != kAckley && OBJ != kUser ? 2 : 1;

template <int OBJ, int G, int CPL, class T>
__global__ __launch_bounds__(kBfgsBlock) __attribute__((amdgpu_waves_per_eu(kLbfgsWaves<OBJ, CPL>)))
void lbfgs_kernel(const ReqDev *reqs, int nreq, BatchDev *hdr, int64_t total) {
  constexpr bool kMixed = sizeof(T) != sizeof(double);
  constexpr int S = 64 / G;  // groups per wave
  constexpr int SLOTS = G * CPL;
  extern __shared__ double smem[];
  const GroupLanes<G> L;
  const int j = L.j;
  double *xs, *ps, *al, *acc;
  StartCounts *cnt;  // the start's pair skips and direction resets (lane 0)
  ReqHot *qh;
  {
    double *base = smem + (size_t)((threadIdx.x >> 6) * S + L.grp) * lbfgs_stride(SLOTS);
    xs = base;
    ps = base + SLOTS;
    al = base + 2 * SLOTS;
    acc = al + kTabTrials;
    cnt = reinterpret_cast<StartCounts *>(acc + kMaxSums);
    qh = reinterpret_cast<ReqHot *>(acc + kMaxSums + 1);
  }

  bool own[CPL];
  double xj[CPL], gj[CPL], pj[CPL], sj[CPL];
  double hs[kHist][CPL], hy[kHist][CPL], hrho[kHist];  // pairs, oldest first
  int count = 0;                                         // pairs stored
  double f = 0.0;
  int64_t idx = -1;
  int k = 0, ls_trials = 0;
  bool fresh = false, first = true;
  bool hi = !kMixed;
#pragma unroll
  for (int c = 0; c < CPL; ++c) own[c] = false, xj[c] = gj[c] = pj[c] = sj[c] = 0.0;
  const int es_pass = es_pass_of(hdr);
  int claims = 0;  // starts claimed after the first (second early-stop pass)
  int cur_ri = -1;  // the request whose scalars and step lengths the group's LDS holds
  bool have_acc = false;  // acc holds the term sums at xs (value_grad_slots)

  for (;;) {
    // -- claim a start when idle (as the BFGS kernel) -----------------------
    if (idx < 0) {
      const unsigned long long groups = (unsigned long long)gridDim.x * (kBfgsBlock / G);
      const unsigned long long self =
          (unsigned long long)blockIdx.x * (kBfgsBlock / G) + (threadIdx.x >> 6) * S + L.grp;
      unsigned long long got = 0;
      if (first) {
        got = self;
        first = false;
      } else if (es_pass == 2) {
        got = strided_claim(self, groups, ++claims);
      } else {
        if (j == 0) got = groups + atomicAdd((unsigned long long *)&hdr->queue, 1ull);
        got = __shfl(got, L.grp * G, 64);
      }
      if (got >= (unsigned long long)total) break;
      const int ri = request_of(reqs, nreq, (int64_t)got);
      const ReqDev &rq = reqs[ri];
      idx = (int64_t)got - rq.start_offset + rq.slice_first;
      if (es_pass == 2 && !es_rerun(rq, idx)) {  // keeps its first-pass result
        idx = -1;
        continue;
      }
      const int d0 = rq.d;
      if (ri != cur_ri) {  // the LDS slice still holds the previous start's request
        if (j == 0) load_hot<OBJ>(*qh, rq, ri, es_pass);
        fill_step_lengths(al, rq.shrink, j, G);
        cur_ri = ri;
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int jj = j + G * c;
        own[c] = jj < d0;
        xj[c] = own[c] ? rq.ws.x[idx * d0 + jj] : 0.0;  // x <- swarm[i]
        xs[jj] = xj[c];
      }
      if (j == 0) *cnt = StartCounts{0, 0};
      count = 0;
      k = 0;
      ls_trials = 0;
      fresh = true;
      hi = !kMixed;
    }
    wave_sync();
    const ReqHot &q = *qh;
    const int d = q.d;
    // the group's stopping bound, read early (its use is at the termination
    // test) and taken from one lane: the bound falls while the kernel runs
    const int bound = __shfl(es_bound(q), L.grp * G, 64);

    // -- value and gradient at xs ---------------------------------------------
    double gn[CPL];
    double fn;
    if (hi)
      fn = value_grad_slots<OBJ, G, CPL, double>(L, d, xs, gn, have_acc ? acc : nullptr);
    else
      fn = value_grad_slots<OBJ, G, CPL, T>(L, d, xs, gn, have_acc ? acc : nullptr);
    have_acc = false;

    // -- after a step: keep (s, y) when y's > 0, dropping the oldest pair ----
    if (!fresh) {
      double yj[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) yj[c] = gn[c] - gj[c];
      const double sy = slot_dot<G, CPL>(yj, sj);
      if (sy > 0.0) {
        const int m = q.m_hist;
        if (count == m) {  // full: shift the pairs one place towards the front
#pragma unroll
          for (int i = 0; i + 1 < kHist; ++i)
            if (i + 1 < m) {
#pragma unroll
              for (int c = 0; c < CPL; ++c) {
                hs[i][c] = hs[i + 1][c];
                hy[i][c] = hy[i + 1][c];
              }
              hrho[i] = hrho[i + 1];
            }
          --count;
        }
        const double rho = 1.0 / sy;
#pragma unroll
        for (int i = 0; i < kHist; ++i)
          if (i == count) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
              hs[i][c] = sj[c];
              hy[i][c] = yj[c];
            }
            hrho[i] = rho;
          }
        ++count;
      } else if (j == 0) {
        ++cnt->skips;
      }
      ++k;
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) gj[c] = gn[c];
    f = fn;
    fresh = false;
    if (q.trace_len && k < q.trace_len)
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        if (own[c]) reqs[q.ri].trace[(idx * q.trace_len + k) * d + j + G * c] = xj[c];

    // -- termination -------------------------------------------------------------
    bool bad = !__builtin_isfinite(f);
#pragma unroll
    for (int c = 0; c < CPL; ++c) bad = bad || (own[c] && !__builtin_isfinite(gj[c]));
    const bool any_bad = L.ballot(bad) != 0ull;
    const double gg = slot_dot<G, CPL>(gj, gj);
    if (kMixed && !hi && (any_bad || norm_below(gg, 10.0 * q.tol))) {
      hi = true;  // escalate: re-evaluate this point in FP64
      fresh = true;
      continue;
    }
    int status = -1;
    if (any_bad)
      status = ZEUS_ST_NONFINITE;
    else if (norm_below(gg, q.tol))
      status = ZEUS_ST_CONVERGED;
    else
      status = budget_status(q, k, bound);
    if (status >= 0) {
      const ReqDev &rq = reqs[q.ri];
      const int tl = q.trace_len;
      if (status == ZEUS_ST_CONVERGED && q.es && j == 0) es_converged(q.es, k, q.iter_bfgs, q.es_c);
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        if (own[c]) rq.out_x[idx * d + j + G * c] = xj[c];
      if (kMixed && !hi) f = value_slots<OBJ, G, CPL, double>(L, d, xs);
      if (j == 0) {
        rq.out_f[idx] = f;
        rq.out_iters[idx] = k;
        rq.out_status[idx] = status;
        if (rq.out_ls) rq.out_ls[idx] = ls_trials;
        if (rq.out_skips) rq.out_skips[idx] = cnt->skips;
        if (rq.out_resets) rq.out_resets[idx] = cnt->resets;
      }
      if (tl)
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          if (own[c])
            for (int kk = k + 1; kk < tl; ++kk)
              rq.trace[(idx * tl + kk) * d + j + G * c] = __builtin_nan("");
      idx = -1;
      continue;
    }

    // -- search direction: two-loop recursion over the stored pairs -------------
    double qv[CPL], alpha[kHist];
#pragma unroll
    for (int c = 0; c < CPL; ++c) qv[c] = gj[c];
#pragma unroll
    for (int i = kHist - 1; i >= 0; --i) {
      alpha[i] = 0.0;
      if (i < count) {  // newest pair first: alpha_i = rho_i s_i'q, q <- q - alpha_i y_i
        alpha[i] = hrho[i] * slot_dot<G, CPL>(hs[i], qv);
#pragma unroll
        for (int c = 0; c < CPL; ++c) qv[c] = __builtin_fma(-alpha[i], hy[i][c], qv[c]);
      }
    }
    if (count > 0) {  // r = gamma q, gamma = s'y / y'y of the newest pair
      double sn[CPL], yn[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) sn[c] = yn[c] = 0.0;
#pragma unroll
      for (int i = 0; i < kHist; ++i)
        if (i == count - 1)
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            sn[c] = hs[i][c];
            yn[c] = hy[i][c];
          }
      const double gamma = slot_dot<G, CPL>(sn, yn) / slot_dot<G, CPL>(yn, yn);
#pragma unroll
      for (int c = 0; c < CPL; ++c) qv[c] = gamma * qv[c];
    }
#pragma unroll
    for (int i = 0; i < kHist; ++i)
      if (i < count) {  // oldest pair first: beta = rho_i y_i'r, r <- r + (alpha_i - beta) s_i
        const double beta = hrho[i] * slot_dot<G, CPL>(hy[i], qv);
#pragma unroll
        for (int c = 0; c < CPL; ++c) qv[c] = __builtin_fma(alpha[i] - beta, hs[i][c], qv[c]);
      }
#pragma unroll
    for (int c = 0; c < CPL; ++c) pj[c] = own[c] ? -qv[c] : 0.0;
    double ddir = slot_dot<G, CPL>(gj, pj);
    if (!(ddir < 0.0)) {  // not a descent direction: forget the pairs, p = -g
      if (j == 0) ++cnt->resets;
      count = 0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) pj[c] = own[c] ? -gj[c] : 0.0;
      ddir = slot_dot<G, CPL>(gj, pj);
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) ps[j + G * c] = pj[c];
    wave_sync();

    // -- Armijo backtracking ---------------------------------------------------
    int taken;
    if (hi) {
      taken = armijo_search<OBJ, G, SLOTS, double>(L, xs, ps, al, q, f, ddir, acc);
    } else {
      taken = armijo_search<OBJ, G, SLOTS, T>(L, xs, ps, al, q, f, ddir, acc);
      if (taken < 0) {
        ls_trials += q.iter_ls;
        hi = true;
        fresh = true;
        continue;
      }
    }
    // the accepted trial's term sums are those of the next evaluation
    have_acc = taken >= 0 && !whole_form<Elem<OBJ>>::value;
    const int nshrink = taken >= 0 ? taken : q.iter_ls;
    ls_trials += taken >= 0 ? taken + 1 : q.iter_ls;
    const double a = step_length(al, q.shrink, nshrink);

    // -- step ---------------------------------------------------------------------
    wave_sync();  // every lane has read xs and ps in the line search
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const double xnew = xj[c] + a * pj[c];
      sj[c] = own[c] ? xnew - xj[c] : 0.0;
      xj[c] = own[c] ? xnew : 0.0;
      xs[j + G * c] = xj[c];
    }
  }
}

}  // namespace
}  // namespace zeus
