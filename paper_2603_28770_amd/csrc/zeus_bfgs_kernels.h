// zeus_bfgs_kernels.h -- the BFGS kernel template for d <= 64 on gfx950
// (Alg. 4 / Alg. 10 with the dual-number gradient of Alg. 5 and the Armijo
// line search of Alg. 6).
//
// Mapping (the finer-grained parallelism the paper defers to future work, Sec. IV):
//  * one group of G lanes (G a power of two >= dim, G <= 64) runs one start;
//    a 64-lane wavefront holds 64/G groups, a 256-thread block four waves;
//  * lane j owns coordinate j; the inverse Hessian H stays in the group's
//    registers for the whole run (H never touches HBM), in tiles of R rows by
//    16 columns (zeus_group.h Tile);
//  * gradient: lane j evaluates on dual numbers seeded with the tangent e_j,
//    so the G lanes compute the dim passes of Alg. 5 at once;
//  * line search: each round evaluates consecutive trials of the
//    backtracking sequence in parallel; the first trial that satisfies the
//    Armijo condition is exactly the step the sequential loop of Alg. 6
//    would return;
//  * the small vectors the lanes exchange (x, p, g, s, y, u) go through the
//    group's slice of LDS;
//  * each group first takes the start with its own index, then claims starts
//    from an agent-scope work counter, so a group that finishes early takes
//    the next start instead of idling; results do not depend on which group
//    ran which start.
// The loop is flattened so that every trip does one gradient evaluation and
// one line search for every group of a wave, whatever iteration each group's
// start is in.
#pragma once

#include "zeus_bfgs_common.h"

namespace zeus {
namespace {

// Per-group LDS slice: the vectors that every lane of the group reads in
// full.  Entries from the dimension on are zero.
struct GroupShm {
  double *xs;  // [G] iterate under evaluation (x, then x_new)
  double *ps;  // [G] search direction
  double *vs;  // operand of the next matrix-vector product (y, then g)
  double *ss;  // s = x_new - x
  double *us;  // u = H y  (vs, ss, us: tile_vec_len(G) doubles, padded layout)
  double *al;  // [kTabTrials] step lengths of the start's request
  ReqHot *q;   // the start's request
};

// Doubles per group slice.
__device__ __host__ __forceinline__ constexpr int group_stride(int G) {
  return 2 * G + 3 * tile_vec_len(G) + kTabTrials + kHotDoubles;
}

// T = double: every step in FP64.
// T = float (mixed precision): a start evaluates the objective, its dual
// numbers and the term sums in FP32 at the FP32-rounded point, while x, p, H,
// Hg, g'p, the Armijo comparison, s, y and y's stay FP64.  Near a minimum FP32
// can no longer resolve the Armijo decrease nor a gradient below the tolerance,
// so a start escalates to FP64 evaluation for the rest of its run, re-evaluating
// its current point, when (a) its FP32 gradient norm falls below 10 Theta,
// (b) an FP32 value or gradient is not finite, or (c) an FP32 line search finds
// no step.  Convergence and non-finite outcomes are therefore always decided
// on FP64 values; the value reported for a start is FP64 at its final x.
//
// Every reduction below runs with all lanes of the group active: the control
// flow splits only on values the whole group shares.
// Waves per SIMD the register allocation must allow.  Left to itself the
// compiler keeps the 64-lane kernels of the transcendental objectives at one
// wave (256 VGPRs plus AGPRs); asking for two costs a few dozen spilled
// registers but hides far more latency (Ackley d = 50: 1.5x faster), and
// three waves help Rastrigin's 16-lane kernel the same way.  Other kernels
// reach their occupancy without the request.
template <int OBJ, int G>
constexpr int kBfgsWaves = G == 64 ? 2 : (G == 16 && OBJ == kRastrigin) ? 3 : 1;

template <int OBJ, int G, class T>
__global__ __launch_bounds__(kBfgsBlock) __attribute__((amdgpu_waves_per_eu(kBfgsWaves<OBJ, G>)))
void bfgs_kernel(const ReqDev *reqs, int nreq,
                                                          BatchDev *hdr, int64_t total) {
  using E = Elem<OBJ>;
  constexpr bool kMixed = sizeof(T) != sizeof(double);
  constexpr int S = 64 / G;  // groups per wave
  extern __shared__ double smem[];
  const GroupLanes<G> L;
  const int j = L.j;
  GroupShm sh;
  {
    double *base = smem + (size_t)((threadIdx.x >> 6) * S + L.grp) * group_stride(G);
    sh.xs = base;
    sh.ps = base + G;
    constexpr int VL = tile_vec_len(G);
    sh.vs = base + 2 * G;
    sh.ss = sh.vs + VL;
    sh.us = sh.ss + VL;
    sh.al = sh.us + VL;
    sh.q = reinterpret_cast<ReqHot *>(sh.al + kTabTrials);
  }

  bool own = false;
  Tile<G> H;  // this lane's tile of the inverse Hessian (identity in the padding)
  double xj = 0.0, gj = 0.0, pj = 0.0, sj = 0.0, f = 0.0;
  int64_t idx = -1;
  int k = 0, ls_trials = 0;
  StartCounts cnt{0, 0};  // the start's update skips and direction resets
  bool fresh = false, first = true;
  bool hi = !kMixed;  // evaluating in FP64 (always, unless mixed precision)
  const int es_pass = es_pass_of(hdr);
  int claims = 0;  // starts claimed after the first (second early-stop pass)
  int cur_ri = -1;  // the request whose scalars and step lengths the group's LDS holds

  for (;;) {
    // -- claim a start when idle ------------------------------------------
    if (idx < 0) {
      // the first start of a group is its own index; later ones come from
      // the counter, after the starts taken that way
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
        if (j == 0) load_hot<OBJ>(*sh.q, rq, ri, es_pass);
        fill_step_lengths(sh.al, rq.shrink, j, G);
        cur_ri = ri;
      }
      own = j < d0;
      xj = own ? rq.ws.x[idx * d0 + j] : 0.0;  // x <- swarm[i]
      sh.xs[j] = xj;
      H.identity(j);  // H <- I
      cnt = StartCounts{0, 0};
      k = 0;
      ls_trials = 0;
      fresh = true;
      hi = !kMixed;
    }
    wave_sync();
    const ReqHot &q = *sh.q;
    const int d = q.d;
    // the group's stopping bound, read early (its use is at the termination
    // test) and taken from one lane: the bound falls while the kernel runs
    const int bound = __shfl(es_bound(q), L.grp * G, 64);

    // -- value and gradient at xs (dual numbers, one direction per lane) ----
    double gn, fn;
    if (hi)
      fn = group_value_grad<OBJ, G, double>(L, d, sh.xs, &gn);
    else
      fn = group_value_grad<OBJ, G, T>(L, d, sh.xs, &gn);

    // y's and g'g are formed together (independent butterflies overlap);
    // right after a claim or an escalation y's is not used
    const double yj = gn - gj;  // zero beyond the dimension
    const double sy = lane_tree_sum<G, double>(yj * sj);
    const double gg = lane_tree_sum<G, double>(gn * gn);

    // -- after a step: y and the rank-2 inverse-Hessian update --------------
    if (!fresh) {
      if (sy > 0.0) {  // curvature condition; skip the update otherwise
        const double rho = 1.0 / sy;
        // every lane: the tile sums cross lanes.  From 16 lanes on the tiles
        // take the vector by row broadcasts from the lanes' own entries.
        double uj;
        if constexpr (kTileCols<G> == 16) {
          uj = H.matvec_bcast(yj);
        } else {
          sh.vs[vpos<G>(j)] = yj;
          wave_sync();
          uj = H.matvec(sh.vs, j);
        }
        uj = own ? uj : 0.0;
        const double yu = lane_tree_sum<G, double>(yj * uj);
        if constexpr (kTileRows<G> > 1 || kTileCols<G> < 16) {  // rows of other lanes
          sh.us[vpos<G>(j)] = uj;
          sh.ss[vpos<G>(j)] = sj;
          wave_sync();
        }
        const double beta = (rho * rho) * yu + rho;
        // H+ = H - rho (s u' + u s') + beta s s'   (u = H y); inf * 0 would
        // have reached the padding when a coefficient is not finite
        bool fin;
        if constexpr (kTileCols<G> == 16)
          fin = H.rank2_bcast(rho, beta, sh.us, sh.ss, uj, sj, j, sj, uj);
        else
          fin = H.rank2(rho, beta, sh.us, sh.ss, j, sj, uj);
        if (!fin) H.restore_padding(j, d);
      } else {
        ++cnt.skips;
      }
      ++k;
    }
    gj = gn;
    f = fn;
    fresh = false;
    if (q.trace_len && own && k < q.trace_len) reqs[q.ri].trace[(idx * q.trace_len + k) * d + j] = xj;

    // -- termination: non-finite, ||g|| < Theta, budget ---------------------
    const bool bad = (own && !__builtin_isfinite(gj)) || !__builtin_isfinite(f);
    const bool any_bad = L.ballot(bad) != 0ull;
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
      if (own) rq.out_x[idx * d + j] = xj;
      if (kMixed && !hi) f = group_value<OBJ, G, double>(L, d, sh.xs);  // FP64 value at x
      if (j == 0) {
        rq.out_f[idx] = f;
        rq.out_iters[idx] = k;
        rq.out_status[idx] = status;
        if (rq.out_ls) rq.out_ls[idx] = ls_trials;
        if (rq.out_skips) rq.out_skips[idx] = cnt.skips;
        if (rq.out_resets) rq.out_resets[idx] = cnt.resets;
      }
      if (tl && own)
        for (int kk = k + 1; kk < tl; ++kk)
          rq.trace[(idx * tl + kk) * d + j] = __builtin_nan("");
      idx = -1;
      continue;
    }

    // -- search direction p = -H g (reset to -g if not a descent direction) -
    double hg;  // every lane: the tile sums cross lanes
    if constexpr (kTileCols<G> == 16) {
      hg = H.matvec_bcast(gj);
    } else {
      sh.vs[vpos<G>(j)] = gj;
      wave_sync();
      hg = H.matvec(sh.vs, j);
    }
    pj = own ? -hg : 0.0;
    double ddir = lane_tree_sum<G, double>(gj * pj);
    if (!(ddir < 0.0)) {
      H.identity(j);
      pj = own ? -gj : 0.0;
      ddir = lane_tree_sum<G, double>(gj * pj);
      ++cnt.resets;
    }
    sh.ps[j] = pj;
    wave_sync();

    // -- Armijo backtracking (Alg. 6) ---------------------------------------
    int taken;
    if (hi) {
      taken = armijo_search<OBJ, G, G, double>(L, sh.xs, sh.ps, sh.al, *sh.q, f, ddir);
    } else {
      taken = armijo_search<OBJ, G, G, T>(L, sh.xs, sh.ps, sh.al, *sh.q, f, ddir);
      if (taken < 0) {
        ls_trials += q.iter_ls;
        hi = true;  // escalate: FP32 cannot resolve this decrease
        fresh = true;
        continue;
      }
    }
    const int nshrink = taken >= 0 ? taken : q.iter_ls;
    ls_trials += taken >= 0 ? taken + 1 : q.iter_ls;
    const double alpha = step_length(sh.al, q.shrink, nshrink);

    // -- step: x_new = x + alpha p, s = x_new - x -----------------------------
    const double xnew = xj + alpha * pj;
    sj = own ? xnew - xj : 0.0;
    xj = own ? xnew : 0.0;
    wave_sync();  // every lane has read xs in the line search
    sh.xs[j] = xj;
  }
}

}  // namespace
}  // namespace zeus
