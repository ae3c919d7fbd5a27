// zeus_bfgs_tile_kernels.h -- the BFGS phase for 64 < d <= 128 with the
// inverse Hessian on chip (Alg. 4 / Alg. 10 with the dual-number gradient of
// Alg. 5 and the Armijo search of Alg. 6): one block of four wavefronts per
// start.  Built into the library (zeus_bfgs_tile.hip) and into the run-time
// program of a user objective.
//
//  * H is 128 x 128 (zero-padded past the dimension, ones on the padded
//    diagonal) and split into four 64 x 64 quarters, one per wavefront:
//    wavefront w holds rows 64 (w & 1) .. + 63 and columns 64 (w >> 1) .. + 63
//    in its registers, in the 4 x 16 tiles of the narrow kernel's 64-lane
//    groups (zeus_group.h Tile), so H never leaves the chip;
//  * a row's product with a vector is a fused multiply-add chain over each
//    block of 16 consecutive columns, the block sums added pairwise: inside a
//    wavefront the four blocks of its quarter meet in two lane-swap levels,
//    then the two quarters of a row are added through LDS, which is the
//    pairwise tree over the eight blocks (the order of every other kernel);
//    lane i of wavefronts w and w + 2 both end with row 64 (w & 1) + i;
//  * lanes 0 .. 127 own the coordinates (x, g, p, s, y); the vectors the
//    tiles read (y, g, u, s) go through LDS in the padded layout, written
//    before a reduction whose barrier publishes them (six barriers per
//    iteration with an update, plus one per line-search round: the value at
//    a new iterate takes the accepted trial's term sums, block_eval);
//  * gradient, sums, line search (four trials per round, one per wavefront),
//    termination and retirement are those of the device-memory block kernel
//    (zeus_block.h), with the term slots cut to 128;
//  * starts are claimed as by the other kernels: first the block's own index,
//    then an agent-scope work counter.
// The control flow is uniform across the block (one start per block), so
// every barrier is reached by all its threads.
#pragma once

#include "zeus_block.h"

namespace zeus {
namespace {

constexpr int kTDim = kTileBlockDim;            // rows and columns of the padded H
constexpr int kQuarter = 64;                    // rows and columns of a wavefront's part
constexpr int kTVec = tile_vec_len(kTDim);      // doubles of a padded operand vector
static_assert(kTDim == 2 * kQuarter, "four wavefronts hold two by two quarters");

struct TileShm {
  double xs[kTDim];  // iterate under evaluation (x, then x_new), zero past d
  double ps[kTDim];  // search direction
  double vs[kTVec];  // y, operand of u = H y, padded layout
  double gs[kTVec];  // g, operand of p = -H g, padded layout
  double ss[kTVec];  // s = x_new - x, padded layout
  double us[kTVec];  // u = H y, padded layout
  double part[kBlockWaves][kQuarter];  // each wavefront's products over its quarter
  double red[2][3][kBlockWaves];       // [phase][sum][wave] partial sums
  double tsum[2 * kBlockWaves][kMaxSums];   // [phase * waves + wave][sum] line-search trials' term sums
  double al[kTabTrials];
  int pass[2][kBlockWaves];            // [phase][wave] line-search outcome
  StartCounts cnt;                     // update skips and direction resets (thread 0)
  unsigned long long got;
  int bound;                           // early-stop bound of this iteration
  ReqHot q;
};

// Row products of H with the padded vector v (in LDS): lane i of wavefront w
// returns row 64 (w & 1) + i, its quarter's sum plus the other quarter's
// (the same bits in wavefronts w and w ^ 2: IEEE addition commutes).
__device__ __forceinline__ double tile_block_matvec(const Tile<64> &H, const double *v, TileShm &sh,
                                                    int lane, int w, int c0) {
  const double mine = H.matvec_bcast(v[vpos<kTDim>(c0 + lane)]);
  sh.part[w][lane] = mine;
  __syncthreads();
  return mine + sh.part[w ^ 2][lane];
}

// See the narrow kernel for the mixed-precision rules (T = float).
template <int OBJ, class T>
__global__ __launch_bounds__(kBlockLanes) __attribute__((amdgpu_waves_per_eu(2)))
void bfgs_tile_kernel(const ReqDev *reqs, int nreq, BatchDev *hdr, int64_t total) {
  constexpr bool kMixed = sizeof(T) != sizeof(double);
  __shared__ TileShm sh;
  const int j = threadIdx.x;  // coordinate of lanes below kTDim
  const int lane = j & 63, w = j >> 6;
  const int r0 = kQuarter * (w & 1), c0 = kQuarter * (w >> 1);  // this wavefront's quarter
  const bool coord = j < kTDim;
  const int ci = j & (kTDim - 1);  // row whose products this lane receives
  Tile<64> H;
  int phase = 0, lsphase = 0;
  int acc = -1;  // slot of sh.tsum with the accepted trial's term sums (block_armijo), or -1
  bool own = false, first = true, fresh = false, hi = !kMixed;
  double xj = 0.0, gj = 0.0, pj = 0.0, sj = 0.0, f = 0.0;
  int64_t idx = -1;
  int k = 0, ls_trials = 0;
  const int es_pass = es_pass_of(hdr);
  int claims = 0;  // starts claimed after the first (second early-stop pass; thread 0)

  for (;;) {
    if (idx < 0) {
      if (j == 0) {
        sh.got = first           ? (unsigned long long)blockIdx.x
                 : es_pass == 2 ? strided_claim(blockIdx.x, gridDim.x, ++claims)
                                : gridDim.x + atomicAdd((unsigned long long *)&hdr->queue, 1ull);
      }
      first = false;
      __syncthreads();
      const unsigned long long got = sh.got;
      if (got >= (unsigned long long)total) break;
      const int ri = request_of(reqs, nreq, (int64_t)got);
      const ReqDev &rq = reqs[ri];
      idx = (int64_t)got - rq.start_offset + rq.slice_first;
      if (es_pass == 2 && !es_rerun(rq, idx)) {  // keeps its first-pass result
        idx = -1;
        __syncthreads();  // every thread has read sh.got before the next claim writes it
        continue;
      }
      const int d0 = rq.d;
      if (j == 0) {
        load_hot<OBJ>(sh.q, rq, ri, es_pass);
        sh.cnt = StartCounts{0, 0};
      }
      fill_step_lengths(sh.al, rq.shrink, j, kBlockLanes);
      own = j < d0;
      xj = own ? rq.ws.x[idx * d0 + j] : 0.0;  // x <- swarm[i]
      if (coord) sh.xs[j] = xj;
      k = 0;  // H <- I before the first product (below)
      ls_trials = 0;
      fresh = true;
      hi = !kMixed;
    }
    // the stopping bound, read early (its use is at the termination test) by
    // one thread for the block: the bound falls while the kernel runs
    if (j == 0) sh.bound = es_bound(sh.q);
    __syncthreads();  // xs, the request and the bound are visible; earlier reads are done
    const ReqHot &q = sh.q;
    const int d = q.d;
    const int bound = sh.bound;

    // -- value and gradient at xs -------------------------------------------
    double gn, fn;
    if (hi)
      fn = block_eval<OBJ, double, true>(d, sh.xs, &gn, sh, phase, acc);
    else
      fn = block_eval<OBJ, T, true>(d, sh.xs, &gn, sh, phase, acc);
    acc = -1;

    // y's, g'g and the non-finite test in one reduction, whose barrier also
    // publishes y and g for the products below; right after a claim or an
    // escalation y's is not used
    const double yj = gn - gj;  // zero beyond the dimension and on lanes >= kTDim
    if (coord) {
      sh.vs[vpos<kTDim>(j)] = yj;
      sh.gs[vpos<kTDim>(j)] = gn;
    }
    const bool bad = (own && !__builtin_isfinite(gn)) || !__builtin_isfinite(fn);
    double sums[3] = {yj * sj, gn * gn, bad ? 1.0 : 0.0};
    block_tree_sums<3, double>(sums, sh, phase);
    const double sy = sums[0], gg = sums[1];
    const bool any_bad = sums[2] != 0.0;

    // -- after a step: u = H y and the rank-2 update --------------------------
    if (!fresh) {
      if (sy > 0.0) {  // curvature condition; skip the update otherwise
        const double rho = 1.0 / sy;
        double uj = tile_block_matvec(H, sh.vs, sh, lane, w, c0);
        uj = ci < d ? uj : 0.0;
        if (coord) {  // published by the barrier of the next reduction
          sh.us[vpos<kTDim>(j)] = uj;
          sh.ss[vpos<kTDim>(j)] = sj;
        }
        const double yu = block_tree_sum(coord ? yj * uj : 0.0, sh, phase);
        const double beta = (rho * rho) * yu + rho;
        // H+ = H - rho (s u' + u s') + beta s s'   (u = H y); inf * 0 would
        // have reached the padding when a coefficient is not finite
        if (!H.rank2_bcast(rho, beta, sh.us + vpos<kTDim>(r0), sh.ss + vpos<kTDim>(r0),
                           sh.us[vpos<kTDim>(c0 + lane)], sh.ss[vpos<kTDim>(c0 + lane)], lane, 0.0,
                           0.0))
          H.restore_padding_at(lane, d, r0, c0);
      } else if (j == 0) {
        ++sh.cnt.skips;
      }
      ++k;
    }
    gj = gn;
    f = fn;
    fresh = false;
    if (q.trace_len && own && k < q.trace_len) reqs[q.ri].trace[(idx * q.trace_len + k) * d + j] = xj;

    // -- termination: non-finite, ||g|| < Theta, budget ---------------------
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
      if (kMixed && !hi) f = block_eval<OBJ, double, false>(d, sh.xs, nullptr, sh, phase);
      if (j == 0) {
        rq.out_f[idx] = f;
        rq.out_iters[idx] = k;
        rq.out_status[idx] = status;
        if (rq.out_ls) rq.out_ls[idx] = ls_trials;
        if (rq.out_skips) rq.out_skips[idx] = sh.cnt.skips;
        if (rq.out_resets) rq.out_resets[idx] = sh.cnt.resets;
      }
      if (tl && own)
        for (int kk = k + 1; kk < tl; ++kk) rq.trace[(idx * tl + kk) * d + j] = __builtin_nan("");
      idx = -1;
      continue;
    }

    // -- search direction p = -H g (reset to -g if not a descent direction) -
    // H is the identity until the first update (k = 0).  Setting it here
    // rather than at the claim keeps the old tile's registers from being
    // live beside the new one's (the claim path rejoins the loop with H).
    if (k == 0) H.identity_at(lane, r0, c0);
    const double hg = tile_block_matvec(H, sh.gs, sh, lane, w, c0);
    pj = own ? -hg : 0.0;
    if (coord) sh.ps[j] = pj;  // published by the barrier of the next reduction
    double ddir = block_tree_sum(gj * pj, sh, phase);
    if (!(ddir < 0.0)) {
      if (j == 0) ++sh.cnt.resets;
      H.identity_at(lane, r0, c0);
      pj = own ? -gj : 0.0;
      if (coord) sh.ps[j] = pj;
      ddir = block_tree_sum(gj * pj, sh, phase);
    }

    // -- Armijo backtracking (Alg. 6) ---------------------------------------
    int taken;
    if (hi) {
      taken = block_armijo<OBJ, double, kTDim>(sh, f, ddir, lsphase, &acc);
    } else {
      taken = block_armijo<OBJ, T, kTDim>(sh, f, ddir, lsphase, &acc);
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
    // every lane has read xs and ps before the last barrier of the line search
    const double xnew = xj + alpha * pj;
    sj = own ? xnew - xj : 0.0;
    xj = own ? xnew : 0.0;
    if (coord) sh.xs[j] = xj;
  }
}

}  // namespace
}  // namespace zeus
