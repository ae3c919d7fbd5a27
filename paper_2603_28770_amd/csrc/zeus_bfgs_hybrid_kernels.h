// zeus_bfgs_hybrid_kernels.h -- the BFGS phase for 128 < d <= 208 with the
// inverse Hessian on chip, in registers and LDS (Alg. 4 / Alg. 10 with the
// dual-number gradient of Alg. 5 and the Armijo search of Alg. 6): one block
// of eight wavefronts per start.  Built into the library
// (zeus_bfgs_hybrid.hip) and into the run-time program of a user objective.
//
//  * H is 208 x 208 (zero-padded past the dimension, ones on the padded
//    diagonal).  Rows and columns 0 .. 191 form a 3 x 3 grid of 64 x 64
//    tiles; eight of them sit in the registers of the eight wavefronts, in
//    the 4 x 16 lane tiles of the narrow kernel's 64-lane groups (zeus_group.h
//    Tile).  The rest -- the ninth tile (rows and columns 128 .. 191), the
//    column strip (rows 0 .. 191, columns 192 .. 207) and the row strip (rows
//    192 .. 207, all columns) -- is held in LDS as chains of 16 consecutive
//    columns of one row, 656 chains, element k of chain q at hl[k][q] so that
//    the lanes of a wavefront read consecutive addresses; lane t owns chain t
//    and lanes 0 .. 143 chain t + 512 as well;
//  * a row's product with a vector is a fused multiply-add chain over each
//    block of 16 consecutive columns, the block sums added pairwise over the
//    13 blocks (the order of every other kernel): a register tile's four
//    blocks meet in two lane-swap levels, the LDS chains are summed one per
//    lane, and lane i < 208 adds row i's pieces in the tree's order;
//  * chains that lie wholly in the padding are skipped: their products are
//    exact zeros and the update leaves them as they are;
//  * lanes 0 .. 207 own the coordinates (x, g, p, s, y); the vectors the
//    tiles and chains read go through LDS in the padded layout, written
//    before a reduction whose barrier publishes them;
//  * gradient, sums, line search (eight trials per round, one per wavefront),
//    termination and retirement are those of the other block kernels
//    (zeus_block.h), over 256 term slots;
//  * starts are claimed as by the other kernels: first the block's own index,
//    then an agent-scope work counter.
// The control flow is uniform across the block (one start per block), so
// every barrier is reached by all its threads.  One block fills a CU's LDS.
#pragma once

#include "zeus_block.h"

namespace zeus {
namespace {

constexpr int kHD = kHybridDim;            // rows and columns of the padded H
constexpr int kHW = 8;                     // wavefronts per start
constexpr int kHLanes = 64 * kHW;          // lanes per start
constexpr int kHB = kHD / 16;              // column blocks
constexpr int kHReg = 192;                 // rows and columns of the 3 x 3 tile grid
constexpr int kQT = 256;                   // chains of tile (2, 2): rows 128..191, blocks 8..11
constexpr int kQC = kHReg;                 // column strip: rows 0..191, block 12
constexpr int kQR = 16 * kHB;              // row strip: rows 192..207, blocks 0..12
constexpr int kQ = kQT + kQC + kQR;        // chains in LDS
constexpr int kHVec = tile_vec_len(256);   // doubles of a padded operand vector (vpos<256>)
constexpr int kHSlots = 256;               // term slots of a line-search trial
static_assert(kHD == kHReg + 16 && kHB == 13, "one 16-wide strip past the tile grid");

struct HybridShm {
  double xs[kHSlots];            // iterate under evaluation (x, then x_new), zero past d
  double ps[kHSlots];            // search direction
  double vs[kHVec];              // y, operand of u = H y, padded layout
  double gs[kHVec];              // g, operand of p = -H g, padded layout
  double ss[kHVec];              // s = x_new - x, padded layout
  double us[kHVec];              // u = H y, padded layout
  double tpart[kHW][64];         // each wavefront's products over its register tile
  double cpart[kQ];              // the chains' products
  double red[2][3][kHW];         // [phase][sum][wave] partial sums
  double tsum[2 * kHW][kMaxSums];     // [phase * waves + wave][sum] line-search trials' term sums
  double al[kTabTrials];
  int pass[2][kHW];              // [phase][wave] line-search outcome
  StartCounts cnt;               // update skips and direction resets (thread 0)
  int pad_hl[2];                 // places hl (below)
  unsigned long long got;
  int bound;                     // early-stop bound of this iteration
  ReqHot q;
  // last: the fields above stay within reach of the 16-bit offsets of LDS
  // instructions from one base, which keeps their addresses out of registers
  double hl[16][kQ];             // the LDS part of H, element k of chain q at hl[k][q]
};
// The chain array 8 bytes past a 16-byte boundary: 16-byte aligned, the
// d = 200 solve took 2% longer (230.4 against 225.7 ms).
static_assert(__builtin_offsetof(HybridShm, hl) % 16 == 8, "the chain array's placement in LDS");

// Row and column block of chain q.
__device__ __forceinline__ int chain_row(int q) {
  return q < kQT ? 128 + (q & 63) : q < kQT + kQC ? q - kQT : kHReg + ((q - kQT - kQC) & 15);
}
__device__ __forceinline__ int chain_block(int q) {
  return q < kQT ? 8 + (q >> 6) : q < kQT + kQC ? kHB - 1 : (q - kQT - kQC) >> 4;
}

// The chains of lane t: t and t + 512, so lanes 0 .. 143 hold two.  The
// wavefronts with the extra chains are the block's first ones: issue favours
// a SIMD's older wavefronts, so there the longer path between two barriers is
// served first.  Given instead to the wavefronts without gradient work (lanes
// 256 .. 399) the same chains made the d = 200 solve 12% slower.
// (A loop, not unrolled: two inlined copies of a chain's work would keep
// both chains' loads in flight and spill.)
template <class F>
__device__ __forceinline__ void for_lane_chains(int t, F &&f) {
#pragma unroll 1
  for (int q = t; q < kQ; q += kHLanes) f(q);
}

// A chain with no row or no column below the dimension lies in the padding.
__device__ __forceinline__ bool chain_live(int q, int d) {
  return chain_row(q) < d && 16 * chain_block(q) < d;
}

// Identity entries of the LDS part (all chains).
__device__ __forceinline__ void chains_identity(HybridShm &sh, int t) {
  for_lane_chains(t, [&](int q) {
    const int r = chain_row(q), c0 = 16 * chain_block(q);
#pragma unroll
    for (int k = 0; k < 16; ++k) sh.hl[k][q] = r == c0 + k ? 1.0 : 0.0;
  });
}

// Row i of H v (lane i < kHD) from the register tiles' products (tpart) and
// the chains' (cpart): the pairwise tree over the 13 blocks,
// ((b0..b3 + b4..b7) + (b8..b11 + b12)).
__device__ __forceinline__ double hybrid_row(const HybridShm &sh, int i) {
  if (i < kHReg) {
    const int a = i >> 6, l = i & 63;
    const double t0 = sh.tpart[3 * a][l], t1 = sh.tpart[3 * a + 1][l];
    const double t2 = a < 2 ? sh.tpart[3 * a + 2][l]
                            : (sh.cpart[l] + sh.cpart[64 + l]) + (sh.cpart[128 + l] + sh.cpart[192 + l]);
    return (t0 + t1) + (t2 + sh.cpart[kQT + i]);
  }
  const double *c = sh.cpart + kQT + kQC + (i - kHReg);  // block b at c[16 b]
  const double lo = ((c[0] + c[16]) + (c[32] + c[48])) + ((c[64] + c[80]) + (c[96] + c[112]));
  const double hi = ((c[128] + c[144]) + (c[160] + c[176])) + c[192];
  return lo + hi;
}

// H v for the padded vector vec (in LDS): every lane forms its register
// tile's products and its chains' products, then lane i < kHD returns row i
// (other lanes 0).
__device__ __forceinline__ double hybrid_matvec(const Tile<64> &H, const double *vec, HybridShm &sh,
                                                int t, int lane, int w, int c0, int d) {
  sh.tpart[w][lane] = H.matvec_bcast(vec[vpos<256>(c0 + lane)]);
  for_lane_chains(t, [&](int q) {
    double acc = 0.0;
    if (chain_live(q, d)) {
      const double *v = vec + vpos<256>(16 * chain_block(q));  // 16 consecutive entries
      // four columns at a time: a memory clobber between chunks keeps the
      // next chunk's loads from being hoisted, which bounds the live registers
#pragma unroll
      for (int k0 = 0; k0 < 16; k0 += 4) {
        if (k0 > 0) asm volatile("" ::: "memory");
#pragma unroll
        for (int k = k0; k < k0 + 4; ++k) acc = __builtin_fma(sh.hl[k][q], v[k], acc);
      }
    }
    sh.cpart[q] = acc;
  });
  __syncthreads();
  return t < kHD ? hybrid_row(sh, t) : 0.0;
}

// The rank-2 update of the chains (the register tiles update themselves):
// element (r, c) by fma(e_r, s_c, fma(a_r, u_c, H_rc)), a_r = -rho s_r,
// e_r = beta s_r - rho u_r; a chain whose coefficients are not finite gets
// its padding back.
__device__ __forceinline__ void chains_rank2(HybridShm &sh, int t, int d, double rho, double beta) {
  for_lane_chains(t, [&](int q) {
    if (!chain_live(q, d)) return;
    const int r = chain_row(q), c0 = 16 * chain_block(q);
    const double sr = sh.ss[vpos<256>(r)], ur = sh.us[vpos<256>(r)];
    const double a = -rho * sr;
    const double e = beta * sr - rho * ur;
    const double *uc = sh.us + vpos<256>(c0), *sc = sh.ss + vpos<256>(c0);
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
      if (k0 > 0) asm volatile("" ::: "memory");
#pragma unroll
      for (int k = k0; k < k0 + 4; ++k)
        sh.hl[k][q] = __builtin_fma(e, sc[k], __builtin_fma(a, uc[k], sh.hl[k][q]));
    }
    if (!(__builtin_isfinite(a) && __builtin_isfinite(e)))
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (c0 + k >= d) sh.hl[k][q] = r == c0 + k ? 1.0 : 0.0;
  });
}

// See the narrow kernel for the mixed-precision rules (T = float).
template <int OBJ, class T>
__global__ __launch_bounds__(kHLanes) __attribute__((amdgpu_waves_per_eu(2)))
void bfgs_hybrid_kernel(const ReqDev *reqs, int nreq, BatchDev *hdr, int64_t total) {
  constexpr bool kMixed = sizeof(T) != sizeof(double);
  __shared__ HybridShm sh;
  const int j = threadIdx.x;  // coordinate of lanes below kHD
  const int lane = j & 63, w = j >> 6;
  const int r0 = 64 * (w / 3), c0 = 64 * (w % 3);  // this wavefront's register tile
  const bool coord = j < kHD;
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
      fill_step_lengths(sh.al, rq.shrink, j, kHLanes);
      own = j < d0;
      xj = own ? rq.ws.x[idx * d0 + j] : 0.0;  // x <- swarm[i]
      if (coord) sh.xs[j] = xj;
      chains_identity(sh, j);  // H <- I (the register tiles before the first product)
      k = 0;
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
    const double yj = gn - gj;  // zero beyond the dimension and on lanes >= kHD
    if (coord) {
      sh.vs[vpos<256>(j)] = yj;
      sh.gs[vpos<256>(j)] = gn;
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
        double uj = hybrid_matvec(H, sh.vs, sh, j, lane, w, c0, d);
        uj = own ? uj : 0.0;
        if (coord) {  // published by the barrier of the next reduction
          sh.us[vpos<256>(j)] = uj;
          sh.ss[vpos<256>(j)] = sj;
        }
        const double yu = block_tree_sum(yj * uj, sh, phase);
        const double beta = (rho * rho) * yu + rho;
        // H+ = H - rho (s u' + u s') + beta s s'   (u = H y); inf * 0 would
        // have reached the padding when a coefficient is not finite
        if (!H.rank2_bcast(rho, beta, sh.us + vpos<256>(r0), sh.ss + vpos<256>(r0),
                           sh.us[vpos<256>(c0 + lane)], sh.ss[vpos<256>(c0 + lane)], lane, 0.0, 0.0))
          H.restore_padding_at(lane, d, r0, c0);
        chains_rank2(sh, j, d, rho, beta);
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
    // The register tiles are the identity until the first update (k = 0);
    // setting them here rather than at the claim keeps the old tile's
    // registers from being live beside the new one's.
    if (k == 0) H.identity_at(lane, r0, c0);
    const double hg = hybrid_matvec(H, sh.gs, sh, j, lane, w, c0, d);
    pj = own ? -hg : 0.0;
    if (coord) sh.ps[j] = pj;  // published by the barrier of the next reduction
    double ddir = block_tree_sum(gj * pj, sh, phase);
    if (!(ddir < 0.0)) {
      if (j == 0) ++sh.cnt.resets;
      H.identity_at(lane, r0, c0);
      chains_identity(sh, j);
      pj = own ? -gj : 0.0;
      if (coord) sh.ps[j] = pj;
      ddir = block_tree_sum(gj * pj, sh, phase);
    }

    // -- Armijo backtracking (Alg. 6) ---------------------------------------
    int taken;
    if (hi) {
      taken = block_armijo<OBJ, double, kHSlots>(sh, f, ddir, lsphase, &acc);
    } else {
      taken = block_armijo<OBJ, T, kHSlots>(sh, f, ddir, lsphase, &acc);
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
