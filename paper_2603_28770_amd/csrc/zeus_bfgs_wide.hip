// zeus_bfgs_wide.hip -- the BFGS phase with the inverse Hessian in device
// memory (Alg. 4 / Alg. 10 with the dual-number gradient of Alg. 5 and the
// Armijo search of Alg. 6): one block of 256 lanes per start.  It runs
// 208 < d <= 256, where H no longer fits on chip, and any d > 64 when the
// tiling is forced (ZEUS_TILE_LANES=256), which the tests use to compare it
// with the on-chip kernels.
//
//  * lane i owns coordinate i and row i of the inverse Hessian H;
//  * a row of up to 256 doubles does not fit in registers, so H lives in a
//    slot of device memory owned by the block, stored column by column
//    (element (i, c) at c * CS + i, CS = the dimension rounded up to 64):
//    every pass over H reads or writes consecutive addresses across the
//    lanes.  A block keeps its slot for every start it runs;
//  * per iteration H is read once by u = H y and once more by the rank-2
//    update, which writes the new rows and forms p = -H_new g_new from them in
//    the same pass (the search direction needs no third pass);
//  * a row's product with a vector is a fused multiply-add chain over each
//    block of 16 consecutive columns, the block sums added pairwise (the
//    order of the tile layout of the narrow kernel);
//  * sums over coordinates and terms are the pairwise trees used everywhere:
//    a butterfly inside each wavefront, then the four wavefront sums added
//    pairwise through LDS;
//  * the line search evaluates four trials per round, one per wavefront;
//  * starts are claimed as by the narrow kernel: first the block's own index,
//    then an agent-scope work counter.
// The control flow is uniform across the block (one start per block), so
// every barrier is reached by all its threads.
#include "zeus_block.h"

namespace zeus {
namespace {

constexpr int kWide = kBlockLanes;   // lanes (threads) per start
constexpr int kWaves = kBlockWaves;  // wavefronts per start == trials per round

struct WideShm {
  double xs[kWide];  // iterate under evaluation (x, then x_new)
  double ps[kWide];  // search direction
  double vs[kWide];  // y, operand of u = H y
  double gs[kWide];  // gradient, operand of p = -H g
  double ss[kWide];  // s = x_new - x
  double us[kWide];  // u = H y
  double red[2][2][kWaves];  // [phase][sum][wave] partial sums
  double tsum[2 * kWaves][kMaxSums];  // [phase * waves + wave][sum] line-search trials' term sums
  double al[kTabTrials];
  int pass[2][kWaves];       // [phase][wave] line-search outcome
  StartCounts cnt;           // update skips and direction resets (thread 0)
  unsigned long long got;
  int bound;                 // early-stop bound of this iteration
  ReqHot q;
};

// See the narrow kernel for the mixed-precision rules (T = float): FP32
// evaluation with escalation to FP64 near the minimum, on a non-finite value
// or on a failed FP32 line search; H, s, y, p, g'p and Armijo stay FP64.
//
// Row products: blocks of kHBlock columns, the block sums added over the
// zero-padded pairwise tree of kHBlocks leaves.  The tree is folded as the
// blocks complete, like a binary counter: s[l] holds the finished subtree of
// 2^l blocks waiting for its right sibling.  The block index is the same on
// every lane, so the branches are uniform and the column loops stay short.
constexpr int kHBlock = 16;
constexpr int kHBlocks = kMaxDim / kHBlock;
static_assert(kHBlocks == 16, "the fold below has four levels");

__device__ __forceinline__ void fold_block(double x, int b, double (&s)[4], double &total) {
  if (!(b & 1)) { s[0] = x; return; }
  x = s[0] + x;
  if (!(b & 2)) { s[1] = x; return; }
  x = s[1] + x;
  if (!(b & 4)) { s[2] = x; return; }
  x = s[2] + x;
  if (!(b & 8)) { s[3] = x; return; }
  total = s[3] + x;
}

// sum_c H(j, c) v[c] for the column-major row starting at hc
__device__ __forceinline__ double slot_row_dot(const double *hc, int64_t cs, const double *v, int d) {
  double s[4] = {0.0, 0.0, 0.0, 0.0}, total = 0.0;
  int b = 0;
  for (; b * kHBlock < d; ++b) {
    const int c0 = b * kHBlock;
    double acc = 0.0;
    if (c0 + kHBlock <= d) {
#pragma unroll
      for (int k = 0; k < kHBlock; ++k) acc = __builtin_fma(hc[(int64_t)(c0 + k) * cs], v[c0 + k], acc);
    } else {
      for (int c = c0; c < d; ++c) acc = __builtin_fma(hc[(int64_t)c * cs], v[c], acc);
    }
    fold_block(acc, b, s, total);
  }
  for (; b < kHBlocks; ++b) fold_block(0.0, b, s, total);
  return total;
}
template <int OBJ, class T>
__global__ __launch_bounds__(kWide) void bfgs_wide_kernel(const ReqDev *reqs, int nreq,
                                                          BatchDev *hdr, int64_t total,
                                                          double *hslots, int cs, int64_t slot) {
  constexpr bool kMixed = sizeof(T) != sizeof(double);
  __shared__ WideShm sh;
  const int j = threadIdx.x;
  double *H = hslots + (int64_t)blockIdx.x * slot;  // column c of row j at H[c * cs + j]
  int phase = 0, lsphase = 0;
  int acc = -1;  // slot of sh.tsum with the accepted trial's term sums (block_armijo), or -1
  bool own = false, first = true, fresh = false, hi = !kMixed;
  double xj = 0.0, gj = 0.0, pj = 0.0, sj = 0.0, f = 0.0;
  int64_t idx = -1;
  int k = 0, ls_trials = 0;
  bool have_p = false;  // p = -H g already formed by the update pass
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
      fill_step_lengths(sh.al, rq.shrink, j, kWide);
      own = j < d0;
      xj = own ? rq.ws.x[idx * d0 + j] : 0.0;  // x <- swarm[i]
      sh.xs[j] = xj;
      if (own)  // H <- I
        for (int c = 0; c < d0; ++c) H[(int64_t)c * cs + j] = (c == j) ? 1.0 : 0.0;
      k = 0;
      ls_trials = 0;
      fresh = true;
      hi = !kMixed;
      have_p = false;
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

    // -- after a step: y, u = H y, the rank-2 update and p = -H_new g_new ----
    have_p = false;
    if (!fresh) {
      const double yj = gn - gj;
      const double sy = block_tree_sum(yj * sj, sh, phase);
      if (sy > 0.0) {
        const double rho = 1.0 / sy;
        sh.vs[j] = yj;
        sh.gs[j] = gn;
        __syncthreads();
        const double uj = own ? slot_row_dot(H + j, cs, sh.vs, d) : 0.0;
        const double yu = block_tree_sum(yj * uj, sh, phase);
        sh.us[j] = uj;
        sh.ss[j] = sj;
        __syncthreads();
        const double beta = (rho * rho) * yu + rho;
        const double au = -rho * sj;
        const double as = beta * sj - rho * uj;
        // H+ = H - rho (s u' + u s') + beta s s'   (row j), then p_j = -(H+ g)_j
        double total = 0.0;
        if (own) {
          double *hc = H + j;
          double s[4] = {0.0, 0.0, 0.0, 0.0};
          auto upd = [&](int c, double acc) {
            const double hn =
                __builtin_fma(as, sh.ss[c], __builtin_fma(au, sh.us[c], hc[(int64_t)c * cs]));
            hc[(int64_t)c * cs] = hn;
            return __builtin_fma(hn, sh.gs[c], acc);
          };
          int b = 0;
          for (; b * kHBlock < d; ++b) {
            const int c0 = b * kHBlock;
            double acc = 0.0;
            if (c0 + kHBlock <= d) {
#pragma unroll
              for (int k = 0; k < kHBlock; ++k) acc = upd(c0 + k, acc);
            } else {
              for (int c = c0; c < d; ++c) acc = upd(c, acc);
            }
            fold_block(acc, b, s, total);
          }
          for (; b < kHBlocks; ++b) fold_block(0.0, b, s, total);
        }
        pj = own ? -total : 0.0;
        have_p = true;
      } else if (j == 0) {
        ++sh.cnt.skips;
      }
      ++k;
    }
    gj = gn;
    f = fn;
    fresh = false;
    if (q.trace_len && own && k < q.trace_len) reqs[q.ri].trace[(idx * q.trace_len + k) * d + j] = xj;

    // -- termination ----------------------------------------------------------
    const bool bad = (own && !__builtin_isfinite(gj)) || !__builtin_isfinite(f);
    const bool any_bad = __syncthreads_or(bad) != 0;
    const double gg = block_tree_sum(gj * gj, sh, phase);
    if (kMixed && !hi && (any_bad || norm_below(gg, 10.0 * q.tol))) {
      hi = true;
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

    // -- search direction p = -H g (formed above after an update) ------------
    if (!have_p) {
      sh.gs[j] = gj;
      __syncthreads();
      pj = own ? -slot_row_dot(H + j, cs, sh.gs, d) : 0.0;
    }
    double ddir = block_tree_sum(gj * pj, sh, phase);
    if (!(ddir < 0.0)) {  // not a descent direction: H <- I, p = -g
      if (j == 0) ++sh.cnt.resets;
      if (own)
        for (int c = 0; c < d; ++c) H[(int64_t)c * cs + j] = (c == j) ? 1.0 : 0.0;
      pj = own ? -gj : 0.0;
      ddir = block_tree_sum(gj * pj, sh, phase);
    }
    sh.ps[j] = pj;
    __syncthreads();

    // -- Armijo backtracking -----------------------------------------------------
    int taken;
    if (hi) {
      taken = block_armijo<OBJ, double, kWide>(sh, f, ddir, lsphase, &acc);
    } else {
      taken = block_armijo<OBJ, T, kWide>(sh, f, ddir, lsphase, &acc);
      if (taken < 0) {
        ls_trials += q.iter_ls;
        hi = true;
        fresh = true;
        continue;
      }
    }
    const int nshrink = taken >= 0 ? taken : q.iter_ls;
    ls_trials += taken >= 0 ? taken + 1 : q.iter_ls;
    const double alpha = step_length(sh.al, q.shrink, nshrink);

    // -- step -------------------------------------------------------------------
    const double xnew = xj + alpha * pj;
    sj = own ? xnew - xj : 0.0;
    xj = own ? xnew : 0.0;
    __syncthreads();  // every lane has read xs and ps in the line search
    sh.xs[j] = xj;
  }
}

template <int OBJ, class T>
hipError_t launch_wide_t(const Group &g, int64_t want, int cus) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void *>(&bfgs_wide_kernel<OBJ, T>), kWide, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int64_t cap = (int64_t)cus * per_cu;
  if (g.resident) {
    *g.resident = cap;
    return hipSuccess;
  }
  if (cap > g.wide_slots) cap = g.wide_slots;
  const int blocks = (int)(want < cap ? want : cap);
  hipLaunchKernelGGL((bfgs_wide_kernel<OBJ, T>), dim3(blocks), dim3(kWide), 0, g.stream, g.reqs,
                     g.nreq, g.hdr, g.total_starts, g.hslots, g.wide_cs, g.wide_slot_doubles);
  return hipGetLastError();
}

template <class T>
hipError_t launch_wide_prec(const Group &g, int64_t want, int cus) {
  switch (g.objective) {
    case kRosenbrock: return launch_wide_t<kRosenbrock, T>(g, want, cus);
    case kRastrigin: return launch_wide_t<kRastrigin, T>(g, want, cus);
    case kAckley: return launch_wide_t<kAckley, T>(g, want, cus);
    case kStyblinskiTang: return launch_wide_t<kStyblinskiTang, T>(g, want, cus);
    case kSphere: return launch_wide_t<kSphere, T>(g, want, cus);
    case kQuartic: return launch_wide_t<kQuartic, T>(g, want, cus);
    default: return hipErrorInvalidValue;  // Goldstein-Price has d == 2
  }
}

}  // namespace

hipError_t launch_bfgs_wide(const Group &g, int cus) {
  if (!g.hslots || g.wide_slots < 1) return hipErrorInvalidValue;
  const int64_t want = g.total_starts;
  if (g.precision == ZEUS_MIXED) return launch_wide_prec<float>(g, want, cus);
  return launch_wide_prec<double>(g, want, cus);
}

}  // namespace zeus
