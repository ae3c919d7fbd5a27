// zeus_bfgs.hip -- the BFGS phase on gfx950 (Alg. 4 / Alg. 10 with the
// dual-number gradient of Alg. 5 and the Armijo line search of Alg. 6), plus
// the final best-of-N reduction (Alg. 7).
//
// Mapping (the "more levels of parallelism" the paper leaves for later):
//  * one group of G lanes (G a power of two >= dim, G <= 64) runs one start;
//    a 64-lane wavefront holds 64/G groups, a 256-thread block four waves;
//  * lane j owns coordinate j and row j of the inverse Hessian H, which stays
//    in registers for the whole run (H never touches HBM);
//  * gradient: lane j evaluates the objective on dual numbers seeded with the
//    tangent e_j, so the G lanes compute the dim passes of Alg. 5 at once;
//  * line search: lane j evaluates trial j (alpha = shrink^j) of the
//    backtracking sequence; the first trial that satisfies the Armijo
//    condition is taken, which is exactly the step the sequential loop of
//    Alg. 6 would return, in one objective evaluation instead of several;
//  * the small vectors a lane needs in full (x, p, g, s, y, u) are exchanged
//    through the group's slice of LDS;
//  * each group first takes the start with its own index, then claims starts
//    from an agent-scope work counter, so a group that finishes early takes
//    the next start instead of idling; results do not depend on which group
//    ran which start.
// The loop is flattened so that every trip does one gradient evaluation and
// one line search for every group of a wave, whatever iteration each group's
// start is in.
#include <cstdlib>

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
  bool fresh = false, first = true;
  bool hi = !kMixed;  // evaluating in FP64 (always, unless mixed precision)

  for (;;) {
    // -- claim a start when idle ------------------------------------------
    if (idx < 0) {
      // the first start of a group is its own index; later ones come from
      // the counter, after the starts taken that way
      const unsigned long long groups = (unsigned long long)gridDim.x * (kBfgsBlock / G);
      unsigned long long got = 0;
      if (first) {
        got = (unsigned long long)blockIdx.x * (kBfgsBlock / G) + (threadIdx.x >> 6) * S + L.grp;
        first = false;
      } else {
        if (j == 0) got = groups + atomicAdd((unsigned long long *)&hdr->queue, 1ull);
        got = __shfl(got, L.grp * G, 64);
      }
      if (got >= (unsigned long long)total) break;
      const int ri = request_of(reqs, nreq, (int64_t)got);
      const ReqDev &rq = reqs[ri];
      idx = (int64_t)got - rq.start_offset;
      const int d0 = rq.d;
      if (j == 0) load_hot<OBJ>(*sh.q, rq, ri);
      own = j < d0;
      fill_step_lengths(sh.al, rq.shrink, j, G);
      xj = own ? rq.ws.x[idx * d0 + j] : 0.0;  // x <- swarm[i]
      sh.xs[j] = xj;
      H.identity(j);  // H <- I
      k = 0;
      ls_trials = 0;
      fresh = true;
      hi = !kMixed;
    }
    wave_sync();
    const ReqHot &q = *sh.q;
    const int d = q.d;

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
        sh.vs[vpos<G>(j)] = yj;
        wave_sync();
        double uj = H.matvec(sh.vs, j);  // every lane: the tile sums cross lanes
        uj = own ? uj : 0.0;
        const double yu = lane_tree_sum<G, double>(yj * uj);
        sh.us[vpos<G>(j)] = uj;
        sh.ss[vpos<G>(j)] = sj;
        wave_sync();
        const double beta = (rho * rho) * yu + rho;
        // H+ = H - rho (s u' + u s') + beta s s'   (u = H y); inf * 0 would
        // have reached the padding when a coefficient is not finite
        if (!H.rank2(rho, beta, sh.us, sh.ss, j, sj, uj)) H.restore_padding(j, d);
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
    if (kMixed && !hi && (any_bad || sqrt(gg) < 10.0 * q.tol)) {
      hi = true;  // escalate: re-evaluate this point in FP64
      fresh = true;
      continue;
    }
    int status = -1;
    if (any_bad)
      status = ZEUS_ST_NONFINITE;
    else if (sqrt(gg) < q.tol)
      status = ZEUS_ST_CONVERGED;
    else if (k == q.iter_bfgs)
      status = q.stop_status;  // MAXITER, or STOPPED at an early-stop cap
    if (status >= 0) {
      const ReqDev &rq = reqs[q.ri];
      const int tl = q.trace_len;
      if (own) rq.out_x[idx * d + j] = xj;
      if (kMixed && !hi) f = group_value<OBJ, G, double>(L, d, sh.xs);  // FP64 value at x
      if (j == 0) {
        rq.out_f[idx] = f;
        rq.out_iters[idx] = k;
        rq.out_status[idx] = status;
        if (rq.out_ls) rq.out_ls[idx] = ls_trials;
      }
      if (tl && own)
        for (int kk = k + 1; kk < tl; ++kk)
          rq.trace[(idx * tl + kk) * d + j] = __builtin_nan("");
      idx = -1;
      continue;
    }

    // -- search direction p = -H g (reset to -g if not a descent direction) -
    sh.vs[vpos<G>(j)] = gj;
    wave_sync();
    const double hg = H.matvec(sh.vs, j);  // every lane: the tile sums cross lanes
    pj = own ? -hg : 0.0;
    double ddir = lane_tree_sum<G, double>(gj * pj);
    if (!(ddir < 0.0)) {
      H.identity(j);
      pj = own ? -gj : 0.0;
      ddir = lane_tree_sum<G, double>(gj * pj);
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

// Best-of-N and counts over all starts of one request per block
// (deterministic: (f, index) minimum over finite f, exact integer sums).
constexpr int kSumBlock = 1024;

__global__ __launch_bounds__(kSumBlock) void summary_kernel(const ReqDev *reqs) {
  __shared__ double sk[kSumBlock / 64];
  __shared__ int64_t si[kSumBlock / 64];
  __shared__ int64_t sc[4][kSumBlock / 64];
  const ReqDev &rq = reqs[blockIdx.x];
  const int64_t n = rq.n;
  const double *f = rq.out_f;
  double key = __builtin_huge_val();
  int64_t idx = INT64_MAX;
  int64_t nconv = 0, nnf = 0, it = 0, lt = 0;
  // U elements per thread per trip, their loads issued together
  constexpr int U = 8;
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += (int64_t)kSumBlock * U) {
    double fv[U];
    int32_t sv[U], iv[U], lv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * kSumBlock;
      const bool in = i < n;
      fv[u] = in ? f[i] : __builtin_huge_val();
      sv[u] = in ? rq.out_status[i] : -1;
      iv[u] = in ? rq.out_iters[i] : 0;
      lv[u] = (in && rq.out_ls) ? rq.out_ls[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * kSumBlock;
      if (__builtin_isfinite(fv[u]) && key_less(fv[u], i, key, idx)) {
        key = fv[u];
        idx = i;
      }
      nconv += sv[u] == ZEUS_ST_CONVERGED;
      nnf += sv[u] == ZEUS_ST_NONFINITE;
      it += iv[u];
      lt += lv[u];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ok = __shfl_xor(key, off, 64);
    const int64_t oi = __shfl_xor(idx, off, 64);
    if (key_less(ok, oi, key, idx)) {
      key = ok;
      idx = oi;
    }
    nconv += __shfl_xor(nconv, off, 64);
    nnf += __shfl_xor(nnf, off, 64);
    it += __shfl_xor(it, off, 64);
    lt += __shfl_xor(lt, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sk[wave] = key;
    si[wave] = idx;
    sc[0][wave] = nconv;
    sc[1][wave] = nnf;
    sc[2][wave] = it;
    sc[3][wave] = lt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int wv = 1; wv < kSumBlock / 64; ++wv) {
      if (key_less(sk[wv], si[wv], key, idx)) {
        key = sk[wv];
        idx = si[wv];
      }
      nconv += sc[0][wv];
      nnf += sc[1][wv];
      it += sc[2][wv];
      lt += sc[3][wv];
    }
    const bool found = idx != INT64_MAX;
    zeus_summary *out = rq.summary;
    out->best_index = found ? idx : -1;
    out->best_f = found ? f[idx] : __builtin_nan("");
    out->n_converged = nconv;
    out->n_nonfinite = nnf;
    out->total_iters = it;
    out->total_ls_trials = lt;
    out->pso_best_index = rq.ws.best->idx;
    out->pso_best_f = rq.ws.best->f;
  }
}

// The kernel is persistent: it gets as many blocks as can be resident at once
// (more would only start once the work counter is spent).
template <int OBJ, int G, class T>
hipError_t launch_g(const Group &g, int64_t want, int cus) {
  const size_t lds = sizeof(double) * (size_t)group_stride(G) * (kBfgsBlock / G);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void *>(&bfgs_kernel<OBJ, G, T>), kBfgsBlock, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int64_t cap = (int64_t)cus * per_cu;
  const int blocks = (int)(want < cap ? want : cap);
  hipLaunchKernelGGL((bfgs_kernel<OBJ, G, T>), dim3(blocks), dim3(kBfgsBlock), lds, g.stream,
                     g.reqs, g.nreq, g.hdr, g.total_starts);
  return hipGetLastError();
}

template <int OBJ, class T>
hipError_t launch_obj(const Group &g, int64_t want, int cus) {
  switch (g.g_bfgs) {
    case 2: return launch_g<OBJ, 2, T>(g, want, cus);
    case 4: return launch_g<OBJ, 4, T>(g, want, cus);
    case 8: return launch_g<OBJ, 8, T>(g, want, cus);
    case 16: return launch_g<OBJ, 16, T>(g, want, cus);
    case 32: return launch_g<OBJ, 32, T>(g, want, cus);
    case 64: return launch_g<OBJ, 64, T>(g, want, cus);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t launch_prec(const Group &g, int64_t want, int cus) {
  switch (g.objective) {
    case kRosenbrock: return launch_obj<kRosenbrock, T>(g, want, cus);
    case kRastrigin: return launch_obj<kRastrigin, T>(g, want, cus);
    case kAckley: return launch_obj<kAckley, T>(g, want, cus);
    case kStyblinskiTang: return launch_obj<kStyblinskiTang, T>(g, want, cus);
    case kGoldsteinPrice: return launch_obj<kGoldsteinPrice, T>(g, want, cus);
    case kSphere: return launch_obj<kSphere, T>(g, want, cus);
    case kQuartic: return launch_obj<kQuartic, T>(g, want, cus);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Tiling: lanes per start (2..64, a power of two >= dim: one group per start,
// H in registers) or kWideLanes (one block per start, H in device memory).
// Every tiling computes the same pairwise trees, so results do not depend on
// it; only speed does.  The rules come from the autotuner's table; a start
// no rule covers gets the smallest power of two >= max(dim, 4), or the block
// above 64 dimensions.  ZEUS_TILE_LANES forces a tiling (the autotuner uses
// it to time the candidates).
#include "zeus_tiling.inc"

namespace {
bool tiling_valid(int lanes, int dim) {
  if (lanes == kWideLanes) return dim <= kMaxDim;
  return lanes >= 2 && lanes <= kMaxNarrowDim && (lanes & (lanes - 1)) == 0 && lanes >= dim;
}
}  // namespace

int group_lanes(int objective, int precision, int dim) {
  if (const char *e = getenv("ZEUS_TILE_LANES")) {
    const int v = atoi(e);
    if (v > 0 && tiling_valid(v, dim)) return v;
  }
  if (dim > kMaxNarrowDim) return kWideLanes;
  for (const TileRule &r : kTileRules)
    if (r.objective == objective && r.precision == precision && dim >= r.dmin && dim <= r.dmax &&
        tiling_valid(r.lanes, dim))
      return r.lanes;
  int g = 4;
  while (g < dim) g <<= 1;
  return g;
}

hipError_t launch_bfgs(const Group &g) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (cus <= 0) cus = 256;
  if (g.method == 1) return launch_lbfgs(g, cus);
  if (g.g_bfgs == kWideLanes) return launch_bfgs_wide(g, cus);
  if (g.g_bfgs > kMaxNarrowDim) return hipErrorInvalidValue;
  const int64_t starts_per_block = (int64_t)(kBfgsBlock / g.g_bfgs);
  const int64_t want = (g.total_starts + starts_per_block - 1) / starts_per_block;
  if (g.precision == ZEUS_MIXED) return launch_prec<float>(g, want, cus);
  return launch_prec<double>(g, want, cus);
}

int wide_slots(int64_t total_starts) {
  return (int)(total_starts < kWideMaxSlots ? total_starts : kWideMaxSlots);
}

int wide_cs(int dmax) { return (dmax + 63) / 64 * 64; }

size_t wide_hslot_bytes(int64_t total_starts, int dmax) {
  return sizeof(double) * (size_t)wide_slots(total_starts) * (size_t)dmax * (size_t)wide_cs(dmax);
}

hipError_t launch_summary(const Group &g) {
  hipLaunchKernelGGL(summary_kernel, dim3(g.nreq), dim3(kSumBlock), 0, g.stream, g.reqs);
  return hipGetLastError();
}

}  // namespace zeus
