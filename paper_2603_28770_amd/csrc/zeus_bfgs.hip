// zeus_bfgs.hip -- the BFGS phase on gfx950: kernel launches and tiling (the
// kernel template is in zeus_bfgs_kernels.h), plus the final best-of-N
// reduction (Alg. 7).
#include <cstdlib>

#include "zeus_bfgs_kernels.h"

namespace zeus {
namespace {

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

// Between the two BFGS passes of a group with early stop: K* of every request
// that stops early, from its complete count of convergences up to K*, and
// the work counter reset for the second pass.
__global__ __launch_bounds__(64) void es_finish_kernel(const ReqDev *reqs, int nreq, BatchDev *hdr) {
  for (int r = threadIdx.x; r < nreq; r += blockDim.x) {
    const ReqDev &rq = reqs[r];
    if (rq.ws.es) rq.ws.es[kEsKstar] = es_search(rq.ws.es, rq.iter_bfgs + 1, rq.required_c);
  }
  if (threadIdx.x == 0) {
    hdr->queue = 0ull;
    hdr->es_pass = 2u;
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
  if (g.resident) {
    *g.resident = cap * (kBfgsBlock / G);
    return hipSuccess;
  }
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
// H in registers), kTileBlockDim (one block of four wavefronts per start, H in
// their registers, dim <= 128), kHybridDim (one block of eight wavefronts per
// start, H in their registers and LDS, dim <= 208) or kWideLanes (one block
// per start, H in device memory).
// Every tiling computes the same pairwise trees, so results do not depend on
// it; only speed does.  The rules come from the autotuner's table; a start
// no rule covers gets the smallest power of two >= max(dim, 4), or above 64
// dimensions the block with H on chip (in registers up to 128, in registers
// and LDS up to 208; the device-memory block above).  A user objective up to 8 dimensions gets 32 lanes:
// evaluated as a whole it tries one step length per lane in a line-search
// round, and on four user sources (d = 2..5, 1.9 to 12 trials per iteration)
// 32 lanes took 0.71 of the time of the smallest group in geometric mean.
// ZEUS_TILE_LANES forces a tiling (the autotuner uses it to time the
// candidates).
#include "zeus_tiling.inc"

namespace {
bool tiling_valid(int lanes, int dim) {
  if (lanes == kWideLanes) return dim <= kMaxDim;
  if (lanes == kTileBlockDim) return dim <= kTileBlockDim;
  if (lanes == kHybridDim) return dim <= kHybridDim;
  return lanes >= 2 && lanes <= kMaxNarrowDim && (lanes & (lanes - 1)) == 0 && lanes >= dim;
}
}  // namespace

int group_lanes(int objective, int precision, int dim) {
  if (const char *e = getenv("ZEUS_TILE_LANES")) {
    const int v = atoi(e);
    if (v > 0 && tiling_valid(v, dim)) return v;
  }
  if (dim > kMaxNarrowDim)
    return dim <= kTileBlockDim ? kTileBlockDim : dim <= kHybridDim ? kHybridDim : kWideLanes;
  for (const TileRule &r : kTileRules)
    if (r.objective == objective && r.precision == precision && dim >= r.dmin && dim <= r.dmax &&
        tiling_valid(r.lanes, dim))
      return r.lanes;
  if (objective == kUser && dim <= 8) return 32;
  int g = 4;
  while (g < dim) g <<= 1;
  return g;
}

size_t bfgs_lds_bytes(int lanes) {
  return sizeof(double) * (size_t)group_stride(lanes) * (kBfgsBlock / lanes);
}

hipError_t launch_bfgs(const Group &g) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (cus <= 0) cus = 256;
  // ZEUS_BFGS_CUS sizes the persistent grid for fewer compute units: the
  // tests use it to show that results do not depend on how many groups or
  // blocks share the starts (nor on which of them runs which start)
  if (const char *e = getenv("ZEUS_BFGS_CUS")) {
    const int v = atoi(e);
    if (v > 0 && v < cus) cus = v;
  }
  if (g.method == 1) return launch_lbfgs(g, cus);
  if (g.g_bfgs == kWideLanes) return launch_bfgs_wide(g, cus);
  if (g.g_bfgs == kTileBlockDim || g.g_bfgs == kHybridDim) {
    if (g.objective == kUser) return launch_user_bfgs(g, g.total_starts, cus);
    return g.g_bfgs == kTileBlockDim ? launch_bfgs_tile(g, cus) : launch_bfgs_hybrid(g, cus);
  }
  if (g.g_bfgs > kMaxNarrowDim) return hipErrorInvalidValue;
  const int64_t starts_per_block = (int64_t)(kBfgsBlock / g.g_bfgs);
  const int64_t want = (g.total_starts + starts_per_block - 1) / starts_per_block;
  if (g.objective == kUser) return launch_user_bfgs(g, want, cus);
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

hipError_t launch_es_finish(const Group &g) {
  hipLaunchKernelGGL(es_finish_kernel, dim3(1), dim3(64), 0, g.stream, g.reqs, g.nreq, g.hdr);
  return hipGetLastError();
}

hipError_t launch_summary(const Group &g) {
  hipLaunchKernelGGL(summary_kernel, dim3(g.nreq), dim3(kSumBlock), 0, g.stream, g.reqs);
  return hipGetLastError();
}

}  // namespace zeus
