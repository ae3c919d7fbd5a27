// zeus_pso.hip -- swarm phase on gfx950: initialisation (Alg. 2 / Alg. 8) and
// synchronous updates (Alg. 3 / Alg. 9), one thread per particle.
//
// The paper's kernels take the global best with an atomicMin on the value
// followed by an unsynchronised copy of the position, which lets two winners
// interleave their copies.  Here every launch ends with a deterministic
// reduction instead: each block reduces (value, index) pairs to its best, and
// the last block to finish (an agent-scope counter) reduces the block results
// in index order and refreshes the global best once, on strict improvement,
// lowest index on ties.  A NaN value ranks as +infinity.
//
// Particle state is struct-of-arrays in HBM, row-major [n][dim] doubles.
#include "zeus_device.h"
#include "zeus_internal.h"

namespace zeus {
namespace {

struct PsoArgs {
  int64_t n;
  int d;
  int t;            // PSO iteration (1-based); 0 for the initialisation
  double lo, hi;    // sampling box
  double vh;        // velocity half-range
  double w, c1, c2; // inertia, cognitive, social
  uint64_t k0, k1;  // Philox key (seed, request id)
  Workspace ws;
};

// Block-wide (key, index) minimum; result valid in thread 0.
__device__ void block_argmin(double &key, int64_t &idx, double *sk, int64_t *si) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ok = __shfl_xor(key, off, 64);
    const int64_t oi = __shfl_xor(idx, off, 64);
    if (key_less(ok, oi, key, idx)) {
      key = ok;
      idx = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sk[wave] = key;
    si[wave] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int wv = 1; wv < kPsoBlock / 64; ++wv)
      if (key_less(sk[wv], si[wv], key, idx)) {
        key = sk[wv];
        idx = si[wv];
      }
  }
  __syncthreads();
}

// Publishes this block's best; the last block of the grid then reduces all
// block results and updates the global best (always for the initial swarm,
// on strict improvement afterwards) and copies its position to gx.
__device__ void finish_global_best(const PsoArgs &a, double key, int64_t idx, bool initial) {
  __shared__ double sk[kPsoBlock / 64];
  __shared__ int64_t si[kPsoBlock / 64];
  __shared__ bool last;
  __shared__ int64_t winner;
  block_argmin(key, idx, sk, si);
  __threadfence();  // make this block's particle writes visible device-wide
  __syncthreads();
  if (threadIdx.x == 0) {
    a.ws.partial_key[blockIdx.x] = key;
    a.ws.partial_idx[blockIdx.x] = idx;
    __threadfence();
    const uint32_t done = atomicAdd(a.ws.pso_counter, 1u);
    last = (done == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();  // acquire the other blocks' results
  double k = __builtin_huge_val();
  int64_t i = INT64_MAX;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kPsoBlock) {
    const double kb = __hip_atomic_load(&a.ws.partial_key[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t ib = __hip_atomic_load(&a.ws.partial_idx[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (key_less(kb, ib, k, i)) {
      k = kb;
      i = ib;
    }
  }
  block_argmin(k, i, sk, si);
  if (threadIdx.x == 0) {
    const double fm = a.ws.pf[i];
    bool take = initial || rank_key(fm) < rank_key(a.ws.best->f);
    if (take) {
      a.ws.best->f = fm;
      a.ws.best->idx = i;
    }
    winner = take ? i : -1;
    *a.ws.pso_counter = 0u;  // ready for the next launch
  }
  __syncthreads();
  if (winner >= 0)
    for (int j = threadIdx.x; j < a.d; j += kPsoBlock) a.ws.gx[j] = a.ws.px[winner * a.d + j];
}

template <int OBJ>
__global__ __launch_bounds__(kPsoBlock) void pso_init_kernel(PsoArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kPsoBlock + threadIdx.x;
  double key = __builtin_huge_val();
  int64_t idx = INT64_MAX;
  if (i < a.n) {
    const int d = a.d;
    double *xr = a.ws.x + i * d, *vr = a.ws.v + i * d, *pr = a.ws.px + i * d;
    const double vlo = -a.vh, vhi = a.vh;
    for (int jb = 0; jb * 4 < d; ++jb) {
      const u64x4 rx = philox4x64_10((uint64_t)jb, (uint64_t)i, 0, kTagX0, a.k0, a.k1);
      const u64x4 rv = philox4x64_10((uint64_t)jb, (uint64_t)i, 0, kTagV0, a.k0, a.k1);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jb * 4 + q;
        if (j < d) {
          // UniformSample(lo, hi) = lo + u (hi - lo)
          const double xv = a.lo + u01(rx.w[q]) * (a.hi - a.lo);
          const double vv = vlo + u01(rv.w[q]) * (vhi - vlo);
          xr[j] = xv;
          vr[j] = vv;
          pr[j] = xv;
        }
      }
    }
    const double f = Obj<OBJ>::template eval<double>(d, [=](int j) { return xr[j]; });
    a.ws.pf[i] = f;
    key = rank_key(f);
    idx = i;
  }
  finish_global_best(a, key, idx, true);
}

template <int OBJ>
__global__ __launch_bounds__(kPsoBlock) void pso_step_kernel(PsoArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kPsoBlock + threadIdx.x;
  double key = __builtin_huge_val();
  int64_t idx = INT64_MAX;
  if (i < a.n) {
    const int d = a.d;
    double *xr = a.ws.x + i * d, *vr = a.ws.v + i * d, *pr = a.ws.px + i * d;
    const double *gx = a.ws.gx;
    for (int jb = 0; jb * 4 < d; ++jb) {
      const u64x4 r1w = philox4x64_10((uint64_t)jb, (uint64_t)i, (uint64_t)a.t, kTagR1, a.k0, a.k1);
      const u64x4 r2w = philox4x64_10((uint64_t)jb, (uint64_t)i, (uint64_t)a.t, kTagR2, a.k0, a.k1);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jb * 4 + q;
        if (j < d) {
          const double r1 = u01(r1w.w[q]), r2 = u01(r2w.w[q]);
          const double x = xr[j], v = vr[j];
          // v' = w v + c1 r1 (p - x) + c2 r2 (g - x);  x' = x + v'
          const double inertia = a.w * v;
          const double cog = (a.c1 * r1) * (pr[j] - x);
          const double soc = (a.c2 * r2) * (gx[j] - x);
          const double vn = (inertia + cog) + soc;
          vr[j] = vn;
          xr[j] = x + vn;
        }
      }
    }
    const double fx = Obj<OBJ>::template eval<double>(d, [=](int j) { return xr[j]; });
    double pf = a.ws.pf[i];
    if (rank_key(fx) < rank_key(pf)) {  // personal best, strict
      pf = fx;
      a.ws.pf[i] = fx;
      for (int j = 0; j < d; ++j) pr[j] = xr[j];
    }
    key = rank_key(pf);
    idx = i;
  }
  finish_global_best(a, key, idx, false);
}

__global__ void ws_init_kernel(Workspace ws) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *ws.pso_counter = 0u;
    *ws.queue = 0ull;
  }
}

PsoArgs make_args(const Launch &L, int t) {
  const zeus_problem &p = *L.pb;
  PsoArgs a;
  a.n = p.n_starts;
  a.d = p.dim;
  a.t = t;
  a.lo = p.lower;
  a.hi = p.upper;
  a.vh = p.v_half > 0.0 ? p.v_half : (p.upper - p.lower);
  a.w = p.w;
  a.c1 = p.c1;
  a.c2 = p.c2;
  a.k0 = p.seed;
  a.k1 = p.request_id;
  a.ws = L.ws;
  return a;
}

template <template <int> class K>
hipError_t launch_obj(int obj, dim3 grid, hipStream_t s, const PsoArgs &a) {
  switch (obj) {
    case kRosenbrock: hipLaunchKernelGGL(K<kRosenbrock>::fn, grid, dim3(kPsoBlock), 0, s, a); break;
    case kRastrigin: hipLaunchKernelGGL(K<kRastrigin>::fn, grid, dim3(kPsoBlock), 0, s, a); break;
    case kAckley: hipLaunchKernelGGL(K<kAckley>::fn, grid, dim3(kPsoBlock), 0, s, a); break;
    case kStyblinskiTang: hipLaunchKernelGGL(K<kStyblinskiTang>::fn, grid, dim3(kPsoBlock), 0, s, a); break;
    case kGoldsteinPrice: hipLaunchKernelGGL(K<kGoldsteinPrice>::fn, grid, dim3(kPsoBlock), 0, s, a); break;
    case kSphere: hipLaunchKernelGGL(K<kSphere>::fn, grid, dim3(kPsoBlock), 0, s, a); break;
    case kQuartic: hipLaunchKernelGGL(K<kQuartic>::fn, grid, dim3(kPsoBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int OBJ> struct InitK { static constexpr auto fn = pso_init_kernel<OBJ>; };
template <int OBJ> struct StepK { static constexpr auto fn = pso_step_kernel<OBJ>; };

}  // namespace

int pso_blocks(int64_t n) { return (int)((n + kPsoBlock - 1) / kPsoBlock); }

hipError_t launch_ws_init(const Launch &L) {
  hipLaunchKernelGGL(ws_init_kernel, dim3(1), dim3(64), 0, L.stream, L.ws);
  return hipGetLastError();
}

hipError_t launch_pso_init(const Launch &L) {
  const PsoArgs a = make_args(L, 0);
  return launch_obj<InitK>(L.pb->objective, dim3(L.ws.pso_blocks), L.stream, a);
}

hipError_t launch_pso_step(const Launch &L, int t) {
  const PsoArgs a = make_args(L, t);
  return launch_obj<StepK>(L.pb->objective, dim3(L.ws.pso_blocks), L.stream, a);
}

}  // namespace zeus
