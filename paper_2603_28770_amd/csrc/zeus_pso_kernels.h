// zeus_pso_kernels.h -- swarm kernel templates for gfx950: initialisation (Alg. 2 / Alg. 8) and
// synchronous updates (Alg. 3 / Alg. 9).
//
// One group of G lanes per particle: lane j draws, updates and stores
// coordinate j (consecutive lanes touch consecutive addresses), the group
// evaluates the objective term-parallel and keeps the personal best.
// A launch serves a table of requests (one request, or a bucket of a batch);
// each request owns P = min(#particle groups, 1024) consecutive blocks that
// stride over its particles.
//
// Global best.  The paper's kernels take it with an atomicMin on the value and
// an unsynchronised copy of the position, which lets two winners interleave
// their copies.  Here it is a deterministic reduction in three stages, with no
// device-wide fence anywhere: (1) each block reduces its particles to one
// (rank key, index) pair and stores it, with the winner's position, in slot
// t & 1; (2) every block of the next launch reduces those P block results
// itself (after the kernel boundary they are visible to all), compares the
// winner with the previous global best (strict improvement, lowest index on
// ties, NaN ranking as +infinity) and so starts the sweep with the global best
// of sweep t; block 0 also records it for later launches; (3) after the last
// sweep a one-block launch performs stage (2) once more to publish the result.
#pragma once

#include "zeus_device.h"
#include "zeus_group.h"
#include "zeus_internal.h"

namespace zeus {
namespace {

// Index of the table entry whose [offset, next offset) holds v (offsets are
// ascending and start at 0).
template <class Off>
__device__ __forceinline__ int find_entry(const ReqDev *reqs, int nreq, int64_t v, Off off) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off(reqs[mid]) <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Block-wide minimum of (key, idx) carrying two payloads; the result is left
// in every thread.
template <int NT>
__device__ void block_argmin(double &key, int64_t &idx, double &val, int64_t &aux) {
  __shared__ double sk[NT / 64], sv[NT / 64];
  __shared__ int64_t si[NT / 64], sa[NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ok = __shfl_xor(key, off, 64);
    const int64_t oi = __shfl_xor(idx, off, 64);
    const double ov = __shfl_xor(val, off, 64);
    const int64_t oa = __shfl_xor(aux, off, 64);
    if (key_less(ok, oi, key, idx)) {
      key = ok;
      idx = oi;
      val = ov;
      aux = oa;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sk[wave] = key;
    si[wave] = idx;
    sv[wave] = val;
    sa[wave] = aux;
  }
  __syncthreads();
  key = sk[0];
  idx = si[0];
  val = sv[0];
  aux = sa[0];
  for (int wv = 1; wv < NT / 64; ++wv)
    if (key_less(sk[wv], si[wv], key, idx)) {
      key = sk[wv];
      idx = si[wv];
      val = sv[wv];
      aux = sa[wv];
    }
  __syncthreads();
}

// Stage (2): the global best after sweep `done` (>= 0) from the block results
// of that sweep and the global best after sweep done-1.  Leaves its position
// in gx_sh[0..d) for every thread of the block.  When `publish`, the result is
// also stored for later launches (and in final_best / final_gx if given).
//
// It is split in two so that a caller can issue the loads of the block
// results (stage_two_load) and do unrelated work while they are in flight.
template <int NT>
struct StageTwo {
  static constexpr int kPer = (kPsoMaxBlocks + NT - 1) / NT;  // block results per thread
  double kb[kPer], fb[kPer];
  int64_t ib[kPer];
};

template <int NT>
__device__ __forceinline__ void stage_two_load(const ReqDev &a, int done, StageTwo<NT> &s) {
  const int P = a.ws.pso_blocks, slot = done & 1;
#pragma unroll
  for (int r = 0; r < StageTwo<NT>::kPer; ++r) {
    const int b = threadIdx.x + r * NT;
    s.kb[r] = __builtin_huge_val();
    s.ib[r] = INT64_MAX;
    s.fb[r] = __builtin_nan("");
    if (b < P) {
      s.kb[r] = a.ws.part_key[slot * P + b];
      s.ib[r] = a.ws.part_idx[slot * P + b];
      s.fb[r] = a.ws.part_f[slot * P + b];
    }
  }
}

template <int NT>
__device__ void global_best_after(const ReqDev &a, int done, double *gx_sh, bool publish,
                                  PsoBest *final_best, double *final_gx, const StageTwo<NT> &s) {
  const int d = a.d, slot = done & 1, P = a.ws.pso_blocks;
  double key = __builtin_huge_val(), val = __builtin_nan("");
  int64_t idx = INT64_MAX, blk = 0;
#pragma unroll
  for (int r = 0; r < StageTwo<NT>::kPer; ++r)
    if (key_less(s.kb[r], s.ib[r], key, idx)) {
      key = s.kb[r];
      idx = s.ib[r];
      val = s.fb[r];
      blk = threadIdx.x + r * NT;
    }
  block_argmin<NT>(key, idx, val, blk);
  bool take = true;
  PsoBest prev{0.0, 0};
  if (done > 0) {
    prev = a.ws.best_store[(done - 1) & 1];
    take = rank_key(val) < rank_key(prev.f);  // strict improvement
  }
  for (int j = threadIdx.x; j < d; j += NT)
    gx_sh[j] = take ? a.ws.part_x[((size_t)slot * P + blk) * d + j]
                    : a.ws.gx_store[((done - 1) & 1) * d + j];
  __syncthreads();
  if (publish) {
    const PsoBest nb = take ? PsoBest{val, idx} : prev;
    if (threadIdx.x == 0) {
      a.ws.best_store[slot] = nb;
      if (final_best) *final_best = nb;
    }
    for (int j = threadIdx.x; j < d; j += NT) {
      a.ws.gx_store[slot * d + j] = gx_sh[j];
      if (final_gx) final_gx[j] = gx_sh[j];
    }
  }
}

// G lanes per particle, each owning CPL coordinates j, j + G, ...
template <int OBJ, int G, int CPL>
__global__ __launch_bounds__(pso_threads(G * CPL)) void pso_kernel(const ReqDev *reqs, int nreq,
                                                                  int t) {
  constexpr int NT = pso_threads(G * CPL);
  constexpr int kGroups = NT / G;
  constexpr int kSlots = G * CPL;
  // Uniforms of up to kBatch particles per group are drawn together, so
  // that the 2 ceil(d / 4) Philox blocks of each particle keep more of the
  // group's lanes busy (d = 10: 12 blocks over 16 lanes instead of 6).
  constexpr int kBatch = CPL == 1 && G >= 4 ? 3 : 1;
  __shared__ double xs_all[kGroups][kSlots];
  __shared__ double uw_all[kGroups][kBatch][2][kSlots + 4];  // [particle][stream][coordinate]
  __shared__ double gx_sh[kMaxDim];
  const int r = find_entry(reqs, nreq, blockIdx.x, [](const ReqDev &q) { return (int64_t)q.block_offset; });
  const ReqDev &a = reqs[r];
  if (t > a.iter_pso) return;  // this request's swarm is done
  const int blk = (int)blockIdx.x - a.block_offset;  // block within the request
  const GroupLanes<G> L;
  const int gib = threadIdx.x / G;  // group in block
  double *xs = xs_all[gib];
  const int d = a.d, j = L.j, P = a.ws.pso_blocks;
  const int nb = (d + 3) >> 2;  // Philox blocks per stream

  const uint64_t tag_a = t == 0 ? kTagX0 : kTagR1, tag_b = t == 0 ? kTagV0 : kTagR2;
  const int64_t stride = (int64_t)P * kGroups;
  const int64_t first = (int64_t)blk * kGroups + gib;
  // particles per batch: as many as fit their Philox blocks into G lanes
  const int pb = kBatch == 1 ? 1 : (G / (2 * nb) < 1 ? 1 : (G / (2 * nb) > kBatch ? kBatch : G / (2 * nb)));
  // Philox blocks b = j, j + G, ... below pb 2 nb of the batch starting at
  // particle k0: particle b / (2 nb) of the batch, block (b mod 2 nb) mod nb
  // of stream a (the first nb) or stream b
  auto draw = [&](int64_t k0) {
    for (int b = j; b < pb * 2 * nb; b += G) {
      const int pp = b / (2 * nb), bb = b - pp * 2 * nb;
      const int64_t ip = first + (k0 + pp) * stride;
      if (ip >= a.n) continue;
      const int sb = bb >= nb, jb = sb ? bb - nb : bb;
      const u64x4 rw = philox4x64_10((uint64_t)jb, (uint64_t)ip, (uint64_t)t, sb ? tag_b : tag_a,
                                     a.k0, a.k1);
#pragma unroll
      for (int q = 0; q < 4; ++q) uw_all[gib][pp][sb][jb * 4 + q] = u01(rw.w[q]);
    }
  };

  // stage (2), its loads in flight while the first batch is drawn
  StageTwo<NT> s2;
  if (t > 0) stage_two_load<NT>(a, t - 1, s2);
  draw(0);
  if (t > 0) global_best_after<NT>(a, t - 1, gx_sh, blk == 0, nullptr, nullptr, s2);
  double gxj[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) gxj[c] = (t > 0 && j + G * c < d) ? gx_sh[j + G * c] : 0.0;

  // this block's best particle of the sweep, tracked by each group's lane 0
  double key = __builtin_huge_val(), val = __builtin_nan("");
  int64_t idx = INT64_MAX, unused = 0;
  for (int64_t k0 = 0;; k0 += pb) {
    if (__ballot(first + k0 * stride < a.n) == 0ull) break;  // the whole wave is past the end
    if (k0 > 0) {
      wave_sync();  // the previous batch's uniforms have been read
      draw(k0);
    }
    wave_sync();
    for (int pp = 0; pp < pb; ++pp) {
      const int64_t i = first + (k0 + pp) * stride;
      const bool live = i < a.n;
      if (__ballot(live) == 0ull) break;
      const double (*uw)[kSlots + 4] = uw_all[gib][pp];
      double x[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int jj = j + G * c;
        x[c] = 0.0;
        if (!(live && jj < d)) continue;
        const int64_t o = i * d + jj;
        const double ua = uw[0][jj], ub = uw[1][jj];
        if (t == 0) {
          const double vlo = -a.vh, vhi = a.vh;
          // UniformSample(lo, hi) = lo + u (hi - lo)
          x[c] = a.lo + ua * (a.hi - a.lo);
          const double v = vlo + ub * (vhi - vlo);
          a.ws.x[o] = x[c];
          a.ws.v[o] = v;
          a.ws.px[o] = x[c];
        } else {
          const double x0 = a.ws.x[o], v = a.ws.v[o];
          // v' = w v + c1 r1 (p - x) + c2 r2 (g - x);  x' = x + v'
          const double inertia = a.w * v;
          const double cog = (a.c1 * ua) * (a.ws.px[o] - x0);
          const double soc = (a.c2 * ub) * (gxj[c] - x0);
          const double vn = (inertia + cog) + soc;
          x[c] = x0 + vn;
          a.ws.v[o] = vn;
          a.ws.x[o] = x[c];
        }
        xs[jj] = x[c];
      }
      wave_sync();
      if (live) {
        const double f = group_value_slots<OBJ, G, CPL, double>(L, d, xs);
        bool improved = true;
        double pf = f;
        if (t > 0) {
          const double old = a.ws.pf[i];
          improved = rank_key(f) < rank_key(old);  // personal best, strict
          pf = improved ? f : old;
          if (improved)
#pragma unroll
            for (int c = 0; c < CPL; ++c)
              if (j + G * c < d) a.ws.px[i * d + j + G * c] = x[c];
        }
        if (j == 0) {
          if (improved) a.ws.pf[i] = pf;
          if (key_less(rank_key(pf), i, key, idx)) {
            key = rank_key(pf);
            idx = i;
            val = pf;
          }
        }
      }
      wave_sync();  // the group's LDS is reused by its next particle
    }
  }
  block_argmin<NT>(key, idx, val, unused);
  // stage (1): this block's result and its winner's personal-best position
  // (written by this block in this launch, so visible after the barrier)
  const int slot = t & 1;
  if (threadIdx.x == 0) {
    a.ws.part_key[slot * P + blk] = key;
    a.ws.part_idx[slot * P + blk] = idx;
    a.ws.part_f[slot * P + blk] = val;
  }
  if (idx != INT64_MAX)
    for (int jj = threadIdx.x; jj < d; jj += NT)
      a.ws.part_x[((size_t)slot * P + blk) * d + jj] = a.ws.px[idx * d + jj];
}

}  // namespace
}  // namespace zeus
