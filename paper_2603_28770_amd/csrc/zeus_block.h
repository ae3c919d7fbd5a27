// zeus_block.h -- pieces shared by the block-per-start BFGS kernels (64 < d):
// one block of four or eight wavefronts runs a start.
// Lane j owns coordinate j; the block exchanges vectors through its LDS
// struct (a type with the members these helpers name: xs, ps, red, tsum,
// pass, al and q) and finishes every sum across its wavefronts there.
#pragma once

#include "zeus_bfgs_common.h"

namespace zeus {

constexpr int kBlockLanes = kWideLanes;     // lanes (threads) per start (four wavefronts)
constexpr int kBlockWaves = kBlockLanes / 64;  // wavefronts per start == trials per round
static_assert(kBlockWaves == 4, "the device-memory and on-chip blocks have four wavefronts");

// The wavefronts of the block (4 or 8), from the LDS struct's sum slots.
template <class Shm>
constexpr int shm_waves() {
  return (int)(sizeof(Shm::red[0][0]) / sizeof(double));
}

// Pairwise sum over the block's lanes (NW wavefronts of 64) of K values per
// lane: a butterfly inside each wavefront, then the NW wavefront sums added
// pairwise through LDS.  Alternating phases let one barrier per reduction
// suffice: a phase's slots are written again only two reductions later, after
// every thread has passed the barrier of the reduction in between (and so has
// read them).
template <int K, class T, class Shm>
__device__ __forceinline__ void block_tree_sums(T (&v)[K], Shm &sh, int &phase) {
  constexpr int NW = shm_waves<Shm>();
  static_assert(NW == 4 || NW == 8, "blocks of four or eight wavefronts");
  static_assert(K <= (int)(sizeof(Shm::red[0]) / sizeof(Shm::red[0][0])),
                "more sums than the LDS struct has slots for");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    v[k] = lane_tree_sum<64, T>(v[k]);
    if (lane == 0) sh.red[phase][k][w] = (double)v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double *r = sh.red[phase][k];
    const T lo = ((T)r[0] + (T)r[1]) + ((T)r[2] + (T)r[3]);
    if constexpr (NW == 4) {
      v[k] = lo;
    } else {
      v[k] = lo + (((T)r[4] + (T)r[5]) + ((T)r[6] + (T)r[7]));
    }
  }
  phase ^= 1;
}

template <class Shm>
__device__ __forceinline__ double block_tree_sum(double v, Shm &sh, int &phase) {
  double a[1] = {v};
  block_tree_sums<1, double>(a, sh, phase);
  return a[0];
}

// Objective value at xs in number type T (every thread returns it); lane j
// also returns df/dx_j in *gj when kGrad (0 beyond the dimension).  Lane j
// evaluates on dual numbers seeded with e_j the terms whose window holds x_j,
// as the narrow kernel does.
//
// acc >= 0 names the accepted trial of the line search that produced xs
// (block_armijo): its term sums, left in sh.tsum[acc], are the sums this
// evaluation would form -- the same terms at the same point (the step
// computes x + alpha p exactly as the trial did) in the same number type,
// over the same pairwise tree (the value's tree runs over every lane of the
// block, the trial's over the first SLOTS slots, and the slots between hold
// exact zeros) -- so they are taken as they are, and the sum and its
// barrier are skipped (d = 128: 89.5 -> 87.3 ms, d = 200: 231.4 -> 225.4 ms).
// acc is uniform across the block.
template <int OBJ, class T, bool kGrad, class Shm>
__device__ __forceinline__ double block_eval(int d, const double *xs, double *gj, Shm &sh,
                                             int &phase, int acc = -1) {
  using E = Elem<OBJ>;
  if constexpr (whole_form<E>::value) {
    // no term structure: Alg. 5 as written, lane j < d evaluating the whole
    // function on dual numbers seeded with e_j (pass j); the primal part is
    // the same on every lane
    const int j = threadIdx.x;
    if (!kGrad) return E::template value<T>(xs, d);
    double g;
    const double f = E::template value_grad<T>(xs, d, j < d ? j : -1, &g);
    *gj = j < d ? g : 0.0;
    return f;
  } else {
  static_assert(E::W <= 2, "the tangent sum assumes at most two terms per coordinate");
  const int m = E::terms(d);
  const int j = threadIdx.x;
  T tan[E::K], val[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) {
    tan[k] = T(0);
    val[k] = T(0);
  }
  if (kGrad) {
    if (j < d) {
#pragma unroll
      for (int back = E::W - 1; back >= 0; --back) {
        const int i = j - back;
        if (i >= 0 && i < m) {
          dual<T> w[E::W], out[E::K];
#pragma unroll
          for (int q = 0; q < E::W; ++q) w[q] = dual<T>{(T)xs[i + q], q == back ? T(1) : T(0)};
          E::template term<dual<T>>(w, out);
#pragma unroll
          for (int k = 0; k < E::K; ++k) tan[k] = tan[k] + out[k].t;
          if (back == 0)
#pragma unroll
            for (int k = 0; k < E::K; ++k) val[k] = out[k].v;
        }
      }
    }
  } else if (j < m) {
    T w[E::W];
#pragma unroll
    for (int q = 0; q < E::W; ++q) w[q] = (T)xs[j + q];
    E::template term<T>(w, val);
  }
  if (acc >= 0) {
#pragma unroll
    for (int k = 0; k < E::K; ++k) val[k] = (T)sh.tsum[acc][k];
  } else {
    block_tree_sums<E::K, T>(val, sh, phase);
  }
  if (!kGrad) return (double)E::template outer<T>(d, val);
  dual<T> sd[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) sd[k] = dual<T>{val[k], tan[k]};
  const dual<T> r = E::template outer<dual<T>>(d, sd);
  *gj = (j < d) ? (double)r.t : 0.0;
  return (double)r.v;
  }
}

// One Armijo search (Alg. 6) with the objective in number type U over SLOTS
// term slots (SLOTS a multiple of 64, at least the number of terms):
// wavefront w of the NW evaluates trial base + w of each round; lane c of it
// takes the term slots B c .. B c + B - 1 (B = SLOTS / 64) and adds them
// pairwise, the wavefront finishes the pairwise sum.  Returns the index of the
// first passing trial, or -1.  *acc receives the slot of sh.tsum that holds
// the passing trial's term sums (-1 when none passed or the objective has no
// term structure); the slot is written again two rounds later, so it holds
// until the next search's second round.
template <int OBJ, class U, int SLOTS, class Shm>
__device__ __forceinline__ int block_armijo(Shm &sh, double f, double ddir, int &lsphase,
                                            int *acc) {
  using E = Elem<OBJ>;
  static_assert(SLOTS % 64 == 0, "term slots come in whole wavefronts");
  constexpr int B = SLOTS / 64;  // term slots per lane
  constexpr int NW = shm_waves<Shm>();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const ReqHot &q = sh.q;
  const int d = q.d, m = q.m;
  static_assert(E::K <= (int)(sizeof(Shm::tsum[0]) / sizeof(Shm::tsum[0][0])),
                "more term sums than the LDS struct has slots for");
  static_assert((int)(sizeof(Shm::tsum) / sizeof(Shm::tsum[0])) == 2 * NW, "one slot per phase and wave");
  *acc = -1;
  if constexpr (whole_form<E>::value) {
    // no term structure: one trial per lane, trials base .. base + 64 NW - 1
    // in a round; wavefront w reports its first passing lane
    for (int base = 0; base < q.iter_ls; base += 64 * NW) {
      const int t = base + (int)threadIdx.x;
      bool ok = false;
      if (t < q.iter_ls) {
        const double alpha = step_length(sh.al, q.shrink, t);
        ok = E::template trial<U>(sh.xs, sh.ps, alpha, d) <= f + (q.armijo_c * alpha) * ddir;
      }
      const uint64_t hit = __ballot(ok);
      if (lane == 0) sh.pass[lsphase][w] = hit ? __ffsll((unsigned long long)hit) : 0;
      __syncthreads();
      int first = -1;
#pragma unroll
      for (int v = NW - 1; v >= 0; --v)
        if (sh.pass[lsphase][v]) first = 64 * v + sh.pass[lsphase][v] - 1;
      lsphase ^= 1;
      if (first >= 0) return base + first;
    }
    return -1;
  } else {
  for (int base = 0; base < q.iter_ls; base += NW) {
    const int t = base + w;
    const double alpha = step_length(sh.al, q.shrink, t);
    U tv[E::K][B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int i = lane * B + b;
      U out[E::K];
#pragma unroll
      for (int kk = 0; kk < E::K; ++kk) out[kk] = U(0);
      if (i < m) {
        U wv[E::W];
#pragma unroll
        for (int e = 0; e < E::W; ++e) wv[e] = (U)(sh.xs[i + e] + alpha * sh.ps[i + e]);
        E::template term<U>(wv, out);
      }
#pragma unroll
      for (int kk = 0; kk < E::K; ++kk) tv[kk][b] = out[kk];
    }
    U sums[E::K];
#pragma unroll
    for (int kk = 0; kk < E::K; ++kk) sums[kk] = lane_tree_sum<64, U>(reg_tree_sum<B, U>(tv[kk]));
    const double ft = (double)E::template outer<U>(d, sums);
    const bool ok = t < q.iter_ls && ft <= f + (q.armijo_c * alpha) * ddir;
    if (lane == 0) {
      sh.pass[lsphase][w] = ok ? 1 : 0;
#pragma unroll
      for (int kk = 0; kk < E::K; ++kk) sh.tsum[lsphase * NW + w][kk] = (double)sums[kk];
    }
    __syncthreads();
    int first = -1;
#pragma unroll
    for (int v = NW - 1; v >= 0; --v)
      if (sh.pass[lsphase][v]) first = v;
    if (first >= 0) *acc = lsphase * NW + first;
    lsphase ^= 1;
    if (first >= 0) return base + first;
  }
  return -1;
  }
}

}  // namespace zeus
