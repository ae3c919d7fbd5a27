// zeus_block.h -- pieces shared by the two block-per-start BFGS kernels
// (64 < d): one block of kBlockLanes lanes (four wavefronts) runs a start.
// Lane j owns coordinate j; the block exchanges vectors through its LDS
// struct (a type with the members these helpers name: xs, ps, red, pass, al
// and q) and finishes every sum across its four wavefronts there.
#pragma once

#include "zeus_bfgs_common.h"

namespace zeus {

constexpr int kBlockLanes = kWideLanes;     // lanes (threads) per start
constexpr int kBlockWaves = kBlockLanes / 64;  // wavefronts per start == trials per round
static_assert(kBlockWaves == 4, "the pairwise combination of wave sums assumes four waves");

// Pairwise sum over the block's 256 lanes of K values per lane: a butterfly
// inside each wavefront, then the four wavefront sums added pairwise through
// LDS.  Alternating phases let one barrier per reduction suffice: a phase's
// slots are written again only two reductions later, after every thread has
// passed the barrier of the reduction in between (and so has read them).
template <int K, class T, class Shm>
__device__ __forceinline__ void block_tree_sums(T (&v)[K], Shm &sh, int &phase) {
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
    v[k] = ((T)r[0] + (T)r[1]) + ((T)r[2] + (T)r[3]);
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
template <int OBJ, class T, bool kGrad, class Shm>
__device__ __forceinline__ double block_eval(int d, const double *xs, double *gj, Shm &sh,
                                             int &phase) {
  using E = Elem<OBJ>;
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
  block_tree_sums<E::K, T>(val, sh, phase);
  if (!kGrad) return (double)E::template outer<T>(d, val);
  dual<T> sd[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) sd[k] = dual<T>{val[k], tan[k]};
  const dual<T> r = E::template outer<dual<T>>(d, sd);
  *gj = (j < d) ? (double)r.t : 0.0;
  return (double)r.v;
}

// One Armijo search (Alg. 6) with the objective in number type U over SLOTS
// term slots (SLOTS a multiple of 64, at least the number of terms):
// wavefront w evaluates trial base + w of each round; lane c of it takes the
// term slots B c .. B c + B - 1 (B = SLOTS / 64) and adds them pairwise, the
// wavefront finishes the pairwise sum.  Returns the index of the first
// passing trial, or -1.
template <int OBJ, class U, int SLOTS, class Shm>
__device__ __forceinline__ int block_armijo(Shm &sh, double f, double ddir, int &lsphase) {
  using E = Elem<OBJ>;
  static_assert(SLOTS % 64 == 0, "term slots come in whole wavefronts");
  constexpr int B = SLOTS / 64;  // term slots per lane
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const ReqHot &q = sh.q;
  const int d = q.d, m = q.m;
  for (int base = 0; base < q.iter_ls; base += kBlockWaves) {
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
    if (lane == 0) sh.pass[lsphase][w] = ok ? 1 : 0;
    __syncthreads();
    int first = -1;
#pragma unroll
    for (int v = kBlockWaves - 1; v >= 0; --v)
      if (sh.pass[lsphase][v]) first = v;
    lsphase ^= 1;
    if (first >= 0) return base + first;
  }
  return -1;
}

}  // namespace zeus
