// zeus_group.h -- a group of G lanes (G a power of two, G <= 64, so a group
// never spans two wavefronts) working on one particle or one start.  Lane j
// owns coordinate j; the group exchanges vectors through its own slice of LDS.
#pragma once

#include "zeus_device.h"

namespace zeus {

// Orders this wave's LDS traffic.  LDS operations of one wavefront complete
// in issue order, so only the compiler must be kept from moving them.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int G>
struct GroupLanes {
  int j;          // lane index inside the group
  int grp;        // group index inside the wavefront
  uint64_t mask;  // this group's bits in a wavefront ballot
  __device__ __forceinline__ GroupLanes() {
    const int lane = threadIdx.x & 63;
    j = lane & (G - 1);
    grp = lane / G;
    mask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (grp * G));
  }
  // ballot of pred over the group, shifted so that bit j is lane j
  __device__ __forceinline__ uint64_t ballot(bool pred) const {
    return (__ballot(pred) & mask) >> (grp * G);
  }
};

// Index-order reductions over zero-padded LDS vectors.  Entries from n up to
// the next multiple of the chunk size CH are exact zeros, so they can be added
// without a per-element test: x + 0 == x (up to the sign of a zero result),
// and the result rounds exactly like a left-to-right loop over the first n
// entries starting from 0.0.  Each chunk's loads are issued together.
template <int G>
struct Chunk {
  static constexpr int CH = G < 8 ? G : 8;
  __device__ __forceinline__ static int padded(int n) { return (n + CH - 1) / CH * CH; }
};

template <int G, class T>
__device__ __forceinline__ T sum_ordered(const T *a, int n) {
  constexpr int CH = Chunk<G>::CH;
  T acc = T(0);
  for (int c0 = 0; c0 < n; c0 += CH) {
    T v[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) v[q] = a[c0 + q];
#pragma unroll
    for (int q = 0; q < CH; ++q) acc = acc + v[q];
  }
  return acc;
}

// sum_i a_i b_i in index order, products and sums rounded separately
template <int G>
__device__ __forceinline__ double dot_ordered(const double *a, const double *b, int n) {
  constexpr int CH = Chunk<G>::CH;
  double acc = 0.0;
  for (int c0 = 0; c0 < n; c0 += CH) {
    double va[CH], vb[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      va[q] = a[c0 + q];
      vb[q] = b[c0 + q];
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) acc = acc + va[q] * vb[q];
  }
  return acc;
}

// Sequential sums S_k = tv[k][0] + ... + tv[k][m-1] for the K term sums of a
// [K][G] term buffer whose entries from m on are zero.
template <int K, int G, class T>
__device__ __forceinline__ void ordered_sums(const T *tv, int m, T *s) {
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = sum_ordered<G, T>(tv + k * G, m);
}

// Value of the objective at the point whose coordinates are xs[0..d-1] in the
// group's LDS, evaluated in number type T: lane c < m evaluates term c and
// stores it in tv[k*G + c], then every lane adds the terms up in index order.
// tv[k*G + c] must be zero for c >= m.  All lanes of the group must call it.
template <int OBJ, int G, class T>
__device__ __forceinline__ double group_value(const GroupLanes<G> &L, int d, const double *xs,
                                              T *tv) {
  using E = Elem<OBJ>;
  const int m = E::terms(d);
  if (L.j < m) {
    T w[E::W], out[E::K];
#pragma unroll
    for (int q = 0; q < E::W; ++q) w[q] = (T)xs[L.j + q];
    E::template term<T>(w, out);
#pragma unroll
    for (int k = 0; k < E::K; ++k) tv[k * G + L.j] = out[k];
  }
  wave_sync();
  T s[E::K];
  ordered_sums<E::K, G, T>(tv, m, s);
  return (double)E::template outer<T>(d, s);
}

// Value and gradient at xs (forward mode, Alg. 5) in number type T: lane
// j < d returns df/dx_j in *gj; every lane returns f.  Lane j evaluates on
// dual numbers seeded with e_j the terms whose window holds x_j (in ascending
// term order, the order in which the full pass adds them), and its own term's
// value for the shared sums.
template <int OBJ, int G, class T>
__device__ __forceinline__ double group_value_grad(const GroupLanes<G> &L, int d,
                                                   const double *xs, T *tv, double *gj) {
  using E = Elem<OBJ>;
  const int m = E::terms(d);
  const int j = L.j;
  T tan[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) tan[k] = T(0);
  if (j < d) {
#pragma unroll
    for (int back = E::W - 1; back >= 0; --back) {
      const int i = j - back;  // term i holds x_j at window slot `back`
      if (i >= 0 && i < m) {
        dual<T> w[E::W], out[E::K];
#pragma unroll
        for (int q = 0; q < E::W; ++q) w[q] = dual<T>{(T)xs[i + q], q == back ? T(1) : T(0)};
        E::template term<dual<T>>(w, out);
#pragma unroll
        for (int k = 0; k < E::K; ++k) tan[k] = tan[k] + out[k].t;
        if (back == 0)
#pragma unroll
          for (int k = 0; k < E::K; ++k) tv[k * G + j] = out[k].v;
      }
    }
  }
  wave_sync();
  T sv[E::K];
  ordered_sums<E::K, G, T>(tv, m, sv);
  dual<T> sd[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) sd[k] = dual<T>{sv[k], tan[k]};
  const dual<T> r = E::template outer<dual<T>>(d, sd);
  *gj = (j < d) ? (double)r.t : 0.0;
  return (double)r.v;
}

}  // namespace zeus
