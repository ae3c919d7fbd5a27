// zeus_group.h -- a group of G lanes (G a power of two, G <= 64, so a group
// never spans two wavefronts) working on one particle or one start.  Lane j
// owns coordinate j; the group exchanges whole vectors through its own slice
// of LDS and reduces across its lanes in registers.
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

// ---------------------------------------------------------------------------
// Sums.  Every sum over an objective's terms or over coordinates is the
// balanced pairwise sum: a sum of n > 1 values is the sum of its first h
// values plus the sum of the rest, h the largest power of two below n.  Over
// a zero-padded power-of-two block of P >= n slots this is the complete
// binary tree ((v0 + v1) + (v2 + v3)) + ..., because a subtree holding only
// padding contributes an exact zero (x + 0 == x up to the sign of a zero).
//
// Across lanes the tree is a butterfly: at each level a lane adds the partial
// sum of the lane that mirrors it in the next larger aligned block.  IEEE
// addition is commutative, so both partners get the same bits and after
// log2(N) levels every lane of an aligned N-lane block holds the block's sum.
// The first four levels use DPP lane permutations (quad_perm, row_half_mirror,
// row_mirror) that stay inside rows of 16 lanes; the last two go through
// ds_bpermute.  Callers must have every lane of the block active.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm(1,0,3,2)
constexpr int kDppXor2 = 0x4E;        // quad_perm(2,3,0,1)
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within 16

template <int N, class T>
__device__ __forceinline__ T lane_tree_sum(T v) {
  static_assert(N >= 1 && N <= 64 && (N & (N - 1)) == 0, "N must be a power of two <= 64");
  if constexpr (N >= 2) v = v + dpp_move<kDppXor1>(v);
  if constexpr (N >= 4) v = v + dpp_move<kDppXor2>(v);
  if constexpr (N >= 8) v = v + dpp_move<kDppHalfMirror>(v);
  if constexpr (N >= 16) v = v + dpp_move<kDppMirror>(v);
  if constexpr (N >= 32) v = v + __shfl_xor(v, 16, 64);
  if constexpr (N >= 64) v = v + __shfl_xor(v, 32, 64);
  return v;
}

// Pairwise sum of B (a power of two) consecutive values held by one lane.
template <int B, class T>
__device__ __forceinline__ T reg_tree_sum(const T *v) {
  if constexpr (B == 1) {
    return v[0];
  } else {
    return reg_tree_sum<B / 2, T>(v) + reg_tree_sum<B / 2, T>(v + B / 2);
  }
}

// ---------------------------------------------------------------------------
// Row j of H against vectors that every lane reads from the group's LDS.  The
// vectors are read in chunks, the next chunk's loads written before the
// current chunk's arithmetic, so that the scheduler issues them early and a
// wave waits for LDS about once per chunk instead of once per pair of
// elements.
// ---------------------------------------------------------------------------
template <int G>
constexpr int kRowChunk = G < 16 ? G : 16;

template <int N>
__device__ __forceinline__ void lds_load(double (&b)[N], const double *v) {
#pragma unroll
  for (int c = 0; c < N; ++c) b[c] = v[c];
}

// sum_c h[c] v[c] as one fused multiply-add chain in column order.
template <int G>
__device__ __forceinline__ double row_dot(const double (&h)[G], const double *v) {
  constexpr int CH = kRowChunk<G>, NC = G / CH;
  double buf[2][CH];
  lds_load(buf[0], v);
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (k + 1 < NC) lds_load(buf[(k + 1) & 1], v + (k + 1) * CH);
#pragma unroll
    for (int c = 0; c < CH; ++c) acc = __builtin_fma(h[k * CH + c], buf[k & 1][c], acc);
  }
  return acc;
}

// h[c] <- fma(as, s[c], fma(au, u[c], h[c])) for every column c.
template <int G>
__device__ __forceinline__ void row_rank2(double (&h)[G], double au, const double *u, double as,
                                          const double *s) {
  constexpr int CH = kRowChunk<G> / 2 > 0 ? kRowChunk<G> / 2 : 1, NC = G / CH;
  double bu[2][CH], bs[2][CH];
  lds_load(bu[0], u);
  lds_load(bs[0], s);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (k + 1 < NC) {
      lds_load(bu[(k + 1) & 1], u + (k + 1) * CH);
      lds_load(bs[(k + 1) & 1], s + (k + 1) * CH);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c)
      h[k * CH + c] = __builtin_fma(as, bs[k & 1][c], __builtin_fma(au, bu[k & 1][c], h[k * CH + c]));
  }
}

// Value of the objective at the point whose coordinates are xs[0..d-1] in the
// group's LDS, evaluated in number type T.  The group covers G * CPL term
// slots: lane c evaluates the terms c, c + G, ..., c + (CPL-1) G (zero past
// the last term); each block of G consecutive slots is summed by the lane
// butterfly and the CPL block sums are added pairwise, which is the pairwise
// tree over all G * CPL slots.  All lanes of the group must call it.
template <int OBJ, int G, int CPL, class T>
__device__ __forceinline__ double group_value_slots(const GroupLanes<G> &L, int d,
                                                    const double *xs) {
  using E = Elem<OBJ>;
  const int m = E::terms(d);
  T blk[E::K][CPL];
#pragma unroll
  for (int r = 0; r < CPL; ++r) {
    const int i = L.j + G * r;
    T out[E::K];
#pragma unroll
    for (int k = 0; k < E::K; ++k) out[k] = T(0);
    if (i < m) {
      T w[E::W];
#pragma unroll
      for (int q = 0; q < E::W; ++q) w[q] = (T)xs[i + q];
      E::template term<T>(w, out);
    }
#pragma unroll
    for (int k = 0; k < E::K; ++k) blk[k][r] = lane_tree_sum<G, T>(out[k]);
  }
  T s[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) s[k] = reg_tree_sum<CPL, T>(blk[k]);
  return (double)E::template outer<T>(d, s);
}

template <int OBJ, int G, class T>
__device__ __forceinline__ double group_value(const GroupLanes<G> &L, int d, const double *xs) {
  return group_value_slots<OBJ, G, 1, T>(L, d, xs);
}

// Value and gradient at xs (forward mode, Alg. 5) in number type T: lane
// j < d returns df/dx_j in *gj (0 for j >= d); every lane returns f.  Lane j
// evaluates on dual numbers seeded with e_j the terms whose window holds x_j
// (in ascending term order) and keeps its own term's value for the shared
// sums.  Every other term of Alg. 5's pass j has a zero tangent, and with at
// most two nonzero tangents (window W <= 2) the pairwise sum of pass j adds
// exactly these, so lane j gets the tangent of the full pass j.
template <int OBJ, int G, class T>
__device__ __forceinline__ double group_value_grad(const GroupLanes<G> &L, int d,
                                                   const double *xs, double *gj) {
  using E = Elem<OBJ>;
  static_assert(E::W <= 2, "the tangent sum assumes at most two terms per coordinate");
  const int m = E::terms(d);
  const int j = L.j;
  T tan[E::K], val[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) {
    tan[k] = T(0);
    val[k] = T(0);
  }
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
          for (int k = 0; k < E::K; ++k) val[k] = out[k].v;
      }
    }
  }
  dual<T> sd[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) sd[k] = dual<T>{lane_tree_sum<G, T>(val[k]), tan[k]};
  const dual<T> r = E::template outer<dual<T>>(d, sd);
  *gj = (j < d) ? (double)r.t : 0.0;
  return (double)r.v;
}

}  // namespace zeus
