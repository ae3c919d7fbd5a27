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
// row_mirror) that stay inside rows of 16 lanes; the last two use the gfx950
// lane swaps between the halves of 32- and 64-lane blocks (no LDS round
// trip).  Callers must have every lane of the block active.
// ---------------------------------------------------------------------------
// Every lane's source lane is valid for the permutations used here and all
// rows and banks are written, so no "old" value is needed: mov_dpp leaves it
// undefined and the compiler does not seed the destination first (which
// cost two extra moves per level of a double butterfly).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm(1,0,3,2)
constexpr int kDppXor2 = 0x4E;        // quad_perm(2,3,0,1)
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within 16

// Sum across the two halves of every aligned block of 2 * HALF lanes
// (HALF = 16 or 32), from two values per lane: a lane in a lower half returns
// its own a plus the a of the lane HALF above it, a lane in an upper half the
// b of the lane HALF below it plus its own b.  v_permlane{16,32}_swap moves
// the upper half of its first operand into the lower half of its second and
// back, so the two results of a swap of (a, b) hold exactly those operands.
template <int HALF>
__device__ __forceinline__ void lane_swap(uint32_t &x, uint32_t &y) {
  static_assert(HALF == 16 || HALF == 32, "HALF must be 16 or 32");
  if constexpr (HALF == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  }
}
template <int HALF>
__device__ __forceinline__ float half_pair_sum(float a, float b) {
  uint32_t x = __builtin_bit_cast(uint32_t, a), y = __builtin_bit_cast(uint32_t, b);
  lane_swap<HALF>(x, y);
  return __builtin_bit_cast(float, x) + __builtin_bit_cast(float, y);
}
template <int HALF>
__device__ __forceinline__ double half_pair_sum(double a, double b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  uint32_t xl = (uint32_t)ua, yl = (uint32_t)ub, xh = (uint32_t)(ua >> 32), yh = (uint32_t)(ub >> 32);
  lane_swap<HALF>(xl, yl);
  lane_swap<HALF>(xh, yh);
  return __builtin_bit_cast(double, ((uint64_t)xh << 32) | xl) +
         __builtin_bit_cast(double, ((uint64_t)yh << 32) | yl);
}

template <int N, class T>
__device__ __forceinline__ T lane_tree_sum(T v) {
  static_assert(N >= 1 && N <= 64 && (N & (N - 1)) == 0, "N must be a power of two <= 64");
  if constexpr (N >= 2) v = v + dpp_move<kDppXor1>(v);
  if constexpr (N >= 4) v = v + dpp_move<kDppXor2>(v);
  if constexpr (N >= 8) v = v + dpp_move<kDppHalfMirror>(v);
  if constexpr (N >= 16) v = v + dpp_move<kDppMirror>(v);
  if constexpr (N >= 32) v = half_pair_sum<16>(v, v);
  if constexpr (N >= 64) v = half_pair_sum<32>(v, v);
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
// The inverse Hessian of a start, G x G (zero-padded past the dimension, with
// ones on the padded diagonal), spread over the G lanes of its group in
// tiles: with C = min(G, 16) columns and R = G / C rows per tile, lane j
// holds rows (j mod C) + C t, t < R, at columns C * (j / C) + k, k < C.  For
// G <= 16 that is row j whole.
//
// A row's product with a vector is a fused multiply-add chain over each block
// of 16 consecutive columns, the block sums added pairwise.  In the tile
// layout a lane forms one chain for each of its R rows, and the R = 2 or 4
// blocks of a row meet in one or two lane-swap levels (16 lanes apart, then
// 32): level one adds blocks (0, 1) and (2, 3), level two their sums, which
// is the pairwise tree; each level also halves the rows a lane carries, so
// that lane j ends with row j.
//
// The vectors the tiles read (y or g, u, s) sit in the group's LDS with two
// doubles of padding after every 16, so that the four column blocks read by
// one instruction fall in different banks.
// ---------------------------------------------------------------------------
// LDS operands are read in chunks, the next chunk's loads written before the
// current chunk's arithmetic, so that the scheduler issues them early and a
// wave waits for LDS about once per chunk.
template <int N>
__device__ __forceinline__ void lds_load(double (&b)[N], const double *v) {
#pragma unroll
  for (int c = 0; c < N; ++c) b[c] = v[c];
}

// Row broadcasts for the tiles: v_fmac_f64 with DPP row_newbcast:K on its
// first operand multiplies by the value of lane K of the lane's row of 16
// lanes.  In a tile with 16 columns per row, the lane at position K of a row
// holds entry K of the row's 16-column block of a vector, which is what
// every lane of the row needs for its column K, so the products and the
// update read their vector operands from registers, not LDS.  Each asm
// statement starts with s_nop 1: a DPP read needs two wait states after a
// VALU write of its source.  Wait states and operand order are the only
// difference from __builtin_fma: fma(a, b, c) == fma(b, a, c) bit for bit.
template <int K>
struct IntK {
  static constexpr int value = K;
};
template <int K, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (K < N) {
    f(IntK<K>{});
    static_for<K + 1, N>(f);
  }
}

// acc_t += bcast_K(v) * h_t for the R = 1, 2 or 4 rows of a tile column
template <int K>
__device__ __forceinline__ void fmac_bcast(double &a0, double v, double h0) {
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
      : "+v"(a0)
      : "v"(v), "v"(h0), "n"(K));
}
template <int K>
__device__ __forceinline__ void fmac_bcast(double &a0, double &a1, double v, double h0, double h1) {
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %2, %3 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %2, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf"
      : "+v"(a0), "+v"(a1)
      : "v"(v), "v"(h0), "v"(h1), "n"(K));
}
template <int K>
__device__ __forceinline__ void fmac_bcast(double &a0, double &a1, double &a2, double &a3, double v,
                                           double h0, double h1, double h2, double h3) {
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %4, %5 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %4, %6 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %4, %7 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %4, %8 row_newbcast:%9 row_mask:0xf bank_mask:0xf"
      : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
      : "v"(v), "v"(h0), "v"(h1), "v"(h2), "v"(h3), "n"(K));
}
// x_t = fma(e_t, bcast_K(s), fma(a_t, bcast_K(u), x_t)) for the rows of a tile column
template <int K>
__device__ __forceinline__ void upd_bcast(double &x0, double u, double s, double a0, double e0) {
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %1, %3 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %2, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf"
      : "+v"(x0)
      : "v"(u), "v"(s), "v"(a0), "v"(e0), "n"(K));
}
template <int K>
__device__ __forceinline__ void upd_bcast(double &x0, double &x1, double u, double s, double a0,
                                          double a1, double e0, double e1) {
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %2, %4 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %2, %5 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %3, %6 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %3, %7 row_newbcast:%8 row_mask:0xf bank_mask:0xf"
      : "+v"(x0), "+v"(x1)
      : "v"(u), "v"(s), "v"(a0), "v"(a1), "v"(e0), "v"(e1), "n"(K));
}
template <int K>
__device__ __forceinline__ void upd_bcast(double &x0, double &x1, double &x2, double &x3, double u,
                                          double s, const double (&a)[4], const double (&e)[4]) {
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %4, %6 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %4, %7 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %4, %8 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %4, %9 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %5, %10 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %5, %11 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %5, %12 row_newbcast:%14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %5, %13 row_newbcast:%14 row_mask:0xf bank_mask:0xf"
      : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3)
      : "v"(u), "v"(s), "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(e[0]), "v"(e[1]),
        "v"(e[2]), "v"(e[3]), "n"(K));
}

template <int G>
constexpr int kTileCols = G < 16 ? G : 16;
template <int G>
constexpr int kTileRows = G / kTileCols<G>;
// doubles of a padded tile operand vector
__host__ __device__ constexpr int tile_vec_len(int G) { return G <= 16 ? G : G + 2 * (G / 16); }

// LDS position of coordinate c in a tile operand vector
template <int G>
__device__ __forceinline__ int vpos(int c) {
  return G <= 16 ? c : c + 2 * (c >> 4);
}

template <int G>
struct Tile {
  double h[kTileRows<G> * kTileCols<G>];  // h[t * C + k] = H(row(t), col(k))
  static constexpr int C = kTileCols<G>, R = kTileRows<G>;
  __device__ __forceinline__ static int row(int j, int t) { return (j % C) + C * t; }
  __device__ __forceinline__ static int col(int j, int k) { return C * (j / C) + k; }

  // The identity pattern depends on the lane only; an opaque copy of the
  // lane index keeps the compiler from hoisting the G comparisons out of the
  // start loop and holding them in registers for the whole kernel (they are
  // needed once per start).
  __device__ __forceinline__ static int opaque(int j) {
    asm volatile("" : "+v"(j));
    return j;
  }

  __device__ __forceinline__ void identity(int j) {
    j = opaque(j);
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
      for (int k = 0; k < C; ++k) h[t * C + k] = row(j, t) == col(j, k) ? 1.0 : 0.0;
  }

  // The same for a tile that holds the block of a larger matrix whose first
  // row is r0 and first column c0 (the identity's block there: its ones lie
  // on the diagonal of the larger matrix).
  __device__ __forceinline__ void identity_at(int j, int r0, int c0) {
    j = opaque(j);
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
      for (int k = 0; k < C; ++k) h[t * C + k] = r0 + row(j, t) == c0 + col(j, k) ? 1.0 : 0.0;
  }

  // Puts the padding (row or column >= d) back to the identity's.
  __device__ __forceinline__ void restore_padding(int j, int d) {
    j = opaque(j);
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
      for (int k = 0; k < C; ++k)
        if (row(j, t) >= d || col(j, k) >= d) h[t * C + k] = row(j, t) == col(j, k) ? 1.0 : 0.0;
  }

  __device__ __forceinline__ void restore_padding_at(int j, int d, int r0, int c0) {
    j = opaque(j);
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const int r = r0 + row(j, t), c = c0 + col(j, k);
        if (r >= d || c >= d) h[t * C + k] = r == c ? 1.0 : 0.0;
      }
  }

  // (H v)_j for lane j; v in the padded layout (vpos).  For G > 16 the rows
  // are finished across lanes, so every lane of the group must call it (not
  // under a condition that differs between the group's lanes).
  __device__ __forceinline__ double matvec(const double *v, int j) const {
    constexpr int CH = R == 1 ? C : 8, NC = C / CH;
    const double *vb = v + vpos<G>(col(j, 0));
    double buf[2][CH];
    double part[R];
#pragma unroll
    for (int t = 0; t < R; ++t) part[t] = 0.0;
    lds_load(buf[0], vb);
#pragma unroll
    for (int kc = 0; kc < NC; ++kc) {
      if (kc + 1 < NC) lds_load(buf[(kc + 1) & 1], vb + (kc + 1) * CH);
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int t = 0; t < R; ++t)
          part[t] = __builtin_fma(h[t * C + kc * CH + c], buf[kc & 1][c], part[t]);
    }
    if constexpr (R == 1) {
      return part[0];
    } else if constexpr (R == 2) {
      return half_pair_sum<16>(part[0], part[1]);
    } else {
      static_assert(R == 4, "tiles have 1, 2 or 4 rows");
      const double q0 = half_pair_sum<16>(part[0], part[1]);
      const double q1 = half_pair_sum<16>(part[2], part[3]);
      return half_pair_sum<32>(q0, q1);
    }
  }

  // The same product with the vector's entry of column col(j, k) taken from
  // lane k of the lane's row of 16 (row broadcasts): vc is the vector's entry
  // of column col(j, 0) + (j mod 16), i.e. of this lane's position in its
  // block (for a tile of the whole matrix, lane j's own entry).  Needs 16
  // columns per tile row (G >= 16).
  __device__ __forceinline__ double matvec_bcast(double vc) const {
    static_assert(C == 16, "row broadcasts need 16 columns per tile row");
    double part[R];
#pragma unroll
    for (int t = 0; t < R; ++t) part[t] = 0.0;
    static_for<0, C>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      if constexpr (R == 4)
        fmac_bcast<k>(part[0], part[1], part[2], part[3], vc, h[k], h[C + k], h[2 * C + k], h[3 * C + k]);
      else if constexpr (R == 2)
        fmac_bcast<k>(part[0], part[1], vc, h[k], h[C + k]);
      else
        fmac_bcast<k>(part[0], vc, h[k]);
    });
    if constexpr (R == 1) {
      return part[0];
    } else if constexpr (R == 2) {
      return half_pair_sum<16>(part[0], part[1]);
    } else {
      const double q0 = half_pair_sum<16>(part[0], part[1]);
      const double q1 = half_pair_sum<16>(part[2], part[3]);
      return half_pair_sum<32>(q0, q1);
    }
  }

  // H <- H - rho (s u' + u s') + beta s s', element (r, c) by
  // fma(e_r, s_c, fma(a_r, u_c, H_rc)) with a_r = -rho s_r and
  // e_r = beta s_r - rho u_r; u and s in the padded layout, sj and uj this
  // lane's own entries.  Returns false when some a_r or e_r is not finite
  // (then the padding must be restored).
  __device__ __forceinline__ bool rank2(double rho, double beta, const double *us, const double *ss,
                                        int j, double sj, double uj) {
    return rank2_rc(rho, beta, us, ss, us, ss, j, sj, uj);
  }

  // The update with the columns' entries of u and s taken by row broadcasts
  // (uc, sc: the entries of this lane's position in its block, as for
  // matvec_bcast); the rows' entries are read from ur_v and sr_v (padded
  // layout, from the tile's first row) when R > 1, else they are uj and sj.
  __device__ __forceinline__ bool rank2_bcast(double rho, double beta, const double *ur_v,
                                              const double *sr_v, double uc, double sc, int j,
                                              double sj, double uj) {
    static_assert(C == 16, "row broadcasts need 16 columns per tile row");
    double a[R], e[R];
    bool fin = true;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const double sr = R == 1 ? sj : sr_v[vpos<G>(row(j, t))];
      const double ur = R == 1 ? uj : ur_v[vpos<G>(row(j, t))];
      a[t] = -rho * sr;
      e[t] = beta * sr - rho * ur;
      fin = fin && __builtin_isfinite(a[t]) && __builtin_isfinite(e[t]);
    }
    static_for<0, C>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      if constexpr (R == 4)
        upd_bcast<k>(h[k], h[C + k], h[2 * C + k], h[3 * C + k], uc, sc, a, e);
      else if constexpr (R == 2)
        upd_bcast<k>(h[k], h[C + k], uc, sc, a[0], a[1], e[0], e[1]);
      else
        upd_bcast<k>(h[k], uc, sc, a[0], e[0]);
    });
    return fin;
  }

  // The update of a tile that holds a block of a larger matrix: the rows'
  // entries of u and s are read from ur_v and sr_v, the columns' from us and
  // ss (each in the padded layout, from the block's first row or column).
  __device__ __forceinline__ bool rank2_rc(double rho, double beta, const double *ur_v,
                                           const double *sr_v, const double *us,
                                           const double *ss, int j, double sj, double uj) {
    double a[R], e[R];
    bool fin = true;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const double sr = R == 1 ? sj : sr_v[vpos<G>(row(j, t))];
      const double ur = R == 1 ? uj : ur_v[vpos<G>(row(j, t))];
      a[t] = -rho * sr;
      e[t] = beta * sr - rho * ur;
      fin = fin && __builtin_isfinite(a[t]) && __builtin_isfinite(e[t]);
    }
    constexpr int CH = R == 1 ? (C > 1 ? C / 2 : 1) : 4, NC = C / CH;
    const double *ub = us + vpos<G>(col(j, 0));
    const double *sb = ss + vpos<G>(col(j, 0));
    double bu[2][CH], bs[2][CH];
    lds_load(bu[0], ub);
    lds_load(bs[0], sb);
#pragma unroll
    for (int kc = 0; kc < NC; ++kc) {
      if (kc + 1 < NC) {
        lds_load(bu[(kc + 1) & 1], ub + (kc + 1) * CH);
        lds_load(bs[(kc + 1) & 1], sb + (kc + 1) * CH);
      }
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int t = 0; t < R; ++t) {
          double &x = h[t * C + kc * CH + c];
          x = __builtin_fma(e[t], bs[kc & 1][c], __builtin_fma(a[t], bu[kc & 1][c], x));
        }
    }
    return fin;
  }
};

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
  if constexpr (whole_form<E>::value) {
    return E::template value<T>(xs, d);
  } else {
  const int m = E::terms(d);
  T blk[E::K][CPL];
#pragma unroll
  for (int r = 0; r < CPL; ++r) {
    const int i = L.j + G * r;
    // evaluated on every slot (index clamped), zero past the last term
    T w[E::W], out[E::K];
#pragma unroll
    for (int q = 0; q < E::W; ++q) w[q] = (T)xs[i + q < G * CPL ? i + q : G * CPL - 1];
    E::template term<T>(w, out);
#pragma unroll
    for (int k = 0; k < E::K; ++k) blk[k][r] = lane_tree_sum<G, T>(i < m ? out[k] : T(0));
  }
  T s[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) s[k] = reg_tree_sum<CPL, T>(blk[k]);
  return (double)E::template outer<T>(d, s);
  }
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
  const int j = L.j;
  if constexpr (whole_form<E>::value) {
    // Alg. 5 as written: one evaluation on dual numbers seeded with e_j
    double g;
    const double f = E::template value_grad<T>(xs, d, j < d ? j : -1, &g);
    *gj = j < d ? g : 0.0;
    return f;
  } else {
  static_assert(E::W <= 2, "the tangent sum assumes at most two terms per coordinate");
  const int m = E::terms(d);
  T tan[E::K], val[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) {
    tan[k] = T(0);
    val[k] = T(0);
  }
  // Both window positions are evaluated on every lane (indices clamped into
  // the vector) and a term that does not exist contributes an exact zero
  // afterwards, so the loads are not behind branches.
#pragma unroll
  for (int back = E::W - 1; back >= 0; --back) {
    const int i = j - back;  // term i holds x_j at window slot `back`
    const bool valid = j < d && i >= 0 && i < m;
    dual<T> w[E::W], out[E::K];
#pragma unroll
    for (int q = 0; q < E::W; ++q) {
      int iq = i + q < 0 ? 0 : i + q;
      iq = iq < G ? iq : G - 1;
      w[q] = dual<T>{(T)xs[iq], q == back ? T(1) : T(0)};
    }
    E::template term<dual<T>>(w, out);
#pragma unroll
    for (int k = 0; k < E::K; ++k) tan[k] = tan[k] + (valid ? out[k].t : T(0));
    if (back == 0)
#pragma unroll
      for (int k = 0; k < E::K; ++k) val[k] = valid ? out[k].v : T(0);
  }
  dual<T> sd[E::K];
#pragma unroll
  for (int k = 0; k < E::K; ++k) sd[k] = dual<T>{lane_tree_sum<G, T>(val[k]), tan[k]};
  const dual<T> r = E::template outer<dual<T>>(d, sd);
  *gj = (j < d) ? (double)r.t : 0.0;
  return (double)r.v;
  }
}

}  // namespace zeus
