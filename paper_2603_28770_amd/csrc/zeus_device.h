// zeus_device.h -- device-side building blocks for gfx950: the counter-based
// random stream, dual numbers and the objectives (written once, templated on
// the number type so that the same code gives primal values and, on dual
// numbers, directional derivatives).
//
// All code here is compiled with -ffp-contract=off: every multiply and add
// rounds separately unless a kernel asks for a fused multiply-add explicitly
// with __builtin_fma.  Each objective is split into per-term values and an
// outer function of their sums; the kernels add the terms by the balanced
// pairwise tree, so an evaluation rounds exactly as a plain sequential
// evaluation with pairwise sums does.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zeus {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Stateless: every draw is
// a pure function of (counter, key), generated in registers when needed
// (the on-demand generation of Sec. IV-A, without stored generator states).
// ---------------------------------------------------------------------------
struct u64x4 {
  uint64_t w[4];
};

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kMul1 = 0xCA5A826395121157ull;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(kMul0, c0), lo0 = kMul0 * c0;
    const uint64_t hi1 = __umul64hi(kMul1, c2), lo1 = kMul1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return u64x4{{c0, c1, c2, c3}};
}

// Word q (0..3) of a block without indexing a register array at run time.
__device__ __forceinline__ uint64_t word(const u64x4 &b, int q) {
  return q == 0 ? b.w[0] : q == 1 ? b.w[1] : q == 2 ? b.w[2] : b.w[3];
}

// 64 random bits -> double in [0, 1): top 53 bits times 2^-53 (exact).
__device__ __forceinline__ double u01(uint64_t w) {
  return static_cast<double>(w >> 11) * (1.0 / 9007199254740992.0);
}

// Stream tags: the fourth counter word.
enum : uint64_t { kTagX0 = 0, kTagV0 = 1, kTagR1 = 2, kTagR2 = 3 };

// ---------------------------------------------------------------------------
// Dual numbers a + b eps, eps^2 = 0 (Sec. III-C).  T = double or float.
// ---------------------------------------------------------------------------
template <class T>
struct dual {
  T v, t;  // value, tangent
};

template <class T>
__device__ __forceinline__ dual<T> operator+(dual<T> a, dual<T> b) {
  return {a.v + b.v, a.t + b.t};
}
template <class T>
__device__ __forceinline__ dual<T> operator-(dual<T> a, dual<T> b) {
  return {a.v - b.v, a.t - b.t};
}
// (a + b eps)(c + e eps) = ac + (ae + bc) eps
template <class T>
__device__ __forceinline__ dual<T> operator*(dual<T> a, dual<T> b) {
  return {a.v * b.v, a.v * b.t + a.t * b.v};
}

// Mixed constant/number operations, one overload set per number type.
__device__ __forceinline__ double scale(double k, double a) { return k * a; }
__device__ __forceinline__ float scale(float k, float a) { return k * a; }
template <class T>
__device__ __forceinline__ dual<T> scale(T k, dual<T> a) { return {k * a.v, k * a.t}; }

__device__ __forceinline__ double divk(double a, double k) { return a / k; }
__device__ __forceinline__ float divk(float a, float k) { return a / k; }
template <class T>
__device__ __forceinline__ dual<T> divk(dual<T> a, T k) { return {a.v / k, a.t / k}; }

__device__ __forceinline__ double addk(double k, double a) { return k + a; }
__device__ __forceinline__ float addk(float k, float a) { return k + a; }
template <class T>
__device__ __forceinline__ dual<T> addk(T k, dual<T> a) { return {k + a.v, a.t}; }

__device__ __forceinline__ double ksub(double k, double a) { return k - a; }
__device__ __forceinline__ float ksub(float k, float a) { return k - a; }
template <class T>
__device__ __forceinline__ dual<T> ksub(T k, dual<T> a) { return {k - a.v, -a.t}; }

// ---------------------------------------------------------------------------
// sin, cos, exp in double: Cody-Waite argument reduction (Cody and Waite,
// "Software Manual for the Elementary Functions", 1980) and the Taylor series
// of the reduced argument by Horner's rule with fused multiply-adds (about
// one ulp).  Every rounding step is explicit, so the value does not depend on
// the device math library (from |x| = 2^48 on sin and cos are NaN, see sincos).
// ---------------------------------------------------------------------------
namespace zm {
constexpr double kPio2A = 0x1.921fb54442d18p+0;   // pi/2 = A + B + C
constexpr double kPio2B = 0x1.1a62633145c07p-54;
constexpr double kPio2C = -0x1.f1976b7ed8fbcp-110;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kLn2A = 0x1.62e42fefa39efp-1;    // ln 2 = A + B
constexpr double kLn2B = 0x1.abc9e3b39803fp-56;
constexpr double kLog2e = 0x1.71547652b82fep+0;
constexpr double kTrigMax = 0x1p48;

__device__ __forceinline__ double sin_taylor(double r) {  // |r| <= pi/4, to r^17
  const double z = r * r;
  double p = 1.0 / 355687428096000.0;
  p = __builtin_fma(p, z, -1.0 / 1307674368000.0);
  p = __builtin_fma(p, z, 1.0 / 6227020800.0);
  p = __builtin_fma(p, z, -1.0 / 39916800.0);
  p = __builtin_fma(p, z, 1.0 / 362880.0);
  p = __builtin_fma(p, z, -1.0 / 5040.0);
  p = __builtin_fma(p, z, 1.0 / 120.0);
  p = __builtin_fma(p, z, -1.0 / 6.0);
  return __builtin_fma(r * z, p, r);
}

__device__ __forceinline__ double cos_taylor(double r) {  // |r| <= pi/4, to r^16
  const double z = r * r;
  double q = 1.0 / 20922789888000.0;
  q = __builtin_fma(q, z, -1.0 / 87178291200.0);
  q = __builtin_fma(q, z, 1.0 / 479001600.0);
  q = __builtin_fma(q, z, -1.0 / 3628800.0);
  q = __builtin_fma(q, z, 1.0 / 40320.0);
  q = __builtin_fma(q, z, -1.0 / 720.0);
  q = __builtin_fma(q, z, 1.0 / 24.0);
  q = __builtin_fma(q, z, -1.0 / 2.0);
  return __builtin_fma(z, q, 1.0);
}

// x = k pi/2 + r for |x| < 2^48, where k = rint(x 2/pi) is the nearest
// integer and each fused step rounds at the remainder's magnitude (accurate to
// about an ulp of 1); from 2^48 on, and for non-finite x, sin and cos are NaN.
// No library call: its large-argument reduction would raise the register
// use of every kernel this is inlined into.
__device__ __forceinline__ void sincos(double x, double &s, double &c) {
  if (!(__builtin_fabs(x) < kTrigMax)) {
    s = c = __builtin_nan("");
    return;
  }
  const double k = __builtin_rint(x * kTwoOverPi);  // x = k pi/2 + r
  double r = __builtin_fma(-k, kPio2A, x);
  r = __builtin_fma(-k, kPio2B, r);
  r = __builtin_fma(-k, kPio2C, r);
  const double sr = sin_taylor(r), cr = cos_taylor(r);
  const int q = (int)(k - 4.0 * __builtin_floor(k * 0.25));
  s = (q == 0) ? sr : (q == 1) ? cr : (q == 2) ? -sr : -cr;
  c = (q == 0) ? cr : (q == 1) ? -sr : (q == 2) ? -cr : sr;
}

__device__ __forceinline__ double exp(double x) {
  if (x != x) return x;
  if (x > 710.0) return __builtin_huge_val();
  if (x < -746.0) return 0.0;
  const double k = __builtin_rint(x * kLog2e);  // x = k ln2 + r
  double r = __builtin_fma(-k, kLn2A, x);
  r = __builtin_fma(-k, kLn2B, r);
  double p = 1.0 / 6227020800.0;
  p = __builtin_fma(p, r, 1.0 / 479001600.0);
  p = __builtin_fma(p, r, 1.0 / 39916800.0);
  p = __builtin_fma(p, r, 1.0 / 3628800.0);
  p = __builtin_fma(p, r, 1.0 / 362880.0);
  p = __builtin_fma(p, r, 1.0 / 40320.0);
  p = __builtin_fma(p, r, 1.0 / 5040.0);
  p = __builtin_fma(p, r, 1.0 / 720.0);
  p = __builtin_fma(p, r, 1.0 / 120.0);
  p = __builtin_fma(p, r, 1.0 / 24.0);
  p = __builtin_fma(p, r, 1.0 / 6.0);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return __builtin_ldexp(p, (int)k);
}
}  // namespace zm

__device__ __forceinline__ double dcos(double a) {
  double s, c;
  zm::sincos(a, s, c);
  return c;
}
// FP32 (mixed precision): the hardware sine, cosine and exponential
// (v_sin_f32, v_cos_f32, v_exp_f32; absolute error around 1e-6 for moderate
// arguments), with the library functions beyond |x| = 2^10.  FP32 results only
// steer a start until it escalates to FP64 near its minimum.
__device__ __forceinline__ void sincos32(float a, float &s, float &c) {
  if (__builtin_fabsf(a) <= 1024.0f) {
    __sincosf(a, &s, &c);
  } else {
    sincosf(a, &s, &c);
  }
}
__device__ __forceinline__ float dcos(float a) {
  float s, c;
  sincos32(a, s, c);
  return c;
}
__device__ __forceinline__ double dexp(double a) { return zm::exp(a); }
__device__ __forceinline__ float dexp(float a) { return __expf(a); }
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float dsqrt(float a) { return sqrtf(a); }

// cos(a + b eps) = cos a - b sin a eps
__device__ __forceinline__ dual<double> dcos(dual<double> a) {
  double s, c;
  zm::sincos(a.v, s, c);
  return {c, -(a.t * s)};
}
__device__ __forceinline__ dual<float> dcos(dual<float> a) {
  float s, c;
  sincos32(a.v, s, c);
  return {c, -(a.t * s)};
}
// exp(a + b eps) = e^a + b e^a eps
template <class T>
__device__ __forceinline__ dual<T> dexp(dual<T> a) {
  const T e = dexp(a.v);
  return {e, a.t * e};
}
// sqrt(a + b eps) = sqrt a + b / (2 sqrt a) eps
template <class T>
__device__ __forceinline__ dual<T> dsqrt(dual<T> a) {
  const T s = dsqrt(a.v);
  return {s, a.t / (T(2) * s)};
}

template <class N> struct scalar_of { using type = N; };
template <class T> struct scalar_of<dual<T>> { using type = T; };

template <class N>
__device__ __forceinline__ N make_const(typename scalar_of<N>::type c);
template <>
__device__ __forceinline__ double make_const<double>(double c) { return c; }
template <>
__device__ __forceinline__ float make_const<float>(float c) { return c; }
template <>
__device__ __forceinline__ dual<double> make_const<dual<double>>(double c) { return {c, 0.0}; }
template <>
__device__ __forceinline__ dual<float> make_const<dual<float>>(float c) { return {c, 0.0f}; }

// ---------------------------------------------------------------------------
// Objectives (Sec. V-B; Styblinski-Tang; sphere and quartic for tests), in
// element form: every objective here is partially separable,
//     f(x) = outer(S_0, ..., S_{K-1}),   S_k = sum_{i<m} phi_k(x_i, .., x_{i+W-1}),
// with m terms of window W.  A term is written once over a number type N
// (double, float or their dual numbers), so the same code gives values and,
// seeded with a unit tangent, directional derivatives (Sec. III-C).
//
// The kernels evaluate the terms in parallel (one lane per term) and then add
// the term values up in index order, so a value is the same sum, operation for
// operation, as a left-to-right evaluation of the whole function.  For the
// gradient, lane j evaluates on dual numbers seeded with e_j only the (at most
// W) terms whose window contains x_j: every other term of Alg. 5's pass j has a
// zero tangent, and adding exact zeros changes no nonzero sum, so lane j gets
// the same tangent as the full pass j.
// ---------------------------------------------------------------------------
enum Objective : int {
  kRosenbrock = 0,
  kRastrigin = 1,
  kAckley = 2,
  kStyblinskiTang = 3,
  kGoldsteinPrice = 4,
  kSphere = 5,
  kQuartic = 6,
  kUser = 7  // a user objective compiled at run time (zeus_user.h)
};

template <int OBJ>
struct Elem;

// An objective in "whole" form (user code, no term structure) declares
// kWhole = true and provides value / value_grad / trial evaluations; the
// kernels then evaluate it as one function instead of term by term.
template <class E, class = void>
struct whole_form {
  static constexpr bool value = false;
};
template <class E>
struct whole_form<E, decltype(void(E::kWhole))> {
  static constexpr bool value = E::kWhole;
};

// sum_{i<d-1} (1 - x_i)^2 + 100 (x_{i+1} - x_i^2)^2
template <>
struct Elem<kRosenbrock> {
  static constexpr int K = 1, W = 2;
  __host__ __device__ __forceinline__ static int terms(int d) { return d - 1; }
  template <class N>
  __device__ __forceinline__ static void term(const N *w, N *out) {
    using S = typename scalar_of<N>::type;
    const N a = ksub(S(1), w[0]);
    const N b = w[1] - w[0] * w[0];
    out[0] = a * a + scale(S(100), b * b);
  }
  template <class N>
  __device__ __forceinline__ static N outer(int, const N *s) { return s[0]; }
};

// 10 d + sum (x_i^2 - 10 cos(2 pi x_i))
template <>
struct Elem<kRastrigin> {
  static constexpr int K = 1, W = 1;
  __host__ __device__ __forceinline__ static int terms(int d) { return d; }
  template <class N>
  __device__ __forceinline__ static void term(const N *w, N *out) {
    using S = typename scalar_of<N>::type;
    const N c = dcos(scale(S(6.283185307179586), w[0]));
    out[0] = w[0] * w[0] - scale(S(10), c);
  }
  template <class N>
  __device__ __forceinline__ static N outer(int d, const N *s) {
    using S = typename scalar_of<N>::type;
    return addk(S(10) * S(d), s[0]);
  }
};

// -20 exp(-0.2 sqrt(sum x^2 / d)) - exp(sum cos(2 pi x) / d) + 20 + e
template <>
struct Elem<kAckley> {
  static constexpr int K = 2, W = 1;
  __host__ __device__ __forceinline__ static int terms(int d) { return d; }
  template <class N>
  __device__ __forceinline__ static void term(const N *w, N *out) {
    using S = typename scalar_of<N>::type;
    out[0] = w[0] * w[0];
    out[1] = dcos(scale(S(6.283185307179586), w[0]));
  }
  template <class N>
  __device__ __forceinline__ static N outer(int d, const N *s) {
    using S = typename scalar_of<N>::type;
    const N a = scale(S(-20), dexp(scale(S(-0.2), dsqrt(divk(s[0], S(d))))));
    const N b = dexp(divk(s[1], S(d)));
    N r = a - b;
    r = addk(S(20), r);
    r = addk(S(2.718281828459045), r);
    return r;
  }
};

// 0.5 sum (x^4 - 16 x^2 + 5 x)
template <>
struct Elem<kStyblinskiTang> {
  static constexpr int K = 1, W = 1;
  __host__ __device__ __forceinline__ static int terms(int d) { return d; }
  template <class N>
  __device__ __forceinline__ static void term(const N *w, N *out) {
    using S = typename scalar_of<N>::type;
    const N x2 = w[0] * w[0];
    const N x4 = x2 * x2;
    out[0] = (x4 - scale(S(16), x2)) + scale(S(5), w[0]);
  }
  template <class N>
  __device__ __forceinline__ static N outer(int, const N *s) {
    using S = typename scalar_of<N>::type;
    return scale(S(0.5), s[0]);
  }
};

// Goldstein-Price, d = 2: one term over the whole window
template <>
struct Elem<kGoldsteinPrice> {
  static constexpr int K = 1, W = 2;
  __host__ __device__ __forceinline__ static int terms(int) { return 1; }
  template <class N>
  __device__ __forceinline__ static void term(const N *w, N *out) {
    using S = typename scalar_of<N>::type;
    const N x1 = w[0], x2 = w[1];
    const N a = addk(S(1), x1 + x2);
    N pa = ksub(S(19), scale(S(14), x1));
    pa = pa + scale(S(3), x1 * x1);
    pa = pa - scale(S(14), x2);
    pa = pa + scale(S(6), x1 * x2);
    pa = pa + scale(S(3), x2 * x2);
    const N A = addk(S(1), (a * a) * pa);
    const N b = scale(S(2), x1) - scale(S(3), x2);
    N pb = ksub(S(18), scale(S(32), x1));
    pb = pb + scale(S(12), x1 * x1);
    pb = pb + scale(S(48), x2);
    pb = pb - scale(S(36), x1 * x2);
    pb = pb + scale(S(27), x2 * x2);
    const N B = addk(S(30), (b * b) * pb);
    out[0] = A * B;
  }
  template <class N>
  __device__ __forceinline__ static N outer(int, const N *s) { return s[0]; }
};

// 0.5 sum x^2
template <>
struct Elem<kSphere> {
  static constexpr int K = 1, W = 1;
  __host__ __device__ __forceinline__ static int terms(int d) { return d; }
  template <class N>
  __device__ __forceinline__ static void term(const N *w, N *out) { out[0] = w[0] * w[0]; }
  template <class N>
  __device__ __forceinline__ static N outer(int, const N *s) {
    using S = typename scalar_of<N>::type;
    return scale(S(0.5), s[0]);
  }
};

// sum x^4
template <>
struct Elem<kQuartic> {
  static constexpr int K = 1, W = 1;
  __host__ __device__ __forceinline__ static int terms(int d) { return d; }
  template <class N>
  __device__ __forceinline__ static void term(const N *w, N *out) {
    const N x2 = w[0] * w[0];
    out[0] = x2 * x2;
  }
  template <class N>
  __device__ __forceinline__ static N outer(int, const N *s) { return s[0]; }
};

// NaN ranks as +infinity in every best-of comparison.
__device__ __forceinline__ double rank_key(double f) {
  return (f != f) ? __builtin_huge_val() : f;
}

// (key, index) lexicographic minimum: lowest value, lowest index on ties.
struct KeyIdx {
  double key;
  int64_t idx;
};
__device__ __forceinline__ bool key_less(double ka, int64_t ia, double kb, int64_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

}  // namespace zeus
