// zeus_user.h -- user-defined objectives (the paper's f is user code: a
// function of the point, templated on the number type, Sec. III-C / IV).
//
// A user objective is C++ source compiled at run time with hipRTC together
// with this header and the kernel templates.  It defines
//
//     template <class T, class X>
//     ZEUS_FN T objective(const X &x, int d);
//
// where x[i] (i < d) yields a T, and T is double or zeus::Dual (FP64), or, for
// the FP32 evaluations of mixed precision, zeus::F32 or zeus::DualF.  It may
// use +, -, *, / between Ts and doubles (a double takes part as the dual
// number (k, 0), rounded to FP32 in the FP32 types), unary minus, and zsin,
// zcos, zexp, zlog, zsqrt; constants may sit in namespace-scope constexpr
// arrays.  The same source, compiled for the CPU against the oracle's own
// number type, gives the oracle's values.  All four instantiations are
// compiled, so the source must be generic over T (as it must already be for
// the dual numbers).
//
// The kernels see a user objective in "whole" form: no term structure is
// known, so a value is one evaluation of the function; the gradient is Alg. 5
// as written (lane j evaluates the function once on dual numbers seeded with
// e_j, so the G lanes perform the d passes together); a line-search round
// evaluates one trial per lane.
#pragma once

#include "zeus_device.h"

#define ZEUS_FN __device__ __forceinline__

namespace zeus {

// A dual number a + b eps for user code (Sec. III-C): value v, tangent t.
struct Dual {
  double v, t;
  Dual() = default;
  __device__ __forceinline__ Dual(double c) : v(c), t(0.0) {}
  __device__ __forceinline__ Dual(double v_, double t_) : v(v_), t(t_) {}
};

__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.t + b.t}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.t - b.t}; }
// (a + b eps)(c + e eps) = ac + (a e + b c) eps
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.v * b.t + a.t * b.v}; }
// (a + b eps) / (c + e eps) = a / c + (b c - a e) / c^2 eps
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.t * b.v - a.v * b.t) / (b.v * b.v)};
}
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.t}; }
__device__ __forceinline__ Dual operator+(Dual a, double k) { return a + Dual(k); }
__device__ __forceinline__ Dual operator+(double k, Dual a) { return Dual(k) + a; }
__device__ __forceinline__ Dual operator-(Dual a, double k) { return a - Dual(k); }
__device__ __forceinline__ Dual operator-(double k, Dual a) { return Dual(k) - a; }
__device__ __forceinline__ Dual operator*(Dual a, double k) { return a * Dual(k); }
__device__ __forceinline__ Dual operator*(double k, Dual a) { return Dual(k) * a; }
__device__ __forceinline__ Dual operator/(Dual a, double k) { return a / Dual(k); }
__device__ __forceinline__ Dual operator/(double k, Dual a) { return Dual(k) / a; }

namespace zm {
// Natural logarithm: x = m 2^e with sqrt(1/2) <= m < sqrt(2) (exact), then
// log m = 2 atanh(s) = 2 s + 2 s (z/3 + z^2/5 + ... + z^11/23) with
// s = (m - 1) / (m + 1), z = s^2 <= 0.0295 (the series of atanh, by Horner's
// rule with fused multiply-adds), and log x = e ln2_hi + (e ln2_lo + log m)
// with ln 2 split so that e ln2_hi is exact: ln2_hi is the double nearest
// ln 2 with its low 20 significand bits cleared, ln2_lo the double nearest
// ln 2 - ln2_hi.
constexpr double kLogLn2Hi = 0x1.62e42fefp-1;
constexpr double kLogLn2Lo = 0x1.473de6af278edp-34;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;

__device__ __forceinline__ double log(double x) {
  if (!(x > 0.0)) return x == 0.0 ? -__builtin_huge_val() : __builtin_nan("");
  if (x == __builtin_huge_val()) return x;
  int e;
  double m = __builtin_frexp(x, &e);  // x = m 2^e, 1/2 <= m < 1
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e = e - 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double p = 1.0 / 23.0;
  p = __builtin_fma(p, z, 1.0 / 21.0);
  p = __builtin_fma(p, z, 1.0 / 19.0);
  p = __builtin_fma(p, z, 1.0 / 17.0);
  p = __builtin_fma(p, z, 1.0 / 15.0);
  p = __builtin_fma(p, z, 1.0 / 13.0);
  p = __builtin_fma(p, z, 1.0 / 11.0);
  p = __builtin_fma(p, z, 1.0 / 9.0);
  p = __builtin_fma(p, z, 1.0 / 7.0);
  p = __builtin_fma(p, z, 1.0 / 5.0);
  p = __builtin_fma(p, z, 1.0 / 3.0);
  const double t = p * z;
  const double s2 = s + s;
  const double lm = __builtin_fma(s2, t, s2);
  const double k = (double)e;
  const double r = __builtin_fma(k, kLogLn2Lo, lm);
  return __builtin_fma(k, kLogLn2Hi, r);
}
}  // namespace zm

__device__ __forceinline__ double zsin(double a) {
  double s, c;
  zm::sincos(a, s, c);
  return s;
}
__device__ __forceinline__ double zcos(double a) {
  double s, c;
  zm::sincos(a, s, c);
  return c;
}
__device__ __forceinline__ double zexp(double a) { return zm::exp(a); }
__device__ __forceinline__ double zlog(double a) { return zm::log(a); }
__device__ __forceinline__ double zsqrt(double a) { return __builtin_sqrt(a); }
// sin(a + b eps) = sin a + b cos a eps
__device__ __forceinline__ Dual zsin(Dual a) {
  double s, c;
  zm::sincos(a.v, s, c);
  return {s, a.t * c};
}
// cos(a + b eps) = cos a - b sin a eps
__device__ __forceinline__ Dual zcos(Dual a) {
  double s, c;
  zm::sincos(a.v, s, c);
  return {c, -(a.t * s)};
}
// exp(a + b eps) = e^a + b e^a eps
__device__ __forceinline__ Dual zexp(Dual a) {
  const double e = zm::exp(a.v);
  return {e, a.t * e};
}
// log(a + b eps) = log a + b / a eps
__device__ __forceinline__ Dual zlog(Dual a) { return {zm::log(a.v), a.t / a.v}; }
// sqrt(a + b eps) = sqrt a + b / (2 sqrt a) eps
__device__ __forceinline__ Dual zsqrt(Dual a) {
  const double s = __builtin_sqrt(a.v);
  return {s, a.t / (2.0 * s)};
}

// FP32 numbers for the mixed-precision evaluations: every operation in FP32,
// a double operand rounded to FP32 first.  No conversion back to double, so
// a source cannot leave FP32 by accident.
struct F32 {
  float v;
  F32() = default;
  __device__ __forceinline__ F32(double c) : v((float)c) {}
  __device__ __forceinline__ static F32 of(float c) {
    F32 r;
    r.v = c;
    return r;
  }
};
__device__ __forceinline__ F32 operator+(F32 a, F32 b) { return F32::of(a.v + b.v); }
__device__ __forceinline__ F32 operator-(F32 a, F32 b) { return F32::of(a.v - b.v); }
__device__ __forceinline__ F32 operator*(F32 a, F32 b) { return F32::of(a.v * b.v); }
__device__ __forceinline__ F32 operator/(F32 a, F32 b) { return F32::of(a.v / b.v); }
__device__ __forceinline__ F32 operator-(F32 a) { return F32::of(-a.v); }
__device__ __forceinline__ F32 operator+(F32 a, double k) { return a + F32(k); }
__device__ __forceinline__ F32 operator+(double k, F32 a) { return F32(k) + a; }
__device__ __forceinline__ F32 operator-(F32 a, double k) { return a - F32(k); }
__device__ __forceinline__ F32 operator-(double k, F32 a) { return F32(k) - a; }
__device__ __forceinline__ F32 operator*(F32 a, double k) { return a * F32(k); }
__device__ __forceinline__ F32 operator*(double k, F32 a) { return F32(k) * a; }
__device__ __forceinline__ F32 operator/(F32 a, double k) { return a / F32(k); }
__device__ __forceinline__ F32 operator/(double k, F32 a) { return F32(k) / a; }

// The FP32 dual number, with the product and quotient rules of Dual.
struct DualF {
  float v, t;
  DualF() = default;
  __device__ __forceinline__ DualF(double c) : v((float)c), t(0.0f) {}
  __device__ __forceinline__ static DualF of(float v_, float t_) {
    DualF r;
    r.v = v_;
    r.t = t_;
    return r;
  }
};
__device__ __forceinline__ DualF operator+(DualF a, DualF b) { return DualF::of(a.v + b.v, a.t + b.t); }
__device__ __forceinline__ DualF operator-(DualF a, DualF b) { return DualF::of(a.v - b.v, a.t - b.t); }
__device__ __forceinline__ DualF operator*(DualF a, DualF b) {
  return DualF::of(a.v * b.v, a.v * b.t + a.t * b.v);
}
__device__ __forceinline__ DualF operator/(DualF a, DualF b) {
  return DualF::of(a.v / b.v, (a.t * b.v - a.v * b.t) / (b.v * b.v));
}
__device__ __forceinline__ DualF operator-(DualF a) { return DualF::of(-a.v, -a.t); }
__device__ __forceinline__ DualF operator+(DualF a, double k) { return a + DualF(k); }
__device__ __forceinline__ DualF operator+(double k, DualF a) { return DualF(k) + a; }
__device__ __forceinline__ DualF operator-(DualF a, double k) { return a - DualF(k); }
__device__ __forceinline__ DualF operator-(double k, DualF a) { return DualF(k) - a; }
__device__ __forceinline__ DualF operator*(DualF a, double k) { return a * DualF(k); }
__device__ __forceinline__ DualF operator*(double k, DualF a) { return DualF(k) * a; }
__device__ __forceinline__ DualF operator/(DualF a, double k) { return a / DualF(k); }
__device__ __forceinline__ DualF operator/(double k, DualF a) { return DualF(k) / a; }

// FP32 functions: sine, cosine and exponential as the built-in objectives
// take them in FP32 (hardware approximations, absolute error around 1e-6 for
// moderate arguments), the library's FP32 logarithm and square root.  FP32
// results only steer a start until it escalates to FP64 near its minimum.
__device__ __forceinline__ F32 zsin(F32 a) {
  float s, c;
  sincos32(a.v, s, c);
  return F32::of(s);
}
__device__ __forceinline__ F32 zcos(F32 a) {
  float s, c;
  sincos32(a.v, s, c);
  return F32::of(c);
}
__device__ __forceinline__ F32 zexp(F32 a) { return F32::of(dexp(a.v)); }
__device__ __forceinline__ F32 zlog(F32 a) { return F32::of(logf(a.v)); }
__device__ __forceinline__ F32 zsqrt(F32 a) { return F32::of(sqrtf(a.v)); }
__device__ __forceinline__ DualF zsin(DualF a) {
  float s, c;
  sincos32(a.v, s, c);
  return DualF::of(s, a.t * c);
}
__device__ __forceinline__ DualF zcos(DualF a) {
  float s, c;
  sincos32(a.v, s, c);
  return DualF::of(c, -(a.t * s));
}
__device__ __forceinline__ DualF zexp(DualF a) {
  const float e = dexp(a.v);
  return DualF::of(e, a.t * e);
}
__device__ __forceinline__ DualF zlog(DualF a) { return DualF::of(logf(a.v), a.t / a.v); }
__device__ __forceinline__ DualF zsqrt(DualF a) {
  const float s = sqrtf(a.v);
  return DualF::of(s, a.t / (2.0f * s));
}

// The number types of an evaluation in precision P (double or float): the
// plain number S and the dual number D.
template <class P> struct UserNum;
template <> struct UserNum<double> {
  using S = double;
  using D = Dual;
  __device__ __forceinline__ static double val(double a) { return a; }
  __device__ __forceinline__ static double val(Dual a) { return a.v; }
  __device__ __forceinline__ static double tan(Dual a) { return a.t; }
};
template <> struct UserNum<float> {
  using S = F32;
  using D = DualF;
  __device__ __forceinline__ static double val(F32 a) { return (double)a.v; }
  __device__ __forceinline__ static double val(DualF a) { return (double)a.v; }
  __device__ __forceinline__ static double tan(DualF a) { return (double)a.t; }
};

// Views of the point handed to the user's function, in precision P; the FP32
// views round each coordinate (of x, or of the trial point formed in FP64)
// to FP32, as the built-in objectives' FP32 evaluations do.
template <class P>
struct PlainView {  // the point in LDS
  const double *xs;
  __device__ __forceinline__ typename UserNum<P>::S operator[](int i) const {
    return typename UserNum<P>::S((double)(P)xs[i]);
  }
};
template <class P>
struct SeededView {  // the point as dual numbers with tangent e_j (none if j < 0)
  const double *xs;
  int j;
  __device__ __forceinline__ typename UserNum<P>::D operator[](int i) const {
    typename UserNum<P>::D r((double)(P)xs[i]);
    r.t = i == j ? 1 : 0;
    return r;
  }
};
template <class P>
struct TrialView {  // the trial point x + alpha p, each coordinate rounded
  const double *xs, *ps;
  double alpha;
  __device__ __forceinline__ typename UserNum<P>::S operator[](int i) const {
    return typename UserNum<P>::S((double)(P)(xs[i] + alpha * ps[i]));
  }
};

}  // namespace zeus

// The user's source is at namespace scope: make the number type and the
// functions visible there (for double arguments no lookup reaches zeus::).
using zeus::Dual;
using zeus::DualF;
using zeus::F32;
using zeus::zcos;
using zeus::zexp;
using zeus::zlog;
using zeus::zsin;
using zeus::zsqrt;
