// user_objective.hpp -- oracle side of user-defined objectives (test
// infrastructure).  The user's source is written over a number type T that is
// double or zeus::Dual, with zsin, zcos, zexp, zlog, zsqrt; here those are the
// oracle's own: dual numbers by the rules of Sec. III-C (a double k taking
// part as the dual number (k, 0)) over the oracle's sin, cos, exp and log.
// oracle/user.py compiles a user source with this header into a shared
// library whose two entry points are registered with zo_set_user.
#pragma once

#include <cmath>

extern "C" {
double zo_sin(double x);
double zo_cos(double x);
double zo_exp(double x);
double zo_log(double x);
}

#define ZEUS_FN inline

namespace zeus {

struct Dual {
  double v, t;  // value, tangent
  Dual() = default;
  Dual(double c) : v(c), t(0.0) {}
  Dual(double v_, double t_) : v(v_), t(t_) {}
};

// (a + b eps) +- (c + e eps) = (a +- c) + (b +- e) eps
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.t + b.t); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.t - b.t); }
// (a + b eps)(c + e eps) = ac + (a e + b c) eps
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.v * b.t + a.t * b.v); }
// (a + b eps) / (c + e eps) = a / c + (b c - a e) / c^2 eps
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.t * b.v - a.v * b.t) / (b.v * b.v)); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.t); }
inline Dual operator+(Dual a, double k) { return a + Dual(k); }
inline Dual operator+(double k, Dual a) { return Dual(k) + a; }
inline Dual operator-(Dual a, double k) { return a - Dual(k); }
inline Dual operator-(double k, Dual a) { return Dual(k) - a; }
inline Dual operator*(Dual a, double k) { return a * Dual(k); }
inline Dual operator*(double k, Dual a) { return Dual(k) * a; }
inline Dual operator/(Dual a, double k) { return a / Dual(k); }
inline Dual operator/(double k, Dual a) { return Dual(k) / a; }

inline double zsin(double a) { return zo_sin(a); }
inline double zcos(double a) { return zo_cos(a); }
inline double zexp(double a) { return zo_exp(a); }
inline double zlog(double a) { return zo_log(a); }
inline double zsqrt(double a) { return std::sqrt(a); }
// sin(a + b eps) = sin a + b cos a eps;  cos(a + b eps) = cos a - b sin a eps
inline Dual zsin(Dual a) { return Dual(zo_sin(a.v), a.t * zo_cos(a.v)); }
inline Dual zcos(Dual a) { return Dual(zo_cos(a.v), -(a.t * zo_sin(a.v))); }
// exp(a + b eps) = e^a + b e^a eps;  log(a + b eps) = log a + b / a eps
inline Dual zexp(Dual a) {
  const double e = zo_exp(a.v);
  return Dual(e, a.t * e);
}
inline Dual zlog(Dual a) { return Dual(zo_log(a.v), a.t / a.v); }
// sqrt(a + b eps) = sqrt a + b / (2 sqrt a) eps
inline Dual zsqrt(Dual a) {
  const double s = std::sqrt(a.v);
  return Dual(s, a.t / (2.0 * s));
}

}  // namespace zeus

using zeus::Dual;
using zeus::zcos;
using zeus::zexp;
using zeus::zlog;
using zeus::zsin;
using zeus::zsqrt;
