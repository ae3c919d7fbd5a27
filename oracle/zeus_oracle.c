/*
 * zeus_oracle.c -- plain CPU oracle (TEST INFRASTRUCTURE ONLY; see header).
 *
 * Follows the paper's algorithms step by step:
 *   Sec. IV-A      on-demand counter-based random numbers (Philox replaces the
 *                  paper's cuRAND states; one draw per start, iteration,
 *                  stream and dimension)
 *   Alg. 2         swarm initialisation
 *   Alg. 3 / 9     swarm update, applied synchronously (see zo_pso)
 *   Alg. 4 / 10    BFGS with the rank-2 inverse-Hessian update
 *   Alg. 5         forward-mode AD with dual numbers, one pass per direction
 *   Alg. 6         Armijo backtracking line search
 *   Alg. 7         final best-of-N reduction
 * Objectives: Sec. V-B (Rosenbrock, Rastrigin, Ackley, Goldstein-Price) plus
 * the standard Styblinski-Tang function and two test-only objectives.
 *
 * Two builds of this one file:
 *   default        the order of every rounding is fixed by the readings
 *                  written next to the code (balanced pairwise sums, 16-column
 *                  fused row products, the two-FMA update, sin/cos/exp by
 *                  Cody-Waite reduction and Taylor series);
 *   -DZO_PLAIN     the textbook order instead: sums strictly left to right,
 *                  row products and the update unfused in index order, and
 *                  the C library's sin, cos, exp and log.  It takes no reading
 *                  of the paper's silences that a particular implementation
 *                  of the method could have chosen for its own convenience.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fopenmp -fPIC -shared [-DZO_PLAIN]
 */
#include "zeus_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ======================================================================== */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As   */
/* Easy as 1, 2, 3", SC'11): 10 rounds of the 4x64 S-box, key bumped by the  */
/* Weyl constants between rounds.                                           */
/* ======================================================================== */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void zo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                      uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, &hi0, &lo0);
    mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double zo_uniform(uint64_t seed, uint64_t request_id, uint64_t i, uint64_t t,
                  uint64_t tag, uint64_t j) {
  uint64_t ctr[4] = {j / 4, i, t, tag};
  uint64_t key[2] = {seed, request_id};
  uint64_t out[4];
  zo_philox4x64_10(ctr, key, out);
  /* top 53 bits scaled by 2^-53: a double in [0, 1) */
  return (double)(out[j % 4] >> 11) * (1.0 / 9007199254740992.0);
}

#ifdef ZO_PLAIN
/* ======================================================================== */
/* Plain build: sin, cos, exp and log are the C library's.                  */
/* ======================================================================== */
static void zo_sincos(double x, double *s, double *c) {
  *s = sin(x);
  *c = cos(x);
}
double zo_sin(double x) { return sin(x); }
double zo_cos(double x) { return cos(x); }
double zo_exp(double x) { return exp(x); }
double zo_log(double x) { return log(x); }
#else
/* ======================================================================== */
/* sin, cos and exp in double precision, by Cody-Waite argument reduction    */
/* (Cody and Waite, "Software Manual for the Elementary Functions", 1980)    */
/* followed by the Taylor series of the reduced argument, evaluated by       */
/* Horner's rule with fused multiply-adds.  Accurate to about one ulp.  The  */
/* objectives use these instead of the C library so that their rounding is   */
/* specified here, operation by operation.                                  */
/* ======================================================================== */

/* pi/2 as an unevaluated sum of three doubles, and 2/pi rounded. */
static const double ZM_PIO2_1 = 0x1.921fb54442d18p+0;
static const double ZM_PIO2_2 = 0x1.1a62633145c07p-54;
static const double ZM_PIO2_3 = -0x1.f1976b7ed8fbcp-110;
static const double ZM_2_OVER_PI = 0x1.45f306dc9c883p-1;
/* ln 2 as a sum of two doubles, and log2(e) rounded. */
static const double ZM_LN2_1 = 0x1.62e42fefa39efp-1;
static const double ZM_LN2_2 = 0x1.abc9e3b39803fp-56;
static const double ZM_LOG2E = 0x1.71547652b82fep+0;

/* sin r and cos r for |r| <= pi/4 (Taylor series to r^17 and r^16). */
static double sin_taylor(double r) {
  double z = r * r;
  double p = 1.0 / 355687428096000.0;     /*  1/17! */
  p = fma(p, z, -1.0 / 1307674368000.0);  /* -1/15! */
  p = fma(p, z, 1.0 / 6227020800.0);      /*  1/13! */
  p = fma(p, z, -1.0 / 39916800.0);       /* -1/11! */
  p = fma(p, z, 1.0 / 362880.0);          /*  1/9!  */
  p = fma(p, z, -1.0 / 5040.0);           /* -1/7!  */
  p = fma(p, z, 1.0 / 120.0);             /*  1/5!  */
  p = fma(p, z, -1.0 / 6.0);              /* -1/3!  */
  return fma(r * z, p, r);
}

static double cos_taylor(double r) {
  double z = r * r;
  double q = 1.0 / 20922789888000.0;      /*  1/16! */
  q = fma(q, z, -1.0 / 87178291200.0);    /* -1/14! */
  q = fma(q, z, 1.0 / 479001600.0);       /*  1/12! */
  q = fma(q, z, -1.0 / 3628800.0);        /* -1/10! */
  q = fma(q, z, 1.0 / 40320.0);           /*  1/8!  */
  q = fma(q, z, -1.0 / 720.0);            /* -1/6!  */
  q = fma(q, z, 1.0 / 24.0);              /*  1/4!  */
  q = fma(q, z, -1.0 / 2.0);              /* -1/2!  */
  return fma(z, q, 1.0);
}

/* x = k pi/2 + r, |r| <= pi/4 (about).  Each fused multiply-add rounds once
 * at the magnitude of the running remainder, so with pi/2 split in three
 * doubles the reduced argument is accurate to about an ulp of 1 as long as
 * k = rint(x 2/pi) is the nearest integer, which holds with margin below
 * |x| = 2^48 (ulp(x 2/pi) <= 1/16).  The paper does not say how large
 * arguments are handled; here sin and cos are NaN from |x| = 2^48 on (and for
 * an infinity or NaN), so an objective evaluated there is non-finite. */
static const double ZM_TRIG_MAX = 0x1p48;

static void zo_sincos(double x, double *s, double *c) {
  if (!(fabs(x) < ZM_TRIG_MAX)) {
    *s = *c = NAN;
    return;
  }
  double k = rint(x * ZM_2_OVER_PI);
  double r = fma(-k, ZM_PIO2_1, x);
  r = fma(-k, ZM_PIO2_2, r);
  r = fma(-k, ZM_PIO2_3, r);
  double sr = sin_taylor(r), cr = cos_taylor(r);
  double q = k - 4.0 * floor(k * 0.25);
  switch ((int)q) {
    case 0: *s = sr; *c = cr; break;
    case 1: *s = cr; *c = -sr; break;
    case 2: *s = -sr; *c = -cr; break;
    default: *s = -cr; *c = sr; break;
  }
}

double zo_sin(double x) { double s, c; zo_sincos(x, &s, &c); return s; }
double zo_cos(double x) { double s, c; zo_sincos(x, &s, &c); return c; }

double zo_exp(double x) {
  if (x != x) return x;
  if (x > 710.0) return INFINITY;
  if (x < -746.0) return 0.0;
  /* x = k ln2 + r, |r| <= ln2/2; e^x = 2^k e^r */
  double k = rint(x * ZM_LOG2E);
  double r = fma(-k, ZM_LN2_1, x);
  r = fma(-k, ZM_LN2_2, r);
  double p = 1.0 / 6227020800.0;          /* 1/13! */
  p = fma(p, r, 1.0 / 479001600.0);       /* 1/12! */
  p = fma(p, r, 1.0 / 39916800.0);        /* 1/11! */
  p = fma(p, r, 1.0 / 3628800.0);         /* 1/10! */
  p = fma(p, r, 1.0 / 362880.0);          /* 1/9!  */
  p = fma(p, r, 1.0 / 40320.0);           /* 1/8!  */
  p = fma(p, r, 1.0 / 5040.0);            /* 1/7!  */
  p = fma(p, r, 1.0 / 720.0);             /* 1/6!  */
  p = fma(p, r, 1.0 / 120.0);             /* 1/5!  */
  p = fma(p, r, 1.0 / 24.0);              /* 1/4!  */
  p = fma(p, r, 1.0 / 6.0);               /* 1/3!  */
  p = fma(p, r, 0.5);                     /* 1/2!  */
  p = fma(p, r, 1.0);                     /* 1/1!  */
  p = fma(p, r, 1.0);                     /* 1/0!  */
  return ldexp(p, (int)k);
}

/* Natural logarithm.  x = m 2^e with sqrt(1/2) <= m < sqrt(2) (frexp, then
 * one doubling), log m = 2 atanh(s) with s = (m - 1)/(m + 1): the atanh
 * series 2 s (1 + z/3 + z^2/5 + ... + z^11/23), z = s^2 <= 0.0295, summed by
 * Horner's rule with fused multiply-adds as 2s + 2s (z/3 + ...), and
 * log x = e ln2_hi + (e ln2_lo + log m), where ln2_hi is ln 2 rounded to a
 * double with its low 20 significand bits cleared (so e ln2_hi is exact) and
 * ln2_lo the double nearest ln 2 - ln2_hi. */
#define ZM_LOG_LN2_HI 0x1.62e42fefp-1
#define ZM_LOG_LN2_LO 0x1.473de6af278edp-34
#define ZM_SQRT_HALF 0x1.6a09e667f3bcdp-1

double zo_log(double x) {
  if (!(x > 0.0)) return x == 0.0 ? -INFINITY : NAN;
  if (x == INFINITY) return x;
  int e;
  double m = frexp(x, &e);
  if (m < ZM_SQRT_HALF) {
    m = m * 2.0;
    e = e - 1;
  }
  double f = m - 1.0;
  double s = f / (2.0 + f);
  double z = s * s;
  double p = 1.0 / 23.0;
  p = fma(p, z, 1.0 / 21.0);
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  double t2 = p * z;
  double s2 = s + s;
  double lm = fma(s2, t2, s2);
  double k = (double)e;
  double r = fma(k, ZM_LOG_LN2_LO, lm);
  return fma(k, ZM_LOG_LN2_HI, r);
}
#endif /* ZO_PLAIN */

/* ======================================================================== */
/* Dual numbers a + b*eps with eps^2 = 0 (Sec. III-C).  v = value, t = tangent.*/
/* ======================================================================== */

typedef struct { double v, t; } dual;

static dual dd(double v, double t) { dual r; r.v = v; r.t = t; return r; }
static dual d_add(dual a, dual b) { return dd(a.v + b.v, a.t + b.t); }
static dual d_sub(dual a, dual b) { return dd(a.v - b.v, a.t - b.t); }
/* (a + b eps)(c + e eps) = ac + (ae + bc) eps */
static dual d_mul(dual a, dual b) { return dd(a.v * b.v, a.v * b.t + a.t * b.v); }
/* constant k times dual */
static dual d_scale(double k, dual a) { return dd(k * a.v, k * a.t); }
/* dual divided by constant k */
static dual d_divk(dual a, double k) { return dd(a.v / k, a.t / k); }
/* constant k plus / minus dual */
static dual d_addk(double k, dual a) { return dd(k + a.v, a.t); }
static dual d_ksub(double k, dual a) { return dd(k - a.v, -a.t); }
/* cos(a + b eps) = cos a - b sin a eps */
static dual d_cos(dual a) {
  double sv, cv;
  zo_sincos(a.v, &sv, &cv);
  return dd(cv, -(a.t * sv));
}
/* exp(a + b eps) = e^a + b e^a eps */
static dual d_exp(dual a) { double e = zo_exp(a.v); return dd(e, a.t * e); }
/* sqrt(a + b eps) = sqrt a + b / (2 sqrt a) eps */
static dual d_sqrt(dual a) { double s = sqrt(a.v); return dd(s, a.t / (2.0 * s)); }

/* ======================================================================== */
/* Sums.  The paper fixes no order for the sums over an objective's terms or */
/* over coordinates (dot products).  Default build: every such sum is a      */
/* balanced pairwise sum -- a sum of n > 1 values is the sum of its first h  */
/* values plus the sum of the remaining n - h, h being the largest power of  */
/* two below n; a sum of one value is that value.  Plain build: strictly     */
/* left to right, ((v0 + v1) + v2) + ...                                    */
/* ======================================================================== */

#ifndef ZO_PLAIN
static int pw_split(int n) {
  int h = 1;
  while (2 * h < n) h *= 2;
  return h;
}
#endif

/* sum_{i<n} a_i b_i, each product rounded, then summed */
static double pw_dot(const double *a, const double *b, int n) {
  if (n <= 0) return 0.0;
#ifdef ZO_PLAIN
  double acc = a[0] * b[0];
  for (int i = 1; i < n; ++i) acc = acc + a[i] * b[i];
  return acc;
#else
  if (n == 1) return a[0] * b[0];
  int h = pw_split(n);
  return pw_dot(a, b, h) + pw_dot(a + h, b + h, n - h);
#endif
}

/* Products of a row of the inverse Hessian with a vector (u = H y in the
 * update, p = -H g for the direction; Alg. 4).  The paper fixes no order for
 * these sums either.  Default build: the columns fall into blocks of
 * ZO_HBLOCK consecutive columns (the last block may be shorter); each block's
 * products are accumulated left to right by fused multiply-adds, starting
 * from zero, and the block sums are added pairwise as above.  For
 * dim <= ZO_HBLOCK this is one fused multiply-add chain over the row.  Plain
 * build: sum_c hrow[c] v[c] with every product rounded, columns ascending. */
#ifdef ZO_PLAIN
double zo_hrow_dot(const double *hrow, const double *v, int d) {
  double acc = 0.0;
  for (int c = 0; c < d; ++c) acc = acc + hrow[c] * v[c];
  return acc;
}
#else
#define ZO_HBLOCK 16

static double hrow_blocks(const double *h, const double *v, int d, int b0, int nb) {
  if (nb == 1) {
    int c1 = (b0 + 1) * ZO_HBLOCK < d ? (b0 + 1) * ZO_HBLOCK : d;
    double acc = 0.0;
    for (int c = b0 * ZO_HBLOCK; c < c1; ++c) acc = fma(h[c], v[c], acc);
    return acc;
  }
  int hb = pw_split(nb);
  return hrow_blocks(h, v, d, b0, hb) + hrow_blocks(h, v, d, b0 + hb, nb - hb);
}

double zo_hrow_dot(const double *hrow, const double *v, int d) {
  if (d <= 0) return 0.0;
  return hrow_blocks(hrow, v, d, 0, (d + ZO_HBLOCK - 1) / ZO_HBLOCK);
}
#endif

/* sum of the terms lo .. lo+n-1 of an objective, each term a dual number */
typedef dual (*term_fn)(const dual *x, int i);
static dual pw_terms(term_fn term, const dual *x, int lo, int n) {
#ifdef ZO_PLAIN
  dual acc = term(x, lo);
  for (int i = 1; i < n; ++i) acc = d_add(acc, term(x, lo + i));
  return acc;
#else
  if (n == 1) return term(x, lo);
  int h = pw_split(n);
  return d_add(pw_terms(term, x, lo, h), pw_terms(term, x, lo + h, n - h));
#endif
}

static const double ZO_TWO_PI = 6.283185307179586;  /* 2*pi rounded to double */
static const double ZO_E = 2.718281828459045;       /* e rounded to double    */

/* ======================================================================== */
/* Objectives, each written once over dual numbers; the primal value is the  */
/* value part of an evaluation with all tangents zero.                      */
/* ======================================================================== */

/* Sec. V-B: sum_{i=1}^{d-1} [(1 - x_i)^2 + 100 (x_{i+1} - x_i^2)^2]
 * (the paper's upper index n needs x_{n+1}; the sum stops at d-1). */
static dual rosenbrock_term(const dual *x, int i) {
  dual a = d_ksub(1.0, x[i]);
  dual b = d_sub(x[i + 1], d_mul(x[i], x[i]));
  return d_add(d_mul(a, a), d_scale(100.0, d_mul(b, b)));
}
static dual obj_rosenbrock(const dual *x, int d) {
  return pw_terms(rosenbrock_term, x, 0, d - 1);
}

/* Sec. V-B: A*d + sum [x_i^2 - A cos(2 pi x_i)], A = 10. */
static dual rastrigin_term(const dual *x, int i) {
  dual c = d_cos(d_scale(ZO_TWO_PI, x[i]));
  return d_sub(d_mul(x[i], x[i]), d_scale(10.0, c));
}
static dual obj_rastrigin(const dual *x, int d) {
  return d_addk(10.0 * (double)d, pw_terms(rastrigin_term, x, 0, d));
}

/* Sec. V-B: -20 exp(-0.2 sqrt(sum x_i^2 / d)) - exp(sum cos(2 pi x_i) / d)
 *           + 20 + e. */
static dual square_term(const dual *x, int i) { return d_mul(x[i], x[i]); }
static dual cos2pi_term(const dual *x, int i) { return d_cos(d_scale(ZO_TWO_PI, x[i])); }
static dual obj_ackley(const dual *x, int d) {
  dual s1 = pw_terms(square_term, x, 0, d);
  dual s2 = pw_terms(cos2pi_term, x, 0, d);
  dual a = d_scale(-20.0, d_exp(d_scale(-0.2, d_sqrt(d_divk(s1, (double)d)))));
  dual b = d_exp(d_divk(s2, (double)d));
  dual r = d_sub(a, b);
  r = d_addk(20.0, r);
  r = d_addk(ZO_E, r);
  return r;
}

/* Styblinski-Tang: 0.5 * sum (x_i^4 - 16 x_i^2 + 5 x_i). */
static dual st_term(const dual *x, int i) {
  dual x2 = d_mul(x[i], x[i]);
  dual x4 = d_mul(x2, x2);
  return d_add(d_sub(x4, d_scale(16.0, x2)), d_scale(5.0, x[i]));
}
static dual obj_styblinski_tang(const dual *x, int d) {
  return d_scale(0.5, pw_terms(st_term, x, 0, d));
}

/* Sec. V-B: Goldstein-Price, d = 2. */
static dual obj_goldstein_price(const dual *x, int d) {
  (void)d;
  dual x1 = x[0], x2 = x[1];
  dual a = d_addk(1.0, d_add(x1, x2));
  dual pa = d_ksub(19.0, d_scale(14.0, x1));
  pa = d_add(pa, d_scale(3.0, d_mul(x1, x1)));
  pa = d_sub(pa, d_scale(14.0, x2));
  pa = d_add(pa, d_scale(6.0, d_mul(x1, x2)));
  pa = d_add(pa, d_scale(3.0, d_mul(x2, x2)));
  dual A = d_addk(1.0, d_mul(d_mul(a, a), pa));
  dual b = d_sub(d_scale(2.0, x1), d_scale(3.0, x2));
  dual pb = d_ksub(18.0, d_scale(32.0, x1));
  pb = d_add(pb, d_scale(12.0, d_mul(x1, x1)));
  pb = d_add(pb, d_scale(48.0, x2));
  pb = d_sub(pb, d_scale(36.0, d_mul(x1, x2)));
  pb = d_add(pb, d_scale(27.0, d_mul(x2, x2)));
  dual B = d_addk(30.0, d_mul(d_mul(b, b), pb));
  return d_mul(A, B);
}

/* test-only: 0.5 * sum x_i^2 */
static dual obj_sphere(const dual *x, int d) {
  return d_scale(0.5, pw_terms(square_term, x, 0, d));
}

/* test-only: sum x_i^4 */
static dual fourth_term(const dual *x, int i) {
  dual x2 = d_mul(x[i], x[i]);
  return d_mul(x2, x2);
}
static dual obj_quartic(const dual *x, int d) { return pw_terms(fourth_term, x, 0, d); }

/* User objective (ZO_USER): the value in double and one evaluation on dual
 * numbers, both from the user's source compiled for the CPU (zo_set_user). */
static zo_user_value_fn g_user_value = NULL;
static zo_user_dual_fn g_user_dual = NULL;

void zo_set_user(zo_user_value_fn value, zo_user_dual_fn dual_eval) {
  g_user_value = value;
  g_user_dual = dual_eval;
}

static dual obj_user(const dual *x, int d) {
  double *xv = (double *)malloc(sizeof(double) * (size_t)(2 * d + 1));
  double *xt = xv + d;
  for (int i = 0; i < d; ++i) {
    xv[i] = x[i].v;
    xt[i] = x[i].t;
  }
  double t = NAN;
  double v = g_user_dual ? g_user_dual(xv, xt, d, &t) : NAN;
  free(xv);
  return dd(v, t);
}

static dual eval_dual(int objective, const dual *x, int d) {
  switch (objective) {
    case ZO_USER: return obj_user(x, d);
    case ZO_ROSENBROCK: return obj_rosenbrock(x, d);
    case ZO_RASTRIGIN: return obj_rastrigin(x, d);
    case ZO_ACKLEY: return obj_ackley(x, d);
    case ZO_STYBLINSKI_TANG: return obj_styblinski_tang(x, d);
    case ZO_GOLDSTEIN_PRICE: return obj_goldstein_price(x, d);
    case ZO_SPHERE: return obj_sphere(x, d);
    case ZO_QUARTIC: return obj_quartic(x, d);
    default: return dd(NAN, NAN);
  }
}

double zo_f(int objective, const double *x, int dim) {
  if (objective == ZO_USER) return g_user_value ? g_user_value(x, dim) : NAN;
  dual *xd = (dual *)malloc(sizeof(dual) * (size_t)dim);
  for (int i = 0; i < dim; ++i) xd[i] = dd(x[i], 0.0);
  double f = eval_dual(objective, xd, dim).v;
  free(xd);
  return f;
}

/* Alg. 5: one dual pass per direction i; tangent of the result is df/dx_i. */
void zo_grad(int objective, const double *x, int dim, double *f, double *g) {
  dual *xd = (dual *)malloc(sizeof(dual) * (size_t)dim);
  for (int i = 0; i < dim; ++i) xd[i] = dd(x[i], 0.0);
  double fv = NAN;
  for (int i = 0; i < dim; ++i) {
    xd[i].t = 1.0;
    dual r = eval_dual(objective, xd, dim);
    g[i] = r.t;
    fv = r.v;
    xd[i].t = 0.0;
  }
  free(xd);
  *f = fv;
}

/* ======================================================================== */
/* Validation                                                               */
/* ======================================================================== */

int zo_validate(const zo_problem *pb) {
  if (!pb) return -1;
  if (pb->objective == ZO_USER) {
    if (!g_user_value || !g_user_dual) return -1;
  } else if (pb->objective < ZO_ROSENBROCK || pb->objective > ZO_QUARTIC) {
    return -1;
  }
  if (pb->dim < 1) return -1;
  if (pb->objective == ZO_ROSENBROCK && pb->dim < 2) return -1;
  if (pb->objective == ZO_GOLDSTEIN_PRICE && pb->dim != 2) return -1;
  if (pb->n < 1) return -1;
  if (!isfinite(pb->lower) || !isfinite(pb->upper) || !(pb->lower < pb->upper))
    return -1;
  if (pb->iter_pso < 0 || pb->iter_bfgs < 0 || pb->iter_ls < 1) return -1;
  if (!isfinite(pb->w) || !isfinite(pb->c1) || !isfinite(pb->c2) ||
      !isfinite(pb->v_half))
    return -1;
  if (!isfinite(pb->grad_tol) || !(pb->grad_tol > 0.0)) return -1;
  if (!(pb->armijo_c > 0.0 && pb->armijo_c < 1.0)) return -1;
  if (!(pb->ls_shrink > 0.0 && pb->ls_shrink < 1.0)) return -1;
  if (pb->lbfgs_m < 0) return -1;
  return 0;
}

/* ======================================================================== */
/* PSO (Alg. 2 and Alg. 3)                                                  */
/* ======================================================================== */

/* A NaN objective value ranks as +infinity in every best-comparison. */
static double rank_key(double f) { return isnan(f) ? INFINITY : f; }

static int near_tie(double a, double b) {
  double ka = rank_key(a), kb = rank_key(b);
  if (!isfinite(ka) || !isfinite(kb)) return 0;
  double m = fabs(ka) > fabs(kb) ? fabs(ka) : fabs(kb);
  return fabs(ka - kb) <= 1e-12 * m;
}

/* UniformSample(lo, hi) of Alg. 2: lo + u (hi - lo). */
static double sample_in(double u, double lo, double hi) {
  return lo + u * (hi - lo);
}

/* Global best after a sweep: lowest personal-best value, lowest index among
 * equal values (Alg. 2 scans in index order with a strict '<'). */
static int64_t argmin_pf(const double *pf, int64_t n) {
  int64_t best = 0;
  for (int64_t i = 1; i < n; ++i)
    if (rank_key(pf[i]) < rank_key(pf[best])) best = i;
  return best;
}

int zo_pso(const zo_problem *pb, zo_swarm *sw) {
  if (zo_validate(pb) != 0 || !sw) return -1;
  const int d = pb->dim;
  const int64_t n = pb->n;
  const double vh = pb->v_half > 0.0 ? pb->v_half : (pb->upper - pb->lower);
  int64_t ties = 0;

  /* Alg. 2: x ~ U(lower, upper), v ~ U(-vel_range, vel_range), pX = x,
   * pVal = f(x); global best over the initial swarm. */
  for (int64_t i = 0; i < n; ++i) {
    double *xi = sw->x + i * d, *vi = sw->v + i * d, *pi = sw->px + i * d;
    for (int j = 0; j < d; ++j) {
      double ux = zo_uniform(pb->seed, pb->request_id, (uint64_t)i, 0, ZO_TAG_X0, (uint64_t)j);
      double uv = zo_uniform(pb->seed, pb->request_id, (uint64_t)i, 0, ZO_TAG_V0, (uint64_t)j);
      xi[j] = sample_in(ux, pb->lower, pb->upper);
      vi[j] = sample_in(uv, -vh, vh);
      pi[j] = xi[j];
    }
    sw->pf[i] = zo_f(pb->objective, xi, d);
  }
  int64_t g = argmin_pf(sw->pf, n);
  for (int64_t i = 0; i < n; ++i)
    if (i != g && near_tie(sw->pf[i], sw->pf[g])) ++ties;
  sw->gf = sw->pf[g];
  sw->gidx = g;
  memcpy(sw->gx, sw->px + g * d, sizeof(double) * (size_t)d);

  /* Alg. 3, read synchronously: every particle of sweep t uses the global
   * best from the end of sweep t-1; the global best is refreshed once per
   * sweep, only on strict improvement. */
  double *gx_prev = (double *)malloc(sizeof(double) * (size_t)d);
  for (int t = 1; t <= pb->iter_pso; ++t) {
    memcpy(gx_prev, sw->gx, sizeof(double) * (size_t)d);
    for (int64_t i = 0; i < n; ++i) {
      double *xi = sw->x + i * d, *vi = sw->v + i * d, *pi = sw->px + i * d;
      for (int j = 0; j < d; ++j) {
        double r1 = zo_uniform(pb->seed, pb->request_id, (uint64_t)i, (uint64_t)t, ZO_TAG_R1, (uint64_t)j);
        double r2 = zo_uniform(pb->seed, pb->request_id, (uint64_t)i, (uint64_t)t, ZO_TAG_R2, (uint64_t)j);
        /* v' = w v + c1 r1 (p - x) + c2 r2 (g - x);  x' = x + v' */
        double inertia = pb->w * vi[j];
        double cog = (pb->c1 * r1) * (pi[j] - xi[j]);
        double soc = (pb->c2 * r2) * (gx_prev[j] - xi[j]);
        vi[j] = (inertia + cog) + soc;
        xi[j] = xi[j] + vi[j];
      }
      double fv = zo_f(pb->objective, xi, d);
      if (near_tie(fv, sw->pf[i])) ++ties;
      if (rank_key(fv) < rank_key(sw->pf[i])) {  /* personal best, strict */
        sw->pf[i] = fv;
        memcpy(pi, xi, sizeof(double) * (size_t)d);
      }
    }
    int64_t m = argmin_pf(sw->pf, n);
    if (near_tie(sw->pf[m], sw->gf) && m != sw->gidx) ++ties;
    if (rank_key(sw->pf[m]) < rank_key(sw->gf)) {  /* global best, strict */
      sw->gf = sw->pf[m];
      sw->gidx = m;
      memcpy(sw->gx, sw->px + m * d, sizeof(double) * (size_t)d);
    }
  }
  free(gx_prev);
  sw->near_ties = ties;
  return 0;
}

/* ======================================================================== */
/* BFGS pieces                                                              */
/* ======================================================================== */

static double rel_margin(double a, double b) {
  double m = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
  if (!(m > 0.0)) return 0.0;
  double r = fabs(a - b) / m;
  return isnan(r) ? INFINITY : r;
}

/* Alg. 6 with f0 = f(x) passed in and g'p precomputed: start at alpha = 1,
 * accept the first trial with f(x + alpha p) <= f0 + c alpha g'p, otherwise
 * multiply alpha by the shrink factor; at most iter_ls trials.  When no trial
 * is accepted alpha has been shrunk iter_ls times and is returned as is. */
static double line_search_m(const zo_problem *pb, const double *x, double f0,
                            const double *p, double ddir, double *xt,
                            int32_t *trials, int32_t *accepted,
                            double *margin) {
  const int d = pb->dim;
  double alpha = 1.0;
  *trials = 0;
  *accepted = 0;
  for (int tr = 0; tr < pb->iter_ls; ++tr) {
    for (int j = 0; j < d; ++j) xt[j] = x[j] + alpha * p[j];
    double ft = zo_f(pb->objective, xt, d);
    *trials += 1;
    double rhs = f0 + (pb->armijo_c * alpha) * ddir;
    double m = rel_margin(ft, rhs);
    if (margin && m < *margin) *margin = m;
    if (ft <= rhs) {
      *accepted = 1;
      break;
    }
    alpha = alpha * pb->ls_shrink;
  }
  return alpha;
}

double zo_line_search(const zo_problem *pb, const double *x, double f0,
                      const double *p, double ddir, double *xt_scratch,
                      int32_t *trials, int32_t *accepted) {
  return line_search_m(pb, x, f0, p, ddir, xt_scratch, trials, accepted, NULL);
}

/* Rank-2 update of Alg. 4,
 *   H+ = (I - rho s y') H (I - rho y s') + rho s s',  rho = 1 / (y's),
 * expanded with u = H y (H symmetric):
 *   H+ = H - rho (s u' + u s') + (rho^2 y'u + rho) s s'.
 * Skipped when y's is not > 0 (the update would divide by it). */
int zo_bfgs_update(double *H, const double *s, const double *y, int d) {
  double sy = pw_dot(y, s, d);
  if (!(sy > 0.0)) return 0;
  double rho = 1.0 / sy;
  double *u = (double *)calloc((size_t)d, sizeof(double));
  for (int i = 0; i < d; ++i) u[i] = zo_hrow_dot(H + (size_t)i * d, y, d);
  double yu = pw_dot(y, u, d);
  double beta = (rho * rho) * yu + rho;
#ifdef ZO_PLAIN
  /* H_ij - rho (s_i u_j + u_i s_j) + beta s_i s_j, as written */
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      H[i * d + j] = (H[i * d + j] - rho * (s[i] * u[j] + u[i] * s[j])) + (beta * s[i]) * s[j];
#else
  /* row i: H_ij + a_i u_j + e_i s_j with a_i = -rho s_i and
   * e_i = beta s_i - rho u_i, each element by two fused multiply-adds */
  for (int i = 0; i < d; ++i) {
    double a = -rho * s[i];
    double e = beta * s[i] - rho * u[i];
    for (int j = 0; j < d; ++j) H[i * d + j] = fma(e, s[j], fma(a, u[j], H[i * d + j]));
  }
#endif
  free(u);
  return 1;
}

/* a x + y: one fused multiply-add (default build), or rounded twice (plain) */
#ifdef ZO_PLAIN
#define AXPY(a, x, y) ((y) + (a) * (x))
#else
#define AXPY(a, x, y) fma((a), (x), (y))
#endif

void zo_lbfgs_direction(const double *S, const double *Y, const double *rho, int count,
                        const double *g, int d, double *p) {
  double *q = (double *)malloc(sizeof(double) * (size_t)d);
  double *alpha = (double *)malloc(sizeof(double) * (size_t)(count > 0 ? count : 1));
  memcpy(q, g, sizeof(double) * (size_t)d);
  /* first loop, newest pair first: alpha_i = rho_i s_i'q, q <- q - alpha_i y_i */
  for (int i = count - 1; i >= 0; --i) {
    alpha[i] = rho[i] * pw_dot(S + (size_t)i * d, q, d);
    for (int j = 0; j < d; ++j) q[j] = AXPY(-alpha[i], Y[(size_t)i * d + j], q[j]);
  }
  /* r = H0 q with H0 = gamma I */
  if (count > 0) {
    const double *sn = S + (size_t)(count - 1) * d, *yn = Y + (size_t)(count - 1) * d;
    double gamma = pw_dot(sn, yn, d) / pw_dot(yn, yn, d);
    for (int j = 0; j < d; ++j) q[j] = gamma * q[j];
  }
  /* second loop, oldest pair first: beta = rho_i y_i'r, r <- r + (alpha_i - beta) s_i */
  for (int i = 0; i < count; ++i) {
    double beta = rho[i] * pw_dot(Y + (size_t)i * d, q, d);
    for (int j = 0; j < d; ++j) q[j] = AXPY(alpha[i] - beta, S[(size_t)i * d + j], q[j]);
  }
  for (int j = 0; j < d; ++j) p[j] = -q[j];
  free(alpha);
  free(q);
}

int zo_lbfgs_push(double *S, double *Y, double *rho, int *count, int m, const double *s,
                  const double *y, int d) {
  double sy = pw_dot(y, s, d);
  if (!(sy > 0.0)) return 0;
  if (*count == m) { /* full: drop the oldest pair */
    memmove(S, S + d, sizeof(double) * (size_t)(m - 1) * d);
    memmove(Y, Y + d, sizeof(double) * (size_t)(m - 1) * d);
    memmove(rho, rho + 1, sizeof(double) * (size_t)(m - 1));
    --*count;
  }
  memcpy(S + (size_t)*count * d, s, sizeof(double) * (size_t)d);
  memcpy(Y + (size_t)*count * d, y, sizeof(double) * (size_t)d);
  rho[*count] = 1.0 / sy;
  ++*count;
  return 1;
}

/* Track the smallest decision margin and the first iteration at which a
 * margin fell below ZO_TIE_MARGIN (a near-tie: rounding differences of other
 * implementations may legitimately take the other branch there). */
static void note_margin(double m, int32_t k, double *min_margin, int32_t *tie_iter) {
  if (m < *min_margin) *min_margin = m;
  if (m < ZO_TIE_MARGIN && *tie_iter < 0) *tie_iter = k;
}

static int all_finite(const double *a, int d) {
  for (int i = 0; i < d; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

/* One BFGS run (Alg. 4 with Alg. 5 gradients and Alg. 6 line search). */
static void bfgs_one(const zo_problem *pb, const double *x0, int64_t k_out,
                     zo_bfgs_out *out, double *work) {
  const int d = pb->dim;
  double *x = work, *g = x + d, *p = g + d, *xn = p + d, *gn = xn + d;
  double *s = gn + d, *y = s + d, *xt = y + d, *H = xt + d;
  int32_t ls_trials = 0, ls_fail = 0, skips = 0, resets = 0, k = 0, status;
  double min_margin = INFINITY;
  int32_t tie_iter = -1;
  double *trace = out->trace ? out->trace + k_out * (int64_t)out->trace_len * d : NULL;

  const int lm = pb->lbfgs_m;                    /* L-BFGS history (0: BFGS) */
  double *LS = NULL, *LY = NULL, *lrho = NULL;
  int lcount = 0;
  if (lm > 0) {
    LS = (double *)malloc(sizeof(double) * (size_t)lm * d);
    LY = (double *)malloc(sizeof(double) * (size_t)lm * d);
    lrho = (double *)malloc(sizeof(double) * (size_t)lm);
  }
  memcpy(x, x0, sizeof(double) * (size_t)d);    /* x <- swarm[i]        */
  for (int i = 0; i < d; ++i)                    /* H <- I               */
    for (int j = 0; j < d; ++j) H[i * d + j] = (i == j) ? 1.0 : 0.0;
  double f;
  zo_grad(pb->objective, x, d, &f, g);

  for (;;) {
    if (trace && k < out->trace_len) memcpy(trace + (int64_t)k * d, x, sizeof(double) * (size_t)d);
    if (!isfinite(f) || !all_finite(g, d)) { status = ZO_NONFINITE; break; }
    double gnorm = sqrt(pw_dot(g, g, d));
    {
      double m = rel_margin(gnorm, pb->grad_tol);
      note_margin(m, k, &min_margin, &tie_iter);
    }
    if (gnorm < pb->grad_tol) { status = ZO_CONVERGED; break; }
    if (k == pb->iter_bfgs) { status = ZO_MAXITER; break; }

    /* search direction p = -H g (the row products of zo_hrow_dot), or the
     * L-BFGS two-loop recursion over the stored pairs */
    if (lm > 0) {
      zo_lbfgs_direction(LS, LY, lrho, lcount, g, d, p);
    } else {
      for (int i = 0; i < d; ++i) p[i] = -zo_hrow_dot(H + (size_t)i * d, g, d);
    }
    double ddir = pw_dot(g, p, d);
    {
      double m = fabs(ddir) / (gnorm * sqrt(pw_dot(p, p, d)));
      if (!isnan(m)) note_margin(m, k, &min_margin, &tie_iter);
    }
    if (!(ddir < 0.0)) {  /* not a descent direction: restart from H = I */
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) H[i * d + j] = (i == j) ? 1.0 : 0.0;
      lcount = 0;         /* L-BFGS: forget the stored pairs */
      for (int i = 0; i < d; ++i) p[i] = -g[i];
      ddir = pw_dot(g, p, d);
      ++resets;
    }

    int32_t tr, acc;
    double mm = INFINITY;
    double alpha = line_search_m(pb, x, f, p, ddir, xt, &tr, &acc, &mm);
    note_margin(mm, k, &min_margin, &tie_iter);
    ls_trials += tr;
    if (!acc) ++ls_fail;

    for (int i = 0; i < d; ++i) xn[i] = x[i] + alpha * p[i];
    double fn;
    zo_grad(pb->objective, xn, d, &fn, gn);
    for (int i = 0; i < d; ++i) s[i] = xn[i] - x[i];
    for (int i = 0; i < d; ++i) y[i] = gn[i] - g[i];
    {
      double sy = pw_dot(y, s, d);
      double m = fabs(sy) / (sqrt(pw_dot(s, s, d)) * sqrt(pw_dot(y, y, d)));
      if (!isnan(m)) note_margin(m, k, &min_margin, &tie_iter);
    }
    if (lm > 0) {
      if (!zo_lbfgs_push(LS, LY, lrho, &lcount, lm, s, y, d)) ++skips;
    } else if (!zo_bfgs_update(H, s, y, d)) {
      ++skips;
    }

    memcpy(x, xn, sizeof(double) * (size_t)d);
    memcpy(g, gn, sizeof(double) * (size_t)d);
    f = fn;
    ++k;
  }

  free(LS);
  free(LY);
  free(lrho);
  if (trace)
    for (int kk = k + 1; kk < out->trace_len; ++kk)
      for (int j = 0; j < d; ++j) trace[(int64_t)kk * d + j] = NAN;
  memcpy(out->x + k_out * d, x, sizeof(double) * (size_t)d);
  out->f[k_out] = f;
  out->iters[k_out] = k;
  out->status[k_out] = status;
  if (out->ls_trials) out->ls_trials[k_out] = ls_trials;
  if (out->ls_fail) out->ls_fail[k_out] = ls_fail;
  if (out->skips) out->skips[k_out] = skips;
  if (out->resets) out->resets[k_out] = resets;
  if (out->min_margin) out->min_margin[k_out] = min_margin;
  if (out->tie_iter) out->tie_iter[k_out] = tie_iter;
}

int zo_bfgs(const zo_problem *pb, const double *x0, const int64_t *idx,
            int64_t m, zo_bfgs_out *out, int nthreads) {
  if (zo_validate(pb) != 0 || !out || !x0 || m < 0) return -1;
  const int d = pb->dim;
  const size_t wsz = (size_t)(8 * d + d * d);
  int nt = nthreads > 0 ? nthreads : 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
    double *work = (double *)malloc(sizeof(double) * wsz);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < m; ++k) {
      int64_t i = idx ? idx[k] : k;
      bfgs_one(pb, x0 + i * d, k, out, work);
    }
    free(work);
  }
  (void)nt;
  return 0;
}

int64_t zo_best(const double *f, const int32_t *status, int64_t m,
                int64_t *n_conv) {
  int64_t best = -1, nc = 0;
  for (int64_t i = 0; i < m; ++i) {
    if (status && status[i] == ZO_CONVERGED) ++nc;
    if (!isfinite(f[i])) continue;
    if (best < 0 || f[i] < f[best]) best = i;
  }
  if (n_conv) *n_conv = nc;
  return best;
}

int zo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
