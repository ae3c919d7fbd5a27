"""User-defined objectives written as user code (the source text that
zeus_objective_compile takes), used by the tests and the bench.

* ROSENBROCK, GOLDSTEIN_PRICE, RASTRIGIN: the test functions of Sec. V-B
  restated as user code (for d = 2 Rosenbrock and Goldstein-Price perform the
  same operations as the built-in objectives).
* CHAIN_LOG: a non-separable function whose every gradient component depends
  on every coordinate.
* poisson_fit_source: a binned Poisson likelihood fit of a falling
  dijet-like spectrum, standing in for the paper's dijet fit (Sec. V-G),
  whose data are not available.  The histogram is synthetic: 40 bins in
  x = m / sqrt(s) in [0.1, 0.6], expected counts
      mu_b = exp(phi0) (1 - x_b)^p1 / x_b^(p2 + p3 ln x_b)
  at POISSON_TRUE = (phi0, p1, p2, p3), and counts drawn from Poisson(mu_b)
  with numpy's Philox generator keyed 7.  The objective is the negative log
  likelihood sum_b [mu_b(theta) - n_b ln mu_b(theta)] (constant terms
  dropped), with ln mu_b written out so that no log of an exp is taken.
"""
import numpy as np

ROSENBROCK = '''
template <class T, class X>
ZEUS_FN T objective(const X &x, int d) {
  T s = T(0.0);
  for (int i = 0; i + 1 < d; ++i) {
    const T a = 1.0 - x[i];
    const T b = x[i + 1] - x[i] * x[i];
    s = s + (a * a + 100.0 * (b * b));
  }
  return s;
}
'''

GOLDSTEIN_PRICE = '''
template <class T, class X>
ZEUS_FN T objective(const X &x, int) {
  const T x1 = x[0], x2 = x[1];
  const T a = 1.0 + (x1 + x2);
  T pa = 19.0 - 14.0 * x1;
  pa = pa + 3.0 * (x1 * x1);
  pa = pa - 14.0 * x2;
  pa = pa + 6.0 * (x1 * x2);
  pa = pa + 3.0 * (x2 * x2);
  const T A = 1.0 + (a * a) * pa;
  const T b = 2.0 * x1 - 3.0 * x2;
  T pb = 18.0 - 32.0 * x1;
  pb = pb + 12.0 * (x1 * x1);
  pb = pb + 48.0 * x2;
  pb = pb - 36.0 * (x1 * x2);
  pb = pb + 27.0 * (x2 * x2);
  const T B = 30.0 + (b * b) * pb;
  return A * B;
}
'''

RASTRIGIN = '''
template <class T, class X>
ZEUS_FN T objective(const X &x, int d) {
  T s = T(10.0 * d);
  for (int i = 0; i < d; ++i) s = s + (x[i] * x[i] - 10.0 * zcos(6.283185307179586 * x[i]));
  return s;
}
'''

CHAIN_LOG = '''
template <class T, class X>
ZEUS_FN T objective(const X &x, int d) {
  T s = T(0.0), m = T(0.0);
  for (int i = 0; i < d; ++i) {
    const T a = x[i] - 1.0;
    s = s + a * a;
    m = m + x[i];
  }
  for (int i = 0; i + 1 < d; ++i) {
    const T b = x[i + 1] - x[i] * x[i];
    s = s + zlog(1.0 + 10.0 * (b * b));
  }
  return s + (m * m) / (double)d;
}
'''

POISSON_TRUE = (np.log(50.0), 8.0, 4.0, 0.5)
POISSON_BINS = 40


def poisson_histogram(bins=POISSON_BINS, theta=POISSON_TRUE, seed=7):
    """Bin centres x_b, ln(1 - x_b), ln x_b and Poisson counts n_b."""
    edges = np.linspace(0.1, 0.6, bins + 1)
    x = 0.5 * (edges[:-1] + edges[1:])
    l1, lx = np.log1p(-x), np.log(x)
    phi0, p1, p2, p3 = theta
    mu = np.exp(phi0 + p1 * l1 - (p2 + p3 * lx) * lx)
    n = np.random.Generator(np.random.Philox(key=seed)).poisson(mu).astype(np.float64)
    return x, l1, lx, n


POISSON_COUNTS = poisson_histogram()[3]


def _arr(name, v):
    return f"constexpr double {name}[{len(v)}] = {{" + ", ".join(float(t).hex() for t in v) + "};\n"


def poisson_fit_source(counts=None, bins=POISSON_BINS):
    """User source of the binned Poisson negative log likelihood in
    theta = (phi0, p1, p2, p3), its data embedded as exact constants."""
    _, l1, lx, n = poisson_histogram(bins)
    if counts is not None:
        n = np.asarray(counts, dtype=np.float64)
    return (_arr("kL1", l1) + _arr("kLx", lx) + _arr("kN", n) + f'''
template <class T, class X>
ZEUS_FN T objective(const X &x, int) {{
  T s = T(0.0);
  for (int b = 0; b < {bins}; ++b) {{
    const T e = x[0] + (x[1] * kL1[b] - (x[2] + x[3] * kLx[b]) * kLx[b]);
    s = s + (zexp(e) - kN[b] * e);
  }}
  return s;
}}
''')
