// Host-side 1D ingredients of the superconsistent collocation method (FP64).
//
// Overview (i): Lagrange basis on the n+1 Gauss-Lobatto-Legendre (GLL)
// representation points, i.e. +-1 and the n-1 zeros of P_n'.
// Overview (ii), Eq. adv-diff-1d: collocation points move from the zeros of
// P_n' towards the zeros of P_n as eps/|beta| decreases; the discrete
// operators are the representation basis evaluated at the collocation grid.
//
// The superconsistent node formula is not printed in the paper.  Reading used
// (see the header of t2s2.h): theta_i is the zero of eps P_n'(x) - beta P_n(x)
// inside the i-th gap (z_i, z_{i+1}) of the Gauss zeros of P_n, i = 1..n-1.
//
// Methods used here: bracketed, safeguarded Newton iterations for all nodes
// and product-form Lagrange derivatives (running product recurrences), so
// no Vandermonde system is solved.
#include "spectral_host.h"

#include <cmath>
#include <stdexcept>
#include <vector>

namespace t2s2 {

void legendre(int n, double x, double* p, double* dp, double* d2p) {
  // (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}, differentiated once and twice.
  double p0 = 1.0, q0 = 0.0, s0 = 0.0;
  if (n == 0) { *p = p0; *dp = q0; *d2p = s0; return; }
  double p1 = x, q1 = 1.0, s1 = 0.0;
  for (int k = 1; k < n; ++k) {
    const double a = 2.0 * k + 1.0, inv = 1.0 / (k + 1.0);
    const double p2 = (a * x * p1 - k * p0) * inv;
    const double q2 = (a * (p1 + x * q1) - k * q0) * inv;
    const double s2 = (a * (2.0 * q1 + x * s1) - k * s0) * inv;
    p0 = p1; q0 = q1; s0 = s1; p1 = p2; q1 = q2; s1 = s2;
  }
  *p = p1; *dp = q1; *d2p = s1;
}

namespace {

// Root of f in (a, b) where f(a) and f(b) have opposite signs (or one is 0):
// Newton steps kept inside the bracket, bisection otherwise.
template <class F>
double bracketed_root(F f, double a, double b) {
  double fa, dfa, fb, dfb;
  f(a, &fa, &dfa);
  f(b, &fb, &dfb);
  if (fa == 0.0) return a;
  if (fb == 0.0) return b;
  if ((fa > 0) == (fb > 0)) {
    // sign lost to rounding: the zero sits on an end point
    return std::fabs(fa) < std::fabs(fb) ? a : b;
  }
  double x = 0.5 * (a + b);
  for (int it = 0; it < 200; ++it) {
    double fx, dfx;
    f(x, &fx, &dfx);
    if (fx == 0.0) return x;
    if ((fx > 0) == (fa > 0)) { a = x; fa = fx; } else { b = x; fb = fx; }
    double xn = (dfx != 0.0) ? x - fx / dfx : 0.5 * (a + b);
    if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
    const double step = std::fabs(xn - x);
    x = xn;
    if (step <= 2e-16 * std::fmax(1.0, std::fabs(x)) || (b - a) <= 4e-16 * std::fmax(1.0, std::fabs(x))) break;
  }
  // final Newton polish
  double fx, dfx;
  f(x, &fx, &dfx);
  if (dfx != 0.0) {
    const double xn = x - fx / dfx;
    if (xn > a && xn < b) x = xn;
  }
  return x;
}

}  // namespace

std::vector<double> gauss_zeros(int n) {
  if (n < 1) throw std::invalid_argument("degree must be >= 1");
  std::vector<double> z(n);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    // asymptotic first guess, descending in i, then Newton on P_n
    double x = std::cos(pi * (4.0 * (i + 1) - 1.0) / (4.0 * n + 2.0));
    for (int it = 0; it < 100; ++it) {
      double p, dp, d2p;
      legendre(n, x, &p, &dp, &d2p);
      const double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    z[n - 1 - i] = x;
  }
  return z;
}

std::vector<double> gll_nodes(int n) {
  if (n < 1) throw std::invalid_argument("degree must be >= 1");
  std::vector<double> x(n + 1);
  x[0] = -1.0;
  x[n] = 1.0;
  if (n >= 2) {
    // one zero of P_n' between consecutive zeros of P_n
    const std::vector<double> z = gauss_zeros(n);
    auto dP = [n](double t, double* f, double* df) {
      double p, dp, d2p;
      legendre(n, t, &p, &dp, &d2p);
      *f = dp;
      *df = d2p;
    };
    for (int i = 1; i < n; ++i) x[i] = bracketed_root(dP, z[i - 1], z[i]);
  }
  return x;
}

std::vector<double> colloc_nodes(int n, double eps, double beta, int scheme) {
  if (n < 2) throw std::invalid_argument("degree must be >= 2");
  if (!(eps > 0.0)) throw std::invalid_argument("eps must be > 0");
  if (scheme == 0 || beta == 0.0) {
    std::vector<double> x = gll_nodes(n);
    return std::vector<double>(x.begin() + 1, x.end() - 1);
  }
  const std::vector<double> z = gauss_zeros(n);
  auto q = [n, eps, beta](double t, double* f, double* df) {
    double p, dp, d2p;
    legendre(n, t, &p, &dp, &d2p);
    *f = eps * dp - beta * p;
    *df = eps * d2p - beta * dp;
  };
  std::vector<double> th(n - 1);
  for (int i = 0; i < n - 1; ++i) th[i] = bracketed_root(q, z[i], z[i + 1]);
  return th;
}

void lagrange_eval(const double* x, int N, const double* y, int M,
                   double* E, double* D1, double* D2) {
  // l_i(t) = w_i prod_{k != i} (t - x_k), w_i = 1 / prod_{k != i} (x_i - x_k).
  // Value and first two derivatives of the product by the recurrence
  //   (p, p', p'') <- (p h, p' h + p, p'' h + 2 p'),  h = t - x_k.
  std::vector<double> w(N);
  for (int i = 0; i < N; ++i) {
    double prod = 1.0;
    for (int k = 0; k < N; ++k)
      if (k != i) prod *= (x[i] - x[k]);
    w[i] = 1.0 / prod;
  }
  for (int j = 0; j < M; ++j) {
    const double t = y[j];
    for (int i = 0; i < N; ++i) {
      double p = 1.0, dp = 0.0, d2p = 0.0;
      for (int k = 0; k < N; ++k) {
        if (k == i) continue;
        const double h = t - x[k];
        d2p = d2p * h + 2.0 * dp;
        dp = dp * h + p;
        p = p * h;
      }
      E[j * N + i] = w[i] * p;
      D1[j * N + i] = w[i] * dp;
      D2[j * N + i] = w[i] * d2p;
    }
  }
}

}  // namespace t2s2
