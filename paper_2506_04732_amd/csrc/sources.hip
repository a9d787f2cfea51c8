// Separable TT right-hand sides on a problem's collocation grid.
//
// A separable source f(x) = sum_{m < s} prod_l g_ml(x_l) has an exact TT of
// rank s with block-diagonal cores (the TT format of the paper's Methods:
// the right-hand side enters the solve as a TT): core 0 holds g_m0 in column
// m, middle cores g_ml on the diagonal (m, m), the last core g_m,d-1 in row
// m; for d = 1 the single core is the sum.  Every entry, zeros included, is
// written by one pass over the core.
#include "sources.h"

#include <cmath>

namespace t2s2 {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct SrcArgs {
  int kind;        // 0: Gaussian mixture, 1: manufactured sin(pi x) exp(x)
  int d, l, s, m;  // dimensions, core index, rank, interior nodes of dim l
  double eps, beta_l;
  const double* theta;   // m collocation nodes of dimension l
  const double* amp;     // s
  const double* centre;  // s x d
  const double* width;   // s
};

// the 1D factor of term t in dimension l at node x
__device__ inline double factor(const SrcArgs& a, int t, double x) {
  if (a.kind == 0) {
    const double c = a.centre[t * a.d + a.l], w = a.width[t];
    const double g = exp(-(x - c) * (x - c) / (2.0 * w * w));
    return a.l == 0 ? a.amp[t] * g : g;
  }
  // u_l = sin(pi x) e^x; term t differentiates dimension t:
  // (-eps u'' + beta u')(x) = e^x ((-eps (1 - pi^2) + beta) sin(pi x) + (-2 eps + beta) pi cos(pi x))
  const double sn = sin(kPi * x), cs = cos(kPi * x), ex = exp(x);
  if (t != a.l) return sn * ex;
  return ex * ((-a.eps * (1.0 - kPi * kPi) + a.beta_l) * sn + (-2.0 * a.eps + a.beta_l) * kPi * cs);
}

__global__ void source_core_kernel(SrcArgs a, double* __restrict__ core) {
  const int r0 = (a.l == 0) ? 1 : a.s, r1 = (a.l == a.d - 1) ? 1 : a.s;
  const long tot = (long)r0 * a.m * r1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int q = (int)(e % r1);
    const int i = (int)((e / r1) % a.m);
    const int p = (int)(e / ((long)r1 * a.m));
    const double x = a.theta[i];
    double v = 0.0;
    if (a.d == 1) {
      for (int t = 0; t < a.s; ++t) v += factor(a, t, x);
    } else if (a.l == 0) {
      v = factor(a, q, x);
    } else if (a.l == a.d - 1) {
      v = factor(a, p, x);
    } else if (p == q) {
      v = factor(a, p, x);
    }
    core[e] = v;
  }
}

}  // namespace

void separable_source(Problem& P, const Ctx& c, int kind, int s, const double* amp, const double* centre,
                      const double* width, DTT& f) {
  const int d = P.d;
  T2S2_CHECK(s >= 1 && s <= 1024, "source: the number of terms must be in [1, 1024]");
  if (kind == 0) {
    for (int t = 0; t < s; ++t) {
      T2S2_CHECK(std::isfinite(amp[t]) && std::isfinite(width[t]) && width[t] > 0.0,
                 "source: amplitudes must be finite and widths finite and > 0");
      for (int l = 0; l < d; ++l) T2S2_CHECK(std::isfinite(centre[t * d + l]), "source: centres must be finite");
    }
  }
  // parameters and nodes to the device (small, synchronous copies)
  double* dpar = c.sc->get<double>("src.par", (size_t)s * (d + 2));
  size_t msum = 0;
  for (int l = 0; l < d; ++l) msum += P.m[l];
  double* dth = c.sc->get<double>("src.theta", msum);
  if (kind == 0) {
    c.h2d(dpar, amp, s);
    c.h2d(dpar + s, centre, (size_t)s * d);
    c.h2d(dpar + (size_t)s * (d + 1), width, s);
  }
  f.d = d;
  f.n = P.m;
  f.r.assign(d + 1, 1);
  for (int l = 1; l < d; ++l) f.r[l] = s;
  size_t off = 0;
  for (int l = 0; l < d; ++l) {
    c.h2d(dth + off, P.theta[l].data(), P.theta[l].size());
    SrcArgs a{kind, d, l, s, P.m[l], P.eps, P.beta[l], dth + off, dpar, dpar + s, dpar + (size_t)s * (d + 1)};
    off += P.m[l];
    const long tot = (long)f.r[l] * P.m[l] * f.r[l + 1];
    const int grid = (int)std::min<long>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(source_core_kernel, dim3(grid), dim3(256), 0, c.s, a, f.c[l]);
    T2S2_LAUNCH_CHECK();
  }
}

}  // namespace t2s2
