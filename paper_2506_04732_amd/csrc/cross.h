// TT-cross approximation of built-in non-separable sources.  See cross.hip.
#pragma once
#include <vector>

#include "solver.h"

namespace t2s2 {

// Built-in source functions of x in R^d (kinds):
//   0: amp / (1 + sum_l w_l (x_l - c_l)^2)
//   1: amp exp(-sqrt(delta + sum_l w_l (x_l - c_l)^2))
//   2: amp sin(phase + sum_l w_l x_l)
// params: amp, delta (kind 1) or phase (kind 2; unused for 0), w[d], c[d].
struct CrossFunction {
  int kind = 0;
  std::vector<double> params;  // 2 + 2 d values
};

struct CrossInfo {
  int rank = 0;          // rank of the final cross (before rounding)
  double sample_error = 0.0;
  int evaluations = 0;   // function values sampled
};

// f on the problem's collocation grid as a TT: alternating cross with MaxVol
// row selection at ranks r0, 2 r0, .. <= rmax until the relative error on
// `samples` random grid points is <= tol, then rounded at relative tol / 10.
// f_out: caller cores with room for rmax * m_l * rmax doubles; ranks written.
CrossInfo source_cross(Problem& p, const Ctx& c, const CrossFunction& fn, double tol, int r0, int rmax,
                       unsigned long long seed, int samples, DTT& f_out);

}  // namespace t2s2
