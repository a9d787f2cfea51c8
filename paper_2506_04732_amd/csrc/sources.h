// Separable TT right-hand sides on the collocation grid.  See sources.hip.
#pragma once
#include "solver.h"

namespace t2s2 {

// kind 0: f = sum_t amp[t] prod_l exp(-(x_l - centre[t d + l])^2 / (2 width[t]^2));
// kind 1: the source of u = prod_l sin(pi x_l) exp(x_l) (s = d terms; amp,
// centre, width unused).  f.c must hold the cores of ranks (1, s, .., s, 1);
// f's ranks are set.  Host parameter arrays; synchronises the stream.
void separable_source(Problem& P, const Ctx& c, int kind, int s, const double* amp, const double* centre,
                      const double* width, DTT& f);

}  // namespace t2s2
