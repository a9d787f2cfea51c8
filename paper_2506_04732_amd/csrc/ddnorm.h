// TT 2-norm by a double-double Gram recursion.  See ddnorm.hip.
#pragma once
#include "solver.h"

namespace t2s2 {

// ||x||_2 of a TT in device memory, accurate to ~1e-16 relative even when
// the value is a cancellation of terms 1e8 times larger (residual TTs).
// Synchronises the stream.
double tt_norm_dd(const Ctx& c, const DTT& x);

}  // namespace t2s2
