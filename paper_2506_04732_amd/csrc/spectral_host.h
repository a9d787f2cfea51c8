// Host-side 1D spectral ingredients (FP64).  See spectral_host.cpp.
#pragma once
#include <vector>

namespace t2s2 {

// P_n(x), P_n'(x), P_n''(x) by the three-term recurrence.
void legendre(int n, double x, double* p, double* dp, double* d2p);
// Zeros of P_n, ascending.
std::vector<double> gauss_zeros(int n);
// GLL nodes x_0 = -1 < ... < x_n = 1.
std::vector<double> gll_nodes(int n);
// Interior collocation nodes (n-1): superconsistent (scheme 1) or GLL (0).
std::vector<double> colloc_nodes(int n, double eps, double beta, int scheme);
// E[j,i] = l_i(y_j), D1[j,i] = l_i'(y_j), D2[j,i] = l_i''(y_j), row-major M x N,
// for the Lagrange basis of the N points x.
void lagrange_eval(const double* x, int N, const double* y, int M,
                   double* E, double* D1, double* D2);

}  // namespace t2s2
