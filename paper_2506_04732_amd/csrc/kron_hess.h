// Local Kronecker-sum solve with the left interface in upper Hessenberg form.
// See kron_hess.hip.
#pragma once
#include "common.h"

namespace t2s2 {

// In place on h (r1 x m x r2 complex, row-major): for every right index b,
// solves  H Y + Y T^T + lamR[b] Y = G  for the r1 x m slice Y = h[:, :, b],
// i.e. for j = m-1 .. 0
//   (H + (T[j][j] + lamR[b]) I) Y[:, j] = G[:, j] - sum_{j' > j} T[j][j'] Y[:, j'].
// H: real upper Hessenberg r1 x r1 given column-major (Hc[c * r1 + i] = H[i][c];
// entries below the subdiagonal are ignored); T: complex upper triangular
// m x m row-major; lamR: r2 complex shifts.  Requires kron_hess_fits().
void kron_hess_solve(hipStream_t s, int r1, int m, int r2, const double* Hc, const double2* T, const double2* lamR,
                     double2* h);
void kron_hess_solve(hipStream_t s, int r1, int m, int r2, const float* Hc, const float2* T, const float2* lamR,
                     float2* h);
// The mirrored system with the right interface in Hessenberg form: in place
// on h (r1 x m x r2), for every left index a, solves
//   H Z + Z T^T + lamL[a] Z = G
// for the r2 x m slice Z[c][j] = h[a][j][c], H real upper Hessenberg r2 x r2
// (column-major Hc).  Requires kron_hess_fits(r2, m, ...).
void kron_hess_solve_right(hipStream_t s, int r1, int m, int r2, const double* Hc, const double2* T,
                           const double2* lamL, double2* h);
// Whether the kernel supports r1 and m (r1 <= 256 and the m right-hand sides
// of one wavefront fit in LDS) for complex entries of cbytes bytes.
bool kron_hess_fits(int r1, int m, int cbytes);

}  // namespace t2s2
