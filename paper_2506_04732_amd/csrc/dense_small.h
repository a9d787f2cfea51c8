// Single-workgroup dense kernels for small matrices.  See dense_small.hip.
#pragma once
#include "common.h"

namespace t2s2 {

// Upper Cholesky G = R^T R (n x n row-major), skipping columns whose pivot is
// <= tau * max diag(G) (zero row in R, mask 0); count[0] = kept columns.
void chol_skip(hipStream_t s, int n, const double* G, double* R, int* mask, int* count, double tau);
// Inverse of a nonsingular upper-triangular n x n matrix.
void trtri_upper(hipStream_t s, int n, const double* R, double* Rinv);
void trtri_upper(hipStream_t s, int n, const double2* R, double2* Rinv);
// B (k x c) = U Wt, U (k x k) orthogonal, rows of Wt orthogonal and sorted by
// decreasing norm sigma.  B and JT (k x k) are overwritten as workspace;
// info needs k + 1 ints (info[0] = sweeps used).
void jacobi_rows(hipStream_t s, int k, int c, double* B, double* JT, double* U, double* Wt, double* sigma,
                 int* info, int max_sweeps = 60);
// A (n x n) <- H = Q^T A Q upper Hessenberg, QT <- Q^T; work >= 2n doubles.
void hessenberg(hipStream_t s, int n, double* A, double* QT, double* work);
// Hr real upper Hessenberg (n x n); ZT (n x n complex) holds the initial Z^T
// and receives (Z_in Z)^T with Hr = Z T Z^H; T complex upper triangular;
// Hw: n*n complex workspace (used when the packed form exceeds LDS);
// info[0] = QR sweeps (negative if the iteration cap was hit).
void schur_qr(hipStream_t s, int n, const double* Hr, double2* Hw, double2* ZT, double2* T, int* info);
// Unit upper-triangular Y with T Y = Y diag(T).
void trevec(hipStream_t s, int n, const double2* T, double2* Y);

}  // namespace t2s2
