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
void trtri_upper(hipStream_t s, int n, const float2* R, float2* Rinv);
// B (k x c) = U Wt, U (k x k) orthogonal, rows of Wt orthogonal and sorted by
// decreasing norm sigma.  B and JT (k x k) are overwritten as workspace;
// info needs k + 1 ints (info[0] = sweeps used).
void jacobi_rows(hipStream_t s, int k, int c, double* B, double* JT, double* U, double* Wt, double* sigma,
                 int* info, int max_sweeps = 60);
// Whether hessenberg() keeps an n x n matrix of rbytes-sized entries in LDS.
bool hessenberg_fits_lds(int n, int rbytes);
// A (n x n) <- H = Q^T A Q upper Hessenberg (zeros below the subdiagonal),
// H in global memory; the reflector of step k goes to column k of V (n x n)
// and beta[k] (n entries, 0: no reflector), Q = P_0 ... P_{n-3}, P_k =
// I - beta_k v_k v_k^T.  n <= 512.
void hessenberg_global(hipStream_t s, int n, double* A, double* V, double* beta);
// Tinv = strict upper part of S with diagonal 1/beta (1 where beta = 0).
void hess_tinv(hipStream_t s, int n, const double* S, const double* beta, double* Tinv);
// X (n x n) <- identity.
void identity(hipStream_t s, int n, double* X);
// A (n x n) <- H = Q^T A Q upper Hessenberg, QT <- Q^T; work >= 2n doubles.
void hessenberg(hipStream_t s, int n, double* A, double* QT, double* work);
void hessenberg(hipStream_t s, int n, float* A, float* QT, float* work);
// Real Schur form of a real upper Hessenberg H (n x n, n <= 512) by the
// Francis double-shift QR iteration: H = Z T Z^T, T quasi upper triangular
// (1 x 1 and 2 x 2 diagonal blocks).  ZT (n x n) holds an initial Z^T on input
// and receives (Z_in Z)^T; Hwork: n*n doubles (used when H exceeds LDS);
// info[0] = Francis steps (negative if the iteration cap was hit).
void schur_francis(hipStream_t s, int n, const double* H, double* Hwork, double* ZT, double* T, int* info);
void schur_francis(hipStream_t s, int n, const float* H, float* Hwork, float* ZT, float* T, int* info);
// Real Schur form -> complex Schur form: Tc = P^H T P upper triangular and
// ZTc = (Z P)^T with P block diagonal unitary; bstart: n ints, U: 2n complex.
void rsf2csf(hipStream_t s, int n, const double* T, const double* ZT, double2* Tc, double2* ZTc, int* bstart,
             double2* U);
void rsf2csf(hipStream_t s, int n, const float* T, const float* ZT, float2* Tc, float2* ZTc, int* bstart,
             float2* U);
// Unit upper-triangular Y with T Y = Y diag(T).
void trevec(hipStream_t s, int n, const double2* T, double2* Y);
void trevec(hipStream_t s, int n, const float2* T, float2* Y);

}  // namespace t2s2
