// Host-orchestrated linear algebra on device buffers: scratch pool, mode
// products of TT cores, deflating Cholesky QR, truncated SVD, eigen/Schur
// decompositions of small nonsymmetric matrices.
#pragma once
#include <map>
#include <string>
#include <vector>

#include "common.h"
#include "dense_small.h"
#include "gemm.h"
#include "readback.h"
#include "tt_kernels.h"

namespace t2s2 {

// Named device buffers, grown on demand, released on destruction.  The
// block a buffer outgrows is retired, not freed at once: hipFree waits for
// all work on the device, which in the middle of a solve would stall the
// host behind the side streams' eigendecompositions (and, in a batched
// solve, behind every other instance's queue).  release_retired() frees the
// retired blocks; a retired block stays valid until then, so work already
// queued on it completes as before.
class Scratch {
 public:
  ~Scratch();
  void* raw(const std::string& name, size_t bytes);
  template <class T>
  T* get(const std::string& name, size_t count) {
    return static_cast<T*>(raw(name, count * sizeof(T) + 64));
  }
  size_t bytes() const;
  // frees the retired blocks (each hipFree first waits for the device)
  void release_retired();
  bool has_retired() const { return !retired_.empty(); }

 private:
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs_;
  std::vector<void*> retired_;
};

struct Ctx {
  hipStream_t s = nullptr;
  Scratch* sc = nullptr;
  // optional device flag (one int): set to 1 by a Francis QR that stopped at
  // its step limit; read by the caller at its next synchronisation
  int* fail = nullptr;
  void sync() const { T2S2_HIP(hipStreamSynchronize(s)); }
  // after all earlier work on s (host_read: a pinned mailbox for small reads)
  template <class T>
  void d2h(T* h, const T* d, size_t n) const {
    host_read(s, h, d, n * sizeof(T));
  }
  // synchronous: the host buffer may be reused right after the call
  template <class T>
  void h2d(T* d, const T* h, size_t n) const {
    host_write(s, d, h, n * sizeof(T));
  }
  template <class T>
  void d2d(T* d, const T* src, size_t n) const {
    if (n) T2S2_HIP(hipMemcpyAsync(d, src, n * sizeof(T), hipMemcpyDeviceToDevice, s));
  }
  // sum x[i] y[i] (synchronous)
  double dot(const double* x, const double* y, long n) const;
  double nrm2(const double* x, long n) const;
};

// ---- mode products of a core X[r0][m][r1] (row-major, contiguous) ----
// Y[rA][m][r1] = A (rA x r0) x_1 X
template <class T>
void mode1(const Ctx& c, int rA, int r0, int m, int r1, const T* A, const T* X, T* Y, T beta, Op opA = OpN);
// Y[r0][m][rB] = X x_3 B (rB x r1): Y[.., j] = sum_b B[j, b] X[.., b]
template <class T>
void mode3(const Ctx& c, int r0, int m, int r1, int rB, const T* X, const T* B, T* Y, T beta, Op opB = OpT);
// Y[r0][mK][r1] = K (mK x m) x_2 X
template <class T>
void mode2(const Ctx& c, int r0, int mK, int m, int r1, const T* K, const T* X, T* Y, T beta, Op opK = OpN);

// Orthonormal basis of the columns of A (M x n, leading dimension lda):
// A = Q R + E with Q (M x k, ld k) orthonormal, R (k x n, ld n),
// ||E||_F <= drop ||A||_F.  Gram-based (GEMM) with column skipping in the
// Cholesky factor and deflation of skipped columns to further levels, plus a
// second Cholesky QR pass per level for orthogonality.  Q and R must hold
// M*min(M,n) and min(M,n)*n doubles.  Returns k (0 for A = 0).
int dcholqr(const Ctx& c, int M, int n, const double* A, long lda, double* Q, double* R, double drop);

// Truncated SVD of A (M x n): keeps the smallest r with the Frobenius tail of
// the discarded singular values <= delta (1 <= r <= rmax), U (M x r, ld r)
// orthonormal, W (r x n) with A ~ U W.  sigma_out (optional, host) receives
// the singular values.  Returns r.
int trunc_svd(const Ctx& c, int M, int n, const double* A, long lda, double delta, int rmax, double* U, double* W,
              std::vector<double>* sigma_out = nullptr, double* tail_out = nullptr);

// A (n x n real) = V diag(lam) V^{-1}: Hessenberg reduction, complex Schur
// form by shifted QR, triangular eigenvectors.  Outputs complex n x n V, Vinv
// and n eigenvalues.
void eig_nonsym(const Ctx& c, int n, const double* A, double2* lam, double2* V, double2* Vinv);
// The same factorisation of A = Q H Q^T given its Hessenberg form (Hc: H
// column-major, QT = Q^T row-major): Francis QR from H, no reduction.
void eig_from_hessenberg(const Ctx& c, int n, const double* Hc, const double* QT, double2* lam, double2* V,
                         double2* Vinv);
// The same factorisation computed in FP32 from A rounded to FP32.
void eig_nonsym(const Ctx& c, int n, const double* A, float2* lam, float2* V, float2* Vinv);

// A (n x n) <- H = Q^T A Q upper Hessenberg, QT <- Q^T (LDS-resident kernel
// when it fits, else the global-memory reduction with Q formed by compact-WY
// GEMMs).
void hessenberg(const Ctx& c, int n, double* A, double* QT);

// A (n x n real) = Z T Z^H; outputs ZT = Z^T and upper-triangular T.
void schur_real(const Ctx& c, int n, const double* A, double2* ZT, double2* T);

// Iteration limits of the dense factorisations (0 restores the defaults:
// 40 n + 100 Francis steps, 60 Jacobi sweeps).  Process-wide; lowering them
// makes a factorisation give up and report it (tests of the error path).
void set_iteration_limits(int francis_steps, int jacobi_sweeps);
int francis_step_limit(int n);  // defined next to the Francis kernel
int jacobi_sweep_limit();
// *slot <- max(*slot, ||V||_F ||Vi||_F), an upper bound of cond_2(V) of an
// eigenvector basis (n x n complex), on c's stream
void cond_estimate(const Ctx& c, int n, const double2* V, const double2* Vi, double* slot);
// c.fail <- 0 (on c's stream); whether c.fail is set (synchronises c's stream)
void clear_fail(const Ctx& c);
bool read_fail(const Ctx& c);

}  // namespace t2s2
