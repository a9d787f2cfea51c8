// Element-wise, reduction and TT-specific kernels.  See tt_kernels.hip.
#pragma once
#include "common.h"

#include <algorithm>

namespace t2s2 {

constexpr int kDotBlocks = 512;  // partial-sum slots needed by dot_device

// Ahat[a][(i' R1 + b) n + i] = A[a][i'][i][b] (operator core as R0 matrices
// of (n R1) x n, row-major).
void ttm_permute(hipStream_t s, int R0, int R1, int n, const double* A, double* Ahat);
void fill(hipStream_t s, double* x, long n, double v);
void fill(hipStream_t s, double2* x, long n, double2 v);
// dst[r * ldd + c] = alpha src[r * lds + c], batched with strides ss / sd.
void copy2d(hipStream_t s, long rows, long cols, const double* src, long lds, double* dst, long ldd,
            double alpha = 1.0, int batch = 1, long ss = 0, long sd = 0);
void real_to_complex(hipStream_t s, const double* x, double2* y, long n);
void complex_real_part(hipStream_t s, const double2* x, double* y, long n);
// FP64 <-> FP32 conversions of the mixed-precision local solve
void real_to_complex(hipStream_t s, const double* x, float2* y, long n);
void complex_real_part(hipStream_t s, const float2* x, double* y, long n);
void to_float(hipStream_t s, const double* x, float* y, long n);
void axpby(hipStream_t s, long n, double a, const double* x, double b, double* y);
// *out = sum x[i] y[i] (deterministic two-stage reduction); partial holds
// kDotBlocks doubles.
void dot_device(hipStream_t s, const double* x, const double* y, long n, double* partial, double* out);
void row_sumsq(hipStream_t s, const double* x, long rows, long cols, long ld, double* out);
void col_sumsq(hipStream_t s, const double* x, long rows, long cols, long ld, double* out);
// In place: h[a, :, b] <- (T + (lamL[a] + lamR[b]) I)^{-1} h[a, :, b].
void kron_trisolve(hipStream_t s, int r1, int m, int r2, const double2* T, const double2* lamL,
                   const double2* lamR, double2* h);
void kron_trisolve(hipStream_t s, int r1, int m, int r2, const float2* T, const float2* lamL,
                   const float2* lamR, float2* h);

}  // namespace t2s2

namespace t2s2 {
// out[c * ldo + r] = in[r * ldi + c] for r < rows, c < cols (real / complex).
void transpose(hipStream_t s, long rows, long cols, const double* in, long ldi, double* out, long ldo);
void transpose(hipStream_t s, long rows, long cols, const double2* in, long ldi, double2* out, long ldo);
// out[i] = M[i * (ld + 1)] (diagonal), complex.
void diag_complex(hipStream_t s, int n, const double2* M, long ld, double2* out);
void diag_complex(hipStream_t s, int n, const float2* M, long ld, float2* out);
// dst[r * ldd + j] = src[r * lds + idx[j]] for j < k (column gather).
void gather_cols(hipStream_t s, long rows, int k, const double* src, long lds, const int* idx, double* dst, long ldd);
// Seeded standard-normal-like fill (counter-based hash, Box-Muller).
void fill_random(hipStream_t s, double* x, long n, unsigned long long seed);
}  // namespace t2s2
