// Strided-batched GEMM used by every TT contraction.  See gemm.hip.
#pragma once
#include "common.h"

namespace t2s2 {

enum Op { OpN = 0, OpT = 1, OpC = 2, OpR = 3 };  // R: conjugate, no transpose

// Row-major: C_b = alpha op(A_b) op(B_b) + beta C_b for b < batch, with
// X_b = X + b * strideX.  op(A) is M x K, op(B) is K x N.  OpC conjugates and
// transposes, OpR only conjugates.
template <class T>
void gemm(hipStream_t s, Op opA, Op opB, int M, int N, int K, T alpha,
          const T* A, long lda, long strideA, const T* B, long ldb, long strideB,
          T beta, T* C, long ldc, long strideC, int batch, bool timed = true);

// This thread's FP64 GEMMs use kernel v (0 vector ALU, 1 matrix cores)
// regardless of the tuning table; -1 restores the table.
void gemm_force_variant(int v);
// Where the tuning table came from (device and date, or "untuned").
const char* gemm_tune_source();

}  // namespace t2s2
