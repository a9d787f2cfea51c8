// 2-norm of a TT vector by the Gram recursion in double-double arithmetic.
//
// G_0 = 1,  G_{l+1} = sum_i X_l(i)^T G_l X_l(i),  ||x||^2 = G_d.
// The residual TT f - L x is a concatenation whose parts cancel to ~1e-8 of
// their size; a QR sweep built on FP64 Gram matrices (Cholesky QR) loses
// that cancellation, and so does this recursion in FP64.  In double-double
// (a value is an unevaluated sum hi + lo, about 106 significant bits) every
// product of FP64 core entries is exact and every sum is rounded at ~1e-32
// relative to its terms, so the final cancellation leaves ||x||^2 correct to
// ~1e-16 relative even when it is 1e-16 of the terms.  The cores themselves
// are FP64 and are read as exact.
//
// Error-free transformations: two-sum (Knuth), two-product via FMA, and the
// accurate double-double addition that renormalises both the high and the
// low parts (as in Hida, Li and Bailey's double-double arithmetic).  The
// file is compiled without FP contraction so that no a*b + c in them is
// fused behind the code's back.
#include "ddnorm.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "linalg.h"

#pragma clang fp contract(off)

namespace t2s2 {

namespace {

struct dd {
  double hi, lo;
};

__device__ inline dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

__device__ inline dd quick_two_sum(double a, double b) {  // |a| >= |b|
  const double s = a + b;
  return {s, b - (s - a)};
}

__device__ inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}

// a (FP64) times b (double-double)
__device__ inline dd dd_mul_d(double a, dd b) {
  const double p = a * b.hi;
  double e = fma(a, b.hi, -p);
  e = fma(a, b.lo, e);
  return quick_two_sum(p, e);
}

constexpr int TB = 64, TK = 16, NTH = 256;

// a (FP64) times b (double-double), whichever operand of the GEMM is FP64
__device__ inline dd dd_prod(double a, dd b) { return dd_mul_d(a, b); }
__device__ inline dd dd_prod(dd a, double b) { return dd_mul_d(b, a); }

// C (M x N, double-double, row-major ld N) = op(A) (M x K) B (K x N), one of
// A, B FP64 and the other double-double (the tiles are staged in their own
// type, so the FP64 operand's product is exact by construction).  op(A) = A
// (ld lda) or, with transA, A stored K x M (ld lda).  kchunk > 0: split-K
// partial products, slab z of C at C + z * M * N covers K range
// [z kchunk, (z + 1) kchunk).
template <class TA, class TBt>
__global__ void __launch_bounds__(NTH) dd_gemm_kernel(int transA, int M, int N, int K, const TA* __restrict__ A,
                                                      long lda, const TBt* __restrict__ B, long ldb,
                                                      dd* __restrict__ C, int kchunk) {
  static_assert(std::is_same<TA, double>::value != std::is_same<TBt, double>::value,
                "one operand FP64, the other double-double");
  __shared__ TA As[TK][TB + 1];
  __shared__ TBt Bs[TK][TB + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * TB, n0 = blockIdx.x * TB;
  int kbeg = 0, kend = K;
  if (kchunk > 0) {
    kbeg = blockIdx.z * kchunk;
    kend = min(K, kbeg + kchunk);
    C += (long)blockIdx.z * M * N;
  }
  dd acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = {0.0, 0.0};
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
    for (int s = 0; s < (TB * TK) / NTH; ++s) {
      const int e = tid + NTH * s;
      int i, k;
      if (!transA) { i = e / TK; k = e % TK; } else { k = e / TB; i = e % TB; }
      const int gi = m0 + i, gk = k0 + k;
      TA v{};
      if (gi < M && gk < kend) v = transA ? A[(long)gk * lda + gi] : A[(long)gi * lda + gk];
      As[k][i] = v;
    }
#pragma unroll
    for (int s = 0; s < (TB * TK) / NTH; ++s) {
      const int e = tid + NTH * s;
      const int k = e / TB, j = e % TB;
      const int gj = n0 + j, gk = k0 + k;
      TBt v{};
      if (gj < N && gk < kend) v = B[(long)gk * ldb + gj];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < TK; ++k) {
      TA a[4];
      TBt b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = dd_add(acc[i][j], dd_prod(a[i], b[j]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gi = m0 + ty + 16 * i, gj = n0 + tx + 16 * j;
      if (gi < M && gj < N) C[(long)gi * N + gj] = acc[i][j];
    }
}

__global__ void dd_reduce_kernel(long MN, int S, const dd* __restrict__ W, dd* __restrict__ C) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < MN; e += (long)gridDim.x * blockDim.x) {
    dd s = W[e];
    for (int z = 1; z < S; ++z) s = dd_add(s, W[(long)z * MN + e]);
    C[e] = s;
  }
}

__global__ void dd_one_kernel(dd* g) { g[0] = {1.0, 0.0}; }

// the exact (hi + lo) value of a 1 x 1 result, read by the host
__global__ void dd_collapse_kernel(const dd* g, double* out) {
  out[0] = g[0].hi;
  out[1] = g[0].lo;
}

template <class TA, class TBt>
void dd_gemm(const Ctx& c, bool transA, int M, int N, int K, const TA* A, long lda, const TBt* B, long ldb, dd* C) {
  const long tiles = (long)((M + TB - 1) / TB) * ((N + TB - 1) / TB);
  TimedScope ts(c.s, KC_OTHER, 8.0 * ((double)M * K + (double)K * N) + 16.0 * (double)M * N, 2.0 * M * N * (double)K);
  if (tiles < 128 && K >= 1024) {
    int S = (int)std::min<long>((512 + tiles - 1) / tiles, K / 256);
    S = std::max(2, std::min(S, 256));
    int kchunk = (K + S - 1) / S;
    kchunk = ((kchunk + TK - 1) / TK) * TK;
    S = (K + kchunk - 1) / kchunk;
    const long MN = (long)M * N;
    dd* W = c.sc->get<dd>("dd.split", (size_t)S * MN);
    dim3 grid((N + TB - 1) / TB, (M + TB - 1) / TB, S);
    hipLaunchKernelGGL((dd_gemm_kernel<TA, TBt>), grid, dim3(NTH), 0, c.s, (int)transA, M, N, K, A, lda, B, ldb, W,
                       kchunk);
    T2S2_LAUNCH_CHECK();
    const int rb = (int)std::min<long>((MN + 255) / 256, 2048);
    hipLaunchKernelGGL(dd_reduce_kernel, dim3(rb), dim3(256), 0, c.s, MN, S, W, C);
    T2S2_LAUNCH_CHECK();
    return;
  }
  dim3 grid((N + TB - 1) / TB, (M + TB - 1) / TB, 1);
  hipLaunchKernelGGL((dd_gemm_kernel<TA, TBt>), grid, dim3(NTH), 0, c.s, (int)transA, M, N, K, A, lda, B, ldb, C, 0);
  T2S2_LAUNCH_CHECK();
}

}  // namespace

double tt_norm_dd(const Ctx& c, const DTT& x) {
  const int d = x.d;
  size_t gmax = 1, tmax = 1;
  for (int l = 0; l < d; ++l) {
    gmax = std::max(gmax, (size_t)x.r[l + 1] * x.r[l + 1]);
    tmax = std::max(tmax, (size_t)x.r[l] * x.n[l] * x.r[l + 1]);
  }
  dd* G = c.sc->get<dd>("dd.G", gmax);
  dd* T = c.sc->get<dd>("dd.T", tmax);
  hipLaunchKernelGGL(dd_one_kernel, dim3(1), dim3(1), 0, c.s, G);
  T2S2_LAUNCH_CHECK();
  for (int l = 0; l < d; ++l) {
    const int r0 = x.r[l], n = x.n[l], r1 = x.r[l + 1];
    // T (r0 x n r1) = G (r0 x r0) X (r0 x n r1)
    dd_gemm<dd, double>(c, false, r0, n * r1, r0, G, r0, x.c[l], (long)n * r1, T);
    // G' (r1 x r1) = X^T T, both viewed as (r0 n) x r1
    dd_gemm<double, dd>(c, true, r1, r1, r0 * n, x.c[l], r1, T, r1, G);
  }
  double* out = c.sc->get<double>("dd.out", 2);
  hipLaunchKernelGGL(dd_collapse_kernel, dim3(1), dim3(1), 0, c.s, G, out);
  T2S2_LAUNCH_CHECK();
  double h[2] = {0.0, 0.0};
  c.d2h(h, out, 2);
  const double s = h[0] + h[1];
  T2S2_CHECK(std::isfinite(s), "tt norm: non-finite Gram value");
  return std::sqrt(std::max(0.0, s));
}

}  // namespace t2s2
