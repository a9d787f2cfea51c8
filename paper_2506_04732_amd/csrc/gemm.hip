// Strided-batched GEMM for the TT contractions (FP64, complex FP64, FP32).
//
// Row-major convention: C[M x N] = alpha op(A)[M x K] op(B)[K x N] + beta C,
// with op in {N, T, C (conjugate transpose), R (conjugate, no transpose)}.  Every mode product of a TT core
// [r0][m][r1] is one call: mode 1 is a plain GEMM over the (m r1) columns,
// mode 3 a GEMM with transposed right factor, mode 2 a GEMM batched over r0.
//
// Tile: 64 x 64 outputs per 256-thread workgroup, K staged through LDS in
// steps of 16 (the next step prefetched into registers during the current
// one); each thread owns a 4 x 4 register block at stride 16 so that both
// the LDS reads and the global writes of a wavefront are contiguous.  Most
// calls of the solver have thin outputs and long reductions (projections
// onto interfaces, Gram matrices): with fewer than 256 output tiles and
// K >= 256 the reduction is split into ~128-long slabs summed in a fixed
// order by a second kernel, so many short workgroups run at once.
#include "gemm.h"

#include <map>

#include "gemm_tune.h"

#include <algorithm>
#include <type_traits>

namespace t2s2 {

namespace {

template <class T> struct Arith;
template <> struct Arith<double> {
  __device__ static double zero() { return 0.0; }
  __device__ static double fma(double a, double b, double c) { return ::fma(a, b, c); }
  __device__ static double mul(double a, double b) { return a * b; }
  __device__ static double add(double a, double b) { return a + b; }
  __device__ static double conj(double a) { return a; }
  __device__ static bool is_zero(double a) { return a == 0.0; }
  static bool is_zero_host(double a) { return a == 0.0; }
};
template <> struct Arith<float> {
  __device__ static float zero() { return 0.0f; }
  __device__ static float fma(float a, float b, float c) { return ::fmaf(a, b, c); }
  __device__ static float mul(float a, float b) { return a * b; }
  __device__ static float add(float a, float b) { return a + b; }
  __device__ static float conj(float a) { return a; }
  __device__ static bool is_zero(float a) { return a == 0.0f; }
  static bool is_zero_host(float a) { return a == 0.0f; }
};
template <> struct Arith<double2> {
  __device__ static double2 zero() { return make_double2(0.0, 0.0); }
  __device__ static double2 fma(double2 a, double2 b, double2 c) {
    return make_double2(::fma(a.x, b.x, ::fma(-a.y, b.y, c.x)), ::fma(a.x, b.y, ::fma(a.y, b.x, c.y)));
  }
  __device__ static double2 mul(double2 a, double2 b) { return cmul(a, b); }
  __device__ static double2 add(double2 a, double2 b) { return cadd(a, b); }
  __device__ static double2 conj(double2 a) { return cconj(a); }
  __device__ static bool is_zero(double2 a) { return a.x == 0.0 && a.y == 0.0; }
  static bool is_zero_host(double2 a) { return a.x == 0.0 && a.y == 0.0; }
};
template <> struct Arith<float2> {
  __device__ static float2 zero() { return make_float2(0.0f, 0.0f); }
  __device__ static float2 fma(float2 a, float2 b, float2 c) {
    return make_float2(::fmaf(a.x, b.x, ::fmaf(-a.y, b.y, c.x)), ::fmaf(a.x, b.y, ::fmaf(a.y, b.x, c.y)));
  }
  __device__ static float2 mul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  }
  __device__ static float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
  __device__ static float2 conj(float2 a) { return make_float2(a.x, -a.y); }
  __device__ static bool is_zero(float2 a) { return a.x == 0.0f && a.y == 0.0f; }
  static bool is_zero_host(float2 a) { return a.x == 0.0f && a.y == 0.0f; }
};

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

template <class T>
__global__ void __launch_bounds__(NT)
gemm_kernel(int opA, int opB, int M, int N, int K, T alpha,
            const T* __restrict__ A, long lda, long sA,
            const T* __restrict__ B, long ldb, long sB,
            T beta, T* __restrict__ C, long ldc, long sC, int kchunk) {
  // kchunk > 0: split-K partial products, blockIdx.z selects the K range and
  // the output slab C + z * sC; otherwise blockIdx.z is the batch index.
  using AR = Arith<T>;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const long bz = blockIdx.z;
  int kbeg = 0, kend = K;
  if (kchunk > 0) {
    kbeg = (int)bz * kchunk;
    kend = min(K, kbeg + kchunk);
  } else {
    A += bz * sA;
    B += bz * sB;
  }
  C += bz * sC;

  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = AR::zero();

  // the next K tile is fetched into registers while the current one is
  // multiplied from LDS, so a tile's global latency overlaps the arithmetic
  constexpr int SA = (BM * BK) / NT, SB = (BN * BK) / NT;
  const bool ta = (opA == 1 || opA == 2), tb = (opB == 1 || opB == 2);
  T ra[SA], rb[SB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s = 0; s < SA; ++s) {
      const int e = tid + NT * s;
      int i, k;
      if (!ta) { i = e / BK; k = e % BK; } else { k = e / BM; i = e % BM; }
      const int gi = m0 + i, gk = k0 + k;
      T v = AR::zero();
      if (gi < M && gk < kend) {
        v = !ta ? A[(long)gi * lda + gk] : A[(long)gk * lda + gi];
        if (opA >= 2) v = AR::conj(v);
      }
      ra[s] = v;
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const int e = tid + NT * s;
      int j, k;
      if (!tb) { k = e / BN; j = e % BN; } else { j = e / BK; k = e % BK; }
      const int gj = n0 + j, gk = k0 + k;
      T v = AR::zero();
      if (gj < N && gk < kend) {
        v = !tb ? B[(long)gk * ldb + gj] : B[(long)gj * ldb + gk];
        if (opB >= 2) v = AR::conj(v);
      }
      rb[s] = v;
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int s = 0; s < SA; ++s) {
      const int e = tid + NT * s;
      if (!ta) As[e % BK][e / BK] = ra[s]; else As[e / BM][e % BM] = ra[s];
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const int e = tid + NT * s;
      if (!tb) Bs[e / BN][e % BN] = rb[s]; else Bs[e % BK][e / BK] = rb[s];
    }
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = AR::fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  const bool beta_zero = AR::is_zero(beta);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gi = m0 + ty + 16 * i;
    if (gi >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gj = n0 + tx + 16 * j;
      if (gj >= N) continue;
      T* c = C + (long)gi * ldc + gj;
      T v = AR::mul(alpha, acc[i][j]);
      if (!beta_zero) v = AR::add(v, AR::mul(beta, *c));
      *c = v;
    }
  }
}

// FP64 on the matrix cores: the same 64 x 64 tile and K staging as
// gemm_kernel, each of the 4 wavefronts computing a 32 x 32 quarter as 2 x 2
// blocks of V_MFMA_F64_16X16X4_F64 (lane l holds A[l % 16][k0 + l / 16] and
// B[k0 + l / 16][l % 16]; output element (l / 16 + 4 i, l % 16) in slot i).
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(NT)
gemm_mfma_f64_kernel(int opA, int opB, int M, int N, int K, double alpha,
                     const double* __restrict__ A, long lda, long sA,
                     const double* __restrict__ B, long ldb, long sB,
                     double beta, double* __restrict__ C, long ldc, long sC, int kchunk) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const long bz = blockIdx.z;
  int kbeg = 0, kend = K;
  if (kchunk > 0) {
    kbeg = (int)bz * kchunk;
    kend = min(K, kbeg + kchunk);
  } else {
    A += bz * sA;
    B += bz * sB;
  }
  C += bz * sC;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  constexpr int SA = (BM * BK) / NT, SB = (BN * BK) / NT;
  const bool ta = (opA == 1), tb = (opB == 1);
  double ra[SA], rb[SB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s = 0; s < SA; ++s) {
      const int e = tid + NT * s;
      int i, k;
      if (!ta) { i = e / BK; k = e % BK; } else { k = e / BM; i = e % BM; }
      const int gi = m0 + i, gk = k0 + k;
      ra[s] = (gi < M && gk < kend) ? (!ta ? A[(long)gi * lda + gk] : A[(long)gk * lda + gi]) : 0.0;
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const int e = tid + NT * s;
      int j, k;
      if (!tb) { k = e / BN; j = e % BN; } else { j = e / BK; k = e % BK; }
      const int gj = n0 + j, gk = k0 + k;
      rb[s] = (gj < N && gk < kend) ? (!tb ? B[(long)gk * ldb + gj] : B[(long)gj * ldb + gk]) : 0.0;
    }
  };
  if (kbeg < kend) fetch(kbeg);
  const int li = lane & 15, lk = lane >> 4;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int s = 0; s < SA; ++s) {
      const int e = tid + NT * s;
      if (!ta) As[e % BK][e / BK] = ra[s]; else As[e / BM][e % BM] = ra[s];
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const int e = tid + NT * s;
      if (!tb) Bs[e / BN][e % BN] = rb[s]; else Bs[e % BK][e / BK] = rb[s];
    }
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + lk;
      const double a0 = As[kr][wr + li], a1 = As[kr][wr + 16 + li];
      const double b0 = Bs[kr][wc + li], b1 = Bs[kr][wc + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  const bool beta_zero = (beta == 0.0);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gi = m0 + wr + bi * 16 + lk + 4 * i, gj = n0 + wc + bj * 16 + li;
        if (gi >= M || gj >= N) continue;
        double* c = C + (long)gi * ldc + gj;
        double v = alpha * acc[bi][bj][i];
        if (!beta_zero) v += beta * *c;
        *c = v;
      }
}

// C = alpha * sum_z W[z] + beta * C  (split-K epilogue, deterministic order)
template <class T>
__global__ void splitk_reduce_kernel(int M, int N, int S, const T* __restrict__ W, T alpha, T beta,
                                     T* __restrict__ C, long ldc) {
  using AR = Arith<T>;
  const long MN = (long)M * N;
  const bool beta_zero = AR::is_zero(beta);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < MN; e += (long)gridDim.x * blockDim.x) {
    T acc = AR::zero();
    for (int z = 0; z < S; ++z) acc = AR::add(acc, W[z * MN + e]);
    T* c = C + (e / N) * ldc + (e % N);
    T v = AR::mul(alpha, acc);
    if (!beta_zero) v = AR::add(v, AR::mul(beta, *c));
    *c = v;
  }
}

struct SplitWork {
  void* p = nullptr;
  size_t bytes = 0;
  ~SplitWork() {
    if (p) (void)hipFree(p);
  }
};
// one workspace per (host thread, stream): concurrent solves (batched mode)
// drive their own streams from their own threads, and one solve drives a
// second stream for its side work
thread_local std::map<hipStream_t, SplitWork> g_split;

template <class T>
T* split_workspace(hipStream_t s, size_t count) {
  SplitWork& w = g_split[s];
  const size_t want = count * sizeof(T);
  if (w.bytes < want) {
    if (w.p) T2S2_HIP(hipFree(w.p));
    w.p = nullptr;
    w.bytes = 0;
    const size_t alloc = std::max(want, (size_t)1 << 24);
    T2S2_HIP(hipMalloc(&w.p, alloc));
    w.bytes = alloc;
  }
  return static_cast<T*>(w.p);
}

template <class T> bool AR_beta_nonzero(T b) { return !Arith<T>::is_zero_host(b); }

thread_local int g_force_variant = -1;

int tune_bucket(long x) {
  int b = 0;
  while ((1L << (b + 4)) < x && b < kGemmTuneB - 1) ++b;
  return b;
}

template <class T> T one_of();
template <> double one_of<double>() { return 1.0; }
template <> float one_of<float>() { return 1.0f; }
template <> double2 one_of<double2>() { return make_double2(1.0, 0.0); }
template <> float2 one_of<float2>() { return make_float2(1.0f, 0.0f); }
template <class T> T zero_of();
template <> double zero_of<double>() { return 0.0; }
template <> float zero_of<float>() { return 0.0f; }
template <> double2 zero_of<double2>() { return make_double2(0.0, 0.0); }
template <> float2 zero_of<float2>() { return make_float2(0.0f, 0.0f); }

}  // namespace

template <class T>
void gemm(hipStream_t s, Op opA, Op opB, int M, int N, int K, T alpha,
          const T* A, long lda, long strideA, const T* B, long ldb, long strideB,
          T beta, T* C, long ldc, long strideC, int batch, bool timed) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    // C = beta C; K = 0 never occurs in the solver, reject rather than guess
    throw Error(1, "gemm: K must be positive");
  }
  const bool cplx = std::is_same<T, double2>::value || std::is_same<T, float2>::value;
  const double elem = (double)sizeof(T);
  TimedScope ts(s, cplx ? KC_GEMM_C : KC_GEMM,
                elem * ((double)M * K + (double)K * N + (double)M * N * (AR_beta_nonzero(beta) ? 2.0 : 1.0)) * batch,
                (cplx ? 8.0 : 2.0) * (double)M * N * K * batch, timed);
  const long tiles = (long)((N + BN - 1) / BN) * ((M + BM - 1) / BM);
  // real FP64 without conjugation: the matrix-core kernel where the tuning
  // table (or a forced choice) says it is faster
  bool mfma = false;
  if constexpr (std::is_same<T, double>::value) {
    if ((opA == OpN || opA == OpT) && (opB == OpN || opB == OpT)) {
      const int v = g_force_variant >= 0
                        ? g_force_variant
                        : kGemmTune[batch > 1 ? 1 : 0][tune_bucket(M)][tune_bucket(N)][tune_bucket(K)];
      mfma = (v == 1);
    }
  }
  if (batch == 1 && tiles < 256 && K >= 256) {
    // few output tiles, long reduction: split K into slabs of ~128 (each
    // workgroup runs a short loop, many run at once), at most ~1024 slabs
    int S = (int)std::min<long>(K / 128, std::max<long>(2, 1024 / tiles));
    S = std::max(2, std::min(S, 256));
    int kchunk = (K + S - 1) / S;
    kchunk = ((kchunk + BK - 1) / BK) * BK;
    S = (K + kchunk - 1) / kchunk;
    const long MN = (long)M * N;
    T* W = split_workspace<T>(s, (size_t)S * MN);
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, S);
    if constexpr (std::is_same<T, double>::value) {
      if (mfma)
        hipLaunchKernelGGL(gemm_mfma_f64_kernel, grid, dim3(NT), 0, s, (int)opA, (int)opB, M, N, K, 1.0, A, lda, 0L,
                           B, ldb, 0L, 0.0, W, (long)N, MN, kchunk);
    }
    if (!mfma)
      hipLaunchKernelGGL(gemm_kernel<T>, grid, dim3(NT), 0, s, (int)opA, (int)opB, M, N, K, one_of<T>(),
                         A, lda, 0L, B, ldb, 0L, zero_of<T>(), W, (long)N, MN, kchunk);
    T2S2_LAUNCH_CHECK();
    const int rb = (int)std::min<long>((MN + 255) / 256, 2048);
    hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3(rb), dim3(256), 0, s, M, N, S, W, alpha, beta, C, ldc);
    T2S2_LAUNCH_CHECK();
    return;
  }
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
  if constexpr (std::is_same<T, double>::value) {
    if (mfma) {
      hipLaunchKernelGGL(gemm_mfma_f64_kernel, grid, dim3(NT), 0, s, (int)opA, (int)opB, M, N, K, alpha, A, lda,
                         strideA, B, ldb, strideB, beta, C, ldc, strideC, 0);
      T2S2_LAUNCH_CHECK();
      return;
    }
  }
  hipLaunchKernelGGL(gemm_kernel<T>, grid, dim3(NT), 0, s, (int)opA, (int)opB, M, N, K, alpha,
                     A, lda, strideA, B, ldb, strideB, beta, C, ldc, strideC, 0);
  T2S2_LAUNCH_CHECK();
}

template void gemm<double>(hipStream_t, Op, Op, int, int, int, double, const double*, long, long,
                           const double*, long, long, double, double*, long, long, int, bool);
template void gemm<double2>(hipStream_t, Op, Op, int, int, int, double2, const double2*, long, long,
                            const double2*, long, long, double2, double2*, long, long, int, bool);
template void gemm<float>(hipStream_t, Op, Op, int, int, int, float, const float*, long, long,
                          const float*, long, long, float, float*, long, long, int, bool);
template void gemm<float2>(hipStream_t, Op, Op, int, int, int, float2, const float2*, long, long,
                           const float2*, long, long, float2, float2*, long, long, int, bool);

void gemm_force_variant(int v) { g_force_variant = v; }
const char* gemm_tune_source() { return kGemmTuneSource; }

}  // namespace t2s2
