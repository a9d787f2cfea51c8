// Element-wise, reduction and TT-specific kernels of libt2s2.
#include "tt_kernels.h"

namespace t2s2 {

namespace {

constexpr int kBlock = 256;

inline int grid_for(long n, int per_block = kBlock, int cap = 8192) {
  long g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Ahat[a][(ip * R1 + b) * n + i] = A[a][ip][i][b]: the operator core as R0
// row-major (n R1) x n matrices, the left factors of the GEMM form of the
// core product
__global__ void ttm_permute_kernel(int R0, int R1, int n, const double* __restrict__ A, double* __restrict__ Ah) {
  const long tot = (long)R0 * n * n * R1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int b = (int)(e % R1);
    const long t = e / R1;
    const int i = (int)(t % n);
    const long t2 = t / n;
    const int ip = (int)(t2 % n);
    const int a = (int)(t2 / n);
    Ah[(long)a * n * R1 * n + ((long)ip * R1 + b) * n + i] = A[e];
  }
}

// ------------------------------------------------------------ element-wise
template <class T>
__global__ void fill_kernel(T* x, long n, T v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}

// dst[r * ldd + c] = alpha * src[r * lds + c] for r < rows, c < cols, batched.
template <class T>
__global__ void copy2d_kernel(long rows, long cols, const T* __restrict__ src, long lds, long ss,
                              T* __restrict__ dst, long ldd, long sd, double alpha) {
  const long b = blockIdx.y;
  src += b * ss;
  dst += b * sd;
  const long n = rows * cols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const long r = e / cols, c = e % cols;
    dst[r * ldd + c] = src[r * lds + c] * alpha;
  }
}

__global__ void real_to_complex_kernel(const double* __restrict__ x, double2* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = make_double2(x[i], 0.0);
}

__global__ void real_to_complex32_kernel(const double* __restrict__ x, float2* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = make_float2((float)x[i], 0.0f);
}
__global__ void complex32_real_part_kernel(const float2* __restrict__ x, double* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (double)x[i].x;
}
__global__ void to_float_kernel(const double* __restrict__ x, float* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void complex_real_part_kernel(const double2* __restrict__ x, double* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = x[i].x;
}

__global__ void axpby_kernel(long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

// ------------------------------------------------------------ reductions
// partial[block] = sum over the block's grid-stride share of x[i] * y[i]
__global__ void dot_partial_kernel(const double* __restrict__ x, const double* __restrict__ y, long n,
                                   double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  double s = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    s = fma(x[i], y[i], s);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void sum_final_kernel(const double* __restrict__ partial, int n, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Row sums of squares: out[r] = sum_c x[r * ld + c]^2 (one wavefront-strided
// block per row).
__global__ void row_sumsq_kernel(const double* __restrict__ x, long rows, long cols, long ld,
                                 double* __restrict__ out) {
  __shared__ double sh[kBlock];
  for (long r = blockIdx.x; r < rows; r += gridDim.x) {
    double s = 0.0;
    for (long c = threadIdx.x; c < cols; c += blockDim.x) {
      const double v = x[r * ld + c];
      s = fma(v, v, s);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = sh[0];
    __syncthreads();
  }
}

// Column sums of squares: out[c] = sum_r x[r * ld + c]^2.
__global__ void col_sumsq_kernel(const double* __restrict__ x, long rows, long cols, long ld,
                                 double* __restrict__ out) {
  const long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (long r = 0; r < rows; ++r) {
    const double v = x[r * ld + c];
    s = fma(v, v, s);
  }
  out[c] = s;
}

// --------------------------------------------- shifted triangular solves
// y[a, :, b] = (T + (lamL[a] + lamR[b]) I)^{-1} h[a, :, b], T upper triangular
// m x m (complex), h complex [r1][m][r2], in place.  One thread per (a, b):
// the vector lives in registers (compile-time bound MAXM, fully unrolled
// column-oriented back substitution), T is broadcast from LDS.
template <int MAXM, class R>
__global__ void __launch_bounds__(128)
kron_trisolve_kernel(int r1, int m, int r2, const typename CxOf<R>::type* __restrict__ T,
                     const typename CxOf<R>::type* __restrict__ lamL, const typename CxOf<R>::type* __restrict__ lamR,
                     typename CxOf<R>::type* __restrict__ h) {
  using C = typename CxOf<R>::type;
  using CX = CxOf<R>;
  __shared__ C Ts[MAXM * MAXM];
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) Ts[(e / m) * MAXM + (e % m)] = T[e];
  __syncthreads();
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)r1 * r2) return;
  const int a = (int)(t / r2), b = (int)(t % r2);
  const C s = cadd(lamL[a], lamR[b]);
  C* base = h + (long)a * m * r2 + b;
  C v[MAXM];
#pragma unroll
  for (int i = 0; i < MAXM; ++i) v[i] = (i < m) ? base[(long)i * r2] : CX::make(R(0), R(0));
#pragma unroll
  for (int k = MAXM - 1; k >= 0; --k) {
    if (k < m) {
      C dkk = cadd(Ts[k * MAXM + k], s);
      if (dkk.x == R(0) && dkk.y == R(0)) dkk.x = sizeof(R) == 8 ? R(1e-300) : R(1e-37f);
      v[k] = cdiv(v[k], dkk);
#pragma unroll
      for (int i = 0; i < k; ++i) v[i] = csub(v[i], cmul(Ts[i * MAXM + k], v[k]));
    }
  }
#pragma unroll
  for (int i = 0; i < MAXM; ++i)
    if (i < m) base[(long)i * r2] = v[i];
}

template <class T>
__global__ void transpose_kernel(long rows, long cols, const T* __restrict__ in, long ldi, T* __restrict__ out,
                                 long ldo) {
  __shared__ T tile[32][33];
  const long r0 = blockIdx.y * 32L, c0 = blockIdx.x * 32L;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const long r = r0 + k, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[k][threadIdx.x] = in[r * ldi + c];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const long c = c0 + k, r = r0 + threadIdx.x;
    if (r < rows && c < cols) out[c * ldo + r] = tile[threadIdx.x][k];
  }
}

template <class C>
__global__ void diag_complex_kernel(int n, const C* __restrict__ M, long ld, C* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = M[(long)i * (ld + 1)];
}

__global__ void gather_cols_kernel(long rows, int k, const double* __restrict__ src, long lds,
                                   const int* __restrict__ idx, double* __restrict__ dst, long ldd) {
  const long n = rows * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const long r = e / k;
    const int j = (int)(e % k);
    dst[r * ldd + j] = src[r * lds + idx[j]];
  }
}

__device__ inline unsigned long long mix64(unsigned long long z) {
  // SplitMix64 finaliser
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__global__ void fill_random_kernel(double* x, long n, unsigned long long seed) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const unsigned long long a = mix64(seed * 0x100000001B3ULL + 2ULL * i);
    const unsigned long long b = mix64(seed * 0x100000001B3ULL + 2ULL * i + 1ULL);
    const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
    x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

}  // namespace

// ======================================================== host launchers
void ttm_permute(hipStream_t s, int R0, int R1, int n, const double* A, double* Ahat) {
  const long tot = (long)R0 * n * n * R1;
  hipLaunchKernelGGL(ttm_permute_kernel, dim3(grid_for(tot)), dim3(kBlock), 0, s, R0, R1, n, A, Ahat);
  T2S2_LAUNCH_CHECK();
}

void fill(hipStream_t s, double* x, long n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, v);
  T2S2_LAUNCH_CHECK();
}

void fill(hipStream_t s, double2* x, long n, double2 v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel<double2>, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, v);
  T2S2_LAUNCH_CHECK();
}

void copy2d(hipStream_t s, long rows, long cols, const double* src, long lds, double* dst, long ldd,
            double alpha, int batch, long ss, long sd) {
  if (rows <= 0 || cols <= 0 || batch <= 0) return;
  dim3 grid(grid_for(rows * cols, kBlock, 4096), batch);
  hipLaunchKernelGGL(copy2d_kernel<double>, grid, dim3(kBlock), 0, s, rows, cols, src, lds, ss, dst, ldd, sd, alpha);
  T2S2_LAUNCH_CHECK();
}

void real_to_complex(hipStream_t s, const double* x, double2* y, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(real_to_complex_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  T2S2_LAUNCH_CHECK();
}

void real_to_complex(hipStream_t s, const double* x, float2* y, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(real_to_complex32_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  T2S2_LAUNCH_CHECK();
}

void complex_real_part(hipStream_t s, const float2* x, double* y, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(complex32_real_part_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  T2S2_LAUNCH_CHECK();
}

void to_float(hipStream_t s, const double* x, float* y, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(to_float_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  T2S2_LAUNCH_CHECK();
}

void complex_real_part(hipStream_t s, const double2* x, double* y, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(complex_real_part_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  T2S2_LAUNCH_CHECK();
}

void axpby(hipStream_t s, long n, double a, const double* x, double b, double* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, a, x, b, y);
  T2S2_LAUNCH_CHECK();
}

void dot_device(hipStream_t s, const double* x, const double* y, long n, double* partial, double* out) {
  const int g = grid_for(n, kBlock, kDotBlocks);
  hipLaunchKernelGGL(dot_partial_kernel, dim3(g), dim3(kBlock), 0, s, x, y, n, partial);
  T2S2_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(kBlock), 0, s, partial, g, out);
  T2S2_LAUNCH_CHECK();
}

void row_sumsq(hipStream_t s, const double* x, long rows, long cols, long ld, double* out) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(row_sumsq_kernel, dim3((int)std::min<long>(rows, 4096)), dim3(kBlock), 0, s, x, rows, cols, ld, out);
  T2S2_LAUNCH_CHECK();
}

void col_sumsq(hipStream_t s, const double* x, long rows, long cols, long ld, double* out) {
  if (cols <= 0) return;
  hipLaunchKernelGGL(col_sumsq_kernel, dim3((int)((cols + 127) / 128)), dim3(128), 0, s, x, rows, cols, ld, out);
  T2S2_LAUNCH_CHECK();
}

template <class R>
static void kron_trisolve_t(hipStream_t s, int r1, int m, int r2, const typename CxOf<R>::type* T,
                            const typename CxOf<R>::type* lamL, const typename CxOf<R>::type* lamR,
                            typename CxOf<R>::type* h) {
  T2S2_CHECK(m >= 1 && m <= 64, "kron_trisolve: mode size must be in [1, 64]");
  const long nthr = (long)r1 * r2;
  const int grid = (int)((nthr + 127) / 128);
  const double cb = 2.0 * sizeof(R);
  TimedScope ts(s, KC_KRONSOLVE, cb * (2.0 * nthr * m + (double)m * m + r1 + r2), 8.0 * nthr * m * (m + 1) / 2.0);
  if (m <= 16)
    hipLaunchKernelGGL((kron_trisolve_kernel<16, R>), dim3(grid), dim3(128), 0, s, r1, m, r2, T, lamL, lamR, h);
  else if (m <= 32)
    hipLaunchKernelGGL((kron_trisolve_kernel<32, R>), dim3(grid), dim3(128), 0, s, r1, m, r2, T, lamL, lamR, h);
  else
    hipLaunchKernelGGL((kron_trisolve_kernel<64, R>), dim3(grid), dim3(128), 0, s, r1, m, r2, T, lamL, lamR, h);
  T2S2_LAUNCH_CHECK();
}

void kron_trisolve(hipStream_t s, int r1, int m, int r2, const double2* T, const double2* lamL,
                   const double2* lamR, double2* h) {
  kron_trisolve_t<double>(s, r1, m, r2, T, lamL, lamR, h);
}
void kron_trisolve(hipStream_t s, int r1, int m, int r2, const float2* T, const float2* lamL,
                   const float2* lamR, float2* h) {
  kron_trisolve_t<float>(s, r1, m, r2, T, lamL, lamR, h);
}

void transpose(hipStream_t s, long rows, long cols, const double* in, long ldi, double* out, long ldo) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(transpose_kernel<double>, grid, dim3(32, 8), 0, s, rows, cols, in, ldi, out, ldo);
  T2S2_LAUNCH_CHECK();
}

void transpose(hipStream_t s, long rows, long cols, const double2* in, long ldi, double2* out, long ldo) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(transpose_kernel<double2>, grid, dim3(32, 8), 0, s, rows, cols, in, ldi, out, ldo);
  T2S2_LAUNCH_CHECK();
}

void diag_complex(hipStream_t s, int n, const double2* M, long ld, double2* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(diag_complex_kernel<double2>, dim3((n + 255) / 256), dim3(256), 0, s, n, M, ld, out);
  T2S2_LAUNCH_CHECK();
}

void diag_complex(hipStream_t s, int n, const float2* M, long ld, float2* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(diag_complex_kernel<float2>, dim3((n + 255) / 256), dim3(256), 0, s, n, M, ld, out);
  T2S2_LAUNCH_CHECK();
}

void gather_cols(hipStream_t s, long rows, int k, const double* src, long lds, const int* idx, double* dst, long ldd) {
  if (rows <= 0 || k <= 0) return;
  hipLaunchKernelGGL(gather_cols_kernel, dim3(grid_for(rows * k, kBlock, 4096)), dim3(kBlock), 0, s, rows, k, src,
                     lds, idx, dst, ldd);
  T2S2_LAUNCH_CHECK();
}

void fill_random(hipStream_t s, double* x, long n, unsigned long long seed) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_random_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, seed);
  T2S2_LAUNCH_CHECK();
}

}  // namespace t2s2
