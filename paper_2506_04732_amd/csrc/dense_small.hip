// Single-workgroup dense kernels for the small (r x r, r <= 512) matrices of
// the TT solver: Cholesky with column skipping, triangular inverses,
// one-sided Jacobi SVD, Hessenberg reduction, complex Schur form by shifted
// QR, and eigenvectors of triangular matrices.
//
// These matrices (interfaces, R factors, Gram matrices) are a few hundred KB
// at most; one workgroup of 1024 threads works on a copy staged in LDS when
// it fits (160 KB per workgroup on gfx950) and on global (L2-resident)
// memory otherwise.  Every kernel loops a bounded number of times and every
// barrier is reached by all threads of the workgroup.
#include "dense_small.h"
#include "readback.h"

#include <cfloat>
#include <cstring>

namespace t2s2 {

namespace {

constexpr int kNT = 1024;          // threads of the single workgroup
constexpr long kLdsDoubles = 20000;  // LDS budget of these kernels (160000 B)
constexpr long kLdsBytes = 160000;
constexpr int kJacG = 16;            // Jacobi: lanes per row pair
constexpr int kJacBG = 16;           // block Jacobi: lanes per row pair (32 measured slower)
constexpr int kJacBR = 16;           // block Jacobi: row entries per lane (c <= kJacBR kJacBG)

template <class R> struct TinyOf;   // a safe "negligible" magnitude
template <> struct TinyOf<double> { static constexpr double value = 1e-290; };
template <> struct TinyOf<float> { static constexpr float value = 1e-35f; };
template <class R> struct EpsOf;    // unit roundoff
template <> struct EpsOf<double> { static constexpr double value = DBL_EPSILON; };
template <> struct EpsOf<float> { static constexpr float value = FLT_EPSILON; };

__device__ inline double block_max(double v, double* red) {
  // all threads participate; red holds kNT/64 doubles
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < (int)(blockDim.x / 64); ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

// Sum over each aligned group of 16 lanes (a DPP row), left in every lane of
// the group, by data-parallel-primitive moves (VALU, no LDS round trip):
// swap with the xor-1 and xor-2 neighbours in the quad, then with the
// mirrored lane in the half row and in the row.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <class T>
__device__ inline T row16_sum(T v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return v;
}

// ------------------------------------------------------------ Cholesky
// Upper Cholesky G = R^T R of a symmetric positive semi-definite n x n
// matrix (row-major, ld n), skipping every column whose pivot, after the
// updates of the previous columns, is <= tau * max_i G[i][i]: such a column
// gets a zero row in R and mask 0.  count[0] = number of kept columns.
template <bool LDS>
__global__ void __launch_bounds__(kNT) chol_skip_kernel(int n, const double* __restrict__ G, double* R,
                                                       int* __restrict__ mask, int* __restrict__ count,
                                                       double tau) {
  extern __shared__ double lds[];
  __shared__ double red[kNT / 64];
  __shared__ double s_piv;
  __shared__ int s_keep, s_count;
  double* W;
  if constexpr (LDS) W = lds; else W = R;
  const long nn = (long)n * n;
  for (long e = threadIdx.x; e < nn; e += blockDim.x) W[e] = G[e];
  __syncthreads();
  double dm = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dm = fmax(dm, W[(long)i * n + i]);
  const double gmax = block_max(dm, red);
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double d = W[(long)k * n + k];
      const int keep = (d > tau * gmax) && (d > 0.0) && gmax > 0.0;
      s_keep = keep;
      s_piv = keep ? sqrt(d) : 0.0;
      mask[k] = keep;
      s_count += keep;
    }
    __syncthreads();
    const int keep = s_keep;
    const double piv = s_piv;
    if (!keep) {
      for (int j = k + threadIdx.x; j < n; j += blockDim.x) W[(long)k * n + j] = 0.0;
      __syncthreads();
      continue;
    }
    const double inv = 1.0 / piv;
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) W[(long)k * n + j] *= inv;
    if (threadIdx.x == 0) W[(long)k * n + k] = piv;
    __syncthreads();
    const int t = n - k - 1;
    const long tt = (long)t * t;
    for (long e = threadIdx.x; e < tt; e += blockDim.x) {
      const int i = k + 1 + (int)(e / t), j = k + 1 + (int)(e % t);
      if (i <= j) W[(long)i * n + j] -= W[(long)k * n + i] * W[(long)k * n + j];
    }
    __syncthreads();
  }
  for (long e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    R[e] = (j < i) ? 0.0 : W[e];
  }
  if (threadIdx.x == 0) count[0] = s_count;
}

// Register-resident versions for n <= NMAX on one wavefront: lane j holds
// column j in registers and every other entry it needs is read from the lane
// that holds it (compile-time lane and row indices after unrolling), so no
// step waits on LDS or a barrier.  Same arithmetic, in the same order, as the
// workgroup kernels above and below.
__device__ inline double rdl(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline float rdl(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }

// sum over the wavefront, in every lane: DPP sums of the four 16-lane rows,
// then the rows' sums read from lanes 0, 16, 32 and 48
template <class T>
__device__ inline T wave_sum64(T v) {
  v = row16_sum(v);
  return (rdl(v, 0) + rdl(v, 16)) + (rdl(v, 32) + rdl(v, 48));
}

template <int NMAX>
__global__ void __launch_bounds__(64) chol_skip_reg_kernel(int n, const double* __restrict__ G, double* R,
                                                          int* __restrict__ mask, int* __restrict__ count,
                                                          double tau) {
  // row k of the matrix is broadcast through the wavefront's LDS row (one
  // write per lane, then same-address reads) rather than by lane reads
  __shared__ double row[64];
  const int j = threadIdx.x;
  double g[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i) g[i] = (i < n && j < n) ? G[i * n + j] : 0.0;
  double gmax = (j < n) ? G[j * n + j] : 0.0;
  for (int off = 32; off > 0; off >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, off, 64));
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (k < n) {
      __builtin_amdgcn_wave_barrier();
      row[j] = g[k];
      __builtin_amdgcn_wave_barrier();
      const double d = row[k];
      const int keep = (d > tau * gmax) && (d > 0.0) && gmax > 0.0;
      if (j == 0) mask[k] = keep;
      cnt += keep;
      if (!keep) {
        if (j >= k) g[k] = 0.0;
      } else {
        const double piv = sqrt(d);
        const double inv = 1.0 / piv;
        if (j > k) g[k] *= inv;
        if (j == k) g[k] = piv;
#pragma unroll
        for (int i = k + 1; i < NMAX; ++i) {
          if (i < n) {
            const double rki = row[i] * inv;
            if (j >= i && j < n) g[i] -= rki * g[k];
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < n && j < n) R[i * n + j] = (j < i) ? 0.0 : g[i];
  if (j == 0) count[0] = cnt;
}

// Blocked right-looking form of chol_skip_kernel for 32 < n <= 256, columns
// taken kCholP at a time.  Each panel is one pass in which every wavefront
// factors the panel's diagonal block in lanes 0..31 (one column per lane; all
// wavefronts compute the same values) and carries 32 trailing columns
// through the same steps in lanes 32..63.  At step k the diagonal lanes
// write their row-k entries to the wavefront's own LDS row, and every lane
// reads the pivot and the row back (the pivot test is chol_skip_kernel's).
// The trailing upper triangle then receives the panel's updates in 4 x 4
// tiles.  Each entry gets the same operations in the same order as in
// chol_skip_kernel (scaling by the pivot's reciprocal, then one subtraction
// per earlier kept column, in column order), so R is bitwise identical; the
// workgroup meets 2 barriers per panel instead of 3 per column.
// LDS: W holds the matrix (n*n doubles); otherwise W is R in global memory
// and the panel's rows are copied to LDS for the trailing update.
constexpr int kCholP = 32;
constexpr int kCholBlkMax = 256;
constexpr int kCholNT = 512;  // 8 wavefronts: 8 x 32 trailing columns per panel

// The steps of one panel in one wavefront (see chol_blk_kernel): g holds the
// lane's column within the panel rows, row is the wavefront's LDS row.  Lanes
// other than the diagonal block's upper part and the valid trailing columns
// are updated too (their values are never read or stored), which keeps the
// steps free of per-lane conditions.  W = kCholP: a full panel (w == kCholP).
template <int W>
__device__ __forceinline__ void chol_panel(double (&g)[kCholP], double* row, int w, int lane, bool diag, int wv,
                                           double tau, double gmax, int* __restrict__ mask, int* s_keep, int& cnt) {
  if constexpr (W > 0) w = W;
#pragma unroll
  for (int k = 0; k < kCholP; ++k) {
    if (W > 0 || k < w) {
      if (diag) row[lane] = g[k];
      __builtin_amdgcn_wave_barrier();
      const double d = row[k];
      const int keep = (d > tau * gmax) && (d > 0.0) && gmax > 0.0;
      if (wv == 0 && lane == 0) {
        mask[k] = keep;
        s_keep[k] = keep;
      }
      cnt += keep;
      const bool right = !diag || lane > k;  // entries right of the pivot in row k
      if (!keep) {
        if (right || lane == k) g[k] = 0.0;
      } else {
        const double piv = sqrt(d);
        const double inv = 1.0 / piv;
        g[k] = (diag && lane == k) ? piv : (right ? g[k] * inv : g[k]);
#pragma unroll
        for (int i = k + 1; i < kCholP; ++i)
          if (W > 0 || i < w) g[i] -= (row[i] * inv) * g[k];
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <bool LDS>
__global__ void __launch_bounds__(kCholNT) chol_blk_kernel(int n, const double* __restrict__ G, double* R,
                                                           int* __restrict__ mask, int* __restrict__ count,
                                                           double tau) {
  extern __shared__ double lds[];
  __shared__ double red[kNT / 64];
  __shared__ double rows[kCholNT / 64][kCholP];  // per wavefront: the current row of the diagonal block
  __shared__ int s_keep[kCholP];
  double* W;
  if constexpr (LDS) W = lds; else W = R;
  const long nn = (long)n * n;
  for (long e = threadIdx.x; e < nn; e += blockDim.x) W[e] = G[e];
  __syncthreads();
  double dm = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dm = fmax(dm, W[(long)i * n + i]);
  const double gmax = block_max(dm, red);
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const bool diag = lane < kCholP;
  int cnt = 0;  // kept columns, tracked by wavefront 0
  for (int k0 = 0; k0 < n; k0 += kCholP) {
    const int w = min(kCholP, n - k0);
    const int c0 = k0 + w;  // first trailing column
    const int col = diag ? k0 + lane : c0 + kCholP * wv + (lane - kCholP);
    const bool valid = diag ? lane < w : col < n;
    double* P;  // row k of the panel at P[k * n + column]
    if constexpr (LDS) P = W + (long)k0 * n; else P = lds;
    if (wv == 0 || c0 + kCholP * wv < n) {  // wavefronts with trailing columns, and wavefront 0
      double g[kCholP];
#pragma unroll
      for (int i = 0; i < kCholP; ++i)
        g[i] = (i < w && valid && (!diag || i <= lane)) ? W[(long)(k0 + i) * n + col] : 0.0;
      if (w == kCholP)
        chol_panel<kCholP>(g, rows[wv], kCholP, lane, diag, wv, tau, gmax, mask + k0, s_keep, cnt);
      else
        chol_panel<0>(g, rows[wv], w, lane, diag, wv, tau, gmax, mask + k0, s_keep, cnt);
#pragma unroll
      for (int i = 0; i < kCholP; ++i) {
        if (i < w && valid && (!diag || (wv == 0 && i <= lane))) {
          W[(long)(k0 + i) * n + col] = g[i];
          if constexpr (!LDS) if (!diag) P[(long)i * n + col] = g[i];
        }
      }
    }
    __syncthreads();
    // trailing upper triangle: 4 x 4 tiles (bi <= bj), column-major over the tiles;
    // the panel's rows are read 4 at a time
    const int t = n - c0;
    const int T4 = (t + 3) / 4;
    const int ntile = T4 * (T4 + 1) / 2;
    for (int q = threadIdx.x; q < ntile; q += blockDim.x) {
      int bj = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
      while (bj * (bj + 1) / 2 > q) --bj;
      while ((bj + 1) * (bj + 2) / 2 <= q) ++bj;
      const int bi = q - bj * (bj + 1) / 2;
      const int i0 = c0 + 4 * bi, j0 = c0 + 4 * bj;
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = i0 + a, j = j0 + b;
          acc[a][b] = (i <= j && j < n) ? W[(long)i * n + j] : 0.0;
        }
#pragma unroll
      for (int k4 = 0; k4 < kCholP; k4 += 4) {
        if (k4 < w) {
          double u[4][4], v[4][4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const bool in = k4 + kk < w;
              u[kk][a] = (in && i0 + a < n) ? P[(long)(k4 + kk) * n + i0 + a] : 0.0;
              v[kk][a] = (in && j0 + a < n) ? P[(long)(k4 + kk) * n + j0 + a] : 0.0;
            }
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            if (k4 + kk < w && s_keep[k4 + kk]) {
#pragma unroll
              for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] -= u[kk][a] * v[kk][b];
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = i0 + a, j = j0 + b;
          if (i <= j && j < n) W[(long)i * n + j] = acc[a][b];
        }
    }
    __syncthreads();
  }
  for (long e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    R[e] = (j < i) ? 0.0 : W[e];
  }
  if (threadIdx.x == 0) count[0] = cnt;
}

// lane j computes column j of R^{-1}; the dot products keep the eight
// strided partial sums and the pairwise combination of the workgroup kernel
template <int NMAX>
__global__ void __launch_bounds__(64) trtri_reg_kernel(int n, const double* __restrict__ R,
                                                      double* __restrict__ Rinv) {
  // R is staged in LDS; row i's entries are same-address reads for every lane
  __shared__ double Rs[NMAX * NMAX];
  const int j = threadIdx.x;
  double x[NMAX];
  for (int e = j; e < n * n; e += 64) Rs[(e / n) * NMAX + e % n] = R[e];
#pragma unroll
  for (int i = 0; i < NMAX; ++i) x[i] = 0.0;
  __syncthreads();
#pragma unroll
  for (int i = NMAX - 1; i >= 0; --i) {
    if (i < n) {
      const double rii = Rs[i * NMAX + i];
      double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = i + 1; t < NMAX; ++t) {
        if (t < n) {
          const double rit = Rs[i * NMAX + t];
          if (t <= j) p[(t - i - 1) & 7] = fma(rit, x[t], p[(t - i - 1) & 7]);
        }
      }
      const double sm = ((p[0] + p[4]) + (p[2] + p[6])) + ((p[1] + p[5]) + (p[3] + p[7]));
      if (j == i) x[i] = 1.0 / rii;
      else if (j > i) x[i] = (-sm) / rii;
    }
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < n && j < n) Rinv[i * n + j] = x[i];
}

// ------------------------------------------------- triangular inverses
// Rinv = R^{-1} for a nonsingular upper-triangular n x n R (row-major), by
// rows from the bottom: Rinv[i][j] = -(sum_{t=i+1..j} R[i][t] Rinv[t][j]) / R[i][i].
template <class T>
struct TriOps;
template <>
struct TriOps<double> {
  __device__ static double zero() { return 0.0; }
  __device__ static double one() { return 1.0; }
  __device__ static double fma(double a, double b, double c) { return ::fma(a, b, c); }
  __device__ static double div(double a, double b) { return a / b; }
  __device__ static double neg(double a) { return -a; }
};
template <>
struct TriOps<double2> {
  __device__ static double2 zero() { return make_double2(0.0, 0.0); }
  __device__ static double2 one() { return make_double2(1.0, 0.0); }
  // c + a b with explicit fused operations, so every kernel rounds it alike
  __device__ static double2 fma(double2 a, double2 b, double2 c) {
    return make_double2(::fma(a.x, b.x, ::fma(-a.y, b.y, c.x)), ::fma(a.x, b.y, ::fma(a.y, b.x, c.y)));
  }
  __device__ static double2 div(double2 a, double2 b) { return cdiv(a, b); }
  __device__ static double2 neg(double2 a) { return make_double2(-a.x, -a.y); }
};

template <>
struct TriOps<float2> {
  __device__ static float2 zero() { return make_float2(0.0f, 0.0f); }
  __device__ static float2 one() { return make_float2(1.0f, 0.0f); }
  __device__ static float2 fma(float2 a, float2 b, float2 c) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
  }
  __device__ static float2 div(float2 a, float2 b) { return cdiv(a, b); }
  __device__ static float2 neg(float2 a) { return make_float2(-a.x, -a.y); }
};

template <class T>
__device__ inline T shfl_xor_t(T v, int off, int width);
template <>
__device__ inline double shfl_xor_t<double>(double v, int off, int width) { return __shfl_xor(v, off, width); }
template <>
__device__ inline double2 shfl_xor_t<double2>(double2 v, int off, int width) {
  return make_double2(__shfl_xor(v.x, off, width), __shfl_xor(v.y, off, width));
}
template <>
__device__ inline float2 shfl_xor_t<float2>(float2 v, int off, int width) {
  return make_float2(__shfl_xor(v.x, off, width), __shfl_xor(v.y, off, width));
}
template <class T>
__device__ inline T tadd(T a, T b);
template <>
__device__ inline double tadd<double>(double a, double b) { return a + b; }
template <>
__device__ inline double2 tadd<double2>(double2 a, double2 b) { return cadd(a, b); }
template <>
__device__ inline float2 tadd<float2>(float2 a, float2 b) { return cadd(a, b); }

// Each entry's dot product is split over a group of kTriG lanes (strided
// terms, shuffle reduction), so a row's dependent chain is ~n / kTriG long.
constexpr int kTriG = 8;

template <class T>
__global__ void __launch_bounds__(kNT) trtri_upper_kernel(int n, const T* __restrict__ R, T* __restrict__ Rinv) {
  using O = TriOps<T>;
  const long nn = (long)n * n;
  const int grp = threadIdx.x / kTriG, sub = threadIdx.x % kTriG, ngrp = blockDim.x / kTriG;
  for (long e = threadIdx.x; e < nn; e += blockDim.x) Rinv[e] = O::zero();
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    const T rii = R[(long)i * n + i];
    for (int j0 = i; j0 < n; j0 += ngrp) {
      const int j = j0 + grp;
      T s = O::zero();
      if (j < n)
        for (int t = i + 1 + sub; t <= j; t += kTriG) s = O::fma(R[(long)i * n + t], Rinv[(long)t * n + j], s);
      for (int off = kTriG / 2; off > 0; off >>= 1) s = tadd<T>(s, shfl_xor_t<T>(s, off, kTriG));
      if (j < n && sub == 0) Rinv[(long)i * n + j] = (j == i) ? O::div(O::one(), rii) : O::div(O::neg(s), rii);
    }
    __syncthreads();
  }
}

// The value of lane L ^ X (X = 1, 2, 4) within aligned groups of 8 lanes, by
// DPP moves: xor 1 and xor 2 are quad permutations; xor 4 is the half-row
// mirror (L -> L ^ 7) followed by the quad reversal (L -> L ^ 3).  Pure data
// movement, so a butterfly built on it gives the same bits as one built on
// __shfl_xor.
template <int X>
__device__ inline double xor8_move(double v) {
  if constexpr (X == 1) return dpp_move<0xB1>(v);
  else if constexpr (X == 2) return dpp_move<0x4E>(v);
  else return dpp_move<0x1B>(dpp_move<0x141>(v));
}
template <int X>
__device__ inline float xor8_move(float v) {
  if constexpr (X == 1) return dpp_move<0xB1>(v);
  else if constexpr (X == 2) return dpp_move<0x4E>(v);
  else return dpp_move<0x1B>(dpp_move<0x141>(v));
}
template <int X>
__device__ inline double2 xor8_move(double2 v) { return make_double2(xor8_move<X>(v.x), xor8_move<X>(v.y)); }
template <int X>
__device__ inline float2 xor8_move(float2 v) { return make_float2(xor8_move<X>(v.x), xor8_move<X>(v.y)); }

// The columns of R^{-1} are independent, so for n <= kTriColMax each group of
// kTriG lanes of a one-wavefront workgroup computes one column on its own,
// without barriers: workgroup b owns columns kTriG b .. kTriG b + kTriG - 1.
// Lane s of a group keeps the entries x[t] of its column with t = s (mod kTriG)
// in registers.  For row i the lane's partial sum runs over the same terms in
// the same order as lane (s - i - 1) mod kTriG of the workgroup kernel, and
// the xor butterfly pairs the same partial sums, so every entry is bitwise
// identical to that kernel's (for finite R; the butterfly moves data by DPP
// instead of shuffles).  Rows of R are staged in LDS kTriG at a time (the row
// block and the columns up to the group's last one); the next block is
// loaded into registers while the current one is used.
constexpr int kTriColMax = 256;
constexpr int kTriColBlocks = kTriColMax / kTriG;

// Entry i of the eigenvector of column j of a triangular matrix:
// -s / (t_ii - t_jj), the denominator raised to smin = max(ulp |t_jj|, tiny)
// in modulus when smaller (shared by both eigenvector kernels)
template <class C>
struct RealOfCx;
template <>
struct RealOfCx<double2> { using type = double; };
template <>
struct RealOfCx<float2> { using type = float; };
template <class C>
__device__ inline C trevec_entry(C s, C tii, C tjj) {
  using R = typename RealOfCx<C>::type;
  using CX = CxOf<R>;
  C den = csub(tii, tjj);
  const R smin = fmax(EpsOf<R>::value * cabs(tjj), TinyOf<R>::value);
  if (cabs(den) < smin) den = CX::make(smin, R(0.0));
  return cdiv(CX::make(-s.x, -s.y), den);
}

// register slots for the next row block's entries (the rest is loaded when staged)
template <class T>
constexpr int tri_col_slots() { return sizeof(T) > 8 ? kTriColBlocks / 2 : kTriColBlocks; }

// one row block MI of trtri_col_kernel, then the blocks above it
template <class T, bool EV, int MI>
__device__ __forceinline__ void trtri_col_block(int n, int B, int j, int s, int lr, int lc, const T* __restrict__ R,
                                                T* __restrict__ Rinv, T* tile, T (&x)[kTriColBlocks],
                                                T (&pre)[tri_col_slots<T>()], T tjj) {
  if constexpr (MI >= 0) {
    using O = TriOps<T>;
    constexpr int MB = kTriColBlocks, LD = kTriColMax;
    if (MI <= B) {
      if constexpr (MI > 0) {
        const int row = kTriG * (MI - 1) + lr;
#pragma unroll
        for (int q = 0; q <= MB - MI && q < tri_col_slots<T>(); ++q) {
          const int col = kTriG * (MI - 1 + q) + lc;
          if (q <= B - MI + 1) pre[q] = (row < n && col < n) ? R[(long)row * n + col] : O::zero();
        }
      }
      for (int r = kTriG - 1; r >= 0; --r) {
        const int i = kTriG * MI + r;
        if (i >= n) continue;
        // the row's entries are read CH at a time, all in flight before the
        // fused steps.  Terms outside i < t <= j need no test: their x[t] is
        // still exactly zero (rows past the column's last are never set, rows
        // up to i not yet), the staged entries are finite (the tile starts
        // zeroed), and the partial sum starts at +0 so it can never become -0:
        // adding such a term leaves it bitwise unchanged.
        constexpr int CH = sizeof(T) > 8 ? 4 : 8;
        T p = O::zero();
#pragma unroll
        for (int m0 = MI; m0 < MB; m0 += CH) {
          if (m0 <= B) {
            T a[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u)
              if (m0 + u < MB) a[u] = tile[r * LD + s + kTriG * (m0 + u - MI)];
#pragma unroll
            for (int u = 0; u < CH; ++u)
              if (m0 + u < MB) p = O::fma(a[u], x[m0 + u], p);
          }
        }
        p = tadd<T>(p, xor8_move<4>(p));
        p = tadd<T>(p, xor8_move<2>(p));
        p = tadd<T>(p, xor8_move<1>(p));
        const T rii = tile[r * LD + r];
        if constexpr (!EV) {
          if (i <= j) {
            const T xi = (i == j) ? O::div(O::one(), rii) : O::div(O::neg(p), rii);
            if (s == r) x[MI] = xi;
            if (s == 0) Rinv[(long)i * n + j] = xi;
          }
        } else {
          // eigenvector of column j: y_j = 1 (kept out of x: its term T[i][j] is
          // added after the butterfly, as in trevec_kernel)
          if (i < j) {
            const T xi = trevec_entry(tadd<T>(p, tile[r * LD + j - kTriG * MI]), rii, tjj);
            if (s == r) x[MI] = xi;
            if (s == 0) Rinv[(long)i * n + j] = xi;
          } else if (i == j && s == 0) {
            Rinv[(long)i * n + j] = O::one();
          }
        }
      }
      if constexpr (MI > 0) {
        __syncthreads();
        const int row = kTriG * (MI - 1) + lr;
#pragma unroll
        for (int q = 0; q <= MB - MI; ++q) {
          if (q <= B - MI + 1) {
            if (q < tri_col_slots<T>()) {
              tile[lr * LD + kTriG * q + lc] = pre[q];
            } else {
              const int col = kTriG * (MI - 1 + q) + lc;
              tile[lr * LD + kTriG * q + lc] = (row < n && col < n) ? R[(long)row * n + col] : O::zero();
            }
          }
        }
        __syncthreads();
      }
    }
    trtri_col_block<T, EV, MI - 1>(n, B, j, s, lr, lc, R, Rinv, tile, x, pre, tjj);
  }
}

// EV: eigenvectors of the triangular R instead (trevec_kernel's results)
template <class T, bool EV>
__global__ void __launch_bounds__(64) trtri_col_kernel(int n, const T* __restrict__ R, T* __restrict__ Rinv) {
  using O = TriOps<T>;
  __shared__ T tile[kTriG * kTriColMax];
  const int lane = threadIdx.x, s = lane % kTriG;
  const int B = blockIdx.x;                // last row block this workgroup needs
  const int j0 = kTriG * B + lane / kTriG;
  const int j = (j0 < n) ? j0 : -1;        // -1: a group past the last column
  for (int i = j0 + 1 + s; i < n && j >= 0; i += kTriG) Rinv[(long)i * n + j] = O::zero();
  // staging: lane l holds row kTriG mi + l / kTriG, columns kTriG (mi + q) + l % kTriG
  const int lr = lane / kTriG, lc = lane % kTriG;
  for (int e = lane; e < kTriG * kTriColMax; e += 64) tile[e] = O::zero();
  __syncthreads();
  T pre[tri_col_slots<T>()];
  T x[kTriColBlocks];
#pragma unroll
  for (int m = 0; m < kTriColBlocks; ++m) x[m] = O::zero();
  {
    const int row = kTriG * B + lr;
    const int col = kTriG * B + lc;
    tile[lr * kTriColMax + lc] = (row < n && col < n) ? R[(long)row * n + col] : O::zero();
  }
  __syncthreads();
  const T tjj = (EV && j >= 0) ? R[(long)j * n + j] : O::zero();
  trtri_col_block<T, EV, kTriColBlocks - 1>(n, B, j, s, lr, lc, R, Rinv, tile, x, pre, tjj);
}

// ------------------------------------------------ one-sided Jacobi SVD
// 1/x from the hardware estimate refined by two Newton steps (full FP64
// accuracy for finite nonzero x), and 1/sqrt(x) likewise for x in [1, 2]
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double rsq_nr12(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x, y * y, 1.5);
  return y * fma(-0.5 * x, y * y, 1.5);
}

// Rotation (cs, sn), rows (x, y) -> (cs x - sn y, sn x + cs y), that makes
// two rows with squared norms a, b and inner product g orthogonal (the
// smaller of the two angles); false when |g| <= tol sqrt(a b) or the angle
// is below 1e-300.  The reciprocals come from refined hardware estimates:
// the rotation has to be orthogonal to working precision, not correctly
// rounded, and the shorter dependent chain is most of a Jacobi round's
// latency.
__device__ inline bool jacobi_rotation(double a, double b, double g, double tol, double& cs, double& sn) {
  if (g == 0.0 || g * g <= (tol * tol) * (a * b)) return false;
  const double zeta = (b - a) * rcp_nr(2.0 * g);
  const double d = fabs(zeta) + sqrt(fma(zeta, zeta, 1.0));  // >= 1
  if (!(d < 1e300)) return false;  // angle below 1e-300 (or g at underflow): nothing to rotate
  const double ta = rcp_nr(d);
  const double t = (zeta >= 0.0) ? ta : -ta;
  cs = rsq_nr12(fma(t, t, 1.0));
  sn = cs * t;
  return true;
}

// Sweeps stop once no pair had a squared cosine g^2 / (a b) above kJacStop2
// (cosine 1e-2) before its rotation: cyclic one-sided Jacobi converges
// quadratically, so the cosines left after that sweep are ~1e-4.  B = U Wt
// stays exact (U is a product of rotations) and the error of dropping rows of
// Wt is their Frobenius norm whatever their orthogonality, so what is left
// only makes the kept rows marginally less than optimal (a rank at most a
// little above the optimal one for the same error); the sweep that would
// confirm it is not run.
constexpr float kJacStop2 = 1e-4f;
// g^2 / (a b) as the bits of a non-negative float (ordered like ints)
__device__ inline int cos2_bits(double a, double b, double g) {
  const double ab = a * b;
  return __float_as_int(ab > 0.0 ? (float)((g * g) * rcp_nr(ab)) : 0.0f);
}

// Row norms of the rotated B (k x c), rows ranked by decreasing norm (ties by
// index) and scattered: Wt (sorted rows), U (column dest(i) = row i of JT),
// sigma (sorted norms); info[0] = sweeps, info[1..k] scratch.
__device__ void jacobi_finish(int k, int c, const double* Bw, const double* Jw, double* __restrict__ U,
                              double* __restrict__ Wt, double* __restrict__ sigma, int* __restrict__ info,
                              int sweep) {
  const long bsz = (long)k * c, jsz = (long)k * k;
  // row norms, rank by decreasing norm (ties by index), scatter
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double s = 0.0;
    for (int e = 0; e < c; ++e) s = fma(Bw[(long)i * c + e], Bw[(long)i * c + e], s);
    sigma[i] = sqrt(s);  // temporary, unsorted
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double si = sigma[i];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double sj = sigma[j];
      rank += (sj > si) || (sj == si && j < i);
    }
    info[1 + i] = rank;  // scratch: destination of row i
  }
  __syncthreads();
  for (long e = threadIdx.x; e < bsz; e += blockDim.x) {
    const int i = (int)(e / c), col = (int)(e % c);
    Wt[(long)info[1 + i] * c + col] = Bw[e];
  }
  // U = J: column dest(i) of U is row i of JT
  for (long e = threadIdx.x; e < jsz; e += blockDim.x) {
    const int i = (int)(e / k), r = (int)(e % k);
    U[(long)r * k + info[1 + i]] = Jw[e];
  }
  __syncthreads();
  // sorted sigma
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double s = 0.0;
    for (int e = 0; e < c; ++e) s = fma(Wt[(long)i * c + e], Wt[(long)i * c + e], s);
    sigma[i] = sqrt(s);
  }
  if (threadIdx.x == 0) info[0] = sweep;
}


// B (k x c, row-major) = U * Wt with U orthogonal k x k and the rows of Wt
// mutually orthogonal: rotations from the left orthogonalise the rows of B
// (Hestenes' method applied to B^T), the rotations accumulate in U.  Rows are
// then sorted by decreasing norm: sigma[i] = ||Wt[i, :]||, so B = U diag(sigma) V^T
// with V^T the normalised rows of Wt.  Pairs are visited in round-robin
// tournament order, k/2 disjoint pairs per round, one group of kJacG lanes
// per pair.
template <int MODE>
__global__ void __launch_bounds__(kNT) jacobi_rows_kernel(int k, int c, double* __restrict__ B,
                                                          double* __restrict__ JT, double* __restrict__ U,
                                                          double* __restrict__ Wt, double* __restrict__ sigma,
                                                          int* __restrict__ info, int max_sweeps) {
  extern __shared__ double lds[];
  __shared__ int s_rot, s_cmax;
  const long bsz = (long)k * c, jsz = (long)k * k;
  double* Bw;
  double* Jw;
  if constexpr (MODE >= 1) Bw = lds; else Bw = B;
  if constexpr (MODE == 2) Jw = lds + bsz; else Jw = JT;
  for (long e = threadIdx.x; e < bsz; e += blockDim.x) Bw[e] = B[e];
  for (long e = threadIdx.x; e < jsz; e += blockDim.x) Jw[e] = ((e / k) == (e % k)) ? 1.0 : 0.0;
  __syncthreads();
  const int K = k + (k & 1);  // even number of players (k odd: one bye)
  const int npairs = K / 2;
  // one group of kJacG lanes per pair: a round's pairs are independent, so
  // many of them are in flight at once
  const int grp = threadIdx.x / kJacG, sub = threadIdx.x % kJacG, ngrp = blockDim.x / kJacG;
  // rows are rotated until their cosines fall below tol: the factorisation
  // B = U Wt is exact for any tol (U is a product of rotations), so tol only
  // decides how well the energy is compacted into the leading rows
  const double tol = 1e-10;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) {
      s_rot = 0;
      s_cmax = 0;
    }
    __syncthreads();
    // this group's rotation count and largest squared cosine of the sweep
    // (one pair of shared atomics per group after the rounds, not per pair)
    int my_rot = 0, my_cmax = 0;
    for (int round = 0; round < K - 1; ++round) {
      for (int pi = grp; pi < npairs; pi += ngrp) {
        // slots pi and K-1-pi; slot 0 is fixed, the others rotate
        const int s1 = pi, s2 = K - 1 - pi;
        int p = (s1 == 0) ? 0 : ((s1 - 1 + round) % (K - 1)) + 1;
        int q = (s2 == 0) ? 0 : ((s2 - 1 + round) % (K - 1)) + 1;
        if (p >= k || q >= k) continue;
        if (p > q) { const int t = p; p = q; q = t; }
        double* bp = Bw + (long)p * c;
        double* bq = Bw + (long)q * c;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int e = sub; e < c; e += kJacG) {
          const double x = bp[e], y = bq[e];
          a = fma(x, x, a);
          b = fma(y, y, b);
          g = fma(x, y, g);
        }
        static_assert(kJacG == 16, "row16_sum reduces over 16 lanes");
        a = row16_sum(a);
        b = row16_sum(b);
        g = row16_sum(g);
        my_cmax = max(my_cmax, cos2_bits(a, b, g));
        double cs, sn;
        if (!jacobi_rotation(a, b, g, tol, cs, sn)) continue;
        for (int e = sub; e < c; e += kJacG) {
          const double x = bp[e], y = bq[e];
          bp[e] = cs * x - sn * y;
          bq[e] = sn * x + cs * y;
        }
        double* jp = Jw + (long)p * k;
        double* jq = Jw + (long)q * k;
        for (int e = sub; e < k; e += kJacG) {
          const double x = jp[e], y = jq[e];
          jp[e] = cs * x - sn * y;
          jq[e] = sn * x + cs * y;
        }
        ++my_rot;
      }
      __syncthreads();
    }
    if (sub == 0) {
      if (my_rot > 0) atomicAdd(&s_rot, my_rot);
      if (my_cmax > 0) atomicMax(&s_cmax, my_cmax);
    }
    __syncthreads();
    const int rot = s_rot;
    const float cmax = __int_as_float(s_cmax);
    __syncthreads();
    if (rot == 0 || cmax <= kJacStop2) break;
  }
  jacobi_finish(k, c, Bw, Jw, U, Wt, sigma, info, sweep);
}

// One-sided Jacobi for matrices beyond LDS (block Jacobi).  The rows of B
// (k x c) and of the rotation accumulator JT (k x k) are split into blocks of
// bsz rows.  A sweep is one launch in which workgroup b sweeps the row pairs
// inside block b (cross = 0, round-robin over its rows), then one launch per
// round of a round-robin pairing of the blocks (nplay players, a bye when the
// block count is odd) in which one workgroup per block pair (P, Q) rotates
// only the pairs between them (cross = 1: max(pn, qn) rounds of disjoint
// pairs, row i of P with row (i + round) mod max(pn, qn) of Q).  Every row
// pair is thus rotated once per sweep, as in cyclic Jacobi.  A workgroup
// loads its rows of B into LDS, accumulates its rotations in a small
// rows x rows matrix Jl, writes the B rows back and replaces its JT rows by
// Jl times them.  Each lane keeps its share of a row pair in registers
// between the dot products and the rotation (LG lanes per pair, c <= NR LG).  counter
// accumulates the rotations.
template <int NR, int LG>
__global__ void __launch_bounds__(kNT) jacobi_block_kernel(int k, int c, double* __restrict__ B,
                                                           double* __restrict__ JT, int bsz, int nblk, int nplay,
                                                           int round, int cross, int* __restrict__ counter) {
  extern __shared__ double lds[];
  __shared__ int s_rot, s_cmax;
  int P = blockIdx.x, Q = blockIdx.x;
  if (cross) {
    const int s1 = blockIdx.x, s2 = nplay - 1 - blockIdx.x;
    P = (s1 == 0) ? 0 : ((s1 - 1 + round) % (nplay - 1)) + 1;
    Q = (s2 == 0) ? 0 : ((s2 - 1 + round) % (nplay - 1)) + 1;
  }
  if (P >= nblk || Q >= nblk) return;  // bye
  const int p0 = P * bsz, pn = min(bsz, k - p0), q0 = Q * bsz, qn = cross ? min(bsz, k - q0) : 0;
  const int rows = pn + qn;
  double* Bw = lds;                     // rows x c (later: the old JT rows, rows x k, k <= c)
  double* Jl = lds + (long)rows * c;    // rows x rows
  auto grow = [&](int r) { return r < pn ? p0 + r : q0 + (r - pn); };
  for (long e = threadIdx.x; e < (long)rows * c; e += blockDim.x) {
    const int r = (int)(e / c), col = (int)(e % c);
    Bw[e] = B[(long)grow(r) * c + col];
  }
  for (int e = threadIdx.x; e < rows * rows; e += blockDim.x) Jl[e] = ((e / rows) == (e % rows)) ? 1.0 : 0.0;
  if (threadIdx.x == 0) {
    s_rot = 0;
    s_cmax = 0;
  }
  __syncthreads();
  const int RP = rows + (rows & 1);
  const int MQ = max(pn, qn);
  const int nrounds = cross ? MQ : RP - 1, npairs = cross ? pn : RP / 2;
  const int grp = threadIdx.x / LG, sub = threadIdx.x % LG, ngrp = blockDim.x / LG;
  const double tol = 1e-10;
  constexpr int NJ = 8;  // Jl entries per lane of a register-resident row
  // this group's rotation count and largest squared cosine (one pair of
  // shared atomics per group after the rounds, not per pair)
  int my_rot = 0, my_cmax = 0;
  if (cross && pn <= ngrp && rows <= NJ * LG) {
    // group pi keeps row pi of block P and its Jl row in registers through
    // every round; only the row of Q it meets passes through LDS (same
    // operations in the same order as the loop below)
    const bool own = grp < pn;
    double xs[NR], jx[NJ];
    if (own) {
      const double* bp = Bw + (long)grp * c;
      const double* jp = Jl + (long)grp * rows;
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int e = sub + u * LG;
        xs[u] = (e < c) ? bp[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NJ; ++u) {
        const int e = sub + u * LG;
        jx[u] = (e < rows) ? jp[e] : 0.0;
      }
    }
    for (int rr = 0; rr < nrounds; ++rr) {
      int q = own ? (grp + rr) % MQ : qn;
      if (q < qn) {
        q += pn;
        double* bq = Bw + (long)q * c;
        double ys[NR];
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int u = 0; u < NR; ++u) {
          const int e = sub + u * LG;
          ys[u] = (e < c) ? bq[e] : 0.0;
          a = fma(xs[u], xs[u], a);
          b = fma(ys[u], ys[u], b);
          g = fma(xs[u], ys[u], g);
        }
        if constexpr (LG == 16) {
          a = row16_sum(a);
          b = row16_sum(b);
          g = row16_sum(g);
        } else {
          for (int off = LG / 2; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, LG);
            b += __shfl_xor(b, off, LG);
            g += __shfl_xor(g, off, LG);
          }
        }
        my_cmax = max(my_cmax, cos2_bits(a, b, g));
        double cs, sn;
        if (jacobi_rotation(a, b, g, tol, cs, sn)) {
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int e = sub + u * LG;
            const double x = xs[u];
            xs[u] = cs * x - sn * ys[u];
            if (e < c) bq[e] = sn * x + cs * ys[u];
          }
          double* jq = Jl + (long)q * rows;
#pragma unroll
          for (int u = 0; u < NJ; ++u) {
            const int e = sub + u * LG;
            if (e < rows) {
              const double x = jx[u], y = jq[e];
              jx[u] = cs * x - sn * y;
              jq[e] = sn * x + cs * y;
            }
          }
          ++my_rot;
        }
      }
      __syncthreads();
    }
    if (own) {
      double* bp = Bw + (long)grp * c;
      double* jp = Jl + (long)grp * rows;
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int e = sub + u * LG;
        if (e < c) bp[e] = xs[u];
      }
#pragma unroll
      for (int u = 0; u < NJ; ++u) {
        const int e = sub + u * LG;
        if (e < rows) jp[e] = jx[u];
      }
    }
    __syncthreads();
  } else
  for (int rr = 0; rr < nrounds; ++rr) {
    for (int pi = grp; pi < npairs; pi += ngrp) {
      int p, q;
      if (cross) {
        // row pi of block P with row (pi + rr) mod MQ of block Q
        p = pi;
        q = (pi + rr) % MQ;
        if (q >= qn) continue;
        q += pn;
      } else {
        const int t1 = pi, t2 = RP - 1 - pi;
        p = (t1 == 0) ? 0 : ((t1 - 1 + rr) % (RP - 1)) + 1;
        q = (t2 == 0) ? 0 : ((t2 - 1 + rr) % (RP - 1)) + 1;
        if (p >= rows || q >= rows) continue;
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
      }
      double* bp = Bw + (long)p * c;
      double* bq = Bw + (long)q * c;
      double xs[NR], ys[NR];
      double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int e = sub + u * LG;
        xs[u] = (e < c) ? bp[e] : 0.0;
        ys[u] = (e < c) ? bq[e] : 0.0;
        a = fma(xs[u], xs[u], a);
        b = fma(ys[u], ys[u], b);
        g = fma(xs[u], ys[u], g);
      }
      if constexpr (LG == 16) {
        a = row16_sum(a);
        b = row16_sum(b);
        g = row16_sum(g);
      } else {
        for (int off = LG / 2; off > 0; off >>= 1) {
          a += __shfl_xor(a, off, LG);
          b += __shfl_xor(b, off, LG);
          g += __shfl_xor(g, off, LG);
        }
      }
      my_cmax = max(my_cmax, cos2_bits(a, b, g));
      double cs, sn;
      if (!jacobi_rotation(a, b, g, tol, cs, sn)) continue;
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int e = sub + u * LG;
        if (e < c) {
          bp[e] = cs * xs[u] - sn * ys[u];
          bq[e] = sn * xs[u] + cs * ys[u];
        }
      }
      double* jp = Jl + (long)p * rows;
      double* jq = Jl + (long)q * rows;
      for (int e = sub; e < rows; e += LG) {
        const double x = jp[e], y = jq[e];
        jp[e] = cs * x - sn * y;
        jq[e] = sn * x + cs * y;
      }
      ++my_rot;
    }
    __syncthreads();
  }
  if (sub == 0) {
    if (my_rot > 0) atomicAdd(&s_rot, my_rot);
    if (my_cmax > 0) atomicMax(&s_cmax, my_cmax);
  }
  for (long e = threadIdx.x; e < (long)rows * c; e += blockDim.x) {
    const int r = (int)(e / c), col = (int)(e % c);
    B[(long)grow(r) * c + col] = Bw[e];
  }
  __syncthreads();
  // JT rows of the pair <- Jl x (old rows), the old rows staged where Bw was
  for (long e = threadIdx.x; e < (long)rows * k; e += blockDim.x) {
    const int r = (int)(e / k), col = (int)(e % k);
    Bw[e] = JT[(long)grow(r) * k + col];
  }
  __syncthreads();
  // thread: one column, rows r = rs, rs + nrs, ...
  const int nrs = max(1, (int)(blockDim.x / k));
  const int col = threadIdx.x % k, rs = threadIdx.x / k;
  if (rs < nrs && threadIdx.x < nrs * k) {
    for (int r = rs; r < rows; r += nrs) {
      double acc = 0.0;
      for (int s2i = 0; s2i < rows; ++s2i) acc = fma(Jl[r * rows + s2i], Bw[(long)s2i * k + col], acc);
      JT[(long)grow(r) * k + col] = acc;
    }
  }
  if (threadIdx.x == 0) {
    if (s_rot > 0) atomicAdd(counter, s_rot);
    atomicMax(counter + 1, s_cmax);
  }
}

__global__ void __launch_bounds__(kNT) jacobi_finish_kernel(int k, int c, const double* __restrict__ B,
                                                            const double* __restrict__ JT, double* __restrict__ U,
                                                            double* __restrict__ Wt, double* __restrict__ sigma,
                                                            int* __restrict__ info, int sweep) {
  jacobi_finish(k, c, B, JT, U, Wt, sigma, info, sweep);
}

__global__ void set_ints_kernel(int* p, int v, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = v;
}

// ------------------------------------------------- Hessenberg reduction
// A (n x n, real, row-major) -> H = Q^T A Q upper Hessenberg, by Householder
// reflectors on columns 0..n-3.  QT receives Q^T.
// Column sums w[j] = beta sum_{i >= r0} v[i] X[i][j] for j in [c0, n): 16
// row groups of 64 lanes each sum a strided share of the rows of 64
// consecutive columns (coalesced), partial sums meet in LDS.
template <class R>
__device__ void hess_colsum(int n, int r0, int c0, const R* __restrict__ X, const R* v, R beta, R* w, R* part) {
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6, ngrp = blockDim.x >> 6;
  for (int cb = c0; cb < n; cb += 64) {
    const int j = cb + lane;
    R acc = R(0.0);
    if (j < n)
      for (int i = r0 + grp; i < n; i += ngrp) acc = fma(v[i], X[(long)i * n + j], acc);
    part[grp * 64 + lane] = acc;
    __syncthreads();
    if (grp == 0 && j < n) {
      R t = R(0.0);
      for (int g = 0; g < ngrp; ++g) t += part[g * 64 + lane];
      w[j] = beta * t;
    }
    __syncthreads();
  }
}

// A (n x n, real, row-major) -> H = Q^T A Q upper Hessenberg, by Householder
// reflectors on columns 0..n-3.  QT receives Q^T.
template <bool LDS, class R>
__global__ void __launch_bounds__(kNT) hessenberg_kernel(int n, R* __restrict__ A, R* __restrict__ QT,
                                                         R* __restrict__ work) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  R* lds = reinterpret_cast<R*>(lds_raw);
  __shared__ R red[kNT / 64];
  __shared__ R part[kNT];
  __shared__ R s_alpha, s_vnorm2;
  const long nn = (long)n * n;
  constexpr bool in_lds = LDS;
  R* H;
  R* v;  // reflector (n)
  R* w;  // products (n)
  if constexpr (LDS) {
    H = lds;
    v = lds + nn;
    w = lds + nn + n;
  } else {
    H = A;
    v = work;
    w = work + n;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  if (in_lds)
    for (long e = threadIdx.x; e < nn; e += blockDim.x) H[e] = A[e];
  for (long e = threadIdx.x; e < nn; e += blockDim.x) QT[e] = ((e / n) == (e % n)) ? R(1.0) : R(0.0);
  __syncthreads();
  for (int k = 0; k < n - 2; ++k) {
    // x = H[k+1:, k]
    R s = R(0.0);
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) {
      const R x = H[(long)i * n + k];
      v[i] = x;
      s = fma(x, x, s);
    }
    s = wave_sum64(s);
    __syncthreads();
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      R tot = R(0.0);
      for (int i = 0; i < nwave; ++i) tot += red[i];
      const R x0 = v[k + 1];
      const R tail = tot - x0 * x0;
      if (tail <= TinyOf<R>::value * fmax(R(1.0), tot)) {
        s_vnorm2 = R(0.0);  // already in Hessenberg form for this column
      } else {
        const R alpha = (x0 >= R(0.0)) ? -sqrt(tot) : sqrt(tot);
        s_alpha = alpha;
        v[k + 1] = x0 - alpha;
        s_vnorm2 = tail + (x0 - alpha) * (x0 - alpha);
      }
    }
    __syncthreads();
    const R vn2 = s_vnorm2;
    if (vn2 == R(0.0)) continue;
    const R beta = R(2.0) / vn2;
    // left: H[k+1:, :] -= v (beta v^T H[k+1:, :]) ; columns k..n-1 suffice
    hess_colsum<R>(n, k + 1, k, H, v, beta, w, part);
    {
      const int rows = n - k - 1, cols = n - k;
      const long tot = (long)rows * cols;
      for (long e = threadIdx.x; e < tot; e += blockDim.x) {
        const int i = k + 1 + (int)(e / cols), j = k + (int)(e % cols);
        H[(long)i * n + j] -= v[i] * w[j];
      }
    }
    __syncthreads();
    // right: H[:, k+1:] -= (beta H[:, k+1:] v) v^T ; one wavefront per row
    for (int i = wave; i < n; i += nwave) {
      R d = R(0.0);
      for (int j = k + 1 + lane; j < n; j += 64) d = fma(H[(long)i * n + j], v[j], d);
      d = wave_sum64(d);
      if (lane == 0) w[i] = beta * d;
    }
    __syncthreads();
    {
      const int cols = n - k - 1;
      const long tot = (long)n * cols;
      for (long e = threadIdx.x; e < tot; e += blockDim.x) {
        const int i = (int)(e / cols), j = k + 1 + (int)(e % cols);
        H[(long)i * n + j] -= w[i] * v[j];
      }
    }
    __syncthreads();
    // QT = P QT (P symmetric): QT[k+1:, :] -= v (beta v^T QT[k+1:, :])
    hess_colsum<R>(n, k + 1, 0, QT, v, beta, w, part);
    {
      const int rows = n - k - 1;
      const long tot = (long)rows * n;
      for (long e = threadIdx.x; e < tot; e += blockDim.x) {
        const int i = k + 1 + (int)(e / n), j = (int)(e % n);
        QT[(long)i * n + j] -= v[i] * w[j];
      }
    }
    __syncthreads();
    // exact zeros below the subdiagonal of column k
    for (int i = k + 2 + threadIdx.x; i < n; i += blockDim.x) H[(long)i * n + k] = R(0.0);
    __syncthreads();
  }
  if (in_lds)
    for (long e = threadIdx.x; e < nn; e += blockDim.x) A[e] = H[e];
}

// --------------------------------------- eigenvectors of triangular T
// T Y = Y diag(T): Y unit upper triangular, column k solves
// (T[:k,:k] - t_kk I) y = -T[:k, k].  Rows are produced bottom-up for all
// columns at once.  Denominators below smin = max(ulp |t_kk|, tiny) are
// replaced by smin (as in standard eigenvector codes).
template <class R>
__global__ void __launch_bounds__(kNT) trevec_kernel(int n, const typename CxOf<R>::type* __restrict__ T,
                                                     typename CxOf<R>::type* __restrict__ Y) {
  using CX = CxOf<R>;
  using C = typename CxOf<R>::type;
  const long nn = (long)n * n;
  const int grp = threadIdx.x / kTriG, sub = threadIdx.x % kTriG, ngrp = blockDim.x / kTriG;
  for (long e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    Y[e] = (i == j) ? CX::make(R(1.0), R(0.0)) : CX::make(R(0.0), R(0.0));
  }
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    const C tii = T[(long)i * n + i];
    for (int k0 = i + 1; k0 < n; k0 += ngrp) {
      const int k = k0 + grp;
      C s = CX::make(R(0.0), R(0.0));
      if (k < n)
        for (int t = i + 1 + sub; t < k; t += kTriG) s = TriOps<C>::fma(T[(long)i * n + t], Y[(long)t * n + k], s);
      for (int off = kTriG / 2; off > 0; off >>= 1) s = tadd<C>(s, shfl_xor_t<C>(s, off, kTriG));
      if (k < n && sub == 0) {
        s = cadd(s, T[(long)i * n + k]);  // times y_k = 1
        Y[(long)i * n + k] = trevec_entry(s, tii, T[(long)k * n + k]);
      }
    }
    __syncthreads();
  }
}


// Householder reduction to Hessenberg form for matrices that exceed LDS.  H
// stays in global memory (L2-resident).  Per step, one read pass over the
// active block (all rows, columns k..n-1) gives both w = H^T v and t = H v,
// and one read-modify-write pass applies
//   P H P = H - beta v w^T - beta t v^T + beta^2 (v^T t) v v^T.
// Column k is written exactly (alpha on the subdiagonal, zeros below).  The
// reflectors go to V (column k, zero above row k+1) and beta[k] (0: none);
// Q is formed from them afterwards.  Wavefronts stride over rows, lanes over
// columns (coalesced rows of the row-major H).
// kHgCols column slots per lane (n <= 64 kHgCols), kHgRows rows in flight
// per wavefront
template <int kHgCols, int kHgRows>
__global__ void __launch_bounds__(kNT) hess_global_kernel(int n, double* __restrict__ H, double* __restrict__ V,
                                                          double* __restrict__ beta_out) {
  extern __shared__ double sm[];
  double* v = sm;             // n
  double* t = v + n;          // n
  double* w = t + n;          // n
  double* wpart = w + n;      // (kNT / 64) * n
  __shared__ double red[kNT / 64];
  __shared__ double s_beta, s_alpha, s_c;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
  for (int k = 0; k < n - 2; ++k) {
    // ---- reflector from H[k+1:, k]
    double ss = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double x = (i >= k + 1) ? H[(long)i * n + k] : 0.0;
      v[i] = x;
      ss = fma(x, x, ss);
    }
    ss = wave_sum64(ss);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int i = 0; i < NW; ++i) tot += red[i];
      const double x0 = v[k + 1];
      const double tail = tot - x0 * x0;
      if (tail <= TinyOf<double>::value * fmax(1.0, tot)) {
        s_beta = 0.0;
      } else {
        const double alpha = (x0 >= 0.0) ? -sqrt(tot) : sqrt(tot);
        v[k + 1] = x0 - alpha;
        s_beta = 2.0 / (tail + (x0 - alpha) * (x0 - alpha));
        s_alpha = alpha;
      }
    }
    __syncthreads();
    const double beta = s_beta;
    for (int i = threadIdx.x; i < n; i += blockDim.x) V[(long)i * n + k] = (beta != 0.0) ? v[i] : 0.0;
    if (threadIdx.x == 0) beta_out[k] = beta;
    if (beta == 0.0) continue;  // column already reduced
    // ---- read pass: w_j = sum_i v_i H_ij (j >= k), t_i = sum_j H_ij v_j
    double vj[kHgCols], wp[kHgCols];
#pragma unroll
    for (int q = 0; q < kHgCols; ++q) {
      const int j = k + lane + 64 * q;
      vj[q] = (j < n) ? v[j] : 0.0;
      wp[q] = 0.0;
    }
    // kHgRows rows per iteration: their loads are issued together
    for (int i0 = wave; i0 < n; i0 += kHgRows * NW) {
      double hv[kHgRows][kHgCols];
#pragma unroll
      for (int r = 0; r < kHgRows; ++r) {
        const int i = i0 + r * NW;
#pragma unroll
        for (int q = 0; q < kHgCols; ++q) {
          const int j = k + lane + 64 * q;
          hv[r][q] = (i < n && j < n) ? H[(long)i * n + j] : 0.0;
        }
      }
      double tp[kHgRows];
#pragma unroll
      for (int r = 0; r < kHgRows; ++r) {
        const int i = i0 + r * NW;
        const double vi = (i < n) ? v[i] : 0.0;
        tp[r] = 0.0;
#pragma unroll
        for (int q = 0; q < kHgCols; ++q) {
          wp[q] = fma(vi, hv[r][q], wp[q]);
          tp[r] = fma(hv[r][q], vj[q], tp[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < kHgRows; ++r) tp[r] = wave_sum64(tp[r]);
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < kHgRows; ++r)
          if (i0 + r * NW < n) t[i0 + r * NW] = tp[r];
      }
    }
#pragma unroll
    for (int q = 0; q < kHgCols; ++q) {
      const int j = k + lane + 64 * q;
      if (j < n) wpart[(long)wave * n + j] = wp[q];
    }
    __syncthreads();
    for (int j = k + threadIdx.x; j < n; j += blockDim.x) {
      double a = 0.0;
      for (int g = 0; g < NW; ++g) a += wpart[(long)g * n + j];
      w[j] = a;
    }
    // c = v^T t
    double cc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) cc = fma(v[i], t[i], cc);
    cc = wave_sum64(cc);
    if (lane == 0) red[wave] = cc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int i = 0; i < NW; ++i) tot += red[i];
      s_c = tot;
    }
    __syncthreads();
    const double b2c = beta * beta * s_c;
    const double alpha = s_alpha;
    // ---- update pass
    double wj[kHgCols];
#pragma unroll
    for (int q = 0; q < kHgCols; ++q) {
      const int j = k + lane + 64 * q;
      wj[q] = (j < n) ? w[j] : 0.0;
    }
    for (int i0 = wave; i0 < n; i0 += kHgRows * NW) {
      double hv[kHgRows][kHgCols];
#pragma unroll
      for (int r = 0; r < kHgRows; ++r) {
        const int i = i0 + r * NW;
#pragma unroll
        for (int q = 0; q < kHgCols; ++q) {
          const int j = k + lane + 64 * q;
          hv[r][q] = (i < n && j < n) ? H[(long)i * n + j] : 0.0;
        }
      }
#pragma unroll
      for (int r = 0; r < kHgRows; ++r) {
        const int i = i0 + r * NW;
        if (i >= n) continue;
        const double vi = v[i], ti = t[i];
#pragma unroll
        for (int q = 0; q < kHgCols; ++q) {
          const int j = k + lane + 64 * q;
          if (j < n) {
            double h;
            if (j == k)
              h = (i == k + 1) ? alpha : (i > k + 1 ? 0.0 : hv[r][q] - beta * ti * vj[q]);
            else
              h = hv[r][q] - beta * (vi * wj[q] + ti * vj[q]) + b2c * vi * vj[q];
            H[(long)i * n + j] = h;
          }
        }
      }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    for (int k = (n >= 2 ? n - 2 : 0); k < n; ++k) V[(long)i * n + k] = 0.0;
  if (threadIdx.x == 0)
    for (int k = (n >= 2 ? n - 2 : 0); k < n; ++k) beta_out[k] = 0.0;
}

// Tinv = strict upper part of S (= V^T V) with diagonal 1/beta (1 where no
// reflector): the inverse of the compact-WY factor T of P_0 ... P_{n-3}
__global__ void hess_tinv_kernel(int n, const double* __restrict__ S, const double* __restrict__ beta,
                                 double* __restrict__ Tinv) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  double x = 0.0;
  if (j > i) x = S[e];
  else if (j == i) x = (beta[i] != 0.0) ? 1.0 / beta[i] : 1.0;
  Tinv[e] = x;
}

__global__ void identity_kernel(int n, double* __restrict__ X) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  X[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
}

}  // namespace

// ============================================================ launchers
static size_t lds_bytes(long doubles) { return (size_t)std::min<long>(doubles, kLdsDoubles) * sizeof(double); }

void chol_skip(hipStream_t s, int n, const double* G, double* R, int* mask, int* count, double tau) {
  T2S2_CHECK(n >= 1 && n <= 4096, "chol_skip: bad size");
  const long need = (long)n * n;
  TimedScope ts(s, KC_CHOL, 16.0 * need, (double)n * n * n / 3.0);
  if (n <= 32)
    hipLaunchKernelGGL(chol_skip_reg_kernel<32>, dim3(1), dim3(64), 0, s, n, G, R, mask, count, tau);
  else if (n <= kCholBlkMax && need + kCholP * kCholP <= kLdsDoubles)
    hipLaunchKernelGGL(chol_blk_kernel<true>, dim3(1), dim3(kCholNT), need * sizeof(double), s, n, G, R, mask, count,
                       tau);
  else if (n <= kCholBlkMax)
    hipLaunchKernelGGL(chol_blk_kernel<false>, dim3(1), dim3(kCholNT), (size_t)kCholP * n * sizeof(double), s, n, G, R,
                       mask, count, tau);
  else if (need <= kLdsDoubles)
    hipLaunchKernelGGL(chol_skip_kernel<true>, dim3(1), dim3(kNT), lds_bytes(need), s, n, G, R, mask, count, tau);
  else
    hipLaunchKernelGGL(chol_skip_kernel<false>, dim3(1), dim3(kNT), 0, s, n, G, R, mask, count, tau);
  T2S2_LAUNCH_CHECK();
}

template <class T>
static void trtri_launch(hipStream_t s, int n, const T* R, T* Rinv) {
  if (n <= kTriColMax)
    hipLaunchKernelGGL((trtri_col_kernel<T, false>), dim3((n + kTriG - 1) / kTriG), dim3(64), 0, s, n, R, Rinv);
  else
    hipLaunchKernelGGL(trtri_upper_kernel<T>, dim3(1), dim3(kNT), 0, s, n, R, Rinv);
}

void trtri_upper(hipStream_t s, int n, const double* R, double* Rinv) {
  TimedScope ts(s, KC_TRTRI, 8.0 * n * n, (double)n * n * n / 3.0);
  if (n <= 32)
    hipLaunchKernelGGL(trtri_reg_kernel<32>, dim3(1), dim3(64), 0, s, n, R, Rinv);
  else
    trtri_launch(s, n, R, Rinv);
  T2S2_LAUNCH_CHECK();
}

void trtri_upper(hipStream_t s, int n, const double2* R, double2* Rinv) {
  TimedScope ts(s, KC_TRTRI, 16.0 * n * n, 4.0 * n * n * n / 3.0);
  trtri_launch(s, n, R, Rinv);
  T2S2_LAUNCH_CHECK();
}

void trtri_upper(hipStream_t s, int n, const float2* R, float2* Rinv) {
  TimedScope ts(s, KC_TRTRI, 8.0 * n * n, 4.0 * n * n * n / 3.0);
  trtri_launch(s, n, R, Rinv);
  T2S2_LAUNCH_CHECK();
}

void jacobi_rows(hipStream_t s, int k, int c, double* B, double* JT, double* U, double* Wt, double* sigma,
                 int* info, int max_sweeps) {
  T2S2_CHECK(k >= 1 && c >= 1, "jacobi_rows: bad size");
  const long bsz = (long)k * c, jsz = (long)k * k;
  long need = 0;
  if (bsz <= kLdsDoubles) need = (bsz + jsz <= kLdsDoubles) ? bsz + jsz : bsz;
  // beyond LDS: block Jacobi, one workgroup per pair of row blocks
  // block size: 2 blk rows of B and the 2blk x 2blk rotation block in LDS,
  // at least 8 blocks (4 workgroups per round)
  int blk = 1;
  while (2L * (blk + 1) * c + 4L * (blk + 1) * (blk + 1) <= kLdsDoubles) ++blk;
  blk = std::min(blk, std::max(2, (k + 7) / 8));
  if (need < bsz + jsz && k <= c && c <= kJacBR * kJacBG && blk >= 2 && (k + blk - 1) / blk >= 3) {
    TimedScope ts(s, KC_JACOBI, 8.0 * (2.0 * bsz + 2.0 * jsz), 0.0);
    const int nblk = (k + blk - 1) / blk, nplay = nblk + (nblk & 1);
    const size_t lds = (size_t)(2L * blk * c + 4L * blk * blk) * sizeof(double);
    identity(s, k, JT);
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
      hipLaunchKernelGGL(set_ints_kernel, dim3(1), dim3(64), 0, s, info, 0, 2);
      hipLaunchKernelGGL((jacobi_block_kernel<kJacBR, kJacBG>), dim3(nblk), dim3(kNT), lds, s, k, c, B, JT, blk,
                         nblk, nplay, 0, 0, info);
      for (int round = 0; round < nplay - 1; ++round)
        hipLaunchKernelGGL((jacobi_block_kernel<kJacBR, kJacBG>), dim3(nplay / 2), dim3(kNT), lds, s, k, c, B, JT,
                           blk, nblk, nplay, round, 1, info);
      T2S2_LAUNCH_CHECK();
      int st[2] = {0, 0};  // rotations, largest squared cosine (float bits)
      host_read(s, st, info, 2 * sizeof(int));
      float cmax;
      std::memcpy(&cmax, &st[1], sizeof(float));
      if (st[0] == 0 || cmax <= kJacStop2) break;
    }
    hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(kNT), 0, s, k, c, B, JT, U, Wt, sigma, info, sweep);
    T2S2_LAUNCH_CHECK();
    return;
  }
  TimedScope ts(s, KC_JACOBI, 8.0 * (2.0 * bsz + 2.0 * jsz), 0.0);
  if (need == bsz + jsz && need > 0)
    hipLaunchKernelGGL(jacobi_rows_kernel<2>, dim3(1), dim3(kNT), lds_bytes(need), s, k, c, B, JT, U, Wt, sigma,
                       info, max_sweeps);
  else if (need == bsz && need > 0)
    hipLaunchKernelGGL(jacobi_rows_kernel<1>, dim3(1), dim3(kNT), lds_bytes(need), s, k, c, B, JT, U, Wt, sigma,
                       info, max_sweeps);
  else
    hipLaunchKernelGGL(jacobi_rows_kernel<0>, dim3(1), dim3(kNT), 0, s, k, c, B, JT, U, Wt, sigma, info,
                       max_sweeps);
  T2S2_LAUNCH_CHECK();
}

template <class R>
static void hessenberg_t(hipStream_t s, int n, R* A, R* QT, R* work) {
  const long need = ((long)n * n + 2L * n) * (long)sizeof(R);
  // static LDS of the kernel: partial sums (kNT) and the reduction slots
  const long static_bytes = (long)sizeof(R) * (kNT + kNT / 64 + 2);
  TimedScope ts(s, KC_HESS, sizeof(R) * 3.0 * n * n, 14.0 * n * n * n / 3.0);
  if (need <= kLdsBytes - static_bytes)
    hipLaunchKernelGGL((hessenberg_kernel<true, R>), dim3(1), dim3(kNT), (size_t)need, s, n, A, QT, work);
  else
    hipLaunchKernelGGL((hessenberg_kernel<false, R>), dim3(1), dim3(kNT), 0, s, n, A, QT, work);
  T2S2_LAUNCH_CHECK();
}
void hessenberg(hipStream_t s, int n, double* A, double* QT, double* work) { hessenberg_t<double>(s, n, A, QT, work); }
void hessenberg(hipStream_t s, int n, float* A, float* QT, float* work) { hessenberg_t<float>(s, n, A, QT, work); }

template <class R>
static void trevec_t(hipStream_t s, int n, const typename CxOf<R>::type* T, typename CxOf<R>::type* Y) {
  TimedScope ts(s, KC_TREVEC, 2.0 * sizeof(R) * 2.0 * n * n, 8.0 * n * n * n / 6.0);
  using C = typename CxOf<R>::type;
  if (n <= kTriColMax)
    hipLaunchKernelGGL((trtri_col_kernel<C, true>), dim3((n + kTriG - 1) / kTriG), dim3(64), 0, s, n, T, Y);
  else
    hipLaunchKernelGGL(trevec_kernel<R>, dim3(1), dim3(kNT), 0, s, n, T, Y);
  T2S2_LAUNCH_CHECK();
}
void trevec(hipStream_t s, int n, const double2* T, double2* Y) { trevec_t<double>(s, n, T, Y); }
void trevec(hipStream_t s, int n, const float2* T, float2* Y) { trevec_t<float>(s, n, T, Y); }


bool hessenberg_fits_lds(int n, int rbytes) {
  const long need = ((long)n * n + 2L * n) * rbytes;
  const long static_bytes = (long)rbytes * (kNT + kNT / 64 + 2);
  return need <= kLdsBytes - static_bytes;
}

void hessenberg_global(hipStream_t s, int n, double* A, double* V, double* beta) {
  T2S2_CHECK(n >= 1 && n <= 512, "hessenberg_global: n must be in [1, 512]");
  const size_t lds = (size_t)(3L * n + (long)(kNT / 64) * n) * sizeof(double);
  TimedScope ts(s, KC_HESS, sizeof(double) * 3.0 * n * n * n / 2.0, 10.0 * n * n * n / 3.0);
  if (n <= 256)
    hipLaunchKernelGGL((hess_global_kernel<4, 4>), dim3(1), dim3(kNT), lds, s, n, A, V, beta);
  else
    hipLaunchKernelGGL((hess_global_kernel<8, 2>), dim3(1), dim3(kNT), lds, s, n, A, V, beta);
  T2S2_LAUNCH_CHECK();
}

void hess_tinv(hipStream_t s, int n, const double* S, const double* beta, double* Tinv) {
  const long nn = (long)n * n;
  TimedScope ts(s, KC_HESS, sizeof(double) * 2.0 * nn, 0.0);
  hipLaunchKernelGGL(hess_tinv_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, n, S, beta, Tinv);
  T2S2_LAUNCH_CHECK();
}

void identity(hipStream_t s, int n, double* X) {
  const long nn = (long)n * n;
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, n, X);
  T2S2_LAUNCH_CHECK();
}

}  // namespace t2s2
