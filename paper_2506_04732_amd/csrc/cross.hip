// TT-cross approximation of function-generated tensors (Methods: the closing
// paragraph on cross approximation with MaxVol; Oseledets & Tyrtyshnikov,
// Goreinov et al., cited there).  Alternating cross with nested index sets:
// at core l the fiber tensor C(a, i, b) = f(I_{l-1}[a], i, J_l[b]) is
// evaluated on the device, orthonormalised (QR), and MaxVol picks the rows
// whose interpolation Q Q[rows]^{-1} is the new core; the chosen rows extend
// the left index set (left-to-right) or, mirrored, the right one.
#include "cross.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace t2s2 {

namespace {

constexpr int kMvThreads = 512;
constexpr int kMvMaxK = 128;  // LU of the k x k submatrix in LDS

struct FnArgs {
  int kind, d;
  const double* par;   // amp, delta|phase, w[d], c[d]
};

__device__ inline double eval_fn(const FnArgs& a, const double* x) {
  const double amp = a.par[0], aux = a.par[1];
  const double* w = a.par + 2;
  const double* cc = a.par + 2 + a.d;
  if (a.kind == 2) {
    double s = aux;
    for (int k = 0; k < a.d; ++k) s = fma(w[k], x[k], s);
    return amp * sin(s);
  }
  double q = 0.0;
  for (int k = 0; k < a.d; ++k) {
    const double t = x[k] - cc[k];
    q = fma(w[k] * t, t, q);
  }
  if (a.kind == 0) return amp / (1.0 + q);
  return amp * exp(-sqrt(aux + q));
}

constexpr int kMaxD = 16;

// out[(a n + i) rb + b] = f(theta[left[a]], theta_l[i], theta[right[b]])
__global__ void fiber_kernel(FnArgs fa, const double* __restrict__ theta, const int* __restrict__ toff, int l,
                             int n, int ra, int rb, const int* __restrict__ left, const int* __restrict__ right,
                             double* __restrict__ out) {
  const long tot = (long)ra * n * rb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int b = (int)(e % rb);
    const long t = e / rb;
    const int i = (int)(t % n);
    const int a = (int)(t / n);
    double x[kMaxD];
    for (int k = 0; k < l; ++k) x[k] = theta[toff[k] + left[(long)a * l + k]];
    x[l] = theta[toff[l] + i];
    const int nr = fa.d - l - 1;
    for (int k = 0; k < nr; ++k) x[l + 1 + k] = theta[toff[l + 1 + k] + right[(long)b * nr + k]];
    out[e] = eval_fn(fa, x);
  }
}

// f at S sample multi-indices idx (S x d)
__global__ void sample_fn_kernel(FnArgs fa, const double* __restrict__ theta, const int* __restrict__ toff,
                                 int S, const int* __restrict__ idx, double* __restrict__ out) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
    double x[kMaxD];
    for (int k = 0; k < fa.d; ++k) x[k] = theta[toff[k] + idx[(long)s * fa.d + k]];
    out[s] = eval_fn(fa, x);
  }
}

// Vout[s][b] = sum_a Vin[s][a] X[a][idx[s][l]][b] (one TT core applied to S row vectors)
__global__ void sample_tt_kernel(int S, int d, int l, int r0, int n, int r1, const int* __restrict__ idx,
                                 const double* __restrict__ X, const double* __restrict__ Vin,
                                 double* __restrict__ Vout) {
  const long tot = (long)S * r1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int s = (int)(e / r1), b = (int)(e % r1);
    const int i = idx[(long)s * d + l];
    double acc = 0.0;
    for (int a = 0; a < r0; ++a) acc = fma(Vin[(long)s * r0 + a], X[((long)a * n + i) * r1 + b], acc);
    Vout[e] = acc;
  }
}

__device__ inline void block_argmax(double v, int idx, double* sv, int* si) {
  // v >= 0; ties resolved to the smaller index
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = idx;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      const double o = sv[t + h];
      const int oi = si[t + h];
      if (o > sv[t] || (o == sv[t] && oi < si[t])) {
        sv[t] = o;
        si[t] = oi;
      }
    }
    __syncthreads();
  }
}

// MaxVol on A (M x k, row-major, M >= k, full column rank), one workgroup.
// W: M x k work (pivoted elimination), B: M x k output = A A[rows]^{-1}.
// rows: k ints.  info[0] = swaps made (negative: iteration cap reached).
__global__ void __launch_bounds__(kMvThreads) maxvol_kernel(int M, int k, const double* __restrict__ A,
                                                            double* __restrict__ W, double* __restrict__ B,
                                                            int* __restrict__ mark, int* __restrict__ rows,
                                                            int* __restrict__ info, double tol, int max_iters) {
  __shared__ double sv[kMvThreads];
  __shared__ int si[kMvThreads];
  __shared__ int piv[kMvMaxK];
  __shared__ int s_row[kMvMaxK];
  extern __shared__ double LU[];  // k x k
  const int t = threadIdx.x, nt = blockDim.x;
  const long tot = (long)M * k;
  for (long e = t; e < tot; e += nt) W[e] = A[e];
  for (int i = t; i < M; i += nt) mark[i] = 0;
  __syncthreads();
  // 1. start: Gaussian elimination with partial pivoting picks k rows
  for (int j = 0; j < k; ++j) {
    double best = -1.0;
    int bi = M;
    for (int i = t; i < M; i += nt) {
      if (mark[i]) continue;
      const double v = fabs(W[(long)i * k + j]);
      if (v > best || (v == best && i < bi)) {
        best = v;
        bi = i;
      }
    }
    block_argmax(best < 0 ? -1.0 : best, bi, sv, si);
    if (t == 0) {
      s_row[j] = si[0];
      mark[si[0]] = 1;
    }
    __syncthreads();
    const int p = s_row[j];
    const double pv = W[(long)p * k + j];
    for (long e = t; e < tot; e += nt) {
      const int i = (int)(e / k), c = (int)(e % k);
      if (c <= j || mark[i] || pv == 0.0) continue;
      W[e] -= W[(long)i * k + j] / pv * W[(long)p * k + c];
    }
    __syncthreads();
  }
  // 2. B = A A[rows]^{-1}:  A[rows]^T B^T = A^T, LU of A[rows]^T with pivoting
  for (int e = t; e < k * k; e += nt) {
    const int r = e / k, cidx = e % k;
    LU[r * k + cidx] = A[(long)s_row[cidx] * k + r];  // (A[rows]^T)[r][c] = A[rows[c]][r]
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      int p = j;
      for (int r = j + 1; r < k; ++r)
        if (fabs(LU[r * k + j]) > fabs(LU[p * k + j])) p = r;
      piv[j] = p;
      if (p != j)
        for (int cidx = 0; cidx < k; ++cidx) {
          const double tmp = LU[j * k + cidx];
          LU[j * k + cidx] = LU[p * k + cidx];
          LU[p * k + cidx] = tmp;
        }
    }
    __syncthreads();
    const double d = LU[j * k + j];
    for (int e = t; e < (k - j - 1) * (k - j); e += nt) {
      const int r = j + 1 + e / (k - j), cidx = j + e % (k - j);
      if (cidx == j) continue;
      LU[r * k + cidx] -= LU[r * k + j] / d * LU[j * k + cidx];
    }
    __syncthreads();
    for (int r = j + 1 + t; r < k; r += nt) LU[r * k + j] /= d;
    __syncthreads();
  }
  // each thread solves for rows of B: (L U) y = P a, a = row i of A (a column of A^T)
  for (int i = t; i < M; i += nt) {
    double y[kMvMaxK];
    for (int r = 0; r < k; ++r) y[r] = A[(long)i * k + r];
    for (int j = 0; j < k; ++j) {
      const int p = piv[j];
      if (p != j) {
        const double tmp = y[j];
        y[j] = y[p];
        y[p] = tmp;
      }
    }
    for (int r = 0; r < k; ++r)
      for (int q = 0; q < r; ++q) y[r] -= LU[r * k + q] * y[q];
    for (int r = k - 1; r >= 0; --r) {
      for (int q = r + 1; q < k; ++q) y[r] -= LU[r * k + q] * y[q];
      y[r] /= LU[r * k + r];
    }
    for (int r = 0; r < k; ++r) B[(long)i * k + r] = y[r];
  }
  __syncthreads();
  // 3. swaps while some |B_ij| > 1 + tol
  int it = 0;
  for (; it < max_iters; ++it) {
    double best = -1.0;
    int be = -1;
    for (long e = t; e < tot; e += nt) {
      const double v = fabs(B[e]);
      if (v > best) {
        best = v;
        be = (int)e;
      }
    }
    block_argmax(best, be < 0 ? (int)tot : be, sv, si);
    const double bmax = sv[0];
    const int eij = si[0];
    __syncthreads();
    if (bmax <= 1.0 + tol) break;
    const int i = eij / k, j = eij % k;
    const double bij = B[(long)i * k + j];
    // B <- B - B[:, j] (B[i, :] - e_j) / B[i, j]; row i first read into LDS
    for (int cidx = t; cidx < k; cidx += nt) sv[cidx] = (B[(long)i * k + cidx] - (cidx == j ? 1.0 : 0.0)) / bij;
    __syncthreads();
    for (long e = t; e < tot; e += nt) {
      const int r = (int)(e / k), cidx = (int)(e % k);
      if (cidx == j) continue;
      B[e] -= B[(long)r * k + j] * sv[cidx];
    }
    __syncthreads();
    for (int r = t; r < M; r += nt) B[(long)r * k + j] -= B[(long)r * k + j] * sv[j];
    if (t == 0) s_row[j] = i;
    __syncthreads();
  }
  for (int j = t; j < k; j += nt) rows[j] = s_row[j];
  if (t == 0) info[0] = it < max_iters ? it : -it;
}

unsigned long long splitmix(unsigned long long& s) {
  unsigned long long z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

int grid_for(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)); }

}  // namespace

CrossInfo source_cross(Problem& p, const Ctx& c, const CrossFunction& fn, double tol, int r0, int rmax,
                       unsigned long long seed, int samples, DTT& out) {
  const int d = p.d;
  T2S2_CHECK(d >= 1 && d <= kMaxD, "source_cross: d must be in [1, 16]");
  T2S2_CHECK(fn.kind >= 0 && fn.kind <= 2, "source_cross: kind must be 0, 1 or 2");
  T2S2_CHECK((int)fn.params.size() == 2 + 2 * d, "source_cross: 2 + 2 d parameters required");
  for (double v : fn.params) T2S2_CHECK(std::isfinite(v), "source_cross: parameters must be finite");
  T2S2_CHECK(fn.kind != 1 || fn.params[1] >= 0.0, "source_cross: delta must be >= 0");
  T2S2_CHECK(std::isfinite(tol) && tol > 0.0, "source_cross: tol must be > 0");
  T2S2_CHECK(r0 >= 1 && rmax >= r0 && rmax <= kMvMaxK, "source_cross: need 1 <= r0 <= rmax <= 128");
  T2S2_CHECK(samples >= 1, "source_cross: samples must be >= 1");
  const std::vector<int>& n = p.m;
  // device tables: nodes, offsets, parameters
  std::vector<int> toff(d + 1, 0);
  for (int l = 0; l < d; ++l) toff[l + 1] = toff[l] + n[l];
  std::vector<double> th;
  for (int l = 0; l < d; ++l) th.insert(th.end(), p.theta[l].begin(), p.theta[l].end());
  Scratch& S = *c.sc;
  double* dth = S.get<double>("cx.theta", th.size());
  int* dtoff = S.get<int>("cx.toff", d + 1);
  double* dpar = S.get<double>("cx.par", fn.params.size());
  c.h2d(dth, th.data(), th.size());
  c.h2d(dtoff, toff.data(), d + 1);
  c.h2d(dpar, fn.params.data(), fn.params.size());
  FnArgs fa{fn.kind, d, dpar};
  unsigned long long rs = seed * 0x2545F4914F6CDD1DULL + 0x1234567ULL;
  // samples and their f values
  std::vector<int> sidx((size_t)samples * d);
  for (auto& v : sidx) v = 0;
  for (int s = 0; s < samples; ++s)
    for (int l = 0; l < d; ++l) sidx[(size_t)s * d + l] = (int)(splitmix(rs) % (unsigned long long)n[l]);
  int* dsidx = S.get<int>("cx.sidx", sidx.size());
  double* dfs = S.get<double>("cx.fs", samples);
  c.h2d(dsidx, sidx.data(), sidx.size());
  hipLaunchKernelGGL(sample_fn_kernel, dim3(grid_for(samples)), dim3(256), 0, c.s, fa, dth, dtoff, samples, dsidx,
                     dfs);
  T2S2_LAUNCH_CHECK();
  std::vector<double> hfs(samples);
  c.d2h(hfs.data(), dfs, samples);
  double fnorm2 = 0.0;
  for (double v : hfs) fnorm2 += v * v;
  CrossInfo info;
  info.evaluations = samples;
  out.d = d;
  out.n = n;
  out.r.assign(d + 1, 1);
  // feasible ranks for r
  auto feasible = [&](int r) {
    std::vector<int> rr(d + 1, 1);
    for (int l = 1; l < d; ++l) {
      double a = 1, b = 1;
      for (int k = 0; k < l; ++k) a *= n[k];
      for (int k = l; k < d; ++k) b *= n[k];
      rr[l] = (int)std::min<double>({(double)r, a, b});
    }
    return rr;
  };
  std::vector<std::vector<int>> J(d + 1), I(d + 1);   // flattened index sets (rows x width)
  std::vector<int> jr(d + 1, 1), ir(d + 1, 1);        // their sizes
  int r = r0;
  for (;;) {
    const std::vector<int> rr = feasible(r);
    // right index sets J_l (dimensions l .. d-1) for l = d-1 .. 1, keeping earlier ones
    for (int l = d - 1; l >= 1; --l) {
      const int w = d - l;
      std::vector<int> cand = J[l];
      int have = (int)cand.size() / std::max(w, 1);
      if ((int)cand.size() != have * w) cand.clear(), have = 0;
      int guard = 0;
      while (have < rr[l] && guard < 100000) {
        ++guard;
        std::vector<int> v(w);
        for (int k = 0; k < w; ++k) v[k] = (int)(splitmix(rs) % (unsigned long long)n[l + k]);
        bool dup = false;
        for (int q = 0; q < have && !dup; ++q) dup = std::equal(v.begin(), v.end(), cand.begin() + (size_t)q * w);
        if (dup) continue;
        cand.insert(cand.end(), v.begin(), v.end());
        ++have;
      }
      J[l] = cand;
      jr[l] = have;
    }
    J[d].clear();
    jr[d] = 1;
    I[0].clear();
    ir[0] = 1;
    for (int half = 0; half < 4; ++half) {
      const bool l2r = half % 2 == 0;
      if (l2r) {
        for (int l = 0; l + 1 < d; ++l) {
          const int ra = ir[l], rb = jr[l + 1], nl = n[l];
          const long M = (long)ra * nl;
          int* dl = S.get<int>("cx.left", std::max<size_t>(1, I[l].size()));
          int* dr = S.get<int>("cx.right", std::max<size_t>(1, J[l + 1].size()));
          if (!I[l].empty()) c.h2d(dl, I[l].data(), I[l].size());
          if (!J[l + 1].empty()) c.h2d(dr, J[l + 1].data(), J[l + 1].size());
          double* C = S.get<double>("cx.C", (size_t)M * rb);
          hipLaunchKernelGGL(fiber_kernel, dim3(grid_for(M * rb)), dim3(256), 0, c.s, fa, dth, dtoff, l, nl, ra, rb,
                             dl, dr, C);
          T2S2_LAUNCH_CHECK();
          info.evaluations += (int)(M * rb);
          double* Q = S.get<double>("cx.Q", (size_t)M * rb);
          double* R = S.get<double>("cx.R", (size_t)rb * rb);
          int k = dcholqr(c, (int)M, rb, C, rb, Q, R, 1e-14);
          T2S2_CHECK(k >= 1, "source_cross: a fiber tensor vanished (f = 0 on a cross)");
          k = std::min<int>(k, (int)std::min<long>(M, kMvMaxK));
          double* W = S.get<double>("cx.W", (size_t)M * k);
          double* B = S.get<double>("cx.B", (size_t)M * k);
          int* drows = S.get<int>("cx.rows", k + 1);
          int* dmark = S.get<int>("cx.mark", (size_t)M);
          hipLaunchKernelGGL(maxvol_kernel, dim3(1), dim3(kMvThreads), (size_t)k * k * sizeof(double), c.s, (int)M,
                             k, Q, W, B, dmark, drows, drows + k, 0.01, 200);
          T2S2_LAUNCH_CHECK();
          std::vector<int> rows(k + 1);
          c.d2h(rows.data(), drows, k + 1);
          // core l = B (ra x nl x k)
          c.d2d(out.c[l], B, (size_t)M * k);
          out.r[l + 1] = k;
          std::vector<int> nI((size_t)k * (l + 1));
          for (int q = 0; q < k; ++q) {
            const int row = rows[q], a = row / nl, i = row % nl;
            for (int t = 0; t < l; ++t) nI[(size_t)q * (l + 1) + t] = I[l][(size_t)a * l + t];
            nI[(size_t)q * (l + 1) + l] = i;
          }
          I[l + 1] = nI;
          ir[l + 1] = k;
        }
        // last core: the fiber itself
        const int l = d - 1, ra = ir[l], nl = n[l];
        int* dl = S.get<int>("cx.left", std::max<size_t>(1, I[l].size()));
        if (!I[l].empty()) c.h2d(dl, I[l].data(), I[l].size());
        hipLaunchKernelGGL(fiber_kernel, dim3(grid_for((long)ra * nl)), dim3(256), 0, c.s, fa, dth, dtoff, l, nl, ra,
                           1, dl, dl, out.c[l]);
        T2S2_LAUNCH_CHECK();
        info.evaluations += ra * nl;
      } else {
        for (int l = d - 1; l >= 1; --l) {
          const int ra = ir[l], rb = jr[l + 1], nl = n[l];
          const long M = (long)nl * rb;
          int* dl = S.get<int>("cx.left", std::max<size_t>(1, I[l].size()));
          int* dr = S.get<int>("cx.right", std::max<size_t>(1, J[l + 1].size()));
          if (!I[l].empty()) c.h2d(dl, I[l].data(), I[l].size());
          if (!J[l + 1].empty()) c.h2d(dr, J[l + 1].data(), J[l + 1].size());
          double* C = S.get<double>("cx.C", (size_t)ra * M);
          hipLaunchKernelGGL(fiber_kernel, dim3(grid_for(ra * M)), dim3(256), 0, c.s, fa, dth, dtoff, l, nl, ra, rb,
                             dl, dr, C);
          T2S2_LAUNCH_CHECK();
          info.evaluations += (int)(ra * M);
          double* Ct = S.get<double>("cx.Ct", (size_t)ra * M);
          transpose(c.s, ra, M, C, M, Ct, ra);  // (nl rb) x ra
          double* Q = S.get<double>("cx.Q", (size_t)M * ra);
          double* R = S.get<double>("cx.R", (size_t)ra * ra);
          int k = dcholqr(c, (int)M, ra, Ct, ra, Q, R, 1e-14);
          T2S2_CHECK(k >= 1, "source_cross: a fiber tensor vanished (f = 0 on a cross)");
          k = std::min<int>(k, (int)std::min<long>(M, kMvMaxK));
          double* W = S.get<double>("cx.W", (size_t)M * k);
          double* B = S.get<double>("cx.B", (size_t)M * k);
          int* dcols = S.get<int>("cx.rows", k + 1);
          int* dmark = S.get<int>("cx.mark", (size_t)M);
          hipLaunchKernelGGL(maxvol_kernel, dim3(1), dim3(kMvThreads), (size_t)k * k * sizeof(double), c.s, (int)M,
                             k, Q, W, B, dmark, dcols, dcols + k, 0.01, 200);
          T2S2_LAUNCH_CHECK();
          std::vector<int> cols(k + 1);
          c.d2h(cols.data(), dcols, k + 1);
          // core l = B^T (k x nl x rb)
          transpose(c.s, M, k, B, k, out.c[l], M);
          out.r[l] = k;
          const int w = d - l;
          std::vector<int> nJ((size_t)k * w);
          for (int q = 0; q < k; ++q) {
            const int col = cols[q], i = col / rb, b = col % rb;
            nJ[(size_t)q * w] = i;
            for (int t = 1; t < w; ++t) nJ[(size_t)q * w + t] = J[l + 1][(size_t)b * (w - 1) + (t - 1)];
          }
          J[l] = nJ;
          jr[l] = k;
        }
        // first core: the fiber itself
        const int nl = n[0], rb = jr[1];
        int* dr = S.get<int>("cx.right", std::max<size_t>(1, J[1].size()));
        if (!J[1].empty()) c.h2d(dr, J[1].data(), J[1].size());
        hipLaunchKernelGGL(fiber_kernel, dim3(grid_for((long)nl * rb)), dim3(256), 0, c.s, fa, dth, dtoff, 0, nl, 1,
                           rb, dr, dr, out.c[0]);
        T2S2_LAUNCH_CHECK();
        info.evaluations += nl * rb;
      }
    }
    // error on the samples
    int rmx = 1;
    for (int l = 0; l <= d; ++l) rmx = std::max(rmx, out.r[l]);
    double* V0 = S.get<double>("cx.V0", (size_t)samples * rmx);
    double* V1 = S.get<double>("cx.V1", (size_t)samples * rmx);
    fill(c.s, V0, samples, 1.0);
    for (int l = 0; l < d; ++l) {
      hipLaunchKernelGGL(sample_tt_kernel, dim3(grid_for((long)samples * out.r[l + 1])), dim3(256), 0, c.s, samples, d,
                         l, out.r[l], n[l], out.r[l + 1], dsidx, out.c[l], V0, V1);
      T2S2_LAUNCH_CHECK();
      std::swap(V0, V1);
    }
    std::vector<double> tv(samples);
    c.d2h(tv.data(), V0, samples);
    double e2 = 0.0;
    for (int s = 0; s < samples; ++s) e2 += (tv[s] - hfs[s]) * (tv[s] - hfs[s]);
    info.rank = r;
    info.sample_error = fnorm2 > 0 ? std::sqrt(e2 / fnorm2) : std::sqrt(e2);
    T2S2_CHECK(std::isfinite(info.sample_error), "source_cross: non-finite function values");
    if (info.sample_error <= tol || r >= rmax) break;
    r = std::min(2 * r, rmax);
  }
  tt_round(c, out, 0.1 * tol, rmax);
  c.sync();
  return info;
}

}  // namespace t2s2
