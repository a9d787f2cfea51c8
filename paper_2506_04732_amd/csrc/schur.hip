// Real Schur form by the implicit multishift QR iteration (small-bulge
// multishift: several double-shift bulges chased together), and its
// conversion to a complex Schur form, for the small nonsymmetric matrices of
// the TT solver (Hessenberg input, n <= 512).
//
// One workgroup.  The Hessenberg matrix lives in LDS in packed row form (row
// i keeps columns max(0, i-3) .. n-1: a 3 x 3 bulge reaches three below the
// diagonal) whenever it fits (n <= ~191 in FP64, ~271 in FP32), else in
// global memory.  Both precisions share one template.  The Schur vectors
// (rows of Z^T) are updated lazily: the reflectors of a few consecutive
// phases are multiplied into a small matrix G in LDS and applied to the
// affected rows of Z^T in one pass, so the chase itself never waits on
// global memory.
#include <cfloat>

#include "dense_small.h"

namespace t2s2 {

namespace {

constexpr int kFqThreads = 256;

__host__ __device__ inline int row_start(int i) { return i > 3 ? i - 3 : 0; }

// packed-row offset of (i, j): rows 0..3 keep all n columns, row i > 3 keeps
// columns i-3..n-1
__host__ __device__ inline int packed_off(int n, int i, int j) {
  const int d = i > 3 ? i - 3 : 0;
  return i * n - ((d * (d - 1)) >> 1) - d + j;
}

template <bool LDS, class R>
struct HStore {
  R* base;
  int n;
  __device__ R& at(int i, int j) const {
    if constexpr (LDS) return base[packed_off(n, i, j)];
    else return base[(long)i * n + j];
  }
};

// ------------------------------------------------- multishift bulge chase
// KB double-shift bulges chased together (small-bulge multishift QR): the
// shifts of one sweep are the eigenvalues of the trailing 2KB x 2KB block;
// bulge b enters at the top 4b phases after bulge 0, so the bulges stay 4
// rows apart.  Per phase every thread computes the KB reflectors from the
// current H (disjoint rows: no dependence between them), then all row
// updates (left products) are applied, a barrier, then all column updates
// (right products): left and right products of different bulges commute,
// so the result is the product of the same reflectors as in KB successive
// double-shift sweeps.  Deflation is checked between sweeps; active blocks
// smaller than kMsMin use one bulge per sweep (the plain double-shift
// iteration).  Z^T is updated lazily through the batch matrix G as above.
constexpr int kMW = 8;       // steady-state phases per Z batch
constexpr int kMsMin = 24;   // smallest active block chased with KB bulges
constexpr int kMsBulges = 4; // bulges per sweep

template <int KB>
struct MsDims {
  static constexpr int G = 4 * (KB - 1) + 3 + kMW;  // rows covered by one batch
  static constexpr int NS = 2 * KB;                  // shift window
};

template <class R, int KB>
constexpr long kMsLdsBytes = 160000 - (long)(MsDims<KB>::G * MsDims<KB>::G + MsDims<KB>::NS * MsDims<KB>::NS +
                                             2 * MsDims<KB>::NS + 2 * KB) * sizeof(R) -
                             128;

// Eigenvalues of the ns x ns upper Hessenberg Hs (row stride ld) by the
// double-shift QR iteration without Schur vectors, run by one wavefront
// (LDS accesses of one wavefront are ordered, no barrier needed).
template <class R>
__device__ void small_eigs_wave(int ns, R* Hs, int ld, R* wr, R* wi) {
  const int lane = threadIdx.x & 63;
  const R ulp = sizeof(R) == 8 ? (R)1e-14 : (R)FLT_EPSILON;
  int hi = ns - 1, its = 0, guard = 0;
  while (hi >= 0) {
    if (++guard > 30 * ns) {  // no convergence: the diagonal stands in
      for (int i = lane; i <= hi; i += 64) {
        wr[i] = Hs[i * ld + i];
        wi[i] = R(0);
      }
      __builtin_amdgcn_wave_barrier();
      break;
    }
    bool neg = false;
    if (lane >= 1 && lane <= hi) {
      R sc = fabs(Hs[(lane - 1) * ld + lane - 1]) + fabs(Hs[lane * ld + lane]);
      if (sc == R(0)) sc = R(1);
      neg = fabs(Hs[lane * ld + lane - 1]) <= ulp * sc;
    }
    const unsigned long long msk = __ballot(neg);
    const int l = msk ? 63 - __clzll(msk) : 0;
    __builtin_amdgcn_wave_barrier();
    if (l >= 1 && lane == 0) Hs[l * ld + l - 1] = R(0);
    __builtin_amdgcn_wave_barrier();
    if (l == hi) {
      if (lane == 0) {
        wr[hi] = Hs[hi * ld + hi];
        wi[hi] = R(0);
      }
      __builtin_amdgcn_wave_barrier();
      hi -= 1;
      its = 0;
      continue;
    }
    if (l == hi - 1) {
      if (lane == 0) {
        const R a = Hs[(hi - 1) * ld + hi - 1], b = Hs[(hi - 1) * ld + hi];
        const R c = Hs[hi * ld + hi - 1], d = Hs[hi * ld + hi];
        const R pp = R(0.5) * (a - d), bc = b * c, disc = pp * pp + bc;
        if (disc >= R(0)) {
          const R z = pp + copysign(sqrt(disc), pp);
          wr[hi - 1] = d + z;
          wr[hi] = (z != R(0)) ? d - bc / z : d;
          wi[hi - 1] = wi[hi] = R(0);
        } else {
          wr[hi - 1] = wr[hi] = R(0.5) * (a + d);
          wi[hi - 1] = sqrt(-disc);
          wi[hi] = -sqrt(-disc);
        }
      }
      __builtin_amdgcn_wave_barrier();
      hi -= 2;
      its = 0;
      continue;
    }
    const R a = Hs[(hi - 1) * ld + hi - 1], b = Hs[(hi - 1) * ld + hi];
    const R c = Hs[hi * ld + hi - 1], d = Hs[hi * ld + hi];
    R s = a + d, t = a * d - b * c;
    if (its > 0 && its % 10 == 0) {
      const R e = fabs(c) + fabs(Hs[(hi - 1) * ld + hi - 2]);
      s = R(1.5) * e;
      t = e * e;
    }
    ++its;
    const int p = hi - l + 1;
    R x, y, z;
    {
      const R h00 = Hs[l * ld + l], h01 = Hs[l * ld + l + 1], h10 = Hs[(l + 1) * ld + l];
      const R h11 = Hs[(l + 1) * ld + l + 1], h21 = Hs[(l + 2) * ld + l + 1];
      x = h00 * h00 + h01 * h10 - s * h00 + t;
      y = h10 * (h00 + h11 - s);
      z = h10 * h21;
    }
    for (int k = 0; k <= p - 3; ++k) {
      const int a0 = l + k;
      const R sg = sqrt(x * x + y * y + z * z);
      if (sg > R(0) && (y != R(0) || z != R(0))) {
        const R v0 = x + (x >= R(0) ? sg : -sg);
        const R tau = R(2) / (v0 * v0 + y * y + z * z);
        const int c0 = (k > 0) ? a0 - 1 : l;
        const int j = c0 + lane;
        if (j <= hi) {
          const R h0 = Hs[a0 * ld + j], h1 = Hs[(a0 + 1) * ld + j], h2 = Hs[(a0 + 2) * ld + j];
          const R sm = tau * (v0 * h0 + y * h1 + z * h2);
          Hs[a0 * ld + j] = h0 - sm * v0;
          Hs[(a0 + 1) * ld + j] = (k > 0 && j == a0 - 1) ? R(0) : h1 - sm * y;
          Hs[(a0 + 2) * ld + j] = (k > 0 && j == a0 - 1) ? R(0) : h2 - sm * z;
        }
        __builtin_amdgcn_wave_barrier();
        const int r1 = min(a0 + 3, hi);
        const int i = l + lane;
        if (i <= r1) {
          const R h0 = Hs[i * ld + a0], h1 = Hs[i * ld + a0 + 1], h2 = Hs[i * ld + a0 + 2];
          const R sm = tau * (h0 * v0 + h1 * y + h2 * z);
          Hs[i * ld + a0] = h0 - sm * v0;
          Hs[i * ld + a0 + 1] = h1 - sm * y;
          Hs[i * ld + a0 + 2] = h2 - sm * z;
        }
        __builtin_amdgcn_wave_barrier();
      }
      x = Hs[(a0 + 1) * ld + a0];
      y = Hs[(a0 + 2) * ld + a0];
      z = (k < p - 3) ? Hs[(a0 + 3) * ld + a0] : R(0);
    }
    {
      const R sg = sqrt(x * x + y * y);
      if (sg > R(0) && y != R(0)) {
        const R v0 = x + (x >= R(0) ? sg : -sg);
        const R tau = R(2) / (v0 * v0 + y * y);
        const int a0 = hi - 1;
        const int j = hi - 2 + lane;
        if (j <= hi) {
          const R h0 = Hs[a0 * ld + j], h1 = Hs[hi * ld + j];
          const R sm = tau * (v0 * h0 + y * h1);
          Hs[a0 * ld + j] = h0 - sm * v0;
          Hs[hi * ld + j] = (j == hi - 2) ? R(0) : h1 - sm * y;
        }
        __builtin_amdgcn_wave_barrier();
        const int i = l + lane;
        if (i <= hi) {
          const R h0 = Hs[i * ld + a0], h1 = Hs[i * ld + hi];
          const R sm = tau * (h0 * v0 + h1 * y);
          Hs[i * ld + a0] = h0 - sm * v0;
          Hs[i * ld + hi] = h1 - sm * y;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
}

template <bool LDS, class R, int KB>
__global__ void __launch_bounds__(kFqThreads) francis_ms_kernel(int n, const R* __restrict__ Hin, R* __restrict__ Hg,
                                                                R* __restrict__ ZT, R* __restrict__ Tout,
                                                                int* __restrict__ info, int max_sweeps) {
  constexpr int GS = MsDims<KB>::G;
  constexpr int NS = MsDims<KB>::NS;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  R* lds = reinterpret_cast<R*>(lds_raw);
  __shared__ R G[GS * GS];
  __shared__ R Hs[NS * NS];
  __shared__ R s_wr[NS], s_wi[NS];
  __shared__ R s_sh[KB][2];
  __shared__ int s_l, s_hi, s_done;
  HStore<LDS, R> H{LDS ? lds : Hg, n};
  for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (j >= row_start(i)) H.at(i, j) = (j >= i - 1) ? Hin[e] : R(0.0);
  }
  if (threadIdx.x == 0) {
    s_hi = n - 1;
    s_done = 0;
  }
  __syncthreads();

  // Z batch state (identical in every thread)
  int zk0 = 0, zcnt = 0;
  auto flush = [&]() {
    if (zcnt > 0) {
      const int rows = min(GS, n - zk0);
      for (int col = threadIdx.x; col < n; col += blockDim.x) {
        R old[GS];
#pragma unroll
        for (int b = 0; b < GS; ++b) old[b] = (b < rows) ? ZT[(long)(zk0 + b) * n + col] : R(0.0);
#pragma unroll
        for (int a = 0; a < GS; ++a) {
          if (a >= rows) break;
          R acc = R(0.0);
#pragma unroll
          for (int b = 0; b < GS; ++b) acc = fma(G[a * GS + b], old[b], acc);
          ZT[(long)(zk0 + a) * n + col] = acc;
        }
      }
    }
    __syncthreads();
    zcnt = 0;
  };

  const R ulp = sizeof(R) == 8 ? (R)1e-13 : (R)FLT_EPSILON;
  int total = 0, its = 0;
  while (true) {
    // ---- deflation: largest l <= hi with a negligible subdiagonal.  Every
    // thread has read the previous iteration's s_l before thread 0 resets it
    // (a wave released late from the last barrier would otherwise read the
    // reset value and take the other branch)
    __syncthreads();
    if (threadIdx.x == 0) s_l = 0;
    __syncthreads();
    int hi = s_hi;
    for (int i = 1 + threadIdx.x; i <= hi; i += blockDim.x) {
      R sc = fabs(H.at(i - 1, i - 1)) + fabs(H.at(i, i));
      if (sc == R(0.0)) sc = R(1.0);
      if (fabs(H.at(i, i - 1)) <= ulp * sc) atomicMax(&s_l, i);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int l = s_l;
      if (l >= 1 && l <= hi) H.at(l, l - 1) = R(0.0);
      if (hi < 0) {
        s_done = 1;
      } else if (l >= hi - 1) {
        s_hi = l - 1;  // 1 x 1 or 2 x 2 block converged
        s_l = -1;
        if (l - 1 < 0) s_done = 1;
      }
    }
    __syncthreads();
    if (s_done || total >= max_sweeps) break;
    const int l = s_l;
    hi = s_hi;
    if (l < 0) {
      its = 0;
      continue;
    }
    const int p = hi - l + 1;
    const int nb = (p >= kMsMin) ? KB : 1;
    // ---- shifts
    if (nb == 1) {
      if (threadIdx.x == 0) {
        const R a = H.at(hi - 1, hi - 1), b = H.at(hi - 1, hi), c = H.at(hi, hi - 1), d = H.at(hi, hi);
        R sum = a + d, prod = a * d - b * c;
        if (its > 0 && its % 10 == 0) {
          const R e = fabs(c) + fabs(H.at(hi - 1, hi - 2));
          sum = R(1.5) * e;
          prod = e * e;
        }
        s_sh[0][0] = sum;
        s_sh[0][1] = prod;
      }
    } else if (its > 0 && its % 6 == 0) {
      if (threadIdx.x == 0) {
        for (int q = 0; q < KB; ++q) {
          const int i = hi - 2 * q;
          const R ss = fabs(H.at(i, i - 1)) + fabs(H.at(i - 1, i - 2));
          const R aa = R(0.75) * ss + H.at(i, i);
          s_sh[q][0] = R(2) * aa;
          s_sh[q][1] = aa * aa + R(0.4375) * ss * ss;
        }
      }
    } else if (threadIdx.x < 64) {
      const int base = hi - NS + 1;
      for (int e = threadIdx.x; e < NS * NS; e += 64) {
        const int i = e / NS, j = e % NS;
        Hs[e] = (j >= i - 1) ? H.at(base + i, base + j) : R(0);
      }
      __builtin_amdgcn_wave_barrier();
      small_eigs_wave<R>(NS, Hs, NS, s_wr, s_wi);
      __builtin_amdgcn_wave_barrier();
      if (threadIdx.x == 0) {
        // complex pairs as they come, real shifts sorted and paired
        R re[NS];
        int nr = 0, q = 0;
        for (int i = 0; i < NS; ++i) {
          if (s_wi[i] > R(0) && q < KB) {
            s_sh[q][0] = R(2) * s_wr[i];
            s_sh[q][1] = s_wr[i] * s_wr[i] + s_wi[i] * s_wi[i];
            ++q;
          } else if (s_wi[i] == R(0)) {
            re[nr++] = s_wr[i];
          }
        }
        for (int i = 1; i < nr; ++i) {
          const R v = re[i];
          int j = i - 1;
          while (j >= 0 && re[j] > v) {
            re[j + 1] = re[j];
            --j;
          }
          re[j + 1] = v;
        }
        for (int i = 0; i + 1 < nr && q < KB; i += 2) {
          s_sh[q][0] = re[i] + re[i + 1];
          s_sh[q][1] = re[i] * re[i + 1];
          ++q;
        }
        for (; q < KB; ++q) {  // (an odd real count cannot occur; guard anyway)
          s_sh[q][0] = R(2) * H.at(hi, hi);
          s_sh[q][1] = H.at(hi, hi) * H.at(hi, hi);
        }
      }
    }
    __syncthreads();
    R shs[KB], sht[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      shs[q] = s_sh[q][0];
      sht[q] = s_sh[q][1];
    }
    ++its;
    ++total;
    // ---- one sweep: nb bulges, 4 rows apart; thread group b (kFqThreads / nb
    // threads) owns bulge b
    const int nph = (p - 1) + 4 * (nb - 1);
    const int gsz = kFqThreads / nb;
    const int myb = threadIdx.x / gsz, t = threadIdx.x % gsz;
    const R shb = shs[0], thb = sht[0];
    R mys = shb, myt = thb;
#pragma unroll
    for (int q = 1; q < KB; ++q)
      if (q == myb) {
        mys = shs[q];
        myt = sht[q];
      }
    for (int ph = 0; ph < nph; ++ph) {
      // rows touched by the phase (positions are fixed by ph)
      int amin = n, amax = -1;
      for (int b = 0; b < nb; ++b) {
        const int pos = ph - 4 * b;
        if (pos >= 0 && pos <= p - 2) {
          amin = min(amin, l + pos);
          amax = max(amax, l + pos + (pos <= p - 3 ? 2 : 1));
        }
      }
      if (zcnt > 0 && (amin < zk0 || amax > zk0 + GS - 1)) flush();
      if (zcnt == 0) {
        for (int e = threadIdx.x; e < GS * GS; e += blockDim.x) G[e] = ((e / GS) == (e % GS)) ? R(1.0) : R(0.0);
        zk0 = amin;
        __syncthreads();
      }
      // this group's reflector
      bool act = false;
      R v0 = R(0), v1 = R(0), v2 = R(0), tau = R(0);
      int a = 0, w = 3, c0 = 0, r1 = 0, zc = -1;
      {
        const int pos = ph - 4 * myb;
        if (pos >= 0 && pos <= p - 2) {
          a = l + pos;
          R x, y, z;
          if (pos == 0) {
            const R h00 = H.at(l, l), h01 = H.at(l, l + 1), h10 = H.at(l + 1, l), h11 = H.at(l + 1, l + 1);
            const R h21 = H.at(l + 2, l + 1);
            x = h00 * h00 + h01 * h10 - mys * h00 + myt;
            y = h10 * (h00 + h11 - mys);
            z = h10 * h21;
            c0 = l;
            r1 = min(l + 3, hi);
          } else if (pos <= p - 3) {
            x = H.at(a, a - 1);
            y = H.at(a + 1, a - 1);
            z = H.at(a + 2, a - 1);
            c0 = a - 1;
            r1 = min(a + 3, hi);
            zc = a - 1;
          } else {
            x = H.at(a, a - 1);
            y = H.at(a + 1, a - 1);
            z = R(0);
            w = 2;
            c0 = a - 1;
            r1 = hi;
            zc = a - 1;
          }
          const R sg = sqrt(x * x + y * y + z * z);
          if (sg > R(0) && (y != R(0) || z != R(0))) {
            act = true;
            v0 = x + (x >= R(0) ? sg : -sg);
            v1 = y;
            v2 = z;
            tau = R(2) / (v0 * v0 + y * y + z * z);
          }
        }
      }
      // ---- row updates of H (columns c0..n-1) and of G
      if (act) {
        for (int j = c0 + t; j < n; j += gsz) {
          const R h0 = H.at(a, j), h1 = H.at(a + 1, j), h2 = (w == 3) ? H.at(a + 2, j) : R(0.0);
          const R sm = tau * (v0 * h0 + v1 * h1 + v2 * h2);
          H.at(a, j) = h0 - sm * v0;
          if (j == zc) {
            H.at(a + 1, j) = R(0.0);
            if (w == 3) H.at(a + 2, j) = R(0.0);
          } else {
            H.at(a + 1, j) = h1 - sm * v1;
            if (w == 3) H.at(a + 2, j) = h2 - sm * v2;
          }
        }
        const int ga = a - zk0;
        for (int c = t; c < GS; c += gsz) {
          const R g0 = G[ga * GS + c], g1 = G[(ga + 1) * GS + c], g2 = (w == 3) ? G[(ga + 2) * GS + c] : R(0.0);
          const R sm = tau * (v0 * g0 + v1 * g1 + v2 * g2);
          G[ga * GS + c] = g0 - sm * v0;
          G[(ga + 1) * GS + c] = g1 - sm * v1;
          if (w == 3) G[(ga + 2) * GS + c] = g2 - sm * v2;
        }
      }
      __syncthreads();
      // ---- column updates of H (rows 0..r1)
      if (act) {
        for (int i = t; i <= r1; i += gsz) {
          const R h0 = H.at(i, a), h1 = H.at(i, a + 1), h2 = (w == 3) ? H.at(i, a + 2) : R(0.0);
          const R sm = tau * (h0 * v0 + h1 * v1 + h2 * v2);
          H.at(i, a) = h0 - sm * v0;
          H.at(i, a + 1) = h1 - sm * v1;
          if (w == 3) H.at(i, a + 2) = h2 - sm * v2;
        }
      }
      __syncthreads();
      ++zcnt;
    }
  }
  flush();
  for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    Tout[e] = (j >= i - 1 && j >= row_start(i)) ? H.at(i, j) : R(0.0);
  }
  if (threadIdx.x == 0) info[0] = s_done ? total : -total;
}

// Real quasi-triangular T (1 x 1 and 2 x 2 diagonal blocks), real Z^T  ->
// complex upper-triangular Tc = P^H T P and Z'^T = (Z P)^T, with P block
// diagonal: for each 2 x 2 block B, the unitary [v, w], v a unit eigenvector
// of B, makes P^H B P upper triangular.
template <class R>
__global__ void __launch_bounds__(256) rsf2csf_kernel(int n, const R* __restrict__ T, const R* __restrict__ ZT,
                                                      typename CxOf<R>::type* __restrict__ Tc,
                                                      typename CxOf<R>::type* __restrict__ ZTc,
                                                      int* __restrict__ bstart, typename CxOf<R>::type* __restrict__ U) {
  using C = typename CxOf<R>::type;
  using CX = CxOf<R>;
  if (threadIdx.x == 0) {
    int k = 0;
    while (k < n) {
      if (k + 1 < n && T[(long)(k + 1) * n + k] != R(0.0)) {
        const R a = T[(long)k * n + k], b = T[(long)k * n + k + 1];
        const R c = T[(long)(k + 1) * n + k], d = T[(long)(k + 1) * n + k + 1];
        const R hm = R(0.5) * (a - d);
        const R disc = hm * hm + b * c;
        C lam;
        if (disc >= R(0.0)) {
          const R sq = sqrt(disc);
          lam = CX::make(R(0.5) * (a + d) + (hm >= R(0.0) ? sq : -sq), R(0.0));
        } else {
          lam = CX::make(R(0.5) * (a + d), sqrt(-disc));
        }
        // eigenvector of B for lam: (b, lam - a) or (lam - d, c)
        C v0, v1;
        const C la = CX::make(lam.x - a, lam.y), ld = CX::make(lam.x - d, lam.y);
        if (fabs(b) + cabs(la) >= fabs(c) + cabs(ld)) {
          v0 = CX::make(b, R(0.0));
          v1 = la;
        } else {
          v0 = ld;
          v1 = CX::make(c, R(0.0));
        }
        const R nv = sqrt(cabs2(v0) + cabs2(v1));
        v0 = cscale(v0, (R)1 / nv);
        v1 = cscale(v1, (R)1 / nv);
        // U = [[v0, -conj(v1)], [v1, conj(v0)]]
        U[2 * k + 0] = v0;
        U[2 * k + 1] = CX::make(-v1.x, v1.y);
        U[2 * (k + 1) + 0] = v1;
        U[2 * (k + 1) + 1] = cconj(v0);
        bstart[k] = k;
        bstart[k + 1] = k;
        k += 2;
      } else {
        bstart[k] = -1;
        k += 1;
      }
    }
  }
  __syncthreads();
  // P[s+p][s+q] = U[2*(s+p) + q] for a block starting at s; identity otherwise
  auto Pent = [&](int r, int c) -> C {
    const int s = bstart[c];
    if (s < 0) return (r == c) ? CX::make(R(1.0), R(0.0)) : CX::make(R(0.0), R(0.0));
    if (r != s && r != s + 1) return CX::make(R(0.0), R(0.0));
    return U[2 * r + (c - s)];
  };
  const long nn = (long)n * n;
  for (long e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    C acc = CX::make(R(0.0), R(0.0));
    if (j >= i - 1) {
      const int si = bstart[i] < 0 ? i : bstart[i], ni = bstart[i] < 0 ? 1 : 2;
      const int sj = bstart[j] < 0 ? j : bstart[j], nj = bstart[j] < 0 ? 1 : 2;
      for (int a = si; a < si + ni; ++a) {
        const C pa = cconj(Pent(a, i));
        for (int b = sj; b < sj + nj; ++b) {
          const R t = T[(long)a * n + b];
          if (t == R(0.0)) continue;
          acc = cadd(acc, cmul(pa, cscale(Pent(b, j), t)));
        }
      }
    }
    Tc[e] = (j >= i) ? acc : CX::make(R(0.0), R(0.0));
  }
  // Z'^T[j][i] = sum_b P[b][j] ZT[b][i]
  for (long e = threadIdx.x; e < nn; e += blockDim.x) {
    const int j = (int)(e / n), i = (int)(e % n);
    const int sj = bstart[j] < 0 ? j : bstart[j], nj = bstart[j] < 0 ? 1 : 2;
    C acc = CX::make(R(0.0), R(0.0));
    for (int b = sj; b < sj + nj; ++b) acc = cadd(acc, cscale(Pent(b, j), ZT[(long)b * n + i]));
    ZTc[e] = acc;
  }
}

}  // namespace

long francis_packed_doubles(int n) {
  long o = 0;
  for (int i = 0; i < n; ++i) o += n - row_start(i);
  return o;
}

static int g_francis_steps = 0;  // 0: default limit
void set_francis_step_limit(int steps) { g_francis_steps = steps; }
int francis_step_limit(int n) { return g_francis_steps > 0 ? g_francis_steps : 40 * n + 100; }

template <class R>
static void schur_francis_t(hipStream_t s, int n, const R* H, R* Hwork, R* ZT, R* T, int* info) {
  T2S2_CHECK(n >= 1 && n <= 512, "schur_francis: n must be in [1, 512]");
  TimedScope ts(s, KC_SCHUR, sizeof(R) * 4.0 * n * n, 10.0 * (double)n * n * n);
  const long need = francis_packed_doubles(n) * (long)sizeof(R);
  if (need <= kMsLdsBytes<R, kMsBulges>)
    hipLaunchKernelGGL((francis_ms_kernel<true, R, kMsBulges>), dim3(1), dim3(kFqThreads), (size_t)need, s, n, H,
                       Hwork, ZT, T, info, francis_step_limit(n));
  else
    hipLaunchKernelGGL((francis_ms_kernel<false, R, kMsBulges>), dim3(1), dim3(kFqThreads), 0, s, n, H, Hwork, ZT,
                       T, info, francis_step_limit(n));
  T2S2_LAUNCH_CHECK();
}

void schur_francis(hipStream_t s, int n, const double* H, double* Hwork, double* ZT, double* T, int* info) {
  schur_francis_t<double>(s, n, H, Hwork, ZT, T, info);
}
void schur_francis(hipStream_t s, int n, const float* H, float* Hwork, float* ZT, float* T, int* info) {
  schur_francis_t<float>(s, n, H, Hwork, ZT, T, info);
}

template <class R>
static void rsf2csf_t(hipStream_t s, int n, const R* T, const R* ZT, typename CxOf<R>::type* Tc,
                      typename CxOf<R>::type* ZTc, int* bstart, typename CxOf<R>::type* U) {
  TimedScope ts(s, KC_SCHUR, sizeof(R) * 2.0 * n * n + 2.0 * sizeof(R) * 2.0 * n * n, 0.0);
  hipLaunchKernelGGL(rsf2csf_kernel<R>, dim3(1), dim3(256), 0, s, n, T, ZT, Tc, ZTc, bstart, U);
  T2S2_LAUNCH_CHECK();
}

void rsf2csf(hipStream_t s, int n, const double* T, const double* ZT, double2* Tc, double2* ZTc, int* bstart,
             double2* U) {
  rsf2csf_t<double>(s, n, T, ZT, Tc, ZTc, bstart, U);
}
void rsf2csf(hipStream_t s, int n, const float* T, const float* ZT, float2* Tc, float2* ZTc, int* bstart,
             float2* U) {
  rsf2csf_t<float>(s, n, T, ZT, Tc, ZTc, bstart, U);
}

}  // namespace t2s2
