// Local Kronecker-sum solve with the left interface in upper Hessenberg form.
//
// The local operator of the alternating scheme is L (+) K (+) R (a Kronecker
// sum of the left interface, the 1D mode matrix and the right interface).
// With L = Q H Q^T (Hessenberg, orthogonal Q), K = Z T Z^H (complex Schur)
// and R = V diag(lamR) V^{-1}, the transformed system splits over the right
// index b into independent Sylvester equations H Y + Y T^T + lamR[b] Y = G,
// which the Hessenberg-Schur method solves as a chain of m shifted Hessenberg
// systems (j = m-1 .. 0, the right-hand side of j collecting the solved
// columns j' > j through T).
//
// One shifted system B y = g, B = H + sigma I upper Hessenberg, is solved in a
// single bottom-up pass with O(r1) state: column k-1 of B is eliminated
// against the carried column k (2 x 2 column transform E_k, pivoting on the
// larger of the two row-k entries), which completes column k of the upper
// triangular R = B E_{r1-1} ... E_1; row k of R is then complete too, so
// x_k = (g_k - sum_{j>k} R[k][j] x_j) / R[k][k] is back-substituted in the
// same pass.  y = E_{r1-1} ... E_1 x follows by a forward recurrence over the
// stored multipliers and swap flags.  No factor is stored.
//
// One wavefront per right index b; lane l owns rows l, l+64, l+128, ...
// (RPL rows).  H is read column-major from global memory (all wavefronts
// read the same H, so it stays in L2) through a ring of kPD prefetched
// columns; the m right-hand sides of the chain live in LDS.
#include "kron_hess.h"

namespace t2s2 {

namespace {

constexpr int kPD = 4;               // prefetch distance in columns of H
constexpr long kHessLds = 160000;    // dynamic LDS available to one workgroup

template <class R>
__device__ inline R rdlane(R v, int l);
template <>
__device__ inline double rdlane<double>(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <>
__device__ inline float rdlane<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 1/d for d > 0: hardware estimate refined by two Newton steps (FP64), or
// the hardware reciprocal (FP32, 1 ulp)
__device__ inline double rcp_pos(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ inline float rcp_pos(float d) { return __builtin_amdgcn_rcpf(d); }

template <class R>
struct TinyR;
template <>
struct TinyR<double> {
  static constexpr double v = 1e-290;
};
template <>
struct TinyR<float> {
  static constexpr float v = 1e-36f;
};

template <class R, int RPL>
__global__ void __launch_bounds__(64)
kron_hess_kernel(int r1, int m, int r2, const R* __restrict__ Hc, const typename CxOf<R>::type* __restrict__ T,
                 const typename CxOf<R>::type* __restrict__ lamR, typename CxOf<R>::type* __restrict__ h, long sa,
                 long sj, long sb) {
  using C = typename CxOf<R>::type;
  using CX = CxOf<R>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  C* G = reinterpret_cast<C*>(lds_raw);  // [m][RPL][64]
  const int lane = threadIdx.x;
  // workgroups are dispatched round-robin over the 8 XCDs: give each XCD a
  // contiguous range of b so that neighbours share L2 lines of h
  int b = blockIdx.x;
  {
    const int full = (r2 / 8) * 8;
    if (b < full) b = (b % 8) * (r2 / 8) + b / 8;
  }
  const C zero = CX::make(R(0), R(0));
  for (int j = 0; j < m; ++j) {
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int a = 64 * t + lane;
      G[(j * RPL + t) * 64 + lane] = a < r1 ? h[a * sa + j * sj + b * sb] : zero;
    }
  }
  const C lb = lamR[b];
  const R tiny = TinyR<R>::v;

  for (int j = m - 1; j >= 0; --j) {
    const C tjj = T[(long)j * m + j];
    const C sg = CX::make(tjj.x + lb.x, tjj.y + lb.y);
    C cur[RPL], acc[RPL], x[RPL], mu[RPL], rhs[RPL];
    int sw[RPL];
    R ring[kPD][RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int a = 64 * t + lane;
      const R v = a < r1 ? Hc[(long)(r1 - 1) * r1 + a] : R(0);
      cur[t] = CX::make(v + (a == r1 - 1 ? sg.x : R(0)), a == r1 - 1 ? sg.y : R(0));
      acc[t] = zero;
      x[t] = zero;
      mu[t] = zero;
      sw[t] = 0;
      rhs[t] = G[(j * RPL + t) * 64 + lane];
    }
    // ring slot s holds column k-1 for the step k with k % kPD == s
#pragma unroll
    for (int s = 0; s < kPD; ++s) {
      const int k = r1 - 1 - ((r1 - 1 - s + 4 * kPD) % kPD);
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int a = 64 * t + lane;
        ring[s][t] = (k >= 1 && a <= k && a < r1) ? Hc[(long)(k - 1) * r1 + a] : R(0);
      }
    }
    // ---- bottom-up elimination with interleaved back substitution
#pragma unroll
    for (int t = RPL - 1; t >= 0; --t) {
      for (int li0 = 63; li0 >= 0; li0 -= kPD) {
#pragma unroll
        for (int u = 0; u < kPD; ++u) {
          const int li = li0 - u;
          const int k = 64 * t + li;
          const int slot = (3 - u) & (kPD - 1);  // == k % kPD since li0 % kPD == 3
          if (k >= 1 && k <= r1 - 1) {
            const C p1 = CX::make(rdlane(cur[t].x, li), rdlane(cur[t].y, li));
            const R p2 = rdlane(ring[slot][t], li);  // B[k][k-1], real
            const R n1 = cabs2(p1), n2 = p2 * p2;
            const bool swp = n2 > n1;
            const C piv = swp ? CX::make(p2, R(0)) : p1;
            const C oth = swp ? p1 : CX::make(p2, R(0));
            const R den = fmax(swp ? n2 : n1, tiny);
            const R id = rcp_pos(den);
            const C inv = CX::make(piv.x * id, -piv.y * id);
            const C muk = cmul(oth, inv);
            const C dk = CX::make(rdlane(rhs[t].x - acc[t].x, li), rdlane(rhs[t].y - acc[t].y, li));
            const C xk = cmul(dk, inv);
            if (lane == li) {
              x[t] = xk;
              mu[t] = muk;
              sw[t] = swp ? 1 : 0;
            }
#pragma unroll
            for (int tt = 0; tt < RPL; ++tt) {
              if (tt <= t) {
                const int a = 64 * tt + lane;
                const bool dg = (a == k - 1);
                const C nx = CX::make(ring[slot][tt] + (dg ? sg.x : R(0)), dg ? sg.y : R(0));
                const C A = swp ? nx : cur[tt];
                const C Bc = swp ? cur[tt] : nx;
                acc[tt] = CX::make(fma(A.x, xk.x, fma(-A.y, xk.y, acc[tt].x)),
                                   fma(A.x, xk.y, fma(A.y, xk.x, acc[tt].y)));
                cur[tt] = CX::make(fma(-muk.x, A.x, fma(muk.y, A.y, Bc.x)),
                                   fma(-muk.x, A.y, fma(-muk.y, A.x, Bc.y)));
              }
            }
            // prefetch column k-1-kPD for the step k-kPD
            const int kn = k - kPD;
            if (kn >= 1) {
#pragma unroll
              for (int tt = 0; tt < RPL; ++tt) {
                const int a = 64 * tt + lane;
                ring[slot][tt] = (a <= kn && a < r1) ? Hc[(long)(kn - 1) * r1 + a] : R(0);
              }
            }
          }
        }
      }
    }
    // k = 0
    C c0;
    {
      const C p = CX::make(rdlane(cur[0].x, 0), rdlane(cur[0].y, 0));
      const R id = rcp_pos(fmax(cabs2(p), tiny));
      const C inv = CX::make(p.x * id, -p.y * id);
      const C dk = CX::make(rdlane(rhs[0].x - acc[0].x, 0), rdlane(rhs[0].y - acc[0].y, 0));
      c0 = cmul(dk, inv);
    }
    // ---- y = E_{r1-1} ... E_1 x (forward recurrence), into acc
    C c = c0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) acc[t] = zero;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      for (int li = 0; li < 64; ++li) {
        const int k = 64 * t + li;
        if (k < 1 || k > r1 - 1) continue;
        const C xk = CX::make(rdlane(x[t].x, li), rdlane(x[t].y, li));
        const C mk = CX::make(rdlane(mu[t].x, li), rdlane(mu[t].y, li));
        const int sk = __builtin_amdgcn_readlane(sw[t], li);
        const C tmp = csub(xk, cmul(mk, c));
        const C yp = sk ? tmp : c;
        if (!sk) c = tmp;
        // y_{k-1}: row k-1
        if (li > 0) {
          if (lane == li - 1) acc[t] = yp;
        } else if (t > 0) {
          if (lane == 63) acc[t > 0 ? t - 1 : 0] = yp;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < RPL; ++t)
      if (t == (r1 - 1) / 64 && lane == (r1 - 1) % 64) acc[t] = c;
    // ---- output column j, update the right-hand sides of j' < j
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int a = 64 * t + lane;
      if (a < r1) h[a * sa + j * sj + b * sb] = acc[t];
    }
    for (int jp = 0; jp < j; ++jp) {
      const C tj = T[(long)jp * m + j];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        C g = G[(jp * RPL + t) * 64 + lane];
        g = csub(g, cmul(tj, acc[t]));
        G[(jp * RPL + t) * 64 + lane] = g;
      }
    }
  }
}

template <class R>
static void kron_hess_t(hipStream_t s, int r1, int m, int r2, const R* Hc, const typename CxOf<R>::type* T,
                        const typename CxOf<R>::type* lamR, typename CxOf<R>::type* h, long sa, long sj, long sb) {
  using C = typename CxOf<R>::type;
  T2S2_CHECK(r1 >= 1 && m >= 1 && r2 >= 1, "kron_hess_solve: sizes must be positive");
  T2S2_CHECK(kron_hess_fits(r1, m, (int)sizeof(C)), "kron_hess_solve: r1 or m too large for the kernel");
  const int rpl = (r1 + 63) / 64;
  const size_t lds = (size_t)m * rpl * 64 * sizeof(C);
  const double cb = sizeof(C);
  TimedScope ts(s, KC_HESSSOLVE, cb * 2.0 * r1 * m * r2 + sizeof(R) * 0.5 * r1 * r1, 8.0 * r1 * r1 * (double)m * r2);
  switch (rpl) {
    case 1: hipLaunchKernelGGL((kron_hess_kernel<R, 1>), dim3(r2), dim3(64), lds, s, r1, m, r2, Hc, T, lamR, h, sa, sj, sb); break;
    case 2: hipLaunchKernelGGL((kron_hess_kernel<R, 2>), dim3(r2), dim3(64), lds, s, r1, m, r2, Hc, T, lamR, h, sa, sj, sb); break;
    case 3: hipLaunchKernelGGL((kron_hess_kernel<R, 3>), dim3(r2), dim3(64), lds, s, r1, m, r2, Hc, T, lamR, h, sa, sj, sb); break;
    default: hipLaunchKernelGGL((kron_hess_kernel<R, 4>), dim3(r2), dim3(64), lds, s, r1, m, r2, Hc, T, lamR, h, sa, sj, sb); break;
  }
  T2S2_LAUNCH_CHECK();
}

}  // namespace

bool kron_hess_fits(int r1, int m, int cbytes) {
  if (r1 < 1 || r1 > 256 || m < 1) return false;
  const long rpl = (r1 + 63) / 64;
  return (long)m * rpl * 64 * cbytes <= kHessLds;
}

void kron_hess_solve(hipStream_t s, int r1, int m, int r2, const double* Hc, const double2* T, const double2* lamR,
                     double2* h) {
  kron_hess_t<double>(s, r1, m, r2, Hc, T, lamR, h, (long)m * r2, r2, 1);
}
void kron_hess_solve(hipStream_t s, int r1, int m, int r2, const float* Hc, const float2* T, const float2* lamR,
                     float2* h) {
  kron_hess_t<float>(s, r1, m, r2, Hc, T, lamR, h, (long)m * r2, r2, 1);
}
void kron_hess_solve_right(hipStream_t s, int r1, int m, int r2, const double* Hc, const double2* T,
                           const double2* lamL, double2* h) {
  // kernel rows = the Hessenberg index c (stride 1), shifts = the left index
  kron_hess_t<double>(s, r2, m, r1, Hc, T, lamL, h, 1, r2, (long)m * r2);
}

}  // namespace t2s2
