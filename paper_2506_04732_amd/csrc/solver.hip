// Problem set-up, TT building blocks and the alternating TT solver.
//
// Operator (paper: Overview (i)-(iii), Eq. tt-matrix-format): the interior
// collocation system is L = sum_l E_1 x .. x M_l x .. x E_d, a rank-2
// TT-matrix.  The solver works on the equivalent system
//     (x_l E_l^{-1}) L u = (x_l E_l^{-1}) f,   i.e.   (sum_l I x .. K_l .. x I) u = f~,
// K_l = E_l^{-1} M_l: a Kronecker sum, whose Galerkin projections onto
// orthonormal TT bases are again Kronecker sums L_left (+) K_l (+) L_right.
// Every local problem is then solved exactly with eigen-decompositions of the
// two interface matrices and the Schur form of K_l (complex arithmetic),
// followed by FP64 iterative refinement against the real local operator.
//
// Sweeps (the paper's "swaps", Results: Fig. 6) follow one-site AMEn with
// residual enrichment (cited by the paper, not printed): local solve,
// truncated SVD of the new core, enrichment by the residual projected onto
// the far-side basis of an auxiliary rank-kick TT z, QR, interface update.
// The stopping test uses the exact FP64 residual of the original system.
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "ddnorm.h"
#include "kron_hess.h"
#include "spectral_host.h"

namespace t2s2 {

// =============================================================== problem
Problem::~Problem() {
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (auto p : opL.c) fr(p);
  for (auto p : opK.c) fr(p);
  for (auto p : dK) fr(p);
  for (auto p : dEinv) fr(p);
  for (auto p : dEf) fr(p);
  for (auto p : dMf) fr(p);
  for (auto p : dEi) fr(p);
  for (auto p : dMi) fr(p);
  for (auto p : dMx) fr(p);
  for (auto p : dK_ZT) fr(p);
  for (auto p : dK_T) fr(p);
  for (auto p : dK_ZT32) fr(p);
  for (auto p : dK_T32) fr(p);
  for (int k = 0; k < kSides; ++k) {
    if (side[k]) {
      (void)hipStreamSynchronize(side[k]);
      (void)hipStreamDestroy(side[k]);
    }
    if (side_done[k]) (void)hipEventDestroy(side_done[k]);
  }
}

static std::vector<double> host_inverse(int n, std::vector<double> A) {
  std::vector<double> X(n * n, 0.0);
  for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
    if (A[p * n + k] == 0.0) throw Error(1, "singular 1D evaluation matrix");
    if (p != k)
      for (int j = 0; j < n; ++j) {
        std::swap(A[k * n + j], A[p * n + j]);
        std::swap(X[k * n + j], X[p * n + j]);
      }
    const double inv = 1.0 / A[k * n + k];
    for (int j = 0; j < n; ++j) {
      A[k * n + j] *= inv;
      X[k * n + j] *= inv;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = A[i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[i * n + j] -= f * A[k * n + j];
        X[i * n + j] -= f * X[k * n + j];
      }
    }
  }
  return X;
}

template <class T>
static T* dev_alloc(size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw Error(2, "device allocation failed");
  return static_cast<T*>(p);
}

// Rank-2 TT-matrix of sum_l A_1 x .. x B_l x .. x A_d from per-dimension
// (A_l, B_l) blocks: first core [B A], middle [[A 0],[B A]], last [A; B].
static void build_kron_sum(int d, const std::vector<int>& m, const std::vector<std::vector<double>>& Ablk,
                           const std::vector<std::vector<double>>& Bblk, DTTM& out, std::vector<int>& R) {
  out.d = d;
  out.n = m;
  R.assign(d + 1, 2);
  R[0] = R[d] = 1;
  if (d == 1) R[1] = 1;
  out.R = R;
  out.c.resize(d);
  for (int l = 0; l < d; ++l) {
    const int n = m[l], R0 = R[l], R1 = R[l + 1];
    std::vector<double> h((size_t)R0 * n * n * R1, 0.0);
    auto put = [&](int a, int b, const std::vector<double>& blk) {
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) h[(((size_t)a * n + i) * n + j) * R1 + b] = blk[(size_t)i * n + j];
    };
    if (d == 1) {
      put(0, 0, Bblk[l]);
    } else if (l == 0) {
      put(0, 0, Bblk[l]);
      put(0, 1, Ablk[l]);
    } else if (l == d - 1) {
      put(0, 0, Ablk[l]);
      put(1, 0, Bblk[l]);
    } else {
      put(0, 0, Ablk[l]);
      put(1, 0, Bblk[l]);
      put(1, 1, Ablk[l]);
    }
    out.c[l] = dev_alloc<double>(h.size());
    T2S2_HIP(hipMemcpy(out.c[l], h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  }
}

// sum_k c[k] P_k(x), Legendre series by the three-term recurrence
static double legendre_series(const double* c, int nc, double x) {
  double p0 = 1.0, p1 = x, s = c[0];
  if (nc > 1) s += c[1] * x;
  for (int k = 1; k + 1 < nc; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    s += c[k + 1] * p2;
    p0 = p1;
    p1 = p2;
  }
  return s;
}

Problem* problem_create(int d, const int* N, double eps, const double* beta, int scheme, int rank_cap,
                        double rho) {
  T2S2_CHECK(d >= 1 && d <= 16, "d must be in [1, 16]");
  for (int l = 0; l < d; ++l) T2S2_CHECK(std::isfinite(beta[l]), "beta must be finite");
  const std::vector<int> kind(d, 0), nb(d, 1);
  return problem_create_general(d, N, kind.data(), eps, beta, nb.data(), rho, 0.0, scheme, rank_cap);
}

Problem* problem_create_general(int d, const int* N, const int* kind, double eps, const double* beta_coef,
                                const int* nbeta, double rho, double T, int scheme, int rank_cap) {
  T2S2_CHECK(d >= 1 && d <= 16, "d must be in [1, 16]");
  T2S2_CHECK(std::isfinite(eps) && eps > 0.0, "eps must be finite and > 0");
  T2S2_CHECK(std::isfinite(rho), "rho must be finite");
  T2S2_CHECK(scheme == 0 || scheme == 1, "scheme must be 0 (plain) or 1 (superconsistent)");
  T2S2_CHECK(rank_cap >= 1 && rank_cap <= 1024, "rank_cap must be in [1, 1024]");
  bool has_time = false;
  for (int l = 0; l < d; ++l) {
    T2S2_CHECK(kind[l] == 0 || kind[l] == 1, "dimension kind must be 0 (space) or 1 (time)");
    T2S2_CHECK(N[l] >= 3 && N[l] <= 66, "N must be in [3, 66]");
    if (kind[l] == 1) has_time = true;
    else T2S2_CHECK(nbeta[l] >= 1 && nbeta[l] <= 66, "each space dimension needs 1 .. 66 beta coefficients");
  }
  T2S2_CHECK(!has_time || (std::isfinite(T) && T > 0.0), "a time dimension needs a final time T > 0");
  Problem* P = new Problem();
  try {
    P->d = d;
    P->eps = eps;
    P->rho = rho;
    P->scheme = scheme;
    P->rank_cap = rank_cap;
    P->T = has_time ? T : 0.0;
    T2S2_HIP(hipGetDevice(&P->device));
    P->N.assign(N, N + d);
    P->kind.assign(kind, kind + d);
    P->beta.assign(d, 0.0);
    P->m.resize(d);
    std::vector<std::vector<double>> Ieye(d);
    long coff = 0;
    for (int l = 0; l < d; ++l) {
      const int n = N[l] - 1, Nl = N[l];
      const bool time = kind[l] == 1;
      // space: Dirichlet data at both ends, N - 2 unknowns, n - 1 collocation
      // nodes; time (on [0, T]): the value at t = 0 is given, N - 1 unknowns,
      // collocated at the n Gauss points (zeros of P_n)
      const int m = time ? N[l] - 1 : N[l] - 2;
      P->m[l] = m;
      std::vector<double> x = gll_nodes(n);
      std::vector<double> th;
      std::vector<double> bth(m, 0.0);
      if (time) {
        th = gauss_zeros(n);
      } else {
        const double* c = beta_coef + coff;
        coff += nbeta[l];
        for (int k = 0; k < nbeta[l]; ++k) T2S2_CHECK(std::isfinite(c[k]), "beta coefficients must be finite");
        // the node set follows one advection value per dimension: the value
        // of largest magnitude over the GLL nodes, taken positive when beta
        // changes sign there (constant beta: beta itself)
        double bmax = 0.0, bmin = 0.0, bbig = 0.0;
        for (int i = 0; i < Nl; ++i) {
          const double v = legendre_series(c, nbeta[l], x[i]);
          bmax = std::max(bmax, v);
          bmin = std::min(bmin, v);
          if (std::fabs(v) > std::fabs(bbig)) bbig = v;
        }
        const double bnode = (bmax > 0.0 && bmin < 0.0) ? std::max(bmax, -bmin) : bbig;
        P->beta[l] = bnode;
        th = colloc_nodes(n, eps, bnode, scheme);
        for (int j = 0; j < m; ++j) bth[j] = legendre_series(c, nbeta[l], th[j]);
      }
      std::vector<double> Ef((size_t)m * Nl), D1((size_t)m * Nl), D2((size_t)m * Nl);
      lagrange_eval(x.data(), Nl, th.data(), m, Ef.data(), D1.data(), D2.data());
      std::vector<double> E((size_t)m * m), M((size_t)m * m), Mf((size_t)m * Nl);
      // reaction rho u at the collocation nodes is rho (x)E u = sum_l (x)_{k != l} E_k (x) (rho/d) E_l u;
      // time: d/dt = (2 / T) d/ds on [0, T]
      const double rd = rho / d;
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < Nl; ++i) {
          const size_t e = (size_t)j * Nl + i;
          Mf[e] = (time ? (2.0 / T) * D1[e] : -eps * D2[e] + bth[j] * D1[e]) + rd * Ef[e];
        }
      if (time)
        for (auto& t : th) t = 0.5 * T * (t + 1.0);  // reported in physical time
      {
        double* ef = dev_alloc<double>(Ef.size());
        double* mf = dev_alloc<double>(Mf.size());
        P->dEf.push_back(ef);
        P->dMf.push_back(mf);
        T2S2_HIP(hipMemcpy(ef, Ef.data(), Ef.size() * sizeof(double), hipMemcpyHostToDevice));
        T2S2_HIP(hipMemcpy(mf, Mf.data(), Mf.size() * sizeof(double), hipMemcpyHostToDevice));
      }
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
          E[(size_t)j * m + i] = Ef[(size_t)j * Nl + i + 1];
          M[(size_t)j * m + i] = Mf[(size_t)j * Nl + i + 1];
        }
      {
        double* ei = dev_alloc<double>(E.size());
        double* mi = dev_alloc<double>(M.size());
        P->dEi.push_back(ei);
        P->dMi.push_back(mi);
        T2S2_HIP(hipMemcpy(ei, E.data(), E.size() * sizeof(double), hipMemcpyHostToDevice));
        T2S2_HIP(hipMemcpy(mi, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice));
      }
      std::vector<double> Einv = host_inverse(m, E);
      std::vector<double> K((size_t)m * m, 0.0);
      for (int i = 0; i < m; ++i)
        for (int k = 0; k < m; ++k) {
          const double a = Einv[(size_t)i * m + k];
          for (int j = 0; j < m; ++j) K[(size_t)i * m + j] += a * M[(size_t)k * m + j];
        }
      P->gll.push_back(x);
      P->theta.push_back(th);
      P->E.push_back(E);
      P->M.push_back(M);
      P->K.push_back(K);
      P->Einv.push_back(Einv);
      Ieye[l].assign((size_t)m * m, 0.0);
      for (int i = 0; i < m; ++i) Ieye[l][(size_t)i * m + i] = 1.0;
    }
    build_kron_sum(d, P->m, P->E, P->M, P->opL, P->opR);
    std::vector<int> Rk;
    build_kron_sum(d, P->m, Ieye, P->K, P->opK, Rk);
    Ctx c{nullptr, &P->sc};
    c.fail = P->sc.get<int>("ctx.fail", 1);
    clear_fail(c);
    for (int l = 0; l < d; ++l) {
      const int m = P->m[l];
      double* k = dev_alloc<double>((size_t)m * m);
      double* ei = dev_alloc<double>((size_t)m * m);
      T2S2_HIP(hipMemcpy(k, P->K[l].data(), (size_t)m * m * sizeof(double), hipMemcpyHostToDevice));
      T2S2_HIP(hipMemcpy(ei, P->Einv[l].data(), (size_t)m * m * sizeof(double), hipMemcpyHostToDevice));
      P->dK.push_back(k);
      P->dEinv.push_back(ei);
      double2* zt = dev_alloc<double2>((size_t)m * m);
      double2* t = dev_alloc<double2>((size_t)m * m);
      schur_real(c, m, k, zt, t);
      P->dK_ZT.push_back(zt);
      P->dK_T.push_back(t);
      float2* zt32 = dev_alloc<float2>((size_t)m * m);
      float2* t32 = dev_alloc<float2>((size_t)m * m);
      to_float(c.s, reinterpret_cast<const double*>(zt), reinterpret_cast<float*>(zt32), 2L * m * m);
      to_float(c.s, reinterpret_cast<const double*>(t), reinterpret_cast<float*>(t32), 2L * m * m);
      P->dK_ZT32.push_back(zt32);
      P->dK_T32.push_back(t32);
    }
    T2S2_HIP(hipDeviceSynchronize());
    if (read_fail(c)) throw Error(5, "problem set-up: Francis QR of a 1D operator K_l did not converge");
  } catch (...) {
    delete P;
    throw;
  }
  return P;
}

// =============================================================== TT ops
// Device buffer for the permuted operator core (one per host thread, grown
// on demand; the calls of one thread share its stream order).
namespace {
struct CoreWork {
  double* p = nullptr;
  size_t count = 0;
  ~CoreWork() {
    if (p) (void)hipFree(p);
  }
  double* get(size_t n) {
    if (n > count) {
      if (p) T2S2_HIP(hipFree(p));
      p = nullptr;
      count = 0;
      T2S2_HIP(hipMalloc(&p, n * sizeof(double)));
      count = n;
    }
    return p;
  }
};
thread_local CoreWork g_core;
}  // namespace

// Core product Y[(a, p), i', (b, q)] = sum_i A[a, i', i, b] X[p, i, q] as, for
// each a, a GEMM batched over p: Y_p[(i', b), q] = Ahat_a[(i', b), i] X_p[i, q]
// (rows (i', b) of the output are contiguous with stride r1).
// Ah: room for the permuted core (R0 n n R1 doubles); NULL: this thread's
// library-allocated buffer.  timed = false records no events.
static void core_product(const Ctx& c, int R0, int R1, int n, int r0, int r1, const double* A, const double* X,
                         double* Y, double* Ah = nullptr, bool timed = true) {
  const long asz = (long)R0 * n * n * R1;
  TimedScope ts(c.s, KC_TTMV, 8.0 * ((double)r0 * n * r1 + (double)asz + (double)R0 * r0 * n * R1 * r1),
                2.0 * (double)R0 * R1 * n * n * r0 * r1, timed);
  if (!Ah) Ah = g_core.get((size_t)asz);
  ttm_permute(c.s, R0, R1, n, A, Ah);
  const long co = (long)R1 * r1;
  // K = n <= 64: never split-K, so the GEMM uses no workspace
  for (int a = 0; a < R0; ++a)
    gemm<double>(c.s, OpN, OpN, n * R1, r1, n, 1.0, Ah + (long)a * n * R1 * n, n, 0, X, r1, (long)n * r1, 0.0,
                 Y + (long)a * r0 * n * co, r1, (long)n * co, r0, false);
}

void tt_matvec(const Ctx& c, const DTTM& A, const DTT& x, DTT& y) {
  T2S2_CHECK(A.d == x.d, "tt_matvec: dimension mismatch");
  y.d = x.d;
  y.n = x.n;
  y.r.assign(x.d + 1, 1);
  for (int l = 0; l <= x.d; ++l) y.r[l] = A.R[l] * x.r[l];
  for (int l = 0; l < x.d; ++l) {
    T2S2_CHECK(A.n[l] == x.n[l], "tt_matvec: mode size mismatch");
    core_product(c, A.R[l], A.R[l + 1], x.n[l], x.r[l], x.r[l + 1], A.c[l], x.c[l], y.c[l]);
  }
}

// ---- TT-matvec without allocation ------------------------------------------
// The permuted operator core lives in `scratch`, a file-scope device array:
// one copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in): its device
// address is taken once per device with hipGetSymbolAddress and kept.
constexpr long kNoAllocDoubles = 1L << 17;  // 1 MiB: R0 n n R1 <= 131072 per core
static __device__ __align__(256) double scratch[kNoAllocDoubles];
constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[kNoAllocMaxDevices] = {};

static double* noalloc_scratch() {
  int dev = 0;
  T2S2_HIP(hipGetDevice(&dev));
  T2S2_CHECK(dev >= 0 && dev < kNoAllocMaxDevices, "tt_matvec_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    T2S2_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    T2S2_CHECK(ptr != nullptr, "tt_matvec_noalloc: no device address for the scratch array");
    g_noalloc_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_noalloc_ptr[dev];
}

long tt_matvec_noalloc_capacity() { return kNoAllocDoubles; }

void tt_matvec_noalloc(const Ctx& c, const DTTM& A, const DTT& x, DTT& y) {
  T2S2_CHECK(A.d == x.d, "tt_matvec: dimension mismatch");
  for (int l = 0; l < x.d; ++l) {
    T2S2_CHECK(A.n[l] == x.n[l] && A.n[l] <= 64, "tt_matvec: mode sizes must match, <= 64");
    const long asz = (long)A.R[l] * A.n[l] * A.n[l] * A.R[l + 1];
    T2S2_CHECK(asz <= kNoAllocDoubles, "tt_matvec_noalloc: operator core " + std::to_string(l) + " needs " +
                                           std::to_string(asz) + " doubles of scratch, more than the " +
                                           std::to_string(kNoAllocDoubles) + " available");
  }
  double* ws = noalloc_scratch();
  y.d = x.d;
  y.n = x.n;
  y.r.assign(x.d + 1, 1);
  for (int l = 0; l <= x.d; ++l) y.r[l] = A.R[l] * x.r[l];
  for (int l = 0; l < x.d; ++l)
    core_product(c, A.R[l], A.R[l + 1], x.n[l], x.r[l], x.r[l + 1], A.c[l], x.c[l], y.c[l], ws, false);
}

double tt_norm(const Ctx& c, const DTT& x) { return tt_norm_dd(c, x); }

double tt_residual_norm(Problem& p, const Ctx& c, const DTT& x, const DTT& f) {
  const int d = x.d;
  T2S2_CHECK(f.d == d, "residual: dimension mismatch");
  // y = L x in scratch
  DTT y;
  y.d = d;
  y.n = x.n;
  y.r.resize(d + 1);
  y.c.resize(d);
  for (int l = 0; l < d; ++l)
    y.c[l] = c.sc->get<double>("res.y" + std::to_string(l),
                               (size_t)p.opL.R[l] * x.r[l] * x.n[l] * p.opL.R[l + 1] * x.r[l + 1]);
  tt_matvec(c, p.opL, x, y);
  // r = f - y by concatenation
  DTT r;
  r.d = d;
  r.n = x.n;
  r.r.resize(d + 1);
  r.c.resize(d);
  r.r[0] = r.r[d] = 1;
  for (int l = 1; l < d; ++l) r.r[l] = f.r[l] + y.r[l];
  for (int l = 0; l < d; ++l) {
    const int n = x.n[l];
    const size_t sz = (size_t)r.r[l] * n * r.r[l + 1];
    r.c[l] = c.sc->get<double>("res.r" + std::to_string(l), sz);
    if (d == 1) {
      c.d2d(r.c[l], f.c[l], (size_t)n);
      axpby(c.s, n, -1.0, y.c[l], 1.0, r.c[l]);
      continue;
    }
    fill(c.s, r.c[l], (long)sz, 0.0);
    const int fr0 = f.r[l], fr1 = f.r[l + 1], yr0 = y.r[l], yr1 = y.r[l + 1];
    const long ld = r.r[l + 1];
    if (l == 0) {
      copy2d(c.s, n, fr1, f.c[l], fr1, r.c[l], ld);
      copy2d(c.s, n, yr1, y.c[l], yr1, r.c[l] + fr1, ld, -1.0);
    } else if (l == d - 1) {
      copy2d(c.s, (long)fr0 * n, 1, f.c[l], 1, r.c[l], 1);
      copy2d(c.s, (long)yr0 * n, 1, y.c[l], 1, r.c[l] + (long)fr0 * n, 1);
    } else {
      copy2d(c.s, (long)fr0 * n, fr1, f.c[l], fr1, r.c[l], ld);
      copy2d(c.s, (long)yr0 * n, yr1, y.c[l], yr1, r.c[l] + (long)fr0 * n * ld + fr1, ld);
    }
  }
  // norms by the double-double Gram recursion: f and L x cancel to the
  // residual level, which FP64 orthogonalisation cannot resolve
  const double rn = tt_norm_dd(c, r);
  const double fn = tt_norm_dd(c, f);
  T2S2_CHECK(fn > 0.0 && std::isfinite(fn), "residual: ||f|| must be finite and > 0");
  return rn / fn;
}

void tt_round(const Ctx& c, DTT& x, double tol, int rmax) {
  const int d = x.d;
  if (d == 1) return;
  // right-to-left orthogonalisation (in place, ranks never grow)
  for (int l = d - 1; l >= 1; --l) {
    const int r0 = x.r[l], n = x.n[l], r1 = x.r[l + 1];
    const int M = n * r1;  // rows of the transposed unfolding
    double* At = c.sc->get<double>("rnd.At", (size_t)M * r0);
    transpose(c.s, r0, M, x.c[l], M, At, r0);
    const int kmax = std::min(M, r0);
    double* Q = c.sc->get<double>("rnd.Q", (size_t)M * kmax);
    double* R = c.sc->get<double>("rnd.R", (size_t)kmax * r0);
    int k = dcholqr(c, M, r0, At, r0, Q, R, 1e-15);
    if (k == 0) k = 1, fill(c.s, Q, M, 0.0), fill(c.s, R, r0, 0.0);
    transpose(c.s, M, k, Q, k, x.c[l], M);  // core = Q^T (k x n r1)
    const int rp = x.r[l - 1], np = x.n[l - 1];
    double* T = c.sc->get<double>("rnd.T", (size_t)rp * np * k);
    mode3<double>(c, rp, np, r0, k, x.c[l - 1], R, T, 0.0);  // core_{l-1} x3 R
    c.d2d(x.c[l - 1], T, (size_t)rp * np * k);
    x.r[l] = k;
  }
  const double nrm = c.nrm2(x.c[0], (long)x.n[0] * x.r[1]);
  const double delta = tol * nrm / std::sqrt((double)(d - 1));
  for (int l = 0; l + 1 < d; ++l) {
    const int r0 = x.r[l], n = x.n[l], r1 = x.r[l + 1];
    const int M = r0 * n;
    const int kmax = std::min(M, r1);
    double* U = c.sc->get<double>("rnd.U", (size_t)M * kmax);
    double* W = c.sc->get<double>("rnd.W", (size_t)kmax * r1);
    const int r = trunc_svd(c, M, r1, x.c[l], r1, delta, rmax, U, W);
    c.d2d(x.c[l], U, (size_t)M * r);
    const int n1 = x.n[l + 1], r2 = x.r[l + 2];
    double* T = c.sc->get<double>("rnd.T", (size_t)r * n1 * r2);
    mode1<double>(c, r, r1, n1, r2, W, x.c[l + 1], T, 0.0);
    c.d2d(x.c[l + 1], T, (size_t)r * n1 * r2);
    x.r[l + 1] = r;
  }
}

// sum_k coef[k] parts[k] by concatenation (ranks add); out's cores are
// scratch named prefix + l, out.r written
static void tt_concat(const Ctx& c, const std::vector<const DTT*>& parts, const std::vector<double>& coef,
                      const std::string& prefix, DTT& out) {
  const int d = parts[0]->d;
  out.d = d;
  out.n = parts[0]->n;
  out.r.assign(d + 1, 1);
  out.c.resize(d);
  for (int l = 1; l < d; ++l) {
    out.r[l] = 0;
    for (auto* t : parts) out.r[l] += t->r[l];
  }
  for (int l = 0; l < d; ++l) {
    const int n = out.n[l];
    const long sz = (long)out.r[l] * n * out.r[l + 1];
    out.c[l] = c.sc->get<double>(prefix + std::to_string(l), (size_t)sz);
    fill(c.s, out.c[l], sz, 0.0);
    if (d == 1) {
      for (size_t k = 0; k < parts.size(); ++k) axpby(c.s, n, coef[k], parts[k]->c[0], 1.0, out.c[0]);
      continue;
    }
    long o0 = 0, o1 = 0;
    const long ld = out.r[l + 1];
    for (size_t k = 0; k < parts.size(); ++k) {
      const DTT& t = *parts[k];
      const int a0 = t.r[l], a1 = t.r[l + 1];
      if (l == 0) {
        copy2d(c.s, n, a1, t.c[l], a1, out.c[l] + o1, ld, coef[k]);
      } else if (l == d - 1) {
        copy2d(c.s, (long)a0 * n, 1, t.c[l], 1, out.c[l] + o0 * n, 1);
      } else {
        copy2d(c.s, (long)a0 * n, a1, t.c[l], a1, out.c[l] + o0 * n * ld + o1, ld);
      }
      o0 += a0;
      o1 += a1;
    }
  }
}

// y = (sum_l A_1 x .. x B_l x .. x A_d) x with per-dimension blocks A_l (E),
// B_l (M) of mo_l rows and mi_l columns (leading dimension mi_l), applied to
// mode indices off .. off + mi_l - 1 of x's cores (x's mode sizes nx_l): the
// rank-2 Kronecker-sum TT-matrix, block by block (one strided GEMM each)
static void kron_sum_apply(const Ctx& c, const std::vector<int>& mo, const std::vector<int>& mi, int off,
                           const std::vector<double*>& A, const std::vector<double*>& B, const DTT& x,
                           const std::string& prefix, DTT& y) {
  const int d = x.d;
  y.d = d;
  y.n = mo;
  y.r.assign(d + 1, 1);
  y.c.resize(d);
  for (int l = 1; l < d; ++l) y.r[l] = 2 * x.r[l];
  for (int l = 0; l < d; ++l) {
    const int R0 = (l == 0) ? 1 : 2, R1 = (l == d - 1) ? 1 : 2;
    const int r0 = x.r[l], r1 = x.r[l + 1], nx = x.n[l];
    const long sz = (long)R0 * r0 * mo[l] * R1 * r1;
    y.c[l] = c.sc->get<double>(prefix + std::to_string(l), (size_t)sz);
    fill(c.s, y.c[l], sz, 0.0);
    auto block = [&](int a, int b, const double* Blk) {
      gemm<double>(c.s, OpN, OpN, mo[l], r1, mi[l], 1.0, Blk, mi[l], 0, x.c[l] + (long)off * r1, r1, (long)nx * r1,
                   0.0, y.c[l] + (long)a * r0 * mo[l] * R1 * r1 + (long)b * r1, (long)R1 * r1,
                   (long)mo[l] * R1 * r1, r0);
    };
    if (d == 1) {
      block(0, 0, B[l]);
    } else if (l == 0) {
      block(0, 0, B[l]);
      block(0, 1, A[l]);
    } else if (l == d - 1) {
      block(0, 0, A[l]);
      block(1, 0, B[l]);
    } else {
      block(0, 0, A[l]);
      block(1, 0, B[l]);
      block(1, 1, A[l]);
    }
  }
}

void lift_rhs(Problem& p, const Ctx& c, const DTT& f, const DTT& g, DTT& b, int rmax) {
  const int d = p.d;
  T2S2_CHECK(f.d == d && g.d == d, "lift: dimension mismatch");
  for (int l = 0; l < d; ++l) {
    T2S2_CHECK(f.n[l] == p.m[l], "lift: f mode sizes must be N_l - 2");
    T2S2_CHECK(g.n[l] == p.N[l], "lift: g mode sizes must be N_l (GLL grid)");
  }
  DTT y1, y2;
  kron_sum_apply(c, p.m, p.N, 0, p.dEf, p.dMf, g, "lift.y1_", y1);   // L_full g
  kron_sum_apply(c, p.m, p.m, 1, p.dEi, p.dMi, g, "lift.y2_", y2);   // L_int g_int
  tt_concat(c, {&f, &y1, &y2}, {1.0, -1.0, 1.0}, "lift.b", b);
  tt_round(c, b, 1e-14, std::max(1, rmax));
}

Problem* mol_create(int d, const int* N, double eps, const double* beta, double rho, double dt, double theta,
                    int scheme, int rank_cap) {
  T2S2_CHECK(std::isfinite(dt) && dt > 0.0, "dt must be finite and > 0");
  T2S2_CHECK(std::isfinite(theta) && theta > 0.0 && theta <= 1.0, "theta must be in (0, 1]");
  T2S2_CHECK(std::isfinite(rho), "rho must be finite");
  const double cE = 1.0 / (theta * dt), cL = (1.0 - theta) / theta;
  Problem* P = problem_create(d, N, eps, beta, scheme, rank_cap, rho + cE);
  try {
    P->mol_dt = dt;
    P->mol_theta = theta;
    P->rho_phys = rho;
    for (int l = 0; l < d; ++l) {
      const int m = P->m[l];
      // M_l holds M0_l + (rho + cE)/d E_l; the explicit blocks are
      // cE/d E_l - cL (M0_l + rho/d E_l) = (cE/d - cL rho/d) E_l - cL M0_l
      //                                  = (cE/d + cL cE/d) E_l - cL M_l
      std::vector<double> X((size_t)m * m);
      const double a = (cE + cL * cE) / d;
      for (size_t e = 0; e < X.size(); ++e) X[e] = a * P->E[l][e] - cL * P->M[l][e];
      double* dx = dev_alloc<double>(X.size());
      P->dMx.push_back(dx);
      T2S2_HIP(hipMemcpy(dx, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  } catch (...) {
    delete P;
    throw;
  }
  return P;
}

// out[i] = x(idx_0, .., idx_{l-1}, i, idx_{l+1}, ..) for i < n_l: the row
// vector of the slices left of l, the column vector of those right of l
// (chains of slice products), then v X_l(:, i, :) w for every i
void tt_fiber(const Ctx& c, const DTT& x, int l, const std::vector<int>& idx, double* out) {
  const int d = x.d;
  T2S2_CHECK(l >= 0 && l < d && (int)idx.size() == d, "tt_fiber: bad mode or index count");
  for (int k = 0; k < d; ++k) T2S2_CHECK(k == l || (idx[k] >= 0 && idx[k] < x.n[k]), "tt_fiber: index out of range");
  int rmax = 1;
  for (int k = 0; k <= d; ++k) rmax = std::max(rmax, x.r[k]);
  double* v = c.sc->get<double>("fib.v", (size_t)rmax);
  double* v2 = c.sc->get<double>("fib.v2", (size_t)rmax);
  double* w = c.sc->get<double>("fib.w", (size_t)rmax);
  double* w2 = c.sc->get<double>("fib.w2", (size_t)rmax);
  double* Z = c.sc->get<double>("fib.Z", (size_t)rmax * x.n[l]);
  const double one = 1.0;
  c.h2d(v, &one, 1);
  c.h2d(w, &one, 1);
  for (int k = 0; k < l; ++k) {
    // v (1 x r_k) <- v X_k(:, idx_k, :): rows a of the slice at stride n_k r_{k+1}
    const int r0 = x.r[k], n = x.n[k], r1 = x.r[k + 1];
    gemm<double>(c.s, OpN, OpN, 1, r1, r0, 1.0, v, r0, 0, x.c[k] + (long)idx[k] * r1, (long)n * r1, 0, 0.0, v2, r1,
                 0, 1);
    std::swap(v, v2);
  }
  for (int k = d - 1; k > l; --k) {
    // w (r_{k+1}) <- X_k(:, idx_k, :) w
    const int r0 = x.r[k], n = x.n[k], r1 = x.r[k + 1];
    gemm<double>(c.s, OpN, OpN, r0, 1, r1, 1.0, x.c[k] + (long)idx[k] * r1, (long)n * r1, 0, w, 1, 0, 0.0, w2, 1,
                 0, 1);
    std::swap(w, w2);
  }
  const int r0 = x.r[l], n = x.n[l], r1 = x.r[l + 1];
  gemm<double>(c.s, OpN, OpN, r0 * n, 1, r1, 1.0, x.c[l], r1, 0, w, 1, 0, 0.0, Z, 1, 0, 1);   // Z[a][i]
  gemm<double>(c.s, OpN, OpN, 1, n, r0, 1.0, v, r0, 0, Z, n, 0, 0.0, out, n, 0, 1);
}

// ================================================================ solver
namespace {

// Device time per solve phase: an event on the solve's stream at every phase
// change; the time between two events is charged to the earlier phase.
struct PhaseClock {
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> ph;
  size_t used = 0;
  ~PhaseClock() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  void mark(int phase) {
    if (used == ev.size()) {
      hipEvent_t e;
      T2S2_HIP(hipEventCreate(&e));
      ev.push_back(e);
      ph.push_back(0);
    }
    T2S2_HIP(hipEventRecord(ev[used], s));
    ph[used] = phase;
    ++used;
  }
  // after the stream has completed every marked event
  void collect(double* out) {
    for (size_t i = 0; i + 1 < used; ++i) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) out[ph[i]] += ms;
    }
  }
};

// Interface factorisation L = V diag(lam) V^{-1} (complex), FP64 or FP32.
template <class C>
struct EigT {
  C* lam = nullptr;
  C* V = nullptr;
  C* Vi = nullptr;
};
using Eig = EigT<double2>;
using Eig32 = EigT<float2>;

template <class C>
inline C cx_zero() {
  C z;
  z.x = 0;
  z.y = 0;
  return z;
}

// out = (L (+) K (+) R)^{-1} g on r1 x ml x r2 tensors (real in, real out),
// L = VL diag(lamL) VL^{-1}, K = Z T Z^H (ZT = Z^T), R = VR diag(lamR) VR^{-1}:
// mode transforms into the eigen/Schur bases, the triangular Kronecker-sum
// solve along the mode index, transforms back; w0, w1: complex work of size
// r1 ml r2
template <class C>
void kron_inverse_eig(const Ctx& c, int r1, int ml, int r2, const C* ZT, const C* T, const EigT<C>& eL,
                      const EigT<C>& eR, const double* g, double* out, C* w0, C* w1) {
  const long n = (long)r1 * ml * r2;
  const C z0 = cx_zero<C>();
  real_to_complex(c.s, g, w0, n);
  mode3<C>(c, r1, ml, r2, r2, w0, eR.Vi, w1, z0);
  mode2<C>(c, r1, ml, ml, r2, ZT, w1, w0, z0, OpR);
  mode1<C>(c, r1, r1, ml, r2, eL.Vi, w0, w1, z0);
  kron_trisolve(c.s, r1, ml, r2, T, eL.lam, eR.lam, w1);
  mode1<C>(c, r1, r1, ml, r2, eL.V, w1, w0, z0);
  mode2<C>(c, r1, ml, ml, r2, ZT, w0, w1, z0, OpT);
  mode3<C>(c, r1, ml, r2, r2, w1, eR.V, w0, z0);
  complex_real_part(c.s, w0, out, n);
}

// The same inverse with L = Q H Q^T (QT = Q^T row-major, Hc = H column-major,
// H upper Hessenberg): Q^T on the real data, the mode-2/3 transforms, one
// Hessenberg-Schur chain per right eigenvalue, back again; wr: real work of
// size r1 ml r2
template <class C, class R>
void kron_inverse_hess(const Ctx& c, int r1, int ml, int r2, const C* ZT, const C* T, const double* QT, const R* Hc,
                       const EigT<C>& eR, const double* g, double* out, C* w0, C* w1, double* wr) {
  const long n = (long)r1 * ml * r2;
  const C z0 = cx_zero<C>();
  mode1<double>(c, r1, r1, ml, r2, QT, g, wr, 0.0);
  real_to_complex(c.s, wr, w0, n);
  mode3<C>(c, r1, ml, r2, r2, w0, eR.Vi, w1, z0);
  mode2<C>(c, r1, ml, ml, r2, ZT, w1, w0, z0, OpR);
  kron_hess_solve(c.s, r1, ml, r2, Hc, T, eR.lam, w0);
  mode2<C>(c, r1, ml, ml, r2, ZT, w0, w1, z0, OpT);
  mode3<C>(c, r1, ml, r2, r2, w1, eR.V, w0, z0);
  complex_real_part(c.s, w0, wr, n);
  mode1<double>(c, r1, r1, ml, r2, QT, wr, out, 0.0, OpT);
}

// The same inverse with the right interface R = Q H Q^T (QT = Q^T row-major,
// Hc = H column-major) and the left one L = VL diag(lamL) VL^{-1}: Q^T on the
// real data along mode 3, the mode-1/2 transforms, one Hessenberg-Schur chain
// per left eigenvalue, back again
void kron_inverse_hess_right(const Ctx& c, int r1, int ml, int r2, const double2* ZT, const double2* T,
                             const Eig& eL, const double* QT, const double* Hc, const double* g, double* out,
                             double2* w0, double2* w1, double* wr) {
  const long n = (long)r1 * ml * r2;
  const double2 z0 = cx_zero<double2>();
  mode3<double>(c, r1, ml, r2, r2, g, QT, wr, 0.0);
  real_to_complex(c.s, wr, w0, n);
  mode1<double2>(c, r1, r1, ml, r2, eL.Vi, w0, w1, z0);
  mode2<double2>(c, r1, ml, ml, r2, ZT, w1, w0, z0, OpR);
  kron_hess_solve_right(c.s, r1, ml, r2, Hc, T, eL.lam, w0);
  mode2<double2>(c, r1, ml, ml, r2, ZT, w0, w1, z0, OpT);
  mode1<double2>(c, r1, r1, ml, r2, eL.V, w1, w0, z0);
  complex_real_part(c.s, w0, wr, n);
  mode3<double>(c, r1, ml, r2, r2, wr, QT, out, 0.0, OpN);
}

struct Amen {
  Problem& p;
  const Ctx& c;
  SolveOptions o;
  int d, cap, kick, smax;
  std::vector<int> m;
  // interfaces per bond position 0..d (matrices in row-major, [test][trial])
  std::vector<double*> L, XB, ZXI, ZXL, ZB;
  std::vector<Eig> eig;
  std::vector<Eig32> eig32;       // mixed precision: FP32 factors per bond
  std::vector<char> ok64;         // eig[pos] holds the factors of the current L[pos]
  std::vector<char> ok32;         // eig32[pos] holds the FP32 factors of the current L[pos]
  std::vector<char> need64;       // mixed: bond pos needed FP64 factors once, keep them
  // left interfaces in Hessenberg form L = Q H Q^T: the local solve then
  // needs no eigendecomposition of L (Hessenberg-Schur chain per right
  // eigenvalue); QT = Q^T row-major, Hc = H column-major, Hc32 its FP32 copy
  struct HessF {
    double* QT = nullptr;
    double* Hc = nullptr;
    float* Hc32 = nullptr;
  };
  std::vector<HessF> hf;
  std::vector<char> lhess;        // L[pos] is held as HessF (else as eig / eig32)
  bool mixed = false;
  PhaseClock pc;
  // FP64 overlap mode: each new interface is reduced to Hessenberg form on
  // the solve's stream (the next local solve needs it at once) and
  // eigendecomposed on one of the problem's side streams (only the opposite
  // sweep needs that form), so Francis QR leaves the sweep's critical path
  bool overlap = false;
  Ctx cs[Problem::kSides];             // side-stream contexts
  int next_side = 0;
  std::vector<hipEvent_t> ev_eig;      // per bond: its eigendecomposition is done
  hipEvent_t ev_main = nullptr;        // the interface an eigendecomposition reads is ready
  std::vector<char> eig_pending;       // ev_eig recorded, the solve's stream has not waited yet
  std::vector<char> has_eig, has_hess; // forms held for the current interface of each bond
  enum { M_HL = 0, M_HR = 1, M_EIG = 2 };
  std::vector<int> xr, zr, sr;  // ranks of x, z, f~ per bond
  std::vector<double*> xc, zc, bc;  // cores
  std::vector<int> maxrank;     // structural bound per bond
  // work
  double *u, *f, *res, *y, *T1, *T2, *A1, *S, *kick_buf, *zbuf, *U, *W, *tmp, *Qk, *Rk;
  double* cond = nullptr;  // per bond: largest ||V||_F ||V^-1||_F seen (device)
  double2 *h0, *h1;
  float2 *g0, *g1;
  double* hr;

  Amen(Problem& p_, const Ctx& c_, const SolveOptions& o_) : p(p_), c(c_), o(o_) {}
  ~Amen() {
    // side work may still run: the next solve on this problem waits for it
    if (overlap)
      for (int k = 0; k < Problem::kSides; ++k)
        if (cs[k].s) (void)hipEventRecord(p.side_done[k], cs[k].s);
    for (auto e : ev_eig)
      if (e) (void)hipEventDestroy(e);
    if (ev_main) (void)hipEventDestroy(ev_main);
  }

  // ---- overlap mode -------------------------------------------------------
  // Hessenberg form of the interface at bond pos for the local solves of site
  // `site` (false if the chain kernel cannot take it)
  bool hess_into(int pos, int n, int site) {
    if (site < 0 || site >= d || !kron_hess_fits(n, m[site], (int)sizeof(double2))) return false;
    double* Hw = buf("hess.H", (size_t)n * n);
    c.d2d(Hw, L[pos], (size_t)n * n);
    hessenberg(c, n, Hw, hf[pos].QT);
    transpose(c.s, n, n, Hw, n, hf[pos].Hc, n);
    return true;
  }
  // eigendecomposition of the interface at bond pos on a side stream (from
  // its Hessenberg form when it has one)
  void eig_async(int pos, int n) {
    const Ctx& x = cs[next_side];
    next_side = (next_side + 1) % Problem::kSides;
    T2S2_HIP(hipEventRecord(ev_main, c.s));
    T2S2_HIP(hipStreamWaitEvent(x.s, ev_main, 0));
    if (has_hess[pos])
      eig_from_hessenberg(x, n, hf[pos].Hc, hf[pos].QT, eig[pos].lam, eig[pos].V, eig[pos].Vi);
    else
      eig_nonsym(x, n, L[pos], eig[pos].lam, eig[pos].V, eig[pos].Vi);
    cond_estimate(x, n, eig[pos].V, eig[pos].Vi, cond + pos);
    T2S2_HIP(hipEventRecord(ev_eig[pos], x.s));
    eig_pending[pos] = 1;
    has_eig[pos] = 1;
  }
  void wait_eig(int pos) {
    if (!eig_pending[pos]) return;
    T2S2_HIP(hipStreamWaitEvent(c.s, ev_eig[pos], 0));
    eig_pending[pos] = 0;
  }
  void need_eig(int pos, int n) {
    if (has_eig[pos]) {
      wait_eig(pos);
      return;
    }
    eig_nonsym(c, n, L[pos], eig[pos].lam, eig[pos].V, eig[pos].Vi);
    cond_estimate(c, n, eig[pos].V, eig[pos].Vi, cond + pos);
    has_eig[pos] = 1;
  }
  // a new interface at bond pos (size n), left or right of the sites that use
  // it next; hess: reduce it now (the next site needs it)
  void new_interface(int pos, int n, bool left, bool hess) {
    has_hess[pos] = hess && hess_into(pos, n, left ? pos : pos - 1);
    has_eig[pos] = 0;
    // the opposite sweep uses the eigendecomposition, except of the left
    // interface at bond d-1 (site d-1 is solved with its Hessenberg form)
    if (left && pos == d - 1 && has_hess[pos]) return;
    if (has_hess[pos] || !hess) eig_async(pos, n);
    else need_eig(pos, n);
  }
  // form of the local solve at site l going in direction dir
  int pick_mode(int l, int dir, int r1, int r2) {
    const bool fwd = dir > 0 || l == d - 1;
    if (fwd && has_hess[l]) {
      need_eig(l + 1, r2);
      return M_HL;
    }
    if (!fwd && has_hess[l + 1]) {
      need_eig(l, r1);
      return M_HR;
    }
    need_eig(l, r1);
    need_eig(l + 1, r2);
    return M_EIG;
  }
  void local_solve_ov(int mode, int l, int r1, int r2, const double* g, double* out) {
    if (mode == M_HL)
      kron_inverse_hess<double2, double>(c, r1, m[l], r2, p.dK_ZT[l], p.dK_T[l], hf[l].QT, hf[l].Hc, eig[l + 1], g,
                                         out, h0, h1, hr);
    else if (mode == M_HR)
      kron_inverse_hess_right(c, r1, m[l], r2, p.dK_ZT[l], p.dK_T[l], eig[l], hf[l + 1].QT, hf[l + 1].Hc, g, out,
                              h0, h1, hr);
    else
      kron_inverse_eig<double2>(c, r1, m[l], r2, p.dK_ZT[l], p.dK_T[l], eig[l], eig[l + 1], g, out, h0, h1);
  }

  double* buf(const std::string& n, size_t cnt) { return c.sc->get<double>("am." + n, cnt); }

  void local_apply(int l, int r1, int r2, const double* LL, const double* LR, const double* x, double* out) {
    const int ml = m[l];
    mode1<double>(c, r1, r1, ml, r2, LL, x, out, 0.0);
    mode2<double>(c, r1, ml, ml, r2, p.dK[l], x, out, 1.0);
    mode3<double>(c, r1, ml, r2, r2, x, LR, out, 1.0);
  }

  // out = B^{-1} g for B = L_L (+) K_l (+) L_R via the eigen/Schur factors
  // out = B^{-1} g for B = L_L (+) K_l (+) L_R with the FP64 factors
  void local_solve(int l, int r1, int r2, const Eig& eL, const Eig& eR, const double* g, double* out) {
    if (lhess[l])
      kron_inverse_hess<double2, double>(c, r1, m[l], r2, p.dK_ZT[l], p.dK_T[l], hf[l].QT, hf[l].Hc, eR, g, out, h0,
                                         h1, hr);
    else
      kron_inverse_eig<double2>(c, r1, m[l], r2, p.dK_ZT[l], p.dK_T[l], eL, eR, g, out, h0, h1);
  }

  // same solve with the FP32 factors (FP64 in, FP64 out; the orthogonal
  // Hessenberg transform stays FP64)
  void local_solve32(int l, int r1, int r2, const Eig32& eL, const Eig32& eR, const double* g, double* out) {
    if (lhess[l])
      kron_inverse_hess<float2, float>(c, r1, m[l], r2, p.dK_ZT32[l], p.dK_T32[l], hf[l].QT, hf[l].Hc32, eR, g, out,
                                       g0, g1, hr);
    else
      kron_inverse_eig<float2>(c, r1, m[l], r2, p.dK_ZT32[l], p.dK_T32[l], eL, eR, g, out, g0, g1);
  }

  // factorise a left interface at bond pos (size n): Hessenberg form when the
  // chain kernel supports the local system of site pos, else as factor()
  void factor_left(int pos, int n) {
    if (!(pos < d && kron_hess_fits(n, m[pos], (int)sizeof(double2)))) {
      factor(pos, n);
      return;
    }
    double* Hw = buf("hess.H", (size_t)n * n);
    c.d2d(Hw, L[pos], (size_t)n * n);
    hessenberg(c, n, Hw, hf[pos].QT);
    transpose(c.s, n, n, Hw, n, hf[pos].Hc, n);
    if (mixed) to_float(c.s, hf[pos].Hc, hf[pos].Hc32, (long)n * n);
    lhess[pos] = 1;
    ok64[pos] = 1;
    ok32[pos] = 1;
  }

  // factorise the interface at bond pos (size n) in the working precision
  void factor(int pos, int n) {
    lhess[pos] = 0;
    if (mixed && !need64[pos]) {
      eig_nonsym(c, n, L[pos], eig32[pos].lam, eig32[pos].V, eig32[pos].Vi);
      ok32[pos] = 1;
      ok64[pos] = 0;
    } else {
      eig_nonsym(c, n, L[pos], eig[pos].lam, eig[pos].V, eig[pos].Vi);
      cond_estimate(c, n, eig[pos].V, eig[pos].Vi, cond + pos);
      ok64[pos] = 1;
      ok32[pos] = 0;
    }
  }
  void ensure64(int pos, int n) {
    if (!lhess[pos] && !ok64[pos]) {
      eig_nonsym(c, n, L[pos], eig[pos].lam, eig[pos].V, eig[pos].Vi);
      cond_estimate(c, n, eig[pos].V, eig[pos].Vi, cond + pos);
      ok64[pos] = 1;
    }
  }

  void set_boundary(int pos) {
    // 1 x 1 interfaces: L = 0, XB = 1, ZXI = 1, ZXL = 0, ZB = 1
    const double zero = 0.0, one = 1.0;
    c.h2d(L[pos], &zero, 1);
    c.h2d(XB[pos], &one, 1);
    c.h2d(ZXI[pos], &one, 1);
    c.h2d(ZXL[pos], &zero, 1);
    c.h2d(ZB[pos], &one, 1);
    const double2 z = make_double2(0.0, 0.0), o1 = make_double2(1.0, 0.0);
    c.h2d(eig[pos].lam, &z, 1);
    c.h2d(eig[pos].V, &o1, 1);
    c.h2d(eig[pos].Vi, &o1, 1);
    const float2 zf = make_float2(0.0f, 0.0f), of = make_float2(1.0f, 0.0f);
    c.h2d(eig32[pos].lam, &zf, 1);
    c.h2d(eig32[pos].V, &of, 1);
    c.h2d(eig32[pos].Vi, &of, 1);
    ok64[pos] = 1;
    ok32[pos] = 1;
    // left boundary: also as a (trivial) Hessenberg factor H = 0, Q = 1
    lhess[pos] = 0;
    if (pos == 0 && kron_hess_fits(1, m[0], (int)sizeof(double2))) {
      const float zf1 = 0.0f;
      c.h2d(hf[pos].QT, &one, 1);
      c.h2d(hf[pos].Hc, &zero, 1);
      c.h2d(hf[pos].Hc32, &zf1, 1);
      lhess[pos] = 1;
    }
    has_eig[pos] = 1;
    has_hess[pos] = lhess[pos];
    eig_pending[pos] = 0;
    c.sync();
  }

  // ---- interface updates ------------------------------------------------
  // left interfaces at pos l+1 from pos l and cores x_l (r0 x m x r1), z_l (q0 x m x q1)
  void update_left(int l) {
    const int r0 = xr[l], r1 = xr[l + 1], q0 = zr[l], q1 = zr[l + 1], s0 = sr[l], s1 = sr[l + 1], ml = m[l];
    const double* X = xc[l];
    const double* Z = zc[l];
    if (overlap) wait_eig(l + 1);  // the side stream may still read L[l+1]
    // L' = X^T (L x1 X + K x2 X)
    mode1<double>(c, r0, r0, ml, r1, L[l], X, T1, 0.0);
    mode2<double>(c, r0, ml, ml, r1, p.dK[l], X, T1, 1.0);
    gemm<double>(c.s, OpT, OpN, r1, r1, r0 * ml, 1.0, X, r1, 0, T1, r1, 0, 0.0, L[l + 1], r1, 0, 1);
    // XB' = X^T (XB x1 b)
    mode1<double>(c, r0, s0, ml, s1, XB[l], bc[l], T1, 0.0);
    gemm<double>(c.s, OpT, OpN, r1, s1, r0 * ml, 1.0, X, r1, 0, T1, s1, 0, 0.0, XB[l + 1], s1, 0, 1);
    // ZXI' = Z^T (ZXI x1 X);  ZXL' = Z^T (ZXL x1 X + K x2 (ZXI x1 X))
    mode1<double>(c, q0, r0, ml, r1, ZXI[l], X, T1, 0.0);
    gemm<double>(c.s, OpT, OpN, q1, r1, q0 * ml, 1.0, Z, q1, 0, T1, r1, 0, 0.0, ZXI[l + 1], r1, 0, 1);
    mode1<double>(c, q0, r0, ml, r1, ZXL[l], X, T2, 0.0);
    mode2<double>(c, q0, ml, ml, r1, p.dK[l], T1, T2, 1.0);
    gemm<double>(c.s, OpT, OpN, q1, r1, q0 * ml, 1.0, Z, q1, 0, T2, r1, 0, 0.0, ZXL[l + 1], r1, 0, 1);
    // ZB' = Z^T (ZB x1 b)
    mode1<double>(c, q0, s0, ml, s1, ZB[l], bc[l], T1, 0.0);
    gemm<double>(c.s, OpT, OpN, q1, s1, q0 * ml, 1.0, Z, q1, 0, T1, s1, 0, 0.0, ZB[l + 1], s1, 0, 1);
    if (overlap) new_interface(l + 1, r1, true, true);
    else factor_left(l + 1, r1);
  }

  // right interfaces at pos l from pos l+1 and cores x_l, z_l; hess: also
  // reduce L[l] to Hessenberg form for the next site (l-1) of a backward sweep
  void update_right(int l, bool hess = true) {
    const int r0 = xr[l], r1 = xr[l + 1], q0 = zr[l], q1 = zr[l + 1], s0 = sr[l], s1 = sr[l + 1], ml = m[l];
    const double* X = xc[l];
    const double* Z = zc[l];
    if (overlap) wait_eig(l);  // the side stream may still read L[l]
    // L' = X_mat (K x2 X + X x3 L)^T
    mode2<double>(c, r0, ml, ml, r1, p.dK[l], X, T1, 0.0);
    mode3<double>(c, r0, ml, r1, r1, X, L[l + 1], T1, 1.0);
    gemm<double>(c.s, OpN, OpT, r0, r0, ml * r1, 1.0, X, (long)ml * r1, 0, T1, (long)ml * r1, 0, 0.0, L[l], r0, 0, 1);
    // XB' = X_mat (b x3 XB)^T   (r0 x s0)
    mode3<double>(c, s0, ml, s1, r1, bc[l], XB[l + 1], T1, 0.0);
    gemm<double>(c.s, OpN, OpT, r0, s0, ml * r1, 1.0, X, (long)ml * r1, 0, T1, (long)ml * r1, 0, 0.0, XB[l], s0, 0, 1);
    // ZXI' = Z_mat (X x3 ZXI)^T ; ZXL' = Z_mat (K x2 (X x3 ZXI) + X x3 ZXL)^T
    mode3<double>(c, r0, ml, r1, q1, X, ZXI[l + 1], T1, 0.0);
    gemm<double>(c.s, OpN, OpT, q0, r0, ml * q1, 1.0, Z, (long)ml * q1, 0, T1, (long)ml * q1, 0, 0.0, ZXI[l], r0, 0, 1);
    mode3<double>(c, r0, ml, r1, q1, X, ZXL[l + 1], T2, 0.0);
    mode2<double>(c, r0, ml, ml, q1, p.dK[l], T1, T2, 1.0);
    gemm<double>(c.s, OpN, OpT, q0, r0, ml * q1, 1.0, Z, (long)ml * q1, 0, T2, (long)ml * q1, 0, 0.0, ZXL[l], r0, 0, 1);
    // ZB' = Z_mat (b x3 ZB)^T  (q0 x s0)
    mode3<double>(c, s0, ml, s1, q1, bc[l], ZB[l + 1], T1, 0.0);
    gemm<double>(c.s, OpN, OpT, q0, s0, ml * q1, 1.0, Z, (long)ml * q1, 0, T1, (long)ml * q1, 0, 0.0, ZB[l], s0, 0, 1);
    if (overlap) new_interface(l, r0, false, hess);
    else factor(l, r0);
  }

  // right-orthogonalise a TT held in cores (in place); ranks updated
  void right_orth(std::vector<double*>& cores, std::vector<int>& r) {
    for (int l = d - 1; l >= 1; --l) {
      const int r0 = r[l], n = m[l], r1 = r[l + 1];
      const int M = n * r1;
      transpose(c.s, r0, M, cores[l], M, tmp, r0);
      int k = dcholqr(c, M, r0, tmp, r0, Qk, Rk, 1e-15);
      T2S2_CHECK(k >= 1, "solver: zero core in orthogonalisation");
      transpose(c.s, M, k, Qk, k, cores[l], M);
      mode3<double>(c, r[l - 1], m[l - 1], r0, k, cores[l - 1], Rk, tmp, 0.0);
      c.d2d(cores[l - 1], tmp, (size_t)r[l - 1] * m[l - 1] * k);
      r[l] = k;
    }
  }

  int run(const DTT& fin, const DTT* x0, DTT& xout, SolveReport& rep) {
    auto t_start = std::chrono::steady_clock::now();
    pc.s = c.s;
    pc.mark(0);
    d = p.d;
    m = p.m;
    cap = o.rank_cap > 0 ? std::min(o.rank_cap, p.rank_cap) : p.rank_cap;
    kick = std::max(0, std::min(o.kick, cap));
    T2S2_CHECK(fin.d == d, "solve: f has the wrong dimension");
    for (int l = 0; l < d; ++l) T2S2_CHECK(fin.n[l] == m[l], "solve: f mode sizes must be N_l - 2");
    maxrank.assign(d + 1, 1);
    {
      // bond l bound: min(prod_{k<l} m_k, prod_{k>=l} m_k, cap)
      for (int l = 1; l < d; ++l) {
        double a = 1, b = 1;
        for (int k = 0; k < l; ++k) a *= m[k];
        for (int k = l; k < d; ++k) b *= m[k];
        maxrank[l] = (int)std::min<double>({a, b, (double)cap});
      }
    }
    smax = 1;
    sr.assign(d + 1, 1);
    for (int l = 0; l <= d; ++l) {
      sr[l] = fin.r[l];
      smax = std::max(smax, sr[l]);
    }
    int mmax = *std::max_element(m.begin(), m.end());
    const size_t big = (size_t)cap * mmax * cap;
    const size_t kk = (size_t)std::max(kick, 1);
    // f~ = (x E^{-1}) f
    bc.resize(d);
    for (int l = 0; l < d; ++l) {
      bc[l] = buf("b" + std::to_string(l), (size_t)sr[l] * m[l] * sr[l + 1]);
      mode2<double>(c, sr[l], m[l], m[l], sr[l + 1], p.dEinv[l], fin.c[l], bc[l], 0.0);
    }
    L.resize(d + 1);
    XB.resize(d + 1);
    ZXI.resize(d + 1);
    ZXL.resize(d + 1);
    ZB.resize(d + 1);
    eig.resize(d + 1);
    eig32.resize(d + 1);
    ok64.assign(d + 1, 0);
    ok32.assign(d + 1, 0);
    need64.assign(d + 1, 0);
    hf.resize(d + 1);
    lhess.assign(d + 1, 0);
    mixed = (o.precision == 1);
    overlap = !mixed && o.overlap != 0;
    eig_pending.assign(d + 1, 0);
    has_eig.assign(d + 1, 0);
    has_hess.assign(d + 1, 0);
    if (overlap) {
      for (int k = 0; k < Problem::kSides; ++k) {
        if (!p.side[k]) {
          T2S2_HIP(hipStreamCreateWithFlags(&p.side[k], hipStreamNonBlocking));
          T2S2_HIP(hipEventCreateWithFlags(&p.side_done[k], hipEventDisableTiming));
          T2S2_HIP(hipEventRecord(p.side_done[k], p.side[k]));
        }
        cs[k].s = p.side[k];
        cs[k].sc = &p.sc_side[k];
        cs[k].fail = c.fail;
        // side work of an earlier solve on this problem reads interfaces and
        // writes factors and the failure flag, all rewritten from here on
        T2S2_HIP(hipStreamWaitEvent(c.s, p.side_done[k], 0));
      }
      ev_eig.assign(d + 1, nullptr);
      for (auto& e : ev_eig) T2S2_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      T2S2_HIP(hipEventCreateWithFlags(&ev_main, hipEventDisableTiming));
    }
    clear_fail(c);
    for (int l = 0; l <= d; ++l) {
      const std::string t = std::to_string(l);
      L[l] = buf("L" + t, (size_t)cap * cap);
      XB[l] = buf("XB" + t, (size_t)cap * smax);
      ZXI[l] = buf("ZXI" + t, kk * cap);
      ZXL[l] = buf("ZXL" + t, kk * cap);
      ZB[l] = buf("ZB" + t, kk * smax);
      eig[l].lam = c.sc->get<double2>("am.lam" + t, cap);
      eig[l].V = c.sc->get<double2>("am.V" + t, (size_t)cap * cap);
      eig[l].Vi = c.sc->get<double2>("am.Vi" + t, (size_t)cap * cap);
      eig32[l].lam = c.sc->get<float2>("am.lam32" + t, cap);
      eig32[l].V = c.sc->get<float2>("am.V32" + t, (size_t)cap * cap);
      eig32[l].Vi = c.sc->get<float2>("am.Vi32" + t, (size_t)cap * cap);
      hf[l].QT = buf("QT" + t, (size_t)cap * cap);
      hf[l].Hc = buf("Hc" + t, (size_t)cap * cap);
      hf[l].Hc32 = c.sc->get<float>("am.Hc32" + t, (size_t)cap * cap);
    }
    u = buf("u", big);
    f = buf("f", big);
    res = buf("res", big);
    y = buf("y", big);
    T1 = buf("T1", std::max(big, (size_t)cap * mmax * smax));
    T2 = buf("T2", big);
    A1 = buf("A1", (size_t)cap * mmax * kk);
    S = buf("S", (size_t)cap * mmax * kk);
    kick_buf = buf("kick", (size_t)cap * mmax * kk);
    zbuf = buf("zc", kk * mmax * kk);
    U = buf("U", big);
    W = buf("W", (size_t)cap * cap);
    tmp = buf("tmp", big);
    Qk = buf("Qk", big + kk * mmax * ((size_t)cap + kk));
    Rk = buf("Rk", (size_t)cap * std::max<size_t>(cap, mmax * kk));
    h0 = c.sc->get<double2>("am.h0", big);
    h1 = c.sc->get<double2>("am.h1", big);
    g0 = c.sc->get<float2>("am.g0", big);
    g1 = c.sc->get<float2>("am.g1", big);
    hr = buf("hr", big);
    cond = buf("cond", (size_t)d + 1);
    fill(c.s, cond, d + 1, 0.0);
    if (x0 && o.warm_judge) {
      // the given start is kept only if its FP64 residual beats that of the
      // seeded random start a cold solve would use (the fallback)
      rep.warm_residual = tt_residual_norm(p, c, *x0, fin);
      DTT cold;
      cold.d = d;
      cold.n = m;
      cold.r.assign(d + 1, 1);
      cold.c.resize(d);
      for (int l = 1; l < d; ++l) cold.r[l] = std::min(std::max(1, o.init_rank), maxrank[l]);
      for (int l = 0; l < d; ++l) {
        const long sz = (long)cold.r[l] * m[l] * cold.r[l + 1];
        cold.c[l] = buf("cold" + std::to_string(l), (size_t)sz);
        fill_random(c.s, cold.c[l], sz, o.seed * 1315423911ULL + 17ULL * l + 1ULL);
      }
      rep.cold_residual = tt_residual_norm(p, c, cold, fin);
      if (!(rep.warm_residual < rep.cold_residual)) x0 = nullptr;
    }
    rep.warm_start_used = x0 ? 1 : 0;
    // initial x (caller's buffers) and z (scratch)
    xr.assign(d + 1, 1);
    zr.assign(d + 1, 1);
    xc = xout.c;
    zc.resize(d);
    for (int l = 1; l < d; ++l) {
      xr[l] = x0 ? std::min(x0->r[l], maxrank[l]) : std::min(std::max(1, o.init_rank), maxrank[l]);
      zr[l] = std::min((int)kk, maxrank[l]);
    }
    for (int l = 0; l < d; ++l) {
      zc[l] = buf("z" + std::to_string(l), kk * mmax * kk);
      if (x0) {
        T2S2_CHECK(x0->r[l] <= cap && x0->r[l + 1] <= cap, "solve: x0 ranks exceed rank_cap");
        if (x0->c[l] != xc[l]) c.d2d(xc[l], x0->c[l], (size_t)x0->r[l] * m[l] * x0->r[l + 1]);
      } else {
        fill_random(c.s, xc[l], (long)xr[l] * m[l] * xr[l + 1], o.seed * 1315423911ULL + 17ULL * l + 1ULL);
      }
      fill_random(c.s, zc[l], (long)zr[l] * m[l] * zr[l + 1], o.seed * 2654435761ULL + 31ULL * l + 7ULL);
    }
    if (x0) xr = x0->r;
    right_orth(xc, xr);
    right_orth(zc, zr);
    set_boundary(0);
    set_boundary(d);
    // the first sweep goes left to right: it needs the eigendecompositions
    // of the right interfaces, not their Hessenberg forms
    for (int l = d - 1; l >= 1; --l) update_right(l, false);

    const double loc_tol = o.tol / std::sqrt((double)d);
    int status = 3;
    int direction = +1;
    int sweeps = 0;
    double last_res = -1.0;
    for (int sw = 0; sw < o.max_sweeps; ++sw) {
      sweeps = sw + 1;
      double max_res = 0.0;
      for (int step = 0; step < d; ++step) {
        pc.mark(1);
        const int l = direction > 0 ? step : d - 1 - step;
        const int r1 = xr[l], r2 = xr[l + 1], ml = m[l], s0 = sr[l], s1 = sr[l + 1];
        const long n = (long)r1 * ml * r2;
        // local right-hand side f = XB_l x1 b x3 XB_{l+1}
        mode1<double>(c, r1, s0, ml, s1, XB[l], bc[l], T1, 0.0);
        mode3<double>(c, r1, ml, s1, r2, T1, XB[l + 1], f, 0.0);
        const double fn = c.nrm2(f, n);
        // residual of the current core, refinement with the exact solver
        c.d2d(u, xc[l], n);
        local_apply(l, r1, r2, L[l], L[l + 1], u, res);
        axpby(c.s, n, 1.0, f, -1.0, res);
        double rn = c.nrm2(res, n);
        T2S2_CHECK(std::isfinite(rn) && std::isfinite(fn), "solve: non-finite local residual");
        const double res0 = fn > 0 ? rn / fn : 0.0;
        max_res = std::max(max_res, res0);
        if (res0 > loc_tol) {
          // iterative refinement: FP64 residual and update, correction from
          // the exact solver's factors (FP64, or FP32 in mixed precision
          // with a switch to FP64 factors when they contract too slowly)
          ++rep.local_systems;
          // FP32 corrections need current FP32 factors on both sides; a bond
          // that keeps FP64 factors makes its neighbours' systems FP64 too
          bool use64 = !mixed || !(ok32[l] && ok32[l + 1]);
          const int mode = overlap ? pick_mode(l, direction, r1, r2) : -1;
          if (use64 && !overlap) {
            ensure64(l, r1);
            ensure64(l + 1, r2);
          }
          double prev = rn;
          for (int it = 0, it32 = 0, it64 = 0; it < 14; ++it) {
            if (overlap) {
              local_solve_ov(mode, l, r1, r2, res, y);
              ++it64;
            } else if (use64) {
              local_solve(l, r1, r2, eig[l], eig[l + 1], res, y);
              ++it64;
            } else {
              local_solve32(l, r1, r2, eig32[l], eig32[l + 1], res, y);
              ++it32;
            }
            ++rep.refinement_steps;
            axpby(c.s, n, 1.0, y, 1.0, u);
            local_apply(l, r1, r2, L[l], L[l + 1], u, res);
            axpby(c.s, n, 1.0, f, -1.0, res);
            rn = c.nrm2(res, n);
            if (rn <= 0.1 * loc_tol * fn) break;
            if (use64 && it64 >= 6) break;
            if (!use64 && (rn > 0.25 * prev || it32 >= 8)) {
              ensure64(l, r1);
              ensure64(l + 1, r2);
              need64[l] = need64[l + 1] = 1;
              use64 = true;
              ++rep.fp64_fallbacks;
            }
            prev = rn;
          }
          if (rn > 0.1 * loc_tol * fn) ++rep.refinement_capped;
        }
        const bool last = (direction > 0 && l == d - 1) || (direction < 0 && l == 0);
        if (last) {
          c.d2d(xc[l], u, n);
          continue;
        }
        const double unorm = c.nrm2(u, n);
        const double delta = o.tol * unorm / std::sqrt((double)d);
        pc.mark(2);
        if (direction > 0) step_right(l, delta);
        else step_left(l, delta);
      }
      direction = -direction;
      rep.hist_local.push_back(max_res);
      int mr = 0;
      for (int l = 0; l <= d; ++l) mr = std::max(mr, xr[l]);
      rep.hist_rank.push_back(mr);
      double gres = -1.0;
      // FP64 residual: every check_every sweeps, or (check_every = 0) once the
      // largest local residual suggests the target may be met, and at the end
      const bool near = max_res <= 10.0 * o.target;
      const bool check = (o.check_every == 1) || (o.check_every > 1 && sweeps % o.check_every == 0) ||
                         (o.check_every == 0 && near) || (sweeps == o.max_sweeps);
      if (check) {
        pc.mark(4);
        DTT xd;
        xd.d = d;
        xd.n = m;
        xd.r = xr;
        xd.c = xc;
        gres = tt_residual_norm(p, c, xd, fin);
        last_res = gres;
      }
      if (read_fail(c))
        throw Error(5, "solve: Francis QR of an interface matrix did not converge (sweep " +
                           std::to_string(sweeps) + ")");
      rep.hist_res.push_back(gres);
      const double ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
      rep.hist_time.push_back(ms);
      if (o.verbose)
        std::fprintf(stderr, "[t2s2] sweep %d  max local res %.3e  residual %.3e  max rank %d  %.1f ms\n", sweeps,
                     max_res, gres, mr, ms);
      if (gres >= 0.0 && gres <= o.target) {
        status = 0;
        break;
      }
    }
    if (last_res < 0.0) {
      pc.mark(4);
      DTT xd;
      xd.d = d;
      xd.n = m;
      xd.r = xr;
      xd.c = xc;
      last_res = tt_residual_norm(p, c, xd, fin);
      status = last_res <= o.target ? 0 : 3;
    }
    xout.r = xr;
    rep.status = status;
    rep.sweeps = sweeps;
    rep.residual = last_res;
    rep.ranks = xr;
    rep.max_rank = *std::max_element(xr.begin(), xr.end());
    pc.mark(0);
    c.sync();
    pc.collect(rep.phase_ms);
    {
      // eigendecompositions still running on the side streams are left out
      std::vector<double> hc(d + 1);
      c.d2h(hc.data(), cond, d + 1);
      for (double v : hc) rep.max_eig_cond = std::max(rep.max_eig_cond, v);
    }
    if (read_fail(c)) throw Error(5, "solve: Francis QR of an interface matrix did not converge");
    rep.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return status;
  }

  // ---- left-to-right split at core l (l < d-1) ---------------------------
  void step_right(int l, double delta) {
    const int r1 = xr[l], r2 = xr[l + 1], ml = m[l], s0 = sr[l], s1 = sr[l + 1];
    const int q0 = zr[l], q2 = zr[l + 1], r3 = xr[l + 2], m1 = m[l + 1];
    const int M = r1 * ml;
    const int room = std::max(1, maxrank[l + 1]);
    const int r = trunc_svd(c, M, r2, u, r2, delta, room, U, W);
    // uk = U W (truncated solution)
    gemm<double>(c.s, OpN, OpN, M, r2, r, 1.0, U, r, 0, W, r2, 0, 0.0, y, r2, 0, 1);
    int kk = 0, kq = 0;
    if (kick > 0 && q2 > 0) {
      // A1 = uk x3 ZXI_{l+1};  S = K x2 A1 + uk x3 ZXL_{l+1}
      mode3<double>(c, r1, ml, r2, q2, y, ZXI[l + 1], A1, 0.0);
      mode2<double>(c, r1, ml, ml, q2, p.dK[l], A1, S, 0.0);
      mode3<double>(c, r1, ml, r2, q2, y, ZXL[l + 1], S, 1.0);
      // kick = (XB_l x1 b) x3 ZB_{l+1} - (L_l x1 A1 + S)      (r1 m x q2)
      mode1<double>(c, r1, s0, ml, s1, XB[l], bc[l], T1, 0.0);
      mode3<double>(c, r1, ml, s1, q2, T1, ZB[l + 1], kick_buf, 0.0);
      axpby(c.s, (long)M * q2, -1.0, S, 1.0, kick_buf);
      mode1<double>(c, r1, r1, ml, q2, L[l], A1, T2, 0.0);
      axpby(c.s, (long)M * q2, -1.0, T2, 1.0, kick_buf);
      // z core: (ZB_l x1 b) x3 ZB_{l+1} - (ZXL_l x1 A1 + ZXI_l x1 S)   (q0 m x q2)
      mode1<double>(c, q0, s0, ml, s1, ZB[l], bc[l], T1, 0.0);
      mode3<double>(c, q0, ml, s1, q2, T1, ZB[l + 1], zbuf, 0.0);
      mode1<double>(c, q0, r1, ml, q2, ZXL[l], A1, T2, 0.0);
      mode1<double>(c, q0, r1, ml, q2, ZXI[l], S, T2, 1.0);
      axpby(c.s, (long)q0 * ml * q2, -1.0, T2, 1.0, zbuf);
      // orthogonalise the kick against U (two passes) and orthonormalise it
      for (int pass = 0; pass < 2; ++pass) {
        gemm<double>(c.s, OpT, OpN, r, q2, M, 1.0, U, r, 0, kick_buf, q2, 0, 0.0, Rk, q2, 0, 1);
        gemm<double>(c.s, OpN, OpN, M, q2, r, -1.0, U, r, 0, Rk, q2, 0, 1.0, kick_buf, q2, 0, 1);
      }
      const int room_k = std::min(room - r, q2);
      if (room_k > 0) {
        kq = dcholqr(c, M, q2, kick_buf, q2, Qk, Rk, 1e-13);
        kk = std::min(kq, room_k);
      }
      // new z core
      int kz = dcholqr(c, q0 * ml, q2, zbuf, q2, Qk + (size_t)M * q2, Rk, 1e-13);
      if (kz == 0) {
        fill_random(c.s, zbuf, (long)q0 * ml * q2, 977ULL + l);
        kz = dcholqr(c, q0 * ml, q2, zbuf, q2, Qk + (size_t)M * q2, Rk, 1e-13);
      }
      c.d2d(zc[l], Qk + (size_t)M * q2, (size_t)q0 * ml * kz);
      zr[l + 1] = kz;
    }
    const int rn = r + kk;
    // x_l = [U | Qk(:, :kk)]
    copy2d(c.s, M, r, U, r, xc[l], rn);
    if (kk > 0) copy2d(c.s, M, kk, Qk, kq, xc[l] + r, rn);
    // x_{l+1} = [W; 0] x1 x_{l+1}
    mode1<double>(c, r, r2, m1, r3, W, xc[l + 1], tmp, 0.0);
    c.d2d(xc[l + 1], tmp, (size_t)r * m1 * r3);
    if (kk > 0) fill(c.s, xc[l + 1] + (size_t)r * m1 * r3, (long)kk * m1 * r3, 0.0);
    xr[l + 1] = rn;
    // the next z core's left rank follows z_l; its content is rebuilt at l+1
    pc.mark(3);
    update_left(l);
  }

  // ---- right-to-left split at core l (l > 0) -----------------------------
  void step_left(int l, double delta) {
    const int r1 = xr[l], r2 = xr[l + 1], ml = m[l], s0 = sr[l], s1 = sr[l + 1];
    const int q1 = zr[l], q2 = zr[l + 1], r0 = xr[l - 1], mp = m[l - 1];
    const int M = ml * r2;
    const int room = std::max(1, maxrank[l]);
    // u^T (m r2 x r1) = U W  ->  u = W^T U^T
    transpose(c.s, r1, M, u, M, tmp, r1);
    const int r = trunc_svd(c, M, r1, tmp, r1, delta, room, U, W);
    // uk = W^T U^T  (r1 x m r2)
    gemm<double>(c.s, OpT, OpT, r1, M, r, 1.0, W, r1, 0, U, r, 0, 0.0, y, M, 0, 1);
    int kk = 0, kq = 0;
    if (kick > 0 && q1 > 0) {
      // A1 = ZXI_l x1 uk (q1 x m x r2);  S = K x2 A1 + ZXL_l x1 uk
      mode1<double>(c, q1, r1, ml, r2, ZXI[l], y, A1, 0.0);
      mode2<double>(c, q1, ml, ml, r2, p.dK[l], A1, S, 0.0);
      mode1<double>(c, q1, r1, ml, r2, ZXL[l], y, S, 1.0);
      // kick = (ZB_l x1 b) x3 XB_{l+1} - (S + A1 x3 L_{l+1})   (q1 x m r2)
      mode1<double>(c, q1, s0, ml, s1, ZB[l], bc[l], T1, 0.0);
      mode3<double>(c, q1, ml, s1, r2, T1, XB[l + 1], kick_buf, 0.0);
      axpby(c.s, (long)q1 * M, -1.0, S, 1.0, kick_buf);
      mode3<double>(c, q1, ml, r2, r2, A1, L[l + 1], T2, 0.0);
      axpby(c.s, (long)q1 * M, -1.0, T2, 1.0, kick_buf);
      // z core: (ZB_l x1 b) x3 ZB_{l+1} - (S x3 ZXI_{l+1} + A1 x3 ZXL_{l+1})  (q1 x m x q2)
      mode3<double>(c, q1, ml, s1, q2, T1, ZB[l + 1], zbuf, 0.0);
      mode3<double>(c, q1, ml, r2, q2, S, ZXI[l + 1], T2, 0.0);
      mode3<double>(c, q1, ml, r2, q2, A1, ZXL[l + 1], T2, 1.0);
      axpby(c.s, (long)q1 * ml * q2, -1.0, T2, 1.0, zbuf);
      // kick^T (M x q1), orthogonalise against U (M x r), orthonormalise
      transpose(c.s, q1, M, kick_buf, M, T2, q1);
      for (int pass = 0; pass < 2; ++pass) {
        gemm<double>(c.s, OpT, OpN, r, q1, M, 1.0, U, r, 0, T2, q1, 0, 0.0, Rk, q1, 0, 1);
        gemm<double>(c.s, OpN, OpN, M, q1, r, -1.0, U, r, 0, Rk, q1, 0, 1.0, T2, q1, 0, 1);
      }
      const int room_k = std::min(room - r, q1);
      if (room_k > 0) {
        kq = dcholqr(c, M, q1, T2, q1, Qk, Rk, 1e-13);
        kk = std::min(kq, room_k);
      }
      // new z core (rows orthonormal): zbuf (q1 x m q2) -> transpose -> QR
      transpose(c.s, q1, (long)ml * q2, zbuf, (long)ml * q2, T2, q1);
      double* Qz = Qk + (size_t)M * q1;
      int kz = dcholqr(c, ml * q2, q1, T2, q1, Qz, Rk, 1e-13);
      if (kz == 0) {
        fill_random(c.s, T2, (long)ml * q2 * q1, 1777ULL + l);
        kz = dcholqr(c, ml * q2, q1, T2, q1, Qz, Rk, 1e-13);
      }
      transpose(c.s, (long)ml * q2, kz, Qz, kz, zc[l], (long)ml * q2);
      zr[l] = kz;
    }
    const int rn = r + kk;
    // x_l = [U^T ; Qk^T]  (rn x m r2)
    transpose(c.s, M, r, U, r, xc[l], M);
    if (kk > 0) transpose(c.s, M, kk, Qk, kq, xc[l] + (size_t)r * M, M);
    // x_{l-1} = x_{l-1} x3 [W^T | 0]:  new[.., j] = sum_b x[.., b] W[j, b] for j < r
    double* out = tmp;
    mode3<double>(c, r0, mp, r1, r, xc[l - 1], W, out, 0.0);
    copy2d(c.s, (long)r0 * mp, r, out, r, xc[l - 1], rn);
    if (kk > 0) {
      // zero columns r..rn-1
      double* zcol = T2;
      fill(c.s, zcol, (long)r0 * mp * kk, 0.0);
      copy2d(c.s, (long)r0 * mp, kk, zcol, kk, xc[l - 1] + r, rn);
    }
    xr[l] = rn;
    pc.mark(3);
    update_right(l);
  }
};

}  // namespace

void local_kron_solve(const Ctx& c0, int r1, int m, int r2, const double* Lint, const double* K, const double* Rint,
                      const double* g, double* u, int method) {
  T2S2_CHECK(r1 >= 1 && m >= 1 && r2 >= 1, "local_solve: sizes must be positive");
  T2S2_CHECK(r1 <= 512 && r2 <= 512 && m <= 64, "local_solve: r1, r2 <= 512 and m <= 64 required");
  T2S2_CHECK(method >= 0 && method <= 2,
             "local_solve: method must be 0 (eigen), 1 (Hessenberg left) or 2 (Hessenberg right)");
  T2S2_CHECK(method != 1 || kron_hess_fits(r1, m, (int)sizeof(double2)),
             "local_solve: method 1 needs r1 <= 256 and the m right-hand sides of a chain in LDS");
  T2S2_CHECK(method != 2 || kron_hess_fits(r2, m, (int)sizeof(double2)),
             "local_solve: method 2 needs r2 <= 256 and the m right-hand sides of a chain in LDS");
  Scratch& S = *c0.sc;
  Ctx c = c0;
  c.fail = S.get<int>("ctx.fail", 1);
  clear_fail(c);
  const long n = (long)r1 * m * r2;
  double2* ZT = S.get<double2>("loc.ZT", (size_t)m * m);
  double2* T = S.get<double2>("loc.T", (size_t)m * m);
  schur_real(c, m, K, ZT, T);
  double2* w0 = S.get<double2>("loc.w0", n);
  double2* w1 = S.get<double2>("loc.w1", n);
  if (method == 2) {
    Eig eL;
    eL.lam = S.get<double2>("loc.lamL", r1);
    eL.V = S.get<double2>("loc.VL", (size_t)r1 * r1);
    eL.Vi = S.get<double2>("loc.ViL", (size_t)r1 * r1);
    eig_nonsym(c, r1, Lint, eL.lam, eL.V, eL.Vi);
    double* Hw = S.get<double>("loc.H", (size_t)r2 * r2);
    double* QT = S.get<double>("loc.QT", (size_t)r2 * r2);
    double* Hc = S.get<double>("loc.Hc", (size_t)r2 * r2);
    double* wr = S.get<double>("loc.wr", n);
    c.d2d(Hw, Rint, (size_t)r2 * r2);
    hessenberg(c, r2, Hw, QT);
    transpose(c.s, r2, r2, Hw, r2, Hc, r2);
    kron_inverse_hess_right(c, r1, m, r2, ZT, T, eL, QT, Hc, g, u, w0, w1, wr);
    c.sync();
    if (read_fail(c)) throw Error(5, "local_solve: Francis QR did not converge");
    return;
  }
  Eig eR;
  eR.lam = S.get<double2>("loc.lamR", r2);
  eR.V = S.get<double2>("loc.VR", (size_t)r2 * r2);
  eR.Vi = S.get<double2>("loc.ViR", (size_t)r2 * r2);
  eig_nonsym(c, r2, Rint, eR.lam, eR.V, eR.Vi);
  if (method == 0) {
    Eig eL;
    eL.lam = S.get<double2>("loc.lamL", r1);
    eL.V = S.get<double2>("loc.VL", (size_t)r1 * r1);
    eL.Vi = S.get<double2>("loc.ViL", (size_t)r1 * r1);
    eig_nonsym(c, r1, Lint, eL.lam, eL.V, eL.Vi);
    kron_inverse_eig<double2>(c, r1, m, r2, ZT, T, eL, eR, g, u, w0, w1);
  } else {
    double* Hw = S.get<double>("loc.H", (size_t)r1 * r1);
    double* QT = S.get<double>("loc.QT", (size_t)r1 * r1);
    double* Hc = S.get<double>("loc.Hc", (size_t)r1 * r1);
    double* wr = S.get<double>("loc.wr", n);
    c.d2d(Hw, Lint, (size_t)r1 * r1);
    hessenberg(c, r1, Hw, QT);
    transpose(c.s, r1, r1, Hw, r1, Hc, r1);
    kron_inverse_hess<double2, double>(c, r1, m, r2, ZT, T, QT, Hc, eR, g, u, w0, w1, wr);
  }
  c.sync();
  if (read_fail(c)) throw Error(5, "local_solve: Francis QR did not converge");
}

int mol_step(Problem& p, const Ctx& c, const DTT& u, const DTT* b, const SolveOptions& o, DTT& x,
             SolveReport& rep) {
  T2S2_CHECK(p.mol_theta > 0.0, "mol_step: the problem was not created for time stepping (t2s2_mol_create)");
  T2S2_CHECK(u.d == p.d, "mol_step: u has the wrong dimension");
  for (int l = 0; l < p.d; ++l) T2S2_CHECK(u.n[l] == p.m[l], "mol_step: u mode sizes must be N_l - 2");
  DTT y;
  kron_sum_apply(c, p.m, p.m, 0, p.dEi, p.dMx, u, "mol.y", y);
  std::vector<const DTT*> parts{&y};
  std::vector<double> coef{1.0};
  if (b) {
    T2S2_CHECK(b->d == p.d, "mol_step: b has the wrong dimension");
    for (int l = 0; l < p.d; ++l) T2S2_CHECK(b->n[l] == p.m[l], "mol_step: b mode sizes must be N_l - 2");
    parts.push_back(b);
    coef.push_back(1.0 / p.mol_theta);
  }
  DTT f;
  tt_concat(c, parts, coef, "mol.f", f);
  const int cap = o.rank_cap > 0 ? std::min(o.rank_cap, p.rank_cap) : p.rank_cap;
  tt_round(c, f, 1e-14, cap);
  return solve(p, c, f, &u, o, x, rep);
}

// Frees the blocks that scratch buffers outgrew (Scratch::release_retired)
// when that cannot stall the host behind queued work: before a solve queues
// anything, and after it if no side stream still runs its eigendecompositions
// (otherwise at the next solve, or when the problem is destroyed).
thread_local bool t_defer_release = false;

void defer_scratch_release(bool on) { t_defer_release = on; }

void free_retired_scratch(Problem& p) {
  p.sc.release_retired();
  for (int k = 0; k < Problem::kSides; ++k) p.sc_side[k].release_retired();
}

static void release_scratch(Problem& p, bool only_if_sides_idle) {
  if (t_defer_release) return;
  bool any = p.sc.has_retired();
  for (int k = 0; k < Problem::kSides; ++k) any = any || p.sc_side[k].has_retired();
  if (!any) return;
  if (only_if_sides_idle)
    for (int k = 0; k < Problem::kSides; ++k) {
      if (!p.side[k]) continue;
      const hipError_t q = hipStreamQuery(p.side[k]);
      if (q == hipErrorNotReady) {
        (void)hipGetLastError();  // not an error: the side stream is busy
        return;
      }
      T2S2_HIP(q);
    }
  free_retired_scratch(p);
}

int solve(Problem& p, const Ctx& c0, const DTT& f, const DTT* x0, const SolveOptions& o, DTT& x, SolveReport& rep) {
  Ctx c = c0;
  release_scratch(p, false);
  c.fail = c.sc->get<int>("ctx.fail", 1);
  int st;
  {
    Amen a(p, c, o);
    st = a.run(f, x0, x, rep);
  }
  release_scratch(p, true);
  return st;
}

}  // namespace t2s2
