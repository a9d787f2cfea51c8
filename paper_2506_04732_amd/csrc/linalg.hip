// Host orchestration of the device linear algebra.  See linalg.h.
#include "linalg.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace t2s2 {

namespace {
__global__ void flag_if_negative_kernel(const int* __restrict__ info, int* __restrict__ fail) {
  if (threadIdx.x == 0 && info[0] < 0) fail[0] = 1;
}
__global__ void clear_int_kernel(int* __restrict__ x) {
  if (threadIdx.x == 0) x[0] = 0;
}
// after a Francis QR: raise c.fail when it stopped at its step limit
void flag_francis(const Ctx& c, const int* info) {
  if (!c.fail) return;
  hipLaunchKernelGGL(flag_if_negative_kernel, dim3(1), dim3(64), 0, c.s, info, c.fail);
  T2S2_LAUNCH_CHECK();
}
int g_jacobi_sweeps = 0;

// slot[0] = max(slot[0], ||V||_F ||Vi||_F), one workgroup of 256
__global__ void cond_fro_kernel(long nn, const double2* __restrict__ V, const double2* __restrict__ Vi,
                                double* __restrict__ slot) {
  __shared__ double sa[256], sb[256];
  double a = 0.0, b = 0.0;
  for (long e = threadIdx.x; e < nn; e += blockDim.x) {
    a += V[e].x * V[e].x + V[e].y * V[e].y;
    b += Vi[e].x * Vi[e].x + Vi[e].y * Vi[e].y;
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sa[threadIdx.x] += sa[threadIdx.x + h];
      sb[threadIdx.x] += sb[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double cnd = sqrt(sa[0]) * sqrt(sb[0]);
    if (!(slot[0] >= cnd)) slot[0] = cnd;
  }
}
}  // namespace

void cond_estimate(const Ctx& c, int n, const double2* V, const double2* Vi, double* slot) {
  hipLaunchKernelGGL(cond_fro_kernel, dim3(1), dim3(256), 0, c.s, (long)n * n, V, Vi, slot);
  T2S2_LAUNCH_CHECK();
}

void set_iteration_limits(int francis_steps, int jacobi_sweeps);
void set_francis_step_limit(int steps);  // schur.hip

void set_iteration_limits(int francis_steps, int jacobi_sweeps) {
  set_francis_step_limit(std::max(0, francis_steps));
  g_jacobi_sweeps = std::max(0, jacobi_sweeps);
}
int jacobi_sweep_limit() { return g_jacobi_sweeps > 0 ? g_jacobi_sweeps : 60; }

void clear_fail(const Ctx& c) {
  if (!c.fail) return;
  hipLaunchKernelGGL(clear_int_kernel, dim3(1), dim3(64), 0, c.s, c.fail);
  T2S2_LAUNCH_CHECK();
}

bool read_fail(const Ctx& c) {
  if (!c.fail) return false;
  int h = 0;
  c.d2h(&h, c.fail, 1);
  return h != 0;
}

Scratch::~Scratch() {
  release_retired();
  for (auto& kv : bufs_)
    if (kv.second.p) (void)hipFree(kv.second.p);
}

void Scratch::release_retired() {
  for (void* p : retired_) (void)hipFree(p);
  retired_.clear();
}

void* Scratch::raw(const std::string& name, size_t bytes) {
  Buf& b = bufs_[name];
  if (b.bytes >= bytes && b.p) return b.p;
  if (b.p) retired_.push_back(b.p);
  b.p = nullptr;
  b.bytes = 0;
  // grow geometrically to limit reallocations
  size_t want = std::max(bytes, (size_t)4096);
  want = std::max(want, b.bytes + b.bytes / 2);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    throw Error(2, "device allocation of " + std::to_string(want) + " bytes failed for " + name);
  }
  b.bytes = want;
  return b.p;
}

size_t Scratch::bytes() const {
  size_t t = 0;
  for (auto& kv : bufs_) t += kv.second.bytes;
  return t;
}

double Ctx::dot(const double* x, const double* y, long n) const {
  if (n <= 0) return 0.0;
  double* partial = sc->get<double>("ctx.dot.partial", kDotBlocks);
  double* out = sc->get<double>("ctx.dot.out", 1);
  dot_device(s, x, y, n, partial, out);
  double h = 0.0;
  d2h(&h, out, 1);
  return h;
}

double Ctx::nrm2(const double* x, long n) const { return std::sqrt(std::max(0.0, dot(x, x, n))); }

template <class T>
static T one_v();
template <>
double one_v<double>() { return 1.0; }
template <>
double2 one_v<double2>() { return make_double2(1.0, 0.0); }
template <>
float2 one_v<float2>() { return make_float2(1.0f, 0.0f); }

template <class T>
void mode1(const Ctx& c, int rA, int r0, int m, int r1, const T* A, const T* X, T* Y, T beta, Op opA) {
  const long ldA = (opA == OpN || opA == OpR) ? r0 : rA;
  gemm<T>(c.s, opA, OpN, rA, m * r1, r0, one_v<T>(), A, ldA, 0, X, (long)m * r1, 0, beta, Y, (long)m * r1, 0, 1);
}

template <class T>
void mode3(const Ctx& c, int r0, int m, int r1, int rB, const T* X, const T* B, T* Y, T beta, Op opB) {
  // op(B) must be r1 x rB; with opB = T, B is stored rB x r1
  const long ldB = (opB == OpT || opB == OpC) ? r1 : rB;
  gemm<T>(c.s, OpN, opB, r0 * m, rB, r1, one_v<T>(), X, r1, 0, B, ldB, 0, beta, Y, rB, 0, 1);
}

template <class T>
void mode2(const Ctx& c, int r0, int mK, int m, int r1, const T* K, const T* X, T* Y, T beta, Op opK) {
  const long ldK = (opK == OpN || opK == OpR) ? m : mK;
  gemm<T>(c.s, opK, OpN, mK, r1, m, one_v<T>(), K, ldK, 0, X, r1, (long)m * r1, beta, Y, r1, (long)mK * r1, r0);
}

template void mode1<double>(const Ctx&, int, int, int, int, const double*, const double*, double*, double, Op);
template void mode1<double2>(const Ctx&, int, int, int, int, const double2*, const double2*, double2*, double2, Op);
template void mode3<double>(const Ctx&, int, int, int, int, const double*, const double*, double*, double, Op);
template void mode3<double2>(const Ctx&, int, int, int, int, const double2*, const double2*, double2*, double2, Op);
template void mode2<double>(const Ctx&, int, int, int, int, const double*, const double*, double*, double, Op);
template void mode2<double2>(const Ctx&, int, int, int, int, const double2*, const double2*, double2*, double2, Op);
template void mode1<float2>(const Ctx&, int, int, int, int, const float2*, const float2*, float2*, float2, Op);
template void mode3<float2>(const Ctx&, int, int, int, int, const float2*, const float2*, float2*, float2, Op);
template void mode2<float2>(const Ctx&, int, int, int, int, const float2*, const float2*, float2*, float2, Op);

// ------------------------------------------------------------ dcholqr
// Host reads per level: one for the kept-pivot count and mask, one for the
// two orthogonality passes' counts together with the remainder norm of the
// deflation (both passes and, when the level leaves columns unrepresented,
// the deflation run before that read, on the usual outcome that no column
// becomes dependent in a pass).  If a pass did lose a column, the level's
// passes are redone one at a time from their saved input.
int dcholqr(const Ctx& c, int M, int n, const double* A, long lda, double* Qout, double* Rout, double drop) {
  T2S2_CHECK(M >= 1 && n >= 1, "dcholqr: empty matrix");
  const int kmax = std::min(M, n);
  Scratch& S = *c.sc;
  double* Aw = S.get<double>("dq.A", (size_t)M * n);
  double* Work = S.get<double>("dq.W", (size_t)M * n);
  double* Q = S.get<double>("dq.Q", (size_t)M * kmax);
  double* G = S.get<double>("dq.G", (size_t)n * n);
  double* Rl = S.get<double>("dq.Rl", (size_t)n * n);
  double* Ak = S.get<double>("dq.Ak", (size_t)M * n);
  double* Qk = S.get<double>("dq.Qk", (size_t)M * n);
  double* Qc = S.get<double>("dq.Qc", (size_t)M * n);
  double* R11 = S.get<double>("dq.R11", (size_t)n * n);
  double* R11i = S.get<double>("dq.R11i", (size_t)n * n);
  double* C = S.get<double>("dq.C", (size_t)kmax * n);
  double* partial = S.get<double>("dq.partial", kDotBlocks);
  // status block read back in one piece: [0] ||A||^2, [1] remainder norm^2,
  // then ints: level count, pass-0 count, pass-1 count, level mask (n)
  double* st = S.get<double>("dq.st", 2 + ((size_t)n + 4) / 2 + 1);
  int* sti = reinterpret_cast<int*>(st + 2);
  int* mask = sti + 3;
  int* pmask = S.get<int>("dq.pmask", n);
  int* idx = S.get<int>("dq.idx", n);
  // A (contiguous) is read in place
  const double* Ain = A;
  if (lda != n) {
    copy2d(c.s, M, n, A, lda, Aw, n);
    Ain = Aw;
  }
  const double* Wk = Ain;      // the part of A not yet represented (level 0: A)
  double normA2 = -1.0;        // ||A||^2, computed with the first deflation
  std::vector<int> hlev(3 + (size_t)n), hidx;
  struct {
    double nrm[2];
    int cnt[3];
  } hst;
  int k = 0;
  for (int level = 0; level < 5 && k < kmax; ++level) {
    gemm<double>(c.s, OpT, OpN, n, n, M, 1.0, Wk, n, 0, Wk, n, 0, 0.0, G, n, 0, 1);
    chol_skip(c.s, n, G, Rl, mask, sti, 1e-11);
    c.d2h(hlev.data(), sti, 3 + (size_t)n);
    int kl = hlev[0];
    if (kl == 0) break;
    const double* Ablk;   // the kept columns of Wk (M x kl)
    const double* Rblk;   // their Cholesky factor (kl x kl)
    if (kl == n && n <= kmax - k) {
      // every column kept: no gathers
      Ablk = Wk;
      Rblk = Rl;
    } else {
      hidx.clear();
      for (int j = 0; j < n && (int)hidx.size() < kmax - k; ++j)
        if (hlev[3 + j]) hidx.push_back(j);
      kl = (int)hidx.size();
      if (kl == 0) break;
      c.h2d(idx, hidx.data(), kl);
      gather_cols(c.s, M, kl, Wk, n, idx, Ak, kl);
      // R11 = Rl[idx][idx]: gather columns, then rows (via transposes)
      gather_cols(c.s, n, kl, Rl, n, idx, R11i, kl);           // n x kl: columns idx
      transpose(c.s, n, kl, R11i, kl, G, n);                   // kl x n
      gather_cols(c.s, kl, kl, G, n, idx, R11, kl);            // kl x kl = (R11)^T
      transpose(c.s, kl, kl, R11, kl, G, kl);                  // R11
      Ablk = Ak;
      Rblk = G;
    }
    trtri_upper(c.s, kl, Rblk, R11i);
    gemm<double>(c.s, OpN, OpN, M, kl, kl, 1.0, Ablk, kl, 0, R11i, kl, 0, 0.0, Qk, kl, 0, 1);
    // ---- both orthogonality passes (reorthogonalise against earlier levels,
    // then a Cholesky QR pass on the new block): Qk -> Ak -> Qc
    auto pass = [&](double* in, double* out, int* cnt) {
      if (k > 0) {
        gemm<double>(c.s, OpT, OpN, k, kl, M, 1.0, Q, kmax, 0, in, kl, 0, 0.0, C, kl, 0, 1);
        gemm<double>(c.s, OpN, OpN, M, kl, k, -1.0, Q, kmax, 0, C, kl, 0, 1.0, in, kl, 0, 1);
      }
      gemm<double>(c.s, OpT, OpN, kl, kl, M, 1.0, in, kl, 0, in, kl, 0, 0.0, G, kl, 0, 1);
      chol_skip(c.s, kl, G, R11, pmask, cnt, 1e-14);
      trtri_upper(c.s, kl, R11, R11i);
      gemm<double>(c.s, OpN, OpN, M, kl, kl, 1.0, in, kl, 0, R11i, kl, 0, 0.0, out, kl, 0, 1);
    };
    // Qk is kept for a redo; the reorthogonalisation against earlier levels
    // works in place, so from the second level on pass 0 runs on a copy
    if (k > 0) {
      c.d2d(Ak, Qk, (size_t)M * kl);
      pass(Ak, Qc, sti + 1);
    } else {
      pass(Qk, Qc, sti + 1);
    }
    pass(Qc, Ak, sti + 2);
    const bool more = k + kl < kmax;  // columns left for a further level
    if (more) {
      // deflation: Work = A - Q Q^T A, ||Work||^2 (and ||A||^2 once)
      copy2d(c.s, M, kl, Ak, kl, Q + k, kmax);
      const int kn = k + kl;
      gemm<double>(c.s, OpT, OpN, kn, n, M, 1.0, Q, kmax, 0, Ain, n, 0, 0.0, C, n, 0, 1);
      c.d2d(Work, Ain, (size_t)M * n);
      gemm<double>(c.s, OpN, OpN, M, n, kn, -1.0, Q, kmax, 0, C, n, 0, 1.0, Work, n, 0, 1);
      dot_device(c.s, Work, Work, (long)M * n, partial, st + 1);
      if (normA2 < 0.0) dot_device(c.s, Ain, Ain, (long)M * n, partial, st);
    }
    c.d2h(reinterpret_cast<unsigned char*>(&hst), reinterpret_cast<const unsigned char*>(st), sizeof(hst));
    if (hst.cnt[1] == kl && hst.cnt[2] == kl) {
      if (!more) {
        copy2d(c.s, M, kl, Ak, kl, Q + k, kmax);
        k += kl;
        break;  // full rank: nothing left to represent
      }
      k += kl;
      if (normA2 < 0.0) {
        normA2 = hst.nrm[0];
        T2S2_CHECK(std::isfinite(normA2), "dcholqr: non-finite input");
      }
      Wk = Work;
      if (hst.nrm[1] <= drop * drop * normA2) break;
      continue;
    }
    // ---- a pass lost a column: redo the passes one at a time from Qk
    double* qa = Qk;
    double* qb = Ak;
    for (int p = 0; p < 2; ++p) {
      if (k > 0) {
        gemm<double>(c.s, OpT, OpN, k, kl, M, 1.0, Q, kmax, 0, qa, kl, 0, 0.0, C, kl, 0, 1);
        gemm<double>(c.s, OpN, OpN, M, kl, k, -1.0, Q, kmax, 0, C, kl, 0, 1.0, qa, kl, 0, 1);
      }
      gemm<double>(c.s, OpT, OpN, kl, kl, M, 1.0, qa, kl, 0, qa, kl, 0, 0.0, G, kl, 0, 1);
      chol_skip(c.s, kl, G, R11, pmask, sti + 1, 1e-14);
      int k2 = 0;
      c.d2h(&k2, sti + 1, 1);
      if (k2 < kl) {
        // a column became dependent after reorthogonalisation: keep the rest
        std::vector<int> m2(kl), id2;
        c.d2h(m2.data(), pmask, kl);
        for (int j = 0; j < kl; ++j)
          if (m2[j]) id2.push_back(j);
        if (id2.empty()) { kl = 0; break; }
        c.h2d(idx, id2.data(), id2.size());
        gather_cols(c.s, M, (int)id2.size(), qa, kl, idx, qb, (long)id2.size());
        kl = (int)id2.size();
        std::swap(qa, qb);
        --p;  // redo this pass on the reduced block
        continue;
      }
      trtri_upper(c.s, kl, R11, R11i);
      gemm<double>(c.s, OpN, OpN, M, kl, kl, 1.0, qa, kl, 0, R11i, kl, 0, 0.0, qb, kl, 0, 1);
      std::swap(qa, qb);
    }
    if (kl == 0) break;
    copy2d(c.s, M, kl, qa, kl, Q + k, kmax);
    k += kl;
    if (k >= kmax) break;  // full rank: nothing left to represent
    // deflate: Work = A - Q Q^T A
    if (normA2 < 0.0) {
      normA2 = c.dot(Ain, Ain, (long)M * n);
      T2S2_CHECK(std::isfinite(normA2), "dcholqr: non-finite input");
    }
    gemm<double>(c.s, OpT, OpN, k, n, M, 1.0, Q, kmax, 0, Ain, n, 0, 0.0, C, n, 0, 1);
    c.d2d(Work, Ain, (size_t)M * n);
    gemm<double>(c.s, OpN, OpN, M, n, k, -1.0, Q, kmax, 0, C, n, 0, 1.0, Work, n, 0, 1);
    Wk = Work;
    const double rem = c.dot(Work, Work, (long)M * n);
    if (rem <= drop * drop * normA2) break;
  }
  if (k == 0) {
    // zero matrix (or a non-finite one, which is an error)
    const double a2 = c.dot(Ain, Ain, (long)M * n);
    T2S2_CHECK(std::isfinite(a2), "dcholqr: non-finite input");
    return 0;
  }
  gemm<double>(c.s, OpT, OpN, k, n, M, 1.0, Q, kmax, 0, Ain, n, 0, 0.0, Rout, n, 0, 1);
  copy2d(c.s, M, k, Q, kmax, Qout, k);
  return k;
}

// ------------------------------------------------------------ truncated SVD
int trunc_svd(const Ctx& c, int M, int n, const double* A, long lda, double delta, int rmax, double* U, double* W,
              std::vector<double>* sigma_out, double* tail_out) {
  Scratch& S = *c.sc;
  const int kmax = std::min(M, n);
  double* Q = S.get<double>("ts.Q", (size_t)M * kmax);
  double* R = S.get<double>("ts.R", (size_t)kmax * n);
  int k = dcholqr(c, M, n, A, lda, Q, R, 1e-15);
  if (k == 0) {
    // zero matrix: rank 1 with the first unit vector
    fill(c.s, U, M, 0.0);
    const double one = 1.0;
    c.h2d(U, &one, 1);
    fill(c.s, W, n, 0.0);
    c.sync();
    if (sigma_out) sigma_out->assign(1, 0.0);
    if (tail_out) *tail_out = 0.0;
    return 1;
  }
  double* JT = S.get<double>("ts.JT", (size_t)k * k);
  double* J = S.get<double>("ts.J", (size_t)k * k);
  double* Wt = S.get<double>("ts.Wt", (size_t)k * n);
  // sigma (k doubles) and the Jacobi info (k + 1 ints) share one buffer, so
  // one copy returns both
  double* sig = S.get<double>("ts.sig", (size_t)k + (k + 2) / 2 + 1);
  int* info = reinterpret_cast<int*>(sig + k);
  const int max_sw = jacobi_sweep_limit();
  jacobi_rows(c.s, k, n, R, JT, J, Wt, sig, info, max_sw);
  std::vector<double> hsi((size_t)k + 1);
  c.d2h(hsi.data(), sig, (size_t)k + 1);
  int sweeps_used = 0;
  std::memcpy(&sweeps_used, hsi.data() + k, sizeof(int));
  if (sweeps_used >= max_sw)
    throw Error(5, "truncated SVD: one-sided Jacobi did not converge within " + std::to_string(max_sw) +
                       " sweeps (k = " + std::to_string(k) + ")");
  std::vector<double> hs(hsi.begin(), hsi.begin() + k);
  // smallest r with tail(r) = sqrt(sum_{j >= r} s_j^2) <= delta
  std::vector<double> tail(k + 1, 0.0);
  for (int j = k - 1; j >= 0; --j) tail[j] = tail[j + 1] + hs[j] * hs[j];
  int r = k;
  for (int j = 1; j <= k; ++j)
    if (std::sqrt(tail[j]) <= delta) { r = j; break; }
  r = std::max(1, std::min(r, std::min(rmax, k)));
  gemm<double>(c.s, OpN, OpN, M, r, k, 1.0, Q, k, 0, J, k, 0, 0.0, U, r, 0, 1);
  c.d2d(W, Wt, (size_t)r * n);
  if (sigma_out) *sigma_out = hs;
  if (tail_out) *tail_out = std::sqrt(tail[r]);
  return r;
}

// ------------------------------------------------------------ eigen / Schur
void hessenberg(const Ctx& c, int n, double* A, double* QT) {
  Scratch& S = *c.sc;
  if (hessenberg_fits_lds(n, (int)sizeof(double))) {
    double* work = S.get<double>("hq.work", 2 * (size_t)n);
    hessenberg(c.s, n, A, QT, work);
    return;
  }
  // H in global memory; Q^T = I - V W^T, W = V T, T^{-1} = striu(V^T V) + diag(1/beta)
  double* V = S.get<double>("hq.V", (size_t)n * n);
  double* beta = S.get<double>("hq.beta", n);
  double* G = S.get<double>("hq.G", (size_t)n * n);
  double* T = S.get<double>("hq.T", (size_t)n * n);
  double* W = S.get<double>("hq.W", (size_t)n * n);
  hessenberg_global(c.s, n, A, V, beta);
  gemm<double>(c.s, OpT, OpN, n, n, n, 1.0, V, n, 0, V, n, 0, 0.0, G, n, 0, 1);
  hess_tinv(c.s, n, G, beta, W);
  trtri_upper(c.s, n, W, T);
  gemm<double>(c.s, OpN, OpN, n, n, n, 1.0, V, n, 0, T, n, 0, 0.0, W, n, 0, 1);
  identity(c.s, n, QT);
  gemm<double>(c.s, OpN, OpT, n, n, n, -1.0, V, n, 0, W, n, 0, 1.0, QT, n, 0, 1);
}

// real upper Hessenberg H = Q^T A Q (row-major) with QT = Q^T (overwritten)
// -> complex Schur form A = Z T Z^H, ZT = Z^T
static void schur_from_hess(const Ctx& c, int n, const double* H, double* QT, double2* ZT, double2* T) {
  Scratch& S = *c.sc;
  double* Hw = S.get<double>("eig.Hw", (size_t)n * n);
  double* Tr = S.get<double>("eig.Tr", (size_t)n * n);
  int* info = S.get<int>("eig.info", 1);
  int* bstart = S.get<int>("eig.bstart", n);
  double2* U = S.get<double2>("eig.U2", 2 * (size_t)n);
  schur_francis(c.s, n, H, Hw, QT, Tr, info);
  flag_francis(c, info);
  rsf2csf(c.s, n, Tr, QT, T, ZT, bstart, U);
}

void schur_real(const Ctx& c, int n, const double* A, double2* ZT, double2* T) {
  Scratch& S = *c.sc;
  double* H = S.get<double>("eig.H", (size_t)n * n);
  double* QT = S.get<double>("eig.QT", (size_t)n * n);
  c.d2d(H, A, (size_t)n * n);
  hessenberg(c, n, H, QT);
  schur_from_hess(c, n, H, QT, ZT, T);
}

// complex Schur form -> eigenvectors V = Z Y (Y unit upper triangular,
// T Y = Y diag(T)), V^{-1} = Y^{-1} Z^H, eigenvalues diag(T)
static void eig_from_schur(const Ctx& c, int n, const double2* ZT, const double2* T, double2* lam, double2* V,
                           double2* Vinv) {
  Scratch& S = *c.sc;
  double2* Y = S.get<double2>("eig.Y", (size_t)n * n);
  double2* Yi = S.get<double2>("eig.Yi", (size_t)n * n);
  trevec(c.s, n, T, Y);
  trtri_upper(c.s, n, Y, Yi);
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  gemm<double2>(c.s, OpT, OpN, n, n, n, one, ZT, n, 0, Y, n, 0, zero, V, n, 0, 1);
  gemm<double2>(c.s, OpN, OpR, n, n, n, one, Yi, n, 0, ZT, n, 0, zero, Vinv, n, 0, 1);
  diag_complex(c.s, n, T, n, lam);
}

void eig_nonsym(const Ctx& c, int n, const double* A, double2* lam, double2* V, double2* Vinv) {
  Scratch& S = *c.sc;
  double2* ZT = S.get<double2>("eig.ZT", (size_t)n * n);
  double2* T = S.get<double2>("eig.T", (size_t)n * n);
  schur_real(c, n, A, ZT, T);
  eig_from_schur(c, n, ZT, T, lam, V, Vinv);
}

void eig_from_hessenberg(const Ctx& c, int n, const double* Hc, const double* QT, double2* lam, double2* V,
                         double2* Vinv) {
  Scratch& S = *c.sc;
  double* H = S.get<double>("eig.H", (size_t)n * n);
  double* Q = S.get<double>("eig.QT", (size_t)n * n);
  double2* ZT = S.get<double2>("eig.ZT", (size_t)n * n);
  double2* T = S.get<double2>("eig.T", (size_t)n * n);
  transpose(c.s, n, n, Hc, n, H, n);
  c.d2d(Q, QT, (size_t)n * n);
  schur_from_hess(c, n, H, Q, ZT, T);
  eig_from_schur(c, n, ZT, T, lam, V, Vinv);
}

void eig_nonsym(const Ctx& c, int n, const double* A, float2* lam, float2* V, float2* Vinv) {
  Scratch& S = *c.sc;
  float* H = S.get<float>("eig32.H", (size_t)n * n);
  float* QT = S.get<float>("eig32.QT", (size_t)n * n);
  float* work = S.get<float>("eig32.work", 2 * (size_t)n);
  float* Hw = S.get<float>("eig32.Hw", (size_t)n * n);
  float* Tr = S.get<float>("eig32.Tr", (size_t)n * n);
  int* info = S.get<int>("eig32.info", 1);
  int* bstart = S.get<int>("eig32.bstart", n);
  float2* U = S.get<float2>("eig32.U2", 2 * (size_t)n);
  float2* ZT = S.get<float2>("eig32.ZT", (size_t)n * n);
  float2* T = S.get<float2>("eig32.T", (size_t)n * n);
  float2* Y = S.get<float2>("eig32.Y", (size_t)n * n);
  float2* Yi = S.get<float2>("eig32.Yi", (size_t)n * n);
  if (hessenberg_fits_lds(n, (int)sizeof(float))) {
    to_float(c.s, A, H, (long)n * n);
    hessenberg(c.s, n, H, QT, work);
  } else {
    // beyond the FP32 LDS size: FP64 reduction, rounded to FP32
    double* Hd = S.get<double>("eig32.Hd", (size_t)n * n);
    double* QTd = S.get<double>("eig32.QTd", (size_t)n * n);
    c.d2d(Hd, A, (size_t)n * n);
    hessenberg(c, n, Hd, QTd);
    to_float(c.s, Hd, H, (long)n * n);
    to_float(c.s, QTd, QT, (long)n * n);
  }
  schur_francis(c.s, n, H, Hw, QT, Tr, info);
  flag_francis(c, info);
  rsf2csf(c.s, n, Tr, QT, T, ZT, bstart, U);
  trevec(c.s, n, T, Y);
  trtri_upper(c.s, n, Y, Yi);
  const float2 one = make_float2(1.0f, 0.0f), zero = make_float2(0.0f, 0.0f);
  gemm<float2>(c.s, OpT, OpN, n, n, n, one, ZT, n, 0, Y, n, 0, zero, V, n, 0, 1);
  gemm<float2>(c.s, OpN, OpR, n, n, n, one, Yi, n, 0, ZT, n, 0, zero, Vinv, n, 0, 1);
  diag_complex(c.s, n, T, n, lam);
}

}  // namespace t2s2
