// C ABI of libt2s2 (declared in include/t2s2.h).  Argument checks, error
// translation and marshalling only; the work happens in solver.hip.
#include "../../include/t2s2.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "cross.h"
#include "readback.h"
#include "mlp.h"
#include "solver.h"
#include "sources.h"
#include "spectral_host.h"

struct t2s2_mlp {
  t2s2::Mlp* N = nullptr;
};

struct t2s2_problem {
  t2s2::Problem* P = nullptr;
  std::vector<int> n, R;
  std::vector<double*> cores;
};

namespace t2s2 {
void timing_set(bool on);
void timing_select(unsigned mask);
void timing_read(int cls, double* ms, long* launches, double* bytes, double* flops);
static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace t2s2

namespace {

template <class F>
int guarded(F&& f) {
  try {
    t2s2::set_last_error("");
    return f();
  } catch (const t2s2::Error& e) {
    t2s2::set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    t2s2::set_last_error("host allocation failed");
    return T2S2_ENOMEM;
  } catch (const std::exception& e) {
    t2s2::set_last_error(e.what());
    return T2S2_EINVAL;
  }
}

t2s2::DTT to_dtt(const t2s2_tt* t) {
  T2S2_CHECK(t && t->d >= 1 && t->d <= T2S2_MAX_DIM && t->n && t->ranks && t->cores, "invalid TT descriptor");
  t2s2::DTT x;
  x.d = t->d;
  x.n.assign(t->n, t->n + t->d);
  x.r.assign(t->ranks, t->ranks + t->d + 1);
  x.c.assign(t->cores, t->cores + t->d);
  T2S2_CHECK(x.r[0] == 1 && x.r[x.d] == 1, "TT boundary ranks must be 1");
  for (int l = 0; l < x.d; ++l) {
    T2S2_CHECK(x.n[l] >= 1 && x.r[l + 1] >= 1, "TT sizes and ranks must be positive");
    T2S2_CHECK(x.c[l] != nullptr, "TT core pointer is NULL");
  }
  return x;
}

t2s2::Ctx ctx_for(t2s2_problem* p, void* stream) {
  t2s2::Ctx c;
  c.s = static_cast<hipStream_t>(stream);
  c.sc = &p->P->sc;
  return c;
}

t2s2::SolveOptions parse_options(const t2s2_options* opts) {
  t2s2::SolveOptions o;
  if (opts) {
    T2S2_CHECK(std::isfinite(opts->tol) && opts->tol > 0.0 && std::isfinite(opts->target), "bad tolerances");
    T2S2_CHECK(opts->max_sweeps >= 1 && opts->kick >= 0 && opts->init_rank >= 1, "bad sweep/kick/rank options");
    o.tol = opts->tol;
    o.target = opts->target;
    o.max_sweeps = opts->max_sweeps;
    o.kick = opts->kick;
    o.rank_cap = opts->rank_cap;
    o.init_rank = opts->init_rank;
    o.seed = opts->seed;
    o.check_every = opts->check_every;
    o.verbose = opts->verbose;
    T2S2_CHECK(opts->precision == T2S2_PRECISION_FP64 || opts->precision == T2S2_PRECISION_MIXED,
               "precision must be T2S2_PRECISION_FP64 or T2S2_PRECISION_MIXED");
    o.precision = opts->precision;
    o.warm_judge = opts->warm_judge;
    o.overlap = opts->overlap;
  }
  return o;
}

// a TT of the problem's interior grid within the rank cap (checked before any device copy)
t2s2::DTT interior_tt(t2s2_problem* p, const t2s2_tt* t, int cap, const char* what) {
  t2s2::DTT x = to_dtt(t);
  T2S2_CHECK(x.d == p->P->d, std::string(what) + " has the wrong dimension");
  for (int l = 0; l < x.d; ++l) {
    T2S2_CHECK(x.n[l] == p->P->m[l], std::string(what) + " mode sizes must be N_l - 2");
    T2S2_CHECK(x.r[l + 1] <= cap, std::string(what) + " ranks exceed the rank cap");
  }
  return x;
}

void fill_report(t2s2_report* rep, const t2s2::SolveReport& r, int st, int d, int precision) {
  if (!rep) return;
  std::memset(rep, 0, sizeof(*rep));
  rep->status = st == 0 ? T2S2_OK : T2S2_ENOTCONV;
  rep->sweeps = r.sweeps;
  rep->max_rank = r.max_rank;
  for (int l = 0; l <= d && l <= T2S2_MAX_DIM; ++l) rep->ranks[l] = r.ranks[l];
  rep->residual = r.residual;
  rep->time_ms = r.time_ms;
  const int h = std::min<int>((int)r.hist_res.size(), T2S2_MAX_HISTORY);
  rep->history_len = h;
  rep->precision = precision;
  rep->local_systems = r.local_systems;
  rep->refinement_steps = r.refinement_steps;
  rep->fp64_fallbacks = r.fp64_fallbacks;
  rep->warm_start_used = r.warm_start_used;
  rep->warm_residual = r.warm_residual;
  rep->cold_residual = r.cold_residual;
  rep->refinement_capped = r.refinement_capped;
  rep->max_eig_cond = r.max_eig_cond;
  for (int i = 0; i < T2S2_PHASES; ++i) rep->phase_ms[i] = r.phase_ms[i];
  for (int i = 0; i < h; ++i) {
    rep->history_residual[i] = r.hist_res[i];
    rep->history_local[i] = r.hist_local[i];
    rep->history_max_rank[i] = r.hist_rank[i];
    rep->history_time_ms[i] = r.hist_time[i];
  }
}

// One solve on stream s; throws on argument or runtime errors, returns
// T2S2_OK or T2S2_ENOTCONV.  mol_u: a time step from u (then g and x0 are NULL).
int solve_one(t2s2_problem* p, const t2s2_tt* f, const t2s2_tt* g, const t2s2_tt* x0, const t2s2_options* opts,
              t2s2_tt* x_out, t2s2_report* rep, hipStream_t stream, const t2s2_tt* mol_u = nullptr) {
  T2S2_CHECK(p && x_out && (f || mol_u), "NULL argument");
  const t2s2::SolveOptions o = parse_options(opts);
  const int cap = o.rank_cap > 0 ? std::min(o.rank_cap, p->P->rank_cap) : p->P->rank_cap;
  t2s2::DTT fd;
  if (f) fd = interior_tt(p, f, 1 << 30, "f");
  T2S2_CHECK(x_out->d == p->P->d && x_out->cores && x_out->ranks, "invalid x_out descriptor");
  t2s2::DTT xd;
  xd.d = p->P->d;
  xd.n = p->P->m;
  xd.r.assign(xd.d + 1, 1);
  xd.c.assign(x_out->cores, x_out->cores + xd.d);
  t2s2::Ctx c = ctx_for(p, stream);
  t2s2::SolveReport r;
  int st;
  if (mol_u) {
    const t2s2::DTT ud = interior_tt(p, mol_u, cap, "u");
    st = t2s2::mol_step(*p->P, c, ud, f ? &fd : nullptr, o, xd, r);
  } else {
    t2s2::DTT x0d;
    const t2s2::DTT* x0p = nullptr;
    if (x0) {
      x0d = interior_tt(p, x0, cap, "x0");
      x0p = &x0d;
    }
    if (g) {
      t2s2::DTT gd = to_dtt(g);
      T2S2_CHECK(gd.d == p->P->d, "g has the wrong dimension");
      for (int l = 0; l < gd.d; ++l) T2S2_CHECK(gd.n[l] == p->P->N[l], "g mode sizes must be N_l (GLL grid)");
      t2s2::DTT bd;
      t2s2::lift_rhs(*p->P, c, fd, gd, bd, cap);
      fd = bd;
    }
    st = t2s2::solve(*p->P, c, fd, x0p, o, xd, r);
  }
  for (int l = 0; l <= xd.d; ++l) x_out->ranks[l] = xd.r[l];
  fill_report(rep, r, st, xd.d, o.precision);
  if (st != 0) t2s2::set_last_error("tolerance not met within max_sweeps");
  return st == 0 ? T2S2_OK : T2S2_ENOTCONV;
}

}  // namespace

extern "C" {

const char* t2s2_last_error(void) { return t2s2::g_last_error.c_str(); }

int t2s2_nodes(int N, double eps, double beta, int scheme, double* gll_out, double* colloc_out) {
  return guarded([&] {
    T2S2_CHECK(N >= 3 && N <= 257, "N must be in [3, 257]");
    T2S2_CHECK(std::isfinite(eps) && eps > 0.0 && std::isfinite(beta), "eps must be > 0, beta finite");
    T2S2_CHECK(scheme == 0 || scheme == 1, "scheme must be 0 or 1");
    T2S2_CHECK(gll_out && colloc_out, "output pointers must not be NULL");
    const std::vector<double> x = t2s2::gll_nodes(N - 1);
    const std::vector<double> th = t2s2::colloc_nodes(N - 1, eps, beta, scheme);
    std::memcpy(gll_out, x.data(), N * sizeof(double));
    std::memcpy(colloc_out, th.data(), (N - 2) * sizeof(double));
    return T2S2_OK;
  });
}

int t2s2_matrices_1d(int N, double eps, double beta, int scheme, double* E, double* D1, double* D2) {
  return guarded([&] {
    T2S2_CHECK(N >= 3 && N <= 257, "N must be in [3, 257]");
    T2S2_CHECK(std::isfinite(eps) && eps > 0.0 && std::isfinite(beta), "eps must be > 0, beta finite");
    T2S2_CHECK(scheme == 0 || scheme == 1, "scheme must be 0 or 1");
    T2S2_CHECK(E && D1 && D2, "output pointers must not be NULL");
    const std::vector<double> x = t2s2::gll_nodes(N - 1);
    const std::vector<double> th = t2s2::colloc_nodes(N - 1, eps, beta, scheme);
    t2s2::lagrange_eval(x.data(), N, th.data(), N - 2, E, D1, D2);
    return T2S2_OK;
  });
}

static t2s2_problem* wrap_problem(t2s2::Problem* P) {
  t2s2_problem* h = new t2s2_problem();
  h->P = P;
  h->n = P->m;
  h->R = P->opL.R;
  h->cores = P->opL.c;
  return h;
}

int t2s2_problem_create(int d, const int* N, double eps, const double* beta, int scheme, int rank_cap,
                        t2s2_problem** out) {
  return guarded([&] {
    T2S2_CHECK(out && N && beta, "NULL argument");
    T2S2_CHECK(d >= 1 && d <= T2S2_MAX_DIM, "d must be in [1, 16]");
    *out = wrap_problem(t2s2::problem_create(d, N, eps, beta, scheme, rank_cap));
    return T2S2_OK;
  });
}

int t2s2_problem_create_reaction(int d, const int* N, double eps, const double* beta, double rho, int scheme,
                                 int rank_cap, t2s2_problem** out) {
  return guarded([&] {
    T2S2_CHECK(out && N && beta, "NULL argument");
    T2S2_CHECK(d >= 1 && d <= T2S2_MAX_DIM, "d must be in [1, 16]");
    *out = wrap_problem(t2s2::problem_create(d, N, eps, beta, scheme, rank_cap, rho));
    return T2S2_OK;
  });
}

int t2s2_problem_create_general(int d, const int* N, const int* kind, double eps, const double* beta_coef,
                                const int* nbeta, double rho, double T, int scheme, int rank_cap,
                                t2s2_problem** out) {
  return guarded([&] {
    T2S2_CHECK(out && N && kind && beta_coef && nbeta, "NULL argument");
    T2S2_CHECK(d >= 1 && d <= T2S2_MAX_DIM, "d must be in [1, 16]");
    *out = wrap_problem(t2s2::problem_create_general(d, N, kind, eps, beta_coef, nbeta, rho, T, scheme, rank_cap));
    return T2S2_OK;
  });
}

int t2s2_mol_create(int d, const int* N, double eps, const double* beta, double rho, double dt, double theta,
                    int scheme, int rank_cap, t2s2_problem** out) {
  return guarded([&] {
    T2S2_CHECK(out && N && beta, "NULL argument");
    T2S2_CHECK(d >= 1 && d <= T2S2_MAX_DIM, "d must be in [1, 16]");
    *out = wrap_problem(t2s2::mol_create(d, N, eps, beta, rho, dt, theta, scheme, rank_cap));
    return T2S2_OK;
  });
}

int t2s2_mol_step(t2s2_problem* p, const t2s2_tt* u, const t2s2_tt* b, const t2s2_options* opts,
                  t2s2_tt* u_next, t2s2_report* rep, void* stream) {
  return guarded([&] {
    T2S2_CHECK(u, "NULL argument");
    return solve_one(p, b, nullptr, nullptr, opts, u_next, rep, static_cast<hipStream_t>(stream), u);
  });
}

int t2s2_problem_destroy(t2s2_problem* p) {
  return guarded([&] {
    if (!p) return T2S2_OK;
    delete p->P;
    delete p;
    return T2S2_OK;
  });
}

int t2s2_problem_operator(const t2s2_problem* p, t2s2_ttm* out) {
  return guarded([&] {
    T2S2_CHECK(p && out, "NULL argument");
    out->d = p->P->d;
    out->n = p->n.data();
    out->ranks = p->R.data();
    out->cores = p->cores.data();
    return T2S2_OK;
  });
}

int t2s2_problem_colloc(const t2s2_problem* p, int l, double* theta_out) {
  return guarded([&] {
    T2S2_CHECK(p && theta_out, "NULL argument");
    T2S2_CHECK(l >= 0 && l < p->P->d, "dimension index out of range");
    const auto& th = p->P->theta[l];
    std::memcpy(theta_out, th.data(), th.size() * sizeof(double));
    return T2S2_OK;
  });
}

static int tt_matvec_common(const t2s2_ttm* A, const t2s2_tt* x, t2s2_tt* y, void* stream, bool noalloc) {
  T2S2_CHECK(A && A->cores && A->ranks && A->n, "invalid TT-matrix descriptor");
  t2s2::DTT xd = to_dtt(x);
  T2S2_CHECK(y && y->cores && y->ranks && y->d == xd.d, "invalid output TT descriptor");
  T2S2_CHECK(A->d == xd.d, "operator and vector dimensions differ");
  t2s2::DTTM Ad;
  Ad.d = A->d;
  Ad.n.assign(A->n, A->n + A->d);
  Ad.R.assign(A->ranks, A->ranks + A->d + 1);
  Ad.c.assign(A->cores, A->cores + A->d);
  T2S2_CHECK(Ad.R[0] == 1 && Ad.R[Ad.d] == 1, "operator boundary ranks must be 1");
  for (int l = 0; l < xd.d; ++l) {
    T2S2_CHECK(Ad.n[l] == xd.n[l] && Ad.n[l] <= 64, "mode sizes must match, <= 64");
    T2S2_CHECK(Ad.R[l + 1] >= 1 && Ad.c[l] != nullptr, "operator ranks must be positive, cores non-NULL");
  }
  t2s2::DTT yd;
  yd.c.assign(y->cores, y->cores + y->d);
  t2s2::Ctx c;
  c.s = static_cast<hipStream_t>(stream);
  if (noalloc) t2s2::tt_matvec_noalloc(c, Ad, xd, yd);
  else t2s2::tt_matvec(c, Ad, xd, yd);
  for (int l = 0; l <= xd.d; ++l) y->ranks[l] = yd.r[l];
  return T2S2_OK;
}

int t2s2_tt_matvec(const t2s2_ttm* A, const t2s2_tt* x, t2s2_tt* y, void* stream) {
  return guarded([&] { return tt_matvec_common(A, x, y, stream, false); });
}

int t2s2_tt_matvec_noalloc(const t2s2_ttm* A, const t2s2_tt* x, t2s2_tt* y, void* stream) {
  return guarded([&] { return tt_matvec_common(A, x, y, stream, true); });
}

int t2s2_tt_fiber(t2s2_problem* p, const t2s2_tt* x, int l, const int* idx, double* out, void* stream) {
  return guarded([&] {
    T2S2_CHECK(p && idx && out, "NULL argument");
    const t2s2::DTT xd = to_dtt(x);
    T2S2_CHECK(l >= 0 && l < xd.d, "mode index out of range");
    std::vector<int> iv(idx, idx + xd.d);
    t2s2::Ctx c = ctx_for(p, stream);
    t2s2::tt_fiber(c, xd, l, iv, out);
    return T2S2_OK;
  });
}

int t2s2_tt_norm(t2s2_problem* p, const t2s2_tt* x, double* out, void* stream) {
  return guarded([&] {
    T2S2_CHECK(p && out, "NULL argument");
    t2s2::DTT xd = to_dtt(x);
    t2s2::Ctx c = ctx_for(p, stream);
    *out = t2s2::tt_norm(c, xd);
    return T2S2_OK;
  });
}

int t2s2_tt_residual_norm(t2s2_problem* p, const t2s2_tt* x, const t2s2_tt* f, double* out, void* stream) {
  return guarded([&] {
    T2S2_CHECK(p && out, "NULL argument");
    t2s2::DTT xd = to_dtt(x), fd = to_dtt(f);
    T2S2_CHECK(xd.d == p->P->d && fd.d == p->P->d, "dimension mismatch with the problem");
    for (int l = 0; l < xd.d; ++l)
      T2S2_CHECK(xd.n[l] == p->P->m[l] && fd.n[l] == p->P->m[l], "mode sizes must be N_l - 2");
    t2s2::Ctx c = ctx_for(p, stream);
    *out = t2s2::tt_residual_norm(*p->P, c, xd, fd);
    return T2S2_OK;
  });
}

int t2s2_tt_round(t2s2_problem* p, t2s2_tt* x, double tol, int rmax, void* stream) {
  return guarded([&] {
    T2S2_CHECK(p, "NULL argument");
    T2S2_CHECK(std::isfinite(tol) && tol >= 0.0 && rmax >= 1, "tol must be >= 0 and rmax >= 1");
    t2s2::DTT xd = to_dtt(x);
    t2s2::Ctx c = ctx_for(p, stream);
    t2s2::tt_round(c, xd, tol, rmax);
    c.sync();
    for (int l = 0; l <= xd.d; ++l) x->ranks[l] = xd.r[l];
    return T2S2_OK;
  });
}

int t2s2_local_solve(int r1, int m, int r2, const double* Lint, const double* K, const double* Rint, const double* g,
                     double* u, int method, void* stream) {
  return guarded([&] {
    T2S2_CHECK(Lint && K && Rint && g && u, "NULL argument");
    t2s2::Scratch sc;
    t2s2::Ctx c;
    c.s = static_cast<hipStream_t>(stream);
    c.sc = &sc;
    t2s2::local_kron_solve(c, r1, m, r2, Lint, K, Rint, g, u, method);
    return T2S2_OK;
  });
}

int t2s2_timing_enable(int on) {
  return guarded([&] {
    t2s2::timing_set(on != 0);
    return T2S2_OK;
  });
}

int t2s2_timing_classes(unsigned int mask) {
  return guarded([&] {
    t2s2::timing_select(mask);
    return T2S2_OK;
  });
}

int t2s2_timing_read(int cls, double* total_ms, long long* launches, double* bytes, double* flops) {
  return guarded([&] {
    T2S2_CHECK(cls >= 0 && cls < t2s2::KC_COUNT, "timing class out of range");
    T2S2_CHECK(total_ms && launches && bytes && flops, "NULL argument");
    long n = 0;
    t2s2::timing_read(cls, total_ms, &n, bytes, flops);
    *launches = n;
    return T2S2_OK;
  });
}

const char* t2s2_timing_class_name(int cls) {
  static const char* names[] = {"gemm_f64", "gemm_c128", "ttm_matvec", "schur_qr", "hessenberg", "jacobi_svd",
                                "cholesky", "trtri", "trevec", "kron_trisolve", "hess_solve", "other"};
  if (cls < 0 || cls >= t2s2::KC_COUNT) return "";
  return names[cls];
}

void t2s2_default_options(t2s2_options* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->target = 1e-8;
  o->max_sweeps = 40;
  o->kick = 8;
  o->rank_cap = 0;
  o->init_rank = 2;
  o->seed = 0;
  o->check_every = 1;
  o->verbose = 0;
  o->precision = T2S2_PRECISION_FP64;
  o->warm_judge = 0;
  o->overlap = 1;
}

int t2s2_solve(t2s2_problem* p, const t2s2_tt* f, const t2s2_tt* g, const t2s2_tt* x0, const t2s2_options* opts,
               t2s2_tt* x_out, t2s2_report* rep, void* stream) {
  return guarded([&] { return solve_one(p, f, g, x0, opts, x_out, rep, static_cast<hipStream_t>(stream)); });
}

int t2s2_debug_gemm(int variant, int opA, int opB, int M, int N, int K, int batch, double alpha, const double* A,
                    long long lda, long long sA, const double* B, long long ldb, long long sB, double beta,
                    double* C, long long ldc, long long sC, void* stream) {
  return guarded([&] {
    T2S2_CHECK(variant >= -1 && variant <= 1, "variant must be -1, 0 or 1");
    T2S2_CHECK((opA == 0 || opA == 1) && (opB == 0 || opB == 1), "opA, opB must be 0 (N) or 1 (T)");
    T2S2_CHECK(M >= 1 && N >= 1 && K >= 1 && batch >= 1 && A && B && C, "bad sizes or NULL pointer");
    T2S2_CHECK(lda >= (opA == 0 ? K : M) && ldb >= (opB == 0 ? N : K) && ldc >= N, "leading dimensions too small");
    t2s2::gemm_force_variant(variant);
    try {
      t2s2::gemm<double>(static_cast<hipStream_t>(stream), static_cast<t2s2::Op>(opA), static_cast<t2s2::Op>(opB), M,
                         N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, false);
    } catch (...) {
      t2s2::gemm_force_variant(-1);
      throw;
    }
    t2s2::gemm_force_variant(-1);
    return T2S2_OK;
  });
}

const char* t2s2_gemm_tune_source(void) { return t2s2::gemm_tune_source(); }

int t2s2_debug_readback(const void* dev, void* host, long long bytes, void* stream) {
  return guarded([&] {
    T2S2_CHECK(bytes >= 0 && (bytes == 0 || (dev && host)), "t2s2_debug_readback: NULL pointer or negative size");
    t2s2::host_read(static_cast<hipStream_t>(stream), host, dev, (size_t)bytes);
    return T2S2_OK;
  });
}

int t2s2_debug_iteration_limits(int francis_steps, int jacobi_sweeps) {
  return guarded([&] {
    T2S2_CHECK(francis_steps >= 0 && jacobi_sweeps >= 0, "iteration limits must be >= 0");
    t2s2::set_iteration_limits(francis_steps, jacobi_sweeps);
    return T2S2_OK;
  });
}

int t2s2_solve_batched(int count, t2s2_problem* const* probs, const t2s2_tt* const* f, const t2s2_tt* const* g,
                       const t2s2_tt* const* x0, const t2s2_options* opts, t2s2_tt* const* x_out,
                       t2s2_report* reps, int workers, void* stream) {
  return guarded([&] {
    T2S2_CHECK(count >= 0, "count must be >= 0");
    if (count == 0) return T2S2_OK;
    T2S2_CHECK(probs && f && x_out, "NULL argument");
    T2S2_CHECK(workers >= 0 && workers <= 64, "workers must be in [0, 64]");
    std::vector<t2s2_problem*> ps(probs, probs + count);
    for (int i = 0; i < count; ++i) T2S2_CHECK(ps[i] && f[i] && x_out[i], "NULL problem, f or x_out entry");
    {
      std::vector<t2s2_problem*> sorted = ps;
      std::sort(sorted.begin(), sorted.end());
      T2S2_CHECK(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(),
                 "each instance needs its own t2s2_problem");
    }
    const int nw = std::min(count, workers > 0 ? workers : 16);
    // longest first: cost ~ sum_l m_l * log10(10 / eps) (more unknowns per
    // core and thinner layers need more rank)
    std::vector<int> order(count);
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) {
      order[i] = i;
      double sm = 0.0;
      for (int m : ps[i]->P->m) sm += m;
      cost[i] = sm * std::log10(10.0 / ps[i]->P->eps);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    int device = 0;
    T2S2_HIP(hipGetDevice(&device));
    // every worker stream starts after the work already queued on stream
    hipEvent_t ready;
    T2S2_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    T2S2_HIP(hipEventRecord(ready, static_cast<hipStream_t>(stream)));
    std::vector<int> codes(count, T2S2_OK);
    std::vector<std::string> msgs(count);
    std::atomic<int> next{0};
    auto work = [&]() {
      hipStream_t s = nullptr;
      std::string fail;
      if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
          hipStreamWaitEvent(s, ready, 0) != hipSuccess)
        fail = "worker stream set-up failed";
      // outgrown scratch blocks are freed after the batch, not between the
      // instances (a hipFree would wait for every other worker's queue)
      t2s2::defer_scratch_release(true);
      for (int k = next++; k < count; k = next++) {
        const int i = order[k];
        if (!fail.empty()) {
          codes[i] = T2S2_EHIP;
          msgs[i] = fail;
          continue;
        }
        codes[i] = guarded([&] {
          return solve_one(ps[i], f[i], g ? g[i] : nullptr, x0 ? x0[i] : nullptr, opts, x_out[i],
                           reps ? &reps[i] : nullptr, s);
        });
        if (codes[i] != T2S2_OK) msgs[i] = t2s2_last_error();
      }
      if (s) (void)hipStreamDestroy(s);
    };
    std::vector<std::thread> pool;
    pool.reserve(nw);
    for (int w = 0; w < nw; ++w) pool.emplace_back(work);
    for (auto& t : pool) t.join();
    (void)hipEventDestroy(ready);
    for (int i = 0; i < count; ++i) t2s2::free_retired_scratch(*ps[i]->P);
    // a hard error outranks "not converged"; report the first of the worst
    int worst = T2S2_OK;
    std::string first;
    for (int pass = 0; pass < 2 && worst == T2S2_OK; ++pass)
      for (int i = 0; i < count; ++i) {
        const bool hard = codes[i] != T2S2_OK && codes[i] != T2S2_ENOTCONV;
        if ((pass == 0 && hard) || (pass == 1 && codes[i] == T2S2_ENOTCONV)) {
          worst = codes[i];
          first = "instance " + std::to_string(i) + ": " + msgs[i];
          break;
        }
      }
    if (worst != T2S2_OK) t2s2::set_last_error(first);
    return worst;
  });
}

// ------------------------------------------------------- sources
static int source_common(t2s2_problem* p, int kind, int s, const double* amp, const double* centre,
                         const double* width, t2s2_tt* f_out, void* stream) {
  T2S2_CHECK(p && f_out && f_out->cores && f_out->ranks && f_out->d == p->P->d, "invalid problem or output TT");
  if (kind == 0) T2S2_CHECK(amp && centre && width, "NULL parameter array");
  t2s2::DTT fd;
  fd.c.assign(f_out->cores, f_out->cores + f_out->d);
  t2s2::Ctx c = ctx_for(p, stream);
  t2s2::separable_source(*p->P, c, kind, s, amp, centre, width, fd);
  for (int l = 0; l <= fd.d; ++l) f_out->ranks[l] = fd.r[l];
  c.sync();
  return T2S2_OK;
}

int t2s2_source_gaussians(t2s2_problem* p, int s, const double* amp, const double* centre, const double* width,
                          t2s2_tt* f_out, void* stream) {
  return guarded([&] { return source_common(p, 0, s, amp, centre, width, f_out, stream); });
}

int t2s2_source_cross(t2s2_problem* p, int kind, const double* params, double tol, int r0, int rmax,
                      unsigned long long seed, t2s2_tt* f_out, int* rank_out, double* sample_error_out,
                      void* stream) {
  return guarded([&] {
    T2S2_CHECK(p && params && f_out && f_out->cores && f_out->ranks && f_out->d == p->P->d,
               "invalid problem, parameters or output TT");
    t2s2::CrossFunction fn;
    fn.kind = kind;
    fn.params.assign(params, params + 2 + 2 * p->P->d);
    t2s2::DTT fd;
    fd.c.assign(f_out->cores, f_out->cores + f_out->d);
    t2s2::Ctx c = ctx_for(p, stream);
    const t2s2::CrossInfo info = t2s2::source_cross(*p->P, c, fn, tol, r0, rmax, seed, 1000, fd);
    for (int l = 0; l <= fd.d; ++l) f_out->ranks[l] = fd.r[l];
    if (rank_out) *rank_out = info.rank;
    if (sample_error_out) *sample_error_out = info.sample_error;
    return T2S2_OK;
  });
}

int t2s2_source_manufactured(t2s2_problem* p, t2s2_tt* f_out, void* stream) {
  return guarded([&] {
    T2S2_CHECK(p, "NULL problem");
    return source_common(p, 1, p->P->d, nullptr, nullptr, nullptr, f_out, stream);
  });
}

// ------------------------------------------------------- learned warm start
int t2s2_mlp_create(int n_layers, const int* widths, unsigned long long seed, t2s2_mlp** out) {
  return guarded([&] {
    T2S2_CHECK(out && widths && n_layers >= 1 && n_layers <= 15, "mlp_create: bad arguments");
    *out = nullptr;
    std::vector<int> w(widths, widths + n_layers + 1);
    auto* h = new t2s2_mlp();
    try {
      h->N = t2s2::mlp_create(w, seed);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return T2S2_OK;
  });
}

void t2s2_mlp_destroy(t2s2_mlp* net) {
  if (!net) return;
  delete net->N;
  delete net;
}

int t2s2_mlp_param_count(const t2s2_mlp* net, long long* count) {
  return guarded([&] {
    T2S2_CHECK(net && count, "NULL argument");
    *count = net->N->nparam;
    return T2S2_OK;
  });
}

int t2s2_mlp_get_params(t2s2_mlp* net, float* dst, int which, void* stream) {
  return guarded([&] {
    T2S2_CHECK(net && dst && (which == 0 || which == 1), "mlp_get_params: bad arguments");
    const float* src = which == 0 ? net->N->params : net->N->grad;
    T2S2_HIP(hipMemcpyAsync(dst, src, sizeof(float) * net->N->nparam, hipMemcpyDeviceToDevice,
                            static_cast<hipStream_t>(stream)));
    return T2S2_OK;
  });
}

int t2s2_mlp_set_params(t2s2_mlp* net, const float* src, void* stream) {
  return guarded([&] {
    T2S2_CHECK(net && src, "NULL argument");
    t2s2::Mlp& N = *net->N;
    hipStream_t s = static_cast<hipStream_t>(stream);
    T2S2_HIP(hipMemcpyAsync(N.params, src, sizeof(float) * N.nparam, hipMemcpyDeviceToDevice, s));
    T2S2_HIP(hipMemsetAsync(N.m, 0, sizeof(float) * N.nparam, s));
    T2S2_HIP(hipMemsetAsync(N.v, 0, sizeof(float) * N.nparam, s));
    N.t = 0;
    N.bf16_valid = false;
    return T2S2_OK;
  });
}

int t2s2_mlp_forward(t2s2_mlp* net, int batch, const float* x, float* y, void* stream) {
  return guarded([&] {
    T2S2_CHECK(net && x && y && batch >= 1, "mlp_forward: bad arguments");
    t2s2::mlp_forward(*net->N, static_cast<hipStream_t>(stream), batch, x, y);
    return T2S2_OK;
  });
}

int t2s2_mlp_backward(t2s2_mlp* net, int batch, const float* x, const float* dy, void* stream) {
  return guarded([&] {
    T2S2_CHECK(net && x && dy && batch >= 1, "mlp_backward: bad arguments");
    t2s2::mlp_backward(*net->N, static_cast<hipStream_t>(stream), batch, x, dy);
    return T2S2_OK;
  });
}

int t2s2_mlp_adam_step(t2s2_mlp* net, float lr, float beta1, float beta2, float eps, void* stream) {
  return guarded([&] {
    T2S2_CHECK(net && std::isfinite(lr) && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f,
               "mlp_adam_step: bad arguments");
    t2s2::mlp_adam(*net->N, static_cast<hipStream_t>(stream), lr, beta1, beta2, eps);
    return T2S2_OK;
  });
}

int t2s2_mlp_infer_bf16(t2s2_mlp* net, int batch, const float* x, float* y, void* stream) {
  return guarded([&] {
    T2S2_CHECK(net && x && y && batch >= 1, "mlp_infer_bf16: bad arguments");
    t2s2::mlp_infer_bf16(*net->N, static_cast<hipStream_t>(stream), batch, x, y);
    return T2S2_OK;
  });
}

int t2s2_mlp_train(t2s2_mlp* net, int count, const float* x, const float* targets, int d, const int* n, int rank,
                   int epochs, int batch, float lr, unsigned long long seed, float* epoch_loss, void* stream) {
  return guarded([&] {
    T2S2_CHECK(net && x && targets && n && count >= 1 && epochs >= 0 && batch >= 1 && lr > 0.f,
               "mlp_train: bad arguments");
    const auto h = t2s2::mlp_train(*net->N, static_cast<hipStream_t>(stream), count, x, targets, d, n, rank, epochs,
                                   batch, lr, seed);
    if (epoch_loss) std::copy(h.begin(), h.end(), epoch_loss);
    return T2S2_OK;
  });
}

int t2s2_tt_fit_loss(int batch, int d, const int* n, int rank, const float* pred, const float* target, float* loss,
                     float* dpred, void* stream) {
  return guarded([&] {
    T2S2_CHECK(n && pred && target && loss && dpred && batch >= 0, "tt_fit_loss: bad arguments");
    t2s2::tt_fit_loss(static_cast<hipStream_t>(stream), batch, d, n, rank, pred, target, loss, dpred, 1.0f);
    return T2S2_OK;
  });
}

int t2s2_tt_pack(const t2s2_tt* x, int rank, int canonical, float* out, void* stream) {
  return guarded([&] {
    T2S2_CHECK(out, "NULL argument");
    const t2s2::DTT xd = to_dtt(x);
    t2s2::tt_pack(static_cast<hipStream_t>(stream), xd, rank, canonical ? 1 : 0, out);
    return T2S2_OK;
  });
}

int t2s2_tt_unpack(int d, const int* n, int rank, const float* in, t2s2_tt* x_out, void* stream) {
  return guarded([&] {
    T2S2_CHECK(n && in && x_out && x_out->d == d && x_out->cores && x_out->ranks, "tt_unpack: bad arguments");
    t2s2::DTT xd;
    xd.c.assign(x_out->cores, x_out->cores + d);
    t2s2::tt_unpack(static_cast<hipStream_t>(stream), d, n, rank, in, xd);
    for (int l = 0; l <= d; ++l) x_out->ranks[l] = xd.r[l];
    return T2S2_OK;
  });
}

}  // extern "C"
