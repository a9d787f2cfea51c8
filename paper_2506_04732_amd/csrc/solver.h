// Problem, device TT containers and the TT solver of libt2s2.
#pragma once
#include <vector>

#include "linalg.h"

namespace t2s2 {

// TT vector in device memory; cores[l] is [r[l]][n[l]][r[l+1]] row-major.
struct DTT {
  int d = 0;
  std::vector<int> n, r;
  std::vector<double*> c;
};

// TT-matrix in device memory; cores [R[l]][n[l]][n[l]][R[l+1]].
struct DTTM {
  int d = 0;
  std::vector<int> n, R;
  std::vector<double*> c;
};

struct Problem {
  int d = 0;
  std::vector<int> N, m;        // nodes and interior unknowns per dimension
  double eps = 0.0;
  std::vector<double> beta;
  double rho = 0.0;  // constant reaction of the operator solved (M_l carries rho / d E_l)
  std::vector<int> kind;  // per dimension: 0 space (Dirichlet at both ends), 1 time (initial value)
  double T = 0.0;         // final time of a time dimension (on [0, T])
  // method of lines (theta > 0): the solve operator is A + (1 / (theta dt)) I
  // with A the operator of reaction rho_phys; dMx holds the explicit-part
  // blocks (1/(theta dt d) - (1-theta)/theta rho_phys / d) E_l - (1-theta)/theta M0_l
  double mol_dt = 0.0, mol_theta = 0.0, rho_phys = 0.0;
  std::vector<double*> dMx;
  int scheme = 1;
  int rank_cap = 0;
  int device = 0;
  // host copies of the 1D data (interior blocks, m x m, row-major)
  std::vector<std::vector<double>> gll, theta, E, M, K, Einv;
  // device: original operator (E, M blocks) and the scaled Kronecker sum
  // operator (I, K blocks), both as rank-2 TT-matrices
  DTTM opL, opK;
  std::vector<double*> dK, dEinv;
  // the same blocks on all N_l GLL columns (m_l x N_l, boundary columns
  // included) and on the interior columns (m_l x m_l): the lift of Dirichlet data
  std::vector<double*> dEf, dMf, dEi, dMi;
  std::vector<double2*> dK_ZT, dK_T;  // Schur form of K_l
  std::vector<float2*> dK_ZT32, dK_T32;  // the same rounded to FP32
  std::vector<int> opR;
  Scratch sc;
  // side streams of the solves (eigendecompositions of interfaces, overlapped
  // with the sweep), each with its own scratch; created on first use.
  // side_done[k]: recorded after the last side work of a solve; the next
  // solve waits for it before it rewrites what that work reads
  static constexpr int kSides = 2;
  hipStream_t side[kSides] = {};
  hipEvent_t side_done[kSides] = {};
  Scratch sc_side[kSides];
  ~Problem();
};

struct SolveOptions {
  double tol = 1e-10;
  double target = 1e-8;
  int max_sweeps = 40;
  int kick = 8;
  int rank_cap = 0;
  int init_rank = 2;
  unsigned long long seed = 0;
  int check_every = 1;
  int verbose = 0;
  int precision = 0;  // 0 FP64, 1 mixed (FP32 factors inside FP64 refinement)
  int warm_judge = 0;  // 1: use x0 only if its FP64 residual beats the seeded cold start's
  int overlap = 1;     // FP64: interface eigendecompositions on a side stream (0: on the solve's stream)
};

struct SolveReport {
  int status = 0, sweeps = 0, max_rank = 0;
  std::vector<int> ranks;
  double residual = -1.0, time_ms = 0.0;
  std::vector<double> hist_res, hist_local, hist_time;
  std::vector<int> hist_rank;
  int local_systems = 0, refinement_steps = 0, fp64_fallbacks = 0;
  int refinement_capped = 0;  // local refinements stopped at the step cap above 0.1 tol / sqrt(d)
  double max_eig_cond = 0.0;  // largest ||V||_F ||V^-1||_F of the FP64 interface eigenvector bases
  // device time per phase (events on the solve's stream): 0 set-up (start,
  // orthogonalisation, first interfaces, warm-start judge), 1 local solves,
  // 2 splits (truncated SVD, enrichment, QR), 3 interface updates and
  // factorisations, 4 FP64 residual checks
  double phase_ms[5] = {0, 0, 0, 0, 0};
  int warm_start_used = 0;
  double warm_residual = -1.0, cold_residual = -1.0;
};

Problem* problem_create(int d, const int* N, double eps, const double* beta, int scheme, int rank_cap,
                        double rho = 0.0);
// General problem: per dimension a kind (0 space: Dirichlet data at both
// ends, N_l - 2 unknowns, superconsistent or plain collocation nodes; 1 time
// on [0, T]: the value at t = 0 given, N_l - 1 unknowns collocated at the
// Gauss points), a variable separable advection beta_l(x_l) = sum_k
// c_{l,k} P_k(x_l) (nbeta[l] Legendre coefficients per space dimension,
// concatenated in beta_coef), constant eps and reaction rho.
Problem* problem_create_general(int d, const int* N, const int* kind, double eps, const double* beta_coef,
                                const int* nbeta, double rho, double T, int scheme, int rank_cap);
// A problem for theta-scheme time steps of du/dt + A u = b (A with reaction
// rho): the operator solved per step has reaction rho + 1 / (theta dt).
Problem* mol_create(int d, const int* N, double eps, const double* beta, double rho, double dt, double theta,
                    int scheme, int rank_cap);
// One step: f = (1/(theta dt)) E u - ((1-theta)/theta) (L + rho E) u + b / theta
// (b nullable), rounded at relative 1e-14, then the solve from x0 = u.
int mol_step(Problem& p, const Ctx& c, const DTT& u, const DTT* b, const SolveOptions& o, DTT& x,
             SolveReport& rep);

// y = A x, y's cores preallocated by the caller (ranks R r).
void tt_matvec(const Ctx& c, const DTTM& A, const DTT& x, DTT& y);
// The same with the permuted operator core in a static device array (no
// allocation; R_l n_l^2 R_{l+1} <= tt_matvec_noalloc_capacity() per core,
// n_l <= 64).  Calls that overlap on one GPU share the array and race.
void tt_matvec_noalloc(const Ctx& c, const DTTM& A, const DTT& x, DTT& y);
long tt_matvec_noalloc_capacity();
// out (device, n_l doubles) = the fiber of x along mode l through idx.
void tt_fiber(const Ctx& c, const DTT& x, int l, const std::vector<int>& idx, double* out);
// ||x||_2 (double-double Gram recursion).
double tt_norm(const Ctx& c, const DTT& x);
// ||f - L x|| / ||f|| with the problem's original operator.
double tt_residual_norm(Problem& p, const Ctx& c, const DTT& x, const DTT& f);
// In-place rounding; x's cores must hold the input ranks.
void tt_round(const Ctx& c, DTT& x, double tol, int rmax);
// u = (Lint (+) K (+) Rint)^{-1} g on r1 x m x r2 tensors (device buffers),
// method 0: eigendecompositions of Lint and Rint, 1: Hessenberg form of Lint,
// 2: Hessenberg form of Rint (eigendecomposition of Lint).
void local_kron_solve(const Ctx& c, int r1, int m, int r2, const double* Lint, const double* K, const double* Rint,
                      const double* g, double* u, int method);
// Right-hand side of the interior system for Dirichlet data g (a TT on the
// N_l-point GLL grids; only its boundary values matter):
//   b = f - L_full g + L_int g_int,
// L_full the collocation operator on all GLL columns, g_int the interior
// slices of g.  Exact TT sum (ranks s + 4 s_g), then rounded at relative
// 1e-14 with rank <= rmax; b's cores are scratch of p.
void lift_rhs(Problem& p, const Ctx& c, const DTT& f, const DTT& g, DTT& b, int rmax);
// TT solve of the interior system; x holds the start (or is random) and
// receives the solution; its cores need rank_cap * m * rank_cap doubles.
int solve(Problem& p, const Ctx& c, const DTT& f, const DTT* x0, const SolveOptions& o, DTT& x, SolveReport& rep);

// Scratch blocks outgrown during a solve are normally freed when the solve
// ends (or starts) with no side work queued; each hipFree waits for all work
// on the device.  While concurrent solves run (a batch), the calling thread
// defers those frees (on = true) so that no solve waits for the others'
// queues; free_retired_scratch then frees a problem's deferred blocks.
void defer_scratch_release(bool on);
void free_retired_scratch(Problem& p);

}  // namespace t2s2
