/*
 * t2s2.h -- C ABI of libt2s2, the MI355X (gfx950) tensor-train solver for the
 * superconsistent spectral collocation system of steady advection-diffusion
 * (T^2S^2).
 *
 * Problem (paper: Eq. advection-diffusion with Eq. pblm:time:B):
 *     -eps Lap u + beta . grad u = f   in [-1, 1]^d,   u = g on the boundary,
 * with constant eps > 0 and constant beta in R^d (g = 0 unless Dirichlet
 * data are passed to t2s2_solve).
 *
 * Discretisation (paper: Overview (i)-(iii), Fig. 3):
 *   - N_l nodes per dimension, polynomial degree n_l = N_l - 1; representation
 *     grid = Gauss-Lobatto-Legendre (GLL) nodes (+-1 and the zeros of P_n');
 *   - collocation grid per dimension = superconsistent nodes (scheme SC) or
 *     the interior GLL nodes (scheme PLAIN).  The paper does not print the
 *     superconsistent node formula; this library reads it as: theta_i is the
 *     zero of eps P_n'(x) - beta_l P_n(x) inside the i-th gap (z_i, z_{i+1})
 *     of the zeros z_1 < ... < z_n of P_n (i = 1 .. n-1).  beta_l = 0 gives
 *     the interior GLL nodes;
 *   - interior system  L u = f,  L = sum_l E_1 (x) .. (x) M_l (x) .. (x) E_d,
 *     E_l[j,i] = Lagrange basis i of the GLL grid at theta_j, M_l =
 *     -eps D2_l + beta_l D1_l (first/second derivatives of that basis), all
 *     restricted to interior columns (zero Dirichlet data).  m_l = N_l - 2
 *     unknowns per dimension.
 *
 * Tensor trains (paper: Methods, Eq. TT-format:elementwise and
 * Eq. tt-matrix-format): core l of a TT vector is a C-contiguous FP64 array
 * [r_{l-1}][n_l][r_l] in device memory, r_0 = r_d = 1; the full vector is in
 * C order (index 1 slowest).  TT-matrix cores are [R_{l-1}][n_l (row)][n_l
 * (column)][R_l].  The operator L is held as a rank-2 TT-matrix: first core
 * [M_1 E_1], middle cores [[E 0],[M E]], last core [E_d; M_d].
 *
 * Conventions for every entry point:
 *   - return value is a status code (T2S2_OK on success);
 *   - a failing call leaves a message readable by t2s2_last_error()
 *     (thread-local, valid until the next failing call on that thread);
 *   - "stream" is a hipStream_t passed as void* (NULL = default stream);
 *     device work is enqueued on it; calls that return host scalars
 *     synchronise that stream;
 *   - the caller allocates and owns every input and output buffer (device
 *     buffers for TT cores, host buffers for arrays documented as host);
 *     the library owns only the scratch memory behind a t2s2_problem,
 *     allocated on demand and released by t2s2_problem_destroy;
 *   - calls that share one t2s2_problem must not run concurrently.
 */
#ifndef T2S2_H
#define T2S2_H

#ifdef __cplusplus
extern "C" {
#endif

#define T2S2_OK 0
#define T2S2_EINVAL 1      /* bad argument: sizes, ranks, non-finite data  */
#define T2S2_ENOMEM 2      /* device allocation failed                     */
#define T2S2_ENOTCONV 3    /* solve stopped at max_sweeps above target     */
#define T2S2_EHIP 4        /* HIP runtime error (text in t2s2_last_error)  */
#define T2S2_EFACTOR 5     /* a dense factorisation (Francis QR of an
                              interface or 1D operator, one-sided Jacobi of a
                              truncated SVD) stopped at its iteration limit */

#define T2S2_SCHEME_PLAIN 0
#define T2S2_SCHEME_SC 1

/* Arithmetic of the local solves (t2s2_options.precision).  FP64: local
 * systems are factorised and solved in FP64.  MIXED: the eigen/Schur
 * factorisations of the interface matrices and the complex transforms of
 * the local solve run in FP32, inside FP64 iterative refinement of each
 * local system (FP64 local residual and update); should the FP32 factors
 * contract the residual too slowly, that local system switches to FP64
 * factors.  Truncations, orthogonalisation, interfaces and the global
 * residual test are FP64 in both modes, so the stopping test is the same. */
#define T2S2_PRECISION_FP64 0
#define T2S2_PRECISION_MIXED 1

#define T2S2_MAX_DIM 16
#define T2S2_MAX_HISTORY 128
#define T2S2_PHASES 5

typedef struct t2s2_problem t2s2_problem;

/* TT vector.  n, ranks, cores are host arrays of length d, d+1, d.
 * cores[l] is a device pointer to at least ranks[l]*n[l]*ranks[l+1] doubles
 * (outputs: to the capacity documented by the call).  Outputs overwrite
 * ranks[] with the ranks actually produced. */
typedef struct {
  int d;
  const int* n;
  int* ranks;
  double** cores;
} t2s2_tt;

/* TT-matrix (square modes).  ranks has d+1 entries; cores[l] is a device
 * pointer to ranks[l]*n[l]*n[l]*ranks[l+1] doubles. */
typedef struct {
  int d;
  const int* n;
  const int* ranks;
  double* const* cores;
} t2s2_ttm;

/* Solver options (alternating sweeps with residual enrichment; the paper's
 * "swaps", Results: Superconsistent Stabilization, Fig. 6). */
typedef struct {
  double tol;          /* relative truncation threshold of the core splits   */
  double target;       /* stop once ||f - L x||_2 / ||f||_2 <= target (FP64) */
  int max_sweeps;      /* sweeps (one pass over all cores, alternating)      */
  int kick;            /* enrichment rank per split                          */
  int rank_cap;        /* max TT rank of x (<= the problem's rank_cap)       */
  int init_rank;       /* rank of the seeded random start when x0 is NULL    */
  unsigned long long seed;
  int check_every;     /* FP64 residual every this many sweeps; 0: only once
                          the largest local residual is <= 10 * target      */
  int verbose;         /* 1: print one line per sweep on stderr              */
  int precision;       /* T2S2_PRECISION_FP64 or T2S2_PRECISION_MIXED        */
  int warm_judge;      /* 1: keep x0 only if its FP64 residual ||f - L x0|| /
                          ||f|| is below that of the seeded random start of a
                          cold solve, else start cold; 0: always use x0     */
  int overlap;         /* FP64 precision: 1 (default) reduces each new
                          interface to Hessenberg form on the solve's stream
                          and computes its eigendecomposition (needed only by
                          the opposite sweep) on a second stream owned by the
                          problem, concurrently with the sweep; 0 computes
                          every factorisation on the solve's stream.  Same
                          arithmetic either way, up to rounding.           */
} t2s2_options;

/* Per-solve report (host struct filled by t2s2_solve). */
typedef struct {
  int status;
  int sweeps;
  int max_rank;
  int ranks[T2S2_MAX_DIM + 1];
  double residual;                              /* final ||f - Lx||/||f||  */
  double time_ms;                               /* wall time of the solve   */
  int history_len;
  double history_residual[T2S2_MAX_HISTORY];    /* per sweep, -1 if unchecked */
  double history_local[T2S2_MAX_HISTORY];       /* max local rel. residual  */
  int history_max_rank[T2S2_MAX_HISTORY];
  double history_time_ms[T2S2_MAX_HISTORY];
  int precision;                                /* as requested             */
  int local_systems;                            /* local systems solved     */
  int refinement_steps;                         /* preconditioned FP64 steps */
  int fp64_fallbacks;                           /* MIXED: FP32 factors too
                                                   weak, FP64 ones used     */
  int warm_start_used;                          /* x0 given and kept        */
  double warm_residual;                         /* residual of x0 when judged,
                                                   else -1                  */
  double cold_residual;                         /* residual of the cold start
                                                   when judged, else -1     */
  int refinement_capped;                        /* local refinements that
                                                   stopped at their step cap
                                                   above 0.1 tol / sqrt(d)  */
  double max_eig_cond;                          /* largest ||V||_F ||V^-1||_F
                                                   (>= cond_2(V)) of the FP64
                                                   eigenvector bases of the
                                                   interface matrices; the
                                                   FP64 refinement absorbs
                                                   the error they cause     */
  double phase_ms[T2S2_PHASES];                 /* device time per phase on
                                                   the solve's stream: 0 set-up
                                                   (Dirichlet lift, start,
                                                   orthogonalisation, first
                                                   interfaces, warm-start
                                                   judge), 1 local solves,
                                                   2 splits (truncated SVD,
                                                   enrichment, QR), 3 interface
                                                   updates and factorisations,
                                                   4 FP64 residual checks   */
} t2s2_report;

/* Message of the last failing call on this thread ("" if none). */
const char* t2s2_last_error(void);

/* ---------------------------------------------------------------- host ---
 * 1D ingredients (paper: Overview (i)-(ii)).  Host only, no GPU needed.
 *   N      nodes (degree N-1), 3 <= N <= 257
 *   eps    > 0; beta any finite value; scheme T2S2_SCHEME_SC or _PLAIN
 *   gll_out     host, N doubles, ascending GLL nodes
 *   colloc_out  host, N-2 doubles, ascending collocation nodes
 * EINVAL on bad sizes or non-finite parameters. */
int t2s2_nodes(int N, double eps, double beta, int scheme,
               double* gll_out, double* colloc_out);

/* Lagrange matrices of the GLL basis at the collocation nodes, row-major
 * (N-2) x N host arrays: E[j,i] = l_i(theta_j), D1 = l_i', D2 = l_i''. */
int t2s2_matrices_1d(int N, double eps, double beta, int scheme,
                     double* E, double* D1, double* D2);

/* ------------------------------------------------------------ problem ---
 * Build the 1D ingredients and the rank-2 TT-matrix operator of the
 * interior system on the current HIP device.
 *   d        1 .. T2S2_MAX_DIM;  N  host array of d node counts (3..66)
 *   eps > 0; beta host array of d finite values; scheme as above
 *   rank_cap maximum TT rank any solve on this problem may reach (>= 1)
 * On success *out owns device copies of the operator cores and 1D data.
 * EINVAL, ENOMEM or EHIP otherwise (*out untouched). */
int t2s2_problem_create(int d, const int* N, double eps, const double* beta,
                        int scheme, int rank_cap, t2s2_problem** out);
/* The same problem with a constant reaction term (paper: Eq. pblm:time:A,
 * rho f):  -eps Lap u + beta . grad u + rho u = f.  Collocated, rho u is
 * rho ((x)_l E_l) u = sum_l (x)_{k != l} E_k (x) (rho / d) E_l u, so the
 * operator stays a rank-2 Kronecker sum with M_l = -eps D2_l + beta_l D1_l +
 * (rho / d) E_l (and K_l = E_l^{-1} M_l shifted by rho / d).  rho finite;
 * otherwise as t2s2_problem_create (rho = 0 gives the same problem). */
int t2s2_problem_create_reaction(int d, const int* N, double eps, const double* beta, double rho, int scheme,
                                 int rank_cap, t2s2_problem** out);
int t2s2_problem_destroy(t2s2_problem* p);

/* General problem (paper: Eq. pblm:time:A-C and the unified space-time
 * formulation of the Overview): per dimension a kind
 *   T2S2_DIM_SPACE (0): x_l in [-1, 1], Dirichlet data at both ends (u = g),
 *       N_l - 2 unknowns at the interior GLL nodes, rows at the n_l - 1
 *       superconsistent (or plain) collocation nodes;
 *   T2S2_DIM_TIME (1): t in [0, T], the value at t = 0 given (initial
 *       condition, Eq. pblm:time:C), N_l - 1 unknowns at the GLL nodes
 *       t_1 .. t_n, rows at the n_l Gauss points (zeros of P_n; the
 *       superconsistent limit for a first-order operator: the paper applies
 *       superconsistency to the spatial dimensions only); operator
 *       (2 / T) d/ds of the reference coordinate s;
 * and a variable separable advection beta_l(x_l) = sum_k c_{l,k} P_k(x_l)
 * (Legendre series, nbeta[l] >= 1 coefficients per space dimension,
 * concatenated over the space dimensions in beta_coef; nbeta is ignored for
 * time dimensions), evaluated at the collocation nodes.  The node set of a
 * space dimension follows one advection value: the largest |beta_l| over the
 * GLL nodes, with its sign, or positive when beta_l changes sign there
 * (the paper's variable-coefficient cases take positive directions).
 * Operator: sum_l (x)_{k != l} E_k (x) M_l, M_l = -eps D2_l + diag(beta_l(theta))
 * D1_l + (rho / d) E_l (space), (2/T) D1_l + (rho / d) E_l (time): still a
 * rank-2 Kronecker sum, so t2s2_solve applies unchanged.  The initial
 * condition (and spatial Dirichlet data) enter through t2s2_solve's g: a TT
 * on the full grid (N_l values per dimension) whose values at t = 0 and on
 * the spatial boundary are used, e.g. u0(x) (x) (1, .., 1)(t) for u0
 * vanishing on the spatial boundary.  f and the solution live on the
 * unknown grid (N_l - 2 per space, N_l - 1 per time dimension);
 * t2s2_problem_colloc returns physical times for time dimensions.
 * EINVAL: bad kinds or sizes, T <= 0 with a time dimension, non-finite
 * coefficients. */
#define T2S2_DIM_SPACE 0
#define T2S2_DIM_TIME 1
int t2s2_problem_create_general(int d, const int* N, const int* kind, double eps, const double* beta_coef,
                                const int* nbeta, double rho, double T, int scheme, int rank_cap,
                                t2s2_problem** out);

/* ------------------------------------------------------ method of lines ---
 * Time stepping of du/dt - eps Lap u + beta . grad u + rho u = b with u = 0
 * on the boundary (paper: Overview, the method-of-lines formulation; Eq.
 * ttss-backward-Euler and Eq. ttss-Crank-Nicolson).  Both schemes are the
 * theta-scheme (u^{k+1} - u^k)/dt + theta A u^{k+1} + (1 - theta) A u^k = b,
 * theta = 1 backward Euler, theta = 1/2 Crank-Nicolson, A = -eps Lap +
 * beta . grad + rho.  In collocation form
 *   (E + theta dt (L + rho E)) u^{k+1} = (E - (1-theta) dt (L + rho E)) u^k + dt b
 * (E = (x)_l E_l, L the interior collocation operator), i.e. per step the
 * steady problem with reaction rho + 1/(theta dt) and right-hand side
 *   f = (1/(theta dt)) E u^k - ((1-theta)/theta) (L + rho E) u^k + b / theta,
 * solved by the alternating sweeps with the exact local solver (the identity
 * only shifts K_l).
 * t2s2_mol_create: such a problem (dt > 0, 0 < theta <= 1, rho finite; the
 * rest as t2s2_problem_create); t2s2_solve on it solves the steady problem
 * with reaction rho + 1/(theta dt).
 * t2s2_mol_step: one step from u (interior values, mode sizes N_l - 2, ranks
 * within the cap) to u_next (as x_out of t2s2_solve; it may alias u).  b:
 * NULL or the step's source at the collocation nodes (theta b(t_{k+1}) +
 * (1 - theta) b(t_k) for a time-dependent source).  f is formed as one
 * rank-2 Kronecker-sum TT-matvec of u plus b (ranks 2 r + s), rounded at
 * relative 1e-14; the solve starts from u.  Status and report as
 * t2s2_solve (the residual is that of the step's system); EINVAL if p was
 * not made by t2s2_mol_create. */
int t2s2_mol_create(int d, const int* N, double eps, const double* beta, double rho, double dt, double theta,
                    int scheme, int rank_cap, t2s2_problem** out);
int t2s2_mol_step(t2s2_problem* p, const t2s2_tt* u, const t2s2_tt* b, const t2s2_options* opts,
                  t2s2_tt* u_next, t2s2_report* rep, void* stream);

/* Device pointers of the operator's TT-matrix cores (owned by p; valid until
 * destroy).  out->n and out->ranks point into p. */
int t2s2_problem_operator(const t2s2_problem* p, t2s2_ttm* out);

/* Host copy of the m_l = N_l - 2 collocation nodes of dimension l. */
int t2s2_problem_colloc(const t2s2_problem* p, int l, double* theta_out);

/* ------------------------------------------------------ building blocks -- */

/* y = A x (paper: Methods, structure-preserving operations): core l of y is
 * Y[(a,p), i', (b,q)] = sum_i A_l[a, i', i, b] X_l[p, i, q], so y's ranks are
 * R_l * r_l.  y->cores[l] must hold R_l r_l n_l R_{l+1} r_{l+1} doubles;
 * y->ranks is written.  Asynchronous on stream. */
int t2s2_tt_matvec(const t2s2_ttm* A, const t2s2_tt* x, t2s2_tt* y, void* stream);

/* y = A x exactly as t2s2_tt_matvec, allocating nothing: for callers that
 * cannot call hipMalloc (code under HIP graph capture, serving loops or
 * harnesses that forbid allocation).  The caller passes x and y as for
 * t2s2_tt_matvec; the only scratch, the permuted operator core, lives in a
 * static device array of 131072 doubles (1 MiB) that each GPU holds until
 * the process ends, so every core must satisfy R_l n_l^2 R_{l+1} <= 131072
 * (and n_l <= 64), else T2S2_EINVAL before any work is queued.  The array's
 * device address is looked up on the first call on each device.  Calls that
 * overlap on one GPU share that array and race: serialise them (one stream,
 * or events).  Results are bitwise those of t2s2_tt_matvec.  Asynchronous on
 * stream. */
int t2s2_tt_matvec_noalloc(const t2s2_ttm* A, const t2s2_tt* x, t2s2_tt* y, void* stream);

/* One fiber of a TT (paper: Fig. 2, an entry is the product of one slice
 * per core): out[i] = x(idx_0, .., idx_{l-1}, i, idx_{l+1}, .., idx_{d-1})
 * for i < n_l, the quantity behind the oscillation count along a line
 * through the grid (Results: Superconsistent Stabilization).  idx: host
 * array of d indices (idx[l] is ignored); out: device array of n_l doubles.
 * Uses p's scratch; asynchronous on stream.  EINVAL for a bad mode or index. */
int t2s2_tt_fiber(t2s2_problem* p, const t2s2_tt* x, int l, const int* idx, double* out, void* stream);

/* ||x||_2 (Frobenius) by the Gram recursion G_l = sum_i X_l(i)^T G_{l-1}
 * X_l(i) carried in double-double arithmetic (error-free products and
 * two-sum accumulation), so ||x||^2 is resolved to ~1e-16 of itself; uses
 * p's scratch.  Synchronises stream; result in *out (host). */
int t2s2_tt_norm(t2s2_problem* p, const t2s2_tt* x, double* out, void* stream);

/* ||f - L x||_2 / ||f||_2 with L the problem's operator (paper: Results,
 * Fig. 6 residual per swap): L x by the TT-matvec, f and -L x concatenated
 * into the exact TT of f - L x (ranks s + 2 r), whose norm, and that of f,
 * come from the double-double Gram recursion of t2s2_tt_norm.  The
 * expansion ||f||^2 - 2<f, Lx> + ||Lx||^2 is never formed (it cancels below
 * FP64 at residuals of 1e-8).  Synchronises stream. */
int t2s2_tt_residual_norm(t2s2_problem* p, const t2s2_tt* x, const t2s2_tt* f,
                          double* out, void* stream);

/* In-place rounding rndg(x) (paper: Methods, rounding paragraph):
 * right-to-left QR orthogonalisation, then left-to-right truncated SVDs with
 * delta = tol ||x|| / sqrt(d-1) per split and rank <= rmax, so that
 * ||x - rndg(x)|| <= tol ||x||.  x->cores must have room for the input
 * ranks (output ranks never exceed them); x->ranks is updated.
 * Synchronises stream. */
int t2s2_tt_round(t2s2_problem* p, t2s2_tt* x, double tol, int rmax, void* stream);

/* Local system of the alternating solver (paper: Results, stabilisation of
 * convection-dominated problems -- AMEn solves one local problem per TT core,
 * whose direct solution costs O((r_{l-1} n_l r_l)^3) when formed densely).
 * For the Kronecker-sum operator the local matrix is itself a Kronecker sum
 *   B = Lint (+) K (+) Rint,  (B u)[a,i,b] = sum_a' Lint[a][a'] u[a',i,b]
 *        + sum_i' K[i][i'] u[a,i',b] + sum_b' Rint[b][b'] u[a,i,b'],
 * on u of shape r1 x m x r2 (row-major), and this entry solves B u = g
 * without forming B, as the solver's local solves do:
 *   method 0: eigendecompositions of Lint and Rint, complex Schur form of K,
 *             triangular solves along the mode index;
 *   method 1: Hessenberg form of Lint, eigendecomposition of Rint, Schur form
 *             of K, and per eigenvalue of Rint one Hessenberg-Schur chain
 *             (requires r1 <= 256 and m * ceil(r1/64) * 1024 <= 160000);
 *   method 2: the mirror image: Hessenberg form of Rint, eigendecomposition
 *             of Lint, one chain per eigenvalue of Lint (requires r2 <= 256
 *             and m * ceil(r2/64) * 1024 <= 160000).
 * All arrays are FP64 device buffers owned by the caller, row-major: Lint
 * (r1 x r1), K (m x m), Rint (r2 x r2), g and u (r1 * m * r2); u must not
 * alias g.  One application in FP64, no refinement.  Sizes: r1, r2 <= 512,
 * m <= 64.  Returns T2S2_EINVAL for bad sizes or method, and T2S2_EFACTOR if
 * a Francis QR stops at its step limit (see t2s2_debug_iteration_limits).
 * Synchronises stream. */
int t2s2_local_solve(int r1, int m, int r2, const double* Lint, const double* K, const double* Rint,
                     const double* g, double* u, int method, void* stream);

/* ------------------------------------------------------------- sources ---
 * Separable right-hand sides sampled on the problem's collocation grid
 * (paper: the source enters the solve as a TT, Methods; a sum of s
 * separable terms has exact TT rank s with block-diagonal cores).  f_out's
 * cores are caller-owned device buffers for ranks (1, s, ..., s, 1) (d = 1:
 * one core, the sum); its ranks are written.  Host parameter arrays.
 * Synchronises stream. */
/* f(x) = sum_{t<s} amp[t] prod_l exp(-(x_l - centre[t*d + l])^2 / (2 width[t]^2)).
 * EINVAL: s outside [1, 1024], non-finite values, width <= 0. */
int t2s2_source_gaussians(t2s2_problem* p, int s, const double* amp,
                          const double* centre, const double* width,
                          t2s2_tt* f_out, void* stream);
/* A non-separable source on the collocation grid by TT-cross approximation
 * (paper: Methods, the closing paragraph on cross approximation: a TT from
 * a few sampled entries, rows and columns chosen by MaxVol; Oseledets &
 * Tyrtyshnikov and Goreinov et al. are cited there).  Built-in functions of
 * x in R^d, params = {amp, aux, w_0..w_{d-1}, c_0..c_{d-1}} (host, 2 + 2d):
 *   kind 0: amp / (1 + sum_l w_l (x_l - c_l)^2)
 *   kind 1: amp exp(-sqrt(aux + sum_l w_l (x_l - c_l)^2)), aux >= 0
 *   kind 2: amp sin(aux + sum_l w_l x_l)      (exact TT rank 2)
 * Alternating cross with nested index sets: two pairs of half sweeps at
 * ranks r0, 2 r0, ... <= rmax (<= 128); at each core the fiber tensor
 * f(I_{l-1}, i, J_l) is evaluated on the device, orthonormalised, and a
 * one-workgroup MaxVol kernel (start from pivoted elimination, swaps while
 * an entry of Q Q[rows]^{-1} exceeds 1.01) gives the rows and the core.  It
 * stops when the relative error on 1000 seeded random grid points is <= tol
 * (or at rmax), then rounds at relative tol / 10.  f_out: cores with room for
 * rmax * (N_l - 2) * rmax doubles; ranks written.  rank_out and
 * sample_error_out (host, nullable) receive the last cross rank and its
 * sampled error.  EINVAL for a bad kind, sizes or non-finite parameters or
 * function values.  Synchronises stream. */
int t2s2_source_cross(t2s2_problem* p, int kind, const double* params, double tol, int r0, int rmax,
                      unsigned long long seed, t2s2_tt* f_out, int* rank_out, double* sample_error_out,
                      void* stream);
/* The source of the manufactured solution u = prod_l sin(pi x_l) exp(x_l):
 * f = sum_l (-eps u_l'' + beta_l u_l')(x_l) prod_{k != l} u_k(x_k), rank d. */
int t2s2_source_manufactured(t2s2_problem* p, t2s2_tt* f_out, void* stream);

/* ---------------------------------------------------------------- solve ---
 * Solve the collocation system in TT format by alternating sweeps with
 * exact local solves and residual enrichment (the paper cites AMEn for this
 * step).
 *   f      TT right-hand side on the collocation grid (device cores, mode
 *          sizes N_l - 2)
 *   g      optional Dirichlet data (paper: Eq. pblm:time:B, u = g on the
 *          boundary): a TT on the GLL grid, mode sizes N_l, whose values at
 *          boundary nodes are used (interior values are ignored).  The
 *          boundary rows are then u = g and the interior unknowns solve
 *          L x = b with b = f - L_full g + L g_int (L_full: the collocation
 *          rows on all GLL columns, g_int: g's interior slices), formed as
 *          an exact TT sum and rounded at relative 1e-14 (rank <= rank_cap).
 *          NULL: g = 0, b = f.
 *   x0     optional TT start (NULL: seeded random TT of rank init_rank);
 *          d and mode sizes N_l - 2 must match the problem and its ranks
 *          must not exceed the rank cap, else T2S2_EINVAL before any copy
 *   x_out  output TT of the interior values (mode sizes N_l - 2; with g the
 *          boundary values of the solution are g's); cores[l] must hold
 *          rank_cap*(N_l-2)*rank_cap doubles (first/last: (N_l-2)*rank_cap);
 *          ranks written
 *   rep    optional host report; its residual is ||b - L x|| / ||b||
 * Returns T2S2_OK when the FP64 residual meets opts->target, T2S2_ENOTCONV
 * (x_out still holds the last iterate) when max_sweeps is reached first,
 * T2S2_EINVAL for bad descriptors or a precision other than
 * T2S2_PRECISION_FP64 / _MIXED, T2S2_EFACTOR when a factorisation gives up. */
int t2s2_solve(t2s2_problem* p, const t2s2_tt* f, const t2s2_tt* g,
               const t2s2_tt* x0, const t2s2_options* opts, t2s2_tt* x_out,
               t2s2_report* rep, void* stream);

/* Batched solve of count independent instances of uneven size (each its own
 * d, N_l, eps, beta, source; the batched workload of hundreds of small
 * problems).  Instance i is solved exactly as t2s2_solve(probs[i], f[i],
 * g ? g[i] : NULL, x0 ? x0[i] : NULL, opts, x_out[i], reps ? &reps[i] : NULL)
 * would, so its
 * result is bitwise the same; instances run concurrently, up to `workers`
 * at a time (0: 16, at most 64), each on its own non-blocking HIP stream of
 * default priority driven by its own host thread, taken from a shared
 * queue in decreasing order of an estimated cost (sum of m_l times
 * log10(10 / eps)).  Every worker stream first waits for the work already
 * queued on `stream`; all work is complete when the call returns.  Device
 * scratch that an instance outgrows while the batch runs is released when
 * the call returns (a release in between would wait for every worker), so
 * the call's peak device memory can reach about twice the problems' final
 * scratch on top of it (79 GiB against 56 GiB for the 256-instance
 * benchmark batch).
 *   probs  count distinct problems (a problem is not shared between
 *          concurrent solves: EINVAL if a pointer repeats)
 *   g      NULL, or count entries each NULL or Dirichlet data (as t2s2_solve)
 *   x0     NULL, or count entries each NULL or a start TT
 *   opts   one option set for every instance (NULL: defaults)
 *   reps   NULL or count host reports
 * Returns T2S2_OK if every instance converged; otherwise the worst code
 * (a hard error before T2S2_ENOTCONV), with the first such instance named
 * in t2s2_last_error; reps[i].status holds each instance's outcome. */
int t2s2_solve_batched(int count, t2s2_problem* const* probs,
                       const t2s2_tt* const* f, const t2s2_tt* const* g,
                       const t2s2_tt* const* x0,
                       const t2s2_options* opts, t2s2_tt* const* x_out,
                       t2s2_report* reps, int workers, void* stream);

/* -------------------------------------------------- learned warm start ---
 * A systems addition (the paper trains nothing): a multilayer perceptron
 * maps an instance's parameters to TT cores that start the sweeps.  Widths
 * w_0 .. w_L; hidden layers tanh(W h + b), output linear.  Parameters are one
 * flat FP32 device vector: per layer W_k (w_{k+1} x w_k, row-major), then b_k.
 * The network owns its parameters, gradient, Adam moments, a BF16 copy and
 * scratch (device memory of the current device), released by destroy.
 * All arrays below are FP32 device arrays, batch-major (row b = sample b).
 * Calls on one network must not run concurrently. */
typedef struct t2s2_mlp t2s2_mlp;

/* Glorot-uniform weights (seeded), zero biases.  1 <= n_layers <= 15,
 * widths has n_layers + 1 entries in [1, 65536].  EINVAL on bad sizes. */
int t2s2_mlp_create(int n_layers, const int* widths, unsigned long long seed,
                    t2s2_mlp** out);
void t2s2_mlp_destroy(t2s2_mlp* net);
int t2s2_mlp_param_count(const t2s2_mlp* net, long long* count);
/* Copy the parameters (which = 0) or the last gradient (which = 1) into dst
 * (param_count floats, device); set_params copies src in and resets Adam. */
int t2s2_mlp_get_params(t2s2_mlp* net, float* dst, int which, void* stream);
int t2s2_mlp_set_params(t2s2_mlp* net, const float* src, void* stream);
/* y (batch x w_L) = net(x (batch x w_0)) in FP32; keeps the activations. */
int t2s2_mlp_forward(t2s2_mlp* net, int batch, const float* x, float* y,
                     void* stream);
/* Gradient of sum(dy * y) for the forward pass just made on the same x and
 * batch (EINVAL otherwise) into the network's gradient buffer. */
int t2s2_mlp_backward(t2s2_mlp* net, int batch, const float* x,
                      const float* dy, void* stream);
/* One Adam step (Kingma and Ba) with that gradient. */
int t2s2_mlp_adam_step(t2s2_mlp* net, float lr, float beta1, float beta2,
                       float eps, void* stream);
/* Inference with weights and biases rounded to BF16 (round to nearest
 * even), FP32 activations and accumulation. */
int t2s2_mlp_infer_bf16(t2s2_mlp* net, int batch, const float* x, float* y,
                        void* stream);
/* Flat TT layout: cores of uniform interior rank r (boundary ranks 1) one
 * after another, core l [r_{l-1}][n_l][r_l] C-contiguous; 1 <= d <= 16,
 * n_l <= 64, r <= 16.
 * Gauge-invariant fitting loss per sample, loss[b] = ||P - T||^2 / ||T||^2
 * of the TTs held in pred and target (Methods: the TT representation is not
 * unique, so cores are never compared directly), and dpred = d loss / d pred,
 * by left/right contractions of the TT format. */
int t2s2_tt_fit_loss(int batch, int d, const int* n, int rank,
                     const float* pred, const float* target, float* loss,
                     float* dpred, void* stream);
/* Training: epochs of shuffled (seeded) mini-batches of the mean fitting
 * loss, backward, Adam (betas 0.9, 0.999, eps 1e-8).  x: count x w_0,
 * targets: count x w_L flat TTs, w_L must equal the flat size of (d, n,
 * rank).  epoch_loss (host, optional, epochs floats) receives the mean
 * training loss of each epoch.  On a network that has taken no Adam step
 * yet, the output bias is first set to the mean target and the output
 * weights are scaled by 0.1 (the start is then a typical TT, whose
 * multilinear gradients do not vanish).  Synchronises stream. */
int t2s2_mlp_train(t2s2_mlp* net, int count, const float* x,
                   const float* targets, int d, const int* n, int rank,
                   int epochs, int batch, float lr, unsigned long long seed,
                   float* epoch_loss, void* stream);
/* TT (FP64 cores, ranks <= rank) -> flat FP32 vector, zero-padded to rank.
 * canonical = 1 also fixes the sign of each rank column of cores 0..d-2 so
 * that its largest-magnitude entry is positive (undone in the next core, so
 * the tensor is unchanged): for a left-orthonormal TT from rounding this
 * makes the packed vector a function of the tensor alone. */
int t2s2_tt_pack(const t2s2_tt* x, int rank, int canonical, float* out,
                 void* stream);
/* Flat FP32 vector -> TT with FP64 cores of ranks (1, rank, .., rank, 1);
 * x_out->cores must hold them; x_out->ranks is written. */
int t2s2_tt_unpack(int d, const int* n, int rank, const float* in,
                   t2s2_tt* x_out, void* stream);

/* --------------------------------------------------------- diagnostics ---
 * Kernel-class timing for benchmarks.  While enabled, every library kernel
 * launch is bracketed by two HIP events on its stream (a small overhead per
 * launch) and its algorithmic bytes and flops (the operands the operation
 * must read and write once, and its arithmetic count) are accumulated.
 * t2s2_timing_enable(1) resets the counters; (0) stops recording.
 * Classes: 0 real GEMM, 1 complex GEMM, 2 TT-matvec core, 3 Schur QR,
 * 4 Hessenberg, 5 Jacobi SVD, 6 Cholesky, 7 triangular inverse,
 * 8 triangular eigenvectors, 9 Kronecker-sum triangular solves,
 * 10 Hessenberg-Schur chains, 11 other.
 * t2s2_timing_classes(mask) restricts recording to the classes whose bit is
 * set in mask (bit c = class c; default all): each recorded launch costs two
 * event records on the host, so a timed run can record only the classes it
 * reports.  t2s2_timing_read synchronises the device work it reads; EINVAL
 * for a bad class. */
int t2s2_timing_enable(int on);
int t2s2_timing_classes(unsigned int mask);
int t2s2_timing_read(int cls, double* total_ms, long long* launches, double* bytes, double* flops);
const char* t2s2_timing_class_name(int cls);

/* One strided-batched FP64 GEMM with the library's kernels, row-major:
 * C_b = alpha op(A_b) op(B_b) + beta C_b, X_b = X + b * sX, op 0 = N, 1 = T,
 * op(A) M x K, op(B) K x N.  variant: 0 the vector-ALU kernel, 1 the
 * matrix-core kernel (V_MFMA_F64_16X16X4_F64), -1 the choice of the tuning
 * table that every FP64 GEMM of the solver uses (written by
 * paper_2506_04732_amd/autotune.py from timings of both kernels on the GPU;
 * t2s2_gemm_tune_source names where it came from).  For tests and tuning;
 * device buffers, asynchronous on stream; EINVAL for bad arguments. */
int t2s2_debug_gemm(int variant, int opA, int opB, int M, int N, int K, int batch, double alpha, const double* A,
                    long long lda, long long sA, const double* B, long long ldb, long long sB, double beta,
                    double* C, long long ldc, long long sC, void* stream);
const char* t2s2_gemm_tune_source(void);

/* Copy `bytes` bytes from device memory `dev` to host memory `host` after all
 * earlier work on `stream`, through the library's read-back path (the path
 * that returns pivot counts, ranks, flags and norms to the host during a
 * solve: a pinned mailbox for up to 64 KiB, the runtime's copy beyond).
 * Synchronous; no alignment required; EINVAL for NULL pointers or a negative
 * size.  For tests. */
int t2s2_debug_readback(const void* dev, void* host, long long bytes, void* stream);

/* Iteration limits of the dense factorisations, process-wide (0 restores a
 * default: 40 n + 100 Francis double-shift steps for an n x n matrix, 60
 * one-sided Jacobi sweeps).  For tests of the error path: with a lowered
 * limit the kernels stop normally and the calls that ran them return
 * T2S2_EFACTOR.  EINVAL for negative values. */
int t2s2_debug_iteration_limits(int francis_steps, int jacobi_sweeps);

/* Defaults: tol 1e-10, target 1e-8, max_sweeps 40, kick 8, rank_cap = the
 * problem's, init_rank 2, seed 0, check_every 1, verbose 0, precision FP64,
 * warm_judge 0, overlap 1. */
void t2s2_default_options(t2s2_options* opts);

#ifdef __cplusplus
}
#endif
#endif /* T2S2_H */
