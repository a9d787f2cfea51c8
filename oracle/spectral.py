"""1D spectral ingredients (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

Paper passages followed:

* Overview (i): Lagrange basis on n+1 representation points, the two interval
  ends plus the n-1 zeros of P_n' (Gauss-Lobatto-Legendre, "GLL"); one
  dimension has n+1 degrees of freedom.
* Overview (ii), Eq. adv-diff-1d and Fig. 1: the collocation points move from
  the zeros of P_n' (diffusion-optimal) towards the zeros of P_n
  (convection-optimal) as eps/|beta| decreases; they depend only on that ratio
  and on n; the discrete operators are the Lagrange basis of the
  representation grid evaluated at the collocation grid.

The paper does not print the node formula (its Methods section on
superconsistency is absent).  Reading used here: for degree n, the
superconsistent collocation nodes are, for i = 1..n-1, the unique zero of

    Q(x) = eps * P_n'(x) - beta * P_n(x)

inside the i-th gap (z_i, z_{i+1}) of the Gauss zeros z_1 < ... < z_n of P_n.
Q is, up to the factor n(n+1), the 1D operator -eps d2/dx2 + beta d/dx applied
to the GLL nodal polynomial (1 - x^2) P_n'(x).  Q changes sign across every
gap, so each gap holds exactly one zero and the n-th zero of Q (outside the
gaps, on the outflow side) is dropped.  beta = 0 gives the interior GLL nodes,
i.e. plain spectral collocation.  The limits stated in Overview (ii) follow:
eps/|beta| -> inf gives the zeros of P_n', eps/|beta| -> 0 gives z_i + eps/beta.

Pins (tests/test_oracle_spectral.py): closed-form GLL nodes for n = 2, 3, 4;
exactness of the GLL quadrature up to degree 2n-1; exact interpolation and
differentiation of polynomials of degree <= n; interlacing, both limits and
mirror symmetry of the collocation nodes; the closed-form solution of
Eq. adv-diff-1d (spectral convergence, no oscillation with superconsistent
nodes, oscillation with plain collocation).  The exact node positions of the
paper's figures are parity unpinned (figure only).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

SCHEME_PLAIN = 0
SCHEME_SC = 1


def legendre_with_derivs(n: int, x):
    """Return P_n(x), P_n'(x), P_n''(x) by the three-term recurrence.

    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}, differentiated once and twice.
    """
    x = np.asarray(x, dtype=np.float64)
    p0, d0, s0 = np.ones_like(x), np.zeros_like(x), np.zeros_like(x)
    if n == 0:
        return p0, d0, s0
    p1, d1, s1 = x.copy(), np.ones_like(x), np.zeros_like(x)
    for k in range(1, n):
        p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
        d2 = ((2 * k + 1) * (p1 + x * d1) - k * d0) / (k + 1)
        s2 = ((2 * k + 1) * (2 * d1 + x * s1) - k * s0) / (k + 1)
        p0, d0, s0, p1, d1, s1 = p1, d1, s1, p2, d2, s2
    return p1, d1, s1


def gauss_nodes(n: int) -> np.ndarray:
    """Zeros z_1 < ... < z_n of P_n (Legendre-Gauss points)."""
    z, _ = np.polynomial.legendre.leggauss(n)
    # one Newton step on P_n polishes the library values
    p, dp, _ = legendre_with_derivs(n, z)
    return np.sort(z - p / dp)


def gll_nodes(n: int) -> np.ndarray:
    """GLL representation nodes x_0 = -1 < x_1 < ... < x_n = 1 (Overview (i)).

    Interior nodes = zeros of P_n' = zeros of the Jacobi(1,1) polynomial of
    degree n-1, taken as eigenvalues of its symmetric Jacobi matrix (monic
    recurrence p_{k+1} = x p_k - g_k p_{k-1}, g_k = k(k+2)/((2k+1)(2k+3))),
    then polished by Newton on P_n'.
    """
    if n < 1:
        raise ValueError("degree n must be >= 1")
    if n == 1:
        return np.array([-1.0, 1.0])
    k = np.arange(1, n - 1, dtype=np.float64)
    off = np.sqrt(k * (k + 2) / ((2 * k + 1) * (2 * k + 3)))
    jac = np.diag(off, 1) + np.diag(off, -1)
    y = np.linalg.eigvalsh(jac) if n > 2 else np.zeros(1)
    for _ in range(3):
        _, dp, d2p = legendre_with_derivs(n, y)
        y = y - dp / d2p
    return np.concatenate(([-1.0], np.sort(y), [1.0]))


def gll_weights(n: int) -> np.ndarray:
    """GLL quadrature weights w_j = 2 / (n (n+1) P_n(x_j)^2)."""
    x = gll_nodes(n)
    p, _, _ = legendre_with_derivs(n, x)
    return 2.0 / (n * (n + 1) * p * p)


def sc_nodes(n: int, eps: float, beta: float) -> np.ndarray:
    """Superconsistent collocation nodes theta_1 < ... < theta_{n-1}.

    One zero of eps P_n' - beta P_n per gap of the Gauss zeros (reading stated
    in the module header).  beta = 0 returns the interior GLL nodes.
    """
    if n < 2:
        raise ValueError("degree n must be >= 2 to have interior nodes")
    if eps <= 0:
        raise ValueError("eps must be positive")
    if beta == 0.0:
        return gll_nodes(n)[1:-1].copy()
    z = gauss_nodes(n)

    def q(t):
        p, dp, _ = legendre_with_derivs(n, np.array([t]))
        return float(eps * dp[0] - beta * p[0])

    theta = np.empty(n - 1)
    for i in range(n - 1):
        a, b = z[i], z[i + 1]
        qa, qb = q(a), q(b)
        if qa == 0.0:
            theta[i] = a
        elif qb == 0.0:
            theta[i] = b
        elif qa * qb > 0:
            # eps so small that the zero sits on z_i (or z_{i+1}) to rounding
            theta[i] = a if beta > 0 else b
        else:
            theta[i] = brentq(q, a, b, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)
    return theta


def collocation_nodes(n: int, eps: float, beta: float, scheme: int) -> np.ndarray:
    """Interior collocation grid: superconsistent (scheme=1) or plain GLL (0)."""
    if scheme == SCHEME_PLAIN:
        return gll_nodes(n)[1:-1].copy()
    if scheme == SCHEME_SC:
        return sc_nodes(n, eps, beta)
    raise ValueError(f"unknown scheme {scheme}")


def _orthonormal_legendre_vandermonde(n: int, x):
    """Columns k = 0..n of sqrt((2k+1)/2) P_k and its first two derivatives."""
    x = np.asarray(x, dtype=np.float64)
    V = np.empty((x.size, n + 1))
    V1 = np.empty_like(V)
    V2 = np.empty_like(V)
    for k in range(n + 1):
        p, dp, d2p = legendre_with_derivs(k, x)
        s = np.sqrt((2 * k + 1) / 2.0)
        V[:, k], V1[:, k], V2[:, k] = s * p, s * dp, s * d2p
    return V, V1, V2


def lagrange_matrices(x_rep, y_eval):
    """E, D1, D2 with E[j,i] = l_i(y_j), D1[j,i] = l_i'(y_j), D2[j,i] = l_i''(y_j).

    l_i is the Lagrange basis polynomial of the representation nodes x_rep
    (degree n = len(x_rep) - 1).  Built as V(y) V(x)^{-1} with the orthonormal
    Legendre Vandermonde (Overview (ii): basis of the representation grid
    evaluated at the collocation grid).
    """
    x_rep = np.asarray(x_rep, dtype=np.float64)
    n = x_rep.size - 1
    Vx, _, _ = _orthonormal_legendre_vandermonde(n, x_rep)
    Vy, Vy1, Vy2 = _orthonormal_legendre_vandermonde(n, y_eval)
    # M V(x)^{-1} computed as solve(V(x)^T, M^T)^T
    E = np.linalg.solve(Vx.T, Vy.T).T
    D1 = np.linalg.solve(Vx.T, Vy1.T).T
    D2 = np.linalg.solve(Vx.T, Vy2.T).T
    return E, D1, D2


def operator_1d(N: int, eps: float, beta: float, scheme: int = SCHEME_SC) -> dict:
    """All 1D pieces for one dimension with N = n+1 nodes (degree n = N-1).

    Returns the GLL grid ``x`` (N), the collocation grid ``theta`` (N-2), the
    (N-2) x N matrices ``E``, ``D1``, ``D2`` and the 1D operator
    ``M = -eps D2 + beta D1`` (rows: collocation points, columns: nodal
    values on the representation grid).
    """
    if N < 3:
        raise ValueError("need N >= 3 nodes per dimension")
    n = N - 1
    x = gll_nodes(n)
    theta = collocation_nodes(n, eps, beta, scheme)
    E, D1, D2 = lagrange_matrices(x, theta)
    M = -eps * D2 + beta * D1
    return {"n": n, "x": x, "theta": theta, "E": E, "D1": D1, "D2": D2, "M": M}


def solve_1d(N: int, eps: float, beta: float, rhs, scheme: int = SCHEME_SC,
             g_left: float = 0.0, g_right: float = 0.0) -> dict:
    """Collocation solve of -eps f'' + beta f' = rhs on [-1,1], f(-1)=g_left, f(1)=g_right.

    ``rhs`` is a callable evaluated at the collocation nodes.  Boundary rows are
    identity rows at the two GLL end points (Dirichlet data, Eq. pblm:time:B).
    Dense LU (numpy.linalg.solve).
    """
    op = operator_1d(N, eps, beta, scheme)
    A = np.zeros((N, N))
    b = np.zeros(N)
    A[0, 0] = 1.0
    b[0] = g_left
    A[-1, -1] = 1.0
    b[-1] = g_right
    A[1:-1, :] = op["M"]
    b[1:-1] = rhs(op["theta"])
    u = np.linalg.solve(A, b)
    return {"x": op["x"], "u": u, "op": op}


def closed_form_1d(x, eps: float, beta: float):
    """Exact solution of beta f' - eps f'' = 1, f(-1) = f(1) = 0 (Eq. adv-diff-1d).

    f(x) = (x+1)/beta - (2/beta) (exp(beta(x+1)/eps) - 1) / (exp(2 beta/eps) - 1),
    evaluated in an overflow-free form for beta > 0.
    """
    x = np.asarray(x, dtype=np.float64)
    if beta <= 0:
        raise ValueError("closed form written for beta > 0")
    a = beta / eps
    # (e^{a(x+1)} - 1)/(e^{2a} - 1) = e^{a(x-1)} (1 - e^{-a(x+1)}) / (1 - e^{-2a})
    frac = np.exp(a * (x - 1.0)) * (-np.expm1(-a * (x + 1.0))) / (-np.expm1(-2.0 * a))
    return (x + 1.0) / beta - (2.0 / beta) * frac
