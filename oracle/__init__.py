"""FP64 CPU oracle for the T^2S^2 tensor-train collocation solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (``paper_2506_04732_amd``); the only module both sides import
is ``workloads``, which draws seeded problem parameters and holds none of
the method's arithmetic.

Everything here is plain NumPy/SciPy in float64, written to be read
against the paper:

* ``spectral``     -- 1D ingredients: Legendre polynomials, Gauss-Lobatto-
                      Legendre representation nodes, superconsistent
                      collocation nodes, Lagrange evaluation/derivative
                      matrices (Overview (i), (ii); Eq. adv-diff-1d).
* ``collocation``  -- tensor-product collocation system, dense LU and
                      complex-Schur full-format solves, manufactured data
                      (Overview (iii); Eq. advection-diffusion).
* ``tt``           -- tensor-train format, TT-SVD, rounding, TT-matrix
                      arithmetic (Methods, Tensor Train representation).
* ``amen``         -- alternating linear solver in TT format with residual
                      enrichment ("swaps"; Results, Fig. 6).
* ``metrics``      -- relative Frobenius error, oscillation count,
                      compression ratio (Results).
* ``mlp``          -- FP64 network, gauge-invariant TT fitting loss and
                      Adam step of the learned warm start (a systems
                      addition; the paper trains nothing), with gradients
                      pinned by finite differences.

Parity status of every function is listed in its module header.
"""
