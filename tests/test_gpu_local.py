"""GPU parity of the local Kronecker-sum solve (t2s2_local_solve) against a
dense FP64 solve of the assembled local operator (oracle.amen.kron_sum_dense
and LU).

Inputs are shaped like the solver's local systems: the left and right
interfaces are Galerkin projections of Kronecker sums of scaled 1D
advection-diffusion operators onto random orthonormal bases, K is a scaled 1D
operator.  Sizes span 1..4 row slots of the Hessenberg-Schur kernel (r1 = 1,
37, 70, 130, 200, 256), ragged m and r2.

Bar: the three methods (eigendecompositions of both interfaces; Hessenberg
form of the left one; Hessenberg form of the right one) solve in FP64
through similarity transforms, so their
forward error is bounded by a modest multiple of the unit roundoff times
cond(B) and the condition numbers of the eigenvector bases used:
||u - u*|| <= 64 eps cond(B) cond(V_L) cond(V_R) ||u*|| (cond(V_L) taken as 1
for the orthogonal Hessenberg transform would also hold; the looser bound is
used for both).  cond(B) is the 2-norm condition number up to 4000 rows and
LAPACK's 1-norm estimate beyond (the 19600-row case).
"""
import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

import paper_2506_04732_amd as t2s2  # noqa: E402
from oracle import amen as oamen  # noqa: E402
from oracle import collocation as oc  # noqa: E402


def _say(*a):
    print("[case]", *a, flush=True)


def _k1d(N, eps, beta):
    Es, Ms = oc.interior_factors(oc.build_ops(1, N, eps, [beta]))
    return np.linalg.solve(Es[0], Ms[0])


def _interface(rng, r, Ks):
    A = Ks[0]
    for Kk in Ks[1:]:
        A = np.kron(A, np.eye(Kk.shape[0])) + np.kron(np.eye(A.shape[0]), Kk)
    X, _ = np.linalg.qr(rng.standard_normal((A.shape[0], r)))
    return X.T @ A @ X


def _case(seed, r1, m, r2):
    rng = np.random.default_rng(seed)
    N1 = max(18, int(np.ceil(np.sqrt(r1))) + 3)        # (N1 - 2)^2 >= r1
    KL = _interface(rng, r1, [_k1d(N1, 2e-3, 0.4), _k1d(N1, 2e-3, -0.7)]) if r1 > 1 else np.zeros((1, 1))
    K = _k1d(m + 2, 2e-3, 0.3)
    if r2 <= 6:
        KR = _interface(rng, r2, [_k1d(8, 2e-3, 0.5)]) if r2 > 1 else np.zeros((1, 1))
    else:
        N2 = max(18, int(np.ceil(np.sqrt(r2))) + 3)
        KR = _interface(rng, r2, [_k1d(N2, 2e-3, -0.3), _k1d(N2, 2e-3, 0.8)])
    g = rng.standard_normal((r1, m, r2))
    return KL, K, KR, g


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


CASES = [(1, 6, 4), (37, 5, 3), (70, 6, 5), (130, 4, 3), (200, 3, 2), (256, 2, 2), (64, 9, 1),
         (3, 6, 130), (4, 5, 200), (2, 3, 256), (40, 7, 70)]


def _dense_reference(B, g):
    """Dense FP64 solve of B u = g and cond(B).  Up to 4000 rows the 2-norm
    condition number (SVD); beyond, LAPACK's 1-norm estimate from the LU
    factors (dgecon), which is within a factor n of it, since an SVD of a
    19600 x 19600 matrix takes minutes of host time."""
    n = B.shape[0]
    if n <= 4000:
        return np.linalg.solve(B, g), np.linalg.cond(B)
    lu, piv = sla.lu_factor(B, check_finite=False)
    u = sla.lu_solve((lu, piv), g, check_finite=False)
    rcond, info = sla.lapack.dgecon(lu, np.abs(B).sum(axis=0).max(), norm="1")
    assert info == 0 and rcond > 0
    return u, 1.0 / rcond


@pytest.mark.parametrize("r1,m,r2", CASES)
def test_local_solve_matches_dense(r1, m, r2):
    KL, K, KR, g = _case(100 + r1, r1, m, r2)
    _say("dense reference", r1 * m * r2, "rows")
    B = oamen.kron_sum_dense(KL, K, KR)
    ref, cond_b = _dense_reference(B, g.ravel())
    ref = ref.reshape(r1, m, r2)
    del B
    cond = cond_b * np.linalg.cond(np.linalg.eig(KL)[1]) * np.linalg.cond(np.linalg.eig(KR)[1])
    bar = 64 * np.finfo(np.float64).eps * cond
    outs = {}
    methods = [t2s2.LOCAL_EIG]
    if r1 <= 256:
        methods.append(t2s2.LOCAL_HESS)
    if r2 <= 256:
        methods.append(t2s2.LOCAL_HESS_RIGHT)
    for method in methods:
        _say("local solve", r1, m, r2, "method", method)
        u = t2s2.local_solve(_cuda(KL), _cuda(K), _cuda(KR), _cuda(g), method=method).cpu().numpy()
        err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
        _say(f"  rel err {err:.2e} (bar {bar:.2e})")
        assert err <= bar
        outs[method] = u
    for method in methods[1:]:
        assert np.linalg.norm(outs[0] - outs[method]) <= 2 * bar * np.linalg.norm(ref)


def test_local_solve_eigen_path_beyond_256_rows():
    """r1 = 300: both interfaces by eigendecomposition (Hessenberg reduction of
    a matrix beyond 256 rows, Francis QR from global memory); same bar."""
    r1, m, r2 = 300, 2, 2
    KL, K, KR, g = _case(300, r1, m, r2)
    B = oamen.kron_sum_dense(KL, K, KR)
    ref = np.linalg.solve(B, g.ravel()).reshape(r1, m, r2)
    cond = np.linalg.cond(B) * np.linalg.cond(np.linalg.eig(KL)[1]) * np.linalg.cond(np.linalg.eig(KR)[1])
    bar = 64 * np.finfo(np.float64).eps * cond
    _say("local solve", r1, m, r2, "method 0")
    u = t2s2.local_solve(_cuda(KL), _cuda(K), _cuda(KR), _cuda(g), method=t2s2.LOCAL_EIG).cpu().numpy()
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    _say(f"  rel err {err:.2e} (bar {bar:.2e})")
    assert err <= bar


def test_local_solve_rejects_unsupported_sizes():
    KL, K, KR, g = _case(7, 4, 3, 2)
    with pytest.raises(t2s2.T2S2Error):
        # Hessenberg-Schur chains hold at most 256 rows
        big = np.eye(300)
        t2s2.local_solve(_cuda(big), _cuda(K), _cuda(KR), _cuda(np.zeros((300, 3, 2))), method=t2s2.LOCAL_HESS)
    with pytest.raises(t2s2.T2S2Error):
        t2s2.local_solve(_cuda(KR), _cuda(K), _cuda(big), _cuda(np.zeros((2, 3, 300))),
                         method=t2s2.LOCAL_HESS_RIGHT)
    with pytest.raises(t2s2.T2S2Error):
        t2s2.local_solve(_cuda(KL), _cuda(K), _cuda(KR), _cuda(g), method=5)
