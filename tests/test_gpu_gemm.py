"""The FP64 GEMM kernels (vector ALU and matrix cores, V_MFMA_F64_16X16X4_F64)
against numpy float64 products: ragged sizes around the 16/64 tiles, both
transposes, batches, the split-K path (few output tiles, K >= 256), alpha and
beta.  Bar: |C - C_ref| <= 32 eps K max|A| max|B| element-wise (any order of
summation of K products meets it) -- and the two kernels agree to the same bar."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_04732_amd as t2s2  # noqa: E402
from paper_2506_04732_amd import _lib  # noqa: E402

CASES = [(1, 1, 1, 1, 0, 0), (17, 33, 5, 1, 0, 0), (64, 64, 64, 1, 1, 0), (70, 130, 45, 1, 0, 1),
         (129, 65, 200, 1, 1, 1), (200, 30, 4320, 1, 1, 0), (33, 200, 1000, 1, 0, 0), (30, 200, 30, 150, 0, 0),
         (144, 6000, 144, 1, 0, 0), (5, 3, 7, 9, 1, 1)]


def _run(variant, M, N, K, batch, ta, tb, alpha, beta, A, B, C0):
    import torch
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.from_numpy(C0.copy()).cuda()
    lda = M if ta else K
    ldb = K if tb else N
    sA, sB, sC = A[0].size, B[0].size, C0[0].size
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    t2s2.check(_lib.lib().t2s2_debug_gemm(variant, ta, tb, M, N, K, batch, alpha, C.c_void_p(dA.data_ptr()), lda,
                                           sA, C.c_void_p(dB.data_ptr()), ldb, sB, beta,
                                           C.c_void_p(dC.data_ptr()), N, sC, stream))
    return dC.cpu().numpy()


@pytest.mark.parametrize("M,N,K,batch,ta,tb", CASES)
def test_gemm_kernels_match_numpy(M, N, K, batch, ta, tb):
    print("[case] gemm", M, N, K, batch, ta, tb, flush=True)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((batch, K, M) if ta else (batch, M, K))
    B = rng.standard_normal((batch, N, K) if tb else (batch, K, N))
    C0 = rng.standard_normal((batch, M, N))
    alpha, beta = 0.7, -1.3
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = alpha * np.matmul(opA, opB) + beta * C0
    bar = 32 * np.finfo(np.float64).eps * K * np.abs(A).max() * np.abs(B).max() + 8 * np.finfo(np.float64).eps * np.abs(ref).max()
    outs = [_run(v, M, N, K, batch, ta, tb, alpha, beta, A, B, C0) for v in (0, 1, -1)]
    for v, out in zip((0, 1, -1), outs):
        err = np.abs(out - ref).max()
        print(f"[case]   variant {v}: max err {err:.2e} (bar {bar:.2e})", flush=True)
        assert err <= bar
    assert np.abs(outs[0] - outs[1]).max() <= 2 * bar
