"""GPU check of the MFMA GEMM (the Schur-update kernel) against an FP64 CPU
product: FP64 to rounding; FP32 / BF16 operand rounding within their unit
roundoff bounds.  Odd sizes exercise every tile edge; 2944 x 2950 takes the
128 x 128 tiles, K = 300 more than 256 (the index staging's limit)."""
import numpy as np
import pytest

from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-14), ("fp32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("M,N,K", [(16, 16, 4), (130, 257, 33), (300, 129, 128), (7, 5, 3),
                                   (96, 80, 300), (2944, 2950, 128)])
def test_gemm_matches_cpu(prec, tol, M, N, K):
    import torch
    import paper_1208_2451_amd as prrp
    announce("gemm", prec, M, N, K)
    g = np.random.default_rng(M * 7 + N + K)
    A = g.standard_normal((M, K))
    B = g.standard_normal((K, N))
    C0 = g.standard_normal((M, N))
    Ct = torch.from_numpy(C0.copy()).cuda()
    prrp.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), Ct, alpha=-1.0, beta=1.0,
              precision=prec)
    torch.cuda.synchronize()
    ref = C0 - A @ B
    err = np.abs(Ct.cpu().numpy() - ref).max()
    scale = (np.abs(A) @ np.abs(B)).max()
    assert err <= tol * scale


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gemm_beta_zero_ignores_c(prec):
    # beta = 0: C's prior contents (NaN here) are not read
    import torch
    import paper_1208_2451_amd as prrp
    announce("gemm beta=0", prec)
    g = np.random.default_rng(17)
    M, N, K = 200, 77, 64
    A = g.standard_normal((M, K))
    B = g.standard_normal((K, N))
    Ct = torch.full((M, N), float("nan"), dtype=torch.float64).cuda()
    prrp.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), Ct, alpha=2.0, beta=0.0,
              precision=prec)
    torch.cuda.synchronize()
    out = Ct.cpu().numpy()
    assert np.isfinite(out).all()
    tol = 1e-14 if prec == "fp64" else 2e-6
    assert np.abs(out - 2.0 * (A @ B)).max() <= tol * 2.0 * (np.abs(A) @ np.abs(B)).max()
