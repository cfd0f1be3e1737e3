"""GPU solve, doubled-precision residual and iterative refinement vs the oracle.

Bars: the triangular solves agree with the oracle's solves on the same factors
to 1e-12 relative; the residual agrees with the oracle's Dot2 residual within
the Dot2 bound (u |r| + gamma_n^2 (|A||x| + |b|), doubled for two
evaluation orders); refined solutions are within 1e-12 (relative, max norm)
of the oracle's converged reference solution."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import lu as olu
from oracle import solve as osolve
from paper_1208_2451_amd import inputs
from tests.gpu_util import announce, gpu_factor

pytestmark = pytest.mark.gpu


def _x_ref(A, B):
    lu_, piv = sla.lu_factor(A)
    perm = np.arange(A.shape[0])
    for j, p in enumerate(piv):
        perm[[j, p]] = perm[[p, j]]
    x, _, _ = osolve.refine(A, lu_, perm, B, tol=1e-16, max_iter=12)
    return x


@pytest.mark.parametrize("n,nrhs", [(300, 1), (300, 3), (257, 9), (64, 1), (1, 1)])
def test_solve_matches_oracle_on_same_factors(n, nrhs):
    import torch
    import paper_1208_2451_amd as prrp
    A, _ = inputs.randn_system(n, 40 + n)
    B = np.random.default_rng(n).standard_normal((n, nrhs))
    announce("solve n=%d nrhs=%d" % (n, nrhs))
    LU, perm, st, At, r = gpu_factor(A, min(32, n))
    X = prrp.solve(At, r.perm, torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    Xo = osolve.solve(LU, perm, B)
    assert np.abs(X.cpu().numpy() - Xo).max() <= 1e-12 * max(1.0, np.abs(Xo).max())


@pytest.mark.parametrize("n,nrhs", [(200, 1), (513, 4), (129, 10)])
def test_residual_within_dot2_bound(n, nrhs):
    import torch
    import paper_1208_2451_amd as prrp
    A, _ = inputs.randn_system(n, 7 + n)
    g = np.random.default_rng(3)
    X = np.linalg.solve(A, g.standard_normal((n, nrhs)))
    B = A @ X + 1e-13 * g.standard_normal((n, nrhs))
    announce("residual n=%d nrhs=%d" % (n, nrhs))
    R = prrp.residual(torch.from_numpy(A).cuda(), torch.from_numpy(X).cuda(), torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    Ro = osolve.residual_dot2(A, X, B)
    u = 2.0 ** -53
    gam = n * u / (1 - n * u)
    bound = 2 * u * np.abs(Ro) + 4 * gam * gam * (np.abs(A) @ np.abs(X) + np.abs(B))
    assert np.all(np.abs(R.cpu().numpy() - Ro) <= bound)
    # and a plain FP64 residual would not meet it (the test has teeth)
    assert not np.all(np.abs((B - A @ X) - Ro) <= 0.01 * bound)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_refine_kappa_1e6_to_1e12(precision):
    import torch
    import paper_1208_2451_amd as prrp
    n = 512
    A = inputs.kappa_matrix(n, 5, 1e6)
    B = inputs.rhs(n, 5, 1)
    x_ref = _x_ref(A, B[:, 0])
    announce("refine", precision, "n=%d" % n)
    _, _, st, At, r = gpu_factor(A, 64, precision=precision)
    X, it, rel, status = prrp.refine(torch.from_numpy(A).cuda(), At, r.perm, torch.from_numpy(B).cuda(),
                             tol=1e-14, max_iter=40)
    torch.cuda.synchronize()
    err = np.abs(X.cpu().numpy()[:, 0] - x_ref).max() / np.abs(x_ref).max()
    assert err <= 1e-12, (err, it, rel)


def test_refine_multiple_rhs():
    import torch
    import paper_1208_2451_amd as prrp
    n, nrhs = 384, 16
    A = inputs.kappa_matrix(n, 8, 1e6)
    B = inputs.rhs(n, 8, nrhs)
    announce("refine 16 rhs n=%d" % n)
    _, _, st, At, r = gpu_factor(A, 64)
    X, it, rel, status = prrp.refine(torch.from_numpy(A).cuda(), At, r.perm, torch.from_numpy(B).cuda(),
                             tol=1e-14, max_iter=20)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    for c in (0, 7, 15):
        x_ref = _x_ref(A, B[:, c])
        assert np.abs(Xh[:, c] - x_ref).max() <= 1e-12 * np.abs(x_ref).max()
