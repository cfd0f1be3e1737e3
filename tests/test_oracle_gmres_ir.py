"""Pins of the oracle's componentwise backward error, GMRES and GMRES-based
refinement (oracle/gmres_ir.py) against facts fixed outside it: exact
rational arithmetic, the finite termination of GMRES, the minimal-residual
property over an explicitly formed Krylov space, and exactly representable
solutions."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import gmres_ir as og
from oracle import lu as olu

U = 2.0 ** -53


def _exact_w(A, x, b):
    n = len(b)
    best = Fraction(0)
    for i in range(n):
        r = Fraction(b[i]) - sum(Fraction(A[i, j]) * Fraction(x[j]) for j in range(n))
        den = sum(abs(Fraction(A[i, j])) * abs(Fraction(x[j])) for j in range(n)) + abs(Fraction(b[i]))
        best = max(best, abs(r) / den)
    return best


def test_comp_w_matches_exact_rationals():
    g = np.random.default_rng(5)
    n = 9
    A = g.standard_normal((n, n))
    x = np.linalg.solve(A, g.standard_normal(n))
    b = A @ x + 1e-9 * g.standard_normal(n)
    w = og.comp_w(A, x, b)
    we = _exact_w(A, x, b)
    assert abs(w - float(we)) <= 1e-12 * float(we)
    # a swapped numerator / denominator, or |A x| for |A||x|, fails this
    assert w < 1e-8


def test_gmres_terminates_in_number_of_distinct_eigenvalues():
    g = np.random.default_rng(1)
    n = 14
    S = g.standard_normal((n, n))
    lam = np.array([1.0, 3.0, -2.0] * 5)[:n]          # 3 distinct eigenvalues
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    b = g.standard_normal(n)
    op = lambda v: A @ v  # noqa: E731
    x, k, hist = og.gmres(op, b, 1e-12, n)
    assert k <= 3
    assert np.linalg.norm(b - A @ x) <= 1e-9 * np.linalg.norm(b)
    _, _, h2 = og.gmres(op, b, 1e-30, 2)
    assert h2[-1] > 1e-4 * np.linalg.norm(b)            # two steps are not enough


def _exact_krylov_minres(A, b, k):
    """argmin over x in span{b, Ab, ..., A^(k-1) b} of ||b - A x||_2, exactly."""
    n = len(b)
    Af = [[Fraction(int(v)) for v in row] for row in A]
    bf = [Fraction(int(v)) for v in b]
    K = [bf]
    for _ in range(k - 1):
        v = K[-1]
        K.append([sum(Af[i][j] * v[j] for j in range(n)) for i in range(n)])
    AK = [[sum(Af[i][j] * K[c][j] for j in range(n)) for i in range(n)] for c in range(k)]
    # normal equations (AK)^T (AK) y = (AK)^T b
    M = [[sum(AK[p][i] * AK[q][i] for i in range(n)) for q in range(k)] for p in range(k)]
    rhs = [sum(AK[p][i] * bf[i] for i in range(n)) for p in range(k)]
    for c in range(k):                                  # Gauss-Jordan, exact
        piv = next(r for r in range(c, k) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        rhs[c], rhs[piv] = rhs[piv], rhs[c]
        for r in range(k):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [M[r][q] - f * M[c][q] for q in range(k)]
                rhs[r] -= f * rhs[c]
    y = [rhs[c] / M[c][c] for c in range(k)]
    x = [sum(y[c] * K[c][i] for c in range(k)) for i in range(n)]
    res = [bf[i] - sum(Af[i][j] * x[j] for j in range(n)) for i in range(n)]
    return [float(v) for v in x], float(sum(v * v for v in res))


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_gmres_iterate_minimises_residual_over_krylov_space(k):
    A = np.array([[4, 1, 0, 2, -1, 0], [1, 3, -1, 0, 0, 2], [0, -1, 5, 1, 1, 0],
                  [2, 0, 1, 6, 0, -1], [-1, 0, 1, 0, 2, 1], [0, 2, 0, -1, 1, 7]], dtype=float)
    b = np.array([1, -2, 3, 0, 1, -1], dtype=float)
    x, steps, _ = og.gmres(lambda v: A @ v, b, 0.0, k)
    assert steps == k
    xe, res2 = _exact_krylov_minres(A, b, k)
    assert np.abs(x - xe).max() <= 1e-12 * max(1.0, np.abs(xe).max())
    got = float(np.sum((b - A @ x) ** 2))
    assert abs(got - res2) <= 1e-10 * max(res2, 1e-30) + 1e-24


def test_gmres_ir_recovers_exact_solution_from_perturbed_factors():
    g = np.random.default_rng(11)
    n = 40
    A = np.round(8 * g.standard_normal((n, n)))
    x_true = np.round(16 * g.standard_normal(n))
    b = A @ x_true                                     # exact: small integers
    # factors of a perturbed matrix: a poor but usable preconditioner
    f = olu.lu_prrp(A + 0.05 * g.standard_normal((n, n)), 8, 2.0)
    x, outer, inner, w_b, hist, status = og.gmres_ir(A, f.LU, f.perm, b, gmres_tol=1e-8)
    assert status in ("converged", "stagnated")
    assert hist[-1] <= 2 * U
    assert np.abs(x - x_true).max() <= 4 * U * np.abs(x_true).max()
    assert w_b > 1e-6                                  # the unrefined solution was poor


def test_refine_w_stagnates_where_gmres_ir_converges():
    g = np.random.default_rng(3)
    n = 60
    Q1, _ = np.linalg.qr(g.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(g.standard_normal((n, n)))
    A = Q1 @ np.diag(np.logspace(0, -6, n)) @ Q2.T    # kappa 1e6
    b = g.standard_normal(n)
    # factors carrying relative errors far above 1 / kappa (as low-precision
    # Schur updates would): one triangular solve per step no longer contracts
    f = olu.lu_prrp(A * (1 + 2e-3 * g.standard_normal((n, n))), 8, 2.0)
    _, n_ir, w_b, hist_ir, st_ir = og.refine_w(A, f.LU, f.perm, b, max_iter=30)
    assert st_ir in ("stagnated", "cap") and min(hist_ir) > 1e-12
    x, outer, inner, _, hist, st = og.gmres_ir(A, f.LU, f.perm, b, gmres_tol=1e-10, max_inner=60)
    assert hist[-1] <= 2 * U, (hist, inner)
    x_ref = np.linalg.solve(A, b)
    assert np.abs(x - x_ref).max() <= 1e-8 * np.abs(x_ref).max()   # kappa u bound of x_ref


def test_refine_w_converges_with_good_factors():
    from paper_1208_2451_amd import inputs
    A, b = inputs.randn_system(96, 4)
    f = olu.lu_prrp(A, 16, 2.0)
    x, n_ir, w_b, hist, status = og.refine_w(A, f.LU, f.perm, b[:, 0])
    assert n_ir <= 3
    assert (hist[-1] if hist else w_b) <= 2 * U
