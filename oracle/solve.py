"""Solves and iterative refinement -- oracle (test infrastructure).

``solve`` applies A = Pi L U (the problem statement of the introduction):
x = U^-1 L^-1 b[perm].  ``residual_dot2`` evaluates r = b - A x as if in twice
the working precision and then rounds once, using the error-free
transformations TwoSum (Knuth) and TwoProduct (Dekker, with Veltkamp's split)
accumulated as in Ogita, Rump and Oishi's Dot2 algorithm ("Accurate sum and
dot product", SIAM J. Sci. Comput. 26, 2005).  ``refine`` is classical
iterative refinement (used in the paper's linear-solver experiments, with the
componentwise backward error as its stopping test; here the stopping test is
the relative size of the correction, and w is reported).

Pinned by tests/test_oracle_solve.py: the residual equals the exact rational
residual rounded once on small systems, refined solutions agree with LAPACK
getrs-based refinement to a few ulps of the solution, and a system with a known
exactly representable solution is solved to full accuracy.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

_SPLIT = 134217729.0  # 2^27 + 1


def solve(LU: np.ndarray, perm: np.ndarray, B: np.ndarray) -> np.ndarray:
    """x = U^-1 L^-1 B[perm] for the in-place factors of A[perm] = L U."""
    B = np.asarray(B, dtype=np.float64)
    y = solve_triangular(LU, B[perm], lower=True, unit_diagonal=True)
    return solve_triangular(LU, y, lower=False)


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _split(a):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    return p, al * bl - (((p - ah * bh) - al * bh) - ah * bl)


def residual_dot2(A: np.ndarray, X: np.ndarray, B: np.ndarray, block: int = 512) -> np.ndarray:
    """r = B - A X with Dot2 accuracy (one rounding at the end).

    The sum for row i runs over the terms B[i], -A[i,0] X[0], ..., -A[i,n-1] X[n-1]
    in that order; rows and right-hand sides are processed as vectors.
    """
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
        B = B[:, None]
    n = A.shape[1]
    p = B.copy()
    s = np.zeros_like(p)
    Xh, Xl = _split(-X)
    for j0 in range(0, n, block):
        Ab = A[:, j0:j0 + block]
        Ah, Al = _split(Ab)
        for jj in range(Ab.shape[1]):
            j = j0 + jj
            a = Ab[:, jj:jj + 1]
            x = -X[j:j + 1, :]
            h = a * x
            r = Al[:, jj:jj + 1] * Xl[j:j + 1, :] - (((h - Ah[:, jj:jj + 1] * Xh[j:j + 1, :])
                                                       - Al[:, jj:jj + 1] * Xh[j:j + 1, :])
                                                      - Ah[:, jj:jj + 1] * Xl[j:j + 1, :])
            p, q = _two_sum(p, h)
            s += q + r
    out = p + s
    return out[:, 0] if vec else out


def refine(A, LU, perm, B, tol: float = 1e-14, max_iter: int = 30):
    """Iterative refinement x <- x + solve(r), r from ``residual_dot2``.

    Stops when ||d||_inf <= tol ||x||_inf, when the correction fails to halve,
    or after ``max_iter`` corrections.  Returns (x, iterations, history of
    ||d||/||x||).
    """
    x = solve(LU, perm, B)
    hist = []
    prev = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        r = residual_dot2(A, x, B)
        d = solve(LU, perm, r)
        x = x + d
        rel = float(np.abs(d).max() / max(np.abs(x).max(), np.finfo(float).tiny))
        hist.append(rel)
        if rel <= tol or rel > 0.5 * prev:
            break
        prev = rel
    return x, it, hist
