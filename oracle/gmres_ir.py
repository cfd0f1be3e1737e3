"""Refinement on the componentwise backward error, and GMRES-based
refinement -- oracle (test infrastructure).

The paper's linear-solver experiments (Section 3.3, the paragraph on Tables
"bcaluprrp_gepp" and "fcaluprrp_gepp") refine the solution with the
componentwise backward error w of equation "comp" as the measure:
w_b is w before refinement, N_IR the number of refinement steps.
``refine_w`` is that loop, with the classical stopping rule (Skeel; Arioli,
Demmel and Duff, "Solving sparse linear systems with sparse backward error",
SIAM J. Matrix Anal. Appl. 10, 1989): stop once w is at most the unit
roundoff, once a step fails to halve w, or after max_iter steps.  The
residual is formed as if in twice the working precision
(``solve.residual_dot2``).

``gmres`` is the generalized minimal residual method (Saad and Schultz, SIAM
J. Sci. Stat. Comput. 7, 1986): Arnoldi with modified Gram-Schmidt builds an
orthonormal basis of the Krylov space, Givens rotations reduce the
Hessenberg matrix, and the iterate minimises the residual 2-norm over the
space.  ``gmres_ir`` is GMRES-based iterative refinement (Carson and Higham,
"Accelerating the solution of linear systems by iterative refinement in three
precisions", SIAM J. Sci. Comput. 40, 2018): each correction solves A d = r
by GMRES on the left-preconditioned system U^-1 L^-1 A d = U^-1 L^-1 r, the
preconditioner being the (possibly low-precision) LU factors, instead of one
triangular solve; the outer loop stops as ``refine_w`` does.  This is
beyond the paper, which refines in working precision only; it is the
refinement for factors whose Schur updates ran in BF16, where one triangular
solve per step no longer contracts the error.

Pinned by tests/test_oracle_gmres_ir.py: w against its definition in exact
rationals, GMRES's finite termination on matrices with few distinct
eigenvalues, its minimal-residual iterate against a brute-force least-squares
solution over an explicit Krylov basis in exact rationals, and recovery of an
exactly representable solution from perturbed factors.
"""
from __future__ import annotations

import math

import numpy as np

from .solve import residual_dot2, solve

U_ROUND = 2.0 ** -53


def comp_w(A: np.ndarray, x: np.ndarray, b: np.ndarray, r: np.ndarray | None = None) -> float:
    """Componentwise backward error w = max_i |r_i| / (|A| |x| + |b|)_i
    (equation "comp") with r = b - A x from ``residual_dot2``; rows whose
    denominator is zero count only if their residual is non-zero (then w is
    infinite)."""
    if r is None:
        r = residual_dot2(A, x, b)
    den = np.abs(A) @ np.abs(x) + np.abs(b)
    num = np.abs(r)
    w = 0.0
    for i in range(len(num)):
        if den[i] > 0.0:
            w = max(w, float(num[i] / den[i]))
        elif num[i] > 0.0:
            return math.inf
    return w


def refine_w(A, LU, perm, b, max_iter: int = 30):
    """Refinement x <- x + solve(r) measured by w (Section 3.3).

    Returns (x, N_IR, w_b, history of w after each step, status), status
    "converged" (w <= unit roundoff), "stagnated" (a step did not halve w) or
    "cap"."""
    x = solve(LU, perm, b)
    r = residual_dot2(A, x, b)
    w = comp_w(A, x, b, r)
    w_b = w
    hist = []
    status = "converged" if w <= U_ROUND else "cap"
    steps = 0
    while status == "cap" and steps < max_iter:
        x = x + solve(LU, perm, r)
        steps += 1
        r = residual_dot2(A, x, b)
        w_new = comp_w(A, x, b, r)
        hist.append(w_new)
        if w_new <= U_ROUND:
            status = "converged"
        elif not (w_new <= 0.5 * w):
            status = "stagnated"
        w = w_new
    return x, steps, w_b, hist, status


def _givens(a: float, b: float):
    """c, s with [c s; -s c] [a; b] = [h; 0]."""
    if b == 0.0:
        return 1.0, 0.0
    h = math.hypot(a, b)
    return a / h, b / h


def gmres(apply_op, rhs: np.ndarray, tol: float, max_it: int, x0: np.ndarray | None = None):
    """GMRES for op(d) = rhs from x0 (default 0), restarted never.

    Stops when the (rotated) residual norm is at most tol * ||rhs - op(x0)||
    or after max_it steps.  Returns (x, steps, residual-norm history)."""
    n = rhs.shape[0]
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64)
    r0 = rhs - apply_op(x0) if np.any(x0) else rhs.copy()
    beta = float(np.linalg.norm(r0))
    hist = [beta]
    if beta == 0.0 or max_it == 0:
        return x0.copy(), 0, hist
    V = np.zeros((n, max_it + 1))
    H = np.zeros((max_it + 1, max_it))
    cs = np.zeros(max_it)
    sn = np.zeros(max_it)
    g = np.zeros(max_it + 1)
    g[0] = beta
    V[:, 0] = r0 / beta
    k = 0
    for j in range(max_it):
        w = apply_op(V[:, j])
        for i in range(j + 1):                       # modified Gram-Schmidt
            H[i, j] = float(V[:, i] @ w)
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = float(np.linalg.norm(w))
        if H[j + 1, j] > 0.0:
            V[:, j + 1] = w / H[j + 1, j]
        for i in range(j):                           # earlier rotations
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
        H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]))
        if abs(g[j + 1]) <= tol * beta or H[j, j] == 0.0:
            break
    # back substitution on the k x k triangle
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    return x0 + V[:, :k] @ y, k, hist


def gmres_ir(A, LU, perm, b, gmres_tol: float = 1e-6, max_inner: int = 60, max_outer: int = 20,
             tol: float = 0.0):
    """GMRES-based refinement (Carson and Higham 2018) with the LU factors as
    left preconditioner.

    With tol = 0 the stopping measure is w, as in ``refine_w``.  With tol > 0
    it is the size of the correction, as in ``solve.refine``: stop once
    ||d||_inf <= tol ||x||_inf, or once it fails to halve -- w at the unit
    roundoff bounds only the backward error, and the forward error can still
    be kappa times larger, so a forward-error target needs this measure.
    Returns (x, outer steps, total GMRES steps, w_b, history of w, status)
    with status "converged", "stagnated" or "cap"."""
    A = np.asarray(A, dtype=np.float64)

    def prec_op(v):
        return solve(LU, perm, A @ v)

    x = solve(LU, perm, b)
    r = residual_dot2(A, x, b)
    w = comp_w(A, x, b, r)
    w_b = w
    hist = []
    inner = 0
    status = "converged" if (tol == 0.0 and w <= U_ROUND) else "cap"
    steps = 0
    prev = math.inf
    while status == "cap" and steps < max_outer:
        d, k, _ = gmres(prec_op, solve(LU, perm, r), gmres_tol, max_inner)
        inner += k
        x = x + d
        steps += 1
        r = residual_dot2(A, x, b)
        w_new = comp_w(A, x, b, r)
        hist.append(w_new)
        if tol > 0.0:
            rel = float(np.abs(d).max() / max(np.abs(x).max(), np.finfo(float).tiny))
            if rel <= tol:
                status = "converged"
            elif not (rel <= 0.5 * prev):
                status = "stagnated"
            prev = rel
        elif w_new <= U_ROUND:
            status = "converged"
        elif not (w_new <= 0.5 * w):
            status = "stagnated"
        w = w_new
    return x, steps, inner, w_b, hist, status
