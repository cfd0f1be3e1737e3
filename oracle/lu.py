"""GEPP, LU_PRRP and CALU_PRRP -- oracle (test infrastructure).

LU_PRRP follows Section 2.1, Algorithm "LU_PRRP factorization of a matrix A
of size n x n", step by step, for each b-column panel A_j:
  1. strong RRQR of A_j^T gives Pi_j and R_j;  L_2j = (R11^-1 R12)^T;
  2. Pi_j^T is applied to entire rows;
  3. trailing update A22 -= L_2j A12 (equation "update"), A12 before GEPP;
  4. GEPP of the b x b diagonal block, A_jj = Pi_jj L_jj U_jj, its row
     interchanges applied to entire rows;
  5. U12 = L_jj^-1 Pi_jj^T A12.
The stored unit-lower factor is the point form L21 = L_2j Pi_jj L_jj (equal in
exact arithmetic to A21 U_jj^-1), so that on exit A_in[perm] = L U with LAPACK
conventions.

CALU_PRRP follows Section 3.1: the panel's rows are split top-down into tiles,
strong RRQR of each tile's transpose selects b candidates (leaves), candidate
sets are merged pairwise up a binary tree (or along a chain for the flat tree)
and reselected by strong RRQR; the root's rows are the pivots.  The panel is
then factored by QR without pivoting of its transpose with the pivot rows
first, L_2j = (R11^-1 R12)^T, and the step continues as in LU_PRRP.

Readings: Pi_j is applied LAPACK-style as the sequence of
transpositions row k0+i <-> current position of the i-th selected row; tiles
hold ``tile_rows`` rows except a last remainder of at most b rows, which joins
the previous tile; a tree node stacks the left child's candidates over the
right child's, each in increasing row order; an odd node is promoted; the flat
tree stacks the running candidates over the next whole tile.

Pinned by tests/test_oracle_lu.py (b = 1 equals LAPACK getrf, A[perm] = LU,
|L_2j| <= tau, per-step growth bound, Wilkinson and Foster growth printed in
the paper or given in closed form, CALU_PRRP with one tile equals LU_PRRP,
node certificates and the per-step (1 + tau b)^(H+1) bound), and by
tests/test_oracle_exact_rules.py (the tournament against an exact-rational
replay in which a node stacks its left child's candidates over its right
child's).  The growth 1 printed for the Wright matrix and the 1.33 printed
for CALU_PRRP on the Foster matrix are not pins: exact computations there
show that no pivoting attains them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

from . import rules
from .srrqr import strong_rrqr


@dataclass
class Factorization:
    LU: np.ndarray
    perm: np.ndarray
    info: int = 0
    swaps: int = 0
    max_abs_A: float = 0.0
    max_abs_U: float = 0.0
    max_abs_W: float = 0.0          # max over all intermediate active matrices and U
    max_block_L: float = 0.0        # max |L_2j| over panels
    step_growth_ok: bool = True     # max|S_(k+1)| <= (1 + tau b) max|S_k| every step
    step_ratios: list = field(default_factory=list)
    panel_sel: list = field(default_factory=list)   # per panel: selected rows (slot order)
    node_max_M: list = field(default_factory=list)  # CALU_PRRP: max |M| at every tree node
    tree_height: int = 0

    @property
    def g_W(self) -> float:
        return self.max_abs_W / self.max_abs_A

    @property
    def g_U(self) -> float:
        return self.max_abs_U / self.max_abs_A

    def L(self) -> np.ndarray:
        return np.tril(self.LU, -1) + np.eye(self.LU.shape[0])

    def U(self) -> np.ndarray:
        return np.triu(self.LU)


def _swap_rows(A, perm, r1, r2):
    if r1 != r2:
        A[[r1, r2]] = A[[r2, r1]]
        perm[[r1, r2]] = perm[[r2, r1]]


def gepp_inplace(B: np.ndarray):
    """Gaussian elimination with partial pivoting of a square block, in place.

    Pivot = largest |entry| of the column on or below the diagonal under the
    tie rule.  Returns (ipiv, info): ipiv[j] is the row swapped with j at step
    j (LAPACK convention, 0-based); info is the 1-based first zero pivot or 0.
    """
    n = B.shape[0]
    ipiv = np.arange(n)
    info = 0
    for j in range(n):
        p = j + rules.argmax_lowest(np.abs(B[j:, j]))
        ipiv[j] = p
        if p != j:
            B[[j, p]] = B[[p, j]]
        piv = B[j, j]
        if piv == 0.0:
            if info == 0:
                info = j + 1
            continue
        B[j + 1:, j] /= piv
        B[j + 1:, j + 1:] -= np.outer(B[j + 1:, j], B[j, j + 1:])
    return ipiv, info


def gepp(A: np.ndarray, track_growth: bool = False) -> Factorization:
    """Full-matrix GEPP (the paper's baseline), unblocked, with growth tracking."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    perm = np.arange(n)
    f = Factorization(LU=A, perm=perm, max_abs_A=float(np.abs(A).max()))
    wmax = f.max_abs_A
    for j in range(n):
        p = j + rules.argmax_lowest(np.abs(A[j:, j]))
        _swap_rows(A, perm, j, p)
        piv = A[j, j]
        if piv == 0.0:
            f.info = f.info or j + 1
            continue
        A[j + 1:, j] /= piv
        A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j, j + 1:])
        if track_growth and j + 1 < n:
            wmax = max(wmax, float(np.abs(A[j + 1:, j + 1:]).max()))
    f.max_abs_U = float(np.abs(np.triu(A)).max())
    f.max_abs_W = max(wmax, f.max_abs_U)
    return f


def _finish_panel(A, perm, k0, bw, sel, M, rest, tau, f: Factorization):
    """Steps 2-5 of the LU_PRRP panel step given the panel's pivot rows.

    ``sel``: the bw pivot rows (panel-relative, slot order); ``M`` = R11^-1 R12
    with column t belonging to panel row rest[t].
    """
    n = A.shape[0]
    m = n - k0
    amax_before = float(np.abs(A[k0:, k0:]).max())
    # Pi_j^T on entire rows, as transpositions.
    at = np.arange(m)          # at[q]: panel row now at position q
    pos = np.arange(m)         # pos[r]: position of panel row r
    for i, r in enumerate(sel):
        q = int(pos[r])
        if q != i:
            _swap_rows(A, perm, k0 + i, k0 + q)
            ri, rq = at[i], at[q]
            at[i], at[q] = rq, ri
            pos[rq], pos[ri] = i, q
    # Block L in the new row order: L_2j = (R11^-1 R12)^T.
    col_of = {r: t for t, r in enumerate(rest)}
    L2 = M.T[[col_of[int(at[q])] for q in range(bw, m)]] if m > bw else np.zeros((0, bw))
    if L2.size:
        f.max_block_L = max(f.max_block_L, float(np.abs(L2).max()))
    # Trailing update with A12 before the diagonal GEPP (equation "update").
    A12 = A[k0:k0 + bw, k0 + bw:].copy()
    if m > bw:
        A[k0 + bw:, k0 + bw:] -= L2 @ A12
    # GEPP of the diagonal block; its interchanges act on entire rows.
    D = A[k0:k0 + bw, k0:k0 + bw].copy()
    ipiv, info = gepp_inplace(D)
    if info and not f.info:
        f.info = k0 + info
    p11 = np.arange(bw)
    for j in range(bw):
        pj = int(ipiv[j])
        if pj != j:
            _swap_rows(A, perm, k0 + j, k0 + pj)
            p11[[j, pj]] = p11[[pj, j]]
    A[k0:k0 + bw, k0:k0 + bw] = D
    L11 = np.tril(D, -1) + np.eye(bw)
    if m > bw:
        A[k0:k0 + bw, k0 + bw:] = solve_triangular(L11, A[k0:k0 + bw, k0 + bw:],
                                                   lower=True, unit_diagonal=True)
        A[k0 + bw:, k0:k0 + bw] = L2[:, p11] @ L11
        smax = float(np.abs(A[k0 + bw:, k0 + bw:]).max())
    else:
        smax = 0.0
    umax = float(np.abs(np.triu(A[k0:k0 + bw, k0:])).max())
    f.max_abs_U = max(f.max_abs_U, umax)
    f.max_abs_W = max(f.max_abs_W, smax, umax)
    ratio = smax / amax_before if amax_before > 0 else 0.0
    f.step_ratios.append(ratio)
    f.panel_sel.append(list(sel))
    return ratio


def lu_prrp(A: np.ndarray, b: int, tau: float = 2.0, panels: int | None = None) -> Factorization:
    """LU_PRRP (Algorithm "LU_PRRP factorization").  ``panels`` stops after that
    many panels (the trailing matrix is then left partially factored)."""
    if not tau > 1.0:
        raise ValueError("tau must exceed 1")
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    perm = np.arange(n)
    amax = float(np.abs(A).max())
    f = Factorization(LU=A, perm=perm, max_abs_A=amax, max_abs_W=amax)
    for j, k0 in enumerate(range(0, n, b)):
        if panels is not None and j >= panels:
            break
        bw = min(b, n - k0)
        r = strong_rrqr(A[k0:, k0:k0 + bw], tau)
        if r.rank_deficient_step >= 0 and not f.info:
            f.info = k0 + r.rank_deficient_step + 1
        f.swaps += r.swaps
        M = r.M if r.rank_deficient_step < 0 else _qr_ratio(A[k0:, k0:k0 + bw], r.sel, r.rest)
        ratio = _finish_panel(A, perm, k0, bw, r.sel, M, r.rest, tau, f)
        if ratio > (1.0 + tau * bw) * (1.0 + 1e-12):
            f.step_growth_ok = False
    return f


# --------------------------------------------------------------------------
# CALU_PRRP (Section 3.1)
# --------------------------------------------------------------------------

def tile_bounds(m: int, tile_rows: int, b: int):
    """Top-down row tiles of ``tile_rows`` rows; a last tile of <= b rows joins
    its predecessor (a leaf needs at least b + 1 rows)."""
    if tile_rows < b + 1:
        raise ValueError("tile_rows must be at least b + 1")
    starts = list(range(0, m, tile_rows))
    bounds = [[s, min(s + tile_rows, m)] for s in starts]
    if len(bounds) > 1 and bounds[-1][1] - bounds[-1][0] <= b:
        bounds[-2][1] = bounds[-1][1]
        bounds.pop()
    return [tuple(x) for x in bounds]


def tournament(P: np.ndarray, tau: float, tile_rows: int, tree: str = "binary", f=None):
    """Tournament pivoting on panel P (m x b); returns the b pivot rows
    (panel-relative) in the root's slot order, and the tree height."""
    m, b = P.shape
    bounds = tile_bounds(m, tile_rows, b)

    def node(rows):
        """Strong RRQR on the stacked rows (given in increasing row order)."""
        r = strong_rrqr(P[rows], tau)
        if f is not None:
            f.node_max_M.append(r.max_abs_M)
            f.swaps += r.swaps
        return [rows[t] for t in r.sel]

    if len(bounds) == 1:
        return node(list(range(m))), 0
    if tree == "binary":
        level = [node(list(range(a, e))) for a, e in bounds]
        height = 0
        while len(level) > 1:
            nxt = []
            for i in range(0, len(level) - 1, 2):
                nxt.append(node(sorted(level[i]) + sorted(level[i + 1])))
            if len(level) % 2:
                nxt.append(level[-1])
            level = nxt
            height += 1
        return level[0], height
    if tree == "flat":
        a, e = bounds[0]
        acc = node(list(range(a, e)))
        for a, e in bounds[1:]:
            acc = node(sorted(acc) + list(range(a, e)))
        return acc, len(bounds) - 1
    raise ValueError("tree must be 'binary' or 'flat'")


def _qr_ratio(P: np.ndarray, sel, rest) -> np.ndarray:
    """QR without pivoting of the panel transpose with the pivot rows first;
    returns R11^-1 R12 (columns follow ``rest``)."""
    Q, R11 = np.linalg.qr(P[sel].T)
    R12 = Q.T @ P[rest].T
    if np.any(np.diag(R11) == 0.0):
        # Singular pivot block (rank-deficient panel): the factorization is
        # flagged through ``info``; keep the multipliers finite.
        return np.linalg.lstsq(R11, R12, rcond=None)[0]
    return solve_triangular(R11, R12, lower=False)


def calu_prrp(A: np.ndarray, b: int, tau: float = 2.0, tile_rows: int = 512,
              tree: str = "binary", panels: int | None = None) -> Factorization:
    """CALU_PRRP with tournament pivoting (Section 3.1)."""
    if not tau > 1.0:
        raise ValueError("tau must exceed 1")
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    perm = np.arange(n)
    amax = float(np.abs(A).max())
    f = Factorization(LU=A, perm=perm, max_abs_A=amax, max_abs_W=amax)
    for j, k0 in enumerate(range(0, n, b)):
        if panels is not None and j >= panels:
            break
        bw = min(b, n - k0)
        m = n - k0
        P = A[k0:, k0:k0 + bw]
        tiles = tile_bounds(m, tile_rows, bw)
        if len(tiles) == 1:
            # One tile: the tournament is a single strong RRQR (= LU_PRRP step).
            r = strong_rrqr(P, tau)
            f.swaps += r.swaps
            f.node_max_M.append(r.max_abs_M)
            if r.rank_deficient_step >= 0 and not f.info:
                f.info = k0 + r.rank_deficient_step + 1
            sel, rest, M, H = r.sel, r.rest, r.M, 0
            if r.rank_deficient_step >= 0:
                M = _qr_ratio(P, sel, rest)
        else:
            sel, H = tournament(P, tau, tile_rows, tree, f)
            chosen = set(sel)
            rest = [c for c in range(m) if c not in chosen]
            M = _qr_ratio(P, sel, rest)
        f.tree_height = max(f.tree_height, H)
        ratio = _finish_panel(A, perm, k0, bw, sel, M, rest, tau, f)
        if ratio > (1.0 + tau * bw) ** (H + 1) * (1.0 + 1e-12):
            f.step_growth_ok = False
    return f
