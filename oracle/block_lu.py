"""Block parallel and block pairwise LU_PRRP -- oracle (test infrastructure).

Section 5 ("Less stable factorizations that can also minimize communication")
and Appendix E.  A panel is factored once, on the way up a reduction tree:

  * the panel's active rows are split into tiles (the leaves);
  * at every node, strong RRQR of the transpose of the node's rows selects b
    of them; each other row r of the node is eliminated against the selected
    rows: with D = (R11^-1 R12)^T (Appendix E's D = Rbarbar^T Rbar^-T) and
    d_r its row, row r becomes row r - d_r [selected rows] on every column
    right of the panel, and d_r is stored in row r's panel columns;
  * the selected rows of a node move up the tree: a binary tree stacks the
    left child's candidates over the right child's (block parallel), the flat
    tree stacks the running candidates over the next whole tile (block
    pairwise);
  * the root's b rows are the panel's pivot rows: they move to the top
    (Pi_j, as in LU_PRRP), the diagonal block is factored by GEPP with its
    interchanges on entire rows, and U12 = L11^-1 Pi11^T A12.

No further update follows: every row of the trailing matrix was updated once,
at the node that eliminated it, against that node's selected rows (which are
still unmodified then: a row is changed only when it is eliminated).  The
factorization is therefore a product of node transformations and the
diagonal GEPP, A = Pi_0^T D_0^-1 ... Pi_H^T D_H^-1 [Ajj Abar12; 0 Abar22]
(Appendix E), not one unit lower triangle; ``block_solve`` applies it.

Stored form (``BlockFactorization``): ``LU`` holds U on and above the
diagonal, the diagonal blocks' L11 below their diagonal, and below the
diagonal blocks each eliminated row's d_r (in final row order, rows moved as
a whole); ``perm[p]`` is the original row at final position p; ``nodes[j]``
lists panel j's nodes in execution order (leaves first, up to the root) as
(selected rows, eliminated rows), both as original row numbers, the selected
ones in slot order (the order of d_r's entries).

Readings (shared with CALU_PRRP in ``lu``): tiles follow ``lu.tile_bounds``
except that a tile may hold exactly b rows (the block pairwise tree of
height n / b that Section 5 describes stacks the running b rows over b new
ones; a b-row leaf keeps all its rows);
stacking orders and the odd-node promotion follow ``lu.tournament``; a node
of a rank-deficient panel takes its multipliers from ``lu._qr_ratio`` (the
paper leaves that case open).  The growth recorded is the largest magnitude
of any row after its update and of U, over the largest of A.

Pinned by tests/test_oracle_block_lu.py: b = 1 against an exact-rational
replay of parallel pivoting (binary tree) and pairwise pivoting (flat tree)
written from their definitions; one tile against LU_PRRP; the recorded
transformations applied to A reproduce U; |d_r| <= tau; the per-panel growth
bound (1 + tau b); the solve's backward error.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

from .lu import _qr_ratio, _swap_rows, gepp_inplace
from .srrqr import strong_rrqr


def tile_bounds(m: int, tile_rows: int, b: int):
    """Top-down row tiles of ``tile_rows`` (>= b) rows; a last remainder of
    fewer than b + 1 rows joins its predecessor."""
    if tile_rows < b:
        raise ValueError("tile_rows must be at least b")
    starts = list(range(0, m, tile_rows))
    bounds = [[s, min(s + tile_rows, m)] for s in starts]
    if len(bounds) > 1 and bounds[-1][1] - bounds[-1][0] <= b:
        bounds[-2][1] = bounds[-1][1]
        bounds.pop()
    return [tuple(x) for x in bounds]


@dataclass
class BlockFactorization:
    LU: np.ndarray
    perm: np.ndarray
    b: int
    nodes: list = field(default_factory=list)   # per panel: [(sel ids, elim ids), ...]
    info: int = 0
    swaps: int = 0
    max_abs_A: float = 0.0
    max_abs_W: float = 0.0
    max_abs_D: float = 0.0
    panel_growth: list = field(default_factory=list)   # max|updated rows| / max|active| per panel
    tree_height: int = 0

    @property
    def g_W(self) -> float:
        return self.max_abs_W / self.max_abs_A


def block_lu_prrp(A: np.ndarray, b: int, tau: float = 2.0, tile_rows: int = 512,
                  tree: str = "binary") -> BlockFactorization:
    """Block parallel (tree="binary") or block pairwise (tree="flat")
    LU_PRRP (Section 5, Appendix E)."""
    if not tau > 1.0:
        raise ValueError("tau must exceed 1")
    if tree not in ("binary", "flat"):
        raise ValueError("tree must be 'binary' or 'flat'")
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    perm = np.arange(n)
    amax = float(np.abs(A).max()) if A.size else 0.0
    f = BlockFactorization(LU=A, perm=perm, b=b, max_abs_A=amax, max_abs_W=amax)
    for k0 in range(0, n, b):
        bw = min(b, n - k0)
        m = n - k0
        active_max = float(np.abs(A[k0:, k0:]).max())
        upd_max = 0.0
        recs = []

        def node(rows):
            """Strong RRQR of the stacked rows (panel-relative, stacking order),
            then the elimination of the rows it leaves out."""
            nonlocal upd_max
            P = A[k0 + np.asarray(rows), k0:k0 + bw]
            r = strong_rrqr(P, tau)
            f.swaps += r.swaps
            if r.rank_deficient_step >= 0 and not f.info:
                f.info = k0 + r.rank_deficient_step + 1
            M = r.M if r.rank_deficient_step < 0 else _qr_ratio(P, r.sel, r.rest)
            sel = [rows[t] for t in r.sel]
            elim = [rows[t] for t in r.rest]
            if elim:
                D = M.T                                     # row t <-> elim[t]
                ge = k0 + np.asarray(elim)
                gs = k0 + np.asarray(sel)
                A[ge, k0 + bw:] -= D @ A[gs, k0 + bw:]
                A[ge, k0:k0 + bw] = D
                f.max_abs_D = max(f.max_abs_D, float(np.abs(D).max()))
                if k0 + bw < n:
                    upd_max = max(upd_max, float(np.abs(A[ge, k0 + bw:]).max()))
            recs.append(([int(perm[k0 + s]) for s in sel], [int(perm[k0 + e]) for e in elim]))
            return sel

        tiles = tile_bounds(m, tile_rows, bw) if m > bw else [(0, m)]
        if len(tiles) == 1:
            root = node(list(range(m)))
        elif tree == "binary":
            level = [node(list(range(a, e))) for a, e in tiles]
            height = 0
            while len(level) > 1:
                nxt = [node(sorted(level[i]) + sorted(level[i + 1]))
                       for i in range(0, len(level) - 1, 2)]
                if len(level) % 2:
                    nxt.append(level[-1])
                level = nxt
                height += 1
            root = level[0]
            f.tree_height = max(f.tree_height, height)
        else:
            a, e = tiles[0]
            root = node(list(range(a, e)))
            for a, e in tiles[1:]:
                root = node(sorted(root) + list(range(a, e)))
            f.tree_height = max(f.tree_height, len(tiles) - 1)
        f.nodes.append(recs)

        # Pi_j: the root's rows to the top, as transpositions on entire rows
        at = np.arange(m)
        pos = np.arange(m)
        for i, r in enumerate(root):
            q = int(pos[r])
            if q != i:
                _swap_rows(A, perm, k0 + i, k0 + q)
                ri, rq = at[i], at[q]
                at[i], at[q] = rq, ri
                pos[rq], pos[ri] = i, q
        # GEPP of the diagonal block, interchanges on entire rows; U12
        Dg = A[k0:k0 + bw, k0:k0 + bw].copy()
        ipiv, info = gepp_inplace(Dg)
        if info and not f.info:
            f.info = k0 + info
        for j in range(bw):
            pj = int(ipiv[j])
            if pj != j:
                _swap_rows(A, perm, k0 + j, k0 + pj)
        A[k0:k0 + bw, k0:k0 + bw] = Dg
        if m > bw:
            L11 = np.tril(Dg, -1) + np.eye(bw)
            A[k0:k0 + bw, k0 + bw:] = solve_triangular(L11, A[k0:k0 + bw, k0 + bw:],
                                                       lower=True, unit_diagonal=True)
        umax = float(np.abs(np.triu(A[k0:k0 + bw, k0:])).max())
        f.max_abs_W = max(f.max_abs_W, upd_max, umax)
        f.panel_growth.append(upd_max / active_max if active_max > 0 else 0.0)
    return f


def block_forward(f: BlockFactorization, B: np.ndarray) -> np.ndarray:
    """Applies the factorization's row operations to B (rows in original
    order): every panel's node eliminations in execution order, then the
    diagonal block's L11^-1.  Returns the result in final row order."""
    LU, perm, b = f.LU, f.perm, f.b
    n = LU.shape[0]
    Y = np.array(B, dtype=np.float64).reshape(n, -1).copy()
    final = np.empty(n, dtype=np.int64)
    final[perm] = np.arange(n)
    for j, recs in enumerate(f.nodes):
        k0 = j * b
        bw = min(b, n - k0)
        for sel, elim in recs:
            if elim:
                D = LU[final[np.asarray(elim)], k0:k0 + bw]
                Y[np.asarray(elim)] -= D @ Y[np.asarray(sel)]
        top = perm[k0:k0 + bw]
        L11 = np.tril(LU[k0:k0 + bw, k0:k0 + bw], -1) + np.eye(bw)
        Y[top] = solve_triangular(L11, Y[top], lower=True, unit_diagonal=True)
    return Y[perm]


def block_solve(f: BlockFactorization, B: np.ndarray) -> np.ndarray:
    """x with A x = B from the block factorization."""
    Y = block_forward(f, B)
    X = solve_triangular(np.triu(f.LU), Y, lower=False)
    return X.reshape(np.shape(B))
