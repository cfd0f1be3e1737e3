"""Strong rank revealing QR of a panel's transpose -- oracle (test infrastructure).

Follows Appendix A ("Strong RRQR"): first a classical QR with column pivoting of
B^T = P^T, then, while some |(R11^-1 R12)_ij| exceeds tau, interchange the
selected column i with the unselected column j and re-triangularise R.  The
columns of P^T are the rows of the panel P, so the selected columns are the
panel's pivot rows (Section 2.1 picks a panel's b pivot rows by strong RRQR of
the panel's transpose).

Readings where the paper is silent:
  * QRCP recomputes the squared norm of every candidate's trailing part at each
    step (no norm downdating) and picks by ``rules.argmax_lowest``.
  * The exchange loop picks the violating entry of largest magnitude (tie rule:
    lowest row, then lowest slot); the incoming row takes the slot of the
    outgoing one, the outgoing row rejoins the unselected rows, which are kept
    in increasing row order.
  * After an interchange the whole R is re-triangularised by a fresh QR of its
    selected columns (the "QR updates" of Appendix A done by recomputation).
  * If QRCP meets an exactly zero residual (rank-deficient panel) it keeps
    picking the lowest-index remaining rows and the exchange loop is skipped.

Pinned by tests/test_oracle_srrqr.py: brute-force greedy selection in exact
rational arithmetic, LAPACK geqp3 order, Cramer-rule determinant checks of
the final selection, and the |det R11| growth of every interchange; and by
tests/test_oracle_exact_rules.py: every interchange, in order, against an
exact-rational replay of the rule (largest Cramer ratio |det| growth, ties to
the lowest row, then the lowest slot), on panels with and without duplicated
rows.
"""
from __future__ import annotations

from bisect import insort
from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

from . import rules


@dataclass
class SRRQRResult:
    sel: list          # selected panel rows in slot order (panel-relative)
    rest: list         # unselected panel rows, increasing
    M: np.ndarray      # R11^-1 R12, shape (b, len(rest)); column t <-> rest[t]
    R: np.ndarray      # b x m triangular factor, column c <-> panel row c
    swaps: int = 0
    rank_deficient_step: int = -1   # first QRCP step with a zero residual
    qrcp_order: list = field(default_factory=list)
    det_ratios: list = field(default_factory=list)  # |det R11| growth per swap
    swap_log: list = field(default_factory=list)    # (slot, row in, row out) per swap

    @property
    def max_abs_M(self) -> float:
        return float(np.abs(self.M).max()) if self.M.size else 0.0


def qrcp(P: np.ndarray):
    """Householder QR with column pivoting of P^T (P is m x b, m >= b).

    Returns (order, W, rank_deficient_step): ``order`` lists the b chosen
    panel rows in pivot order; ``W`` is the b x m array of P^T after the b
    reflections, i.e. the R factor with its columns left in panel-row order.
    """
    P = np.asarray(P, dtype=np.float64)
    m, b = P.shape
    if m < b:
        raise ValueError("panel needs at least as many rows as columns")
    W = np.array(P.T)                    # b x m
    chosen = np.zeros(m, dtype=bool)
    order = []
    rdef = -1
    for s in range(b):
        tail = W[s:, :]
        nu = (tail * tail).sum(axis=0)   # squared residual norm of each row
        cand = np.flatnonzero(~chosen)
        p = int(cand[rules.argmax_lowest(nu[cand])])
        if nu[p] == 0.0 and rdef < 0:
            rdef = s
        order.append(p)
        chosen[p] = True
        x = W[s:, p].copy()
        nx = np.sqrt((x * x).sum())
        if nx > 0.0:
            alpha = -np.copysign(nx, x[0])
            v = x
            v[0] -= alpha
            beta = 2.0 / (v @ v)
            W[s:, :] -= np.outer(v, beta * (v @ W[s:, :]))
            W[s + 1:, p] = 0.0
            W[s, p] = alpha
    return order, W, rdef


def _ratio_matrix(W: np.ndarray, sel, rest) -> np.ndarray:
    R11 = np.triu(W[:, sel])
    return solve_triangular(R11, W[:, rest], lower=False)


def strong_rrqr(P: np.ndarray, tau: float, max_swaps: int | None = None) -> SRRQRResult:
    """Strong RRQR (empty R22 block) of P^T; Appendix A."""
    P = np.asarray(P, dtype=np.float64)
    m, b = P.shape
    order, W, rdef = qrcp(P)
    sel = list(order)
    in_sel = set(sel)
    rest = [c for c in range(m) if c not in in_sel]
    res = SRRQRResult(sel=sel, rest=rest, M=np.zeros((b, 0)), R=W, qrcp_order=list(order),
                      rank_deficient_step=rdef)
    if not rest:
        return res
    if rdef >= 0:
        res.M = np.full((b, len(rest)), np.nan)
        return res
    cap = max_swaps if max_swaps is not None else 64 * b
    tkey = rules.key(tau)
    while True:
        M = _ratio_matrix(W, sel, rest)
        K = rules.key(np.abs(M))
        kmax = K.max()
        if not kmax > tkey:
            res.M = M
            break
        hit = K == kmax
        j = int(np.flatnonzero(hit.any(axis=0))[0])      # lowest row index
        i = int(np.flatnonzero(hit[:, j])[0])            # then lowest slot
        if res.swaps >= cap:
            raise RuntimeError("strong RRQR exchange did not terminate")
        res.det_ratios.append(abs(M[i, j]))
        out_row = sel[i]
        res.swap_log.append((i, rest[j], out_row))
        sel[i] = rest[j]
        del rest[j]
        insort(rest, out_row)
        # QR of R with the two columns interchanged: re-triangularise.
        Q, _ = np.linalg.qr(W[:, sel])
        W = Q.T @ W
        for t, c in enumerate(sel):
            W[t + 1:, c] = 0.0
        res.swaps += 1
    res.sel, res.rest, res.R = sel, rest, W
    return res
