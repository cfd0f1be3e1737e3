"""Pins of the oracle's QR with column pivoting and strong RRQR (Appendix A).

Each check uses something other than the oracle itself: exact rational
arithmetic (Gram and Cramer determinants), LAPACK's geqp3, and closed-form
reasoning on the Wilkinson panel.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import rules
from oracle.srrqr import qrcp, strong_rrqr
from paper_1208_2451_amd import inputs


def _frac_matrix(X):
    return [[Fraction(float(v)) for v in row] for row in X]


def _det(M):
    """Exact determinant by fraction-valued Gaussian elimination."""
    M = [row[:] for row in M]
    n = len(M)
    det = Fraction(1)
    for j in range(n):
        p = next((i for i in range(j, n) if M[i][j] != 0), None)
        if p is None:
            return Fraction(0)
        if p != j:
            M[j], M[p] = M[p], M[j]
            det = -det
        det *= M[j][j]
        for i in range(j + 1, n):
            f = M[i][j] / M[j][j]
            for k in range(j, n):
                M[i][k] -= f * M[j][k]
    return det


def _gram_det(rows):
    G = [[sum(a * b for a, b in zip(r1, r2)) for r2 in rows] for r1 in rows]
    return _det(G) if rows else Fraction(1)


@pytest.mark.parametrize("seed", range(6))
def test_qrcp_is_greedy_distance_to_span(seed):
    """Step s picks the row farthest from the span of the rows already picked:
    dist^2(r, S) = det Gram(S + r) / det Gram(S), evaluated exactly."""
    g = np.random.default_rng(seed)
    m, b = 9, 4
    P = g.standard_normal((m, b))
    rows = _frac_matrix(P)
    order, _, rdef = qrcp(P)
    assert rdef == -1
    S = []
    for s in range(b):
        gS = _gram_det([rows[i] for i in S])
        d = {c: _gram_det([rows[i] for i in S] + [rows[c]]) / gS for c in range(m) if c not in S}
        best = max(d, key=lambda c: d[c])
        assert order[s] == best
        S.append(best)


@pytest.mark.parametrize("seed", range(4))
def test_qrcp_order_matches_lapack_geqp3(seed):
    g = np.random.default_rng(100 + seed)
    m, b = 80, 12
    P = g.standard_normal((m, b))
    order, W, _ = qrcp(P)
    _, R, piv = sla.qr(P.T, pivoting=True, mode="economic")
    assert list(piv[:b]) == order
    # |R| agrees up to the sign of each row of R (Householder sign convention).
    Rm = np.abs(np.triu(W[:, order]))
    assert np.allclose(Rm, np.abs(R[:, :b]), rtol=1e-12, atol=1e-12)


def test_qrcp_wilkinson_first_panel_tie():
    """Wilkinson panel 1 (n=256, b=16): rows 15..255 all have squared norm 16
    (closed form), so the tie rule must pick row 15; rows 16..255 are equal."""
    W = inputs.wilkinson(256)
    order, _, rdef = qrcp(W[:, :16])
    assert order[0] == 15
    assert rdef == -1
    assert len(set(order)) == 16
    # Rows 16..255 are identical, so at most one of them can be selected.
    assert sum(1 for r in order if r >= 16) == 1
    assert min(r for r in order if r >= 16) == 16


def test_tie_key_ordering():
    v = np.array([1.0, 1.0 + 2.0 ** -40, 1.0 - 2.0 ** -45, 0.5, 2.0])
    k = rules.key(v)
    assert k[0] == k[1] == k[2] or k[0] == k[1]
    assert k[3] < k[0] < k[4]
    assert rules.argmax_lowest(np.array([3.0, 5.0, 5.0, 4.0])) == 1
    # 5.0 opens a bin (its low mantissa bits are zero): values a few ulps above
    # it share its bin and tie; values below it fall into the previous bin.
    assert rules.argmax_lowest(np.array([3.0, 5.0, 5.0 * (1 + 2.0 ** -49)])) == 1
    assert rules.argmax_lowest(np.array([3.0, 5.0 * (1 - 2.0 ** -50), 5.0])) == 2
    assert not rules.exceeds(2.0, 2.0)
    assert rules.exceeds(2.0 * (1 + 2.0 ** -20), 2.0)


@pytest.mark.parametrize("seed", range(8))
def test_strong_rrqr_certificate_by_cramer(seed):
    """Final selection: replacing any selected row i by any other row r changes
    |det A11| by the factor |M[i, r]| (Cramer), which must not exceed tau."""
    g = np.random.default_rng(200 + seed)
    m, b, tau = 10, 3, 1.05
    P = g.standard_normal((m, b))
    res = strong_rrqr(P, tau)
    rows = _frac_matrix(P)
    d0 = _det([rows[i] for i in res.sel])
    assert d0 != 0
    bound = Fraction(tau) * (1 + Fraction(1, 2 ** 32))
    for t, r in enumerate(res.rest):
        for i in range(b):
            sub = [rows[j] for j in res.sel]
            sub[i] = rows[r]
            ratio = abs(_det(sub) / d0)
            assert ratio <= bound
            assert abs(float(ratio) - abs(res.M[i, t])) <= 1e-12 * max(1.0, float(ratio))


@pytest.mark.parametrize("seed", range(8))
def test_strong_rrqr_swaps_grow_det(seed):
    """Each interchange multiplies |det R11| by more than tau (Appendix A), and
    the product of the ratios is the exact |det| ratio between the QRCP
    selection and the final one."""
    g = np.random.default_rng(300 + seed)
    m, b, tau = 12, 4, 1.05
    P = g.standard_normal((m, b))
    res = strong_rrqr(P, tau)
    rows = _frac_matrix(P)
    d_q = abs(_det([rows[i] for i in res.qrcp_order]))
    d_f = abs(_det([rows[i] for i in res.sel]))
    assert all(r > tau for r in res.det_ratios)
    prod = float(np.prod(res.det_ratios)) if res.det_ratios else 1.0
    assert abs(prod - float(d_f / d_q)) <= 1e-10 * float(d_f / d_q)


def test_strong_rrqr_exercises_swaps_at_tau_near_one():
    tot = 0
    for seed in range(20):
        g = np.random.default_rng(400 + seed)
        P = g.standard_normal((64, 8))
        res = strong_rrqr(P, 1.05)
        assert res.max_abs_M <= 1.05 * (1 + 2.0 ** -32)
        tot += res.swaps
    assert tot > 0


def test_strong_rrqr_qrcp_bound_random_tau2():
    """At tau = 2 on random panels QRCP alone usually meets the bound (the
    paper's observation that |R12^T R11^-T| is rarely above 3)."""
    g = np.random.default_rng(7)
    res = strong_rrqr(g.standard_normal((512, 32)), 2.0)
    assert res.max_abs_M <= 2.0 * (1 + 2.0 ** -32)


def test_rank_deficient_panel_flags():
    """Rank 2 panel with exactly zero rows: the third step meets an exactly
    zero residual, flags it, and completes the selection with the lowest
    remaining row."""
    P = np.zeros((10, 3))
    P[3] = [1.0, 2.0, 0.0]
    P[7] = [0.0, 0.0, 5.0]
    res = strong_rrqr(P, 2.0)
    assert res.rank_deficient_step == 2
    assert res.sel == [7, 3, 0]
