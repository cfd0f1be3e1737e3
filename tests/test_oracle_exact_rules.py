"""Exact-rational pins of the oracle's selection rules, and the computations
that rule out two growth factors printed for pathological matrices.

1. The strong RRQR interchange rule (Appendix A, Algorithm "Strong RRQR"):
   every interchange, in order, is replayed in exact rational arithmetic.  The
   ratio |det(A11 with slot i replaced by row j)| / |det A11| is |M_ij|
   (Cramer's rule), and the rule takes the largest ratio above tau, ties to
   the lowest row, then the lowest slot; the incoming row takes slot i.  Cases
   are kept only where the rule is decided by exact comparisons; the suite
   asserts that some steps have a largest violator that is not the first one
   in column order, and some panels hold duplicated rows (exact ties).

2. The tournament of CALU_PRRP (Section 3.1): leaves and tree nodes are
   replayed with exact greedy Gram-determinant selections and exact Cramer
   exchanges, a node stacking its left child's candidates over its right
   child's (each in increasing row order) and exact ties going to the lowest
   stacked position.  Panels whose right tiles hold copies of rows of the
   left tiles make the stacking order decide the winners; the suite asserts
   that the opposite order would change some of them.

3. Foster's matrix (c = 1, h = 1, k = 2/3; Tables "tab_foster", "ftfoster",
   "btfoster"): in the first panel, rows b .. n-1 are identical, so every
   nonsingular choice of b pivot rows is the top block, or the top block
   without one row e plus one copy of that repeated row.  The first Schur
   complement then has an entry of size at least 2.65 in the last column, for
   every such choice and every b of the tables.  The growth factor of Section
   2.2 is a maximum over all intermediate entries, so g_W >= 2.65 for LU_PRRP
   and for CALU_PRRP with any tree, tile layout or tie rule: the 1.33 printed
   for CALU_PRRP cannot be g_W.  It is the largest entry of the first block
   row of U for the two best choices.

4. Wright's matrix (h = 0.3; Tables "tab_wright", "ftwright", "btwright"):
   |det A| > 1 with max|A| = 1, so some pivot of any LU factorization exceeds
   1 in magnitude and g_W > 1: the printed g_W = 1 is not attainable.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import lu, rules
from oracle.srrqr import strong_rrqr
from paper_1208_2451_amd import inputs


# ------------------------------------------------------------ exact helpers

def _det(M):
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
            if f:
                for k in range(j, n):
                    M[i][k] -= f * M[j][k]
    return det


def _gram(rows):
    if not rows:
        return Fraction(1)
    return _det([[sum(a * b for a, b in zip(r1, r2)) for r2 in rows] for r1 in rows])


class _Undecided(Exception):
    """A comparison of the rule is too close for floating point to decide the
    same way (the oracle works in binary64 with tie bins of 2^-33)."""


def _strict_max(items, margin=Fraction(1, 2 ** 20)):
    """items: (value, order) pairs; the largest value, lowest order among exact
    ties.  Raises _Undecided when the runner-up differs by less than margin
    relative without being exactly equal."""
    best = max(v for v, _ in items)
    for v, _ in items:
        if v != best and best - v <= margin * best:
            raise _Undecided()
    return min(o for v, o in items if v == best)


def _exact_srrqr(rows, cand, tau):
    """Exact replay of QRCP + interchanges on the rows listed in ``cand``
    (positions into ``rows``, in stacking order: exact ties go to the earliest
    position).  Returns (selection as positions in slot order, swap log of
    (slot, incoming position, outgoing position), whether some interchange's
    largest violator was not the first violating entry in column order)."""
    b = len(rows[0])
    S = []
    for _ in range(b):
        gS = _gram([rows[c] for c in S])
        items = [(_gram([rows[c] for c in S] + [rows[c]]) / gS, t)
                 for t, c in enumerate(cand) if c not in S]
        S.append(cand[_strict_max(items)])
    log, first_not_max = [], False
    tau = Fraction(tau)
    for _ in range(64 * b):
        d0 = _det([rows[c] for c in S])
        assert d0 != 0
        items, first = [], None
        rest = [c for c in cand if c not in S]
        for t, j in enumerate(rest):               # lowest row first,
            for i in range(b):                     # then lowest slot
                sub = [rows[c] for c in S]
                sub[i] = rows[j]
                r = abs(_det(sub) / d0)
                if r > tau and first is None:
                    first = (i, j)
                if abs(r - tau) <= tau / 2 ** 20 and r != tau:
                    raise _Undecided()
                items.append((r, t * b + i))
        best = _strict_max(items)
        rmax = max(v for v, _ in items)
        if not rmax > tau:
            break
        t, i = divmod(best, b)
        j = rest[t]
        first_not_max |= first != (i, j)
        log.append((i, j, S[i]))
        S[i] = j
    return S, log, first_not_max


def _frac_rows(P):
    return [[Fraction(float(v)) for v in row] for row in P]


# ------------------------------------------------- 1. the interchange rule

def _exchange_cases():
    """Panels whose rows come from a subspace with decaying scales, where
    QR with column pivoting is often not yet within tau = 1.01."""
    cases = []
    g = np.random.default_rng(2024)
    for k in range(32):
        m, b = (14, 4) if k % 2 else (10, 3)
        scales = np.array([1.0, 1e-1, 1e-2, 1e-3])[:b]
        P = g.standard_normal((m, b)) @ (g.standard_normal((b, b)) * scales)
        if k % 4 == 3:      # duplicated rows: exact ties between distinct rows
            src = g.choice(m, size=2, replace=False)
            dst = g.choice([r for r in range(m) if r not in src], size=2, replace=False)
            P[dst] = P[src]
        cases.append(P)
    return cases


def test_exchange_rule_replayed_exactly():
    tau = 1.01
    checked = swaps = bites = dup_cases = 0
    for P in _exchange_cases():
        rows = _frac_rows(P)
        try:
            sel, log, first_not_max = _exact_srrqr(rows, list(range(len(rows))), tau)
        except _Undecided:
            continue
        res = strong_rrqr(P, tau)
        assert res.swap_log == log, (res.swap_log, log)
        assert res.sel == sel
        checked += 1
        swaps += len(log)
        bites += first_not_max
        dup_cases += len({tuple(r) for r in P.tolist()}) < len(P)
    # the replay is decisive: enough panels, interchanges, steps whose largest
    # violator is not the first one, and panels with exact ties
    assert checked >= 20
    assert swaps >= 15
    assert bites >= 2
    assert dup_cases >= 4


def test_exchange_tie_goes_to_lowest_row():
    """Two identical candidate rows violate equally: the lower one enters."""
    g = np.random.default_rng(77)
    for _ in range(200):
        P = g.standard_normal((9, 3))
        res = strong_rrqr(P, 1.01)
        if not res.swap_log:
            continue
        _, j, _ = res.swap_log[0]
        # put a copy of the first incoming row above it and below it
        for pos in (0, 8):
            if pos == j or pos in res.qrcp_order:
                continue
            Q = P.copy()
            Q[pos] = P[j]
            r2 = strong_rrqr(Q, 1.01)
            if not r2.swap_log or r2.qrcp_order != res.qrcp_order:
                continue
            assert r2.swap_log[0][1] == min(pos, j)
            return
    pytest.fail("no panel with a usable first interchange")


# ------------------------------------------------------- 2. the tournament

def _tiles(m, tile_rows, b):
    bounds = [[s, min(s + tile_rows, m)] for s in range(0, m, tile_rows)]
    if len(bounds) > 1 and bounds[-1][1] - bounds[-1][0] <= b:
        bounds[-2][1] = bounds[-1][1]
        bounds.pop()
    return bounds


def _exact_tournament(rows, tile_rows, tree, tau, left_first=True):
    b = len(rows[0])
    bounds = _tiles(len(rows), tile_rows, b)

    def node(stacked):
        return _exact_srrqr(rows, stacked, tau)[0]

    def stack(left, right):
        return sorted(left) + sorted(right) if left_first else sorted(right) + sorted(left)

    if tree == "binary":
        level = [node(list(range(a, e))) for a, e in bounds]
        while len(level) > 1:
            nxt = [node(stack(level[i], level[i + 1])) for i in range(0, len(level) - 1, 2)]
            if len(level) % 2:
                nxt.append(level[-1])
            level = nxt
        return level[0]
    acc = node(list(range(*bounds[0])))
    for a, e in bounds[1:]:
        acc = node(stack(acc, list(range(a, e))))
    return acc


def _tournament_cases():
    g = np.random.default_rng(31)
    out = []
    for k in range(16):
        b = 3
        tile_rows = 5 if k % 2 else 6
        m = tile_rows * (3 + k % 2) + (k % 3)
        P = g.standard_normal((m, b))
        if k % 2 == 0:
            # copies of large rows of the first tile in later tiles: exact ties
            # between the children of a node
            src = g.choice(tile_rows, size=2, replace=False)
            P[src] *= 6.0
            for t, s in enumerate(src):
                P[tile_rows * (t + 1) + 1] = P[s]
        out.append((P, tile_rows, "binary" if k % 4 < 2 else "flat"))
    return out


def test_tournament_replayed_exactly():
    tau = 1.05
    checked = order_matters = 0
    for P, tile_rows, tree in _tournament_cases():
        rows = _frac_rows(P)
        try:
            want = _exact_tournament(rows, tile_rows, tree, tau)
            other = _exact_tournament(rows, tile_rows, tree, tau, left_first=False)
        except _Undecided:
            continue
        got, _ = lu.tournament(P, tau, tile_rows, tree)
        assert got == want, (tree, got, want)
        checked += 1
        order_matters += other != want
    assert checked >= 12
    # the stacking order is decisive in some cases, so a node that stacked the
    # right child first would fail this pin
    assert order_matters >= 3


# ------------------------------------------------ 3. Foster: g_W >= 2.65

def _foster_panel_exact(b):
    third = Fraction(1, 3)
    T = []
    for i in range(b):
        r = [Fraction(0)] * b
        if i == 0:
            r[0] = Fraction(1)
        else:
            r[0] = -third
            for j in range(1, i):
                r[j] = -2 * third
            r[i] = 2 * third
        T.append(r)
    rstar = [-third] + [-2 * third] * (b - 1)
    return T, rstar


@pytest.mark.parametrize("b", [8, 16, 32, 64, 128])
def test_foster_first_schur_complement_forces_growth(b):
    """Every nonsingular pivot choice of the first Foster panel (kh = 2/3,
    c = 1) leaves a last-column entry of at least 2.65 in the first Schur
    complement.  Top rows hold -1 in the last column; the repeated row r*
    (rows b..n-1 restricted to the panel) holds -1, or -1/3 for row n-1."""
    T, rstar = _foster_panel_exact(b)
    x = [Fraction(0)] * b                      # r* = sum_k x_k T_k
    for j in range(b - 1, -1, -1):
        x[j] = (rstar[j] - sum(x[k] * T[k][j] for k in range(j + 1, b))) / T[j][j]
    assert all(v != 0 for v in x)
    forced = {}
    # pivots = top block: rows i >= b get -1 + sum(x) (or -1/3 + sum(x))
    forced["top"] = min(abs(-1 + sum(x)), abs(Fraction(-1, 3) + sum(x)))
    maxM = {"top": max(abs(v) for v in x)}
    for e in range(b):
        # row e = sum_{k != e} mu_k T_k + c r*
        mu = [-x[k] / x[e] for k in range(b) if k != e]
        c = 1 / x[e]
        forced[e] = min(abs(-1 + sum(mu) + c * a) for a in (Fraction(1), Fraction(1, 3)))
        maxM[e] = max([abs(v) for v in mu] + [abs(c), Fraction(1)])
    assert min(forced.values()) >= Fraction(265, 100)
    # the least growth among all choices is excluding row 1 (|M| <= 1), 8/3
    # up to 2^-b terms; LU_PRRP's strong RRQR reaches it
    best = min(forced, key=lambda k: forced[k])
    assert best == 1 and maxM[1] == 1
    assert abs(float(forced[1]) - 8.0 / 3.0) < 0.02


def test_foster_printed_133_is_first_block_row_of_u():
    """For the two best first-panel choices (excluding row 0 or row 1) the
    first block row of U, i.e. the factor of the selected rows, peaks at
    4/3: the only place a 1.33 appears."""
    n, b = 96, 8
    A = inputs.foster(n)
    for e in (0, 1):
        sel = [r for r in range(b) if r != e] + [b]
        _, _, U = sla.lu(A[sel])
        assert abs(np.abs(U).max() - 4.0 / 3.0) < 1e-12


def test_oracle_calu_prrp_foster_meets_the_bound():
    """The oracle's CALU_PRRP reaches the least possible g_W, 8/3, on Foster
    with leaves of 2b rows (binary and flat trees)."""
    n, b = 256, 8
    A = inputs.foster(n)
    for tree in ("binary", "flat"):
        f = lu.calu_prrp(A, b, 2.0, tile_rows=2 * b, tree=tree)
        assert abs(f.g_W - 8.0 / 3.0) < 1e-12


def test_foster_norm_columns_are_tie_decided():
    """Rows b..n-1 of the first Foster panel are identical, so which copy
    enters (and the slot order) is an exact tie.  The lowest-index and the
    highest-index tie rules give the same g_W = 8/3 but ||U||_1 differing by
    more than an order of magnitude: the printed norm columns record the
    paper's rounding-decided choices, not a property of the method."""
    n, b = 256, 8
    A = inputs.foster(n)
    f_lo = lu.lu_prrp(A, b, 2.0)

    def highest(v):
        k = rules.key(v)
        return int(np.flatnonzero(k == k.max())[-1])

    saved = rules.argmax_lowest
    rules.argmax_lowest = highest      # a planted reading, on the CPU oracle only
    try:
        f_hi = lu.lu_prrp(A, b, 2.0)
    finally:
        rules.argmax_lowest = saved
    assert abs(f_lo.g_W - 8.0 / 3.0) < 1e-12 and abs(f_hi.g_W - 8.0 / 3.0) < 1e-12
    u_lo = np.abs(np.triu(f_lo.LU)).sum(0).max()
    u_hi = np.abs(np.triu(f_hi.LU)).sum(0).max()
    assert max(u_lo, u_hi) > 10 * min(u_lo, u_hi)


# ------------------------------------------------- 4. Wright: g_W > 1

def _wright_blocks(n, E):
    A = np.eye(n)
    for i in range(1, n // 2):
        A[2 * i:2 * i + 2, 2 * (i - 1):2 * i] = -E
    A[0:2, n - 2:n] += np.eye(2)
    return A


def test_wright_growth_exceeds_one_for_any_pivoting():
    """|det A| = prod |u_ii| for any A = Pi L U with unit L, so
    max |u_ii| >= |det A|^(1/n) > 1 = max|A| (h = 0.3, n = 2048), with the
    exact exp(M h) and with its first-order form I + M h alike.

    Eliminating the block bidiagonal rows gives det A = det(I + E^(N-1))
    (N = n/2 blocks, E the subdiagonal block with its sign removed), checked
    against a determinant at n = 16; at n = 2048 GEPP is too unstable on this
    matrix for a computed determinant, so the eigenvalues of the symmetric E
    give it instead."""
    h = 0.3
    M = np.array([[-1.0 / 6.0, 1.0], [1.0, -1.0 / 6.0]])
    w, V = np.linalg.eigh(M * h)
    readings = {"exact": (V * np.exp(w)) @ V.T, "first-order": np.eye(2) + M * h}
    assert np.allclose(_wright_blocks(16, readings["exact"]), inputs.wright(16, h), atol=1e-15)
    for name, E in readings.items():
        lam = np.linalg.eigvalsh(E)
        small = _wright_blocks(16, E)
        assert np.linalg.slogdet(small)[1] == pytest.approx(np.log(np.abs(1 + lam ** 7)).sum(), rel=1e-12)
        n = 2048
        logdet = np.log1p(np.abs(lam) ** (n // 2 - 1)).sum()
        assert np.abs(_wright_blocks(n, E)).max() == 1.0
        assert np.exp(logdet / n) > 1.1, name        # max |u_ii| > 1.1 = 1.1 max|A|
    f = lu.lu_prrp(inputs.wright(256, h), 16, 2.0)
    assert f.g_W > 1.0
