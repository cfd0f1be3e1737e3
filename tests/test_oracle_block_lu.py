"""Pins of the block parallel / block pairwise LU_PRRP oracle
(oracle/block_lu.py, Section 5 and Appendix E) against facts fixed outside
it: parallel and pairwise pivoting (its b = 1 case) replayed in exact
rational arithmetic from their definitions, LU_PRRP (its one-tile case, as
Section 5 states for P = 1), the recorded transformations reproducing U, the
strong-RRQR bound on the multipliers and the per-panel growth bound."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import block_lu as ob
from oracle import lu as olu

U = 2.0 ** -53


def _distinct_int_matrix(n, seed):
    g = np.random.default_rng(seed)
    v = g.choice(np.arange(1, 10 ** 6), size=n * n, replace=False)
    s = g.choice([-1, 1], size=n * n)
    return (v * s).reshape(n, n).astype(float)


def _exact_b1(A, tile_rows, tree):
    """Gaussian elimination with parallel pivoting (binary tree) or pairwise
    pivoting (flat tree), exactly: per column, the active rows are cut into
    consecutive groups of tile_rows (a last group of one row joins the one
    before); in each group the row with the largest |entry| is kept and every
    other row r becomes r - (a_r / a_kept) kept, storing the multiplier in
    its column; the kept rows then meet pairwise (binary: neighbours, an odd
    last one passes up; flat: the running row against each next group) in
    the same way; the final row swaps into the pivot position."""
    n = A.shape[0]
    M = [[Fraction(int(x)) for x in row] for row in A]
    perm = list(range(n))
    for k in range(n):
        m = n - k
        starts = list(range(0, m, tile_rows))
        groups = [list(range(k + s, k + min(s + tile_rows, m))) for s in starts]
        if len(groups) > 1 and len(groups[-1]) <= 1:
            last = groups.pop()
            groups[-1] = groups[-1] + last

        def meet(rows):
            mags = [abs(M[r][k]) for r in rows]
            best = max(mags)
            assert mags.count(best) == 1, "exact tie: choose another matrix"
            keep = rows[mags.index(best)]
            for r in rows:
                if r != keep:
                    f = M[r][k] / M[keep][k]
                    for c in range(k + 1, n):
                        M[r][c] -= f * M[keep][c]
                    M[r][k] = f
            return keep

        if len(groups) == 1:
            root = meet(groups[0])
        elif tree == "binary":
            level = [meet(g) for g in groups]
            while len(level) > 1:
                nxt = [meet(sorted([level[i], level[i + 1]])) for i in range(0, len(level) - 1, 2)]
                if len(level) % 2:
                    nxt.append(level[-1])
                level = nxt
            root = level[0]
        else:
            root = meet(groups[0])
            for g in groups[1:]:
                root = meet(sorted([root]) + g)
        if root != k:
            M[k], M[root] = M[root], M[k]
            perm[k], perm[root] = perm[root], perm[k]
    return M, perm


@pytest.mark.parametrize("tree", ["binary", "flat"])
@pytest.mark.parametrize("n,tile_rows,seed", [(9, 2, 1), (12, 3, 2), (11, 4, 3), (10, 1, 4)])
def test_b1_is_parallel_or_pairwise_pivoting_exactly(tree, n, tile_rows, seed):
    # tile_rows = 1 with the flat tree is Sorensen's pairwise pivoting: the
    # running pivot row meets each next row in turn
    A = _distinct_int_matrix(n, seed)
    M, perm = _exact_b1(A, tile_rows, tree)
    f = ob.block_lu_prrp(A, 1, 2.0, tile_rows, tree)
    assert list(f.perm) == perm
    E = np.array([[float(x) for x in row] for row in M])
    scale = np.abs(E).max()
    assert np.abs(f.LU - E).max() <= 1e-13 * scale


def test_b1_binary_and_flat_differ():
    # the two trees are different eliminations (not a relabelling of one)
    A = _distinct_int_matrix(12, 2)
    fb = ob.block_lu_prrp(A, 1, 2.0, 3, "binary")
    ff = ob.block_lu_prrp(A, 1, 2.0, 3, "flat")
    assert not np.allclose(fb.LU, ff.LU)


@pytest.mark.parametrize("n,b", [(48, 8), (40, 16), (37, 8)])
def test_one_tile_is_lu_prrp(n, b):
    g = np.random.default_rng(n + b)
    A = g.standard_normal((n, n))
    f = ob.block_lu_prrp(A, b, 2.0, tile_rows=10 * n, tree="binary")
    r = olu.lu_prrp(A, b, 2.0)
    assert np.array_equal(f.perm, r.perm)
    assert np.abs(np.triu(f.LU) - np.triu(r.LU)).max() <= 1e-12 * np.abs(r.LU).max()
    x_ref = np.linalg.solve(A, np.ones(n))
    assert np.abs(ob.block_solve(f, np.ones(n)) - x_ref).max() <= 1e-9 * np.abs(x_ref).max()


@pytest.mark.parametrize("tree", ["binary", "flat"])
@pytest.mark.parametrize("n,b,tile_rows", [(64, 8, 16), (70, 8, 20), (96, 16, 40)])
def test_recorded_transformations_reproduce_U(tree, n, b, tile_rows):
    g = np.random.default_rng(7 * n + b)
    A = g.standard_normal((n, n))
    f = ob.block_lu_prrp(A, b, 2.0, tile_rows, tree)
    Y = ob.block_forward(f, A)
    # the operations recorded per node, applied to A itself, give U (rows in
    # final order) and annihilate everything below it
    err = np.abs(Y - np.triu(f.LU)).max()
    assert err <= 1e3 * U * f.max_abs_W * n, err
    # every row of A appears exactly once among each panel's nodes
    for j, recs in enumerate(f.nodes):
        ids = [r for sel, el in recs for r in el]
        root = f.perm[j * b:(j + 1) * b]
        active = set(f.perm[j * b:])
        assert len(ids) == len(set(ids)) == len(active) - len(root)
        assert set(ids) | set(root) == active


@pytest.mark.parametrize("tree", ["binary", "flat"])
def test_multipliers_and_per_panel_growth_bounded(tree):
    g = np.random.default_rng(11)
    n, b, tau = 96, 8, 2.0
    A = g.standard_normal((n, n))
    f = ob.block_lu_prrp(A, b, tau, 24, tree)
    assert f.max_abs_D <= tau * (1 + 1e-12)
    assert max(f.panel_growth) <= (1 + tau * b) * (1 + 1e-12)
    assert f.tree_height == (2 if tree == "binary" else 3)


@pytest.mark.parametrize("tree", ["binary", "flat"])
def test_block_solve_backward_error(tree):
    g = np.random.default_rng(5)
    n, b = 128, 16
    A = g.standard_normal((n, n))
    x_true = g.standard_normal(n)
    rhs = A @ x_true
    f = ob.block_lu_prrp(A, b, 2.0, 32, tree)
    x = ob.block_solve(f, rhs)
    eta = np.abs(A @ x - rhs).max() / (np.abs(A).max() * np.abs(x).max() * n)
    assert eta <= 1e-14, eta
