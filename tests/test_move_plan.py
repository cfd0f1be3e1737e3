"""The panel kernel's parallel derivation of the moves of Pi_j.

With look-ahead the strong-RRQR kernel forms the row moves of Pi_j itself
(Algorithm "LU_PRRP factorization": Pi_j is the sequence of interchanges of
position s with the current position of the s-th selected row).  Instead of
replaying the interchanges one by one it uses two facts: slot s's row sits at
Q[s] = sel[s] when step s comes unless sel[s] < s, in which case it has moved
along Q from sel[s] and Q[s] is the first position >= s on that chain; and a
top-block row that is not selected moves along Q from its own position until
it leaves the top block.  This file restates that derivation (lane rounds as
the kernel runs them) and checks it against the interchanges applied one by
one with the oracle's row-swap routine, on random and adversarial selections.
"""
import numpy as np
import pytest

from oracle import lu as olu


def interchanges(sel, m):
    """Row order after Pi_j, applying the interchanges one at a time."""
    A = np.arange(m, dtype=np.float64)[:, None].copy()
    perm = np.arange(m)
    pos = np.arange(m)
    at = np.arange(m)
    for i, r in enumerate(sel):
        q = int(pos[r])
        if q != i:
            olu._swap_rows(A, perm, i, q)
            ri, rq = at[i], at[q]
            at[i], at[q] = rq, ri
            pos[rq], pos[ri] = i, q
    assert np.array_equal(A[:, 0].astype(int), perm)
    return perm


def derive_moves(sel, m, bw):
    """The kernel's rounds: returns (move list, destination of each left-out
    top-block row, number of rounds of each phase)."""
    sel = list(sel)
    # Q by rounds: an unresolved entry holds -1 - (its chase position)
    v = [sel[i] if sel[i] >= i else -1 - sel[i] for i in range(bw)]
    r1 = 0
    while any(x < 0 for x in v):
        r1 += 1
        assert r1 <= bw * bw
        old = list(v)
        for i in range(bw):
            if old[i] < 0:
                c = -1 - old[i]
                qc = old[c]
                if qc >= 0:
                    v[i] = qc if qc >= i else -1 - qc
    chosen = set(x for x in sel if x < bw)
    dest = {}
    r2 = 0
    for u in range(bw):
        if u in chosen:
            continue
        p = u
        while p < bw:
            p = v[p]
            r2 += 1
        dest[u] = p
    moves = [(t, sel[t]) for t in range(bw)] + [(dest[u], u) for u in sorted(dest)]
    return moves, dest, (r1, r2)


def apply_moves(moves, m):
    order = np.arange(m)
    src = np.arange(m)
    for d, s in moves:
        order[d] = src[s]
    return order


def _check(sel, m, bw):
    moves, dest, _ = derive_moves(sel, m, bw)
    want = interchanges(sel, m)
    assert np.array_equal(apply_moves(moves, m), want)
    # every position below the top block receives exactly one row that was
    # not selected (the near update's source-row map)
    srcmap = {}
    for t in range(m):
        if t in set(sel):
            continue
        fp = dest[t] if t < bw else t
        assert bw <= fp < m and fp not in srcmap
        srcmap[fp] = t
    assert sorted(srcmap) == list(range(bw, m))
    for fp, t in srcmap.items():
        assert want[fp] == t


@pytest.mark.parametrize("seed", range(40))
def test_random_selections(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 400))
    bw = int(rng.integers(1, min(m, 128) + 1))
    kind = seed % 3
    if kind == 0:
        sel = rng.permutation(m)[:bw]
    elif kind == 1:
        k = int(rng.integers(0, min(bw, m - bw) + 1)) if m > bw else bw
        top = rng.permutation(bw)[:bw - k] if m > bw else rng.permutation(bw)
        rest = bw + rng.permutation(m - bw)[:k] if m > bw else np.array([], dtype=int)
        sel = rng.permutation(np.concatenate([top, rest]).astype(int))
    else:
        sel = rng.permutation(min(m, 2 * bw))[:bw]
    _check([int(x) for x in sel], m, bw)


@pytest.mark.parametrize("bw", [1, 8, 64, 128])
def test_adversarial_selections(bw):
    m = 3 * bw
    cases = [
        [(i + 1) % bw for i in range(bw)],          # rotation: longest Q chains
        list(range(bw - 1, -1, -1)),                # reversal
        [bw + i for i in range(bw)],                # every row from below
        [2 * bw - 1 - i for i in range(bw)],
        list(range(bw)),                            # identity: no moves
    ]
    for sel in cases:
        _check(sel, m, bw)
    _, _, (r1, _) = derive_moves([(i + 1) % bw for i in range(bw)], m, bw)
    assert r1 <= bw                                 # rounds stay bounded


def test_last_panel_all_rows_selected():
    for bw in (1, 5, 64):
        rng = np.random.default_rng(bw)
        _check([int(x) for x in rng.permutation(bw)], bw, bw)
