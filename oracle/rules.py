"""The deterministic pivot tie rule (the paper leaves tie-breaking open).

QR with column pivoting, the strong RRQR exchange and partial pivoting each pick
the candidate of largest magnitude.  The paper says nothing about equal or
nearly equal candidates, and structured inputs (the Wilkinson matrix) have
exact ties between distinct rows that rounding would otherwise decide.

Reading used here and in the GPU library: two non-negative magnitudes are
*tied* when their binary64 encodings agree after the 19 low mantissa bits are
dropped (they share sign, exponent and the 33 leading mantissa bits, a relative
bin of 2^-33 ~ 1.2e-10).  Among tied candidates the lowest row index of the
current matrix wins; for the exchange step (a row j and a slot i) the lowest
row, then the lowest slot.  The threshold test of the exchange loop,
|M_ij| > tau, is taken on the same truncated encodings, so values within the
bin of tau do not count as violations.
"""
from __future__ import annotations

import numpy as np

DROP_BITS = 19


def key(v) -> np.ndarray:
    """Truncated binary64 encoding of non-negative magnitudes (uint64)."""
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    return a.view(np.uint64) >> np.uint64(DROP_BITS)


def argmax_lowest(v) -> int:
    """Index of the largest magnitude under the tie rule (lowest index on ties).

    ``v`` is a 1-D array of non-negative values ordered by row index.
    """
    k = key(v)
    return int(np.flatnonzero(k == k.max())[0])


def exceeds(v: float, tau: float) -> bool:
    """|v| > tau beyond the tie bin of tau."""
    return bool(key(abs(v)) > key(tau))
