"""Repeated factorizations of one matrix are bitwise identical.

The strong-RRQR kernel exchanges pivots between workgroups through device
memory and LDS; a missing barrier or an unordered read shows up as a run that
differs from the others (and usually from the oracle) only now and then.  Each
case runs several times in one process and every run must equal the first.
"""
import numpy as np
import pytest

from paper_1208_2451_amd import inputs
from tests.gpu_util import announce, gpu_factor

pytestmark = pytest.mark.gpu

REPEATS = 6


@pytest.mark.parametrize("method,tree,n,b,tr", [
    ("lu", None, 384, 16, 0),
    ("lu", None, 520, 64, 0),
    ("calu", "binary", 300, 16, 40),
    ("calu", "flat", 250, 16, 39),
    ("calu", "binary", 200, 8, 24),
])
def test_repeated_runs_identical(method, tree, n, b, tr):
    A, _ = inputs.randn_system(n, 31 * n + b)
    announce("determinism", method, tree, "n=%d b=%d" % (n, b))
    kw = {} if method == "lu" else dict(method="calu", tree=tree, tile_rows=tr)
    LU0, p0, st0, _, _ = gpu_factor(A, b, 2.0, **kw)
    assert st0["info"] == 0
    for _ in range(REPEATS - 1):
        LU, p, st, _, _ = gpu_factor(A, b, 2.0, **kw)
        assert np.array_equal(p, p0)
        assert np.array_equal(LU, LU0)
        assert st["g_W"] == st0["g_W"] and st["swaps"] == st0["swaps"]
