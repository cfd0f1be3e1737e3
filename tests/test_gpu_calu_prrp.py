"""GPU parity of CALU_PRRP (Section 3.1) against the CPU oracle.

Same bar as LU_PRRP: identical permutation, backward error <= 1e-15 n,
factors within 1e-9 max|LU|, interchange count, tree height and the largest
block-L entry equal, per-step growth within (1 + tau b)^(H+1) (checked
through the oracle on the same pivots), and one tile reproduces LU_PRRP
exactly.
"""
import numpy as np
import pytest

from oracle import lu as olu
from paper_1208_2451_amd import inputs
from tests.gpu_util import announce, backward_error, gpu_factor

pytestmark = pytest.mark.gpu


def _compare(A, b, tau, tree, tile_rows, tag=""):
    n = A.shape[0]
    announce("calu_prrp", tag, "n=%d b=%d tau=%g tree=%s tile_rows=%d" % (n, b, tau, tree, tile_rows))
    LUg, permg, st, _, _ = gpu_factor(A, b, tau, method="calu", tree=tree, tile_rows=tile_rows)
    f = olu.calu_prrp(A, b, tau, tile_rows=tile_rows, tree=tree)
    assert st["info"] == f.info == 0
    assert np.array_equal(permg, f.perm), "pivot permutation differs from the oracle"
    assert backward_error(A, LUg, permg) <= 1e-15 * n
    assert np.abs(LUg - f.LU).max() <= 1e-9 * np.abs(f.LU).max()
    assert st["swaps"] == f.swaps
    assert st["tree_height"] == f.tree_height
    assert f.step_growth_ok
    assert st["g_W"] == pytest.approx(f.g_W, rel=1e-9)
    # the root's block L = A21 A11^-1 (formed here through the inverse of the
    # winners' block) against the oracle's (R11^-1 R12)^T
    assert st["max_block_L"] == pytest.approx(f.max_block_L, rel=1e-9)
    return st, f


@pytest.mark.parametrize("tree", ["binary", "flat"])
# b = 12 and 20: the root inverse ends on a block of 4 columns
@pytest.mark.parametrize("n,b,tr", [(256, 16, 32), (300, 16, 40), (250, 16, 39), (200, 8, 24),
                                    (230, 12, 30), (200, 20, 45)])
def test_calu_random(tree, n, b, tr):
    A, _ = inputs.randn_system(n, n + b + tr)
    _compare(A, b, 2.0, tree, tr, tag="randn")


@pytest.mark.parametrize("tree", ["binary", "flat"])
def test_calu_forced_exchanges(tree):
    A, _ = inputs.randn_system(160, 12)
    st, f = _compare(A, 8, 1.05, tree, 24, tag="tau=1.05")
    assert f.swaps > 0


def test_calu_wilkinson_binary():
    _compare(inputs.wilkinson(256), 16, 2.0, "binary", 32, tag="wilkinson")


def test_calu_one_tile_is_lu_prrp():
    A, _ = inputs.randn_system(192, 4)
    announce("calu one tile n=192 b=32")
    LU1, p1, _, _, _ = gpu_factor(A, 32, 2.0)
    LU2, p2, st, _, _ = gpu_factor(A, 32, 2.0, method="calu", tile_rows=1000)
    assert np.array_equal(p1, p2)
    assert np.array_equal(LU1, LU2)
    assert st["tree_height"] == 0


def test_calu_b128_tiles512_n2048():
    A, _ = inputs.randn_system(2048, 31)
    st, f = _compare(A, 128, 2.0, "binary", 512, tag="cfg3-shape")
    assert st["tree_height"] == 2
