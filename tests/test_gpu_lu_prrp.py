"""GPU parity of LU_PRRP (FP64) against the CPU oracle.

Bar (identical for every case): the permutation equals the oracle's exactly;
||A[perm] - L U||_F / (n ||A||_F) <= 1e-15; the factors agree with the
oracle's element by element within 1e-9 max|LU| (same pivots, different
rounding order); growth, block-L certificate and interchange count agree.
"""
import numpy as np
import pytest

from oracle import lu as olu
from paper_1208_2451_amd import inputs
from tests.gpu_util import TAU_TOL, announce, backward_error, gpu_factor

pytestmark = pytest.mark.gpu


def _compare(A, b, tau=2.0, tag=""):
    n = A.shape[0]
    announce("lu_prrp", tag, "n=%d b=%d tau=%g" % (n, b, tau))
    LUg, permg, st, _, _ = gpu_factor(A, b, tau)
    f = olu.lu_prrp(A, b, tau)
    assert st["info"] == f.info == 0
    assert np.array_equal(permg, f.perm), "pivot permutation differs from the oracle"
    assert backward_error(A, LUg, permg) <= 1e-15 * n
    scale = np.abs(f.LU).max()
    assert np.abs(LUg - f.LU).max() <= 1e-9 * scale
    assert st["swaps"] == f.swaps
    assert st["g_W"] == pytest.approx(f.g_W, rel=1e-9)
    assert st["g_U"] == pytest.approx(f.g_U, rel=1e-9)
    if n > b:
        assert st["max_block_L"] <= tau * TAU_TOL
        assert st["max_block_L"] == pytest.approx(f.max_block_L, rel=1e-9)
    return LUg, permg, st, f


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_randn_256_b16(seed):
    A, _ = inputs.randn_system(256, seed)
    _compare(A, 16, tag="randn seed=%d" % seed)


def test_wilkinson_256_b16():
    _compare(inputs.wilkinson(256), 16, tag="wilkinson")


@pytest.mark.parametrize("n,b", [(200, 16), (257, 32), (300, 64), (129, 128), (64, 64), (33, 8)])
def test_ragged_and_single_panel(n, b):
    A, _ = inputs.randn_system(n, 1000 + n)
    _compare(A, b, tag="ragged")


def test_b1_is_gepp():
    A, _ = inputs.randn_system(64, 77)
    _compare(A, 1, tag="b=1")


@pytest.mark.parametrize("n,b", [(128, 16), (96, 8)])
def test_forced_exchanges_tau_near_one(n, b):
    A, _ = inputs.randn_system(n, 5)
    _, _, st, f = _compare(A, b, tau=1.05, tag="tau=1.05")
    assert f.swaps > 0


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny(n):
    A, _ = inputs.randn_system(n, 3)
    _compare(A, 1 if n == 1 else 2 if n == 3 else 1, tag="tiny")


def test_multi_workgroup_panel_1000_b64():
    A, _ = inputs.randn_system(1000, 11)
    _compare(A, 64, tag="multi-wg")


def test_foster_and_wright_512():
    _compare(inputs.foster(512), 32, tag="foster")
    _compare(inputs.wright(512), 32, tag="wright")


def test_singular_matrix_sets_info():
    n = 64
    A, _ = inputs.randn_system(n, 9)
    A[:, 5] = 0.0                       # exactly rank deficient
    announce("lu_prrp singular n=64 b=16")
    _, _, st, _, _ = gpu_factor(A, 16, 2.0)
    f = olu.lu_prrp(A, 16, 2.0)
    assert f.info > 0
    assert st["info"] == f.info


def test_nonfinite_input_sets_info():
    A, _ = inputs.randn_system(48, 4)
    A[3, 7] = np.nan
    announce("lu_prrp nan n=48 b=16")
    _, _, st, _, _ = gpu_factor(A, 16, 2.0)
    assert st["info"] == -1


def test_deterministic_rerun():
    A, _ = inputs.randn_system(512, 21)
    announce("lu_prrp determinism n=512 b=32")
    LU1, p1, _, _, _ = gpu_factor(A, 32)
    LU2, p2, _, _, _ = gpu_factor(A, 32)
    assert np.array_equal(p1, p2)
    assert np.array_equal(LU1, LU2)
