"""Pins of the oracle's solve, refinement, metrics, bounds and flop counts."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import lu, metrics, solve
from paper_1208_2451_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("seed", range(4))
def test_residual_dot2_against_exact_rationals(seed):
    """Dot2 error bound (Ogita-Rump-Oishi): |res - r| <= u|r| + gamma_n^2 (|A||x| + |b|)."""
    g = np.random.default_rng(seed)
    n = 14
    A = g.standard_normal((n, n))
    x = np.linalg.solve(A, g.standard_normal(n))
    b = A @ x + 1e-13 * g.standard_normal(n)      # residual ~1e-13, heavy cancellation
    r = solve.residual_dot2(A, x, b)
    u = 2.0 ** -53
    gam = n * u / (1 - n * u)
    for i in range(n):
        exact = Fraction(float(b[i])) - sum(Fraction(float(A[i, j])) * Fraction(float(x[j]))
                                            for j in range(n))
        err = abs(Fraction(float(r[i])) - exact)
        scale = float(np.abs(A[i]) @ np.abs(x) + abs(b[i]))
        assert float(err) <= u * abs(float(exact)) + 2 * gam * gam * scale


def test_refine_recovers_exact_solution():
    g = np.random.default_rng(3)
    n = 64
    A = np.round(g.standard_normal((n, n)) * 16)
    xt = np.round(g.standard_normal(n) * 8)
    b = A @ xt                         # exact: small integers
    f = lu.lu_prrp(A, 8, 2.0)
    x, it, _ = solve.refine(A, f.LU, f.perm, b)
    assert np.array_equal(x, xt) or np.abs(x - xt).max() <= 1e-15 * np.abs(xt).max()


def test_refine_on_ill_conditioned_matches_lapack_refinement():
    """The refined solution does not depend on the factor used: LU_PRRP-based
    and LAPACK-getrf-based refinement agree to a few ulps (kappa = 1e6)."""
    n = 128
    A = inputs.kappa_matrix(n, 11, 1e6)
    b = np.random.default_rng(4).standard_normal(n)
    f = lu.lu_prrp(A, 16, 2.0)
    x1, _, _ = solve.refine(A, f.LU, f.perm, b)
    lu_, piv = sla.lu_factor(A)
    perm = np.arange(n)
    for j, p in enumerate(piv):
        perm[[j, p]] = perm[[p, j]]
    x2, _, _ = solve.refine(A, lu_, perm, b)
    assert np.abs(x1 - x2).max() <= 1e-14 * np.abs(x2).max()
    x0 = solve.solve(f.LU, f.perm, b)
    assert np.abs(x0 - x2).max() > 1e-14 * np.abs(x2).max()   # refinement did something


def test_solve_matches_scipy():
    A = np.random.default_rng(8).standard_normal((70, 70))
    B = np.random.default_rng(9).standard_normal((70, 3))
    f = lu.lu_prrp(A, 16, 2.0)
    assert np.allclose(solve.solve(f.LU, f.perm, B), sla.solve(A, B), rtol=1e-10, atol=1e-10)


def test_upper_bound_table_bases():
    with open(os.path.join(GOLDEN, "upper_bound.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    for b, base in rows:
        # printed to three decimals (b = 64 truncated rather than rounded)
        assert abs(metrics.growth_base(int(b), 2.0) - float(base)) < 1.1e-3


def test_bounds_closed_forms():
    assert metrics.log10_bound_lu_prrp(256, 16, 2.0) == pytest.approx(16 * math.log10(33))
    assert metrics.log10_bound_gepp(256) == pytest.approx(255 * math.log10(2))
    # Section 3.2: b = 64, tau = 2, P = 128 (H = 7): the per-column base is
    # 129^(8/64) ~ 1.836 with the stated exponent (H+1); the example in the text
    # quotes (1.7)^n, which is 129^(7/64) (exponent H).
    n, b = 64 * 100, 64
    base = 10 ** (metrics.log10_bound_calu_prrp(n, b, 2.0, 7) / n)
    assert base == pytest.approx(129 ** (8 / 64) * 129 ** (-1 / n), rel=1e-12)
    assert 129 ** (7 / 64) == pytest.approx(1.70, abs=0.01)


def test_flop_count_leading_term():
    """Appendix C per-step counts summed over panels: leading term 2n^3/3.
    (The appendix's closed form keeps 3/2 n^2 b where the sum of its own
    per-step counts gives n^2 b / 2 + 5 n b^2 / 6; only the n^3 term is pinned.)"""
    for n, b in [(4096, 64), (8192, 128)]:
        s = metrics.flops_lu_prrp(n, n, b)
        assert s == pytest.approx(2 / 3 * n ** 3 + 0.5 * n * n * b + 5 / 6 * n * b * b, rel=1e-12)
        assert s / metrics.nominal_flops(n) == pytest.approx(1.0, abs=0.02)


def test_backward_metrics_definitions():
    A = np.array([[2.0, 1.0], [1.0, 3.0]])
    x = np.array([1.0, 1.0])
    b = np.array([3.0, 4.5])           # r = (0, 0.5)
    assert metrics.eta(A, x, b) == pytest.approx(0.5 / (4.0 * 2.0 + 7.5))
    assert metrics.comp_w(A, x, b) == pytest.approx(0.5 / (4.0 + 4.5))
    h1, h2, h3 = metrics.hpl(A, x, b)
    eps = 2.0 ** -53
    assert h1 == pytest.approx(0.5 / (eps * 4.0 * 2))
    assert h2 == pytest.approx(0.5 / (eps * 4.0 * 2.0))
    assert h3 == pytest.approx(0.5 / (eps * 4.0 * 1.0 * 2))
