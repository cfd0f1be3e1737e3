"""Accuracy metrics, growth bounds and flop counts -- oracle (test infrastructure).

  * backward error ||A[perm] - L U||_F / ||A||_F (the Frobenius-norm relative
    error of the paper's summary figure);
  * normwise backward error eta (equation "eta", 1-norm) and componentwise
    backward error w (equation "comp");
  * HPL1, HPL2, HPL3 with eps = 2^-53 (the HPL accuracy tests quoted in the
    experiments of Section 2);
  * log10 growth bounds: LU_PRRP (1 + tau b)^(n/b) (Section 2.2), CALU_PRRP
    (1 + tau b)^((n/b)(H+1) - 1) (Table "caluprrp_bound"), GEPP 2^(n-1);
  * the LU_PRRP flop count of Appendix C.

Pinned by tests/test_oracle_metrics.py: the per-column bases of Table
"upper_bound" (tests/golden/upper_bound.txt), the closed-form flop totals of
Appendix C, and metric values recomputed from definitions on small cases.
"""
from __future__ import annotations

import math

import numpy as np

EPS = 2.0 ** -53


def backward_error(A, LU, perm) -> float:
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return float(np.linalg.norm(A[perm] - L @ U) / np.linalg.norm(A))


def eta(A, x, b) -> float:
    r = b - A @ x
    return float(np.abs(r).sum() / (np.abs(A).sum(axis=0).max() * np.abs(x).sum() + np.abs(b).sum()))


def comp_w(A, x, b) -> float:
    r = b - A @ x
    den = np.abs(A) @ np.abs(x) + np.abs(b)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(den > 0, np.abs(r) / den, 0.0)
    return float(q.max())


def hpl(A, x, b):
    n = A.shape[0]
    r = np.abs(A @ x - b).max()
    a1 = np.abs(A).sum(axis=0).max()
    ainf = np.abs(A).sum(axis=1).max()
    return (float(r / (EPS * a1 * n)), float(r / (EPS * a1 * np.abs(x).sum())),
            float(r / (EPS * ainf * np.abs(x).max() * n)))


def log10_bound_lu_prrp(n: int, b: int, tau: float) -> float:
    return (n / b) * math.log10(1.0 + tau * b)


def log10_bound_calu_prrp(n: int, b: int, tau: float, H: int) -> float:
    return ((n / b) * (H + 1) - 1.0) * math.log10(1.0 + tau * b)


def log10_bound_gepp(n: int) -> float:
    return (n - 1) * math.log10(2.0)


def growth_base(b: int, tau: float) -> float:
    """Per-column base c with (1 + tau b)^(n/b) = c^n."""
    return (1.0 + tau * b) ** (1.0 / b)


def flops_step(m: int, n: int, b: int, k: int) -> float:
    """Appendix C: strong RRQR + update + diagonal GEPP of panel k (1-based)."""
    srrqr = 2.0 * (m - (k - 1) * b) * b * b - 2.0 / 3.0 * b ** 3
    update = 2.0 * b * (m - k * b) * (n - k * b)
    gepp = 2.0 / 3.0 * b ** 3 + (n - k * b) * b * b
    return srrqr + update + gepp


def flops_lu_prrp(m: int, n: int, b: int) -> float:
    return sum(flops_step(m, n, b, k) for k in range(1, n // b + 1))


def flops_lu_prrp_closed(n: int, b: int) -> float:
    """Appendix C closed form for a square matrix."""
    return 2.0 / 3.0 * n ** 3 + 1.5 * n * n * b + 2.0 * n * b * b


def nominal_flops(n: int) -> float:
    """The 2n^3/3 convention used for TFLOP/s."""
    return 2.0 * n ** 3 / 3.0
