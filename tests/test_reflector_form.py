"""The Householder reflector form used by the strong-RRQR kernel.

Each QR step of Algorithm "Strong RRQR" (Appendix A) reflects the pivot
column's trailing part x (head x_0, norm nrm) onto alpha e_1 with
H = I - beta v v^T, v = x - alpha e_1, alpha = -sign(x_0) nrm.  The kernel
forms beta = 1 / (nrm (nrm + |x_0|)) from the trailing norm it already has for
the pivot key, instead of 2 / (v^T v).  Both are the same number; this checks
the identity and the reflection numerically, including heads of either sign,
a zero head and tiny and huge scales.
"""
import numpy as np
import pytest


def _forms(x):
    nrm = float(np.sqrt(np.dot(x, x)))
    head = float(x[0])
    alpha = 0.0 if nrm == 0.0 else -np.copysign(nrm, head)
    v = x.copy()
    v[0] = head - alpha
    vtv = float(np.dot(v, v))
    beta_vtv = 2.0 / vtv if vtv > 0 else 0.0
    beta_kernel = 0.0 if nrm == 0.0 else 1.0 / (nrm * (nrm + abs(head)))
    return alpha, v, beta_vtv, beta_kernel


@pytest.mark.parametrize("seed", range(20))
@pytest.mark.parametrize("scale", [1e-150, 1.0, 1e150])
def test_beta_forms_agree_and_reflect(seed, scale):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 129))
    x = rng.standard_normal(m) * scale
    if seed % 4 == 1:
        x[0] = 0.0
    if seed % 4 == 2:
        x[0] = -abs(x[0])
    alpha, v, b1, b2 = _forms(x)
    assert b2 == pytest.approx(b1, rel=4e-16 * m)
    hx = x - b2 * np.dot(v, x) * v
    e = np.zeros(m)
    e[0] = alpha
    assert np.abs(hx - e).max() <= 1e-14 * max(abs(alpha), np.abs(x).max())


def test_zero_column_gives_identity():
    alpha, v, b1, b2 = _forms(np.zeros(7))
    assert alpha == 0.0 and b1 == 0.0 and b2 == 0.0
