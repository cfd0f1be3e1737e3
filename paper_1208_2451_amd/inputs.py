"""Seeded synthetic inputs shaped like the paper's test matrices.

This module only draws and lays out numbers; it performs no step of the
factorization.  Both the GPU path (tests, bench) and the CPU oracle read their
inputs from here so that they see identical bytes.

Families (the paper's experiments section and the CALU_PRRP experiments):
  * ``randn``    -- i.i.d. N(0,1) entries, the paper's ``randn(n,n)`` matrices,
                    with an N(0,1) right-hand side drawn after the matrix from
                    the same generator.
  * ``wilkinson``-- the GEPP worst case in the layout given for the Wilkinson
                    matrix with T = I and theta = 1: 1 on the diagonal, -1
                    strictly below it, 1 in the last column.
  * ``foster``   -- the Volterra quadrature matrix of Foster (parameters c, k, h).
  * ``wright``   -- the multiple-shooting matrix of Wright with M = [[-1/6, 1],
                    [1, -1/6]] and step h (exact matrix exponential).
  * ``kappa``    -- U diag(s) V^T with Haar orthogonal U, V (QR of a Gaussian
                    matrix with the sign of diag(R) folded into Q) and s
                    log-spaced from 1 to 1/kappa.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "randn_system", "wilkinson", "foster", "wright", "kappa_matrix",
    "rhs", "serving_requests",
]


def randn_system(n: int, seed: int, nrhs: int = 1):
    """Return (A, B): A is n x n N(0,1), B is n x nrhs N(0,1), both C-order float64.

    The matrix is drawn first, then the right-hand sides, from one PCG64 stream.
    """
    g = np.random.default_rng(seed)
    A = g.standard_normal((n, n))
    B = g.standard_normal((n, nrhs))
    return np.ascontiguousarray(A), np.ascontiguousarray(B)


def rhs(n: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """N(0,1) right-hand sides from their own stream (seed offset by 2**31)."""
    g = np.random.default_rng(seed + (1 << 31))
    return np.ascontiguousarray(g.standard_normal((n, nrhs)))


def wilkinson(n: int) -> np.ndarray:
    """GEPP growth 2^(n-1) matrix: diag 1, strictly lower -1, last column 1."""
    A = np.tril(-np.ones((n, n)), -1) + np.eye(n)
    A[:, n - 1] = 1.0
    return A


def foster(n: int, c: float = 1.0, k: float = 2.0 / 3.0, h: float = 1.0) -> np.ndarray:
    """Foster's quadrature matrix: first column -kh/2 below the (1,1) entry 1,
    -kh strictly below the diagonal elsewhere, 1 - kh/2 on the diagonal (rows
    2..n), -1/c in the last column, and 1 - 1/c - kh/2 in the corner."""
    kh = k * h
    A = np.tril(np.full((n, n), -kh), -1)
    A[1:, 0] = -kh / 2.0
    A[np.arange(1, n), np.arange(1, n)] = 1.0 - kh / 2.0
    A[0, 0] = 1.0
    A[:, n - 1] = -1.0 / c
    A[n - 1, n - 1] = 1.0 - 1.0 / c - kh / 2.0
    return A


def _expm2(M: np.ndarray) -> np.ndarray:
    """exp of a symmetric 2x2 matrix through its eigen-decomposition."""
    w, V = np.linalg.eigh(M)
    return (V * np.exp(w)) @ V.T


def wright(n: int, h: float = 0.3) -> np.ndarray:
    """Wright's block bidiagonal matrix with 2x2 blocks: I on the diagonal,
    -exp(M h) on the first block subdiagonal, I in the top-right block.  n must
    be even."""
    if n % 2:
        raise ValueError("wright(n) needs an even n")
    M = np.array([[-1.0 / 6.0, 1.0], [1.0, -1.0 / 6.0]])
    E = _expm2(M * h)
    nb = n // 2
    A = np.eye(n)
    for i in range(1, nb):
        A[2 * i:2 * i + 2, 2 * (i - 1):2 * i] = -E
    A[0:2, n - 2:n] += np.eye(2)
    return A


def generalized_wilkinson(n: int, seed: int, r: int = 1) -> np.ndarray:
    """Generalized Wilkinson matrix (Section 2.3; generator of Appendix F):
    the identity, plus a strictly lower triangular part that is the
    transpose of a negative, rank-r semi-separable upper triangle with random
    entries, plus ones in the last column.  The upper triangle is -u v^T
    (u, v uniform on [0, 1), n x r, from this seed's stream); each row of it is
    scaled so that its largest entry right of the diagonal has magnitude
    n / (n + 1).  The paper's runs drew u, v in Matlab with an unstated seed,
    so only the order of magnitude of its growth figures carries over."""
    g = np.random.default_rng(seed)
    u = g.random((n, r))
    v = g.random((n, r))
    T = -np.triu(u @ v.T, 1)
    for i in range(n - 1):
        m = np.abs(T[i, i + 1:]).max()
        if m > 0.0:
            T[i, i + 1:] /= m * (1.0 + 1.0 / n)
    A = T.T + np.eye(n)
    A[: n - 1, n - 1] = 1.0
    return A


def kappa_matrix(n: int, seed: int, kappa: float = 1e6, device: str = "cpu"):
    """U diag(s) V^T with Haar U, V and s_i = kappa^(-i/(n-1)).

    ``device='cpu'`` returns a numpy array; any torch device string returns a
    torch float64 tensor built on that device (the Gaussian draws always come
    from a seeded numpy stream, so the spectrum and seeds are shared).
    """
    g = np.random.default_rng(seed)
    Zu = g.standard_normal((n, n))
    Zv = g.standard_normal((n, n))
    s = kappa ** (-np.arange(n, dtype=np.float64) / max(n - 1, 1))
    if device == "cpu":
        Qu, Ru = np.linalg.qr(Zu)
        Qu *= np.sign(np.diag(Ru))
        Qv, Rv = np.linalg.qr(Zv)
        Qv *= np.sign(np.diag(Rv))
        return np.ascontiguousarray((Qu * s) @ Qv.T)
    import torch
    dev = torch.device(device)
    out = []
    for Z in (Zu, Zv):
        Zt = torch.from_numpy(Z).to(dev)
        Q, R = torch.linalg.qr(Zt)
        out.append(Q * torch.sign(torch.diagonal(R)))
        del Zt, R
    Qu, Qv = out
    st = torch.from_numpy(s).to(dev)
    return ((Qu * st) @ Qv.T).contiguous()


def serving_requests(count: int, seed: int, rate: float, nmin: int = 64,
                     nmax: int = 2048, step: int = 32, max_rhs: int = 8):
    """Poisson stream of solve requests.

    Returns a list of dicts {t_arrival, n, b, nrhs, seed}: exponential
    inter-arrival times at ``rate`` requests/s, n uniform over
    {nmin, nmin+step, ..., nmax}, b = min(32, n/4), nrhs uniform in 1..max_rhs,
    and a per-request matrix seed.  Arrival and matrix seeds come from separate
    streams.
    """
    ga = np.random.default_rng(seed)
    gs = np.random.default_rng(seed + 7919)
    sizes = np.arange(nmin, nmax + 1, step)
    t = np.cumsum(ga.exponential(1.0 / rate, size=count))
    ns = gs.choice(sizes, size=count)
    nr = gs.integers(1, max_rhs + 1, size=count)
    seeds = gs.integers(0, 2**31 - 1, size=count)
    return [dict(t_arrival=float(t[i]), n=int(ns[i]), b=int(min(32, ns[i] // 4)),
                 nrhs=int(nr[i]), seed=int(seeds[i])) for i in range(count)]
