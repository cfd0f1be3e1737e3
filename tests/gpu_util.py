"""Helpers shared by the GPU tests (host-side checks only)."""
import sys

import numpy as np

TAU_TOL = 1.0 + 2.0 ** -32


def announce(*parts):
    """Name the case about to run on the GPU (flushed, so a fault still shows it)."""
    print("[gpu-case]", *parts, file=sys.stderr, flush=True)


def backward_error(A, LU, perm):
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return float(np.linalg.norm(A[perm] - L @ U) / np.linalg.norm(A))


def gpu_factor(A_np, b, tau=2.0, precision="fp64", method="lu", tree="binary", tile_rows=512):
    import torch
    import paper_1208_2451_amd as prrp
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    if method == "lu":
        r = prrp.factor(A, b, tau, precision=precision)
    else:
        r = prrp.calu_factor(A, b, tau, tree=tree, tile_rows=tile_rows, precision=precision)
    torch.cuda.synchronize()
    return A.cpu().numpy(), r.perm.cpu().numpy(), r.stats(), A, r
