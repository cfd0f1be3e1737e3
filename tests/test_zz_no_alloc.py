"""The refinement entry point that allocates nothing
(prrp_refine_async_static): its scratch is a fixed device array inside the
library, so callers that cannot allocate (graph capture, serving loops) can
call it.  Checked against prrp_refine_async on a caller workspace, bit for
bit, on two calls in a row (the second smaller, so stale contents of the
shared scratch would show), and oversize requests are refused on the host."""
import ctypes

import numpy as np
import pytest

from paper_1208_2451_amd import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _case(n, nrhs, seed, precision):
    import torch
    import paper_1208_2451_amd as prrp
    A = inputs.kappa_matrix(n, seed, 1e6)
    B = inputs.rhs(n, seed, nrhs)
    A0 = torch.from_numpy(A).cuda()
    Af = A0.clone()
    r = prrp.factor(Af, min(64, n // 4), 2.0, precision=precision)
    return A0, Af, r.perm, torch.from_numpy(B).cuda()


def test_static_scratch_matches_workspace_variant():
    import torch
    import paper_1208_2451_amd as prrp
    for n, nrhs, seed in ((640, 3, 1), (200, 1, 2)):
        announce("refine_async_static vs refine_async n=%d nrhs=%d" % (n, nrhs))
        A0, Af, perm, B = _case(n, nrhs, seed, "fp32")
        X1, it1, rel1, st1 = prrp.refine_async(A0, Af, perm, B, tol=1e-14, max_iter=30)
        X2, it2, rel2, st2 = prrp.refine_async_static(A0, Af, perm, B, tol=1e-14, max_iter=30)
        torch.cuda.synchronize()
        assert int(it1.item()) == int(it2.item()) and int(it1.item()) > 1
        assert float(rel1.item()) == float(rel2.item())
        assert int(st1.item()) == int(st2.item())
        assert torch.equal(X1, X2)


def test_static_scratch_refuses_oversize():
    import paper_1208_2451_amd as prrp  # noqa: F401
    from paper_1208_2451_amd import _lib
    L = _lib.lib()
    cap = L.prrp_static_scratch_bytes()
    need = ctypes.c_size_t(0)
    n = 8192
    nrhs = 1
    while True:
        assert L.prrp_solve_workspace_size(n, nrhs, ctypes.byref(need)) == 0
        if need.value > cap:
            break
        nrhs *= 2
    announce("static scratch refuses n=%d nrhs=%d (host only)" % (n, nrhs))
    # the pointers are never dereferenced: the size check comes first
    rc = L.prrp_refine_async_static(8, 8, n, n, 8, 8, 8, nrhs, nrhs, 1e-14, 5, None, None, None,
                                    None)
    assert rc == -8
