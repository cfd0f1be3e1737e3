"""Continuous-batching solve server and autotuner.

Bar: every request served in the mix returns exactly (bit for bit) the
solution the same request gets alone, and that solution is within 1e-12
(relative, max norm) of the converged reference solution (LAPACK factors plus
the oracle's doubled-precision refinement).  A memory budget that admits one
request at a time still completes the stream with the same results.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import solve as osolve
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _x_ref(A, B):
    lu_, piv = sla.lu_factor(A)
    perm = np.arange(A.shape[0])
    for j, p in enumerate(piv):
        perm[[j, p]] = perm[[p, j]]
    x, _, _ = osolve.refine(A, lu_, perm, B, tol=1e-16, max_iter=12)
    return x


def _stream(count, seed, rate, nmax):
    from paper_1208_2451_amd import serving
    reqs = serving.make_requests(count, seed, rate, nmin=64, nmax=nmax)
    return serving.materialize(reqs, "cuda")


def test_mix_equals_alone_and_accuracy():
    import torch
    from paper_1208_2451_amd import serving
    reqs = _stream(20, 11, 2000.0, 512)
    announce("serving mix", [r.n for r in reqs])
    srv = serving.Server(max_batch=6, slots=2, precision="fp32", max_iter=10)
    summary = srv.serve(reqs, realtime=True)
    torch.cuda.synchronize()
    assert summary["requests"] == 20
    for r in reqs:
        x_alone, it = serving.solve_alone(r, precision="fp32", max_iter=10)
        assert r.iters == it
        assert torch.equal(r.X, x_alone), r.rid
        A = r.A.cpu().numpy()
        B = r.B.cpu().numpy()
        xr = _x_ref(A, B)
        err = np.abs(r.X.cpu().numpy() - xr).max() / np.abs(xr).max()
        assert err <= 1e-12, (r.rid, r.n, err)


def test_memory_budget_admits_one_at_a_time():
    import torch
    from paper_1208_2451_amd import serving
    reqs = _stream(6, 12, 1e6, 256)
    announce("serving tiny budget")
    srv = serving.Server(max_batch=8, slots=2, mem_budget=1, precision="fp32")
    summary = srv.serve(reqs, realtime=False)
    torch.cuda.synchronize()
    assert summary["requests"] == 6
    for r in reqs:
        x_alone, _ = serving.solve_alone(r, precision="fp32")
        assert torch.equal(r.X, x_alone)


def test_autotune_returns_valid_choices():
    from paper_1208_2451_amd import autotune
    announce("autotune small")
    t = autotune.tune(classes=((64, 128), (160, 256)), batch=4, batch_options=(2, 4), trials=1)
    f = autotune.rows_per_wg_fn(t)
    assert f(100) in (64, 128) and f(200) in (64, 128) and f(4000) in (64, 128)
    assert t["max_batch"] in (2, 4)
