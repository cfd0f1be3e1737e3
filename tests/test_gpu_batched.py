"""Batched LU_PRRP of uneven-size systems, graph replay and device-side refinement.

Bar: every system of a batch gets exactly the factors, permutation and
statistics of the same system factored alone (same kernels, same operation
order: bitwise equality), the alone results match the oracle's permutation
with backward error <= 1e-15 n, and graph replays reproduce the eager run
bit for bit.  The device-side refinement loop returns the host-driven loop's
solution bit for bit with the same iteration count.
"""
import numpy as np
import pytest

from oracle import lu as olu
from paper_1208_2451_amd import inputs
from tests.gpu_util import announce, backward_error

pytestmark = pytest.mark.gpu

SIZES = [64, 96, 160, 257, 300, 512]


def _panel(n):
    return min(32, max(1, n // 4))


def _systems(sizes, seed0):
    return [inputs.randn_system(n, seed0 + i)[0] for i, n in enumerate(sizes)]


def _alone(A_np, b, precision):
    import torch
    import paper_1208_2451_amd as prrp
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    r = prrp.factor(A, b, 2.0, precision=precision)
    torch.cuda.synchronize()
    return A.cpu().numpy(), r.perm.cpu().numpy(), r.stats()


def _batch(mats_np, precision="fp64", rows_per_wg=64, graph=False, runs=1):
    import torch
    import paper_1208_2451_amd as prrp
    orig = [torch.from_numpy(np.ascontiguousarray(M)).cuda() for M in mats_np]
    work = [o.clone() for o in orig]
    plan = prrp.BatchPlan(work, [_panel(M.shape[0]) for M in mats_np], precision=precision,
                          rows_per_wg=rows_per_wg)
    outs = []
    for _ in range(runs):
        for w, o in zip(work, orig):
            w.copy_(o)
        plan.run(graph=graph)
        torch.cuda.synchronize()
        outs.append(([w.cpu().numpy() for w in work], [p.cpu().numpy() for p in plan.perms],
                     [plan.stats(i) for i in range(len(work))]))
    plan.close()
    return outs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_alone(precision):
    mats = _systems(SIZES, 500)
    announce("batched", precision, SIZES)
    (LUs, perms, stats), = _batch(mats, precision)
    for M, LU, p, st in zip(mats, LUs, perms, stats):
        n = M.shape[0]
        LUa, pa, sta = _alone(M, _panel(n), precision)
        assert np.array_equal(p, pa), n
        assert np.array_equal(LU, LUa), n
        for k in ("max_abs_A", "max_abs_W", "max_abs_U", "max_block_L", "swaps", "info"):
            assert st[k] == sta[k], (n, k)


@pytest.mark.parametrize("sizes", [[520], [384, 1000], [700, 1000, 384]])
def test_batch_first_problem_multi_workgroup(sizes):
    # the first problem's slot sets sit at the start of the plan's memory;
    # multi-workgroup panels reuse them every other step
    mats = _systems(sizes, 1100)
    announce("batched first problem multi-wg", sizes)
    (LUs, perms, stats), = _batch(mats)
    for M, LU, p, st in zip(mats, LUs, perms, stats):
        LUa, pa, sta = _alone(M, _panel(M.shape[0]), "fp64")
        assert st["info"] == 0
        assert np.array_equal(p, pa)
        assert np.array_equal(LU, LUa)


def test_batch_fp64_matches_oracle():
    mats = _systems(SIZES, 600)
    announce("batched vs oracle", SIZES)
    (LUs, perms, stats), = _batch(mats)
    for M, LU, p, st in zip(mats, LUs, perms, stats):
        n = M.shape[0]
        f = olu.lu_prrp(M, _panel(n), 2.0)
        assert np.array_equal(p, f.perm), n
        assert backward_error(M, LU, p) <= 1e-15 * n
        assert st["info"] == 0


def test_batch_rows_per_workgroup_128_same_result():
    # fewer, fuller workgroups per strong-RRQR step change no value
    mats = _systems([700, 1000, 384], 700)
    announce("batched rows_per_wg 64 vs 128")
    (a_lu, a_p, _), = _batch(mats, rows_per_wg=64)
    (b_lu, b_p, _), = _batch(mats, rows_per_wg=128)
    for x, y, p, q in zip(a_lu, b_lu, a_p, b_p):
        assert np.array_equal(p, q)
        assert np.array_equal(x, y)


def test_batch_graph_replays_match_eager():
    mats = _systems([128, 200, 333], 800)
    announce("batched graph replays")
    (e_lu, e_p, e_st), = _batch(mats, graph=False)
    outs = _batch(mats, graph=True, runs=3)
    for lu, p, st in outs:
        for x, y, pp, qq in zip(lu, e_lu, p, e_p):
            assert np.array_equal(pp, qq)
            assert np.array_equal(x, y)


def test_batch_bad_system_does_not_disturb_others():
    mats = _systems([96, 128, 160], 900)
    mats[1] = mats[1].copy()
    mats[1][5, 7] = np.nan
    announce("batched with a NaN system")
    (LUs, perms, stats), = _batch(mats)
    assert stats[1]["info"] == -1
    for i in (0, 2):
        LUa, pa, sta = _alone(mats[i], _panel(mats[i].shape[0]), "fp64")
        assert np.array_equal(perms[i], pa)
        assert np.array_equal(LUs[i], LUa)
        assert stats[i]["info"] == 0


def test_refine_async_equals_refine():
    import torch
    import paper_1208_2451_amd as prrp
    n = 384
    A_np = inputs.kappa_matrix(n, 3, 1e6)
    B_np = inputs.rhs(n, 3, 2)
    announce("refine_async vs refine n=%d" % n)
    A0 = torch.from_numpy(A_np).cuda()
    A = A0.clone()
    r = prrp.factor(A, 32, 2.0, precision="fp32")
    B = torch.from_numpy(B_np).cuda()
    X1, it1, rel1, st1 = prrp.refine(A0, A, r.perm, B, tol=1e-14, max_iter=25)
    X2, it2, rel2, st2 = prrp.refine_async(A0, A, r.perm, B, tol=1e-14, max_iter=25)
    torch.cuda.synchronize()
    assert int(it2.item()) == it1
    assert float(rel2.item()) == rel1
    assert torch.equal(X1, X2)


def test_batch_with_refinement():
    import torch
    import paper_1208_2451_amd as prrp
    sizes = [64, 160, 320]
    mats = [inputs.kappa_matrix(n, 10 + n, 1e4) for n in sizes]
    rhs = [inputs.rhs(n, 20 + n, k) for n, k in zip(sizes, (1, 3, 2))]
    announce("batched factor + refinement", sizes)
    orig = [torch.from_numpy(M).cuda() for M in mats]
    work = [o.clone() for o in orig]
    B = [torch.from_numpy(r).cuda() for r in rhs]
    plan = prrp.BatchPlan(work, [_panel(n) for n in sizes], precision="fp32", originals=orig,
                          rhs=B, tol=1e-14, max_iter=20)
    plan.run(graph=True)
    torch.cuda.synchronize()
    its, rels, sts = plan.refine_results()
    for i, n in enumerate(sizes):
        Aw = orig[i].clone()
        r = prrp.factor(Aw, _panel(n), 2.0, precision="fp32")
        X, it, rel, status = prrp.refine(orig[i], Aw, r.perm, B[i], tol=1e-14, max_iter=20)
        torch.cuda.synchronize()
        assert its[i] == it
        assert torch.equal(plan.solutions[i].view(X.shape), X)
        x_ref = np.linalg.solve(mats[i], rhs[i])
        err = np.abs(X.cpu().numpy() - x_ref).max() / np.abs(x_ref).max()
        assert err <= 1e-12
    plan.close()
