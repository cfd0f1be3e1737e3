"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, answers workspace queries, and rejects bad arguments before
touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1208_2451_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "prrp.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(prrp_\w+|calu_prrp_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libprrp.so not built")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(L, name), name
    assert set(names) <= set(_lib._SIGS), "binding misses a declared entry point"


def test_version_and_status(L):
    assert L.prrp_version().decode().startswith("prrp-gfx950")
    assert L.prrp_status_string(0).decode() == "success"


def test_workspace_queries(L):
    w1 = _lib.workspace_size(256, 16, 0, 0)
    w2 = _lib.workspace_size(4096, 64, 0, 0)
    assert 0 < w1 < w2
    assert _lib.workspace_size(16384, 128, 1, 512) > 0
    assert _lib.solve_workspace_size(4096, 16) >= 2 * 4096 * 16 * 8
    with pytest.raises(_lib.PrrpError):
        _lib.workspace_size(100, 129, 0, 0)         # b above the widest panel
    with pytest.raises(_lib.PrrpError):
        _lib.workspace_size(100, 16, 1, 16)         # tile_rows < b + 1


@pytest.mark.parametrize("args,code", [
    ((None, 8, 8, 2, 2.0), -1),        # null A
    ((1, 0, 8, 2, 2.0), -2),           # n < 1
    ((1, 8, 7, 2, 2.0), -3),           # lda < n
    ((1, 8, 8, 0, 2.0), -4),           # b < 1
    ((1, 8, 8, 9, 2.0), -4),           # b > n
    ((1, 8, 8, 2, 1.0), -5),           # tau <= 1
    ((1, 8, 8, 2, float("nan")), -5),  # tau NaN
])
def test_factor_argument_errors(L, args, code):
    A, n, lda, b, tau = args
    rc = L.prrp_factor(A, n, lda, b, tau, 1, 1, 1, 1 << 40, None)
    assert rc == code


def test_factor_null_perm_stats_ws(L):
    assert L.prrp_factor(1, 8, 8, 2, 2.0, None, 1, 1, 1 << 40, None) == -6
    assert L.prrp_factor(1, 8, 8, 2, 2.0, 1, None, 1, 1 << 40, None) == -7
    assert L.prrp_factor(1, 8, 8, 2, 2.0, 1, 1, None, 1 << 40, None) == -8
    assert L.prrp_factor(1, 8, 8, 2, 2.0, 1, 1, 1, 16, None) == -9    # workspace too small


def test_calu_argument_errors(L):
    f = L.calu_prrp_factor
    assert f(1, 64, 64, 8, 2.0, 2, 32, 1, 1, 1, 1 << 40, None, 0) == -6    # tree kind
    assert f(1, 64, 64, 8, 2.0, 0, 8, 1, 1, 1, 1 << 40, None, 0) == -7     # tile_rows <= b
    assert f(1, 64, 64, 8, 2.0, 0, 32, 1, 1, 1, 1 << 40, None, 5) == -13   # precision


def test_solve_and_gemm_argument_errors(L):
    assert L.prrp_solve(None, 8, 8, 1, 1, 1, 1, 1, 1 << 30, None) == -1
    assert L.prrp_solve(1, 8, 8, 1, 1, 0, 1, 1, 1 << 30, None) == -6
    assert L.prrp_solve(1, 8, 8, 1, 1, 2, 1, 1, 1 << 30, None) == -7
    assert L.prrp_residual(1, 8, 4, 1, 1, 1, 1, 1, None) == -3
    assert L.prrp_gemm(4, 4, 4, 1.0, 1, 3, 1, 4, 0.0, 1, 4, 0, None) == -6
    assert L.prrp_gemm(4, 4, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 4, 7, None) == -12


def test_refine_argument_errors(L):
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0)
    st = ctypes.c_int(0)
    f = L.prrp_refine
    assert f(1, 1, 8, 8, 1, 1, 1, 1, 1, -1.0, 5, ctypes.byref(it), ctypes.byref(rel),
             ctypes.byref(st), 1, 1 << 30, None) == -10
    assert f(1, 1, 8, 8, 1, 1, 1, 1, 1, 1e-14, 5, None, None, None, None, 1 << 30, None) == -15
    assert f(1, 1, 8, 8, 1, 1, 1, 1, 1, 1e-14, 5, None, None, None, 1, 16, None) == -16


def test_refine_async_argument_errors(L):
    f = L.prrp_refine_async
    assert f(1, 1, 8, 8, 1, 1, 1, 1, 1, -1.0, 5, None, None, None, 1, 1 << 30, None) == -10
    assert f(1, 1, 8, 8, 1, 1, 1, 1, 1, 1e-14, 5000, None, None, None, 1, 1 << 30, None) == -11
    assert f(1, 1, 8, 8, 1, 1, 1, 1, 1, 1e-14, 5, None, None, None, None, 1 << 30, None) == -15
    assert f(1, 1, 8, 8, 1, 1, 1, 1, 1, 1e-14, 5, None, None, None, 1, 16, None) == -16


def test_refine_status_codes_match_the_binding(L):
    # the header's PRRP_IR_* values, as the binding and the server read them
    with open(os.path.join(ROOT, "include", "prrp.h")) as fh:
        text = fh.read()
    m = re.search(r"enum\s*\{\s*PRRP_IR_CONVERGED\s*=\s*(\d+),\s*PRRP_IR_STAGNATED\s*=\s*(\d+),"
                  r"\s*PRRP_IR_CAP\s*=\s*(\d+)\s*\}", text)
    assert m, "PRRP_IR_* enum not found"
    assert tuple(int(v) for v in m.groups()) == (_lib.PRRP_IR_CONVERGED, _lib.PRRP_IR_STAGNATED,
                                                  _lib.PRRP_IR_CAP)
    assert sorted(_lib.IR_STATUS) == [0, 1, 2]


def test_no_allocating_batched_factor(L):
    # a batch runs through a plan on the caller's workspace; the one-shot
    # entry point that allocated and synchronised is gone
    assert not hasattr(L, "prrp_factor_batched")


def _panel_cus(L, method, n, b, tree=0, tile_rows=0, bpc=2):
    out = ctypes.c_int64(-1)
    rc = L.prrp_panel_cus(method, n, b, tree, tile_rows, bpc, ctypes.byref(out))
    return rc, out.value


def test_panel_residency_requirement(L):
    # LU_PRRP: one panel of n rows over workgroups of at most 128 rows, at
    # least ceil(n / 64) of them up to 64; all resident at once
    assert _panel_cus(L, 0, 8192, 128) == (0, 32)            # 64 workgroups, 2 per CU
    assert _panel_cus(L, 0, 8192, 128, bpc=1) == (0, 64)
    assert _panel_cus(L, 0, 16384, 128) == (0, 64)           # 128 workgroups of 128 rows
    assert _panel_cus(L, 0, 65536, 128) == (0, 256)          # exactly the MI355X's CUs
    rc, cus = _panel_cus(L, 0, 70000, 128)
    assert rc == 0 and cus > 256                            # rejected by the factor call
    # CALU_PRRP: the tiles are small, but the root factors the whole panel
    assert _panel_cus(L, 1, 16384, 128, 0, 512)[0] == 0
    assert _panel_cus(L, 1, 16384, 128, 0, 512)[1] <= 64
    # argument errors
    assert _panel_cus(L, 2, 64, 8)[0] == -1
    assert _panel_cus(L, 0, 0, 8)[0] == -2
    assert _panel_cus(L, 0, 64, 129)[0] == -3
    assert _panel_cus(L, 1, 64, 8, 5, 32)[0] == -4
    assert _panel_cus(L, 1, 64, 8, 0, 8)[0] == -5
    assert _panel_cus(L, 0, 64, 8, bpc=-1)[0] == -6
    assert L.prrp_panel_cus(0, 64, 8, 0, 0, 2, None) == -7


def test_batch_plan_argument_errors(L):
    one_p = (ctypes.c_void_p * 1)(1)
    n8 = (ctypes.c_int64 * 1)(8)
    b2 = (ctypes.c_int * 1)(2)
    h = ctypes.c_void_p(0)
    args = lambda **kw: dict(dict(count=1, A=one_p, n=n8, lda=n8, b=b2, perm=one_p, stats=1,  # noqa: E731
                                  tau=2.0, schur=0, rpw=64), **kw)

    def call(**kw):
        a = args(**kw)
        return L.prrp_batch_plan_create(a["count"], a["A"], a["n"], a["lda"], a["b"], a["perm"],
                                        a["stats"], a["tau"], a["schur"], a["rpw"], None, None,
                                        None, None, 0.0, 0, a.get("ws", None), a.get("wsb", 0),
                                        None, ctypes.byref(h))
    assert call(count=0) == -1
    assert call(tau=1.0) == -8
    assert call(schur=3) == -9
    assert call(rpw=96) == -10
    assert call(b=(ctypes.c_int * 1)(9)) == -5       # b > n
    assert call(lda=(ctypes.c_int64 * 1)(4)) == -4   # lda < n
    assert call() == -17                             # no workspace
    assert call(ws=1, wsb=16) == -18                 # workspace too small
    need = ctypes.c_size_t(0)
    assert L.prrp_batch_plan_workspace_size(1, n8, b2, None, 64, ctypes.byref(need)) == 0
    assert need.value > 8 * 8 * 2
    need2 = ctypes.c_size_t(0)
    nr = (ctypes.c_int64 * 1)(3)
    assert L.prrp_batch_plan_workspace_size(1, n8, b2, nr, 64, ctypes.byref(need2)) == 0
    assert need2.value > need.value                 # refinement needs solve workspace
    assert L.prrp_batch_plan_workspace_size(1, n8, b2, None, 96, ctypes.byref(need)) == -5
    assert L.prrp_batch_plan_run(None, None, 0) == -1
    assert L.prrp_batch_plan_destroy(None) == 0


def test_block_factor_sizes_and_argument_errors(L):
    ws = ctypes.c_size_t(0)
    ne = ctypes.c_int64(0)
    assert L.prrp_block_sizes(1024, 16, 0, 128, ctypes.byref(ws), ctypes.byref(ne)) == 0
    P, MN = 1024 // 16, 2 * 8 - 1                  # 8 tiles of 128 rows: 15 binary-tree nodes
    assert ne.value == 2 + P + P * MN * 16 + P * 1024
    assert ws.value > _lib.workspace_size(1024, 16, 1, 128)
    assert L.prrp_block_sizes(1024, 16, 1, 128, None, ctypes.byref(ne)) == 0
    assert ne.value == 2 + P + P * 8 * 16 + P * 1024   # flat tree: one node per tile
    assert L.prrp_block_sizes(1024, 16, 2, 128, None, None) == -3    # tree kind
    assert L.prrp_block_sizes(1024, 16, 0, 15, None, None) == -4     # tile_rows < b
    assert L.prrp_block_sizes(1024, 16, 1, 16, None, None) == 0      # b-row tiles (pairwise)
    f = L.prrp_block_factor
    big = 1 << 40
    assert f(None, 64, 64, 8, 2.0, 0, 32, 1, 1, big, 1, 1, big, None) == -1
    assert f(1, 64, 64, 8, 1.0, 0, 32, 1, 1, big, 1, 1, big, None) == -5
    assert f(1, 64, 64, 8, 2.0, 3, 32, 1, 1, big, 1, 1, big, None) == -6
    assert f(1, 64, 64, 8, 2.0, 0, 7, 1, 1, big, 1, 1, big, None) == -7
    assert f(1, 64, 64, 8, 2.0, 0, 32, 1, None, big, 1, 1, big, None) == -9
    assert f(1, 64, 64, 8, 2.0, 0, 32, 1, 1, 10, 1, 1, big, None) == -10   # records too short
    assert f(1, 64, 64, 8, 2.0, 0, 32, 1, 1, big, 1, 1, 16, None) == -13   # workspace too small
    s = L.prrp_block_solve
    assert s(1, 64, 64, 8, 1, None, 1, 1, 1, 1, 1, 1, big, None) == -6
    assert s(1, 64, 64, 8, 1, 1, 1, 1, 1, 1, 0, 1, big, None) == -11
    assert s(1, 64, 64, 8, 1, 1, 1, 1, 1, 1, 1, 1, 16, None) == -13
