"""LU_PRRP / CALU_PRRP on MI355X (gfx950).

Thin torch-facing wrappers over the C ABI of libprrp.so (include/prrp.h).
Matrices are CUDA (HIP) float64 tensors, row-major; factorizations run in
place on the caller's stream.
"""
from __future__ import annotations

from dataclasses import dataclass

__all__ = ["factor", "calu_factor", "block_factor", "block_solve", "solve", "residual", "refine",
           "refine_async",
           "refine_async_static", "refine_gmres",
           "gemm",
           "FactorResult", "read_stats", "BatchPlan"]


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return torch.cuda.current_stream().cuda_stream


def _check_matrix(A, name="A"):
    torch = _torch()
    if not isinstance(A, torch.Tensor) or A.device.type != "cuda":
        raise ValueError("%s must be a CUDA tensor" % name)
    if A.dtype != torch.float64:
        raise ValueError("%s must be float64" % name)
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("%s must be 2-D with unit column stride (row-major)" % name)


@dataclass
class FactorResult:
    perm: object        # torch int64 [n] on the device
    stats_raw: object   # torch uint8 [sizeof prrp_stats] on the device
    workspace: object

    def stats(self) -> dict:
        return read_stats(self.stats_raw)


def read_stats(raw) -> dict:
    from ._lib import Stats
    host = raw.cpu().numpy().tobytes()
    s = Stats.from_buffer_copy(host)
    return dict(max_abs_A=s.max_abs_A, max_abs_W=s.max_abs_W, max_abs_U=s.max_abs_U,
                max_block_L=s.max_block_L, swaps=int(s.swaps), info=int(s.info),
                tree_height=int(s.tree_height),
                g_W=(s.max_abs_W / s.max_abs_A) if s.max_abs_A > 0 else float("nan"),
                g_U=(s.max_abs_U / s.max_abs_A) if s.max_abs_A > 0 else float("nan"))


def _alloc(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def factor(A, b: int, tau: float = 2.0, precision: str = "fp64", workspace=None) -> FactorResult:
    """LU_PRRP of A in place (A = Pi L U; A[perm] = L U on exit)."""
    from . import _lib
    torch = _torch()
    _check_matrix(A)
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    ws_bytes = _lib.workspace_size(n, b, 0, 0)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc(ws_bytes, A.device)
    perm = torch.empty(n, dtype=torch.int64, device=A.device)
    stats = torch.zeros(_lib.STATS_BYTES, dtype=torch.uint8, device=A.device)
    code = _lib.lib().prrp_factor_mixed(A.data_ptr(), n, A.stride(0), b, float(tau), perm.data_ptr(),
                                        stats.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                        _stream_ptr(), _lib.PRECISIONS[precision])
    _lib.check(code, "prrp_factor_mixed")
    return FactorResult(perm, stats, workspace)


def calu_factor(A, b: int, tau: float = 2.0, tree: str = "binary", tile_rows: int = 512,
                precision: str = "fp64", workspace=None) -> FactorResult:
    """CALU_PRRP of A in place with tournament pivoting over row tiles."""
    from . import _lib
    torch = _torch()
    _check_matrix(A)
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    ws_bytes = _lib.workspace_size(n, b, 1, tile_rows)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc(ws_bytes, A.device)
    perm = torch.empty(n, dtype=torch.int64, device=A.device)
    stats = torch.zeros(_lib.STATS_BYTES, dtype=torch.uint8, device=A.device)
    code = _lib.lib().calu_prrp_factor(A.data_ptr(), n, A.stride(0), b, float(tau), _lib.TREES[tree],
                                       tile_rows, perm.data_ptr(), stats.data_ptr(),
                                       workspace.data_ptr(), workspace.numel(), _stream_ptr(),
                                       _lib.PRECISIONS[precision])
    _lib.check(code, "calu_prrp_factor")
    return FactorResult(perm, stats, workspace)


@dataclass
class BlockFactorResult:
    perm: object        # torch int64 [n] on the device
    nodes: object       # torch int32 node records on the device (layout in include/prrp.h)
    stats_raw: object
    workspace: object
    b: int

    def stats(self) -> dict:
        return read_stats(self.stats_raw)


def block_factor(A, b: int, tau: float = 2.0, tree: str = "binary", tile_rows: int = 512,
                 workspace=None) -> BlockFactorResult:
    """Block parallel (tree="binary") or block pairwise (tree="flat") LU_PRRP
    of A in place (Section 5, Appendix E)."""
    from . import _lib
    torch = _torch()
    _check_matrix(A)
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    ws_bytes, entries = _lib.block_sizes(n, b, _lib.TREES[tree], tile_rows)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc(ws_bytes, A.device)
    perm = torch.empty(n, dtype=torch.int64, device=A.device)
    nodes = torch.empty(entries, dtype=torch.int32, device=A.device)
    stats = torch.zeros(_lib.STATS_BYTES, dtype=torch.uint8, device=A.device)
    code = _lib.lib().prrp_block_factor(A.data_ptr(), n, A.stride(0), b, float(tau), _lib.TREES[tree],
                                        tile_rows, perm.data_ptr(), nodes.data_ptr(), entries,
                                        stats.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                        _stream_ptr())
    _lib.check(code, "prrp_block_factor")
    return BlockFactorResult(perm, nodes, stats, workspace, b)


def block_solve(LU, r: BlockFactorResult, B, workspace=None):
    """x with A x = B from block_factor's factors; returns a new tensor."""
    from . import _lib
    _check_matrix(LU, "LU")
    n = LU.shape[0]
    Bc = B.contiguous()
    if Bc.dim() == 1:
        Bc = Bc.view(n, 1)
    nrhs = Bc.shape[1]
    X = Bc.clone()
    ws_bytes = _lib.solve_workspace_size(n, nrhs)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc(ws_bytes, LU.device)
    code = _lib.lib().prrp_block_solve(LU.data_ptr(), n, LU.stride(0), r.b, r.perm.data_ptr(),
                                       r.nodes.data_ptr(), Bc.data_ptr(), nrhs, X.data_ptr(), nrhs,
                                       nrhs, workspace.data_ptr(), workspace.numel(), _stream_ptr())
    _lib.check(code, "prrp_block_solve")
    return X.view(B.shape)


def solve(LU, perm, B, workspace=None):
    """X = U^-1 L^-1 B[perm]; returns a new tensor (B is not modified)."""
    from . import _lib
    _check_matrix(LU, "LU")
    n = LU.shape[0]
    X = B.clone().contiguous()
    if X.dim() == 1:
        X = X.view(n, 1)
    nrhs = X.shape[1]
    ws_bytes = _lib.solve_workspace_size(n, nrhs)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc(ws_bytes, LU.device)
    code = _lib.lib().prrp_solve(LU.data_ptr(), n, LU.stride(0), perm.data_ptr(), X.data_ptr(), nrhs,
                                 X.stride(0), workspace.data_ptr(), workspace.numel(), _stream_ptr())
    _lib.check(code, "prrp_solve")
    return X.view(B.shape)


def residual(A, X, B):
    """R = B - A X with a doubled-precision accumulation (rounded once)."""
    from . import _lib
    torch = _torch()
    _check_matrix(A)
    n = A.shape[0]
    X2 = X.contiguous().view(n, -1)
    B2 = B.contiguous().view(n, -1)
    R = torch.empty_like(X2)
    code = _lib.lib().prrp_residual(A.data_ptr(), n, A.stride(0), X2.data_ptr(), B2.data_ptr(),
                                    R.data_ptr(), X2.shape[1], X2.stride(0), _stream_ptr())
    _lib.check(code, "prrp_residual")
    return R.view(B.shape)


def refine(A, LU, perm, B, tol: float = 1e-14, max_iter: int = 30, workspace=None):
    """Iterative refinement; returns (X, iterations, last max|dX|/max|X|,
    status), status one of "converged", "stagnated", "cap"."""
    import ctypes
    from . import _lib
    torch = _torch()
    _check_matrix(A)
    n = A.shape[0]
    B2 = B.contiguous().view(n, -1)
    nrhs = B2.shape[1]
    X = torch.empty_like(B2)
    ws_bytes = _lib.solve_workspace_size(n, nrhs)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc(ws_bytes, A.device)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    status = ctypes.c_int(0)
    code = _lib.lib().prrp_refine(A.data_ptr(), LU.data_ptr(), n, A.stride(0), perm.data_ptr(),
                                  B2.data_ptr(), X.data_ptr(), nrhs, nrhs, float(tol), int(max_iter),
                                  ctypes.byref(it), ctypes.byref(rel), ctypes.byref(status),
                                  workspace.data_ptr(), workspace.numel(), _stream_ptr())
    _lib.check(code, "prrp_refine")
    return X.view(B.shape), it.value, rel.value, _lib.IR_STATUS[status.value]


def refine_async(A, LU, perm, B, tol: float = 1e-14, max_iter: int = 30, workspace=None):
    """Iterative refinement enqueued without host synchronisation.

    Returns (X, iters, rel, status) where iters (int32), rel (float64) and
    status (int32, a PRRP_IR_* value) are one-element device tensors filled
    when the stream reaches them."""
    from . import _lib
    torch = _torch()
    _check_matrix(A)
    n = A.shape[0]
    B2 = B.contiguous().view(n, -1)
    nrhs = B2.shape[1]
    X = torch.empty_like(B2)
    ws_bytes = _lib.solve_workspace_size(n, nrhs)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = _alloc(ws_bytes, A.device)
    it = torch.zeros(1, dtype=torch.int32, device=A.device)
    rel = torch.zeros(1, dtype=torch.float64, device=A.device)
    status = torch.zeros(1, dtype=torch.int32, device=A.device)
    code = _lib.lib().prrp_refine_async(A.data_ptr(), LU.data_ptr(), n, A.stride(0), perm.data_ptr(),
                                        B2.data_ptr(), X.data_ptr(), nrhs, nrhs, float(tol),
                                        int(max_iter), it.data_ptr(), rel.data_ptr(),
                                        status.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                        _stream_ptr())
    _lib.check(code, "prrp_refine_async")
    return X.view(B.shape), it, rel, status


def refine_async_static(A, LU, perm, B, tol: float = 1e-14, max_iter: int = 30):
    """refine_async without any workspace: the library's fixed device scratch
    (no allocation, usable under graph capture).  Calls that overlap on one
    GPU race on that scratch.  Returns (X, iters, rel, status) as
    refine_async (X is allocated here by torch, outside the library)."""
    from . import _lib
    torch = _torch()
    _check_matrix(A)
    n = A.shape[0]
    B2 = B.contiguous().view(n, -1)
    nrhs = B2.shape[1]
    X = torch.empty_like(B2)
    it = torch.zeros(1, dtype=torch.int32, device=A.device)
    rel = torch.zeros(1, dtype=torch.float64, device=A.device)
    status = torch.zeros(1, dtype=torch.int32, device=A.device)
    code = _lib.lib().prrp_refine_async_static(A.data_ptr(), LU.data_ptr(), n, A.stride(0),
                                               perm.data_ptr(), B2.data_ptr(), X.data_ptr(), nrhs,
                                               nrhs, float(tol), int(max_iter), it.data_ptr(),
                                               rel.data_ptr(), status.data_ptr(), _stream_ptr())
    _lib.check(code, "prrp_refine_async_static")
    return X.view(B.shape), it, rel, status


def refine_gmres(A, LU, perm, b, tol: float = 1e-14, gmres_tol: float = 1e-8, max_inner: int = 60,
                 max_outer: int = 20, workspace=None):
    """GMRES-based refinement (one right-hand side).  tol > 0 stops on the
    correction's size (max|d| <= tol max|x|), tol = 0 on the componentwise
    backward error w reaching the unit roundoff.

    Returns (x, outer steps, total GMRES steps, w of the unrefined solution,
    final w, last max|d|/max|x|, status) with status "converged",
    "stagnated" or "cap"."""
    import ctypes
    from . import _lib
    torch = _torch()
    _check_matrix(A)
    n = A.shape[0]
    bv = b.contiguous().view(n)
    x = torch.empty_like(bv)
    need = ctypes.c_size_t(0)
    _lib.check(_lib.lib().prrp_gmres_workspace_size(n, int(max_inner), ctypes.byref(need)),
               "prrp_gmres_workspace_size")
    if workspace is None or workspace.numel() < need.value:
        workspace = _alloc(need.value, A.device)
    outer, inner, st = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    w0, w1, rel = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    code = _lib.lib().prrp_refine_gmres(A.data_ptr(), LU.data_ptr(), n, A.stride(0), perm.data_ptr(),
                                        bv.data_ptr(), x.data_ptr(), float(tol), float(gmres_tol),
                                        int(max_inner), int(max_outer), ctypes.byref(outer),
                                        ctypes.byref(inner), ctypes.byref(w0), ctypes.byref(w1),
                                        ctypes.byref(rel), ctypes.byref(st), workspace.data_ptr(),
                                        workspace.numel(), _stream_ptr())
    _lib.check(code, "prrp_refine_gmres")
    return x, outer.value, inner.value, w0.value, w1.value, rel.value, _lib.IR_STATUS[st.value]


class BatchPlan:
    """Batched LU_PRRP (+ optional refinement) of systems of uneven sizes.

    ``mats``: list of square float64 CUDA tensors factored in place.  With
    ``originals``/``rhs`` given, each system is refined after its
    factorization into the tensors of ``solutions``.  ``run()`` enqueues the
    plan on the current stream (``graph=True`` captures it once into a HIP
    graph and replays it afterwards)."""

    def __init__(self, mats, bs, tau: float = 2.0, precision: str = "fp64", rows_per_wg: int = 64,
                 originals=None, rhs=None, tol: float = 1e-14, max_iter: int = 10):
        import ctypes
        from . import _lib
        torch = _torch()
        count = len(mats)
        if count < 1 or len(bs) != count:
            raise ValueError("one panel width per matrix")
        for M in mats:
            _check_matrix(M)
        dev = mats[0].device
        self.mats = list(mats)
        self.perms = [torch.empty(M.shape[0], dtype=torch.int64, device=dev) for M in mats]
        self.stats_raw = torch.zeros(count * _lib.STATS_BYTES, dtype=torch.uint8, device=dev)
        self.originals = originals
        self.rhs = None
        self.solutions = None
        arr = lambda ct, vals: (ct * count)(*vals)  # noqa: E731
        self._keep = []
        pA = arr(ctypes.c_void_p, [M.data_ptr() for M in mats])
        pn = arr(ctypes.c_int64, [M.shape[0] for M in mats])
        plda = arr(ctypes.c_int64, [M.stride(0) for M in mats])
        pb = arr(ctypes.c_int, [int(b) for b in bs])
        pperm = arr(ctypes.c_void_p, [p.data_ptr() for p in self.perms])
        self._keep += [pA, pn, plda, pb, pperm]
        pA0 = pB = pX = pnr = None
        if originals is not None:
            self.rhs = [r.contiguous().view(M.shape[0], -1) for r, M in zip(rhs, mats)]
            self.solutions = [torch.empty_like(r) for r in self.rhs]
            for O, M in zip(originals, mats):
                _check_matrix(O, "original")
                if O.stride(0) != M.stride(0):
                    raise ValueError("original and factored matrices need equal leading dimensions")
            pA0 = arr(ctypes.c_void_p, [O.data_ptr() for O in originals])
            pB = arr(ctypes.c_void_p, [r.data_ptr() for r in self.rhs])
            pX = arr(ctypes.c_void_p, [x.data_ptr() for x in self.solutions])
            pnr = arr(ctypes.c_int64, [r.shape[1] for r in self.rhs])
            self._keep += [pA0, pB, pX, pnr]
        need = ctypes.c_size_t(0)
        _lib.check(_lib.lib().prrp_batch_plan_workspace_size(count, pn, pb, pnr, int(rows_per_wg),
                                                             ctypes.byref(need)),
                   "prrp_batch_plan_workspace_size")
        self.workspace = _alloc(need.value, dev)
        handle = ctypes.c_void_p(0)
        code = _lib.lib().prrp_batch_plan_create(
            count, pA, pn, plda, pb, pperm, self.stats_raw.data_ptr(), float(tau),
            _lib.PRECISIONS[precision], int(rows_per_wg), pA0, pB, pX, pnr, float(tol),
            int(max_iter), self.workspace.data_ptr(), self.workspace.numel(), _stream_ptr(),
            ctypes.byref(handle))
        _lib.check(code, "prrp_batch_plan_create")
        self._h = handle

    def run(self, graph: bool = False):
        from . import _lib
        _lib.check(_lib.lib().prrp_batch_plan_run(self._h, _stream_ptr(), 1 if graph else 0),
                   "prrp_batch_plan_run")

    def stats(self, i: int) -> dict:
        from . import _lib
        w = _lib.STATS_BYTES
        return read_stats(self.stats_raw[i * w:(i + 1) * w])

    def infos(self) -> list:
        """The numerical status (prrp_stats.info) of every system, one copy
        of the stats records to the host."""
        from ._lib import Stats
        host = self.stats_raw.cpu().numpy().tobytes()
        w = len(host) // len(self.mats)
        return [int(Stats.from_buffer_copy(host[i * w:(i + 1) * w]).info)
                for i in range(len(self.mats))]

    def refine_results(self):
        """(iterations, last ratios, statuses) per system, copied to the host;
        a status is "converged", "stagnated" or "cap"."""
        import ctypes
        from . import _lib
        count = len(self.mats)
        it = (ctypes.c_int32 * count)()
        rel = (ctypes.c_double * count)()
        st = (ctypes.c_int32 * count)()
        _lib.check(_lib.lib().prrp_batch_plan_results(self._h, it, rel, st, _stream_ptr()),
                   "prrp_batch_plan_results")
        return list(it), list(rel), [_lib.IR_STATUS[v] for v in st]

    def close(self, synchronize: bool = True):
        """Releases the plan (its workspace is a torch tensor freed with this
        object).  Waits for the device first unless the caller knows that the
        plan's work has completed (synchronize=False)."""
        from . import _lib
        if getattr(self, "_h", None) is not None and self._h.value:
            if synchronize:
                _torch().cuda.synchronize()
            _lib.lib().prrp_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def gemm(A, B, C=None, alpha: float = 1.0, beta: float = 0.0, precision: str = "fp64"):
    """C = alpha A B + beta C with the library's MFMA kernel (row-major float64)."""
    from . import _lib
    torch = _torch()
    for t, nm in ((A, "A"), (B, "B")):
        _check_matrix(t, nm)
    M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = torch.zeros(M, N, dtype=torch.float64, device=A.device)
    _check_matrix(C, "C")
    code = _lib.lib().prrp_gemm(M, N, K, float(alpha), A.data_ptr(), A.stride(0), B.data_ptr(),
                                B.stride(0), float(beta), C.data_ptr(), C.stride(0),
                                _lib.PRECISIONS[precision], _stream_ptr())
    _lib.check(code, "prrp_gemm")
    return C
