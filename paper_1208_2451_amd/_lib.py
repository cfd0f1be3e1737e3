"""ctypes binding of libprrp.so (argument marshalling only).

Every computation runs in the gfx950 kernels behind the C ABI declared in
include/prrp.h; torch supplies device memory and the current stream.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprrp.so")

PRRP_FP64, PRRP_SCHUR_FP32, PRRP_SCHUR_BF16 = 0, 1, 2
PRRP_TREE_BINARY, PRRP_TREE_FLAT = 0, 1
PRECISIONS = {"fp64": PRRP_FP64, "fp32": PRRP_SCHUR_FP32, "bf16": PRRP_SCHUR_BF16}
PRRP_IR_CONVERGED, PRRP_IR_STAGNATED, PRRP_IR_CAP = 0, 1, 2
IR_STATUS = {PRRP_IR_CONVERGED: "converged", PRRP_IR_STAGNATED: "stagnated", PRRP_IR_CAP: "cap"}
TREES = {"binary": PRRP_TREE_BINARY, "flat": PRRP_TREE_FLAT}


class Stats(ctypes.Structure):
    _fields_ = [
        ("max_abs_A", ctypes.c_double),
        ("max_abs_W", ctypes.c_double),
        ("max_abs_U", ctypes.c_double),
        ("max_block_L", ctypes.c_double),
        ("swaps", ctypes.c_int64),
        ("info", ctypes.c_int32),
        ("tree_height", ctypes.c_int32),
        ("panels", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


STATS_BYTES = ctypes.sizeof(Stats)

_vp, _i64, _i32, _dbl, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t

_SIGS = {
    "prrp_workspace_size": (_i32, [_i64, _i32, _i32, _i64, ctypes.POINTER(_sz)]),
    "prrp_factor": (_i32, [_vp, _i64, _i64, _i32, _dbl, _vp, _vp, _vp, _sz, _vp]),
    "prrp_factor_mixed": (_i32, [_vp, _i64, _i64, _i32, _dbl, _vp, _vp, _vp, _sz, _vp, _i32]),
    "calu_prrp_factor": (_i32, [_vp, _i64, _i64, _i32, _dbl, _i32, _i64, _vp, _vp, _vp, _sz, _vp, _i32]),
    "prrp_solve_workspace_size": (_i32, [_i64, _i64, ctypes.POINTER(_sz)]),
    "prrp_block_sizes": (_i32, [_i64, _i32, _i32, _i64, ctypes.POINTER(_sz), ctypes.POINTER(_i64)]),
    "prrp_block_factor": (_i32, [_vp, _i64, _i64, _i32, _dbl, _i32, _i64, _vp, _vp, _i64, _vp, _vp,
                                 _sz, _vp]),
    "prrp_block_solve": (_i32, [_vp, _i64, _i64, _i32, _vp, _vp, _vp, _i64, _vp, _i64, _i64, _vp,
                                _sz, _vp]),
    "prrp_solve": (_i32, [_vp, _i64, _i64, _vp, _vp, _i64, _i64, _vp, _sz, _vp]),
    "prrp_residual": (_i32, [_vp, _i64, _i64, _vp, _vp, _vp, _i64, _i64, _vp]),
    "prrp_refine": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _i64, _i64, _dbl, _i32,
                           ctypes.POINTER(_i32), ctypes.POINTER(_dbl), ctypes.POINTER(_i32),
                           _vp, _sz, _vp]),
    "prrp_refine_async": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _i64, _i64, _dbl, _i32,
                                 _vp, _vp, _vp, _vp, _sz, _vp]),
    "prrp_static_scratch_bytes": (_sz, []),
    "prrp_refine_async_static": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _i64, _i64, _dbl,
                                        _i32, _vp, _vp, _vp, _vp]),
    "prrp_gmres_workspace_size": (_i32, [_i64, _i32, ctypes.POINTER(_sz)]),
    "prrp_refine_gmres": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _dbl, _dbl, _i32, _i32,
                                 ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_dbl),
                                 ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(_i32),
                                 _vp, _sz, _vp]),
    "prrp_panel_cus": (_i32, [_i32, _i64, _i32, _i32, _i64, _i32, ctypes.POINTER(_i64)]),
    "prrp_batch_plan_workspace_size": (_i32, [_i64, _vp, _vp, _vp, _i32, ctypes.POINTER(_sz)]),
    "prrp_batch_plan_create": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _vp, _dbl, _i32, _i32,
                                      _vp, _vp, _vp, _vp, _dbl, _i32, _vp, _sz, _vp,
                                      ctypes.POINTER(_vp)]),
    "prrp_batch_plan_run": (_i32, [_vp, _vp, _i32]),
    "prrp_batch_plan_results": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "prrp_batch_plan_destroy": (_i32, [_vp]),
    "prrp_gemm": (_i32, [_i64, _i64, _i64, _dbl, _vp, _i64, _vp, _i64, _dbl, _vp, _i64, _i32, _vp]),
    "prrp_profile_enable": (_i32, [_i32]),
    "prrp_profile_read": (_i32, [ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]),
    "prrp_status_string": (ctypes.c_char_p, [_i32]),
    "prrp_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libprrp.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libprrp.so is not built (expected at %s); run "
                "`python -m paper_1208_2451_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PrrpError(RuntimeError):
    pass


def check(code: int, what: str) -> None:
    if code != 0:
        msg = lib().prrp_status_string(code).decode()
        raise PrrpError("%s failed with code %d: %s" % (what, code, msg))


def workspace_size(n: int, b: int, method: int = 0, tile_rows: int = 0) -> int:
    out = ctypes.c_size_t(0)
    check(lib().prrp_workspace_size(n, b, method, tile_rows, ctypes.byref(out)), "prrp_workspace_size")
    return out.value


def solve_workspace_size(n: int, nrhs: int) -> int:
    out = ctypes.c_size_t(0)
    check(lib().prrp_solve_workspace_size(n, nrhs, ctypes.byref(out)), "prrp_solve_workspace_size")
    return out.value


def block_sizes(n: int, b: int, tree: int, tile_rows: int):
    """(workspace bytes, int32 entries of the node records) of prrp_block_factor."""
    ws = ctypes.c_size_t(0)
    ne = ctypes.c_int64(0)
    check(lib().prrp_block_sizes(n, b, tree, tile_rows, ctypes.byref(ws), ctypes.byref(ne)),
          "prrp_block_sizes")
    return ws.value, ne.value


PHASES = ["srrqr", "gepp", "moves", "l21", "u12", "schur", "startup"]


def profile_enable(on: bool = True) -> None:
    lib().prrp_profile_enable(1 if on else 0)


def profile_read() -> dict:
    ms = (ctypes.c_double * len(PHASES))()
    cnt = (ctypes.c_int64 * len(PHASES))()
    lib().prrp_profile_read(ms, cnt)
    return {p: (ms[i], cnt[i]) for i, p in enumerate(PHASES)}
