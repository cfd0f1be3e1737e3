#!/usr/bin/env python
"""LU_PRRP benchmark on one MI355X.

Workload (the metric's configuration): n = 8192, b = 128, tau = 2, matrix
U diag(s) V^T with Haar-random orthogonal U, V and s log-spaced from 1 to
1e-6 (kappa = 1e6), one N(0,1) right-hand side.  A step is one pass of the
whole hot path: restore A from a resident copy, factor it (strong-RRQR
panels, diagonal GEPP, row moves, triangular products, Schur updates), then
solve with iterative refinement (doubled-precision residual) until the
correction is below 1e-13 of the solution.  Each Schur precision (FP64, and
FP32 / BF16 operands with FP32 accumulation) is timed; `value` is the
fastest time-to-solution that reaches the 1e-12 forward-error target,
reported as TFLOP/s with the 2n^3/3 convention.

Prints one JSON line.  Only one GPU is used (--gpus above 1 exits).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LU_PRRP TFLOP/s (2n^3/3) FP64 vs mixed+IR at n=8192; solves/s + p99 latency"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_GBS = 8000.0


def schur_flops(n: int, b: int) -> float:
    tot = 0.0
    for k0 in range(0, n, b):
        bw = min(b, n - k0)
        m = n - k0
        tot += 2.0 * (m - bw) * (n - k0 - bw) * bw
    return tot


def srrqr_flops(n: int, b: int) -> float:
    """Appendix C strong-RRQR count per panel, 2 m b^2 - 2/3 b^3, summed."""
    tot = 0.0
    for k0 in range(0, n, b):
        bw = min(b, n - k0)
        m = n - k0
        tot += 2.0 * m * bw * bw - 2.0 / 3.0 * bw ** 3
    return tot


def measured_traffic(kernel_source: str, summary: str):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
        src = open(os.path.join(ROOT, "paper_1208_2451_amd", "csrc", kernel_source), "rb").read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if "=" in line and line.startswith("    "):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256_prefix") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    return float(vals["traffic_bytes_per_launch"])


def reference_solution(A, b, iters: int = 10, lu_piv=None):
    """Accuracy reference, independent of the library: LAPACK getrf, then
    refinement whose residuals b - A x are accumulated in the host's extended
    precision (x86 long double, 64-bit significand) in row blocks.  Its own
    forward error is a few 1e-14 at kappa = 1e6, far inside the 1e-12 target."""
    import numpy as np
    import scipy.linalg as sla
    if lu_piv is None:
        lu_piv = sla.lu_factor(A)
    x = sla.lu_solve(lu_piv, b)
    for _ in range(iters):
        xl = x.astype(np.longdouble)
        r = np.empty(len(b), dtype=np.float64)
        for i in range(0, A.shape[0], 256):
            r[i:i + 256] = (b[i:i + 256].astype(np.longdouble)
                            - A[i:i + 256].astype(np.longdouble) @ xl).astype(np.float64)
        d = sla.lu_solve(lu_piv, r)
        x = x + d
        if np.abs(d).max() <= 1e-17 * np.abs(x).max():
            break
    return x


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(A_host, b, tau, panels):
    """The oracle as it stands, on the first `panels` panels of the same matrix."""
    import numpy as np
    from oracle import lu as olu
    from oracle import metrics as om
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        threads = os.cpu_count() or 1
    n = A_host.shape[0]
    t0 = time.perf_counter()
    olu.lu_prrp(A_host, b, tau, panels=panels)
    dt = time.perf_counter() - t0
    flops = sum(om.flops_step(n, n, b, k) for k in range(1, panels + 1))
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": "oracle LU_PRRP (NumPy FP64) on the first %d of %d panels of the same "
                      "n=%d, b=%d matrix: %.3g flops (Appendix C per-panel counts) in %.1f s"
                      % (panels, (n + b - 1) // b, n, b, flops, dt),
            "seconds": dt}


def serving_bench(nreq: int, seed: int, rates=(0.3, 0.5, 0.7, 1.0)):
    """Continuous-batching solve server: n uniform in {64, 96, ..., 2048},
    b = min(32, n/4), N(0,1) systems with 1-8 right-hand sides, FP32 Schur
    update and FP64 refinement.  The autotuner picks the launch shapes, a
    saturated run gives the capacity, and Poisson runs of `nreq` requests
    arrive at each fraction of it in `rates` (p50 / p99 per rate)."""
    import torch
    from paper_1208_2451_amd import autotune, serving
    t0 = time.perf_counter()
    tuning = autotune.tune(batch=8, batch_options=(8, 16, 32), trials=1)
    log("autotune %.1f s: %s" % (time.perf_counter() - t0, json.dumps(
        {"rows_per_wg": tuning["rows_per_wg"], "max_batch": tuning["max_batch"]})))
    rpw = autotune.rows_per_wg_fn(tuning)
    srv = serving.Server(max_batch=tuning["max_batch"], slots=3, precision="fp32", max_iter=10,
                         rows_per_wg=rpw)
    warm = serving.materialize(serving.make_requests(24, seed + 5, 1e9), "cuda")
    srv.serve(warm, realtime=False)
    del warm
    sat_reqs = serving.materialize(serving.make_requests(max(48, nreq // 4), seed + 1, 1e9), "cuda")
    sat = srv.serve(sat_reqs, realtime=False)
    del sat_reqs
    log("serving saturated", json.dumps(sat))
    sweep = []
    same = True
    for k, frac in enumerate(rates):
        rate = frac * sat["solves_per_s"]
        reqs = serving.materialize(serving.make_requests(nreq, seed + 2 + k, rate), "cuda")
        run = srv.serve(reqs, realtime=True)
        torch.cuda.synchronize()
        if frac == 0.7:
            for r in reqs[:: max(1, len(reqs) // 8)]:
                x, _ = serving.solve_alone(r, precision="fp32", max_iter=10, rows_per_wg=rpw(r.n))
                same = same and bool(torch.equal(x, r.X))
        run.update({"load": frac, "rate_per_s": rate})
        log("serving load %.1f" % frac, json.dumps(run))
        sweep.append(run)
        del reqs
        torch.cuda.empty_cache()
    head = next(r for r in sweep if r["load"] == 0.7) if 0.7 in rates else sweep[-1]
    out = dict(head)
    out.update({"saturated_solves_per_s": sat["solves_per_s"], "saturated_tflops": sat["tflops"],
                "mix_equals_alone_sampled": same, "max_batch": tuning["max_batch"],
                "rows_per_wg": tuning["rows_per_wg"],
                "sweep": [{k: r[k] for k in ("load", "rate_per_s", "requests", "solves_per_s",
                                             "p50_ms", "p99_ms", "not_converged",
                                             "factor_info_nonzero", "batches",
                                             "plan_build_ms_mean")} for r in sweep],
                "kind": "Poisson arrivals at %s x saturated capacity, %d requests each; n uniform "
                        "in {64..2048} step 32, b = min(32, n/4), 1-8 rhs, FP32 Schur + FP64 "
                        "refinement to 1e-14; latency = completion - arrival; headline fields at "
                        "0.7" % (list(rates), nreq)})
    return out


def hpl_metrics(A, x, b):
    """HPL1, HPL2, HPL3 of the experiments' section (eps = 2^-53), for the
    record (host NumPy on the solution the device returned)."""
    import numpy as np
    eps = 2.0 ** -53
    n = A.shape[0]
    r = float(np.abs(A @ x - b).max())
    a1 = float(np.abs(A).sum(axis=0).max())
    ainf = float(np.abs(A).sum(axis=1).max())
    return {"HPL1": r / (eps * a1 * n), "HPL2": r / (eps * a1 * float(np.abs(x).sum())),
            "HPL3": r / (eps * ainf * float(np.abs(x).max()) * n)}


def calu_bench(n: int, b: int, tile_rows: int, tau: float, seed: int, steps: int, warmup: int):
    """CALU_PRRP, binary tournament over 512-row tiles, on an N(0,1) matrix:
    factor time and TFLOP/s (2n^3/3), and the per-phase device times."""
    import torch
    import paper_1208_2451_amd as prrp
    from paper_1208_2451_amd import _lib
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    A0 = torch.randn(n, n, generator=g, dtype=torch.float64, device=dev)
    A = torch.empty_like(A0)
    ws = torch.empty(_lib.workspace_size(n, b, 1, tile_rows), dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        A.copy_(A0)
        prrp.calu_factor(A, b, tau, tree="binary", tile_rows=tile_rows, workspace=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        A.copy_(A0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = prrp.calu_factor(A, b, tau, tree="binary", tile_rows=tile_rows, workspace=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    st = r.stats()
    _lib.profile_enable(True)
    A.copy_(A0)
    prrp.calu_factor(A, b, tau, tree="binary", tile_rows=tile_rows, workspace=ws)
    torch.cuda.synchronize()
    phases = _lib.profile_read()
    _lib.profile_enable(False)
    ms = 1e3 * sum(times) / len(times)
    nominal = 2.0 * n ** 3 / 3.0
    ph = {k: v[0] for k, v in phases.items()}
    out = {"workload": "CALU_PRRP factor, n=%d, b=%d, tau=%g, binary tree over %d-row tiles, "
                       "N(0,1) matrix" % (n, b, tau, tile_rows),
           "ms_per_factor": ms, "tflops": nominal / (ms * 1e-3) / 1e12, "steps": steps,
           "g_W": st["g_W"], "tree_height": st["tree_height"], "info": st["info"],
           "max_block_L": st["max_block_L"], "swaps": st["swaps"],
           "phase_ms_per_factor": ph,
           "phase_launches_per_factor": {k: v[1] for k, v in phases.items()}}
    # the dominant kernel: the tournament (latency bound) or the Schur GEMM
    dom = max(("srrqr", "schur"), key=lambda k: ph[k])
    if dom == "schur":
        fl = schur_flops(n, b)
        ach = fl / (ph["schur"] * 1e-3) / 1e12
        out["roofline"] = {"kernel": "schur_gemm (gemm_kernel<double>)", "bound": "mfma",
                           "achieved": ach, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                           "frac": ach / PEAK_TFLOPS["fp64"], "traffic": None}
    else:
        out["roofline"] = {"kernel": "srrqr_kernel (tournament nodes and leaves)", "bound": "alu",
                           "ms_per_factor": ph["srrqr"],
                           "note": "latency bound: (tree height + 1) x b dependent pivot steps "
                                   "per panel"}
    del A, A0, ws
    torch.cuda.empty_cache()
    return out


def calu_sweep(n: int, b: int, tau: float, seed: int):
    """Tile-size sweep of CALU_PRRP (binary and flat trees) on one N(0,1)
    matrix: factor time and growth, with g_W / sqrt(n) beside the bands the
    paper reports for random matrices (Section 3.3: binary tree between
    sqrt(n)/2 and 3 sqrt(n)/4, flat tree between sqrt(n)/4 and 3 sqrt(n)/4)."""
    import math
    import torch
    import paper_1208_2451_amd as prrp
    from paper_1208_2451_amd import _lib
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed + 99)
    A0 = torch.randn(n, n, generator=g, dtype=torch.float64, device=dev)
    A = torch.empty_like(A0)
    out = []
    for tree, tiles in (("binary", (256, 512, 1024, 2048)), ("flat", (512, 2048))):
        for tr in tiles:
            ws = torch.empty(_lib.workspace_size(n, b, 1, tr), dtype=torch.uint8, device=dev)
            A.copy_(A0)
            prrp.calu_factor(A, b, tau, tree=tree, tile_rows=tr, workspace=ws)   # warm-up
            A.copy_(A0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = prrp.calu_factor(A, b, tau, tree=tree, tile_rows=tr, workspace=ws)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            st = r.stats()
            lo, hi = (0.5, 0.75) if tree == "binary" else (0.25, 0.75)
            gs = st["g_W"] / math.sqrt(n)
            out.append({"tree": tree, "tile_rows": tr, "ms": ms,
                        "tflops": 2.0 * n ** 3 / 3.0 / (ms * 1e-3) / 1e12,
                        "tree_height": st["tree_height"], "g_W": st["g_W"],
                        "g_W_over_sqrt_n": gs, "paper_band": [lo, hi],
                        "in_band": lo <= gs <= hi})
            del ws
    del A, A0
    torch.cuda.empty_cache()
    return {"n": n, "b": b, "runs": out}


def block_bench(n: int, b: int, tile_rows: int, tree: str, tau: float, seed: int, steps: int,
                warmup: int):
    """Block parallel (binary tree) or block pairwise (flat tree) LU_PRRP
    (Section 5, Appendix E) on an N(0,1) matrix: factor time, TFLOP/s
    (2n^3/3), growth, per-phase device times, and the solve's time and
    backward error."""
    import torch
    import paper_1208_2451_amd as prrp
    from paper_1208_2451_amd import _lib
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed + 7)
    A0 = torch.randn(n, n, generator=g, dtype=torch.float64, device=dev)
    A = torch.empty_like(A0)
    ws_bytes, _ = _lib.block_sizes(n, b, _lib.TREES[tree], tile_rows)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        A.copy_(A0)
        prrp.block_factor(A, b, tau, tree=tree, tile_rows=tile_rows, workspace=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        A.copy_(A0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = prrp.block_factor(A, b, tau, tree=tree, tile_rows=tile_rows, workspace=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    st = r.stats()
    rhs = torch.randn(n, 1, generator=g, dtype=torch.float64, device=dev)
    prrp.block_solve(A, r, rhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = prrp.block_solve(A, r, rhs)
    torch.cuda.synchronize()
    solve_ms = 1e3 * (time.perf_counter() - t0)
    res = (A0 @ x - rhs).abs().max().item()
    eta = res / (A0.abs().max().item() * x.abs().max().item() * n)
    _lib.profile_enable(True)
    A.copy_(A0)
    prrp.block_factor(A, b, tau, tree=tree, tile_rows=tile_rows, workspace=ws)
    torch.cuda.synchronize()
    phases = _lib.profile_read()
    _lib.profile_enable(False)
    ms = 1e3 * sum(times) / len(times)
    ph = {k: v[0] for k, v in phases.items()}
    kind = "block parallel" if tree == "binary" else "block pairwise"
    out = {"workload": "%s LU_PRRP factor, n=%d, b=%d, tau=%g, %s tree over %d-row tiles, N(0,1) "
                       "matrix" % (kind, n, b, tau, tree, tile_rows),
           "ms_per_factor": ms, "tflops": 2.0 * n ** 3 / 3.0 / (ms * 1e-3) / 1e12, "steps": steps,
           "g_W": st["g_W"], "max_abs_d": st["max_block_L"], "tree_height": st["tree_height"],
           "info": st["info"], "swaps": st["swaps"], "solve_ms": solve_ms,
           "backward_error": eta, "phase_ms_per_factor": ph,
           "phase_launches_per_factor": {k: v[1] for k, v in phases.items()},
           "roofline": {"kernel": "srrqr_kernel (tree nodes)", "bound": "alu",
                        "ms_per_factor": ph["srrqr"],
                        "note": "latency bound: every tree level is b dependent pivot steps, "
                                "each followed by its nodes' updates"}}
    del A, A0, ws
    torch.cuda.empty_cache()
    return out


def block_sweep(tau: float, seed: int):
    """Growth of block parallel LU_PRRP at n = 2048 with P = 16, 32 tiles and
    b = 2, 4, 8, 16 (the setting of Figure "bluprrp"), and of block pairwise
    LU_PRRP with the flat tree of height n / b (tiles of b rows) at n = 1024,
    2048 and b = 8, 16, 32 (Figure "fluprrp"), on N(0,1) matrices.  The
    figures are plots without printed values: the shape is what compares
    (Section 5: block parallel growth rising with P, block pairwise growth
    falling with b and staying below n)."""
    import torch
    import paper_1208_2451_amd as prrp
    dev = torch.device("cuda:0")
    out = {"parallel": [], "pairwise": []}

    def one(n, b, tree, tile_rows):
        g = torch.Generator(device=dev)
        g.manual_seed(seed + n + b)
        A = torch.randn(n, n, generator=g, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = prrp.block_factor(A, b, tau, tree=tree, tile_rows=tile_rows)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        st = r.stats()
        return {"n": n, "b": b, "tile_rows": tile_rows, "ms": ms, "g_W": st["g_W"],
                "info": st["info"]}

    for P in (16, 32):
        for b in (2, 4, 8, 16):
            row = one(2048, b, "binary", 2048 // P)
            row["P"] = P
            out["parallel"].append(row)
    for n in (1024, 2048):
        for b in (8, 16, 32):
            row = one(n, b, "flat", b)
            row["below_n"] = row["g_W"] < n
            out["pairwise"].append(row)
    torch.cuda.empty_cache()
    return out


def block_legs(tau: float, seed: int, steps: int, warmup: int):
    """Block parallel at the CALU_PRRP workload (n = 16384, b = 128, 512-row
    tiles), block pairwise at n = 8192 over 512-row tiles, and the growth sweep."""
    steps = max(1, min(3, steps))
    out = {"parallel": block_bench(16384, 128, 512, "binary", tau, seed, steps, warmup)}
    log("block parallel", json.dumps(out["parallel"]))
    out["pairwise"] = block_bench(8192, 128, 512, "flat", tau, seed, steps, warmup)
    log("block pairwise", json.dumps(out["pairwise"]))
    out["growth_sweep"] = block_sweep(tau, seed)
    log("block growth sweep", json.dumps(out["growth_sweep"]))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--b", type=int, default=128)
    ap.add_argument("--tau", type=float, default=2.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precisions", default="fp64,fp32,fp32-gmres,bf16",
                    help="variants: Schur precision (fp64, fp32, bf16), optionally -gmres for "
                         "GMRES-based refinement")
    ap.add_argument("--tol", type=float, default=1e-13)
    ap.add_argument("--cpu-panels", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--solves", type=int, default=200)
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of each Poisson serving run (0 skips serving)")
    ap.add_argument("--no-rhs16", dest="rhs16", action="store_false",
                    help="skip the 16 right-hand-side runs")
    ap.add_argument("--calu-n", type=int, default=16384,
                    help="order of the CALU_PRRP run (0 skips it)")
    ap.add_argument("--calu-only", action="store_true",
                    help="run only the CALU_PRRP leg (for kernel traces) and print its JSON")
    ap.add_argument("--no-block", dest="block", action="store_false",
                    help="skip the block parallel / block pairwise LU_PRRP legs")
    ap.add_argument("--block-only", action="store_true",
                    help="run only the block parallel / pairwise legs and print their JSON")
    ap.add_argument("--host-matrix", action="store_true",
                    help="build the kappa matrix with NumPy on the host (same recipe) and copy it "
                         "in, instead of building it with device QR")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy (neg of the n x n FP64 matrix, 2 n^2 8 bytes) "
                         "first, as the scale for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU; the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1208_2451_amd as prrp
    from paper_1208_2451_amd import _lib, inputs

    if args.calu_only:
        print(json.dumps(calu_bench(args.calu_n or 16384, 128, 512, args.tau, args.seed,
                                    args.steps, args.warmup)), flush=True)
        return
    if args.block_only:
        print(json.dumps(block_legs(args.tau, args.seed, args.steps, args.warmup)), flush=True)
        return

    n, b, tau = args.n, args.b, args.tau
    dev = torch.device("cuda:0")
    if args.host_matrix:
        log("generating kappa=1e6 matrix n=%d on the host" % n)
        A0 = torch.from_numpy(inputs.kappa_matrix(n, args.seed, 1e6)).to(dev)
    else:
        log("generating kappa=1e6 matrix n=%d on the GPU" % n)
        A0 = inputs.kappa_matrix(n, args.seed, 1e6, device="cuda:0")
    B = torch.from_numpy(inputs.rhs(n, args.seed, 1)).to(dev)
    A = torch.empty_like(A0)
    ws = torch.empty(_lib.workspace_size(n, b, 0, 0), dtype=torch.uint8, device=dev)
    sws = torch.empty(_lib.solve_workspace_size(n, 1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    if args.copy_calibration:
        torch.neg(A0, out=A)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (8 * n * n, 8 * n * n))

    x_ref = None
    A_host = A0.cpu().numpy()
    B16 = torch.from_numpy(inputs.rhs(n, args.seed, 16)).to(dev)
    if not args.no_accuracy:
        import scipy.linalg as sla
        log("reference solutions: LAPACK getrf + refinement with extended-precision residuals")
        lu_piv = sla.lu_factor(A_host)
        x_ref = reference_solution(A_host, B.cpu().numpy()[:, 0], lu_piv=lu_piv)
        B16h = B16.cpu().numpy()
        x_ref16 = {c: reference_solution(A_host, B16h[:, c], lu_piv=lu_piv) for c in (0, 15)}
        del lu_piv

    nominal = 2.0 * n ** 3 / 3.0
    variants = {}
    perm64 = None
    gws = None
    for variant in [p.strip() for p in args.precisions.split(",") if p.strip()]:
        # "<schur precision>" refines with one triangular solve per
        # correction; "<schur precision>-gmres" with GMRES-based refinement
        prec, _, how = variant.partition("-")
        gmres = how == "gmres"
        log("variant", variant)

        def step(rhs=B):
            A.copy_(A0)
            r = prrp.factor(A, b, tau, precision=prec, workspace=ws)
            if gmres:
                x, outer, inner, w0, w1, rel, status = prrp.refine_gmres(
                    A0, A, r.perm, rhs[:, 0], tol=args.tol, gmres_tol=1e-8, max_inner=60,
                    max_outer=10, workspace=gws)
                return r, x.view(n, 1), outer, inner, rel, status
            X, it, rel, status = prrp.refine(A0, A, r.perm, rhs, tol=args.tol, max_iter=30,
                                             workspace=sws if rhs is B else None)
            return r, X, it, 0, rel, status

        if gmres and gws is None:
            import ctypes
            need = ctypes.c_size_t(0)
            _lib.check(_lib.lib().prrp_gmres_workspace_size(n, 60, ctypes.byref(need)), "gmres ws")
            gws = torch.empty(need.value, dtype=torch.uint8, device=dev)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        times, iters, inners, rels = [], [], [], []
        t_all = time.perf_counter()
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r, X, it, inner, rel, status = step()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            iters.append(it)
            inners.append(inner)
            rels.append(rel)
        wall = time.perf_counter() - t_all
        ms = 1e3 * wall / args.steps
        st = r.stats()
        perm = r.perm.cpu().numpy()
        if prec == "fp64" and perm64 is None:
            perm64 = perm
        # the factors of the last step are in A: the unrefined solution
        X0 = prrp.solve(A, r.perm, B, workspace=sws)
        torch.cuda.synchronize()
        # factor-only time and per-phase device times (separate profiled steps)
        _lib.profile_enable(True)
        for _ in range(max(1, min(2, args.steps))):
            A.copy_(A0)
            prrp.factor(A, b, tau, precision=prec, workspace=ws)
        torch.cuda.synchronize()
        phases = _lib.profile_read()
        _lib.profile_enable(False)
        nprof = max(1, min(2, args.steps))
        tf0 = time.perf_counter()
        A.copy_(A0)
        prrp.factor(A, b, tau, precision=prec, workspace=ws)
        torch.cuda.synchronize()
        factor_ms = 1e3 * (time.perf_counter() - tf0)
        err = err0 = hpl = None
        if x_ref is not None:
            xg = X.cpu().numpy()[:, 0]
            err = float(np.abs(xg - x_ref).max() / np.abs(x_ref).max())
            err0 = float(np.abs(X0.cpu().numpy()[:, 0] - x_ref).max() / np.abs(x_ref).max())
            hpl = hpl_metrics(A_host, xg, B.cpu().numpy()[:, 0])
        variants[variant] = {
            "ms_per_step": ms, "tflops_to_solution": nominal / (ms * 1e-3) / 1e12,
            "factor_ms": factor_ms, "tflops_factor": nominal / (factor_ms * 1e-3) / 1e12,
            "refinement": "gmres" if gmres else "one solve per correction",
            "ir_iterations": iters[-1], "gmres_steps": inners[-1] if gmres else None,
            "last_correction": rels[-1], "ir_status": status,
            "forward_error": err, "forward_error_unrefined": err0,
            "meets_1e-12": (err is not None and err <= 1e-12), "hpl": hpl,
            "pivots_equal_fp64_fraction": (float(np.mean(perm == perm64))
                                           if perm64 is not None else None),
            "g_W": st["g_W"], "max_block_L": st["max_block_L"], "swaps": st["swaps"], "info": st["info"],
            "phase_ms_per_factor": {k: v[0] / nprof for k, v in phases.items()},
            "phase_launches_per_factor": {k: v[1] // nprof for k, v in phases.items()},
        }
        # 16 right-hand sides (the workload's second configuration)
        if not gmres and args.rhs16:
            for _ in range(max(1, args.warmup)):
                step(B16)
            torch.cuda.synchronize()
            t16 = []
            for _ in range(args.steps):
                t0 = time.perf_counter()
                r16, X16, it16, _, rel16, st16 = step(B16)
                torch.cuda.synchronize()
                t16.append(time.perf_counter() - t0)
            e16 = None
            if x_ref is not None:
                Xh = X16.cpu().numpy()
                e16 = max(float(np.abs(Xh[:, c] - xr).max() / np.abs(xr).max())
                          for c, xr in x_ref16.items())
            variants[variant]["rhs16"] = {"ms_per_step": 1e3 * sum(t16) / len(t16),
                                       "ir_iterations": it16, "ir_status": st16,
                                       "forward_error_cols_0_15": e16,
                                       "meets_1e-12": e16 is not None and e16 <= 1e-12}
        log(variant, json.dumps(variants[variant]))

    # headline: fastest variant that meets the accuracy target (FP64 if none does)
    ok = [p for p, v in variants.items() if v["meets_1e-12"] or x_ref is None]
    head_variant = min(ok, key=lambda p: variants[p]["ms_per_step"]) if ok else "fp64"
    hv = variants[head_variant]
    head = head_variant.partition("-")[0]          # its Schur precision

    # roofline for the dominant kernel of the headline variant
    ph = hv["phase_ms_per_factor"]
    # the panel kernel or the Schur GEMM: the other phases are short kernels
    # off the panel chain (their sums over streams say little on their own)
    dom = max(("srrqr", "schur"), key=lambda k: ph[k])
    if dom == "schur":
        fl = schur_flops(n, b)
        ach = fl / (ph["schur"] * 1e-3) / 1e12
        roof = {"kernel": "schur_gemm (gemm_kernel<%s>)" % {"fp64": "double", "fp32": "float", "bf16": "bf16"}[head],
                "bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[head], "unit": "TFLOP/s",
                "frac": ach / PEAK_TFLOPS[head], "traffic": None,
                "algorithmic": "2 (m-b)(n-k0-b) b flops per panel update, %.4g flops per factorization" % fl}
    else:
        fl = srrqr_flops(n, b)
        ach = fl / (ph[dom] * 1e-3) / 1e12
        traffic = None
        if (n, b) == (8192, 128):
            traffic = measured_traffic("srrqr.hip", "hbm_counters_srrqr_n8192_b128_fp64.md")
        roof = {"kernel": "srrqr_kernel (strong RRQR panel)",
                "bound": "alu", "achieved": ach, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                "frac": ach / PEAK_TFLOPS["fp64"], "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated)",
                "algorithmic": "2 m b^2 - 2/3 b^3 flops per panel (Appendix C), %.4g per factorization" % fl,
                "note": "latency bound: b dependent pivot steps per panel"}
    roof["launches_per_factor"] = hv["phase_launches_per_factor"].get(dom)
    roof["ms_per_factor"] = ph[dom]

    # resident-factor solve latency (one right-hand side per call)
    A.copy_(A0)
    r = prrp.factor(A, b, tau, precision="fp64", workspace=ws)
    torch.cuda.synchronize()
    lat = []
    for _ in range(args.solves):
        t0 = time.perf_counter()
        prrp.solve(A, r.perm, B, workspace=sws)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    lat = np.array(lat) * 1e3
    solves = {"solves_per_s": float(1e3 / lat.mean()), "p50_ms": float(np.percentile(lat, 50)),
              "p99_ms": float(np.percentile(lat, 99)), "kind": "resident FP64 factors, n=%d, 1 rhs, "
              "one synchronized prrp_solve per request" % n}

    serving_out = None
    if args.serving_requests > 0:
        log("serving: %d requests" % args.serving_requests)
        serving_out = serving_bench(args.serving_requests, args.seed)

    calu = None
    if args.calu_n > 0:
        del A, A0
        torch.cuda.empty_cache()
        log("CALU_PRRP n=%d" % args.calu_n)
        calu = calu_bench(args.calu_n, 128, 512, tau, args.seed, max(1, min(3, args.steps)), 1)
        log("calu", json.dumps(calu))
        calu["tile_sweep"] = calu_sweep(8192, 128, tau, args.seed)
        log("calu tile sweep", json.dumps(calu["tile_sweep"]))

    block = None
    if args.block:
        log("block parallel / pairwise LU_PRRP")
        block = block_legs(tau, args.seed, args.steps, 1)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on %d panels" % args.cpu_panels)
        cpu = cpu_baseline(A_host, b, tau, args.cpu_panels)

    out = {
        "metric": METRIC, "value": hv["tflops_to_solution"], "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": hv["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else ("f64+f32" if head == "fp32" else "f64+bf16"),
        "data": "synthetic",
        "config": {"workload": "LU_PRRP factor + refinement to 1e-12, n=%d, b=%d, tau=%g, "
                               "U diag(s) V^T (Haar U,V; s log-spaced 1..1e-6), 1 rhs; variant %s"
                               % (n, b, tau, head_variant),
                   "n": n, "b": b, "tau": tau, "schur_precision": head, "variant": head_variant,
                   "nrhs": 1},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
        "solves": solves,
        "serving": serving_out,
        "calu_prrp": calu,
        "block_lu_prrp": block,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
