"""Continuous-batching solve server over batched LU_PRRP plans.

Requests (a square system with 1-8 right-hand sides, already resident in
device memory) arrive over time.  The server keeps a FIFO of arrived requests
and a few in-flight batch slots, each with its own stream.  Whenever a slot is
free it admits the oldest waiting requests into one batch, as many as fit the
batch limit and the device-memory budget (factor copy, plan workspace and
solution of each request).  Each batch is one plan: batched LU_PRRP with the
Schur update in the chosen precision, then FP64 refinement of every system
(``prrp_batch_plan_*`` in the C ABI).  Batches that arrive while others run
overlap on the device; completions are found by polling events, never by
blocking the host.  Latency is completion minus arrival.

All arithmetic runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    t_arrival: float
    n: int
    b: int
    nrhs: int
    seed: int
    A: object = None          # device float64 n x n (resident payload)
    B: object = None          # device float64 n x nrhs
    X: object = None          # solution, set on completion
    iters: int = -1
    status: str = ""          # refinement outcome: converged / stagnated / cap
    info: int = 0             # the factorization's numerical status (0: ok)
    t_admit: float = -1.0
    t_done: float = -1.0


def materialize(reqs, device):
    """Draws every request's matrix and right-hand sides on the device from
    its own seed (N(0,1) entries), as if uploaded before the run."""
    import torch
    for r in reqs:
        g = torch.Generator(device=device)
        g.manual_seed(int(r.seed))
        r.A = torch.randn(r.n, r.n, generator=g, dtype=torch.float64, device=device)
        r.B = torch.randn(r.n, r.nrhs, generator=g, dtype=torch.float64, device=device)
    return reqs


def make_requests(count: int, seed: int, rate: float, nmin: int = 64, nmax: int = 2048,
                  step: int = 32, max_rhs: int = 8):
    from . import inputs
    out = []
    for i, d in enumerate(inputs.serving_requests(count, seed, rate, nmin, nmax, step, max_rhs)):
        out.append(Request(i, d["t_arrival"], d["n"], d["b"], d["nrhs"], d["seed"]))
    return out


_WS_CACHE: dict = {}


def plan_bytes(n: int, b: int, nrhs: int, rows_per_wg: int) -> int:
    """Device bytes one request holds while in flight: its factor copy, its
    share of the plan workspace and its solution."""
    from . import _lib
    key = (n, b, nrhs, rows_per_wg)
    if key not in _WS_CACHE:
        pn = (ctypes.c_int64 * 1)(n)
        pb = (ctypes.c_int * 1)(b)
        pr = (ctypes.c_int64 * 1)(nrhs)
        need = ctypes.c_size_t(0)
        _lib.check(_lib.lib().prrp_batch_plan_workspace_size(1, pn, pb, pr, rows_per_wg,
                                                             ctypes.byref(need)),
                   "prrp_batch_plan_workspace_size")
        _WS_CACHE[key] = int(need.value) + 8 * n * n + 8 * n * nrhs
    return _WS_CACHE[key]


@dataclass
class Batch:
    reqs: list
    plan: object
    event: object
    bytes: int
    work: list = field(default_factory=list)


class Server:
    def __init__(self, device="cuda:0", max_batch: int = 16, slots: int = 3,
                 mem_budget: int | None = None, precision: str = "fp32", tau: float = 2.0,
                 tol: float = 1e-14, max_iter: int = 10, rows_per_wg=64):
        import torch
        self.device = torch.device(device)
        self.max_batch = int(max_batch)
        self.precision = precision
        self.tau = float(tau)
        self.tol = float(tol)
        self.max_iter = int(max_iter)
        # rows per panel workgroup: a number, or a callable n -> 64 / 128
        self.rows_per_wg = rows_per_wg if callable(rows_per_wg) else (lambda n, v=rows_per_wg: v)
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            mem_budget = int(0.5 * free)
        self.mem_budget = int(mem_budget)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(int(slots))]
        self.plan_ms = []         # host time to build each batch's plan

    def _launch(self, reqs, stream):
        import torch
        from . import BatchPlan
        with torch.cuda.stream(stream):
            work = [r.A.clone() for r in reqs]
            # one rows-per-workgroup value per batch (that of its largest system)
            rpw = self.rows_per_wg(max(r.n for r in reqs))
            t0 = time.perf_counter()
            plan = BatchPlan(work, [r.b for r in reqs], tau=self.tau, precision=self.precision,
                             rows_per_wg=rpw, originals=[r.A for r in reqs],
                             rhs=[r.B for r in reqs], tol=self.tol, max_iter=self.max_iter)
            self.plan_ms.append(1e3 * (time.perf_counter() - t0))
            # a plan is built for one batch's sizes and run once: capturing it
            # into a graph would cost more host time than the launches it saves
            plan.run(graph=False)
            ev = torch.cuda.Event()
            ev.record(stream)
        return plan, ev, work, rpw

    def serve(self, reqs, realtime: bool = True):
        """Runs the requests (sorted by arrival) to completion.  With
        ``realtime`` arrivals follow the wall clock from the call; otherwise
        every request is present at time 0 (saturation).  Returns a summary."""
        import torch
        reqs = sorted(reqs, key=lambda r: r.t_arrival)
        self.plan_ms = []
        waiting, inflight = [], [None] * len(self.streams)
        used = 0
        nxt = 0
        done = 0
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: float("inf"))
        while done < len(reqs):
            progressed = False
            for k, bt in enumerate(inflight):
                if bt is not None and bt.event.query():
                    t = time.perf_counter() - t0
                    with torch.cuda.stream(self.streams[k]):
                        its, _, sts = bt.plan.refine_results()
                        infos = bt.plan.infos()
                    for r, x, it, stt, inf in zip(bt.reqs, bt.plan.solutions, its, sts, infos):
                        r.t_done = t
                        r.X = x
                        r.iters = it
                        r.status = stt
                        r.info = inf
                    bt.plan.close(synchronize=False)
                    used -= bt.bytes
                    done += len(bt.reqs)
                    inflight[k] = None
                    progressed = True
            arrived_by = clock()
            while nxt < len(reqs) and reqs[nxt].t_arrival <= arrived_by:
                waiting.append(reqs[nxt])
                nxt += 1
                progressed = True
            for k in range(len(inflight)):
                if inflight[k] is not None or not waiting:
                    continue
                take, need = [], 0
                for r in waiting:
                    if len(take) >= self.max_batch:
                        break
                    nb = plan_bytes(r.n, r.b, r.nrhs, self.rows_per_wg(r.n))
                    # over budget: wait, unless nothing else holds memory
                    if used + need + nb > self.mem_budget and (take or used > 0):
                        break
                    take.append(r)
                    need += nb
                if not take:
                    break
                waiting = waiting[len(take):]
                t = time.perf_counter() - t0
                for r in take:
                    r.t_admit = t
                plan, ev, work, _ = self._launch(take, self.streams[k])
                inflight[k] = Batch(take, plan, ev, need, work)
                used += need
                progressed = True
            if not progressed:
                if realtime and nxt < len(reqs) and not waiting and all(b is None for b in inflight):
                    time.sleep(max(0.0, min(1e-3, reqs[nxt].t_arrival - (time.perf_counter() - t0))))
                else:
                    time.sleep(20e-6)
        span = max(r.t_done for r in reqs) - (min(r.t_arrival for r in reqs) if realtime else 0.0)
        lat = np.array([r.t_done - (r.t_arrival if realtime else 0.0) for r in reqs]) * 1e3
        flops = sum(2.0 * r.n ** 3 / 3.0 for r in reqs)
        return {
            "requests": len(reqs),
            "solves_per_s": len(reqs) / span,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "tflops": flops / span / 1e12,
            "span_s": span,
            "max_iters": int(max(r.iters for r in reqs)),
            # requests whose refinement stopped short of tol, or whose
            # factorization reported a numerical status: served, but flagged
            "not_converged": int(sum(r.status != "converged" for r in reqs)),
            "factor_info_nonzero": int(sum(r.info != 0 for r in reqs)),
            "batches": len(self.plan_ms),
            "plan_build_ms_mean": float(np.mean(self.plan_ms)) if self.plan_ms else 0.0,
        }


def solve_alone(req, precision="fp32", tau=2.0, tol=1e-14, max_iter=10, rows_per_wg=64):
    """The same request through a batch of one (for the alone-vs-mix check)."""
    import torch
    from . import BatchPlan
    work = [req.A.clone()]
    plan = BatchPlan(work, [req.b], tau=tau, precision=precision, rows_per_wg=rows_per_wg,
                     originals=[req.A], rhs=[req.B], tol=tol, max_iter=max_iter)
    plan.run()
    torch.cuda.synchronize()
    its, _, _ = plan.refine_results()
    x = plan.solutions[0].clone()
    plan.close()
    return x, its[0]
