"""Autotuner for the batched factorization used by the solve server.

Two launch-shape choices are measured rather than guessed:
  * rows per strong-RRQR workgroup (64 or 128) for each size class -- fewer,
    fuller workgroups shorten each pivot step's cross-workgroup exchange but
    lengthen its local work;
  * the largest batch the server forms -- bigger batches amortise launches
    over more systems but make every system wait for the batch's largest.
Each candidate is timed with device events on saturated synthetic batches of
the class's sizes; the fastest wins.  Results are plain dicts (JSON-able).
"""
from __future__ import annotations

import json

import numpy as np

DEFAULT_CLASSES = ((64, 512), (544, 1024), (1056, 2048))


def _batch_ms(sizes, rows_per_wg, precision, seed, trials):
    import torch
    from . import BatchPlan
    dev = torch.device("cuda")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    mats = [torch.randn(n, n, generator=g, dtype=torch.float64, device=dev) for n in sizes]
    rhs = [torch.randn(n, 1, generator=g, dtype=torch.float64, device=dev) for n in sizes]
    work = [m.clone() for m in mats]
    plan = BatchPlan(work, [min(32, n // 4) for n in sizes], precision=precision,
                     rows_per_wg=rows_per_wg, originals=mats, rhs=rhs, tol=1e-14, max_iter=10)
    plan.run()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(trials):
        for w, m in zip(work, mats):
            w.copy_(m)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.run()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    plan.close()
    return best


def tune(classes=DEFAULT_CLASSES, batch=16, batch_options=(8, 16, 32), precision="fp32",
         trials=2, seed=1234, step=32):
    """Returns {"rows_per_wg": [[n_max, value], ...], "max_batch": m, "timings": {...}}."""
    rng = np.random.default_rng(seed)
    out = {"rows_per_wg": [], "timings": {}}
    for lo, hi in classes:
        sizes = [int(v) for v in rng.choice(np.arange(lo, hi + 1, step), size=batch)]
        t = {rpw: _batch_ms(sizes, rpw, precision, seed, trials) for rpw in (64, 128)}
        out["timings"]["%d-%d" % (lo, hi)] = t
        out["rows_per_wg"].append([hi, min(t, key=t.get)])
    rpw_of = rows_per_wg_fn(out)
    allsizes = [int(v) for v in rng.choice(np.arange(classes[0][0], classes[-1][1] + 1, step),
                                            size=max(batch_options) * 2)]
    tb = {}
    for mb in batch_options:
        ms = 0.0
        for i in range(0, len(allsizes), mb):
            chunk = allsizes[i:i + mb]
            ms += _batch_ms(chunk, rpw_of(max(chunk)), precision, seed + i, 1)
        tb[mb] = len(allsizes) / (ms * 1e-3)        # systems per second, one slot
    out["timings"]["max_batch_solves_per_s"] = tb
    out["max_batch"] = max(tb, key=tb.get)
    return out


def rows_per_wg_fn(tuning):
    table = sorted(tuning["rows_per_wg"])

    def f(n):
        for hi, v in table:
            if n <= hi:
                return int(v)
        return int(table[-1][1])
    return f


def save(tuning, path):
    with open(path, "w") as fh:
        json.dump(tuning, fh, indent=1, default=str)


def load(path):
    with open(path) as fh:
        t = json.load(fh)
    t["timings"] = t.get("timings", {})
    return t
