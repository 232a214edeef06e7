"""Autotuner for the work-item shape of a plan.

The Gram kernels' work item is a pair's unique rows within one band of
frequencies, at most ``chunk_rows`` of them (edt_plan_opts).  The best band
and chunk depend on the survey (row counts per pair and frequency, number of
|k| classes, depth count) and on the precision, so the tuner times the
assembly on the GPU for a few candidates and keeps the fastest.  Timing uses
the library's per-kernel HIP-event timer on the launch stream.
"""
from __future__ import annotations

import json
import os
import time

import torch

from .edt import Plan

__all__ = ["candidates", "autotune"]


def candidates(survey):
    """(chunk_rows, gram_band) pairs to try; band 0 = the planner default."""
    nf = len(survey.freqs)
    bands = sorted({0, 4, 8, 16, 32, nf})
    return [(c, b) for c in (1024, 2048) for b in bands if b <= nf]


def _time_assemble(plan, vel, prec, reps):
    g64, g32 = plan.green(vel, want32=prec != "fp64")
    d = torch.zeros(plan.n_rows, 2, dtype=torch.complex128, device=plan.device)
    P, nz = plan.n_pairs, plan.nz
    out = (torch.zeros(P, nz, nz, dtype=torch.float64, device=plan.device),
           torch.empty(P, 2, nz, dtype=torch.float64, device=plan.device),
           torch.empty(P, dtype=torch.float64, device=plan.device))
    plan.assemble(g64, g32, d, prec, out=out)
    torch.cuda.synchronize()
    plan.timing(True)
    plan.timing_read()
    for _ in range(reps):
        plan.assemble(g64, g32, d, prec, out=out)
    torch.cuda.synchronize()
    t = plan.timing_read()
    plan.timing(False)
    return sum(ms for ms, _ in t.values()) / reps


def autotune(survey, prec="bf16x3", reps=3, cands=None, cache=None, log=None):
    """Return {"chunk_rows", "gram_band", "ms", "table"} for the fastest
    assembly of `survey` in precision `prec`.  With `cache` (a JSON path) a
    previous result for the same survey shape is reused."""
    key = f"{survey.dim}:{survey.n_mid}:{getattr(survey, 'n_off', 0)}:{len(survey.freqs)}:{survey.nz}:{prec}"
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            memo = json.load(fh)
        if key in memo:
            return memo[key]
    vel = torch.as_tensor(survey.vel, dtype=torch.float64, device="cuda")
    table = []
    best = None
    for chunk, band in (cands or candidates(survey)):
        t0 = time.perf_counter()
        plan = Plan(survey, chunk_rows=chunk, gram_band=band)
        ms = _time_assemble(plan, vel, prec, reps)
        row = {"chunk_rows": chunk, "gram_band": plan.info["gram_band"], "items": plan.info["n_items"],
               "ms": ms, "wall_s": time.perf_counter() - t0}
        table.append(row)
        if log:
            log(row)
        if best is None or ms < best["ms"]:
            best = dict(row)
        plan.close()
        del plan
        torch.cuda.empty_cache()
    result = {"chunk_rows": best["chunk_rows"], "gram_band": best["gram_band"], "ms": best["ms"], "table": table}
    if cache:
        memo = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                memo = json.load(fh)
        memo[key] = result
        with open(cache, "w") as fh:
            json.dump(memo, fh)
    return result
