"""Autotuner for the work-item shapes of a plan.

Three plan options shape the work of a pass (edt_plan_opts):
* ``chunk_rows`` and ``gram_band``: a Gram work item is a pair's unique rows
  within one band of frequencies, at most chunk_rows of them.  Wider bands
  mean fewer, longer items (less partial-tile traffic, a shorter reduce) but,
  for the FP16x3 Gram, one power-of-two scale over a wider range of row
  magnitudes, which can cost refinement sweeps.
* ``resid_group``: frequencies per residual work item of the refinement
  sweeps (the table slab an item reads against the partials it writes).

The best shapes depend on the survey (rows per pair and frequency, number of
|k| classes, depths) and on the precision, so the tuner times the whole pass
-- green -> assemble -> solve with the refinement of the mixed paths -- on the
GPU for each candidate, with the library's per-kernel HIP-event timer on the
launch stream, and keeps the fastest.  It tunes the Gram shape first, then
the residual grouping with that Gram shape.  Every candidate meets the same
refinement tolerance; the planner's default shape is always a candidate, so
the tuned plan is never slower than the default on the tuning data.

Results are cached in a JSON table keyed by the survey and the precision: the
file named by the environment variable EDT_TUNE_CACHE, else the table shipped
with the package (``tuned_shapes.json``), which ``shapes_for`` reads.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import torch

from .edt import Plan

__all__ = ["candidates", "survey_key", "cache_path", "shapes_for", "autotune", "DEFAULT_SHAPE"]

DEFAULT_SHAPE = {"chunk_rows": 0, "gram_band": 0, "resid_group": 0}
_HERE = os.path.dirname(os.path.abspath(__file__))
PACKAGE_TABLE = os.path.join(_HERE, "tuned_shapes.json")


def survey_key(survey, prec: str) -> str:
    """Key of a survey and precision in the cache: a digest of everything that
    fixes the rows and the work (geometry, frequencies, depths, layers, cut)."""
    fields = [int(survey.dim), int(survey.n_mid), float(survey.d_mid), int(getattr(survey, "n_off", 0)),
              float(getattr(survey, "d_off", 0.0)), [float(f) for f in survey.freqs], float(survey.eps),
              int(survey.nz), float(survey.z0), float(survey.dz), float(survey.kappa),
              [float(v) for v in survey.vel], [float(z) for z in survey.zif]]
    h = hashlib.sha1(json.dumps(fields).encode()).hexdigest()[:16]
    return f"{survey.dim}d-N{survey.n_mid}-nz{survey.nz}-nf{len(survey.freqs)}-{h}:{prec}"


def cache_path() -> str:
    return os.environ.get("EDT_TUNE_CACHE") or PACKAGE_TABLE


def _read(path):
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def shapes_for(survey, prec: str) -> dict:
    """The cached shape (chunk_rows, gram_band, resid_group) of this survey and
    precision: from EDT_TUNE_CACHE if set and holding it, else from the
    package's table, else the planner's default (all 0)."""
    key = survey_key(survey, prec)
    for path in (os.environ.get("EDT_TUNE_CACHE"), PACKAGE_TABLE):
        memo = _read(path)
        if key in memo:
            r = memo[key]
            return {k: int(r[k]) for k in DEFAULT_SHAPE}
    return dict(DEFAULT_SHAPE)


def candidates(survey):
    """Gram shapes (chunk_rows, gram_band) to try, then residual groupings;
    0 = the planner's default."""
    nf = len(survey.freqs)
    bands = sorted({0, 4, 8, 16, 32, nf})
    gram = [(c, b) for c in (0, 1024) for b in bands if b <= nf]
    resid = sorted({0, 1, 4, 8})
    return gram, [g for g in resid if g <= nf]


def _synthetic_rows(plan, vel, seed=7):
    """Data rows for the tuning passes: the Born forward map of a seeded
    random model spectrum plus 5% complex noise (torch's generator), so the
    refinement does the work real data need."""
    gen = torch.Generator(device="cuda").manual_seed(seed)
    g64, _ = plan.green(vel, want32=False)
    v = torch.complex(torch.randn(plan.n_km, plan.nz, generator=gen, device="cuda", dtype=torch.float64),
                      torch.randn(plan.n_km, plan.nz, generator=gen, device="cuda", dtype=torch.float64))
    d = plan.forward(g64, v)
    if plan.n_rows:
        rdt = torch.float32 if d.dtype == torch.complex64 else torch.float64
        sc = 0.05 * float(d.abs().amax()) / np.sqrt(2.0)
        d += sc * torch.complex(torch.randn(d.shape, generator=gen, device="cuda", dtype=rdt),
                                torch.randn(d.shape, generator=gen, device="cuda", dtype=rdt))
    return d


def _time_pass(plan, vel, d_rows, prec, lambda_rel, refine_tol, max_refine, reps):
    """ms per pass (sum of the library's kernel times) and the mean sweeps."""
    from .pipeline import Pipeline
    pipe = Pipeline(plan, vel, d_rows, lambda_rel, prec=prec, refine_tol=refine_tol, max_refine=max_refine)
    pipe.step()
    torch.cuda.synchronize()
    plan.timing(True)
    plan.timing_read()
    for _ in range(reps):
        pipe.step()
    torch.cuda.synchronize()
    t = plan.timing_read()
    plan.timing(False)
    ms = sum(v for v, _ in t.values()) / reps
    sweeps = float(pipe.steps.float().mean()) if prec != "fp64" else 0.0
    bad = int(((pipe.info != 0) & (pipe.info != -1)).sum())
    return ms, sweeps, bad


def autotune(survey, prec="fp16x3", reps=3, lambda_rel=None, refine_tol=3e-6, max_refine=8, data="c128",
             d_rows=None, cache=None, write=True, log=None):
    """Tune the shapes of `survey` in precision `prec`; returns {"chunk_rows",
    "gram_band", "resid_group", "ms", "default_ms", "table"}.  d_rows: data
    rows of the default plan's layout (every shape has the same row order);
    default: seeded synthetic rows.  cache: a JSON path (default
    cache_path()); with write the result is stored there under survey_key."""
    lam = float(survey.lambda_rel if lambda_rel is None else lambda_rel)
    vel = torch.as_tensor(np.asarray(survey.vel, np.float64), device="cuda")
    base = Plan(survey, data=data)
    d = d_rows if d_rows is not None else _synthetic_rows(base.upload(), vel)
    table = []

    def run(shape):
        t0 = time.perf_counter()
        plan = Plan(survey, data=data, **shape)
        ms, sweeps, bad = _time_pass(plan, vel, d, prec, lam, refine_tol, max_refine, reps)
        row = dict(shape)
        row.update({"gram_band_used": plan.info["gram_band"], "resid_group_used": plan.info["resid_group"],
                    "items": plan.info["n_items"], "ms": ms, "sweeps_mean": sweeps, "failed_pairs": bad,
                    "wall_s": time.perf_counter() - t0})
        plan.close()
        del plan
        torch.cuda.empty_cache()
        table.append(row)
        if log:
            log(row)
        return row

    gram_c, resid_c = candidates(survey)
    rows = [run({"chunk_rows": c, "gram_band": b, "resid_group": 0}) for c, b in gram_c]
    ok = [r for r in rows if r["failed_pairs"] == 0] or rows
    best_g = min(ok, key=lambda r: r["ms"])
    rows2 = [best_g] + [run({"chunk_rows": best_g["chunk_rows"], "gram_band": best_g["gram_band"],
                             "resid_group": g}) for g in resid_c if g != 0]
    ok2 = [r for r in rows2 if r["failed_pairs"] == 0] or rows2
    best = min(ok2, key=lambda r: r["ms"])
    default_ms = next(r["ms"] for r in table if all(r[k] == 0 for k in DEFAULT_SHAPE))
    result = {k: int(best[k]) for k in DEFAULT_SHAPE}
    result.update({"ms": best["ms"], "default_ms": default_ms, "prec": prec, "table": table})
    path = cache or cache_path()
    if write and path:
        memo = _read(path)
        memo[survey_key(survey, prec)] = result
        with open(path, "w") as fh:
            json.dump(memo, fh, indent=1, sort_keys=True)
    return result
