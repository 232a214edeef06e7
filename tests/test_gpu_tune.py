"""GPU: the work-item autotuner (paper_0905_0238_amd.tune).

The tuner times whole passes (green -> assemble -> solve, with the
refinement of the mixed paths) over candidate shapes and keeps the fastest;
the planner's default shape is a candidate, so the choice is never slower
than the default on the tuning data.  The tuned plan must still meet the
oracle's bars (FP64 <= 1e-10, mixed <= 1e-6), and the cached table must give
the shape back.
"""
import numpy as np
import pytest

from tests._cases import oracle_case, rel_errors, layered_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")
from paper_0905_0238_amd import tune  # noqa: E402


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("fp16x3", 1e-6)])
def test_tuned_shape_is_valid_no_slower_and_meets_parity(tmp_path, monkeypatch, prec, bar):
    s = layered_small(nz=72, N=48, nf=12, seed=21)
    cache = tmp_path / "shapes.json"
    monkeypatch.setenv("EDT_TUNE_CACHE", str(cache))
    res = tune.autotune(s, prec=prec, reps=2)
    gram_c, resid_c = tune.candidates(s)
    assert (res["chunk_rows"], res["gram_band"]) in gram_c and res["resid_group"] in resid_c
    assert res["ms"] <= res["default_ms"]
    assert all(r["failed_pairs"] == 0 for r in res["table"])
    print(f"{prec}: tuned {res['chunk_rows']}/{res['gram_band']}/{res['resid_group']} {res['ms']:.3f} ms, "
          f"default {res['default_ms']:.3f} ms, {len(res['table'])} candidates", flush=True)
    # the cache gives the shape back, keyed on survey and precision
    shape = tune.shapes_for(s, prec)
    assert shape == {k: res[k] for k in tune.DEFAULT_SHAPE}
    other = "bf16x3" if prec != "bf16x3" else "fp16x3"
    assert tune.shapes_for(s, other) == tune.DEFAULT_SHAPE
    # parity of the tuned plan
    r = oracle_case(s)
    p = E.Plan(s, **shape)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    out = p.run(vel, torch.from_numpy(r["d_rows"]).cuda(), s.lambda_rel, prec=prec, refine_tol=3e-6)
    torch.cuda.synchronize()
    g, per = rel_errors(out["v"].cpu().numpy(), r["V"], r["pl"])
    assert g <= bar and per <= bar, (g, per)
