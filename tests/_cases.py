"""Shared helpers of the GPU parity tests: oracle reference runs and error
measures.  Inputs come from edt_inputs and the oracle only."""
import numpy as np

from edt_inputs import make_custom, vhat
from oracle.rows import plan as oracle_plan
from oracle.solve import gtables, forward, noise_scale, add_noise, solve, pack


def oracle_case(s, pairs_subset=None):
    """Oracle data (packed rows) and solution for survey s."""
    pl = oracle_plan(s)
    tabs = gtables(s, pl)
    clean = forward(s, pl, vhat(s), tabs)
    scale = noise_scale(s, pl, clean)
    data = add_noise(s, pl, clean, scale)
    d_rows, off = pack(pl, data)
    V, info = solve(s, pl, data, tabs)
    return dict(pl=pl, tabs=tabs, clean=clean, data=data, d_rows=d_rows, off=off, V=V, info=info)


def rel_errors(Vg, Vo, pl):
    """Global ||dV||_F/||V||_F and worst per-pair ||dV_p|| / max(||V_p||, 1e-3 max_q ||V_q||)."""
    Vg = np.asarray(Vg)
    Vo = np.asarray(Vo)
    glob = np.linalg.norm(Vg - Vo) / max(np.linalg.norm(Vo), 1e-300)
    norms = []
    errs = []
    for p in pl.pairs:
        idx = [p.u] if p.u == p.u_neg else [p.u, p.u_neg]
        norms.append(np.linalg.norm(Vo[idx]))
        errs.append(np.linalg.norm(Vg[idx] - Vo[idx]))
    norms = np.array(norms)
    floor = 1e-3 * norms.max() if norms.size else 0.0
    per = np.array(errs) / np.maximum(np.maximum(norms, floor), 1e-300)
    return glob, float(per.max()) if per.size else 0.0


def layered_small(nz=40, N=48, nf=12, seed=11, **kw):
    """An 8-layer survey with a ragged depth count (not a multiple of 32)."""
    rng = np.random.default_rng(seed)
    vel = rng.uniform(1500, 4000, 8)
    zif = np.cumsum(rng.uniform(30, 80, 7))
    base = dict(N=N, nz=nz, dx=12.5, dz=8.0, freqs=tuple(np.linspace(3.0, 60.0, nf)), vel=tuple(vel),
                zif=tuple(zif), noise_rel=0.05, seed=seed)
    base.update(kw)
    return make_custom(**base)
