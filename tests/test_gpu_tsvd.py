"""GPU: the paper's truncated-SVD solve (edt_tsvd) against the oracle's
eigen-decomposition (oracle.tsvd), pair by pair.

The truncation is discontinuous where an eigenvalue of a pair's Gram meets the
threshold sigma^2: pairs with an eigenvalue within a relative 1e-6 of sigma^2
have no well-defined answer and are left out (and counted).  Every other pair
must match to the FP64 bar, 1e-10 relative, unless the truncated problem's own
conditioning allows two FP64 computations to differ by more: its forward error
is of order u (lambda_max / lambda_min,kept + lambda_max / gap), u the unit
roundoff and gap the distance of the nearest eigenvalue from sigma^2, so the
bar of a pair is max(1e-10, 100 u (that sum)).  The run prints the worst error
and how many pairs are within 1e-10.
"""
import inspect

import numpy as np
import pytest

from edt_inputs import make_config, make_custom
from oracle.tsvd import tsvd_solve
from tests._cases import oracle_case, layered_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")

GAP = 1e-6


def _cases():
    return {
        "cfg1": lambda: make_config(1),
        "layered-nz40": lambda: layered_small(),
        "layered-nz200": lambda: layered_small(nz=200, N=32, nf=6, seed=3),
        "homogeneous": lambda: make_custom(N=32, nz=33, dx=12.5, dz=8.0, freqs=(6.0, 17.0, 29.0, 41.0),
                                           vel=(2300.0,), zif=(), noise_rel=0.05, seed=11),
        "3d-small": lambda: make_custom(dim=3, N=12, Nh=6, nz=37, dx=25.0, dz=10.0,
                                        freqs=(8.0, 14.0, 20.0), vel=(1800.0, 2500.0, 2100.0),
                                        zif=(60.0, 200.0), noise_rel=0.05, seed=5),
    }


def _gpu_tsvd(s, r, tol, max_iter=None):
    """max_iter None: the binding's default, the one bench.py times."""
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    g64, _ = p.green(vel, want32=False)
    d = torch.from_numpy(r["d_rows"]).cuda()
    gram, rhs, _ = p.assemble(g64, None, d, "fp64")
    kw = {} if max_iter is None else {"max_iter": max_iter}
    x, v, info, iters = p.tsvd(gram, rhs, tol, **kw)
    torch.cuda.synchronize()
    return v.cpu().numpy(), info.cpu().numpy(), iters.cpu().numpy()


@pytest.mark.parametrize("tol", [1e-2, 1e-3])
@pytest.mark.parametrize("name", list(_cases()))
def test_tsvd_matches_the_oracle(name, tol):
    s = _cases()[name]()
    r = oracle_case(s)
    Vo, info_o = tsvd_solve(s, r["pl"], r["data"], r["tabs"], tol)
    # the binding's default step limit (64): every pair away from the
    # threshold converges well inside it
    v, info, iters = _gpu_tsvd(s, r, tol)
    default_iter = inspect.signature(E.Plan.tsvd).parameters["max_iter"].default
    nv = np.linalg.norm(Vo)
    u = np.finfo(np.float64).eps / 2
    checked, ambiguous, tight, within, worst = 0, 0, 0, 0, 0.0
    for q, (p, io) in enumerate(zip(r["pl"].pairs, info_o)):
        idx = [p.u] if p.u == p.u_neg else [p.u, p.u_neg]
        if p.n_rows == 0:
            assert info[q] == -1 and not np.any(v[idx])
            continue
        w, t2 = io["eig"], io["tau2"]
        gap = np.min(np.abs(w - t2))
        if gap <= GAP * t2:
            ambiguous += 1
            continue
        assert info[q] == 0, (name, q, info[q], iters[q])
        assert iters[q] < default_iter, (name, q, int(iters[q]))
        kept = w[w >= t2]
        lmax = w.max()
        kappa = lmax / kept.min() if kept.size else 0.0
        bar = max(1e-10, 100 * u * (kappa + lmax / gap))
        tight += bar == 1e-10
        ref = Vo[idx]
        err = np.linalg.norm(v[idx] - ref) / max(np.linalg.norm(ref), 1e-3 * nv)
        assert err <= bar, (name, tol, q, err, bar, int(iters[q]))
        checked += 1
        within += err <= 1e-10
        worst = max(worst, err)
    assert checked >= 0.9 * (checked + ambiguous) and checked > 0, (checked, ambiguous)
    print(f"{name} tol {tol}: {checked} pairs checked, {ambiguous} ambiguous; bar 1e-10 for {tight}; "
          f"error <= 1e-10 for {within}, worst {worst:.2e}; sign steps max {int(iters.max())}")


def test_tsvd_without_truncation_recovers_the_model():
    """tol = 0 on a full-rank noise-free survey: the least-squares solution is
    the model itself."""
    s = make_custom(N=16, nz=6, dx=20.0, dz=15.0, freqs=tuple(np.linspace(8, 40, 9)),
                    vel=(1700.0, 2400.0), zif=(40.0,), kappa=100.0, lambda_rel=0.0, noise_rel=0.0, seed=5)
    r = oracle_case(s)
    v, info, iters = _gpu_tsvd(s, r, 0.0, max_iter=150)
    Vo, _ = tsvd_solve(s, r["pl"], r["clean"], r["tabs"], 0.0)
    assert np.all(info == 0)
    assert np.linalg.norm(v - Vo) <= 1e-9 * np.linalg.norm(Vo)


def test_tsvd_reports_an_unconverged_sign_iteration():
    s = layered_small()
    r = oracle_case(s)
    v, info, iters = _gpu_tsvd(s, r, 1e-2, max_iter=3)
    nonempty = np.array([p.n_rows > 0 for p in r["pl"].pairs])
    assert np.all(iters[nonempty] == 3)
    assert np.all(info[nonempty] == -2)   # EDT_INFO_NOCONV
