"""Pins of the oracle gradient: central finite differences of the oracle's own
forward solve, with the evanescent-cut mask held fixed (velocity changes do
not move c_top's row selection because the plan is built once)."""
import numpy as np
import pytest

from edt_inputs import make_custom
from oracle.solve import gtables, synth_data, solve
from oracle.grad import grad


@pytest.fixture(scope="module")
def case():
    s = make_custom(N=16, nz=10, dx=25.0, dz=20.0, freqs=(6.0, 9.0, 12.0),
                    vel=(1800.0, 2600.0, 2200.0), zif=(45.0, 120.0), noise_rel=0.05, seed=3)
    pl, tabs, data, _ = synth_data(s)
    rng = np.random.default_rng(0)
    T = rng.normal(size=(pl.n_km, s.nz)) + 1j * rng.normal(size=(pl.n_km, s.nz))
    V, _ = solve(s, pl, data, tabs)
    g = grad(s, pl, data, 2 * (V - T))
    return s, pl, data, T, g


def _loss(s, pl, data, T, vel=None, lr=None):
    t = gtables(s, pl, vel=vel)
    V, _ = solve(s, pl, data, t, lambda_rel=lr)
    return float(np.sum(np.abs(V - T) ** 2))


def test_grad_velocity_fd(case):
    s, pl, data, T, g = case
    for m in range(s.n_layers):
        h = 1e-6 * s.vel[m]
        vp, vm = s.vel.copy(), s.vel.copy()
        vp[m] += h
        vm[m] -= h
        fd = (_loss(s, pl, data, T, vel=vp) - _loss(s, pl, data, T, vel=vm)) / (2 * h)
        assert abs(fd - g["vel"][m]) <= 1e-4 * abs(g["vel"][m])


def test_grad_lambda_fd(case):
    s, pl, data, T, g = case
    h = 1e-6 * s.lambda_rel
    fd = (_loss(s, pl, data, T, lr=s.lambda_rel + h) - _loss(s, pl, data, T, lr=s.lambda_rel - h)) / (2 * h)
    assert abs(fd - g["lambda_rel"]) <= 1e-4 * abs(g["lambda_rel"])


def test_grad_data_fd(case):
    s, pl, data, T, g = case
    for pi, r, e in [(1, 0, 0), (3, 2, 1), (0, 1, 0), (5, 4, 1), (8, 0, 0)]:
        if pl.pairs[pi].n_rows <= r:
            continue
        for part in (1.0, 1j):
            h = 1e-6 * abs(data[pi][e][r])
            dp = [(a.copy(), b.copy()) for a, b in data]
            dm = [(a.copy(), b.copy()) for a, b in data]
            dp[pi][e][r] += h * part
            dm[pi][e][r] -= h * part
            fd = (_loss(s, pl, dp, T) - _loss(s, pl, dm, T)) / (2 * h)
            an = g["d"][pi][e][r]
            an = an.real if part == 1.0 else an.imag
            assert abs(fd - an) <= 1e-4 * max(abs(an), 1e-3 * np.max(np.abs(np.concatenate(
                [np.abs(x[0]) for x in g["d"] if x[0].size]))))
