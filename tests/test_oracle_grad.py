"""Pins of the oracle gradient: central finite differences of the oracle's own
forward solve, with the evanescent-cut mask held fixed (velocity changes do
not move c_top's row selection because the plan is built once); on the 2D line
and on the survey of parallel lines (grad_lines)."""
import numpy as np
import pytest

from edt_inputs import make_custom, make_lines, vhat
from oracle.solve import add_noise, gtables, noise_scale, synth_data, solve
from oracle.grad import grad, grad_lines
from oracle.lines3d import forward_lines, line_tables, plan_lines, solve_lines


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


@pytest.fixture(scope="module")
def line_case():
    s = make_lines(Nx=8, Ny=5, dx=30.0, dy=45.0, nz=8, dz=20.0, freqs=(6.0, 11.0, 15.0),
                   vel=(1800.0, 2600.0, 2200.0), zif=(45.0, 110.0), kappa=1.0, noise_rel=0.05, seed=4)
    pl = plan_lines(s)
    tab = line_tables(s)
    clean = forward_lines(s, pl, vhat(s), tab)
    data = add_noise(s, pl, clean, noise_scale(s, pl, clean))
    rng = np.random.default_rng(1)
    T = rng.normal(size=(pl.n_km, s.nz)) + 1j * rng.normal(size=(pl.n_km, s.nz))
    V, _ = solve_lines(s, pl, data, tab)
    g = grad_lines(s, pl, data, 2 * (V - T))
    return s, pl, data, T, g


def _line_loss(s, pl, data, T, vel=None, lr=None):
    V, _ = solve_lines(s, pl, data, line_tables(s, vel), lambda_rel=lr)
    return float(np.sum(np.abs(V - T) ** 2))


def test_line_grad_velocity_fd(line_case):
    s, pl, data, T, g = line_case
    for m in range(s.n_layers):
        h = 1e-6 * s.vel[m]
        vp, vm = s.vel.copy(), s.vel.copy()
        vp[m] += h
        vm[m] -= h
        fd = (_line_loss(s, pl, data, T, vel=vp) - _line_loss(s, pl, data, T, vel=vm)) / (2 * h)
        assert abs(fd - g["vel"][m]) <= 1e-4 * abs(g["vel"][m]), (m, fd, g["vel"][m])


def test_line_grad_lambda_fd(line_case):
    s, pl, data, T, g = line_case
    h = 1e-6 * s.lambda_rel
    fd = (_line_loss(s, pl, data, T, lr=s.lambda_rel + h)
          - _line_loss(s, pl, data, T, lr=s.lambda_rel - h)) / (2 * h)
    assert abs(fd - g["lambda_rel"]) <= 1e-4 * abs(g["lambda_rel"])


def test_line_grad_data_fd(line_case):
    s, pl, data, T, g = line_case
    big = np.max(np.abs(np.concatenate([x[0] for x in g["d"] if x[0].size])))
    n = 0
    for pi in range(0, len(pl.pairs), 5):
        if pl.pairs[pi].n_rows == 0:
            continue
        for e in (0, 1):
            for part in (1.0, 1j):
                h = 1e-6 * abs(data[pi][e][0])
                dp = [(a.copy(), b.copy()) for a, b in data]
                dm = [(a.copy(), b.copy()) for a, b in data]
                dp[pi][e][0] += h * part
                dm[pi][e][0] -= h * part
                fd = (_line_loss(s, pl, dp, T) - _line_loss(s, pl, dm, T)) / (2 * h)
                an = g["d"][pi][e][0]
                an = an.real if part == 1.0 else an.imag
                assert abs(fd - an) <= 1e-4 * max(abs(an), 1e-3 * big)
                n += 1
    assert n >= 8
