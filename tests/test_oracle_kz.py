"""Pins of the oracle's k_z-disk restriction (paper Section 3.1).

* the basis against numpy's FFT: orthonormal columns whose discrete Fourier
  transform over z vanishes outside the kept indices, and which span every
  kept mode (the projector onto them equals the FFT mask);
* the kept index set against a direct count of the disk's lattice points;
* a disk holding every k_z reduces to the unrestricted truncated SVD;
* on a survey: the solution's transform over z vanishes outside the disk, the
  normal equations hold on the kept modes at tol = 0 (checked through the
  FFT of the residual G x - c), a pair outside the disk is zero, and a model
  band-limited to the disk is recovered from noise-free data.
"""
import numpy as np
import pytest

from edt_inputs import make_custom, make_lines, vhat
from oracle.kz import kz_basis, kz_disk_radius, kz_kept, kz_tsvd_solve, pair_km2
from oracle.rows import plan, row_values
from oracle.solve import gtables, forward, synth_data, normal_equations, INFO_EMPTY
from oracle.tsvd import tsvd_gram, tsvd_solve
from oracle.lines3d import forward_lines, line_row_values, line_tables, plan_lines
from oracle.solve import add_noise, noise_scale


def _mask(nz, kept):
    m = np.zeros(nz, bool)
    for j in kept:
        m[j] = True
        m[(-j) % nz] = True
    return m


@pytest.mark.parametrize("nz,dz,km2,K", [(16, 10.0, 0.0, 0.2), (17, 10.0, 1e-3, 0.15), (32, 8.0, 4e-3, 0.3),
                                         (12, 5.0, 0.0, 10.0), (9, 5.0, 0.05, 0.2)])
def test_basis_is_the_fft_subspace(nz, dz, km2, K):
    kept = kz_kept(nz, dz, km2, K)
    F = kz_basis(nz, dz, km2, K)
    m = _mask(nz, kept)
    assert F.shape[1] == int(m.sum())
    assert np.allclose(F.T @ F, np.eye(F.shape[1]), atol=1e-13)
    Fh = np.fft.fft(F, axis=0)
    assert np.max(np.abs(Fh[~m]), initial=0.0) <= 1e-12
    # the projector F F^T is the FFT mask: it reproduces any kept mode and
    # kills every other one
    P_fft = np.real(np.fft.ifft(np.fft.fft(np.eye(nz), axis=0) * m[:, None], axis=0))
    assert np.allclose(F @ F.T, P_fft, atol=1e-13)


def test_kept_indices_count_the_disk():
    nz, dz = 40, 12.5
    dkz = 2 * np.pi / (nz * dz)
    for km2, K in [(0.0, 0.1), (0.002, 0.1), (0.02, 0.1), (0.0, 1.0)]:
        kept = kz_kept(nz, dz, km2, K)
        ref = [j for j in range(nz // 2 + 1) if np.hypot(j * dkz, np.sqrt(km2)) <= K * (1 + 1e-15)]
        assert kept == ref
    assert kz_kept(nz, dz, 0.02, 0.1) == []    # |k_m| > K: nothing kept


def test_km2_follows_the_fftfreq_order():
    s2 = make_custom(N=12, nz=5, dx=25.0, freqs=(3.0,), vel=(2000.0,))
    dk = 2 * np.pi / (12 * 25.0)
    for u in range(12):
        assert np.isclose(pair_km2(s2, u), (np.fft.fftfreq(12)[u] * 12 * dk) ** 2, rtol=1e-14)
    s3 = make_custom(dim=3, N=8, Nh=4, nz=5, dx=25.0, freqs=(3.0,), vel=(2000.0,))
    dk = 2 * np.pi / (8 * 25.0)
    f = np.fft.fftfreq(8) * 8
    for u in range(64):
        ux, uy = divmod(u, 8)
        assert np.isclose(pair_km2(s3, u), ((f[ux] * dk) ** 2 + (f[uy] * dk) ** 2), rtol=1e-14)


def test_radius():
    s = make_custom(N=8, nz=5, dx=25.0, freqs=(2.0, 5.0, 3.0), vel=(1500.0, 4000.0), zif=(500.0,))
    assert np.isclose(kz_disk_radius(s), 2.2 * 2 * np.pi * 5.0 / 1500.0, rtol=1e-15)


def _survey(**kw):
    base = dict(N=32, nz=24, dx=12.5, dz=8.0, freqs=(6.0, 17.0, 29.0, 41.0), vel=(2300.0, 3100.0),
                zif=(90.0,), noise_rel=0.05, seed=11)
    base.update(kw)
    return make_custom(**base)


def test_disk_holding_every_kz_is_the_plain_tsvd():
    s = _survey()
    pl, tabs, data, _ = synth_data(s)
    Vr, _ = kz_tsvd_solve(s, pl, data, tabs, 1e-2, K=1e3)
    V, _ = tsvd_solve(s, pl, data, tabs, 1e-2)
    assert np.max(np.abs(Vr - V)) <= 1e-9 * np.max(np.abs(V))


def test_restricted_solution_lives_in_the_disk_and_solves_the_restricted_system():
    s = _survey()
    pl, tabs, data, _ = synth_data(s)
    K = 0.7 * kz_disk_radius(s)
    V, info = kz_tsvd_solve(s, pl, data, tabs, 0.0, K)
    nz = s.nz
    n_out = 0
    for p, (d0, d1), inf in zip(pl.pairs, data, info):
        kept = kz_kept(nz, s.dz, pair_km2(s, p.u), K)
        m = _mask(nz, kept)
        x = inf["x"]
        if not kept:
            n_out += 1
            assert not np.any(x)
            continue
        assert np.max(np.abs(np.fft.fft(x, axis=1)[:, ~m]), initial=0.0) <= 1e-10 * np.max(np.abs(x))
        if p.n_rows == 0:
            continue
        A = row_values(s, p, tabs.lookup)
        G, c, _ = normal_equations(A, d0, d1)
        r = np.fft.fft(x @ G - c, axis=1)[:, m]
        assert np.max(np.abs(r)) <= 1e-8 * np.max(np.abs(np.fft.fft(c, axis=1)[:, m]))
    assert n_out > 0


def test_band_limited_model_is_recovered():
    # nz = 8 keeps every restricted pair well conditioned (kappa(F^T G F) < 4e6)
    s = _survey(N=16, nz=8, noise_rel=0.0, freqs=tuple(np.linspace(8, 40, 7)), vel=(1700.0, 2400.0),
                zif=(40.0,), kappa=100.0, lambda_rel=0.0, seed=5)
    pl = plan(s)
    tabs = gtables(s, pl)
    K = kz_disk_radius(s)
    # project the seeded model onto the disk, pair by pair
    vh = vhat(s)
    vb = np.zeros_like(vh)
    for p in pl.pairs:
        F = kz_basis(s.nz, s.dz, pair_km2(s, p.u), K)
        for u in {p.u, p.u_neg}:
            vb[u] = F @ (F.T @ vh[u].real) + 1j * (F @ (F.T @ vh[u].imag))
    assert np.linalg.norm(vb - vh) > 0.01 * np.linalg.norm(vh)    # the disk does cut the model
    clean = forward(s, pl, vb, tabs)
    V, info = kz_tsvd_solve(s, pl, clean, tabs, 0.0, K)
    assert np.max(np.abs(V - vb)) <= 1e-7 * np.max(np.abs(vb))
    assert all(i["info"] != INFO_EMPTY for i in info)


def test_km2_of_the_line_survey_follows_both_fftfreq_orders():
    """u = ux N_y + c: |(k_m, k_y)|^2 with its own spacing on each axis
    (N_x != N_y, so a transposed index fails)."""
    Nx, Ny, dx, dy = 10, 6, 25.0, 40.0
    s = make_lines(Nx=Nx, Ny=Ny, dx=dx, dy=dy, nz=5, freqs=(3.0,), vel=(2000.0,), model="zero")
    fx, fy = np.fft.fftfreq(Nx) * Nx, np.fft.fftfreq(Ny) * Ny
    for u in range(Nx * Ny):
        ux, c = divmod(u, Ny)
        want = (fx[ux] * 2 * np.pi / (Nx * dx)) ** 2 + (fy[c] * 2 * np.pi / (Ny * dy)) ** 2
        assert np.isclose(pair_km2(s, u), want, rtol=1e-14)


def _line_case():
    s = make_lines(Nx=12, Ny=5, dx=25.0, dy=40.0, nz=16, dz=10.0, freqs=(6.0, 14.0, 23.0), vel=(1900.0, 2700.0),
                   zif=(40.0,), kappa=1.0, noise_rel=0.05, seed=8)
    pl = plan_lines(s)
    tab = line_tables(s)
    clean = forward_lines(s, pl, vhat(s), tab)
    return s, pl, tab, add_noise(s, pl, clean, noise_scale(s, pl, clean))


def test_line_disk_holding_every_kz_is_the_plain_tsvd():
    s, pl, tab, data = _line_case()
    Vr, _ = kz_tsvd_solve(s, pl, data, tab, 1e-2, K=1e3)
    V = np.zeros_like(Vr)
    for p, (d0, d1) in zip(pl.pairs, data):
        if not p.n_rows:
            continue
        G, c, _ = normal_equations(line_row_values(s, p, tab), d0, d1)
        x, _, _ = tsvd_gram(G, c, 1e-2)
        if p.self_conjugate:
            x[1] = 0.0
        V[p.u] = x[0] + 1j * x[1]
        if not p.self_conjugate:
            V[p.u_neg] = x[0] - 1j * x[1]
    assert np.max(np.abs(Vr - V)) <= 1e-9 * np.max(np.abs(V))


def test_line_restricted_solution_lives_in_the_disk():
    s, pl, tab, data = _line_case()
    K = 0.6 * kz_disk_radius(s)
    V, info = kz_tsvd_solve(s, pl, data, tab, 0.0, K)
    nz = s.nz
    n_out = n_part = 0
    for p, (d0, d1), inf in zip(pl.pairs, data, info):
        kept = kz_kept(nz, s.dz, pair_km2(s, p.u), K)
        m = _mask(nz, kept)
        x = inf["x"]
        if not kept:
            n_out += 1
            assert not np.any(x)
            continue
        n_part += 0 < len(kept) < nz // 2 + 1
        assert np.max(np.abs(np.fft.fft(x, axis=1)[:, ~m]), initial=0.0) <= 1e-10 * max(np.max(np.abs(x)), 1e-300)
        if p.n_rows == 0:
            continue
        G, c, _ = normal_equations(line_row_values(s, p, tab), d0, d1)
        r = np.fft.fft(x @ G - c, axis=1)[:, m]
        assert np.max(np.abs(r)) <= 1e-8 * np.max(np.abs(np.fft.fft(c, axis=1)[:, m]))
    assert n_out > 0 and n_part > 0
