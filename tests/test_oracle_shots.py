"""Pins of the oracle's shot-record and model transforms (paper Section 2.1).

* brute-force space-domain Born data (oracle.born, a direct sum with no
  transform) go through shots_to_rows to the wavenumber-domain rows of the
  seeded model (odd and even N, with and without the evanescent cut);
* a single plane-wave shot record lands on exactly the row of its (a, b) key,
  with value dx N^2;
* 3D areal (Section 2.2): brute-force Born records of the doubled periodic
  survey (the N-periodic model repeated 2 x 2 times on the 2N x 2N grid) go
  to the rows of every k_m, odd components included; a plane-wave record of
  the doubled survey lands on the rows whose half-grid wavenumbers are its
  own, with value d_mid^2 (2N)^4 / 4;
* 3D parallel lines (Section 2.2): brute-force Born records of the line
  survey [f, line, receiver, source] go to the rows (no evanescent cut: the
  cut drops terms of the rows' quadrature that full Born data keep); a
  plane-wave record lands on the rows keyed by its (a, b, c), at +k and at
  the -k partner, with value d_mid N_y N_x^2;
* model_from_spectrum inverts the spectrum that defines the seeded model, in
  2D, 3D and on the survey of parallel lines; one spectral line of the line
  survey gives its closed-form cosine.
"""
import numpy as np
import pytest

from edt_inputs import make_custom, make_lines, vhat
from oracle.born import born_2d, born_3d, born_lines
from oracle.rows import plan
from oracle.shots import model_from_spectrum, shots_to_rows
from oracle.solve import gtables, forward


@pytest.mark.parametrize("N,kappa", [(12, 100.0), (11, 100.0), (16, 1.0)])
def test_born_shot_records_give_the_rows(N, kappa):
    s = make_custom(N=N, nz=5, dx=25.0, dz=20.0, freqs=(5.0, 9.0), vel=(1800.0, 2600.0, 2100.0),
                    zif=(45.0, 70.0), kappa=kappa, seed=3)
    pl = plan(s)
    tabs = gtables(s, pl)
    clean = forward(s, pl, vhat(s), tabs)
    D = np.stack([born_2d(s.vel, s.zif, f, s.eps, s.v_true, s.d_mid, s.z, s.dz) for f in s.freqs])
    rows = shots_to_rows(s, pl, D)
    scale = max(np.max(np.abs(d0)) for d0, _ in clean if d0.size)
    for (d0, d1), (e0, e1) in zip(clean, rows):
        assert np.max(np.abs(e0 - d0), initial=0) <= 1e-12 * scale
        assert np.max(np.abs(e1 - d1), initial=0) <= 1e-12 * scale


def test_plane_wave_lands_on_its_row():
    N = 10
    s = make_custom(N=N, nz=4, dx=20.0, freqs=(6.0,), vel=(2000.0,), kappa=100.0)
    pl = plan(s)
    a0, b0 = 3, 8
    n = np.arange(N)
    D = np.exp(2j * np.pi * (a0 * n[:, None] + b0 * n[None, :]) / N)[None]
    rows = shots_to_rows(s, pl, D)
    hits = 0
    for p, (d0, d1) in zip(pl.pairs, rows):
        for keys, d in ((p.key0, d0), (p.key1, d1)):
            for (a, b), v in zip(keys, d):
                want = s.d_mid * N * N if (a, b) == (a0, b0) else 0.0
                assert abs(v - want) <= 1e-10 * s.d_mid * N * N
                hits += (a, b) == (a0, b0)
    assert hits >= 1


def test_model_from_its_spectrum():
    s2 = make_custom(N=24, nz=7, dx=12.5, freqs=(5.0,), vel=(2000.0,), seed=2)
    assert np.allclose(model_from_spectrum(s2, vhat(s2)), s2.v_true, rtol=0, atol=1e-13)
    s3 = make_custom(dim=3, N=8, Nh=4, nz=5, dx=25.0, freqs=(3.0,), vel=(2000.0,), seed=4)
    assert np.allclose(model_from_spectrum(s3, vhat(s3)), s3.v_true, rtol=0, atol=1e-13)
    sl = make_lines(Nx=9, Ny=6, nz=4, freqs=(3.0,), vel=(2000.0,), seed=6)
    assert np.allclose(model_from_spectrum(sl, vhat(sl)), sl.v_true, rtol=0, atol=1e-13)


def test_line_model_of_one_spectral_line():
    """One k_m entry (ux, c) = (2, 5) with value w at depth 1, its partner
    (-2, -5) with conj(w): the model is 2 Re(w e^{2 pi i (2 x / N_x + 5 y / N_y)})
    / (N_x N_y) at depth 1 and zero elsewhere."""
    Nx, Ny, nz = 9, 7, 3
    sl = make_lines(Nx=Nx, Ny=Ny, nz=nz, freqs=(3.0,), vel=(2000.0,), model="zero")
    w = 0.7 - 1.3j
    V = np.zeros((Nx * Ny, nz), np.complex128)
    V[2 * Ny + 5, 1] = w
    V[(Nx - 2) * Ny + (Ny - 5), 1] = np.conj(w)
    m = model_from_spectrum(sl, V)
    x, y = np.arange(Nx)[:, None], np.arange(Ny)[None, :]
    want = 2.0 * np.real(w * np.exp(2j * np.pi * (2 * x / Nx + 5 * y / Ny))) / (Nx * Ny)
    assert m.shape == (Nx, Ny, nz)
    assert np.max(np.abs(m[:, :, 1] - want)) <= 1e-15
    assert not m[:, :, 0].any() and not m[:, :, 2].any()


def _signed(u, N):
    return u if u < (N + 1) // 2 else u - N


@pytest.mark.parametrize("N,vel,zif", [(8, (1800.0, 2500.0), (40.0,)), (5, (2100.0, 1700.0, 2900.0), (30.0, 70.0))])
def test_areal_born_records_give_the_rows(N, vel, zif):
    s = make_custom(dim=3, N=N, Nh=N // 2 + 1, nz=3, dx=30.0, dz=25.0, freqs=(6.0, 9.0), vel=vel, zif=zif,
                    kappa=100.0, seed=11)
    pl = plan(s)
    clean = forward(s, pl, vhat(s), gtables(s, pl))
    M = 2 * N
    V2 = np.tile(s.v_true, (2, 2, 1))
    D = np.stack([born_3d(s.vel, s.zif, f, s.eps, V2, s.d_mid, s.z, s.dz).reshape(M, M, M, M)
                  for f in s.freqs])
    rows = shots_to_rows(s, pl, D)
    scale = max(np.max(np.abs(d0)) for d0, _ in clean if d0.size)
    odd = 0
    for p, (d0, d1), (e0, e1) in zip(pl.pairs, clean, rows):
        assert np.max(np.abs(e0 - d0), initial=0) <= 1e-12 * scale
        assert np.max(np.abs(e1 - d1), initial=0) <= 1e-12 * scale
        ux, uy = divmod(p.u, N)
        odd += (ux % 2 or uy % 2) * d0.size
    assert odd > 0


def test_areal_plane_wave_lands_on_its_rows():
    N = 6
    M = 2 * N
    s = make_custom(dim=3, N=N, Nh=N, nz=2, dx=20.0, freqs=(7.0,), vel=(2000.0,), kappa=100.0)
    pl = plan(s)
    a0, b0 = (3, 1), (7, 5)      # receiver and source wavenumber indices on the 2N grid (a - b = 4n)
    g = np.arange(M)
    ph = (a0[0] * g[:, None, None, None] + a0[1] * g[None, :, None, None]
          + b0[0] * g[None, None, :, None] + b0[1] * g[None, None, None, :])
    D = np.exp(2j * np.pi * ph / M)[None]
    rows = shots_to_rows(s, pl, D)
    peak = s.d_mid ** 2 * M ** 4 / 4.0
    hits = 0
    for p, (d0, d1) in zip(pl.pairs, rows):
        ux, uy = divmod(p.u, N)
        q = np.array([_signed(ux, N), _signed(uy, N)])
        n = p.key0[:, 1]
        nv = np.stack([n // s.n_off - s.n_off // 2, n % s.n_off - s.n_off // 2], axis=1)
        r0, s0 = (q + 2 * nv) % M, (q - 2 * nv) % M           # +k_m datum
        r1, s1 = (-s0) % M, (-r0) % M                         # -k_m datum
        for r, sv, d in ((r0, s0, d0), (r1, s1, d1)):
            at = np.all(r == a0, axis=1) & np.all(sv == b0, axis=1)
            want = np.where(at, peak, 0.0)
            assert np.max(np.abs(d - want), initial=0) <= 1e-10 * peak
            hits += int(at.sum())
    assert hits >= 1


@pytest.mark.parametrize("Nx,Ny,kappa", [(8, 6, 100.0), (7, 5, 100.0)])
def test_line_survey_born_records_give_the_rows(Nx, Ny, kappa):
    from oracle.lines3d import forward_lines, line_tables, plan_lines
    s = make_lines(Nx=Nx, Ny=Ny, dx=30.0, dy=45.0, nz=3, dz=25.0, freqs=(6.0, 9.0), vel=(1800.0, 2500.0),
                   zif=(40.0,), kappa=kappa, seed=5)
    pl = plan_lines(s)
    clean = forward_lines(s, pl, vhat(s), line_tables(s))
    D = np.stack([np.transpose(born_lines(s.vel, s.zif, f, s.eps, s.v_true, s.d_mid, s.d_line, s.z, s.dz),
                               (2, 0, 1)) for f in s.freqs])
    rows = shots_to_rows(s, pl, D)
    scale = max(np.max(np.abs(d0)) for d0, _ in clean if d0.size)
    n = 0
    for (d0, d1), (e0, e1) in zip(clean, rows):
        assert np.max(np.abs(e0 - d0), initial=0) <= 1e-12 * scale
        assert np.max(np.abs(e1 - d1), initial=0) <= 1e-12 * scale
        n += d0.size
    assert n > 0


def test_line_survey_plane_wave_lands_on_its_rows():
    from oracle.lines3d import plan_lines
    Nx, Ny = 10, 6
    s = make_lines(Nx=Nx, Ny=Ny, dx=20.0, dy=30.0, nz=2, freqs=(7.0,), vel=(2000.0,), zif=(), kappa=100.0)
    pl = plan_lines(s)
    a0, b0, c0 = 3, 8, 2
    j, n = np.arange(Ny), np.arange(Nx)
    D = np.exp(2j * np.pi * (c0 * j[:, None, None] / Ny + a0 * n[None, :, None] / Nx
                             + b0 * n[None, None, :] / Nx))[None]
    rows = shots_to_rows(s, pl, D)
    peak = s.d_mid * Ny * Nx * Nx
    hits = 0
    for p, (d0, d1) in zip(pl.pairs, rows):
        for keys, d in ((p.key0, d0), (p.key1, d1)):
            at = (keys[:, 0] == a0) & (keys[:, 1] == b0) & (keys[:, 2] == c0)
            assert np.max(np.abs(d - np.where(at, peak, 0.0)), initial=0) <= 1e-10 * peak
            hits += int(at.sum())
    assert hits >= 1
