"""Pins of the oracle's finite-aperture operator (paper Section 2.1, eq. M).

* brute-force space-domain Born records, windowed in full offset, go through
  the record transform to exactly the windowed rows S A applied to the seeded
  model, at +k_m and at -k_m (the window convention, the discrete sinc and
  the pairing; odd and even N);
* the discrete sinc is real and its circulant is an orthogonal projector;
* the windowed Gram lies below the full one (A^H S A <= A^H A), and a window
  holding every offset gives the plain damped solve;
* survey of parallel lines: brute-force line Born records, each line windowed
  in full offset, go through the line record transform to exactly the
  windowed line rows applied to the model (odd and even grids), the data form
  of the window agrees, and the Gram and full-window properties hold.
"""
import numpy as np
import pytest

from edt_inputs import make_custom, make_lines, vhat
from oracle.aperture import aperture_data, aperture_rows, aperture_solve, offset_window, window_kernel
from oracle.born import born_2d, born_lines
from oracle.lines3d import forward_lines, line_row_values, line_tables, plan_lines, solve_lines
from oracle.solve import add_noise, noise_scale
from oracle.rows import plan, row_values
from oracle.shots import shots_to_rows
from oracle.solve import gtables, synth_data, solve


@pytest.mark.parametrize("N,b", [(12, 60.0), (11, 40.0), (16, 70.0)])
def test_windowed_born_records_give_the_windowed_rows(N, b):
    s = make_custom(N=N, nz=4, dx=25.0, dz=20.0, freqs=(5.0, 9.0), vel=(1800.0, 2600.0), zif=(45.0,),
                    kappa=100.0, seed=3)
    pl = plan(s)
    tabs = gtables(s, pl)
    w = offset_window(s, b)
    assert 0 < w.sum() < N
    R = np.arange(N)
    W = w[(R[:, None] - R[None, :]) % N]                   # w(R - S)
    D = np.stack([born_2d(s.vel, s.zif, f, s.eps, s.v_true, s.d_mid, s.z, s.dz) for f in s.freqs]) * W
    rows = shots_to_rows(s, pl, D)
    Sm = window_kernel(w)
    vh = vhat(s)
    scale = max(np.max(np.abs(d0)) for d0, _ in rows if d0.size)
    for p, (d0, d1) in zip(pl.pairs, rows):
        B = aperture_rows(s, p, row_values(s, p, tabs.lookup), Sm)
        assert np.max(np.abs(B @ vh[p.u] - d0)) <= 1e-12 * scale
        assert np.max(np.abs(B @ vh[p.u_neg] - d1)) <= 1e-12 * scale
    # the data form of the window: the unwindowed records' rows, windowed by
    # aperture_data, are the windowed records' rows
    D0 = np.stack([born_2d(s.vel, s.zif, f, s.eps, s.v_true, s.d_mid, s.z, s.dz) for f in s.freqs])
    wd = aperture_data(s, pl, shots_to_rows(s, pl, D0), b)
    for (a0, a1), (d0, d1) in zip(wd, rows):
        assert np.max(np.abs(a0 - d0)) <= 1e-12 * scale
        assert np.max(np.abs(a1 - d1)) <= 1e-12 * scale


def test_discrete_sinc_is_a_real_projector():
    s = make_custom(N=20, nz=3, dx=10.0, freqs=(5.0,), vel=(2000.0,))
    Sm = window_kernel(offset_window(s, 35.0))
    assert np.max(np.abs(Sm.imag)) <= 1e-15
    N = Sm.shape[0]
    n = np.arange(N)
    C = Sm.real[(n[:, None] - n[None, :]) % N]
    assert np.allclose(C @ C, C, atol=1e-14)
    assert np.allclose(C, C.T, atol=1e-15)


def test_windowed_gram_is_below_the_full_one_and_full_window_is_plain():
    s = make_custom(N=24, nz=6, dx=12.5, dz=8.0, freqs=(6.0, 17.0, 29.0), vel=(2300.0, 3100.0), zif=(30.0,),
                    noise_rel=0.05, seed=11, lambda_rel=1e-3)
    pl, tabs, data, _ = synth_data(s)
    Sm = window_kernel(offset_window(s, 40.0))
    for p in pl.pairs:
        if not p.n_rows:
            continue
        A = row_values(s, p, tabs.lookup)
        G = (A.conj().T @ A).real
        Gw = (A.conj().T @ aperture_rows(s, p, A, Sm)).real
        assert np.min(np.linalg.eigvalsh(G - Gw)) >= -1e-12 * np.max(np.abs(G))
        assert np.min(np.linalg.eigvalsh(Gw)) >= -1e-12 * np.max(np.abs(G))
    V, _ = aperture_solve(s, pl, data, tabs, b_max=1e6)
    Vo, _ = solve(s, pl, data, tabs)
    assert np.max(np.abs(V - Vo)) <= 1e-10 * np.max(np.abs(Vo))


def _line_records(s, W=None):
    D = np.stack([np.transpose(born_lines(s.vel, s.zif, f, s.eps, s.v_true, s.d_mid, s.d_line, s.z, s.dz),
                               (2, 0, 1)) for f in s.freqs])
    return D if W is None else D * W[None, None]


@pytest.mark.parametrize("Nx,Ny,b", [(8, 6, 40.0), (7, 5, 35.0)])
def test_windowed_line_born_records_give_the_windowed_line_rows(Nx, Ny, b):
    """No evanescent cut: the cut drops quadrature terms the brute-force
    records keep."""
    s = make_lines(Nx=Nx, Ny=Ny, dx=30.0, dy=45.0, nz=3, dz=25.0, freqs=(6.0, 9.0), vel=(1800.0, 2500.0),
                   zif=(40.0,), kappa=100.0, seed=5)
    pl = plan_lines(s)
    tab = line_tables(s)
    w = offset_window(s, b)
    assert 0 < w.sum() < Nx
    R = np.arange(Nx)
    W = w[(R[:, None] - R[None, :]) % Nx]                  # w(R - S), every line
    rows = shots_to_rows(s, pl, _line_records(s, W))
    Sm = window_kernel(w)
    vh = vhat(s)
    scale = max(np.max(np.abs(d0)) for d0, _ in rows if d0.size)
    n = 0
    for p, (d0, d1) in zip(pl.pairs, rows):
        if not p.n_rows:
            continue
        B = aperture_rows(s, p, line_row_values(s, p, tab), Sm)
        assert np.max(np.abs(B @ vh[p.u] - d0)) <= 1e-12 * scale
        assert np.max(np.abs(B @ vh[p.u_neg] - d1)) <= 1e-12 * scale
        n += p.n_rows
    assert n > 0
    wd = aperture_data(s, pl, shots_to_rows(s, pl, _line_records(s)), b)
    for (a0, a1), (d0, d1) in zip(wd, rows):
        assert np.max(np.abs(a0 - d0), initial=0) <= 1e-12 * scale
        assert np.max(np.abs(a1 - d1), initial=0) <= 1e-12 * scale


def test_windowed_line_gram_is_below_the_full_one_and_full_window_is_plain():
    s = make_lines(Nx=12, Ny=5, dx=25.0, dy=40.0, nz=6, dz=12.0, freqs=(6.0, 14.0, 23.0), vel=(1900.0, 2700.0),
                   zif=(40.0,), kappa=1.0, noise_rel=0.05, seed=8)
    pl = plan_lines(s)
    tab = line_tables(s)
    clean = forward_lines(s, pl, vhat(s), tab)
    data = add_noise(s, pl, clean, noise_scale(s, pl, clean))
    Sm = window_kernel(offset_window(s, 60.0))
    for p in pl.pairs:
        if not p.n_rows:
            continue
        A = line_row_values(s, p, tab)
        G = (A.conj().T @ A).real
        Gw = (A.conj().T @ aperture_rows(s, p, A, Sm)).real
        assert np.min(np.linalg.eigvalsh(G - Gw)) >= -1e-12 * np.max(np.abs(G))
        assert np.min(np.linalg.eigvalsh(Gw)) >= -1e-12 * np.max(np.abs(G))
    V, _ = aperture_solve(s, pl, data, tab, b_max=1e6)
    Vo, _ = solve_lines(s, pl, data, tab)
    assert np.max(np.abs(V - Vo)) <= 1e-10 * np.max(np.abs(Vo))
