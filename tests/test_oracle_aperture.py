"""Pins of the oracle's finite-aperture operator (paper Section 2.1, eq. M).

* brute-force space-domain Born records, windowed in full offset, go through
  the record transform to exactly the windowed rows S A applied to the seeded
  model, at +k_m and at -k_m (the window convention, the discrete sinc and
  the pairing; odd and even N);
* the discrete sinc is real and its circulant is an orthogonal projector;
* the windowed Gram lies below the full one (A^H S A <= A^H A), and a window
  holding every offset gives the plain damped solve.
"""
import numpy as np
import pytest

from edt_inputs import make_custom, vhat
from oracle.aperture import aperture_data, aperture_rows, aperture_solve, offset_window, window_kernel
from oracle.born import born_2d
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
