"""Pins of the oracle's shot-record and model transforms (paper Section 2.1).

* brute-force space-domain Born data (oracle.born, a direct sum with no
  transform) go through shots_to_rows to the wavenumber-domain rows of the
  seeded model (odd and even N, with and without the evanescent cut);
* a single plane-wave shot record lands on exactly the row of its (a, b) key,
  with value dx N^2;
* model_from_spectrum inverts the spectrum that defines the seeded model, in
  2D and 3D.
"""
import numpy as np
import pytest

from edt_inputs import make_custom, vhat
from oracle.born import born_2d
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
