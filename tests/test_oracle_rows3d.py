"""Pins of the oracle's 3D areal rows (paper Section 2.2; the areal geometry
the paper calls ideal, with the midpoint-wavenumber decoupling of eq. DMV).

In units of dk/2 a row of k_m index q_u and k_h index n has k_r = q_u + 2n
and k_s = q_u - 2n.  These half-grid wavenumbers are whole-grid wavenumbers
of a survey with twice the period: the N-periodic model, repeated twice along
each axis, sampled by a full-coverage periodic areal survey on the 2N x 2N
grid.  Its data transform at receiver index a = q_u + 2n and source index
b = q_u - 2n (mod 2N) is the datum of that row at +k_m, and at (-b, -a) the
datum at -k_m, times 4 (the repeated model's spectrum at an even index 2q is
four times the N-grid spectrum at q; at odd indices it vanishes).  Every row,
odd q_u and the Nyquist k_m included, is compared with brute-force
space-domain Born data.
"""
import dataclasses

import numpy as np
import pytest

from edt_inputs import make_custom, vhat
from oracle.born import born_3d
from oracle.rows import plan, kmax_of
from oracle.solve import gtables, forward


def _doubled_survey_spectrum(s, f_hz):
    """d_mid^2 DFT over receivers and sources of the brute-force areal data of
    the model repeated 2 x 2 times on the 2N x 2N periodic grid: [a, b] with
    a, b in (2N)^2 flattened (x*2N + y)."""
    N = s.n_mid
    V2 = np.tile(s.v_true, (2, 2, 1))
    D = born_3d(s.vel, s.zif, f_hz, s.eps, V2, s.d_mid, s.z, s.dz)
    M = 2 * N
    F = (s.d_mid ** 2) * np.fft.fft2(D.reshape(M, M, M, M), axes=(0, 1))
    return np.fft.fft2(F, axes=(2, 3))


@pytest.mark.parametrize("N,vel,zif", [(8, (1800.0, 2500.0), (40.0,)), (6, (2100.0, 1700.0, 2900.0), (30.0, 70.0))])
def test_every_km_row_matches_doubled_periodic_areal_born(N, vel, zif):
    s = make_custom(dim=3, N=N, Nh=N // 2, nz=3, dx=30.0, dz=25.0, freqs=(6.0, 9.0),
                    vel=vel, zif=zif, kappa=100.0, seed=7)
    pl = plan(s)
    tabs = gtables(s, pl)
    clean = forward(s, pl, vhat(s), tabs)
    M = 2 * N
    checked = odd = 0
    for fi, f in enumerate(s.freqs):
        F = _doubled_survey_spectrum(s, f)
        scale = np.max(np.abs(F))
        # data coupling to an odd model index vanish (the repeated model has none)
        ax, ay, bx, by = np.meshgrid(*(np.arange(M),) * 4, indexing="ij")
        odd_sum = ((ax + bx) % 2 == 1) | ((ay + by) % 2 == 1)
        assert np.max(np.abs(F[odd_sum])) <= 1e-12 * scale
        for p, (d0, d1) in zip(pl.pairs, clean):
            ux, uy = divmod(p.u, N)
            qx = ux if ux < (N + 1) // 2 else ux - N
            qy = uy if uy < (N + 1) // 2 else uy - N
            sel = np.nonzero(p.f == fi)[0]
            n = p.key0[sel, 1]
            nh = s.n_off
            nx = n // nh - nh // 2
            ny = n % nh - nh // 2
            ax, ay = (qx + 2 * nx) % M, (qy + 2 * ny) % M
            bx, by = (qx - 2 * nx) % M, (qy - 2 * ny) % M
            ref0 = F[ax, ay, bx, by] / 4.0
            ref1 = F[(-bx) % M, (-by) % M, (-ax) % M, (-ay) % M] / 4.0
            assert np.max(np.abs(ref0 - d0[sel]), initial=0.0) <= 1e-12 * scale
            assert np.max(np.abs(ref1 - d1[sel]), initial=0.0) <= 1e-12 * scale
            checked += sel.shape[0]
            if qx % 2 or qy % 2:
                odd += sel.shape[0]
    assert checked > 50 and odd > checked // 2


def test_doubled_survey_pin_detects_a_wrong_half_grid_wavenumber():
    """A half-grid |k_r| rounded to the whole grid (the mistake the doubled
    survey is there to catch) changes the rows of odd k_m by far more than
    the pin's tolerance."""
    from oracle.rows import row_values
    from oracle.green import green, omega
    N = 8
    s = make_custom(dim=3, N=N, Nh=N // 2, nz=3, dx=30.0, dz=25.0, freqs=(6.0,),
                    vel=(1800.0, 2500.0), zif=(40.0,), kappa=100.0, seed=7)
    pl = plan(s)
    F = _doubled_survey_spectrum(s, s.freqs[0])
    scale = np.max(np.abs(F))
    vh = vhat(s)
    dk = 2 * np.pi / (N * s.d_mid)
    worst = 0.0
    for p in pl.pairs:
        ux, uy = divmod(p.u, N)
        qx = ux if ux < (N + 1) // 2 else ux - N
        qy = uy if uy < (N + 1) // 2 else uy - N
        if not (qx % 2 or qy % 2):
            continue
        wrong = dataclasses.replace(p, kr=np.round(p.kr / dk) * dk)
        A = row_values(s, wrong, lambda fi, k: green(s.vel, s.zif, omega(s.freqs[fi], s.eps), k, s.z))
        d0 = A @ vh[p.u]
        n = p.key0[:, 1]
        nx, ny = n // s.n_off - s.n_off // 2, n % s.n_off - s.n_off // 2
        ref = F[(qx + 2 * nx) % (2 * N), (qy + 2 * ny) % (2 * N), (qx - 2 * nx) % (2 * N),
                (qy - 2 * ny) % (2 * N)] / 4.0
        worst = max(worst, np.max(np.abs(ref - d0)))
    assert worst > 1e-6 * scale


def test_rows_invariant_under_lattice_rotation_and_cut():
    N = 16
    s = make_custom(dim=3, N=N, Nh=N // 2, nz=2, dx=20.0, freqs=(9.0, 21.0),
                    vel=(2000.0, 2500.0), zif=(30.0,), seed=1, model=None)
    pl = plan(s)
    km = kmax_of(s.freqs, s.kappa, s.vel[0])
    by_u = {}
    for p in pl.pairs:
        by_u[p.u] = p
        by_u[p.u_neg] = p
        assert np.all(p.kr <= km[p.f]) and np.all(p.ks <= km[p.f])

    def sig(u):
        p = by_u[u]
        return sorted(zip(p.f.tolist(), np.round(np.minimum(p.kr, p.ks), 9).tolist(),
                          np.round(np.maximum(p.kr, p.ks), 9).tolist()))

    for u in range(N * N):
        ux, uy = divmod(u, N)
        qx = ux if ux < (N + 1) // 2 else ux - N
        qy = uy if uy < (N + 1) // 2 else uy - N
        if abs(qx) >= N // 2 - 1 or abs(qy) >= N // 2 - 1:
            continue               # rotation would leave the fftfreq window
        rx, ry = -qy, qx
        ur = (rx % N) * N + (ry % N)
        assert sig(u) == sig(ur)
    # every kept row of a k_m obeys the cut, and every (n, f) obeying it is kept
    dk = 2 * np.pi / (N * s.d_mid)
    for p in pl.pairs[:40]:
        ux, uy = divmod(p.u, N)
        qx = ux if ux < (N + 1) // 2 else ux - N
        qy = uy if uy < (N + 1) // 2 else uy - N
        cnt = 0
        for f in range(s.n_freq):
            for nx in range(-(N // 4), N // 4):
                for ny in range(-(N // 4), N // 4):
                    kr = 0.5 * dk * np.hypot(qx + 2 * nx, qy + 2 * ny)
                    ks = 0.5 * dk * np.hypot(qx - 2 * nx, qy - 2 * ny)
                    if max(kr, ks) <= km[f] * (1 - 1e-12):
                        cnt += 1
                    elif max(kr, ks) <= km[f] * (1 + 1e-12):
                        pytest.skip("tie at the cut")
        assert cnt == p.n_rows


@pytest.mark.parametrize("dim", [2, 3])
def test_subset_enumeration_lists_the_same_pairs(dim):
    """plan(s, only=...) lists exactly the chosen pairs of the full
    enumeration, row for row, with their survey indices."""
    from edt_inputs import make_custom
    if dim == 2:
        s = make_custom(N=40, nz=3, dx=12.5, freqs=(4.0, 9.0, 20.0), vel=(2100.0,), model=None)
    else:
        s = make_custom(dim=3, N=16, Nh=8, nz=3, dx=20.0, freqs=(9.0, 21.0), vel=(2000.0,), model=None)
    full = plan(s)
    pick = [0, 3, len(full.pairs) - 1]
    sub = plan(s, only=pick)
    assert sub.index == pick and full.index == list(range(len(full.pairs)))
    for i, q in zip(pick, sub.pairs):
        r = full.pairs[i]
        assert (q.u, q.u_neg) == (r.u, r.u_neg)
        for a in ("f", "kr", "ks", "key0", "key1"):
            assert np.array_equal(getattr(q, a), getattr(r, a))
