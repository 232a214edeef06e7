"""Pins of the oracle's 3D areal rows (paper Section 2.2; the areal geometry
the paper calls ideal, with the midpoint-wavenumber decoupling of eq. DMV).

In units of dk/2 a row of k_m index q_u and k_h index n has k_r = q_u + 2n
and k_s = q_u - 2n.  For an even q_u these are whole-grid wavenumbers
a = q_u/2 + n, b = q_u/2 - n, and the row must reproduce the datum (a, b) of a
full-coverage periodic areal survey computed by brute force in space.  Odd
q_u rows use the same formula; they are checked by the lattice symmetries.
"""
import numpy as np
import pytest

from edt_inputs import make_custom, vhat
from oracle.born import born_3d
from oracle.rows import plan, kmax_of
from oracle.solve import gtables, forward


def test_even_km_rows_match_periodic_areal_born():
    N = 8
    s = make_custom(dim=3, N=N, Nh=N // 2, nz=3, dx=30.0, dz=25.0, freqs=(6.0, 9.0),
                    vel=(1800.0, 2500.0), zif=(40.0,), kappa=100.0, seed=7)
    pl = plan(s)
    tabs = gtables(s, pl)
    clean = forward(s, pl, vhat(s), tabs)
    checked = 0
    for fi, f in enumerate(s.freqs):
        D = born_3d(s.vel, s.zif, f, s.eps, s.v_true, s.d_mid, s.z, s.dz)
        F = (s.d_mid ** 2) * np.fft.fft2(D.reshape(N, N, N, N), axes=(0, 1))
        F = np.fft.fft2(F, axes=(2, 3))
        scale = np.max(np.abs(F))
        for p, (d0, d1) in zip(pl.pairs, clean):
            ux, uy = divmod(p.u, N)
            qx = ux if ux < (N + 1) // 2 else ux - N
            qy = uy if uy < (N + 1) // 2 else uy - N
            if qx % 2 or qy % 2 or qx == -N // 2 or qy == -N // 2:
                continue
            sel = np.nonzero(p.f == fi)[0]
            n = p.key0[sel, 1]
            nh = s.n_off
            nx = n // nh - nh // 2
            ny = n % nh - nh // 2
            for sign, d in ((1, d0), (-1, d1)):
                ax = (sign * qx // 2 + nx) % N
                ay = (sign * qy // 2 + ny) % N
                bx = (sign * qx // 2 - nx) % N
                by = (sign * qy // 2 - ny) % N
                ref = F[ax, ay, bx, by]
                assert np.max(np.abs(ref - d[sel])) <= 1e-12 * scale
                checked += sel.shape[0]
    assert checked > 50


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
