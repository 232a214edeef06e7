"""Pins of the oracle's 3D line-survey rows (paper Section 2.2, eq. Born3D and
the decoupled 3D equation with its k_h'' integral).

* Brute-force space-domain Born data of a periodic survey of parallel lines
  (every source to every receiver of its own line), transformed over
  receiver, source and line, equal the rows applied to the model spectrum,
  datum for datum at +k and at the -k partner (odd and even N_x, N_y, two
  layers, no cut): the sum over the line wavenumbers, its weight and the
  pairing.
* Dropping the sum's weight 1/L_y, taking the datum at line index -c, or
  leaving the source's line wavenumber q - c unwrapped fails that check.
* The evanescent cut: every kept term obeys it, and a row is kept iff a term
  is; with the cut, the partner's rows have the same value (the sum over the
  periodic line grid re-indexes).
* The solve: on a noise-free survey without damping and with full column
  rank, the normal equations of the rows recover the model spectrum.
"""
import numpy as np
import pytest
import scipy.linalg

from edt_inputs import make_lines, vhat
from oracle.born import born_lines
from oracle.lines3d import forward_lines, line_row_values, line_tables, plan_lines
from oracle.solve import normal_equations


def _spectrum(s, f_hz):
    D = born_lines(s.vel, s.zif, f_hz, s.eps, s.v_true, s.d_mid, s.d_line, s.z, s.dz)
    return s.d_mid * np.fft.fftn(D, axes=(0, 1, 2))


@pytest.mark.parametrize("Nx,Ny,dx,dy", [(8, 6, 30.0, 45.0), (7, 5, 25.0, 40.0), (6, 4, 40.0, 40.0)])
def test_rows_match_brute_force_line_survey(Nx, Ny, dx, dy):
    s = make_lines(Nx=Nx, Ny=Ny, dx=dx, dy=dy, nz=3, dz=25.0, freqs=(6.0, 9.0), vel=(1800.0, 2500.0),
                   zif=(40.0,), kappa=100.0, seed=3)
    pl = plan_lines(s)
    tab = line_tables(s)
    d = forward_lines(s, pl, vhat(s), tab)
    checked = 0
    for fi, f in enumerate(s.freqs):
        F = _spectrum(s, f)
        scale = np.max(np.abs(F))
        for p, (d0, d1) in zip(pl.pairs, d):
            sel = np.nonzero(p.f == fi)[0]
            k0, k1 = p.key0[sel], p.key1[sel]
            assert np.max(np.abs(F[k0[:, 0], k0[:, 1], k0[:, 2]] - d0[sel]), initial=0.0) <= 1e-12 * scale
            assert np.max(np.abs(F[k1[:, 0], k1[:, 1], k1[:, 2]] - d1[sel]), initial=0.0) <= 1e-12 * scale
            checked += sel.size
    # no cut: every (f, a) of every pair is a row
    assert checked == s.n_freq * Nx * len(pl.pairs)


def test_plausible_mistakes_fail_the_pin():
    """The sum's weight 1/L_y dropped, the datum taken at line index -c, or the
    source's line wavenumber q - c left unwrapped (its non-negative index mod
    N_y instead of the signed one) moves the data far outside the pin's
    tolerance.  (q + c in place of q - c is no mistake: the sum over the whole
    periodic grid is even in c.)"""
    from oracle.green import green, omega
    s = make_lines(Nx=8, Ny=6, dx=30.0, dy=45.0, nz=3, dz=25.0, freqs=(7.0,), vel=(1800.0, 2500.0),
                   zif=(40.0,), kappa=100.0, seed=4)
    pl = plan_lines(s)
    tab = line_tables(s)
    vh = vhat(s)
    F = _spectrum(s, s.freqs[0])
    scale = np.max(np.abs(F))
    Nx, Ny, Ly = s.n_mid, s.n_line, s.n_line * s.d_line
    dkx, dky = 2 * np.pi / (Nx * s.d_mid), 2 * np.pi / Ly
    w = omega(s.freqs[0], s.eps)
    worst_w = worst_c = worst_u = 0.0
    for p in pl.pairs:
        ref0 = F[p.key0[:, 0], p.key0[:, 1], p.key0[:, 2]]
        A = line_row_values(s, p, tab)
        worst_w = max(worst_w, np.max(np.abs((A * Ly) @ vh[p.u] - ref0)))
        worst_c = max(worst_c, np.max(np.abs(A @ vh[p.u] - F[p.key0[:, 0], p.key0[:, 1], (-p.key0[:, 2]) % Ny])))
        qc = p.c if p.c < (Ny + 1) // 2 else p.c - Ny
        B = np.zeros_like(A)
        for r in range(p.n_rows):
            for q in range(-(Ny // 2), Ny - Ny // 2):
                pq = (q - qc) % Ny
                gr = green(s.vel, s.zif, w, np.array([np.hypot(p.a[r] * dkx, q * dky)]), s.z)[0]
                gs = green(s.vel, s.zif, w, np.array([np.hypot(p.b[r] * dkx, pq * dky)]), s.z)[0]
                B[r] += gr * gs
        B *= w * w * s.dz / Ly
        worst_u = max(worst_u, np.max(np.abs(B @ vh[p.u] - ref0)))
    assert worst_w > 1e-3 * scale and worst_c > 1e-6 * scale and worst_u > 1e-6 * scale


def test_cut_and_partner_symmetry():
    s = make_lines(Nx=12, Ny=8, dx=20.0, dy=30.0, nz=4, dz=15.0, freqs=(9.0, 21.0), vel=(2000.0, 2600.0),
                   zif=(30.0,), kappa=1.0, seed=1)
    pl = plan_lines(s)
    tab = line_tables(s)
    Nx, Ny = s.n_mid, s.n_line
    dkx, dky = 2 * np.pi / (Nx * s.d_mid), 2 * np.pi / (Ny * s.d_line)
    n_rows = 0
    for p in pl.pairs:
        qc = p.c if p.c < (Ny + 1) // 2 else p.c - Ny
        for r in range(p.n_rows):
            km = pl.kmax[p.f[r]]
            kept = 0
            for bit in range(Ny):
                q = bit - Ny // 2
                pq = (q - qc) % Ny
                pq = pq if pq < (Ny + 1) // 2 else pq - Ny
                ok = np.hypot(p.a[r] * dkx, q * dky) <= km * (1 + 1e-12) and np.hypot(p.b[r] * dkx, pq * dky) <= km * (1 + 1e-12)
                strict = np.hypot(p.a[r] * dkx, q * dky) <= km * (1 - 1e-12) and np.hypot(p.b[r] * dkx, pq * dky) <= km * (1 - 1e-12)
                bitset = bool((int(p.mask[r]) >> bit) & 1)
                if bitset:
                    assert ok
                    kept += 1
                else:
                    assert not strict
            assert kept > 0
        n_rows += p.n_rows
    assert n_rows > 0
    # the partner (-u, -c) row (-b, -a) of a kept row, summed with the same
    # rule over its own terms, has the same value (the cut is symmetric and
    # the sum over the periodic line grid re-indexes)
    for p in [q for q in pl.pairs if not q.self_conjugate and q.n_rows][:6]:
        A = line_row_values(s, p, tab)
        c = p.u_neg % Ny
        qc = c if c < (Ny + 1) // 2 else c - Ny
        for r in range(p.n_rows):
            km2 = pl.kmax[p.f[r]] ** 2
            a2, b2 = -p.b[r], -p.a[r]
            acc = np.zeros(s.nz, np.complex128)
            for bit in range(Ny):
                qq = bit - Ny // 2
                pq = (qq - qc) % Ny
                pq = pq if pq < (Ny + 1) // 2 else pq - Ny
                kr2 = (a2 * dkx) * (a2 * dkx) + (qq * dky) * (qq * dky)
                ks2 = (b2 * dkx) * (b2 * dkx) + (pq * dky) * (pq * dky)
                if kr2 <= km2 and ks2 <= km2:
                    acc += tab[p.f[r], abs(a2), abs(qq)] * tab[p.f[r], abs(b2), abs(pq)]
            w = 2 * np.pi * s.freqs[p.f[r]] + 1j * s.eps
            assert np.max(np.abs(w * w * s.dz / (Ny * s.d_line) * acc - A[r])) <= 1e-13 * np.max(np.abs(A[r]))


def test_noise_free_full_rank_survey_recovers_the_model():
    s = make_lines(Nx=6, Ny=4, dx=30.0, dy=40.0, nz=3, dz=25.0, freqs=tuple(np.linspace(6.0, 30.0, 7)),
                   vel=(1800.0, 2500.0), zif=(40.0,), kappa=100.0, seed=5)
    pl = plan_lines(s)
    tab = line_tables(s)
    vh = vhat(s)
    d = forward_lines(s, pl, vh, tab)
    for p, (d0, d1) in zip(pl.pairs, d):
        A = line_row_values(s, p, tab)
        G, c, _ = normal_equations(A, d0, d1)
        x = scipy.linalg.solve(G, c.T, assume_a="pos").T
        ref = vh[p.u]
        if p.self_conjugate:
            assert np.max(np.abs(x[0] - ref.real)) <= 1e-8 * np.max(np.abs(ref))
        else:
            assert np.max(np.abs(x[0] + 1j * x[1] - ref)) <= 1e-8 * np.max(np.abs(ref))
