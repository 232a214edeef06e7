"""Pins of the oracle's decoupled problems (paper Section 2.1, eqs. Born,
Dkmh, DMV, M, VSym, Split) and of its damped least-squares solve.

* brute-force space-domain Born data on a tiny periodic line equals, datum for
  datum, the wavenumber-domain rows times the model's DFT (indexing, pairing,
  constants);
* the +/-k_m row symmetry and the evanescent cut, by direct enumeration;
* the Tikhonov solve against numpy's lstsq on the stacked system and against
  SVD filter factors (different algorithms for the same minimiser);
* exact recovery of the model from noise-free data without damping;
* invariance under a common scaling of rows and data (relative damping);
* the real-valuedness of the recovered model (eq. VSym).
"""
import numpy as np
import pytest

from edt_inputs import make_custom, vhat, noise
from oracle.born import born_2d
from oracle.rows import plan, row_values, kmax_of
from oracle.solve import (gtables, forward, synth_data, solve, normal_equations,
                          solve_pair, INFO_EMPTY, pack)


def _small(**kw):
    base = dict(N=12, nz=5, dx=25.0, dz=20.0, freqs=(5.0, 7.0), vel=(1800.0, 2600.0),
                zif=(45.0,), kappa=100.0, seed=3)
    base.update(kw)
    return make_custom(**base)


@pytest.mark.parametrize("N,freqs,kappa", [(12, (7.0,), 100.0), (11, (5.0, 9.0), 100.0),
                                           (16, (6.0, 11.0), 1.0)])
def test_periodic_born_identity(N, freqs, kappa):
    s = _small(N=N, freqs=freqs, kappa=kappa, vel=(1800.0, 2600.0, 2100.0), zif=(45.0, 70.0))
    pl = plan(s)
    tabs = gtables(s, pl)
    clean = forward(s, pl, vhat(s), tabs)
    for fi, f in enumerate(s.freqs):
        D = born_2d(s.vel, s.zif, f, s.eps, s.v_true, s.d_mid, s.z, s.dz)
        F = s.d_mid * np.fft.fft2(D)
        scale = np.max(np.abs(F))
        for p, (d0, d1) in zip(pl.pairs, clean):
            sel = p.f == fi
            e0 = F[p.key0[sel, 0], p.key0[sel, 1]]
            e1 = F[p.key1[sel, 0], p.key1[sel, 1]]
            assert np.max(np.abs(e0 - d0[sel]), initial=0) <= 1e-12 * scale
            assert np.max(np.abs(e1 - d1[sel]), initial=0) <= 1e-12 * scale
    if kappa > 10:   # no cut: every (a, b) datum belongs to exactly one row slot
        nrows = sum(p.n_rows * (1 if p.self_conjugate else 2) for p in pl.pairs)
        assert nrows == N * N * len(freqs)


def test_rows_by_direct_enumeration_and_cut():
    s = make_custom(N=40, nz=4, dx=12.5, freqs=(4.0, 9.0, 20.0), vel=(2100.0, 3000.0),
                    zif=(30.0,), seed=1)
    pl = plan(s)
    N = s.n_mid
    dk = 2 * np.pi / (N * s.d_mid)
    km = kmax_of(s.freqs, s.kappa, s.vel[0])
    for p in pl.pairs:
        for u, keys in ((p.u, p.key0), (p.u_neg, p.key1)):
            # every datum (f, a, b) with a + b = u and both |k| within the cut
            want = set()
            for f in range(s.n_freq):
                for a in range(N):
                    b = (u - a) % N
                    qa = a if a < N // 2 else a - N
                    qb = b if b < N // 2 else b - N
                    if abs(qa) * dk <= km[f] and abs(qb) * dk <= km[f]:
                        want.add((f, a, b))
            got = set(zip(p.f.tolist(), keys[:, 0].tolist(), keys[:, 1].tolist()))
            if u == p.u_neg and u != p.u:
                continue
            if p.u == p.u_neg and N % 2 == 0 and p.u == N // 2:
                # the Nyquist problem: partner rows are rows of the same problem
                assert got <= want
                continue
            assert got == want
        # the +k_m and -k_m data of a row share |k_r|, |k_s| (M even in k_m)
        qa1 = np.where(p.key1[:, 0] < N // 2, p.key1[:, 0], p.key1[:, 0] - N)
        qb1 = np.where(p.key1[:, 1] < N // 2, p.key1[:, 1], p.key1[:, 1] - N)
        assert np.array_equal(np.sort(np.stack([np.abs(qa1) * dk, np.abs(qb1) * dk]), 0),
                              np.sort(np.stack([p.kr, p.ks]), 0))
        # k_h = k_r - k_s is the same for the row and its partner (mod N)
        kh0 = (p.key0[:, 0] - p.key0[:, 1]) % N
        kh1 = (p.key1[:, 0] - p.key1[:, 1]) % N
        assert np.array_equal(kh0, kh1)


def _system(seed=0, R=60, nz=8):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(R, nz)) + 1j * rng.normal(size=(R, nz))
    d0 = rng.normal(size=R) + 1j * rng.normal(size=R)
    d1 = rng.normal(size=R) + 1j * rng.normal(size=R)
    return A, d0, d1


class _P:
    n_rows = 60
    self_conjugate = False


class _S:
    nz = 8
    lambda_rel = 0.3


def test_tikhonov_equals_stacked_lstsq_and_svd_filter():
    A, d0, d1 = _system()
    x, info, lam, tr = solve_pair(_S, _P, A, d0, d1)
    Ah = np.vstack([A.real, A.imag])
    assert np.isclose(tr, np.sum(np.abs(A) ** 2))
    for j, b in enumerate([(d0 + d1) / 2, (d0 - d1) / 2j]):
        bh = np.concatenate([b.real, b.imag])
        M = np.vstack([Ah, np.sqrt(lam) * np.eye(8)])
        rhs = np.concatenate([bh, np.zeros(8)])
        ref = np.linalg.lstsq(M, rhs, rcond=None)[0]
        assert np.max(np.abs(x[j] - ref)) <= 1e-10 * np.max(np.abs(ref))
        U, sv, Vt = np.linalg.svd(Ah, full_matrices=False)
        ref2 = Vt.T @ ((sv / (sv ** 2 + lam)) * (U.T @ bh))
        assert np.max(np.abs(x[j] - ref2)) <= 1e-10 * np.max(np.abs(ref2))


def test_scale_invariance_under_relative_damping():
    A, d0, d1 = _system(3)
    x1 = solve_pair(_S, _P, A, d0, d1)[0]
    x2 = solve_pair(_S, _P, 7.5e3 * A, 7.5e3 * d0, 7.5e3 * d1)[0]
    assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(x1))


def test_exact_recovery_without_damping():
    # enough frequencies and wavenumbers that every pair has full column rank
    s = make_custom(N=16, nz=6, dx=20.0, dz=15.0, freqs=tuple(np.linspace(8, 40, 9)),
                    vel=(1700.0, 2400.0), zif=(40.0,), kappa=100.0, lambda_rel=0.0, seed=5)
    pl = plan(s)
    tabs = gtables(s, pl)
    vh = vhat(s)
    clean = forward(s, pl, vh, tabs)
    V, info = solve(s, pl, clean, tabs)
    assert np.max(np.abs(V - vh)) <= 1e-8 * np.max(np.abs(vh))


def test_recovered_model_is_real_and_symmetric():
    s = make_custom(N=20, nz=7, freqs=(6.0, 12.0, 18.0), vel=(2000.0, 2800.0), zif=(30.0,),
                    noise_rel=0.05, seed=9)
    pl, tabs, data, _ = synth_data(s)
    V, info = solve(s, pl, data, tabs)
    N = s.n_mid
    for u in range(N):
        assert np.allclose(V[(-u) % N], np.conj(V[u]), rtol=0, atol=1e-14 * np.max(np.abs(V)))
    v = np.fft.ifft(V, axis=0)
    assert np.max(np.abs(v.imag)) <= 1e-14 * np.max(np.abs(v.real))


def test_empty_pairs_give_zero():
    # low frequencies and a long line: large |k_m| has no propagating rows
    s = make_custom(N=64, nz=5, dx=25.0, freqs=(2.0, 3.0), vel=(2500.0,), seed=2)
    pl, tabs, data, _ = synth_data(s)
    V, info = solve(s, pl, data, tabs)
    empty = [p for p in pl.pairs if p.n_rows == 0]
    assert empty, "expected some empty pairs"
    for p, inf in zip(pl.pairs, info):
        if p.n_rows == 0:
            assert inf["info"] == INFO_EMPTY
            assert not np.any(V[p.u]) and not np.any(V[p.u_neg])


def test_self_conjugate_nyquist_duplicate_rows():
    # at u = N/2 the partner of row a is row a + N/2 of the same problem with
    # identical A: averaging the two data on duplicated rows gives the same
    # minimiser as solving once per distinct row (damping is relative)
    s = make_custom(N=16, nz=5, freqs=(9.0, 14.0), vel=(1600.0,), kappa=100.0, noise_rel=0.1,
                    seed=4)
    pl, tabs, data, _ = synth_data(s)
    p = [q for q in pl.pairs if q.u == 8][0]
    d0, d1 = data[8]
    A = row_values(s, p, tabs.lookup)
    x = solve_pair(s, p, A, d0, d1)[0]
    # rows a and a+N/2 coincide; keep one of each, data = average of the pair
    N = s.n_mid
    a = p.key0[:, 0]
    keep = np.array([ai < N // 2 for ai in a])
    mate = {}
    for r in range(p.n_rows):
        mate[(int(p.f[r]), int(a[r]))] = r
    avg = np.array([0.5 * (d0[r] + d0[mate[(int(p.f[r]), (int(a[r]) + N // 2) % N)]])
                    for r in np.nonzero(keep)[0]])
    G, c, tr = normal_equations(A[keep], avg, avg)
    lam = s.lambda_rel * tr / s.nz
    ref = np.linalg.solve(G + lam * np.eye(s.nz), c[0])
    assert np.max(np.abs(x[0] - ref)) <= 1e-11 * np.max(np.abs(ref))
    assert not np.any(x[1])


def test_noise_is_counter_based_and_normalised():
    n1 = noise(7, np.arange(5), np.arange(5) * 3, 11)
    n2 = noise(7, np.arange(5)[::-1], (np.arange(5) * 3)[::-1], 11)[::-1]
    assert np.array_equal(n1, n2)
    big = noise(1, 0, np.arange(200000))
    assert abs(np.mean(np.abs(big) ** 2) - 1.0) < 0.02
    assert abs(np.mean(big)) < 0.01


def test_pack_layout():
    s = _small()
    pl, tabs, data, _ = synth_data(s)
    d, off = pack(pl, data)
    assert off[-1] == d.shape[0]
    for i, (d0, d1) in enumerate(data):
        assert np.array_equal(d[off[i]:off[i + 1], 0], d0)
        assert np.array_equal(d[off[i]:off[i + 1], 1], d1)
