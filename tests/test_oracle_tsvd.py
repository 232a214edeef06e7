"""Pins of the oracle's truncated-SVD solve (paper Section 3.1).

* against the SVD of the stacked real rows [Re A; Im A] (numpy.linalg.svd on
  the rows, a different algorithm from the Gram eigen-decomposition), with the
  tolerance placed between two singular values;
* without truncation on a full-rank system: numpy's lstsq on the rows;
* a tolerance above every singular value gives zero;
* invariance under a common scaling of rows and data (relative tolerance);
* on a survey: exact recovery from noise-free data without truncation, empty
  pairs at zero, a real model (eq. VSym).
"""
import numpy as np
import pytest

from edt_inputs import make_custom, vhat
from oracle.rows import plan
from oracle.solve import gtables, forward, synth_data, INFO_EMPTY
from oracle.tsvd import tsvd_gram, tsvd_pair, tsvd_solve, tsvd_threshold


def _system(seed=0, R=60, nz=8):
    rng = np.random.default_rng(seed)
    # rows with a spread of singular values: random complex rows times a
    # geometric column scaling
    A = (rng.normal(size=(R, nz)) + 1j * rng.normal(size=(R, nz))) * np.logspace(0, -4, nz)
    d0 = rng.normal(size=R) + 1j * rng.normal(size=R)
    d1 = rng.normal(size=R) + 1j * rng.normal(size=R)
    return A, d0, d1


class _P:
    n_rows = 60
    self_conjugate = False


class _S:
    nz = 8


@pytest.mark.parametrize("seed,cut", [(0, 3), (1, 5), (2, 1)])
def test_tsvd_equals_row_svd_truncation(seed, cut):
    A, d0, d1 = _system(seed)
    Ah = np.vstack([A.real, A.imag])
    U, sv, Vt = np.linalg.svd(Ah, full_matrices=False)   # descending
    # sigma between singular values cut-1 and cut (a clear gap on this scale)
    sigma = np.sqrt(sv[cut - 1] * sv[cut])
    tol_rel = sigma / np.sqrt(np.sqrt(np.sum(sv ** 4)))    # ||G||_F = sqrt(sum s^4)
    x, info, w, tau2 = tsvd_pair(_S, _P, A, d0, d1, tol_rel)
    assert np.isclose(tau2, sigma ** 2, rtol=1e-12)
    assert np.sum(w >= tau2) == cut
    for j, b in enumerate([(d0 + d1) / 2, (d0 - d1) / 2j]):
        bh = np.concatenate([b.real, b.imag])
        ref = Vt[:cut].T @ ((U[:, :cut].T @ bh) / sv[:cut])
        assert np.max(np.abs(x[j] - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_no_truncation_is_least_squares():
    A, d0, d1 = _system(4)
    x = tsvd_pair(_S, _P, A, d0, d1, 0.0)[0]
    Ah = np.vstack([A.real, A.imag])
    for j, b in enumerate([(d0 + d1) / 2, (d0 - d1) / 2j]):
        bh = np.concatenate([b.real, b.imag])
        ref = np.linalg.lstsq(Ah, bh, rcond=None)[0]
        assert np.max(np.abs(x[j] - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_tolerance_above_everything_gives_zero():
    A, d0, d1 = _system(5)
    x, _, w, tau2 = tsvd_pair(_S, _P, A, d0, d1, 1.01)
    assert tau2 > w.max()
    assert not np.any(x)


def test_threshold_is_relative():
    A, d0, d1 = _system(6)
    x1, _, _, t1 = tsvd_pair(_S, _P, A, d0, d1, 1e-2)
    x2, _, _, t2 = tsvd_pair(_S, _P, 3.0e4 * A, 3.0e4 * d0, 3.0e4 * d1, 1e-2)
    assert np.isclose(t2, 9.0e8 * t1, rtol=1e-12)
    assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(x1))


def test_gram_form_keeps_the_solution_in_the_kept_subspace():
    A, d0, d1 = _system(7)
    G = (A.conj().T @ A).real
    c = np.stack([(A.conj().T @ ((d0 + d1) / 2)).real, (A.conj().T @ ((d0 - d1) / 2j)).real])
    tau2 = tsvd_threshold(G, 3e-2)
    x, w, _ = tsvd_gram(G, c, 3e-2)
    wv, V = np.linalg.eigh(G)
    drop = V[:, wv < tau2]
    assert drop.shape[1] > 0
    assert np.max(np.abs(drop.T @ x.T)) <= 1e-12 * np.max(np.abs(x))
    # on the kept subspace the normal equations hold exactly
    keep = V[:, wv >= tau2]
    assert np.allclose(keep.T @ (G @ x.T), keep.T @ c.T, rtol=1e-10, atol=1e-12 * np.max(np.abs(c)))


def test_survey_exact_recovery_empty_pairs_and_symmetry():
    s = make_custom(N=16, nz=6, dx=20.0, dz=15.0, freqs=tuple(np.linspace(8, 40, 9)),
                    vel=(1700.0, 2400.0), zif=(40.0,), kappa=100.0, lambda_rel=0.0, seed=5)
    pl = plan(s)
    tabs = gtables(s, pl)
    vh = vhat(s)
    clean = forward(s, pl, vh, tabs)
    V, info = tsvd_solve(s, pl, clean, tabs, 0.0)
    assert np.max(np.abs(V - vh)) <= 1e-8 * np.max(np.abs(vh))
    s2 = make_custom(N=64, nz=5, dx=25.0, freqs=(2.0, 3.0), vel=(2500.0,), noise_rel=0.05, seed=2)
    pl2, tabs2, data2, _ = synth_data(s2)
    V2, info2 = tsvd_solve(s2, pl2, data2, tabs2, 1e-2)
    assert any(p.n_rows == 0 for p in pl2.pairs)
    for p, inf in zip(pl2.pairs, info2):
        if p.n_rows == 0:
            assert inf["info"] == INFO_EMPTY and not np.any(V2[p.u])
    N = s2.n_mid
    for u in range(N):
        assert np.allclose(V2[(-u) % N], np.conj(V2[u]), rtol=0, atol=1e-14 * np.max(np.abs(V2)))
