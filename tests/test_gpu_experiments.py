"""GPU: the paper's numerical examples (Section 3.2), run end to end through
the library -- Born data by edt_forward, truncated-SVD solve (with and
without the k_z restriction), model by edt_model -- and checked for the
qualitative outcomes the paper reports, as orderings of the relative model
error in the middle 4 km of the 40 km line.

The geometry is the paper's (a 40 km line at 50 m, depths 800-4000 m at 50 m,
a 1 km square of V = 1, water or water over 4000 m/s below 1 km, 1-10 Hz,
imaginary frequency 0.15 1/s) in the infinite-aperture reading of eq. M; the
tolerance is relative (sigma^2 = tol_rel^2 ||G||_F, since the scale of the
paper's sigma = 1 is unknown).  Outcomes checked:
* homogeneous water, 1-5 Hz: the square at 2000 m is reconstructed worse than
  at 1500 m;
* the two-layer reference reconstructs the square at 2000 m far better than
  water (error below half);
* two-layer: 1-10 Hz beats 1-5 Hz, and 5-10 Hz is worse than 1-10 Hz;
* two-layer, 1-5 and 1-10 Hz: the k_z restriction changes the error little;
* 5% noise of constant modulus and random phase added to the shot records
  (through edt_shots_fft / edt_shots_pack): at a large tolerance the error
  barely grows, at a small one it grows markedly.
One configuration is also run by the oracle, to the FP64 bar.
"""
import numpy as np
import pytest

from edt_inputs import make_square_experiment
from oracle.rows import plan as oracle_plan
from oracle.shots import model_from_spectrum
from oracle.solve import gtables, forward
from oracle.tsvd import tsvd_solve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")

F_1_5 = (1.0, 2.0, 3.0, 4.0, 5.0)
F_1_10 = tuple(float(f) for f in range(1, 11))
F_5_10 = tuple(float(f) for f in range(5, 11))


def _window_error(s, m):
    N = s.n_mid
    n = np.arange(N)
    x = np.where(n < (N + 1) // 2, n, n - N) * s.d_mid
    w = np.abs(x) <= 2000.0
    return float(np.linalg.norm(m[w] - s.v_true[w]) / np.linalg.norm(s.v_true[w]))


def _noisy_rows(p, s, d_clean, rng):
    """Records whose transform is the clean data, plus noise of modulus 0.05
    max|D_f| and uniform phase per record entry, back through the GPU
    transform."""
    rm = p.rowmap()
    f = rm["rows"][:, 0]
    a, b = rm["keys"][:, 0], rm["keys"][:, 1]
    N = s.n_mid
    d = d_clean.cpu().numpy()
    F = np.zeros((s.n_freq, N, N), np.complex128)
    F[f, a, b] = d[:, 0]
    F[f, (-b) % N, (-a) % N] = d[:, 1]
    D = np.fft.ifft2(F, axes=(1, 2)) / s.d_mid
    amp = 0.05 * np.max(np.abs(D), axis=(1, 2))
    D = D + amp[:, None, None] * np.exp(2j * np.pi * rng.random(D.shape))
    rec = torch.from_numpy(D).cuda()
    p.shots_fft(rec)
    return p.shots_pack(rec)


def _run(s, tol, restrict=False, noise_seed=None):
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    g64, _ = p.green(vel, want32=False)
    vt = torch.from_numpy(np.fft.fft(s.v_true, axis=0)).cuda()
    d = p.forward(g64, vt)
    if noise_seed is not None:
        d = _noisy_rows(p, s, d, np.random.default_rng(noise_seed))
    gram, rhs, _ = p.assemble(g64, None, d, "fp64")
    work = p.tsvd_work()
    if restrict:
        p.kz_restrict(gram, rhs, p.kz_disk_radius(2.2), work)
    _, v, info, _ = p.tsvd(gram, rhs, tol, max_iter=150, tsvd_work=work)
    m = p.model(v)
    torch.cuda.synchronize()
    return _window_error(s, m.cpu().numpy()), v.cpu().numpy(), info.cpu().numpy()


TOL = 1e-2


@pytest.fixture(scope="module")
def errors():
    cases = {
        "water-1500-1to5": dict(depth=1500.0, freqs=F_1_5),
        "water-2000-1to5": dict(depth=2000.0, freqs=F_1_5),
        "layers-2000-1to5": dict(depth=2000.0, two_layer=True, freqs=F_1_5),
        "layers-2000-1to10": dict(depth=2000.0, two_layer=True, freqs=F_1_10),
        "layers-2000-5to10": dict(depth=2000.0, two_layer=True, freqs=F_5_10),
    }
    out = {}
    for name, kw in cases.items():
        s = make_square_experiment(**kw)
        for restrict in (False, True):
            e, _, info = _run(s, TOL, restrict)
            assert np.all(info[:] >= -1), (name, info.min())
            out[(name, restrict)] = e
    for k, v in out.items():
        print(f"{k[0]} {'restricted' if k[1] else 'unrestricted'}: relative error {v:.3f}")
    return out


def test_deeper_square_is_worse_in_water(errors):
    for r in (False, True):
        assert errors[("water-2000-1to5", r)] > errors[("water-1500-1to5", r)] + 0.05


def test_two_layer_reference_is_far_better_for_the_deep_square(errors):
    for r in (False, True):
        assert errors[("layers-2000-1to5", r)] < 0.5 * errors[("water-2000-1to5", r)]


def test_frequency_bands(errors):
    for r in (False, True):
        assert errors[("layers-2000-1to10", r)] < errors[("layers-2000-1to5", r)]
        assert errors[("layers-2000-5to10", r)] > errors[("layers-2000-1to10", r)] + 0.05


def test_restriction_changes_little_with_two_layers(errors):
    for name in ("layers-2000-1to5", "layers-2000-1to10"):
        assert abs(errors[(name, True)] - errors[(name, False)]) <= 0.1 * errors[(name, False)]


def test_noise_and_tolerance():
    s = make_square_experiment(depth=2000.0, two_layer=True, freqs=F_1_10)
    big = [_run(s, 1e-2, noise_seed=n)[0] for n in (None, 1)]
    small = [_run(s, 1e-3, noise_seed=n)[0] for n in (None, 1)]
    print(f"tol 1e-2: clean {big[0]:.3f} noisy {big[1]:.3f}; tol 1e-3: clean {small[0]:.3f} noisy {small[1]:.3f}")
    assert big[1] <= 1.05 * big[0]
    assert small[1] >= 1.5 * small[0]


def test_one_example_matches_the_oracle():
    s = make_square_experiment(depth=2000.0, two_layer=True, freqs=F_1_5, N=200)
    e, v, _ = _run(s, TOL)
    pl = oracle_plan(s)
    tabs = gtables(s, pl)
    clean = forward(s, pl, np.fft.fft(s.v_true, axis=0), tabs)
    Vo, _ = tsvd_solve(s, pl, clean, tabs, TOL)
    eo = _window_error(s, model_from_spectrum(s, Vo))
    assert abs(e - eo) <= 1e-8 * eo, (e, eo)
    assert np.linalg.norm(v - Vo) <= 1e-9 * np.linalg.norm(Vo)
