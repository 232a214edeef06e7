"""GPU: the transforms on either side of the decoupled problems
(edt_shots_fft + edt_shots_pack, edt_model) against the oracle's numpy FFTs
(oracle.shots), element by element.

* seeded random shot records -> packed rows, for power-of-two lengths
  (radix-2 path) and others (direct path: even, odd), with and without the
  evanescent cut, and at the full size of the 2D N = 512, 128-frequency
  survey; bar 1e-12 of the largest datum;
* seeded random spectra -> the model, 2D and 3D, up to the 3D 128 x 128,
  nz = 200 grid; bar 1e-12 of the largest model value;
* end to end on a small survey: shot records -> rows -> FP64 solve -> model,
  against the oracle's solve and model, to the FP64 bar 1e-10;
* 3D shot records are refused.
"""
import numpy as np
import pytest

from edt_inputs import make_config, make_custom
from oracle.rows import plan as oracle_plan
from oracle.shots import model_from_spectrum, shots_to_rows
from oracle.solve import pack
from tests._cases import oracle_case, layered_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")


def _shot_cases():
    return {
        "N12-direct": lambda: make_custom(N=12, nz=5, dx=25.0, freqs=(5.0, 9.0), vel=(1800.0, 2600.0),
                                          zif=(45.0,), kappa=100.0, seed=3),
        "N11-odd": lambda: make_custom(N=11, nz=5, dx=25.0, freqs=(5.0, 9.0, 13.0), vel=(1800.0,), seed=3),
        "N16-cut": lambda: make_custom(N=16, nz=5, dx=25.0, freqs=(6.0, 11.0), vel=(1800.0, 2600.0),
                                       zif=(45.0,), kappa=1.0, seed=3),
        "N48-layered": lambda: layered_small(),
        "cfg1-N64": lambda: make_config(1),
    }


def _records(s, seed):
    rng = np.random.default_rng(seed)
    shape = (len(s.freqs), s.n_mid, s.n_mid)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def _gpu_rows(p, D):
    sh = torch.from_numpy(D).cuda()
    p.shots_fft(sh)
    d = p.shots_pack(sh)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def _check_rows(name, pl, d_gpu, rows_o):
    ref, off = pack(pl, rows_o)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(d_gpu - ref))
    print(f"{name}: {ref.shape[0]} rows, max error {err / scale:.2e} of the largest datum")
    assert err <= 1e-12 * scale, (name, err / scale)


@pytest.mark.parametrize("name", list(_shot_cases()))
def test_shot_records_to_rows(name):
    s = _shot_cases()[name]()
    pl = oracle_plan(s)
    D = _records(s, 17)
    p = E.Plan(s)
    _check_rows(name, pl, _gpu_rows(p, D), shots_to_rows(s, pl, D))


def test_shot_records_to_rows_at_full_size():
    s = make_config(2)
    pl = oracle_plan(s)
    D = _records(s, 23)
    p = E.Plan(s)
    _check_rows("2D N=512 nf=128", pl, _gpu_rows(p, D), shots_to_rows(s, pl, D))


@pytest.mark.parametrize("dim,N,nz", [(2, 12, 7), (2, 64, 64), (2, 512, 256), (3, 12, 37), (3, 16, 8),
                                      (3, 128, 200)])
def test_model_from_spectrum(dim, N, nz):
    kw = dict(dim=3, Nh=N // 2) if dim == 3 else {}
    s = make_custom(N=N, nz=nz, dx=12.5, dz=8.0, freqs=(5.0,), vel=(2000.0,), **kw)
    p = E.Plan(s)
    rng = np.random.default_rng(N + nz)
    V = rng.normal(size=(p.n_km, nz)) + 1j * rng.normal(size=(p.n_km, nz))
    m = p.model(torch.from_numpy(V).cuda())
    torch.cuda.synchronize()
    ref = model_from_spectrum(s, V)
    err = np.max(np.abs(m.cpu().numpy() - ref))
    assert err <= 1e-12 * np.max(np.abs(ref)), (dim, N, nz, err)


def test_end_to_end_from_shot_records():
    """Records whose transform is the oracle's noisy data (zero outside the
    kept rows) go through the GPU transform, FP64 solve and model."""
    s = layered_small(N=32, nz=40)
    r = oracle_case(s)
    pl = r["pl"]
    F = np.zeros((len(s.freqs), s.n_mid, s.n_mid), np.complex128)
    for p_, (d0, d1) in zip(pl.pairs, r["data"]):
        F[p_.f, p_.key0[:, 0], p_.key0[:, 1]] = d0
        F[p_.f, p_.key1[:, 0], p_.key1[:, 1]] = d1
    D = np.fft.ifft2(F, axes=(1, 2)) / s.d_mid
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    sh = torch.from_numpy(D).cuda()
    p.shots_fft(sh)
    d = p.shots_pack(sh)
    out = p.run(vel, d, s.lambda_rel, prec="fp64")
    m = p.model(out["v"])
    torch.cuda.synchronize()
    ref = model_from_spectrum(s, r["V"])
    err = np.max(np.abs(m.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print(f"end to end: model error {err:.2e}")
    assert err <= 1e-10


def test_shot_records_of_3d_surveys_are_refused():
    s = make_custom(dim=3, N=12, Nh=6, nz=5, dx=25.0, freqs=(5.0,), vel=(2000.0,))
    p = E.Plan(s)
    sh = torch.zeros(1, 12, 12, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="2D line survey"):
        p.shots_fft(sh)


def test_transforms_longer_than_2048_are_refused():
    s = make_custom(N=2050, nz=2, dx=5.0, freqs=(5.0,), vel=(2000.0,), model="zero")
    p = E.Plan(s)
    sh = torch.zeros(1, 1, 1, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="n_mid > 2048"):
        p.shots_fft(sh)
    v = torch.zeros(p.n_km, s.nz, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="n_mid > 2048"):
        p.model(v)

