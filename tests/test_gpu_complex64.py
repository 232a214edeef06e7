"""Data rows stored in complex64 (the plan option EDT_DATA_C64), through the
C-ABI, against the FP64 oracle fed the same rounded data.

The library reads complex64 rows and widens them to FP64, so a solve on
complex64 rows must meet the FP64 bar (<= 1e-10) against the oracle's solve
of the rounded data (complex64 values held in complex128), and the mixed
paths the mixed bar (<= 1e-6).  Outputs written in the plan's data type (the
forward map, the shot-record gather, the data gradient) are the FP64 results
rounded once to complex64.
"""
import numpy as np
import pytest

from edt_inputs import make_custom, vhat
from oracle.solve import solve
from tests._cases import oracle_case, rel_errors, layered_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rounded_case(s):
    r = oracle_case(s)
    d32 = r["d_rows"].astype(np.complex64)
    d64 = d32.astype(np.complex128)
    off = r["off"]
    data = [(d64[off[i]:off[i + 1], 0], d64[off[i]:off[i + 1], 1]) for i in range(len(r["pl"].pairs))]
    V, _ = solve(s, r["pl"], data, r["tabs"])
    return r, d32, data, V


CASES = {
    "layered-nz40": lambda: layered_small(),
    "layered-nz257": lambda: layered_small(nz=257, N=16, nf=4, seed=4),
    "3d-small": lambda: make_custom(dim=3, N=12, Nh=6, nz=37, dx=25.0, dz=10.0, freqs=(8.0, 14.0, 20.0),
                                    vel=(1800.0, 2500.0, 2100.0), zif=(60.0, 200.0), noise_rel=0.05, seed=5),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_complex64_rows_solve_against_oracle_of_rounded_data(name):
    s = CASES[name]()
    r, d32, data, V = _rounded_case(s)
    p = E.Plan(s, data="c64")
    vel = _dev(np.asarray(s.vel, np.float64))
    d = _dev(d32)
    for prec, bar in (("fp64", 1e-10), ("fp16x3", 1e-6), ("bf16x3", 1e-6)):
        out = p.run(vel, d, s.lambda_rel, prec=prec, refine_tol=3e-7, max_refine=12)
        torch.cuda.synchronize()
        g, per = rel_errors(out["v"].cpu().numpy(), V, r["pl"])
        print(f"{name} c64 {prec}: global {g:.2e} per pair {per:.2e}", flush=True)
        assert g <= bar and per <= bar, (prec, g, per)
    # the rounding of the data is what separates this from the complex128 solve
    g, _ = rel_errors(V, r["V"], r["pl"])
    assert g > 1e-12


@pytest.mark.parametrize("name", ["layered-nz40", "3d-small"])
def test_complex64_forward_rows_are_rounded_fp64_rows(name):
    s = CASES[name]()
    r = oracle_case(s)
    p = E.Plan(s, data="c64")
    g64, _ = p.green(_dev(np.asarray(s.vel, np.float64)), want32=False)
    d = p.forward(g64, _dev(vhat(s)))
    torch.cuda.synchronize()
    assert d.dtype == torch.complex64
    d = d.cpu().numpy().astype(np.complex128)
    clean = np.zeros_like(d)
    for i, (d0, d1) in enumerate(r["clean"]):
        clean[r["off"][i]:r["off"][i + 1], 0] = d0
        clean[r["off"][i]:r["off"][i + 1], 1] = d1
    # one rounding to FP32 per component (2^-24 relative) on top of FP64 rows
    err = np.abs(d - clean)
    assert np.all(err <= 2.0 ** -24 * (np.abs(clean.real) + np.abs(clean.imag)) + 1e-12 * np.max(np.abs(clean)))


def test_complex64_shot_gather_rounds_the_complex128_gather():
    s = make_custom(N=48, nz=8, dx=12.5, dz=8.0, freqs=(5.0, 11.0, 23.0), vel=(2100.0, 2600.0), zif=(40.0,),
                    noise_rel=0.0, seed=3)
    rng = np.random.default_rng(2)
    rec = rng.normal(size=(s.n_freq, s.n_mid, s.n_mid)) + 1j * rng.normal(size=(s.n_freq, s.n_mid, s.n_mid))
    p128, p64 = E.Plan(s), E.Plan(s, data="c64")
    sh = _dev(rec)
    p128.shots_fft(sh)
    a = p128.shots_pack(sh).cpu().numpy()
    b = p64.shots_pack(sh).cpu().numpy()
    assert b.dtype == np.complex64
    assert np.array_equal(b, a.astype(np.complex64))


def test_complex64_data_gradient_against_oracle():
    from oracle.grad import grad
    s = layered_small(nz=24, N=24, nf=6, seed=4)
    r, d32, data, V = _rounded_case(s)
    rng = np.random.default_rng(1)
    T = rng.normal(size=(s.n_mid, s.nz)) + 1j * rng.normal(size=(s.n_mid, s.nz))
    go = grad(s, r["pl"], data, 2.0 * (V - T))
    p = E.Plan(s, data="c64")
    d = _dev(d32).requires_grad_(True)
    lam = torch.tensor(s.lambda_rel, dtype=torch.float64, device="cuda", requires_grad=True)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda", requires_grad=True)
    Vg = E.edt_solve(d, lam, vel, p)
    loss = (Vg - _dev(T)).abs().pow(2).sum()
    loss.backward()
    assert d.grad.dtype == torch.complex64
    gd = d.grad.cpu().numpy().astype(np.complex128)
    ref = np.zeros_like(gd)
    for i, (a0, a1) in enumerate(go["d"]):
        ref[r["off"][i]:r["off"][i + 1], 0] = a0
        ref[r["off"][i]:r["off"][i + 1], 1] = a1
    # the data gradient is formed in FP64 and rounded once to complex64
    assert np.max(np.abs(gd - ref)) <= 1e-7 * np.max(np.abs(ref))
    assert abs(lam.grad.item() - go["lambda_rel"]) <= 1e-10 * np.sum(go["lambda_abs"])
    gv = vel.grad.cpu().numpy()
    assert np.max(np.abs(gv - go["vel"])) <= 1e-8 * np.max(np.abs(go["vel"]))


def test_rows_of_the_wrong_type_are_refused():
    s = layered_small()
    r = oracle_case(s)
    p = E.Plan(s, data="c64")
    g64, g32 = p.green(_dev(np.asarray(s.vel, np.float64)))
    with pytest.raises(ValueError, match="complex64"):
        p.assemble(g64, g32, _dev(r["d_rows"]), "fp16x3")
