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
* 3D areal survey: seeded random records of the doubled periodic survey
  [f, Rx, Ry, Sx, Sy] (2N per axis) -> packed rows, for 2N a power of two,
  even and odd, with the evanescent cut, in complex64 rows, and at 2N = 64
  (whose first pass takes two launches); brute-force Born records of the
  repeated model -> the oracle's clean rows; records -> rows -> FP64 solve ->
  model end to end (bar 1e-10); at the largest grid (n_mid = 128, 69 GB of
  records) a plane wave made on the device lands on exactly its rows, and so
  at the longest 2D transform (n_mid = 2048); n_mid above 128 is refused;
* 3D survey of parallel lines: seeded random records [f, line, R, S] ->
  packed rows, for power-of-two, odd and even lengths, with and without the
  evanescent cut, a single line, and complex64 rows; brute-force Born records
  -> the oracle's clean rows; records -> rows -> FP64 solve against the
  oracle's, and the model from the solution (bar 1e-10); at n_mid = 2048 a
  plane wave made on the device lands on exactly its rows; random spectra ->
  the model [N_x, N_y, nz] (bar 1e-12).
"""
import ctypes

import numpy as np
import pytest

from edt_inputs import make_config, make_custom, make_lines, vhat
from oracle.born import born_3d, born_lines
from oracle.lines3d import forward_lines, line_tables, plan_lines, solve_lines
from oracle.rows import plan as oracle_plan
from oracle.shots import model_from_spectrum, shots_to_rows
from oracle.solve import add_noise, forward, gtables, noise_scale, pack
from tests._cases import layered_small, oracle_case, rel_errors

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
    sh = torch.from_numpy(np.ascontiguousarray(D)).cuda()
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


def _areal_cases():
    kw = dict(dim=3, nz=3, dx=30.0, dz=25.0, vel=(1800.0, 2500.0), zif=(40.0,), seed=5)
    return {
        "N8-radix2": lambda: make_custom(N=8, Nh=4, freqs=(6.0, 9.0), kappa=100.0, **kw),
        "N6-direct": lambda: make_custom(N=6, Nh=6, freqs=(6.0, 9.0, 12.0), kappa=100.0, **kw),
        "N5-odd": lambda: make_custom(N=5, Nh=3, freqs=(7.0,), kappa=100.0, **kw),
        "N16-cut": lambda: make_custom(N=16, Nh=8, freqs=(6.0, 11.0), kappa=1.0, **kw),
        "N32-two-launches": lambda: make_custom(N=32, Nh=16, freqs=(5.0, 8.0), kappa=1.0, **kw),
    }


def _areal_records(s, seed):
    rng = np.random.default_rng(seed)
    shape = (len(s.freqs),) + (2 * s.n_mid,) * 4
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.mark.parametrize("name", list(_areal_cases()))
def test_areal_shot_records_to_rows(name):
    s = _areal_cases()[name]()
    pl = oracle_plan(s)
    D = _areal_records(s, 29)
    p = E.Plan(s)
    assert p.records_shape() == D.shape
    _check_rows(name, pl, _gpu_rows(p, D), shots_to_rows(s, pl, D))


def test_areal_shot_records_to_complex64_rows():
    s = _areal_cases()["N8-radix2"]()
    pl = oracle_plan(s)
    D = _areal_records(s, 31)
    p = E.Plan(s, data="c64")
    d = _gpu_rows(p, D)
    assert d.dtype == np.complex64
    ref, _ = pack(pl, shots_to_rows(s, pl, D))
    scale = np.max(np.abs(ref))
    # the library rounds its FP64 datum once
    err = np.max(np.abs(d.astype(np.complex128) - ref))
    assert err <= 1.2e-7 * scale, err / scale


def test_areal_born_records_give_the_oracle_rows():
    """Brute-force Born records of the N-periodic model repeated 2 x 2 times
    on the doubled grid: the GPU rows equal the oracle's clean rows."""
    s = make_custom(dim=3, N=8, Nh=4, nz=3, dx=30.0, dz=25.0, freqs=(6.0, 9.0), vel=(1800.0, 2500.0),
                    zif=(40.0,), kappa=100.0, seed=7)
    pl = oracle_plan(s)
    clean = forward(s, pl, vhat(s), gtables(s, pl))
    M = 2 * s.n_mid
    V2 = np.tile(s.v_true, (2, 2, 1))
    D = np.stack([born_3d(s.vel, s.zif, f, s.eps, V2, s.d_mid, s.z, s.dz).reshape(M, M, M, M)
                  for f in s.freqs])
    _check_rows("3D Born records", pl, _gpu_rows(E.Plan(s), D), clean)


def test_areal_end_to_end_from_shot_records():
    """Doubled-survey records whose transform holds 4 times the oracle's noisy
    data at the rows' keys (zero elsewhere) -> GPU transform, pack, FP64
    solve and model, against the oracle's solve and model."""
    s = make_custom(dim=3, N=8, Nh=4, nz=12, dx=30.0, dz=15.0, freqs=(5.0, 8.0, 11.0, 14.0),
                    vel=(1800.0, 2500.0), zif=(60.0,), kappa=1.0, noise_rel=0.05, seed=13)
    r = oracle_case(s)
    N, M, nh = s.n_mid, 2 * s.n_mid, s.n_off
    F = np.zeros((len(s.freqs),) + (M,) * 4, np.complex128)
    for p_, (d0, d1) in zip(r["pl"].pairs, r["data"]):
        ux, uy = divmod(p_.u, N)
        qx, qy = (ux if ux < (N + 1) // 2 else ux - N), (uy if uy < (N + 1) // 2 else uy - N)
        n = p_.key0[:, 1]
        nx, ny = n // nh - nh // 2, n % nh - nh // 2
        ax, ay, bx, by = (qx + 2 * nx) % M, (qy + 2 * ny) % M, (qx - 2 * nx) % M, (qy - 2 * ny) % M
        F[p_.f, ax, ay, bx, by] = 4.0 * d0
        F[p_.f, (-bx) % M, (-by) % M, (-ax) % M, (-ay) % M] = 4.0 * d1
    D = np.fft.ifftn(F, axes=(1, 2, 3, 4)) / s.d_mid ** 2
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
    print(f"3D end to end: model error {err:.2e}")
    assert err <= 1e-10


def test_areal_records_at_the_largest_grid():
    """n_mid = 128, the largest grid the transform takes: one frequency of
    records on 256 positions per axis (69 GB), a plane wave made on the device
    (the oracle's transform would not fit the host).  Every row must be zero
    except those whose half-grid wavenumbers are the wave's, which get
    d_mid^2 (2N)^4 / 4; each pass runs as several launches of at most 65,536
    workgroups."""
    N, M = 128, 256
    free, _ = torch.cuda.mem_get_info()
    if free < 80e9:
        pytest.skip("needs about 70 GB of free device memory")
    s = make_custom(dim=3, N=N, Nh=4, nz=2, dx=25.0, freqs=(5.0,), vel=(2000.0,), kappa=100.0, model=None)
    p = E.Plan(s)
    a0, b0 = (3, 1), (7, 5)   # a - b = 4 n with n = (-1, -1), q = (5, 3)
    g = torch.arange(M, device="cuda", dtype=torch.float64)

    def wave(k):
        return torch.polar(torch.ones_like(g), 2.0 * np.pi * k * g / M)
    rec = torch.empty((1, M, M, M, M), dtype=torch.complex128, device="cuda")
    inner = wave(a0[1])[:, None, None] * wave(b0[0])[None, :, None] * wave(b0[1])[None, None, :]
    ex = wave(a0[0])
    for x in range(M):
        rec[0, x] = ex[x] * inner
    del inner
    p.shots_fft(rec)
    d = p.shots_pack(rec)
    torch.cuda.synchronize()
    del rec
    d = d.cpu().numpy()
    m = p.rowmap()
    nh = s.n_off
    u = np.repeat(m["pair_km"][:, 0], np.diff(m["row_off"]))
    ux, uy = u // N, u % N
    qx, qy = np.where(ux < (N + 1) // 2, ux, ux - N), np.where(uy < (N + 1) // 2, uy, uy - N)
    n = m["keys"][:, 0]
    nx, ny = n // nh - nh // 2, n % nh - nh // 2
    ax, ay, bx, by = (qx + 2 * nx) % M, (qy + 2 * ny) % M, (qx - 2 * nx) % M, (qy - 2 * ny) % M
    peak = s.d_mid ** 2 * float(M) ** 4 / 4.0
    hit0 = (ax == a0[0]) & (ay == a0[1]) & (bx == b0[0]) & (by == b0[1])
    hit1 = ((-bx) % M == a0[0]) & ((-by) % M == a0[1]) & ((-ax) % M == b0[0]) & ((-ay) % M == b0[1])
    err0 = np.max(np.abs(d[:, 0] - np.where(hit0, peak, 0.0)))
    err1 = np.max(np.abs(d[:, 1] - np.where(hit1, peak, 0.0)))
    print(f"2N = {M}: {len(d)} rows, {int(hit0.sum())} + {int(hit1.sum())} hits, "
          f"max error {max(err0, err1) / peak:.2e} of the peak")
    assert hit0.sum() + hit1.sum() >= 1
    assert max(err0, err1) <= 1e-10 * peak


def test_areal_records_beyond_n_mid_128_are_refused():
    from paper_0905_0238_amd import _lib
    buf = torch.zeros(16, dtype=torch.complex128, device="cuda")
    sa = make_custom(dim=3, N=130, Nh=2, nz=2, dx=25.0, freqs=(5.0,), vel=(2000.0,), kappa=1.0, model="zero")
    pa = E.Plan(sa)
    pa.upload()
    st = _lib.load().edt_shots_fft(pa._h, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(0))
    assert st == _lib.EDT_EINVAL
    torch.cuda.synchronize()


def _line_cases():
    kw = dict(nz=4, dz=20.0, vel=(1800.0, 2500.0), zif=(40.0,), seed=9)
    return {
        "Nx16-Ny8-radix2": lambda: make_lines(Nx=16, Ny=8, dx=25.0, dy=40.0, freqs=(6.0, 11.0, 17.0),
                                              kappa=100.0, **kw),
        "Nx15-Ny7-odd-cut": lambda: make_lines(Nx=15, Ny=7, dx=20.0, dy=35.0, freqs=(9.0, 14.0, 22.0),
                                               kappa=1.0, **kw),
        "Nx24-Ny12-direct-cut": lambda: make_lines(Nx=24, Ny=12, dx=12.5, dy=25.0, freqs=(8.0, 20.0, 40.0),
                                                   kappa=1.0, **kw),
        "Nx12-Ny1": lambda: make_lines(Nx=12, Ny=1, dx=25.0, dy=40.0, freqs=(6.0, 11.0), kappa=100.0, **kw),
    }


def _line_records(s, seed):
    rng = np.random.default_rng(seed)
    shape = (len(s.freqs), s.n_line, s.n_mid, s.n_mid)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.mark.parametrize("name", list(_line_cases()))
def test_line_survey_shot_records_to_rows(name):
    s = _line_cases()[name]()
    pl = plan_lines(s)
    D = _line_records(s, 37)
    p = E.Plan(s)
    assert p.records_shape() == D.shape
    _check_rows(name, pl, _gpu_rows(p, D), shots_to_rows(s, pl, D))


def test_line_survey_shot_records_to_complex64_rows():
    s = _line_cases()["Nx15-Ny7-odd-cut"]()
    pl = plan_lines(s)
    D = _line_records(s, 41)
    d = _gpu_rows(E.Plan(s, data="c64"), D)
    assert d.dtype == np.complex64
    ref, _ = pack(pl, shots_to_rows(s, pl, D))
    # the library rounds its FP64 datum once
    err = np.max(np.abs(d.astype(np.complex128) - ref))
    assert err <= 1.2e-7 * np.max(np.abs(ref)), err / np.max(np.abs(ref))


@pytest.mark.parametrize("Nx,Ny", [(8, 6), (7, 5)])
def test_line_survey_born_records_give_the_oracle_rows(Nx, Ny):
    """Brute-force Born records of the line survey [f, line, R, S]: the GPU
    rows equal the oracle's clean rows (no evanescent cut, which would drop
    quadrature terms the brute-force records keep)."""
    s = make_lines(Nx=Nx, Ny=Ny, dx=30.0, dy=45.0, nz=3, dz=25.0, freqs=(6.0, 9.0), vel=(1800.0, 2500.0),
                   zif=(40.0,), kappa=100.0, seed=5)
    pl = plan_lines(s)
    clean = forward_lines(s, pl, vhat(s), line_tables(s))
    D = np.stack([np.transpose(born_lines(s.vel, s.zif, f, s.eps, s.v_true, s.d_mid, s.d_line, s.z, s.dz),
                               (2, 0, 1)) for f in s.freqs])
    _check_rows(f"line Born records {Nx} x {Ny}", pl, _gpu_rows(E.Plan(s), D), clean)


def test_line_survey_end_to_end_from_shot_records():
    """Records whose transform holds the oracle's noisy data at the rows'
    keys -> GPU transform, pack and FP64 solve, against the oracle's solve of
    the oracle's rows of the same records."""
    s = make_lines(Nx=12, Ny=6, dx=25.0, dy=40.0, nz=16, dz=15.0, freqs=(5.0, 8.0, 11.0, 14.0),
                   vel=(1800.0, 2500.0), zif=(60.0,), kappa=1.0, noise_rel=0.05, seed=17)
    pl = plan_lines(s)
    tab = line_tables(s)
    clean = forward_lines(s, pl, vhat(s), tab)
    data = add_noise(s, pl, clean, noise_scale(s, pl, clean))
    F = np.zeros((len(s.freqs), s.n_line, s.n_mid, s.n_mid), np.complex128)
    for q, (d0, d1) in zip(pl.pairs, data):
        F[q.f, q.key0[:, 2], q.key0[:, 0], q.key0[:, 1]] = d0
        F[q.f, q.key1[:, 2], q.key1[:, 0], q.key1[:, 1]] = d1
    D = np.fft.ifftn(F, axes=(1, 2, 3)) / s.d_mid
    Vo, _ = solve_lines(s, pl, shots_to_rows(s, pl, D), tab)
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    sh = torch.from_numpy(D).cuda()
    p.shots_fft(sh)
    d = p.shots_pack(sh)
    out = p.run(vel, d, s.lambda_rel, prec="fp64")
    m = p.model(out["v"])
    torch.cuda.synchronize()
    g, per = rel_errors(out["v"].cpu().numpy(), Vo, pl)
    ref = model_from_spectrum(s, Vo)
    err = np.max(np.abs(m.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print(f"line survey end to end: solve error {g:.2e} global, {per:.2e} per pair; model error {err:.2e}")
    assert g <= 1e-10 and per <= 1e-10 and err <= 1e-10


@pytest.mark.parametrize("Nx,Ny,nz", [(16, 8, 5), (15, 7, 33), (24, 1, 4), (128, 32, 70), (2048, 3, 2)])
def test_line_survey_model_from_spectrum(Nx, Ny, nz):
    """Seeded random spectra [N_x N_y, nz] -> the model [N_x, N_y, nz]:
    radix-2 and direct lengths on both axes, a single line, the transform's
    longest x axis; bar 1e-12 of the largest model value."""
    s = make_lines(Nx=Nx, Ny=Ny, nz=nz, freqs=(3.0,), vel=(2000.0,), model="zero")
    rng = np.random.default_rng(Nx * 100 + Ny)
    V = rng.normal(size=(Nx * Ny, nz)) + 1j * rng.normal(size=(Nx * Ny, nz))
    m = E.Plan(s).model(torch.from_numpy(V).cuda())
    torch.cuda.synchronize()
    ref = model_from_spectrum(s, V)
    assert m.shape == ref.shape
    err = np.max(np.abs(m.cpu().numpy() - ref))
    assert err <= 1e-12 * np.max(np.abs(ref)), err / np.max(np.abs(ref))


def test_line_survey_records_at_the_longest_transform():
    """n_mid = 2048 on 4 lines: a plane wave of line index c0, receiver index
    a0 and source index b0 lands on exactly the rows keyed (a0, b0, c0) (at
    +k) and (-b0, -a0, -c0) (at -k), with value d_mid N_y N^2."""
    N, Ny = 2048, 4
    s = make_lines(Nx=N, Ny=Ny, dx=5.0, dy=100.0, nz=2, freqs=(11.0,), vel=(2000.0,), zif=(), kappa=1.0,
                   model="zero")
    p = E.Plan(s)
    a0, b0, c0 = 37, 2048 - 45, 3
    g = torch.arange(N, device="cuda", dtype=torch.float64)
    gy = torch.arange(Ny, device="cuda", dtype=torch.float64)
    wa = torch.polar(torch.ones_like(g), 2.0 * np.pi * a0 * g / N)
    wb = torch.polar(torch.ones_like(g), 2.0 * np.pi * b0 * g / N)
    wc = torch.polar(torch.ones_like(gy), 2.0 * np.pi * c0 * gy / Ny)
    rec = (wc[:, None, None] * wa[None, :, None] * wb[None, None, :])[None].contiguous()
    p.shots_fft(rec)
    d = p.shots_pack(rec)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    m = p.rowmap()
    keys = m["keys"]
    c = np.repeat(m["pair_km"][:, 0] % Ny, np.diff(m["row_off"]))
    peak = s.d_mid * Ny * float(N) ** 2
    hit0 = (keys[:, 0] == a0) & (keys[:, 1] == b0) & (c == c0)
    hit1 = (((-keys[:, 1]) % N) == a0) & (((-keys[:, 0]) % N) == b0) & (((-c) % Ny) == c0)
    err = max(np.max(np.abs(d[:, 0] - np.where(hit0, peak, 0.0))),
              np.max(np.abs(d[:, 1] - np.where(hit1, peak, 0.0))))
    print(f"N = {N}, N_y = {Ny}: {len(d)} rows, {int(hit0.sum())} + {int(hit1.sum())} hits, "
          f"max error {err / peak:.2e} of the peak")
    assert hit0.sum() + hit1.sum() >= 1
    assert err <= 1e-10 * peak, err / peak


def test_line_records_at_the_longest_transform():
    """n_mid = 2048, the longest transform: a plane wave of receiver index a0
    and source index b0 lands on exactly the rows keyed (a0, b0) (at +k_m)
    and (-b0, -a0) (at -k_m), with value d_mid N^2; every other datum is zero."""
    N = 2048
    s = make_custom(N=N, nz=2, dx=5.0, freqs=(6.0, 11.0), vel=(2000.0,), kappa=1.0, model=None)
    p = E.Plan(s)
    a0, b0 = 37, 2048 - 45
    g = torch.arange(N, device="cuda", dtype=torch.float64)
    wa = torch.polar(torch.ones_like(g), 2.0 * np.pi * a0 * g / N)
    wb = torch.polar(torch.ones_like(g), 2.0 * np.pi * b0 * g / N)
    rec = (wa[:, None] * wb[None, :]).expand(len(s.freqs), N, N).contiguous()
    p.shots_fft(rec)
    d = p.shots_pack(rec)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    keys = p.rowmap()["keys"]
    peak = s.d_mid * float(N) ** 2
    hit0 = (keys[:, 0] == a0) & (keys[:, 1] == b0)
    hit1 = (((-keys[:, 1]) % N) == a0) & (((-keys[:, 0]) % N) == b0)
    err = max(np.max(np.abs(d[:, 0] - np.where(hit0, peak, 0.0))),
              np.max(np.abs(d[:, 1] - np.where(hit1, peak, 0.0))))
    assert hit0.sum() + hit1.sum() >= 1
    assert err <= 1e-10 * peak, err / peak


def test_transforms_longer_than_2048_are_refused():
    s = make_custom(N=2050, nz=2, dx=5.0, freqs=(5.0,), vel=(2000.0,), model="zero")
    p = E.Plan(s)
    sh = torch.zeros(1, 2050, 2050, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="n_mid > 2048"):
        p.shots_fft(sh)
    v = torch.zeros(p.n_km, s.nz, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="n_mid > 2048"):
        p.model(v)

