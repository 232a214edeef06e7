"""GPU: the 3D survey of parallel lines (paper Section 2.2) through the C-ABI,
against the FP64 oracle (oracle.lines3d).

* the rows' Gram Re(A^H A), right-hand sides and trace (edt_assemble, FP64)
  against the oracle's rows, to 1e-12 of each pair's largest entry;
* the damped solve (edt_solve without refinement) against the oracle's, to
  1e-10 globally and per pair; complex64 data rows against the oracle fed
  the same rounded data;
* the Born forward map against the oracle's data, to 1e-12;
* the truncated SVD runs on the line Gram;
* the finite aperture (edt_aperture_gram, the offset window on every line):
  the windowed Gram and trace against the oracle's Re(A^H S A) to 1e-12, the
  damped solve of windowed data against the oracle's to 1e-10, a window
  holding every offset gives edt_assemble's Gram, and sampled pairs of the
  larger survey (three chunks of pairs) against the oracle;
* the adjoint (edt_adjoint) against the oracle's gradient: data to 1e-9,
  damping and layer velocities to 1e-8, on the three surveys;
* what the line survey does not cover is refused.
Surveys: odd and even grids, with and without the evanescent cut, depth
counts that span several 64-tiles with a ragged tail, and a larger survey on
sampled pairs.
"""
import numpy as np
import pytest

from edt_inputs import make_lines, vhat
from oracle.lines3d import forward_lines, line_row_values, line_tables, plan_lines, solve_lines
from oracle.aperture import aperture_data, aperture_rows, aperture_solve, offset_window, window_kernel
from oracle.solve import add_noise, noise_scale, normal_equations, pack
from tests._cases import rel_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = {
    "even-nocut": lambda: make_lines(Nx=16, Ny=8, dx=25.0, dy=40.0, nz=24, dz=15.0, freqs=(6.0, 11.0, 17.0),
                                     vel=(1800.0, 2600.0), zif=(45.0,), kappa=100.0, noise_rel=0.05, seed=1),
    "odd-cut": lambda: make_lines(Nx=15, Ny=7, dx=20.0, dy=35.0, nz=33, dz=12.0, freqs=(9.0, 14.0, 22.0, 31.0),
                                  vel=(2000.0, 2600.0, 1900.0), zif=(40.0, 140.0), kappa=1.0, noise_rel=0.05, seed=2),
    "deep-cut": lambda: make_lines(Nx=24, Ny=12, dx=12.5, dy=25.0, nz=150, dz=8.0,
                                   freqs=tuple(np.linspace(8.0, 40.0, 6)), vel=(1700.0, 2400.0, 3100.0),
                                   zif=(120.0, 600.0), kappa=1.0, noise_rel=0.05, seed=3),
}


def _case(s):
    pl = plan_lines(s)
    tab = line_tables(s)
    clean = forward_lines(s, pl, vhat(s), tab)
    data = add_noise(s, pl, clean, noise_scale(s, pl, clean))
    d_rows, off = pack(pl, data)
    return pl, tab, clean, data, d_rows, off


@pytest.mark.parametrize("name", sorted(CASES))
def test_line_gram_rhs_trace_and_solve(name):
    s = CASES[name]()
    pl, tab, clean, data, d_rows, off = _case(s)
    p = E.Plan(s)
    m = p.rowmap()
    assert np.array_equal(m["row_off"], off)
    assert p.n_km == s.n_mid * s.n_line
    vel = _dev(np.asarray(s.vel, np.float64))
    g64, _ = p.green(vel, want32=False)
    d = _dev(d_rows)
    gram, rhs, trace = p.assemble(g64, None, d, "fp64")
    torch.cuda.synchronize()
    G, Rc, T = gram.cpu().numpy(), rhs.cpu().numpy(), trace.cpu().numpy()
    low = np.tril(np.ones((s.nz, s.nz), bool))
    for i, (q, (d0, d1)) in enumerate(zip(pl.pairs, data)):
        if not q.n_rows:
            continue
        A = line_row_values(s, q, tab)
        Go, co, tro = normal_equations(A, d0, d1)
        assert np.max(np.abs(G[i][low] - Go[low])) <= 1e-12 * np.max(np.abs(Go)), (name, i)
        assert np.max(np.abs(Rc[i] - co)) <= 1e-12 * np.max(np.abs(co)), (name, i)
        assert abs(T[i] - tro) <= 1e-12 * tro
    x, v, info, _ = p.solve(g64, d, gram, rhs, trace, s.lambda_rel)
    torch.cuda.synchronize()
    Vo, _ = solve_lines(s, pl, data, tab)
    g, per = rel_errors(v.cpu().numpy(), Vo, pl)
    print(f"{name}: {len(pl.pairs)} pairs, {p.n_rows} rows; solve error {g:.2e} global, {per:.2e} per pair",
          flush=True)
    assert g <= 1e-10 and per <= 1e-10
    info = info.cpu().numpy()
    for q, inf in zip(pl.pairs, info):
        assert inf == (-1 if q.n_rows == 0 else 0)


@pytest.mark.parametrize("name", ["even-nocut", "odd-cut"])
def test_line_forward_map(name):
    s = CASES[name]()
    pl, tab, clean, data, d_rows, off = _case(s)
    ref, _ = pack(pl, clean)
    for dt in ("c128", "c64"):
        p = E.Plan(s, data=dt)
        g64, _ = p.green(_dev(np.asarray(s.vel, np.float64)), want32=False)
        d = p.forward(g64, _dev(vhat(s))).cpu().numpy().astype(np.complex128)
        bar = 1e-12 if dt == "c128" else 2.0 ** -23
        assert np.max(np.abs(d - ref)) <= bar * np.max(np.abs(ref)), (name, dt)


def test_line_solve_on_complex64_rows():
    from oracle.lines3d import solve_lines as sl
    s = CASES["odd-cut"]()
    pl, tab, clean, data, d_rows, off = _case(s)
    d32 = d_rows.astype(np.complex64)
    r64 = d32.astype(np.complex128)
    data_r = [(r64[off[i]:off[i + 1], 0], r64[off[i]:off[i + 1], 1]) for i in range(len(pl.pairs))]
    Vo, _ = sl(s, pl, data_r, tab)
    p = E.Plan(s, data="c64")
    out = p.run(_dev(np.asarray(s.vel, np.float64)), _dev(d32), s.lambda_rel, prec="fp64")
    torch.cuda.synchronize()
    g, per = rel_errors(out["v"].cpu().numpy(), Vo, pl)
    assert g <= 1e-10 and per <= 1e-10


def test_truncated_svd_on_the_line_gram():
    from oracle.tsvd import tsvd_gram
    s = CASES["odd-cut"]()
    pl, tab, clean, data, d_rows, off = _case(s)
    p = E.Plan(s)
    g64, _ = p.green(_dev(np.asarray(s.vel, np.float64)), want32=False)
    gram, rhs, _ = p.assemble(g64, None, _dev(d_rows), "fp64")
    _, v, info, iters = p.tsvd(gram, rhs, 1e-2)
    torch.cuda.synchronize()
    v = v.cpu().numpy()
    u = np.finfo(np.float64).eps / 2
    nv = np.linalg.norm(v)
    checked = 0
    for q, (d0, d1) in zip(pl.pairs, data):
        if not q.n_rows:
            continue
        Go, co, _ = normal_equations(line_row_values(s, q, tab), d0, d1)
        x, w, t2 = tsvd_gram(Go, co, 1e-2)
        if q.self_conjugate:
            x[1] = 0.0
        gap = np.min(np.abs(w - t2))
        if gap <= 1e-6 * t2:
            continue
        kept = w[w >= t2]
        bar = max(1e-10, 100 * u * (w.max() / kept.min() + w.max() / gap))
        idx = [q.u] if q.self_conjugate else [q.u, q.u_neg]
        ref = np.array([x[0] + 1j * x[1]] if q.self_conjugate else [x[0] + 1j * x[1], x[0] - 1j * x[1]])
        err = np.linalg.norm(v[idx] - ref) / max(np.linalg.norm(ref), 1e-3 * nv)
        assert err <= bar, (q.u, err, bar)
        checked += 1
    assert checked > 0


@pytest.mark.parametrize("name,b", [("even-nocut", 60.0), ("odd-cut", 45.0), ("deep-cut", 40.0)])
def test_line_aperture_gram_and_solve(name, b):
    s = CASES[name]()
    pl, tab, clean, data, d_rows, off = _case(s)
    w = offset_window(s, b)
    assert 0 < w.sum() < s.n_mid
    Sm = window_kernel(w)
    dW = aperture_data(s, pl, data, b)
    p = E.Plan(s)
    g64, _ = p.green(_dev(np.asarray(s.vel, np.float64)), want32=False)
    d = _dev(pack(pl, dW)[0])
    gram_full, rhs, trace_full = p.assemble(g64, None, d, "fp64")
    gram, trace = p.aperture_gram(g64, b)
    x, v, info, _ = p.solve(g64, d, gram.clone(), rhs, trace, s.lambda_rel)   # the solve factors in place
    gram_all, trace_all = p.aperture_gram(g64, 1e6)
    torch.cuda.synchronize()
    G, T = gram.cpu().numpy(), trace.cpu().numpy()
    low = np.tril(np.ones((s.nz, s.nz), bool))
    for i, q in enumerate(pl.pairs):
        if not q.n_rows:
            continue
        A = line_row_values(s, q, tab)
        ref = (A.conj().T @ aperture_rows(s, q, A, Sm)).real
        assert np.max(np.abs(G[i][low] - ref[low])) <= 1e-12 * np.max(np.abs(ref)), (name, i)
        assert abs(T[i] - np.trace(ref)) <= 1e-12 * abs(np.trace(ref)), (name, i)
    Vo, _ = aperture_solve(s, pl, dW, tab, b)
    g, per = rel_errors(v.cpu().numpy(), Vo, pl)
    print(f"{name}: aperture b = {b} m ({int(w.sum())} of {s.n_mid} offsets); solve error {g:.2e} global, "
          f"{per:.2e} per pair", flush=True)
    assert g <= 1e-10 and per <= 1e-10
    Ga, Gf = gram_all.cpu().numpy(), gram_full.cpu().numpy()
    for i in range(len(pl.pairs)):
        scale = max(np.max(np.abs(Gf[i][low])), 1e-300)
        assert np.max(np.abs(Ga[i][low] - Gf[i][low])) <= 1e-12 * scale
    assert np.allclose(trace_all.cpu().numpy(), trace_full.cpu().numpy(), rtol=1e-12, atol=0)


@pytest.mark.parametrize("name", sorted(CASES))
def test_line_adjoint_matches_the_oracle_gradient(name):
    from oracle.grad import grad_lines
    s = CASES[name]()
    pl, tab, clean, data, d_rows, off = _case(s)
    rng = np.random.default_rng(3)
    T = rng.normal(size=(pl.n_km, s.nz)) + 1j * rng.normal(size=(pl.n_km, s.nz))
    Vo, _ = solve_lines(s, pl, data, tab)
    gV = 2.0 * (Vo - T)
    go = grad_lines(s, pl, data, gV)
    p = E.Plan(s)
    vel = _dev(np.asarray(s.vel, np.float64))
    d = _dev(d_rows)
    out = p.run(vel, d, s.lambda_rel, prec="fp64")
    gd, gl, gvel = p.adjoint(vel, out["g64"], d, out["gram"], out["trace"], out["x"], s.lambda_rel, _dev(gV))
    torch.cuda.synchronize()
    gd = gd.cpu().numpy()
    ref_d = np.zeros_like(gd)
    for i, (a0, a1) in enumerate(go["d"]):
        ref_d[off[i]:off[i + 1], 0] = a0
        ref_d[off[i]:off[i + 1], 1] = a1
    ed = np.max(np.abs(gd - ref_d)) / np.max(np.abs(ref_d))
    el = abs(gl.item() - go["lambda_rel"]) / abs(go["lambda_rel"])
    ev = np.max(np.abs(gvel.cpu().numpy() - go["vel"])) / np.max(np.abs(go["vel"]))
    print(f"{name}: adjoint errors data {ed:.2e}, damping {el:.2e}, velocities {ev:.2e}", flush=True)
    assert ed <= 1e-9 and el <= 1e-8 and ev <= 1e-8


def test_line_adjoint_on_complex64_rows():
    """A complex64 plan reads its data rows widened to FP64 and writes the data
    gradient rounded once to complex64: against the oracle fed the same
    rounded data, 1.2e-7 of the largest data gradient (the rounding), 1e-8 for
    the damping and the velocities."""
    from oracle.grad import grad_lines
    s = CASES["even-nocut"]()
    pl, tab, clean, data, d_rows, off = _case(s)
    d32 = d_rows.astype(np.complex64)
    r64 = d32.astype(np.complex128)
    data_r = [(r64[off[i]:off[i + 1], 0], r64[off[i]:off[i + 1], 1]) for i in range(len(pl.pairs))]
    rng = np.random.default_rng(7)
    T = rng.normal(size=(pl.n_km, s.nz)) + 1j * rng.normal(size=(pl.n_km, s.nz))
    Vo, _ = solve_lines(s, pl, data_r, tab)
    go = grad_lines(s, pl, data_r, 2.0 * (Vo - T))
    p = E.Plan(s, data="c64")
    vel = _dev(np.asarray(s.vel, np.float64))
    d = _dev(d32)
    out = p.run(vel, d, s.lambda_rel, prec="fp64")
    gd, gl, gvel = p.adjoint(vel, out["g64"], d, out["gram"], out["trace"], out["x"], s.lambda_rel,
                             _dev(2.0 * (Vo - T)))
    torch.cuda.synchronize()
    gd = gd.cpu().numpy()
    assert gd.dtype == np.complex64
    ref_d = np.zeros(gd.shape, np.complex128)
    for i, (a0, a1) in enumerate(go["d"]):
        ref_d[off[i]:off[i + 1], 0] = a0
        ref_d[off[i]:off[i + 1], 1] = a1
    assert np.max(np.abs(gd.astype(np.complex128) - ref_d)) <= 1.2e-7 * np.max(np.abs(ref_d))
    assert abs(gl.item() - go["lambda_rel"]) <= 1e-8 * abs(go["lambda_rel"])
    assert np.max(np.abs(gvel.cpu().numpy() - go["vel"])) <= 1e-8 * np.max(np.abs(go["vel"]))


def test_line_autograd_through_the_solve():
    """torch.autograd through edt_solve on a line survey: the velocity,
    damping and data gradients of |V~ - T|^2 against the oracle's."""
    from oracle.grad import grad_lines
    from paper_0905_0238_amd.autograd import edt_solve
    s = CASES["odd-cut"]()
    pl, tab, clean, data, d_rows, off = _case(s)
    rng = np.random.default_rng(5)
    T = rng.normal(size=(pl.n_km, s.nz)) + 1j * rng.normal(size=(pl.n_km, s.nz))
    Vo, _ = solve_lines(s, pl, data, tab)
    go = grad_lines(s, pl, data, 2.0 * (Vo - T))
    p = E.Plan(s)
    vel = _dev(np.asarray(s.vel, np.float64)).requires_grad_(True)
    lam = torch.tensor(s.lambda_rel, dtype=torch.float64, device="cuda", requires_grad=True)
    d = _dev(d_rows).requires_grad_(True)
    V = edt_solve(d, lam, vel, p)
    loss = torch.sum(torch.abs(V - _dev(T)) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    gv = vel.grad.cpu().numpy()
    assert np.max(np.abs(gv - go["vel"])) <= 1e-8 * np.max(np.abs(go["vel"]))
    assert abs(lam.grad.item() - go["lambda_rel"]) <= 1e-8 * abs(go["lambda_rel"])
    ref_d = np.zeros_like(d_rows)
    for i, (a0, a1) in enumerate(go["d"]):
        ref_d[off[i]:off[i + 1], 0] = a0
        ref_d[off[i]:off[i + 1], 1] = a1
    assert np.max(np.abs(d.grad.cpu().numpy() - ref_d)) <= 1e-9 * np.max(np.abs(ref_d))


def test_line_survey_refusals():
    s = CASES["even-nocut"]()
    pl, tab, clean, data, d_rows, off = _case(s)
    p = E.Plan(s)
    vel = _dev(np.asarray(s.vel, np.float64))
    g64, g32 = p.green(vel)
    d = _dev(d_rows)
    with pytest.raises(RuntimeError, match="FP64 only"):
        p.assemble(g64, g32, d, "fp16x3")
    gram, rhs, trace = p.assemble(g64, None, d, "fp64")
    with pytest.raises(RuntimeError, match="without refinement"):
        p.solve(g64, d, gram, rhs, trace, s.lambda_rel, refine=True)


def test_sampled_pairs_of_a_larger_line_survey():
    """128 lines' worth of positions (N_x = 128 at 12.5 m) on 32 lines 25 m
    apart, nz = 128, 32 frequencies 4-40 Hz, four layers, with the cut: the
    whole survey's Gram and solve on the GPU, 8 pairs (the largest by rows
    among them) against the oracle, their data from the oracle.  FP64 bar
    max(1e-10, 100 u kappa(H)) per pair (H = G + lambda I, kappa from the
    oracle's eigenvalues)."""
    s = make_lines(Nx=128, Ny=32, dx=12.5, dy=25.0, nz=128, dz=10.0, freqs=tuple(np.linspace(4.0, 40.0, 32)),
                   vel=(1600.0, 2200.0, 2900.0, 3500.0), zif=(150.0, 450.0, 900.0), kappa=1.0,
                   noise_rel=0.05, seed=7)
    p = E.Plan(s)
    off = p.rowmap()["row_off"]
    rows = np.diff(off)
    rng = np.random.default_rng(11)
    nonempty = np.nonzero(rows)[0]
    pick = sorted(set([int(np.argmax(rows))] + [int(i) for i in rng.choice(nonempty, 7, replace=False)]))
    pl = plan_lines(s, only=pick)
    assert pl.index == pick
    for q, i in zip(pl.pairs, pick):
        assert q.n_rows == rows[i]
    tab = line_tables(s)
    clean = forward_lines(s, pl, vhat(s), tab)
    data = add_noise(s, pl, clean, noise_scale(s, pl, clean))
    vel = _dev(np.asarray(s.vel, np.float64))
    g64, _ = p.green(vel, want32=False)
    d = p.forward(g64, _dev(vhat(s)))
    for q, i, (d0, d1) in zip(pl.pairs, pick, data):
        d[off[i]:off[i + 1], 0] = _dev(d0)
        d[off[i]:off[i + 1], 1] = _dev(d1)
    gram, rhs, trace = p.assemble(g64, None, d, "fp64")
    G = gram[pick].cpu().numpy()
    x, v, info, _ = p.solve(g64, d, gram, rhs, trace, s.lambda_rel)
    torch.cuda.synchronize()
    v, info = v.cpu().numpy(), info.cpu().numpy()
    low = np.tril(np.ones((s.nz, s.nz), bool))
    u = np.finfo(np.float64).eps / 2
    worst = 0.0
    for j, (q, i, (d0, d1)) in enumerate(zip(pl.pairs, pick, data)):
        A = line_row_values(s, q, tab)
        Go, _, tro = normal_equations(A, d0, d1)
        assert np.max(np.abs(G[j][low] - Go[low])) <= 1e-12 * np.max(np.abs(Go)), i
        from oracle.solve import solve_pair
        xo, info_o, lam, _ = solve_pair(s, q, A, d0, d1)
        assert info[i] == 0 and info_o == 0
        w = np.linalg.eigvalsh(Go + lam * np.eye(s.nz))
        idx = [q.u] if q.self_conjugate else [q.u, q.u_neg]
        ref = np.array([xo[0] + 1j * xo[1], xo[0] - 1j * xo[1]])[:len(idx)]
        err = np.linalg.norm(v[idx] - ref) / np.linalg.norm(ref)
        bar = max(1e-10, 100 * u * w.max() / w.min())
        assert err <= bar, (i, q.n_rows, err, bar)
        worst = max(worst, err)
    print(f"line survey 128x32, nz 128: {len(rows)} pairs, {int(rows.sum())} rows, largest {int(rows.max())}; "
          f"8 sampled pairs worst {worst:.2e}", flush=True)
    # the finite aperture over the whole survey (three chunks of pairs), the
    # sampled pairs against the oracle
    b = 0.15 * s.n_mid * s.d_mid
    Sm = window_kernel(offset_window(s, b))
    gram_w, trace_w = p.aperture_gram(g64, b)
    Gw, Tw = gram_w[pick].cpu().numpy(), trace_w[pick].cpu().numpy()
    for j, (q, i) in enumerate(zip(pl.pairs, pick)):
        A = line_row_values(s, q, tab)
        ref = (A.conj().T @ aperture_rows(s, q, A, Sm)).real
        assert np.max(np.abs(Gw[j][low] - ref[low])) <= 1e-12 * np.max(np.abs(ref)), i
        assert abs(Tw[j] - np.trace(ref)) <= 1e-12 * abs(np.trace(ref)), i
