"""GPU: the finite-aperture Gram (edt_aperture_gram) and its damped solve
against the oracle (oracle.aperture), pair by pair.

* the windowed Gram Re(A^H S A) and its trace against the oracle's product
  with the discrete-sinc matrix, to 1e-12 of the pair's largest entry, for
  power-of-two and other line lengths (both transform paths), ragged depths,
  two half-apertures and a window holding every offset (which must give
  edt_assemble's FP64 Gram);
* the FP64 damped solve (edt_solve without refinement) on that Gram against
  the oracle's solve, to the FP64 bar 1e-10 (global and per pair), both fed
  the windowed data d_W = S d, so that the right-hand sides are the windowed
  normal equations' Re(A^H d_W);
* the paper's pairing, finite aperture with the truncated SVD at the
  binding's default step limit, from windowed data and end to end from
  records windowed in full offset (transform, gather, windowed Gram,
  truncated SVD, model);
* 3D areal surveys are refused (the survey of parallel lines is covered in
  tests/test_gpu_lines3d.py).
"""
import numpy as np
import pytest

from edt_inputs import make_config, make_custom
from oracle.aperture import aperture_data, aperture_rows, aperture_solve, offset_window, window_kernel
from oracle.solve import pack
from oracle.rows import row_values
from tests._cases import oracle_case, layered_small, rel_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")


def _cases():
    return {
        "cfg1-N64": lambda: make_config(1),
        "N48-layered": lambda: layered_small(),
        "N32-nz200": lambda: layered_small(nz=200, N=32, nf=6, seed=3),
        "N32-homogeneous": lambda: make_custom(N=32, nz=33, dx=12.5, dz=8.0, freqs=(6.0, 17.0, 29.0, 41.0),
                                               vel=(2300.0,), zif=(), noise_rel=0.05, seed=11),
    }


def _gpu(s, r, b_max, data=None):
    """Windowed Gram and trace, and edt_assemble's Gram, rhs and trace of the
    given data (default: the oracle case's unwindowed data)."""
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    g64, _ = p.green(vel, want32=False)
    rows = r["d_rows"] if data is None else pack(r["pl"], data)[0]
    d = torch.from_numpy(rows).cuda()
    gram_full, rhs, trace_full = p.assemble(g64, None, d, "fp64")
    gram, trace = p.aperture_gram(g64, b_max)
    torch.cuda.synchronize()
    return p, g64, d, gram, trace, gram_full, rhs, trace_full


@pytest.mark.parametrize("frac", [0.15, 0.3])
@pytest.mark.parametrize("name", list(_cases()))
def test_aperture_gram_and_solve(name, frac):
    s = _cases()[name]()
    r = oracle_case(s)
    b_max = frac * s.n_mid * s.d_mid / 2
    w = offset_window(s, b_max)
    assert 0 < w.sum() < s.n_mid
    Sm = window_kernel(w)
    dW = aperture_data(s, r["pl"], r["data"], b_max)
    p, g64, d, gram, trace, _, rhs, _ = _gpu(s, r, b_max, dW)
    G = gram.cpu().numpy()
    t = trace.cpu().numpy()
    low = np.tril(np.ones((s.nz, s.nz), bool))
    for q, pr in enumerate(r["pl"].pairs):
        if not pr.n_rows:
            continue
        A = row_values(s, pr, r["tabs"].lookup)
        ref = (A.conj().T @ aperture_rows(s, pr, A, Sm)).real
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(G[q][low] - ref[low])) <= 1e-12 * scale, (name, q)
        assert abs(t[q] - np.trace(ref)) <= 1e-12 * abs(np.trace(ref)), (name, q)
    x, v, info, _ = p.solve(g64, d, gram, rhs, trace, s.lambda_rel, refine=False)
    torch.cuda.synchronize()
    Vo, _ = aperture_solve(s, r["pl"], dW, r["tabs"], b_max)
    g, per = rel_errors(v.cpu().numpy(), Vo, r["pl"])
    print(f"{name} b = {b_max:.0f} m ({int(w.sum())} of {s.n_mid} offsets): solve error {g:.2e} global, {per:.2e} per pair")
    assert g <= 1e-10 and per <= 1e-10, (g, per)


def _oracle_aperture_tsvd(s, r, data, b_max, tol):
    """The oracle's truncated-SVD solution of the windowed normal equations
    (eigen-decomposition of Re(A^H S A), right-hand sides Re(A^H d_W)), and
    per pair (pair, eigenvalues, threshold)."""
    from oracle.solve import normal_equations
    from oracle.tsvd import tsvd_gram
    Sm = window_kernel(offset_window(s, b_max))
    Vo = np.zeros((r["pl"].n_km, s.nz), np.complex128)
    checks = []
    for pr, (d0, d1) in zip(r["pl"].pairs, data):
        if not pr.n_rows:
            continue
        A = row_values(s, pr, r["tabs"].lookup)
        Gw = (A.conj().T @ aperture_rows(s, pr, A, Sm)).real
        _, c, _ = normal_equations(A, d0, d1)
        x, w, t2 = tsvd_gram(Gw, c, tol)
        if pr.self_conjugate:
            x[1] = 0.0
        Vo[pr.u] = x[0] + 1j * x[1]
        if not pr.self_conjugate:
            Vo[pr.u_neg] = x[0] - 1j * x[1]
        checks.append((pr, w, t2))
    return Vo, checks


def _check_tsvd(v, info, iters, Vo, checks, what):
    """Per pair, the conditioning-derived bar of the truncated SVD (pairs
    within a relative 1e-6 of the threshold left out and counted); every
    other pair converged inside the binding's default step limit."""
    import inspect
    default_iter = inspect.signature(E.Plan.tsvd).parameters["max_iter"].default
    u = np.finfo(np.float64).eps / 2
    nv = np.linalg.norm(Vo)
    checked = ambiguous = 0
    worst, worst_bar = 0.0, 0.0
    for q, (pr, w, t2) in enumerate(checks):
        gap = np.min(np.abs(w - t2))
        if gap <= 1e-6 * t2:
            ambiguous += 1
            continue
        kept = w[w >= t2]
        bar = max(1e-10, 100 * u * (w.max() / kept.min() + w.max() / gap))
        idx = [pr.u] if pr.u == pr.u_neg else [pr.u, pr.u_neg]
        err = np.linalg.norm(v[idx] - Vo[idx]) / max(np.linalg.norm(Vo[idx]), 1e-3 * nv)
        assert err <= bar, (what, pr.u, err, bar)
        checked += 1
        worst = max(worst, err)
        worst_bar = max(worst_bar, bar)
    assert checked >= 0.9 * (checked + ambiguous) and checked > 0
    nonempty = info != -1
    assert np.all(info[nonempty] != -2) or ambiguous, "a pair away from the threshold did not converge"
    assert int(iters.max()) < default_iter
    print(f"{what}: {checked} pairs, {ambiguous} ambiguous, worst {worst:.2e}, sign steps max {int(iters.max())}")
    return worst_bar


@pytest.mark.parametrize("tol", [1e-2, 1e-3])
def test_truncated_svd_on_the_aperture_gram(tol):
    """The paper's own configuration: finite aperture and the truncated SVD
    (edt_aperture_gram -> edt_tsvd at the default step limit) on windowed data
    against the oracle's eigen-decomposition of its windowed Gram."""
    s = layered_small()
    r = oracle_case(s)
    b_max = 0.3 * s.n_mid * s.d_mid / 2
    dW = aperture_data(s, r["pl"], r["data"], b_max)
    p, g64, d, gram, trace, _, rhs, _ = _gpu(s, r, b_max, dW)
    _, v, info, iters = p.tsvd(gram, rhs, tol)
    torch.cuda.synchronize()
    Vo, checks = _oracle_aperture_tsvd(s, r, dW, b_max, tol)
    _check_tsvd(v.cpu().numpy(), info.cpu().numpy(), iters.cpu().numpy(), Vo, checks,
                f"aperture + truncated SVD tol {tol}")


def test_end_to_end_from_windowed_records():
    """Records whose transform is the oracle's noisy data, windowed in full
    offset |x_R - x_S| <= 2 b, through the GPU record transform and gather,
    the windowed Gram, the truncated SVD and the model transform, against the
    oracle's windowed data (the same window applied to the rows) solved by
    its eigen-decomposition."""
    from oracle.shots import model_from_spectrum
    s = layered_small(N=32, nz=40)
    r = oracle_case(s)
    pl = r["pl"]
    b_max = 0.3 * s.n_mid * s.d_mid / 2
    F = np.zeros((len(s.freqs), s.n_mid, s.n_mid), np.complex128)
    for p_, (d0, d1) in zip(pl.pairs, r["data"]):
        F[p_.f, p_.key0[:, 0], p_.key0[:, 1]] = d0
        F[p_.f, p_.key1[:, 0], p_.key1[:, 1]] = d1
    D = np.fft.ifft2(F, axes=(1, 2)) / s.d_mid
    R = np.arange(s.n_mid)
    D *= offset_window(s, b_max)[(R[:, None] - R[None, :]) % s.n_mid]
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    sh = torch.from_numpy(D).cuda()
    p.shots_fft(sh)
    d = p.shots_pack(sh)
    g64, _ = p.green(vel, want32=False)
    _, rhs, _ = p.assemble(g64, None, d, "fp64")
    gram, trace = p.aperture_gram(g64, b_max)
    _, v, info, iters = p.tsvd(gram, rhs, 1e-2)
    m = p.model(v)
    torch.cuda.synchronize()
    dW = aperture_data(s, pl, r["data"], b_max)
    Vo, checks = _oracle_aperture_tsvd(s, r, dW, b_max, 1e-2)
    bar = _check_tsvd(v.cpu().numpy(), info.cpu().numpy(), iters.cpu().numpy(), Vo, checks,
                      "records -> windowed Gram -> truncated SVD")
    ref = model_from_spectrum(s, Vo)
    err = np.max(np.abs(m.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print(f"end to end with the aperture: model error {err:.2e}")
    assert err <= 10 * bar


def test_window_holding_every_offset_is_the_plain_gram():
    s = layered_small()
    r = oracle_case(s)
    _, _, _, gram, trace, gram_full, _, trace_full = _gpu(s, r, 1e6)
    low = np.tril(np.ones((s.nz, s.nz), bool))
    G, Gf = gram.cpu().numpy(), gram_full.cpu().numpy()
    for q in range(G.shape[0]):
        scale = max(np.max(np.abs(Gf[q][low])), 1e-300)
        assert np.max(np.abs(G[q][low] - Gf[q][low])) <= 1e-12 * scale
    assert np.allclose(trace.cpu().numpy(), trace_full.cpu().numpy(), rtol=1e-12, atol=0)


def test_sampled_pairs_at_full_size():
    """2D N = 512, nz = 256, 128 frequencies, the paper's aperture-to-line
    ratio (b = 0.075 N dx): the Gram of 4 seeded pairs against the oracle."""
    from oracle.rows import plan as oracle_plan
    from oracle.solve import gtables
    s = make_config(2)
    pl = oracle_plan(s)
    rng = np.random.default_rng(9)
    nonempty = [i for i, q in enumerate(pl.pairs) if q.n_rows > 0]
    pick = sorted(rng.choice(nonempty, size=4, replace=False).tolist())
    sub = [pl.pairs[i] for i in pick]
    tabs = gtables(s, pl, pairs=sub)
    b_max = 0.075 * s.n_mid * s.d_mid
    Sm = window_kernel(offset_window(s, b_max))
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    g64, _ = p.green(vel, want32=False)
    gram, trace = p.aperture_gram(g64, b_max)
    torch.cuda.synchronize()
    low = np.tril(np.ones((s.nz, s.nz), bool))
    for i, pr in zip(pick, sub):
        A = row_values(s, pr, tabs.lookup)
        ref = (A.conj().T @ aperture_rows(s, pr, A, Sm)).real
        G = gram[i].cpu().numpy()
        assert np.max(np.abs(G[low] - ref[low])) <= 1e-12 * np.max(np.abs(ref)), i


def test_3d_areal_surveys_are_refused():
    s = make_custom(dim=3, N=12, Nh=6, nz=5, dx=25.0, freqs=(5.0,), vel=(2000.0,))
    p = E.Plan(s)
    g64 = torch.zeros(1, 1, 5, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="2D line survey"):
        p.aperture_gram(g64, 100.0)


def test_bad_half_aperture_is_refused():
    s = layered_small()
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    g64, _ = p.green(vel, want32=False)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(RuntimeError, match="b_max"):
            p.aperture_gram(g64, bad)

