"""GPU parity of the HIP path against the FP64 oracle, through the C-ABI.

Bars: FP64 path <= 1e-10 relative, mixed precision (FP32 or
BF16x3 Gram + FP64 Cholesky + FP64 refinement) <= 1e-6 relative, both as a
global Frobenius ratio and per +-k_m pair (floor 1e-3 of the largest pair).
Intermediate tables, Grams and data are checked at FP64 rounding level.
"""
import numpy as np
import pytest

from edt_inputs import make_config, make_custom, vhat
from oracle.green import green, omega
from oracle.solve import normal_equations
from oracle.rows import row_values
from tests._cases import oracle_case, rel_errors, layered_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _vel(s):
    return _dev(np.asarray(s.vel, np.float64))


def _cases():
    return {
        "cfg1": lambda: make_config(1),
        "layered-nz40": lambda: layered_small(),
        "layered-nz200": lambda: layered_small(nz=200, N=32, nf=6, seed=3),
        # past one 256-depth super-block: a 1-depth second block, and a ragged one
        "layered-nz257": lambda: layered_small(nz=257, N=16, nf=4, seed=4),
        "layered-nz400": lambda: layered_small(nz=400, N=24, nf=5, seed=6, dz=5.0),
        # one layer: the Green's function is the closed form exp(i k_z |z|) i / (2 k_z)
        "homogeneous": lambda: make_custom(N=32, nz=33, dx=12.5, dz=8.0, freqs=(6.0, 17.0, 29.0, 41.0),
                                           vel=(2300.0,), zif=(), noise_rel=0.05, seed=11),
        "3d-small": lambda: make_custom(dim=3, N=12, Nh=6, nz=37, dx=25.0, dz=10.0,
                                        freqs=(8.0, 14.0, 20.0), vel=(1800.0, 2500.0, 2100.0),
                                        zif=(60.0, 200.0), noise_rel=0.05, seed=5),
    }


@pytest.fixture(scope="module")
def refs():
    return {k: (f(), None) for k, f in _cases().items()}


def _ref(refs, name):
    s, r = refs[name]
    if r is None:
        r = oracle_case(s)
        refs[name] = (s, r)
    return s, r


@pytest.mark.parametrize("name", ["cfg1", "layered-nz40", "homogeneous", "3d-small"])
def test_green_tables(refs, name):
    s, r = _ref(refs, name)
    p = E.Plan(s)
    g64, g32 = p.green(_vel(s))
    torch.cuda.synchronize()
    g64 = g64.cpu().numpy()
    g32 = g32.cpu().numpy()
    cls_k = p.rowmap()["cls_k"]
    for f in range(s.n_freq):
        w = omega(s.freqs[f], s.eps)
        ref = green(s.vel, s.zif, w, cls_k, s.z)
        sc = np.max(np.abs(ref), axis=1, keepdims=True)
        assert np.max(np.abs(g64[f] - ref) / sc) <= 1e-12
        ref32 = ref * (abs(w) * np.sqrt(s.dz))
        sc32 = np.max(np.abs(ref32), axis=1, keepdims=True)
        assert np.max(np.abs(g32[f] - ref32) / sc32) <= 2e-6


@pytest.mark.parametrize("name", ["cfg1", "layered-nz40", "3d-small"])
def test_forward_born_rows(refs, name):
    s, r = _ref(refs, name)
    p = E.Plan(s)
    g64, _ = p.green(_vel(s), want32=False)
    d = p.forward(g64, _dev(vhat(s)))
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    clean = np.zeros_like(d)
    for i, (d0, d1) in enumerate(r["clean"]):
        clean[r["off"][i]:r["off"][i + 1], 0] = d0
        clean[r["off"][i]:r["off"][i + 1], 1] = d1
    assert np.max(np.abs(d - clean)) <= 1e-12 * np.max(np.abs(clean))


@pytest.mark.parametrize("name", ["cfg1", "layered-nz40", "homogeneous", "layered-nz200", "layered-nz257",
                                  "layered-nz400", "3d-small"])
def test_fp64_gram_rhs_trace(refs, name):
    s, r = _ref(refs, name)
    p = E.Plan(s)
    g64, _ = p.green(_vel(s), want32=False)
    gram, rhs, trace = p.assemble(g64, None, _dev(r["d_rows"]), "fp64")
    torch.cuda.synchronize()
    gram, rhs, trace = gram.cpu().numpy(), rhs.cpu().numpy(), trace.cpu().numpy()
    low = np.tril(np.ones((s.nz, s.nz), bool))
    for i, q in enumerate(r["pl"].pairs):
        if q.n_rows == 0:
            continue
        A = row_values(s, q, r["tabs"].lookup)
        G, c, tr = normal_equations(A, *r["data"][i])
        assert np.max(np.abs(gram[i][low] - G[low])) <= 1e-12 * np.max(np.abs(G))
        assert np.max(np.abs(rhs[i] - c)) <= 1e-12 * np.max(np.abs(c))
        assert abs(trace[i] - tr) <= 1e-12 * tr


@pytest.mark.parametrize("name", ["cfg1", "layered-nz40", "homogeneous", "layered-nz200", "layered-nz257",
                                  "layered-nz400", "3d-small"])
def test_fp64_solve(refs, name):
    s, r = _ref(refs, name)
    p = E.Plan(s)
    out = p.run(_vel(s), _dev(r["d_rows"]), s.lambda_rel, prec="fp64")
    torch.cuda.synchronize()
    g, per = rel_errors(out["v"].cpu().numpy(), r["V"], r["pl"])
    assert g <= 1e-10 and per <= 1e-10, (g, per)
    info = out["info"].cpu().numpy()
    for q, inf in zip(r["pl"].pairs, info):
        assert inf == (-1 if q.n_rows == 0 else 0)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3", "fp32"])
@pytest.mark.parametrize("name", ["cfg1", "layered-nz40", "homogeneous", "layered-nz200", "layered-nz257",
                                  "layered-nz400", "3d-small"])
def test_mixed_solve_with_refinement(refs, name, prec):
    s, r = _ref(refs, name)
    if prec == "fp32" and s.nz > 256:
        pytest.skip("the FP32 Gram covers nz <= 256 (rejected with EINVAL, tested below)")
    p = E.Plan(s)
    out = p.run(_vel(s), _dev(r["d_rows"]), s.lambda_rel, prec=prec, refine_tol=1e-9, max_refine=10)
    torch.cuda.synchronize()
    g, per = rel_errors(out["v"].cpu().numpy(), r["V"], r["pl"])
    assert g <= 1e-6 and per <= 1e-6, (g, per)
    info = out["info"].cpu().numpy()
    assert np.all((info == 0) | (info == -1))
    steps = out["steps"].cpu().numpy()
    print(name, prec, "global", g, "pair", per, "steps max", steps.max(), "mean", steps.mean())


@pytest.mark.parametrize("name", ["layered-nz40", "layered-nz400"])
def test_mixed_gram_is_close_to_fp64(refs, name):
    s, r = _ref(refs, name)
    p = E.Plan(s)
    g64, g32 = p.green(_vel(s))
    d = _dev(r["d_rows"])
    G64 = p.assemble(g64, g32, d, "fp64")[0].cpu().numpy()
    Gb = p.assemble(g64, g32, d, "bf16x3")[0].cpu().numpy()
    Gh = p.assemble(g64, g32, d, "fp16x3")[0].cpu().numpy()
    Gf = p.assemble(g64, g32, d, "fp32")[0].cpu().numpy() if s.nz <= 256 else G64
    low = np.tril(np.ones((s.nz, s.nz), bool))
    for i in range(G64.shape[0]):
        sc = np.max(np.abs(G64[i]))
        if sc == 0:
            continue
        assert np.max(np.abs(Gb[i][low] - G64[i][low])) <= 1e-4 * sc
        assert np.max(np.abs(Gh[i][low] - G64[i][low])) <= 1e-5 * sc
        assert np.max(np.abs(Gf[i][low] - G64[i][low])) <= 1e-5 * sc


@pytest.mark.parametrize("opts", [dict(chunk_rows=16, gram_band=1), dict(chunk_rows=5, gram_band=2)])
def test_fp64_assemble_with_small_banded_items(refs, opts):
    """Many items per pair (one or two frequencies, a few rows each) and an
    XCD schedule with holes give the same Gram, rhs and trace."""
    s, r = _ref(refs, "layered-nz40")
    p = E.Plan(s, **opts)
    items, sched = p.schedule("gram")
    assert len(items) > 4 * p.n_pairs and np.any(sched < 0)
    g64, _ = p.green(_vel(s), want32=False)
    gram, rhs, trace = p.assemble(g64, None, _dev(r["d_rows"]), "fp64")
    torch.cuda.synchronize()
    gram, rhs, trace = gram.cpu().numpy(), rhs.cpu().numpy(), trace.cpu().numpy()
    low = np.tril(np.ones((s.nz, s.nz), bool))
    for i, q in enumerate(r["pl"].pairs):
        if q.n_rows == 0:
            continue
        A = row_values(s, q, r["tabs"].lookup)
        G, c, tr = normal_equations(A, *r["data"][i])
        assert np.max(np.abs(gram[i][low] - G[low])) <= 1e-12 * np.max(np.abs(G))
        assert np.max(np.abs(rhs[i] - c)) <= 1e-12 * np.max(np.abs(c))
        assert abs(trace[i] - tr) <= 1e-12 * tr
    out = p.run(_vel(s), _dev(r["d_rows"]), s.lambda_rel, prec="bf16x3", refine_tol=1e-9, max_refine=10)
    g, per = rel_errors(out["v"].cpu().numpy(), r["V"], r["pl"])
    assert g <= 1e-6 and per <= 1e-6, (g, per)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3", "fp32"])
def test_mixed_rhs_and_trace(refs, prec):
    """FP32/BF16x3 assembly: the trace (which fixes lambda) is FP32 rows summed
    in FP64, within 1e-7 of FP64; the right-hand side is an FP32 estimate that
    the FP64 refinement residual corrects."""
    s, r = _ref(refs, "layered-nz200")
    p = E.Plan(s)
    g64, g32 = p.green(_vel(s))
    d = _dev(r["d_rows"])
    _, c64, t64 = p.assemble(g64, g32, d, "fp64")
    _, cm, tm = p.assemble(g64, g32, d, prec)
    c64, t64, cm, tm = (a.cpu().numpy() for a in (c64, t64, cm, tm))
    ok = t64 > 0
    assert np.all(np.abs(tm[ok] - t64[ok]) <= 1e-7 * t64[ok])
    for i in np.flatnonzero(ok):
        assert np.max(np.abs(cm[i] - c64[i])) <= 1e-4 * np.max(np.abs(c64[i]))


def test_bf16x3_pivot_failure_escalates_to_fp64(refs):
    """nz = 400 with few rows: lambda is below the BF16x3 Gram error for one
    pair, whose factorisation fails (info = failing column).  Without
    escalation the failure is reported; with it that pair is re-assembled in
    FP64 and every pair meets the mixed-precision bar."""
    s, r = _ref(refs, "layered-nz400")
    p = E.Plan(s)
    vel = _vel(s)
    d = _dev(r["d_rows"])
    g64, g32 = p.green(vel)
    gram, rhs, trace = p.assemble(g64, g32, d, "bf16x3")
    _, _, info0, _ = p.solve(g64, d, gram.clone(), rhs, trace, s.lambda_rel, refine=True, refine_tol=1e-9,
                             max_refine=10, escalate=False)
    info0 = info0.cpu().numpy()
    assert np.any(info0 > 0), "expected a failed BF16x3 factorisation in this case"
    _, v, info1, _ = p.solve(g64, d, gram.clone(), rhs, trace, s.lambda_rel, refine=True, refine_tol=1e-9,
                             max_refine=10, escalate=True)
    info1 = info1.cpu().numpy()
    assert np.all((info1 == 0) | (info1 == -1))
    g, per = rel_errors(v.cpu().numpy(), r["V"], r["pl"])
    assert g <= 1e-6 and per <= 1e-6, (g, per)


@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3"])
def test_solve_reuses_the_data_sums_of_assemble(refs, prec):
    """edt_solve with data_summed takes the data sums that edt_assemble left in
    the workspace: the same refined result, bit for bit, as summing again."""
    s, r = _ref(refs, "layered-nz257")
    p = E.Plan(s)
    vel = _vel(s)
    d = _dev(r["d_rows"])
    g64, g32 = p.green(vel)
    gram, rhs, trace = p.assemble(g64, g32, d, prec)
    x0, v0, i0, s0 = p.solve(g64, d, gram.clone(), rhs, trace, s.lambda_rel, refine=True, refine_tol=1e-9,
                             max_refine=10)
    gram, rhs, trace = p.assemble(g64, g32, d, prec)
    x1, v1, i1, s1 = p.solve(g64, d, gram, rhs, trace, s.lambda_rel, refine=True, refine_tol=1e-9,
                             max_refine=10, data_summed=True)
    for a, b in ((x0, x1), (v0, v1), (i0, i1), (s0, s1)):
        assert torch.equal(a, b)
    g, per = rel_errors(v1.cpu().numpy(), r["V"], r["pl"])
    assert g <= 1e-6 and per <= 1e-6, (g, per)


def test_depth_limits(refs):
    """nz > 256 is served by FP64 and the split Grams; FP32 and the adjoint
    reject it, and nz > 448 is rejected at every entry point."""
    s, r = _ref(refs, "layered-nz400")
    p = E.Plan(s)
    g64, g32 = p.green(_vel(s))
    with pytest.raises(RuntimeError, match="FP32 Gram"):
        p.assemble(g64, g32, _dev(r["d_rows"]), "fp32")
    big = layered_small(nz=449, N=4, nf=2, seed=1)
    pb = E.Plan(big)
    with pytest.raises(RuntimeError, match="nz > 448"):
        pb.green(_vel(big))


def test_empty_and_nonfinite_and_singular():
    s = make_custom(N=64, nz=6, dx=25.0, freqs=(2.0, 3.0), vel=(2500.0,), noise_rel=0.0, seed=2)
    r = oracle_case(s)
    p = E.Plan(s)
    assert p.info["n_empty"] > 0
    out = p.run(_vel(s), _dev(r["d_rows"]), s.lambda_rel)
    info = out["info"].cpu().numpy()
    v = out["v"].cpu().numpy()
    for q, inf in zip(r["pl"].pairs, info):
        if q.n_rows == 0:
            assert inf == -1 and not np.any(v[q.u]) and not np.any(v[q.u_neg])
    # a NaN datum poisons only its own pair, which is flagged
    d = r["d_rows"].copy()
    q = next(i for i, q in enumerate(r["pl"].pairs) if q.n_rows > 0)
    d[r["off"][q], 0] = np.nan
    info2 = p.run(_vel(s), _dev(d), s.lambda_rel)["info"].cpu().numpy()
    assert info2[q] != 0
    others = [i for i in range(len(info2)) if i != q]
    assert np.array_equal(info2[others], info[others])
    # an indefinite system: the factorisation reports the failing pivot
    g64, _ = p.green(_vel(s), want32=False)
    gram, rhs, trace = p.assemble(g64, None, _dev(r["d_rows"]), "fp64")
    eye = torch.eye(s.nz, dtype=torch.float64, device="cuda")
    gram[:] = -eye
    gram[:, 2, 2] = 5.0
    x, v, inf, _ = p.solve(g64, _dev(r["d_rows"]), gram, rhs, torch.ones_like(trace), 0.0)
    inf = inf.cpu().numpy()
    nonempty = np.diff(p.rowmap()["row_off"]) > 0
    assert np.all(inf[nonempty] == 1)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_bitwise_deterministic(refs, prec):
    s, r = _ref(refs, "layered-nz40")
    p = E.Plan(s)
    a = p.run(_vel(s), _dev(r["d_rows"]), s.lambda_rel, prec=prec)["v"].cpu().numpy()
    b = p.run(_vel(s), _dev(r["d_rows"]), s.lambda_rel, prec=prec)["v"].cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_forward_adjoint_dot_product(refs):
    # <A v, d> = <v, A^H d> where A^H d is read off the FP64 right-hand sides:
    # rhs = Re(A^H b+-) with b+ = (d0+d1)/2, b- = (d0-d1)/(2i)
    s, r = _ref(refs, "layered-nz40")
    p = E.Plan(s)
    g64, _ = p.green(_vel(s), want32=False)
    rng = np.random.default_rng(0)
    P = p.n_pairs
    pk = p.rowmap()["pair_km"]
    # a model spectrum that is the transform of a real field
    v = np.fft.fft(rng.normal(size=(s.n_mid, s.nz)), axis=0)
    dd = rng.normal(size=(p.n_rows, 2)) + 1j * rng.normal(size=(p.n_rows, 2))
    fwd = p.forward(g64, _dev(v)).cpu().numpy()
    _, rhs, _ = p.assemble(g64, None, _dev(dd), "fp64")
    rhs = rhs.cpu().numpy()
    lhs = 0.0
    rhs_sum = 0.0
    for i in range(P):
        a, b = r["off"][i], r["off"][i + 1]
        u0, u1 = pk[i]
        # Re sum conj(d) A v over both data columns
        lhs += np.real(np.sum(np.conj(dd[a:b, 0]) * fwd[a:b, 0]) + np.sum(np.conj(dd[a:b, 1]) * fwd[a:b, 1]))
        xp, xm = v[u0].real, v[u0].imag
        # A v(u) = A (x+ + i x-), A v(-u) = A (x+ - i x-): <d, A v> = 2 <b+, A x+> + 2 <b-, A x->
        rhs_sum += 2.0 * (xp @ rhs[i, 0] + xm @ rhs[i, 1])
    assert abs(lhs - rhs_sum) <= 1e-12 * abs(lhs)


def test_adjoint_matches_oracle_gradient():
    from oracle.grad import grad
    s = layered_small(nz=24, N=24, nf=6, seed=4)
    r = oracle_case(s)
    rng = np.random.default_rng(1)
    T = rng.normal(size=(s.n_mid, s.nz)) + 1j * rng.normal(size=(s.n_mid, s.nz))
    gV = 2.0 * (r["V"] - T)
    go = grad(s, r["pl"], r["data"], gV)
    p = E.Plan(s)
    vel = _vel(s)
    d = _dev(r["d_rows"])
    out = p.run(vel, d, s.lambda_rel, prec="fp64")
    gd, gl, gvel = p.adjoint(vel, out["g64"], d, out["gram"], out["trace"], out["x"], s.lambda_rel, _dev(gV))
    torch.cuda.synchronize()
    gd = gd.cpu().numpy()
    ref_d = np.zeros_like(gd)
    for i, (a0, a1) in enumerate(go["d"]):
        ref_d[r["off"][i]:r["off"][i + 1], 0] = a0
        ref_d[r["off"][i]:r["off"][i + 1], 1] = a1
    assert np.max(np.abs(gd - ref_d)) <= 1e-9 * np.max(np.abs(ref_d))
    assert abs(gl.item() - go["lambda_rel"]) <= 1e-8 * abs(go["lambda_rel"])
    gv = gvel.cpu().numpy()
    assert np.max(np.abs(gv - go["vel"])) <= 1e-8 * np.max(np.abs(go["vel"])), (gv, go["vel"])
