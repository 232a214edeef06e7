"""GPU: a survey solved in pair-range batches (one shared Green's table,
workspace and Gram buffer) gives the single-plan result, and the batch plans
of the largest workload (3D, 256 x 256 k_m, 96 x 96 k_h, nz = 400, 160
frequencies, 12 layers) solve sampled pairs to the oracle's bars.

Bars: FP64 <= 1e-10, mixed <= 1e-6 against the oracle (globally and per
pair); FP64 batches bit for bit equal to the single plan when both use the
same work-item shape.  A pair whose damped matrix H = G + lambda I is so ill
conditioned that two FP64 computations differ by more than 1e-10 (the
largest pairs of the 3D 256 x 256 survey: kappa(H) ~ 3e5, and two summation
orders of the oracle's own Gram give solutions 4e-10 apart) takes the
conditioning-derived FP64 bar max(1e-10, 100 u kappa(H)).
"""
import numpy as np
import pytest

from edt_inputs import make_config, make_custom, vhat
from oracle.rows import plan as oracle_plan, row_values
from oracle.solve import gtables, forward, noise_scale, add_noise, solve_pair
from tests._cases import oracle_case, rel_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")


def _survey():
    return make_custom(dim=3, N=12, Nh=6, nz=37, dx=25.0, dz=10.0, freqs=(8.0, 14.0, 20.0),
                       vel=(1800.0, 2500.0, 2100.0), zif=(60.0, 200.0), noise_rel=0.05, seed=5)


@pytest.fixture(scope="module")
def case():
    s = _survey()
    return s, oracle_case(s)


def _stream(s, r, prec, **kw):
    st = E.Stream(s, prec=prec, refine_tol=1e-9, max_refine=10, batch_pairs=8, threads=4, **kw)
    off = np.zeros(len(r["pl"].pairs) + 1, np.int64)
    off[1:] = np.cumsum([q.n_rows for q in r["pl"].pairs])
    for b, (a, e) in enumerate(st.batches):
        st.set_data(b, torch.from_numpy(r["d_rows"][off[a]:off[e]]))
    return st


def test_fp64_batches_equal_the_single_plan_bitwise(case):
    s, r = case
    st = _stream(s, r, "fp64", chunk_rows=64, gram_band=1)
    assert len(st.batches) >= 3
    v = st.step().cpu().numpy()
    p = E.Plan(s, chunk_rows=64, gram_band=1)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    pipe = E.Pipeline(p, vel, torch.from_numpy(r["d_rows"]).cuda(), s.lambda_rel, "fp64")
    v1 = pipe.step().cpu().numpy()
    assert np.array_equal(v, v1)
    assert np.array_equal(st.x.cpu().numpy(), pipe.x.cpu().numpy())
    assert np.array_equal(st.info.cpu().numpy(), pipe.info.cpu().numpy())
    g, per = rel_errors(v, r["V"], r["pl"])
    assert g <= 1e-10 and per <= 1e-10, (g, per)


@pytest.mark.parametrize("prec", ["fp16x3", "bf16x3"])
def test_mixed_batches_meet_the_bar_and_replay(case, prec):
    s, r = case
    st = _stream(s, r, prec)
    v = st.step().cpu().numpy()
    g, per = rel_errors(v, r["V"], r["pl"])
    assert g <= 1e-6 and per <= 1e-6, (g, per)
    info = st.info.cpu().numpy()
    assert np.all((info == 0) | (info == -1))
    st.capture()
    for _ in range(3):
        st.v.zero_()
        vr = st.replay().cpu().numpy()
        assert np.array_equal(vr, v)


def _bf16x3_indefinite(s, cand, k):
    """Up to k of the candidate pairs whose damped Gram, formed from rows split
    into bfloat16 halves (hi^T hi + hi^T lo + lo^T hi, the BF16x3 product), is
    not positive definite: a single-row pair's Gram is a rank-one a a^T, and
    the dropped lo lo^T term (about 2^-16 |a|^2) can exceed the damping
    lambda = 1e-3 |a|^2 / nz, so its BF16x3 factorisation fails and the solve
    must re-assemble it in FP64.  A CPU model of the split used to pick test
    pairs; the expected values still come from the oracle."""
    cand = sorted(int(i) for i in cand)
    pl = oracle_plan(s, only=cand)
    tabs = gtables(s, pl)
    scored = []
    for i, q in zip(cand, pl.pairs):
        A = row_values(s, q, tabs.lookup)
        R = np.concatenate([A.real, A.imag]).astype(np.float32)
        R = R * np.float32(2.0 ** -np.floor(np.log2(np.abs(R).max())))
        h = torch.from_numpy(R).to(torch.bfloat16).to(torch.float32).numpy()
        lo = torch.from_numpy(R - h).to(torch.bfloat16).to(torch.float32).numpy()
        h, lo, R = h.astype(np.float64), lo.astype(np.float64), R.astype(np.float64)
        G3 = h.T @ h + h.T @ lo + lo.T @ h
        lam = s.lambda_rel * np.trace(R.T @ R) / s.nz
        w0 = np.linalg.eigvalsh(G3 + lam * np.eye(s.nz))[0]
        if w0 <= 0:
            scored.append((w0 / lam, i))
    return [i for _, i in sorted(scored)[:k]]


@pytest.mark.parametrize("band", ["mid", "top", "small"])
def test_largest_workload_sampled_pairs(band):
    """Batch plans of the 3D 256 x 256 survey: seeded pairs, each planned as
    its own batch and solved with the survey's full Green's table, from three
    parts of the row distribution: mid-sized pairs (500 to 6000 rows), the
    top 1% by rows with the largest pair, and pairs with fewer rows than
    depths, where the damping can fall below the BF16x3 Gram's error and the
    solve re-assembles the pair in FP64 (escalation)."""
    s = make_config(5)
    rows = E.pair_rows(s)
    rng = np.random.default_rng(105)
    if band == "mid":
        pick = rng.choice(np.flatnonzero((rows >= 500) & (rows <= 6000)), size=3, replace=False).tolist()
    elif band == "top":
        top = np.flatnonzero(rows >= np.quantile(rows, 0.99))
        pick = rng.choice(top, size=2, replace=False).tolist() + [int(np.argmax(rows))]
    else:
        pick = rng.choice(np.flatnonzero((rows >= 1) & (rows <= 100)), size=12, replace=False).tolist()
        pick += _bf16x3_indefinite(s, rng.choice(np.flatnonzero(rows == 1), size=40, replace=False), 4)
    pick = sorted(set(int(i) for i in pick))
    pl = oracle_plan(s, only=pick)
    assert pl.index == pick
    sub = pl.pairs
    assert [q.n_rows for q in sub] == [int(rows[i]) for i in pick]
    print(f"{band}: pairs {pick}, rows {[q.n_rows for q in sub]}", flush=True)
    tabs = gtables(s, pl, pairs=sub)
    clean = forward(s, pl, vhat(s), tabs, pairs=sub)
    data = add_noise(s, pl, clean, noise_scale(s, pl, clean, pairs=sub), pairs=sub)
    del clean
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    escalated = 0
    u = np.finfo(np.float64).eps / 2
    for i, q, (d0, d1) in zip(pick, sub, data):
        x, _, lam, _, G = solve_pair(s, q, row_values(s, q, tabs.lookup), d0, d1, return_gram=True)
        w = np.linalg.eigvalsh(G + lam * np.eye(s.nz))
        kappa = w[-1] / w[0]
        del G
        ref = x[0] + 1j * x[1]
        p = E.Plan(s, pairs=(i, i + 1))
        assert p.n_pairs == 1 and p.n_rows == q.n_rows and p.nz == 400
        d = torch.from_numpy(np.stack([d0, d1], axis=1)).cuda()
        for prec, bar in (("fp64", max(1e-10, 100 * u * kappa)), ("fp16x3", 1e-6), ("bf16x3", 1e-6)):
            pipe = E.Pipeline(p, vel, d, s.lambda_rel, prec=prec, refine_tol=3e-6, max_refine=8)
            v = pipe.step().cpu().numpy()
            e = np.linalg.norm(v[q.u] - ref) / np.linalg.norm(ref)
            if not q.self_conjugate:
                e = max(e, np.linalg.norm(v[q.u_neg] - np.conj(ref)) / np.linalg.norm(ref))
            line = f"pair {i} rows {q.n_rows} kappa {kappa:.2e} {prec}: {e:.3e} (bar {bar:.1e}) " \
                   f"sweeps {int(pipe.steps.cpu()[0])}"
            if prec == "bf16x3":
                # the same factorisation without escalation: a non-positive
                # pivot (info > 0) means the pair above was re-assembled in FP64
                g0, r0, t0 = p.assemble(pipe.G64, pipe.G32, pipe.d, "bf16x3")
                _, _, info0, _ = p.solve(pipe.G64, pipe.d, g0, r0, t0, s.lambda_rel, refine=True,
                                         refine_tol=3e-6, max_refine=8, escalate=False)
                esc = int(info0.cpu()[0]) > 0
                escalated += esc
                line += " (escalated)" if esc else ""
            print(line, flush=True)
            assert e <= bar, (i, prec, e)
            assert int(pipe.info.cpu()[0]) == 0
            del pipe
    print(f"{band}: {escalated} of {len(sub)} pairs escalated under BF16x3", flush=True)
    if band == "small":
        assert escalated >= 1   # the escalation path of the largest workload ran
