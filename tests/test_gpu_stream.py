"""GPU: a survey solved in pair-range batches (one shared Green's table,
workspace and Gram buffer) gives the single-plan result, and the batch plans
of the largest workload (3D, 256 x 256 k_m, 96 x 96 k_h, nz = 400, 160
frequencies, 12 layers) solve sampled pairs to the oracle's bars.

Bars: FP64 <= 1e-10, mixed <= 1e-6 against the oracle (globally and per
pair); FP64 batches bit for bit equal to the single plan when both use the
same work-item shape.
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


def test_largest_workload_sampled_pairs():
    """Batch plans of the 3D 256 x 256 survey: a few seeded pairs, each planned
    as its own batch and solved with the survey's full Green's table."""
    s = make_config(5)
    rows = E.pair_rows(s)
    rng = np.random.default_rng(105)
    ok = np.flatnonzero((rows >= 500) & (rows <= 6000))
    pick = sorted(rng.choice(ok, size=3, replace=False).tolist())
    pl = oracle_plan(s, only=pick)
    assert pl.index == pick
    sub = pl.pairs
    assert [q.n_rows for q in sub] == [int(rows[i]) for i in pick]
    tabs = gtables(s, pl, pairs=sub)
    clean = forward(s, pl, vhat(s), tabs, pairs=sub)
    data = add_noise(s, pl, clean, noise_scale(s, pl, clean, pairs=sub), pairs=sub)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    for i, q, (d0, d1) in zip(pick, sub, data):
        x = solve_pair(s, q, row_values(s, q, tabs.lookup), d0, d1)[0]
        ref = x[0] + 1j * x[1]
        p = E.Plan(s, pairs=(i, i + 1))
        assert p.n_pairs == 1 and p.n_rows == q.n_rows and p.nz == 400
        d = torch.from_numpy(np.stack([d0, d1], axis=1)).cuda()
        for prec, bar in (("fp64", 1e-10), ("fp16x3", 1e-6), ("bf16x3", 1e-6)):
            pipe = E.Pipeline(p, vel, d, s.lambda_rel, prec=prec, refine_tol=3e-6, max_refine=8)
            v = pipe.step().cpu().numpy()
            e = np.linalg.norm(v[q.u] - ref) / np.linalg.norm(ref)
            if not q.self_conjugate:
                e = max(e, np.linalg.norm(v[q.u_neg] - np.conj(ref)) / np.linalg.norm(ref))
            print(f"pair {i} rows {q.n_rows} {prec}: {e:.3e}")
            assert e <= bar, (i, prec, e)
            assert int(pipe.info.cpu()[0]) == 0
            del pipe
