"""GPU tests of the differentiable solve (torch.autograd.Function over the
hand-written adjoint) and of the HIP-graph capture of a full pass.

* EDTSolve's gradients equal the FP64 oracle gradient (adjoint of the normal
  equations plus tangent-mode Green's functions) on a small layered survey,
  on sampled pairs of the 2D gradient workload, and at depth counts that
  take every variant of the velocity-gradient table kernel.
* On the 2D gradient workload (512 traces, nz = 128, 64 frequencies) the
  gradients with respect to every layer velocity, lambda_rel and sampled data
  entries equal central finite differences (h = 1e-6 relative) of the same
  FP64 GPU forward, to 1e-4.
* A captured pass replays bit for bit like the eager pass, with the
  program's own eager work and synchronisations between the replays.
"""
import numpy as np
import pytest

from edt_inputs import make_config, noise, vhat
from tests._cases import oracle_case, rel_errors, layered_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_autograd_matches_oracle_gradient():
    from oracle.grad import grad
    s = layered_small(nz=24, N=24, nf=6, seed=4)
    r = oracle_case(s)
    rng = np.random.default_rng(1)
    T = rng.normal(size=(s.n_mid, s.nz)) + 1j * rng.normal(size=(s.n_mid, s.nz))
    go = grad(s, r["pl"], r["data"], 2.0 * (r["V"] - T))
    p = E.Plan(s)
    d = _dev(r["d_rows"]).requires_grad_(True)
    lam = torch.tensor(s.lambda_rel, dtype=torch.float64, device="cuda", requires_grad=True)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda", requires_grad=True)
    V = E.edt_solve(d, lam, vel, p)
    g, per = rel_errors(V.detach().cpu().numpy(), r["V"], r["pl"])
    assert g <= 1e-10 and per <= 1e-10
    loss = (V - _dev(T)).abs().pow(2).sum()
    loss.backward()
    gd = d.grad.cpu().numpy()
    ref_d = np.zeros_like(gd)
    for i, (a0, a1) in enumerate(go["d"]):
        ref_d[r["off"][i]:r["off"][i + 1], 0] = a0
        ref_d[r["off"][i]:r["off"][i + 1], 1] = a1
    assert np.max(np.abs(gd - ref_d)) <= 1e-9 * np.max(np.abs(ref_d))
    assert abs(lam.grad.item() - go["lambda_rel"]) <= 1e-8 * abs(go["lambda_rel"])
    gv = vel.grad.cpu().numpy()
    assert np.max(np.abs(gv - go["vel"])) <= 1e-8 * np.max(np.abs(go["vel"]))


def _sampled_case(s, n_sample, seed):
    """Oracle data of a seeded sample of non-empty pairs, the loss target on
    their k_m and the oracle gradient of L = sum over the sample's k_m of
    |V~ - T|^2.  Pairs outside the sample get zero data and no loss: they
    add nothing to any gradient, so the sample's oracle gradient is the
    whole gradient."""
    from oracle.grad import grad
    from oracle.rows import plan as oplan
    from oracle.solve import gtables, forward, noise_scale, add_noise, solve
    counts = E.pair_rows(s)
    rng = np.random.default_rng(seed)
    nonempty = np.nonzero(counts > 0)[0]
    pick = nonempty if n_sample >= nonempty.size else np.sort(np.concatenate(
        [[nonempty[np.argmax(counts[nonempty])]],
         rng.choice(nonempty, size=n_sample - 1, replace=False)]))
    pick = np.unique(pick)
    sub = oplan(s, only=pick.tolist())
    tabs = gtables(s, sub)
    clean = forward(s, sub, vhat(s), tabs)
    data = add_noise(s, sub, clean, noise_scale(s, sub, clean))
    V, _ = solve(s, sub, data, tabs)
    T = vhat(s) * (1.0 + 0.1 * rng.normal(size=vhat(s).shape))
    mask = np.zeros(V.shape[0], bool)
    for q in sub.pairs:
        mask[q.u] = mask[q.u_neg] = True
    gV = np.where(mask[:, None], 2.0 * (V - T), 0.0)
    go = grad(s, sub, data, gV)
    return sub, data, V, T, mask, go


@pytest.mark.parametrize("name,n_sample", [
    # the 2D gradient workload (512 traces, nz = 128, 64 frequencies): table
    # kernel with 2 depths per lane
    ("cfg3", 16),
    # nz in (128, 192] and (192, 256]: 3 and 4 depths per lane
    ("nz160", 64), ("nz224", 64)])
def test_adjoint_matches_oracle_gradient_at_size(name, n_sample):
    s = {"cfg3": lambda: make_config(3),
         "nz160": lambda: layered_small(nz=160, N=32, nf=5, seed=8),
         "nz224": lambda: layered_small(nz=224, N=24, nf=4, seed=9)}[name]()
    print(f"adjoint vs oracle gradient: {name}, nz={s.nz}", flush=True)
    sub, data, Vo, T, mask, go = _sampled_case(s, n_sample, seed=5)
    p = E.Plan(s)
    off = p.rowmap()["row_off"]
    d0 = np.zeros((p.n_rows, 2), np.complex128)
    for i, (a0, a1) in zip(sub.index, data):
        assert off[i + 1] - off[i] == a0.shape[0]
        d0[off[i]:off[i + 1], 0] = a0
        d0[off[i]:off[i + 1], 1] = a1
    d = _dev(d0).requires_grad_(True)
    lam = torch.tensor(s.lambda_rel, dtype=torch.float64, device="cuda", requires_grad=True)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda", requires_grad=True)
    V = E.edt_solve(d, lam, vel, p)
    Vg = V.detach().cpu().numpy()
    assert np.max(np.abs(Vg[mask] - Vo[mask])) <= 1e-10 * np.max(np.abs(Vo[mask]))
    m = _dev(mask.astype(np.float64))[:, None]
    loss = ((V - _dev(T)).abs().pow(2) * m).sum()
    loss.backward()
    gd = d.grad.cpu().numpy()
    ref_d = np.zeros_like(gd)
    for i, (a0, a1) in zip(sub.index, go["d"]):
        ref_d[off[i]:off[i + 1], 0] = a0
        ref_d[off[i]:off[i + 1], 1] = a1
    e_d = np.max(np.abs(gd - ref_d)) / np.max(np.abs(ref_d))
    # dL/dlambda_p = -y.x is a dot product whose terms can cancel (pairs with
    # far fewer rows than depths): its rounding error is relative to
    # sum |y x|, not to the result
    e_l = abs(lam.grad.item() - go["lambda_rel"]) / np.sum(go["lambda_abs"])
    gv = vel.grad.cpu().numpy()
    e_v = np.max(np.abs(gv - go["vel"])) / np.max(np.abs(go["vel"]))
    print(f"  pairs {len(sub.pairs)}: grad_d {e_d:.2e}, grad_lambda {e_l:.2e} "
          f"(cancellation {np.sum(go['lambda_abs']) / abs(go['lambda_rel']):.1f}), grad_vel {e_v:.2e}", flush=True)
    assert e_d <= 1e-8 and e_l <= 1e-10 and e_v <= 1e-8


def _synthetic_rows(s, p):
    """Data rows of the survey's model from the FP64 forward map plus the
    counter-based noise (an input, not an expected value)."""
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    g64, _ = p.green(vel, want32=False)
    d = p.forward(g64, _dev(vhat(s))).cpu().numpy()
    m = p.rowmap()
    f = m["rows"][:, 0].astype(np.int64)
    mx = np.zeros(s.n_freq)
    np.maximum.at(mx, f, np.maximum(np.abs(d[:, 0]), np.abs(d[:, 1])))
    keys = m["keys"].astype(np.int64)
    N = s.n_mid
    d[:, 0] += s.noise_rel * mx[f] * noise(s.seed, f, keys[:, 0], keys[:, 1])
    d[:, 1] += s.noise_rel * mx[f] * noise(s.seed, f, (-keys[:, 1]) % N, (-keys[:, 0]) % N)
    return d


def test_autograd_matches_central_differences_on_gradient_workload():
    s = make_config(3)
    p = E.Plan(s)
    d0 = _synthetic_rows(s, p)
    T = _dev(vhat(s))
    vel0 = np.asarray(s.vel, np.float64)

    def loss_of(d, lam, vel):
        V = E.edt_solve(d, lam, vel, p)
        return (V - T).abs().pow(2).sum()

    d = _dev(d0).requires_grad_(True)
    lam = torch.tensor(s.lambda_rel, dtype=torch.float64, device="cuda", requires_grad=True)
    vel = _dev(vel0).requires_grad_(True)
    loss = loss_of(d, lam, vel)
    loss.backward()
    gvel = vel.grad.cpu().numpy()
    glam = lam.grad.item()
    gd = d.grad.cpu().numpy()

    def L(dd=d0, ll=s.lambda_rel, vv=vel0):
        with torch.no_grad():
            return loss_of(_dev(dd), torch.tensor(ll, dtype=torch.float64, device="cuda"), _dev(vv)).item()

    scale = np.max(np.abs(gvel))
    for l in range(len(vel0)):
        h = 1e-6 * vel0[l]
        vp, vm = vel0.copy(), vel0.copy()
        vp[l] += h
        vm[l] -= h
        fd = (L(vv=vp) - L(vv=vm)) / (2 * h)
        assert abs(fd - gvel[l]) <= 1e-4 * scale, (l, fd, gvel[l])
    h = 1e-6 * s.lambda_rel
    fd = (L(ll=s.lambda_rel + h) - L(ll=s.lambda_rel - h)) / (2 * h)
    assert abs(fd - glam) <= 1e-4 * abs(glam), (fd, glam)
    rng = np.random.default_rng(7)
    scale_d = np.max(np.abs(gd))
    for r in rng.choice(len(d0), size=4, replace=False):
        for c in (0, 1):
            for part in (1.0, 1j):
                h = 1e-6 * max(abs(d0[r, c]), 1e-30)
                dp, dm = d0.copy(), d0.copy()
                dp[r, c] += h * part
                dm[r, c] -= h * part
                fd = (L(dd=dp) - L(dd=dm)) / (2 * h)
                an = gd[r, c].real if part == 1.0 else gd[r, c].imag
                assert abs(fd - an) <= 1e-4 * scale_d, (r, c, part, fd, an)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_graph_replay_equals_eager(prec):
    s = layered_small(nz=40, N=48, nf=12, seed=11)
    r = oracle_case(s)
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    pipe = E.Pipeline(p, vel, _dev(r["d_rows"]), s.lambda_rel, prec=prec, refine_tol=1e-9, max_refine=10)
    eager = pipe.step().clone()
    torch.cuda.synchronize()
    g, per = rel_errors(eager.cpu().numpy(), r["V"], r["pl"])
    assert g <= (1e-10 if prec == "fp64" else 1e-6) and per <= (1e-10 if prec == "fp64" else 1e-6)
    pipe.capture()
    ref = eager.cpu().numpy().view(np.uint64)
    for k in range(3):
        # the program's own eager work between the replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        pipe.v.zero_()
        out = pipe.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint64), ref), k
        del junk
