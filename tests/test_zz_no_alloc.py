"""The allocation-free solve (edt_solve_static) against edt_solve, through the
C-ABI: same plan, same assembled Gram, same data; the static variant keeps
its scratch in the library's static device array instead of the plan's
workspace.  The two run the same kernels in the same order, so their
results must agree bit for bit.  Two calls in a row, the second on a smaller
survey, check that nothing of the first call's scratch leaks into the next.
"""
import ctypes as C

import numpy as np
import pytest

from edt_inputs import make_config
from tests._cases import oracle_case, layered_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_0905_0238_amd")
from paper_0905_0238_amd import _lib  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _surveys():
    # a larger survey first, then a smaller one (fewer pairs, rows and depths)
    big = layered_small(nz=72, N=48, nf=12, seed=21)
    small = layered_small(nz=40, N=24, nf=6, seed=22)
    return [big, small]


def _assembled(s, prec):
    r = oracle_case(s)
    p = E.Plan(s)
    vel = _dev(np.asarray(s.vel, np.float64))
    g64, g32 = p.green(vel, want32=prec != "fp64")
    d = _dev(r["d_rows"])
    gram, rhs, trace = p.assemble(g64, g32, d, prec)
    torch.cuda.synchronize()
    return p, g64, d, gram, rhs, trace


@pytest.mark.parametrize("prec,refine,escalate", [("fp64", False, False), ("fp16x3", True, False),
                                                  ("bf16x3", True, True)])
def test_static_solve_equals_workspace_solve_on_two_calls(prec, refine, escalate):
    cases = []
    for s in _surveys():
        p, g64, d, gram, rhs, trace = _assembled(s, prec)
        ref = p.solve(g64, d, gram.clone(), rhs, trace, s.lambda_rel, refine=refine, refine_tol=3e-6,
                      max_refine=8, escalate=escalate)
        torch.cuda.synchronize()
        cases.append((s, p, g64, d, gram, rhs, trace, [t.cpu() for t in ref]))
    # the static calls back to back: the second, smaller survey reuses the
    # array the first one left behind
    outs = []
    for s, p, g64, d, gram, rhs, trace, _ in cases:
        outs.append(p.solve_static(g64, d, gram.clone(), rhs, trace, s.lambda_rel, refine=refine,
                                   refine_tol=3e-6, max_refine=8, escalate=escalate))
    torch.cuda.synchronize()
    for (s, p, *_, ref), out in zip(cases, outs):
        x, v, info, steps = (t.cpu() for t in out)
        rx, rv, rinfo, rsteps = ref
        print(f"{prec} nz={s.nz} pairs={p.n_pairs}: max |dx| {float((x - rx).abs().max()):.3e}", flush=True)
        assert torch.equal(info, rinfo)
        assert torch.equal(x, rx)
        assert torch.equal(v, rv)
        if refine:
            assert torch.equal(steps, rsteps)
        assert int((info > 0).sum()) == 0


def test_static_solve_matches_oracle_after_a_larger_call():
    """The second, smaller call also meets the FP64 bar against the oracle."""
    from tests._cases import rel_errors
    big, small = _surveys()
    for s in (big, small):
        r = oracle_case(s)
        p = E.Plan(s)
        vel = _dev(np.asarray(s.vel, np.float64))
        g64, _ = p.green(vel, want32=False)
        d = _dev(r["d_rows"])
        gram, rhs, trace = p.assemble(g64, None, d, "fp64")
        x, v, info, _ = p.solve_static(g64, d, gram, rhs, trace, s.lambda_rel)
        torch.cuda.synchronize()
        glob, per = rel_errors(v.cpu().numpy(), r["V"], r["pl"])
        print(f"fp64 static nz={s.nz}: global {glob:.3e} per pair {per:.3e}", flush=True)
        assert glob <= 1e-10 and per <= 1e-10


def test_static_solve_refuses_oversized_plans_and_summed_data():
    """A plan whose scratch exceeds the static array is refused with
    EDT_ENOMEM and a message naming the size; data_summed is refused with
    EDT_EINVAL.  Nothing is enqueued in either case."""
    s = make_config(2, with_model=False)
    p = E.Plan(s)
    p.upload()
    L = _lib.load()
    dummy = torch.zeros(64, dtype=torch.float64, device="cuda")
    idummy = torch.zeros(64, dtype=torch.int32, device="cuda")
    ptr = C.c_void_p(dummy.data_ptr())
    iptr = C.c_void_p(idummy.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(refine, escalate, data_summed):
        opts = _lib.SolveOpts(refine, 1e-6, 8, escalate, data_summed)
        return L.edt_solve_static(p._h, ptr, ptr, ptr, ptr, ptr, 1e-3, C.byref(opts), ptr, ptr, iptr, iptr,
                                  stream)

    # the 2D 512-trace survey: refinement fits (about 111 MB), escalation's
    # FP64 Gram partials (1.2 GB) do not
    assert call(1, 1, 0) == _lib.EDT_ENOMEM
    msg = L.edt_last_error().decode()
    assert "bytes of scratch" in msg and str(_lib.STATIC_SCRATCH_BYTES) in msg
    assert call(1, 0, 1) == _lib.EDT_EINVAL
    torch.cuda.synchronize()
    assert float(dummy.abs().sum()) == 0.0 and int(idummy.abs().sum()) == 0
