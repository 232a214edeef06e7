"""Host-side checks of libedt: the C++ planner's pairs, rows, classes and
data keys must equal the oracle's enumeration exactly (integer work), the
library must export every entry point of include/edt.h, and invalid surveys
must be rejected with an error rather than planned."""
import os
import re

import numpy as np
import pytest

from edt_inputs import make_config, make_custom
from oracle.rows import plan as oracle_plan

E = pytest.importorskip("paper_0905_0238_amd")
from paper_0905_0238_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    try:
        return _lib.load()
    except ImportError as e:
        pytest.skip(str(e))


def test_exports_every_declared_entry_point():
    L = _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "edt.h")).read()
    declared = sorted(set(re.findall(r"\b(edt_[a-z_]+)\s*\(", hdr)))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), f"libedt.so does not export {name}"
    assert set(declared) == set(_lib.EXPORTS)


SURVEYS = {
    "cfg1": lambda: make_config(1, with_model=False),
    "2d-even-cut": lambda: make_custom(N=40, nz=7, dx=12.5, freqs=(4.0, 9.0, 20.0),
                                       vel=(2100.0, 3000.0), zif=(30.0,), model=None),
    "2d-odd-nocut": lambda: make_custom(N=11, nz=3, freqs=(5.0, 9.0), kappa=100.0, model=None),
    "2d-empty": lambda: make_custom(N=64, nz=5, dx=25.0, freqs=(2.0, 3.0), vel=(2500.0,), model=None),
    "3d-small": lambda: make_custom(dim=3, N=16, Nh=8, nz=4, dx=20.0, freqs=(9.0, 21.0),
                                    vel=(2000.0, 2500.0), zif=(30.0,), model=None),
    "3d-nocut": lambda: make_custom(dim=3, N=8, Nh=4, nz=3, dx=30.0, freqs=(6.0,), kappa=100.0,
                                    model=None),
}


@pytest.mark.parametrize("name", list(SURVEYS))
def test_rowmap_equals_oracle(name):
    _lib_or_skip()
    s = SURVEYS[name]()
    p = E.Plan(s)
    m = p.rowmap()
    pl = oracle_plan(s)
    assert p.n_pairs == len(pl.pairs)
    assert p.n_km == pl.n_km
    off = np.zeros(len(pl.pairs) + 1, np.int64)
    off[1:] = np.cumsum([q.n_rows for q in pl.pairs])
    assert np.array_equal(m["row_off"], off)
    cls_k = m["cls_k"]
    for i, q in enumerate(pl.pairs):
        a, b = off[i], off[i + 1]
        assert tuple(m["pair_km"][i]) == (q.u, q.u_neg)
        assert np.array_equal(m["rows"][a:b, 0], q.f)
        # classes map to exactly the oracle's |k_r|, |k_s| (bit for bit)
        assert np.array_equal(cls_k[m["rows"][a:b, 1]], q.kr)
        assert np.array_equal(cls_k[m["rows"][a:b, 2]], q.ks)
        if s.dim == 2:
            assert np.array_equal(m["keys"][a:b], q.key0)
        else:
            assert np.array_equal(m["keys"][a:b, 0], q.key0[:, 1])
    if name == "2d-empty":
        assert p.info["n_empty"] > 0


def test_rowmap_equals_oracle_full_size_2d():
    _lib_or_skip()
    s = make_config(3, with_model=False)
    p = E.Plan(s)
    m = p.rowmap()
    pl = oracle_plan(s)
    off = np.zeros(len(pl.pairs) + 1, np.int64)
    off[1:] = np.cumsum([q.n_rows for q in pl.pairs])
    assert np.array_equal(m["row_off"], off)
    f = np.concatenate([q.f for q in pl.pairs])
    kr = np.concatenate([q.kr for q in pl.pairs])
    key = np.concatenate([q.key0 for q in pl.pairs])
    assert np.array_equal(m["rows"][:, 0], f)
    assert np.array_equal(m["cls_k"][m["rows"][:, 1]], kr)
    assert np.array_equal(m["keys"], key)
    # every data row is counted once among the distinct Born rows
    assert 0 < p.info["n_urows"] <= p.n_rows


@pytest.mark.parametrize("bad", ["zif0", "order", "dim", "nz", "vel", "freq", "areal"])
def test_invalid_surveys_are_rejected(bad):
    _lib_or_skip()
    kw = dict(N=16, nz=4, freqs=(5.0,), vel=(2000.0, 2500.0, 3000.0), zif=(30.0, 60.0), model=None)
    s = make_custom(**kw)
    if bad == "zif0":
        s.zif = np.array([0.0, 60.0])
    elif bad == "order":
        s.zif = np.array([60.0, 30.0])
    elif bad == "dim":
        s.dim = 4
    elif bad == "nz":
        s.nz = 0
    elif bad == "vel":
        s.vel = np.array([2000.0, -1.0, 3000.0])
    elif bad == "freq":
        s.freqs = np.array([-5.0])
    elif bad == "areal":
        s = make_custom(dim=3, N=8, Nh=4, nz=2, freqs=(5.0,), model=None)
        s.d_off = s.d_off * 1.5
    with pytest.raises(RuntimeError):
        E.Plan(s)
