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
    # the largest evanescent disk lies inside the k_m grid (class set known in closed form)
    "3d-disk-inside": lambda: make_custom(dim=3, N=32, Nh=16, nz=3, dx=20.0, freqs=(5.0, 9.0),
                                          vel=(2000.0,), model=None),
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


@pytest.mark.parametrize("name", list(SURVEYS))
def test_unique_rows_merge_equal_born_rows(name):
    """A unique row stands for data rows of one pair with the same frequency and
    the same {|k_r|, |k_s|} (equal Born rows by source-receiver reciprocity);
    its multiplicity is their count, and the rows of a pair are sorted by f."""
    _lib_or_skip()
    s = SURVEYS[name]()
    p = E.Plan(s)
    m, u = p.rowmap(), p.urows()
    rows, uo, ur, ru = m["rows"], u["urow_off"], u["urows"], u["row_unique"]
    assert uo[0] == 0 and uo[-1] == len(ur)
    mult = np.bincount(ru, minlength=len(ur))
    assert np.array_equal(mult, ur[:, 1])
    for q in range(p.n_pairs):
        a, b = m["row_off"][q], m["row_off"][q + 1]
        assert np.all((ru[a:b] >= uo[q]) & (ru[a:b] < uo[q + 1]))
        uu = ur[ru[a:b]]
        assert np.array_equal(uu[:, 0], rows[a:b, 0])
        assert np.array_equal(np.sort(uu[:, 2:], 1), np.sort(rows[a:b, 1:], 1))
        seg = ur[uo[q]:uo[q + 1]]
        assert np.all(np.diff(seg[:, 0]) >= 0)
        keys = {(f, min(c1, c2), max(c1, c2)) for f, _, c1, c2 in seg}
        assert len(keys) == len(seg)


@pytest.mark.parametrize("name", ["cfg1", "2d-even-cut", "2d-odd-nocut", "3d-small", "3d-nocut"])
def test_unique_rows_follow_chains_of_shared_columns(name):
    """Within a pair and frequency the unique rows are ordered along chains of
    shared |k| classes, each row oriented (first class, second class) so that
    a chained row's first class is the row before's second.  In 2D a class
    joins at most two unique rows, so the class graph is paths (a class with a
    row to itself ends one) and cycles, and every component is one chain:
    the chain links number the rows less the components."""
    _lib_or_skip()
    s = SURVEYS[name]()
    p = E.Plan(s)
    u = p.urows()
    uo, ur = u["urow_off"], u["urows"]
    links = rows = comps = 0
    for q in range(p.n_pairs):
        seg = ur[uo[q]:uo[q + 1]]
        for f in np.unique(seg[:, 0]):
            g = seg[seg[:, 0] == f]
            k = int(np.sum(g[:-1, 3] == g[1:, 2]))
            parent = {}

            def root(c):
                while parent.setdefault(c, c) != c:
                    c = parent[c]
                return c
            for a, b in g[:, 2:]:
                parent[root(int(a))] = root(int(b))
            nc = len({root(c) for c in list(parent)})
            if s.dim == 2:
                deg = {}
                for a, b in g[:, 2:]:
                    deg[int(a)] = deg.get(int(a), 0) + 1
                    if b != a:
                        deg[int(b)] = deg.get(int(b), 0) + 1
                assert max(deg.values()) <= 2
                assert k == len(g) - nc, (q, f)
            links, rows, comps = links + k, rows + len(g), comps + nc
    assert rows == len(ur) and links >= rows - 2 * comps


def _check_items(p, which, band, max_rows):
    items, sched = p.schedule(which)
    u = p.urows()
    uo, f = u["urow_off"], u["urows"][:, 0]
    # pair-major, contiguous, covering every unique row once
    k = 0
    for q in range(p.n_pairs):
        pos = uo[q]
        while pos < uo[q + 1]:
            pq, b, e = items[k]
            assert (pq, b) == (q, pos) and b < e <= uo[q + 1]
            assert e - b <= max_rows
            assert np.all(f[b:e] // band == f[b] // band)
            # items are maximal: they end at the pair's end, a band edge or the size cap
            assert e == uo[q + 1] or f[e] // band != f[b] // band or e - b == max_rows
            pos, k = e, k + 1
    assert k == len(items)
    # launch order: every item once, holes are -1, length a multiple of the XCD count
    assert len(sched) % 8 == 0
    real = sched[sched >= 0]
    assert np.array_equal(np.sort(real), np.arange(len(items)))
    nrows = items[:, 2] - items[:, 1]
    bands = f[items[:, 1]] // band
    runs = [sched[x::8][sched[x::8] >= 0] for x in range(8)]
    for r in runs:
        # each XCD walks its bands in order, longest items of a band first
        assert np.all(np.diff(bands[r]) >= 0)
        for g in np.unique(bands[r]):
            assert np.all(np.diff(nrows[r][bands[r] == g]) <= 0)
    # the runs are consecutive pieces of the band order and carry about equal work
    order = np.concatenate(runs)
    assert np.all(np.diff(bands[order]) >= 0)
    load = np.array([nrows[r].sum() for r in runs])
    assert load.max() - load.min() <= 2 * nrows.max()


@pytest.mark.parametrize("opts", [dict(), dict(chunk_rows=16, gram_band=1), dict(chunk_rows=7, gram_band=3)])
@pytest.mark.parametrize("name", ["cfg1", "2d-even-cut", "3d-small"])
def test_work_items_and_xcd_schedule(name, opts):
    _lib_or_skip()
    s = SURVEYS[name]()
    p = E.Plan(s, **opts)
    band = p.info["gram_band"]
    if "gram_band" in opts:
        assert band == min(opts["gram_band"], p.table_shape[0])
    assert p.info["chunk_rows"] == opts.get("chunk_rows", 2048)
    _check_items(p, "gram", band, p.info["chunk_rows"])
    assert p.info["resid_group"] >= 2
    _check_items(p, "resid", p.info["resid_group"], 1024)


def _band_rules(p):
    n_f, n_cls, nz = p.table_shape
    l2 = int(2.5e6 // (n_cls * nz * 8))
    per_pf = p.info["n_urows"] / max(1, (p.n_pairs - p.info["n_empty"]) * n_f)
    return l2, int(np.ceil(256 / per_pf)), per_pf


def test_default_band_fits_l2():
    _lib_or_skip()
    s = make_config(2, with_model=False)
    p = E.Plan(s)
    n_cls, nz = p.table_shape[1], p.table_shape[2]
    band = p.info["gram_band"]
    l2, rows, _ = _band_rules(p)
    assert rows <= l2
    # one band's FP32 table slab is at most 2.5 MB and one more frequency would exceed it
    assert band * n_cls * nz * 8 <= 2.5e6 < (band + 1) * n_cls * nz * 8


def test_default_band_widens_for_sparse_rows():
    """3D 128 x 128 survey: one frequency's FP32 slab is near the L2 budget, so
    the band is set by the rows rule (an average item of 256 unique rows);
    residual groups: at least 2 frequencies, widened to 64 rows per item."""
    _lib_or_skip()
    s = make_config(4, with_model=False)
    p = E.Plan(s)
    l2, rows, per_pf = _band_rules(p)
    n_f = p.table_shape[0]
    assert rows > l2
    assert p.info["gram_band"] == min(n_f, rows)
    assert p.info["resid_group"] == min(n_f, max(2, int(np.ceil(64 / per_pf))))


@pytest.mark.parametrize("opts", [dict(chunk_rows=2049), dict(chunk_rows=-1), dict(gram_band=-2)])
def test_invalid_plan_options_are_rejected(opts):
    _lib_or_skip()
    s = SURVEYS["cfg1"]()
    with pytest.raises(RuntimeError):
        E.Plan(s, **opts)


def test_rowmap_equals_oracle_full_size_3d():
    """The narrowed offset loops of the 3D planner keep exactly the rows of the
    oracle's full enumeration (128 x 128 midpoints, 64 x 64 offsets)."""
    _lib_or_skip()
    s = make_config(4, with_model=False)
    p = E.Plan(s)
    m = p.rowmap()
    pl = oracle_plan(s)
    off = np.zeros(len(pl.pairs) + 1, np.int64)
    off[1:] = np.cumsum([q.n_rows for q in pl.pairs])
    assert np.array_equal(m["row_off"], off)
    f = np.concatenate([q.f for q in pl.pairs])
    kr = np.concatenate([q.kr for q in pl.pairs])
    ks = np.concatenate([q.ks for q in pl.pairs])
    key = np.concatenate([q.key0[:, 1] for q in pl.pairs])
    assert np.array_equal(m["rows"][:, 0], f)
    assert np.array_equal(m["cls_k"][m["rows"][:, 1]], kr)
    assert np.array_equal(m["cls_k"][m["rows"][:, 2]], ks)
    assert np.array_equal(m["keys"][:, 0], key)


@pytest.mark.parametrize("name", ["3d-small", "3d-nocut", "3d-disk-inside"])
def test_classes_are_exactly_the_used_wavenumbers(name):
    """The |k| classes are exactly the distinct |k_r|, |k_s| of the oracle's
    rows over the whole survey, also where they are derived without visiting
    every pair."""
    _lib_or_skip()
    s = SURVEYS[name]()
    pl = oracle_plan(s)
    used = np.unique(np.concatenate([np.concatenate([q.kr, q.ks]) for q in pl.pairs if q.n_rows]))
    for pairs in (None, (0, 1)):
        cls_k = E.Plan(s, pairs=pairs).rowmap()["cls_k"]
        assert np.array_equal(np.sort(cls_k), used)


@pytest.mark.parametrize("name", ["cfg1", "2d-even-cut", "2d-empty", "3d-small", "3d-disk-inside"])
def test_pair_range_plans_are_slices_of_the_full_plan(name):
    """A plan of pairs [a, b) (a batch) holds exactly those pairs' rows, data
    keys and unique rows of the full plan, with the full survey's |k| classes
    (so that every batch shares one Green's table)."""
    _lib_or_skip()
    s = SURVEYS[name]()
    full = E.Plan(s)
    m, u = full.rowmap(), full.urows()
    P = full.n_pairs
    cuts = sorted({0, P // 3, P // 3 + 1, P - 1, P})
    for a, b in zip(cuts[:-1], cuts[1:]):
        q = E.Plan(s, pairs=(a, b))
        mq, uq = q.rowmap(), q.urows()
        assert (q.n_pairs, q.n_pairs_all, q.pair_begin, q.n_km) == (b - a, P, a, full.n_km)
        assert q.table_shape == full.table_shape
        assert np.array_equal(mq["cls_k"], m["cls_k"])
        r0, r1 = m["row_off"][a], m["row_off"][b]
        assert np.array_equal(mq["row_off"], m["row_off"][a:b + 1] - r0)
        assert np.array_equal(mq["rows"], m["rows"][r0:r1])
        assert np.array_equal(mq["keys"], m["keys"][r0:r1])
        assert np.array_equal(mq["pair_km"], m["pair_km"][a:b])
        u0, u1 = u["urow_off"][a], u["urow_off"][b]
        assert np.array_equal(uq["urow_off"], u["urow_off"][a:b + 1] - u0)
        assert np.array_equal(uq["urows"], u["urows"][u0:u1])
        assert np.array_equal(uq["row_unique"], u["row_unique"][r0:r1] - u0)


@pytest.mark.parametrize("pairs", [(0, 10 ** 6), (3, 2), (-1, 2)])
def test_invalid_pair_ranges_are_rejected(pairs):
    _lib_or_skip()
    with pytest.raises(RuntimeError):
        E.Plan(SURVEYS["cfg1"](), pairs=pairs)


@pytest.mark.parametrize("kw", [dict(Nx=16, Ny=8, kappa=100.0), dict(Nx=15, Ny=7, kappa=1.0),
                                dict(Nx=24, Ny=12, dx=12.5, dy=25.0, kappa=1.0, freqs=(8.0, 23.0, 40.0))])
def test_line_survey_rows_equal_oracle(kw):
    """The planner's rows of the 3D survey of parallel lines are the oracle's,
    bit for bit: pairs, row order, frequencies and (a, b) keys."""
    from edt_inputs import make_lines
    from oracle.lines3d import plan_lines
    _lib_or_skip()
    s = make_lines(nz=5, model=None, **kw)
    pl = plan_lines(s)
    p = E.Plan(s)
    m = p.rowmap()
    assert p.n_pairs == len(pl.pairs) and p.n_km == s.n_mid * s.n_line
    off = np.zeros(len(pl.pairs) + 1, np.int64)
    off[1:] = np.cumsum([q.n_rows for q in pl.pairs])
    assert np.array_equal(m["row_off"], off)
    assert np.array_equal(m["pair_km"], np.array([[q.u, q.u_neg] for q in pl.pairs], np.int32))
    f = np.concatenate([q.f for q in pl.pairs])
    k = np.concatenate([q.key0[:, :2] for q in pl.pairs])
    assert np.array_equal(m["rows"][:, 0], f) and np.array_equal(m["keys"], k)
    assert np.array_equal(E.pair_rows(s), np.diff(off))
    # classes: every (|a|, |q|) of the grid
    Nx, Ny = s.n_mid, s.n_line
    ia, iq = np.divmod(np.arange(m["cls_k"].size), Ny // 2 + 1)
    ref = np.sqrt((ia * 2 * np.pi / (Nx * s.d_mid)) ** 2 + (iq * 2 * np.pi / (Ny * s.d_line)) ** 2)
    assert np.allclose(m["cls_k"], ref, rtol=1e-15, atol=0)


def test_line_survey_limits_are_refused():
    from edt_inputs import make_lines
    _lib_or_skip()
    with pytest.raises(RuntimeError, match="n_line <= 64"):
        E.Plan(make_lines(Nx=8, Ny=65, model=None))
    s = make_lines(Nx=8, Ny=4, model=None)
    s.dim = 2
    with pytest.raises(RuntimeError, match="dim 3"):
        E.Plan(s)
