"""Host side of batch streaming: per-pair row counts without a plan, and the
cutting of a survey's pairs into contiguous batches under row and pair caps."""
import numpy as np
import pytest

from edt_inputs import make_config, make_custom

E = pytest.importorskip("paper_0905_0238_amd")
from paper_0905_0238_amd import _lib  # noqa: E402


def _lib_or_skip():
    try:
        return _lib.load()
    except ImportError as e:
        pytest.skip(str(e))


@pytest.mark.parametrize("s", [
    make_config(1, with_model=False),
    make_custom(N=40, nz=7, dx=12.5, freqs=(4.0, 9.0, 20.0), vel=(2100.0, 3000.0), zif=(30.0,), model=None),
    make_custom(dim=3, N=16, Nh=8, nz=4, dx=20.0, freqs=(9.0, 21.0), vel=(2000.0, 2500.0), zif=(30.0,),
                model=None),
    make_custom(dim=3, N=32, Nh=16, nz=3, dx=20.0, freqs=(5.0, 9.0), vel=(2000.0,), model=None),
])
def test_pair_rows_match_the_plan(s):
    _lib_or_skip()
    rows = E.pair_rows(s)
    p = E.Plan(s)
    assert len(rows) == p.n_pairs
    assert np.array_equal(rows, np.diff(p.rowmap()["row_off"]))


def test_cut_batches_covers_pairs_under_caps():
    rng = np.random.default_rng(0)
    rows = rng.integers(0, 1000, 500)
    rows[17] = 5000   # a pair larger than the row cap forms a batch of its own
    rows[300:320] = 0
    for cap_r, cap_p in [(2500, 64), (10 ** 9, 50), (1, 10 ** 6)]:
        b = E.cut_batches(rows, cap_r, cap_p)
        assert b[0][0] == 0 and b[-1][1] == len(rows)
        assert all(b[i][1] == b[i + 1][0] for i in range(len(b) - 1))
        for a, e in b:
            assert e > a and e - a <= cap_p
            assert rows[a:e].sum() <= cap_r or e - a == 1
            # maximal: the next pair would break a cap
            if e < len(rows):
                assert rows[a:e + 1].sum() > cap_r or e + 1 - a > cap_p
    with pytest.raises(ValueError):
        E.cut_batches(rows, 0, 4)


def _resident(p):
    """The documented parts of edt_plan_info.resident_bytes, from the plan's
    own query fields."""
    i = p.info
    P, nz = p.n_pairs, p.nz
    datum = 8 if i["data_type"] == _lib.DATA_C64 else 16
    return (i["dev_plan_bytes"] + i["work_bytes"] + p.n_rows * 2 * datum + P * (nz * nz + 4 * nz + 1) * 8
            + P * 8 + p.n_km * nz * 16 + i["table_elems"] * 24)


@pytest.mark.parametrize("data", ["c128", "c64"])
def test_resident_bytes_and_budget_refusal(data):
    _lib_or_skip()
    s = make_custom(N=40, nz=7, dx=12.5, freqs=(4.0, 9.0, 20.0), vel=(2100.0, 3000.0), zif=(30.0,), model=None)
    p = E.Plan(s, data=data)
    need = int(p.info["resident_bytes"])
    assert need == _resident(p)
    assert p.info["data_type"] == _lib.DATA_TYPES[data]
    # a budget of exactly the need is accepted, one byte less is refused
    q = E.Plan(s, data=data, hbm_budget=need)
    assert int(q.info["resident_bytes"]) == need
    with pytest.raises(RuntimeError, match=r"status -2.*need %d device bytes" % need):
        E.Plan(s, data=data, hbm_budget=need - 1)


def test_complex64_data_halves_the_data_rows():
    _lib_or_skip()
    s = make_config(1, with_model=False)
    a, b = E.Plan(s, data="c128"), E.Plan(s, data="c64")
    assert int(a.info["resident_bytes"]) - int(b.info["resident_bytes"]) == a.n_rows * 2 * 8
    with pytest.raises(ValueError):
        E.Plan(s, data="c32")


def test_budget_refuses_a_single_pair_that_does_not_fit():
    """A one-pair batch whose pass needs more than the budget is refused at
    plan time, with the pair range in the message."""
    _lib_or_skip()
    s = make_config(1, with_model=False)
    rows = E.pair_rows(s)
    q = int(np.argmax(rows))
    one = E.Plan(s, pairs=(q, q + 1))
    need = int(one.info["resident_bytes"])
    with pytest.raises(RuntimeError, match=r"pairs \[%d, %d\) need" % (q, q + 1)):
        E.Plan(s, pairs=(q, q + 1), hbm_budget=need // 2)


def test_invalid_data_type_is_refused():
    import ctypes as C
    from paper_0905_0238_amd.edt import _structs
    L = _lib_or_skip()
    s = make_config(1, with_model=False)
    sv, ly, keep = _structs(s)
    h = C.c_void_p()
    opts = _lib.PlanOpts(0, 0, 0, 0, 7, 0, 0)
    assert L.edt_plan_create(C.byref(sv), C.byref(ly), C.byref(opts), C.byref(h)) == _lib.EDT_EINVAL
    assert b"data_type" in L.edt_last_error()


def test_stream_refuses_a_layout_over_budget():
    """Batches that each fit but do not fit together (all batches' plans and
    data stay resident) are refused before any device memory is taken."""
    _lib_or_skip()
    s = make_config(1, with_model=False)
    rows = E.pair_rows(s)
    ranges = E.cut_batches(rows, int(rows.sum()) // 4 + 1, 10 ** 6)
    plans = [E.Plan(s, pairs=r, data="c64") for r in ranges]
    biggest = max(int(p.info["resident_bytes"]) for p in plans)
    with pytest.raises(MemoryError, match="the stream needs"):
        E.Stream(s, batch_rows=int(rows.sum()) // 4 + 1, data="c64", hbm_budget=biggest, device="cpu")
    with pytest.raises(RuntimeError, match="status -2"):
        E.Stream(s, batch_rows=int(rows.sum()) // 4 + 1, data="c64", hbm_budget=biggest // 3, device="cpu")


def test_tuned_shape_table_lookup(tmp_path, monkeypatch):
    """shapes_for: the EDT_TUNE_CACHE table first, then the package's table,
    else the planner default; keys differ by survey and by precision."""
    import json
    from paper_0905_0238_amd import tune
    s = make_config(1, with_model=False)
    s2 = make_config(2, with_model=False)
    assert tune.survey_key(s, "fp16x3") != tune.survey_key(s, "bf16x3")
    assert tune.survey_key(s, "fp16x3") != tune.survey_key(s2, "fp16x3")
    cache = tmp_path / "t.json"
    monkeypatch.setenv("EDT_TUNE_CACHE", str(cache))
    assert tune.shapes_for(s, "fp16x3") == tune.DEFAULT_SHAPE or tune.survey_key(s, "fp16x3") in json.load(
        open(tune.PACKAGE_TABLE))
    cache.write_text(json.dumps({tune.survey_key(s, "fp16x3"): {"chunk_rows": 1024, "gram_band": 8,
                                                                 "resid_group": 4, "ms": 1.0}}))
    assert tune.shapes_for(s, "fp16x3") == {"chunk_rows": 1024, "gram_band": 8, "resid_group": 4}
    # the shape is a valid plan option
    _lib_or_skip()
    p = E.Plan(s, **tune.shapes_for(s, "fp16x3"))
    assert p.info["chunk_rows"] == 1024 and p.info["gram_band"] == 8 and p.info["resid_group"] == 4
