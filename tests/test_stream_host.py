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
