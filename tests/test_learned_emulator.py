"""Property test of the learned split search's logic on the CPU: prediction,
window, bounded search, certificate, fallback (oracle/learned.py).  Whatever
the prediction and the window, the result equals the oracle's split
(Lemma 8), and the fallback runs exactly when the clipped window misses the
true split."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import learned

KEYS = st.integers(min_value=0, max_value=6)  # a small alphabet: long runs of ties


@st.composite
def cases(draw):
    A = sorted(draw(st.lists(KEYS, max_size=24)))
    B = sorted(draw(st.lists(KEYS, max_size=24)))
    d = draw(st.integers(min_value=0, max_value=len(A) + len(B)))
    a_hat = draw(st.integers(min_value=-40, max_value=80))
    wlo = draw(st.integers(min_value=-30, max_value=30))
    whi = draw(st.integers(min_value=wlo, max_value=40))
    return A, B, d, a_hat, wlo, whi


def _clipped(na, nb, d, a_hat, wlo, whi):
    dlo, dhi = max(0, d - nb), min(d, na)
    a_hat = min(max(a_hat, dlo), dhi)
    return min(max(a_hat + wlo, dlo), dhi), min(max(a_hat + whi, dlo), dhi)


@settings(max_examples=3000, deadline=None)
@given(cases())
def test_any_prediction_and_window_give_the_split(orc, case):
    A, B, d, a_hat, wlo, whi = case
    a, fb = learned.learned_split(A, B, d, a_hat, wlo, whi)
    want = int(orc.partition(np.array(A, np.uint32), np.array(B, np.uint32),
                             np.array([d], np.int64))[0])
    assert a == want
    lo, hi = _clipped(len(A), len(B), d, a_hat, wlo, whi)
    assert fb == (not lo <= want <= hi)


@pytest.mark.parametrize("where", ["lo=hi=split", "lo=hi=dlo", "hi=dhi", "lo=dlo",
                                   "just_below", "just_above"])
def test_certificate_edges(orc, where):
    """The certificate's edge cases, each on every diagonal of one pair with
    runs of ties: a zero-width window on the split, on the diagonal's lower
    end, windows reaching a diagonal end, and windows ending one short of
    the split on either side (which must fall back)."""
    A = [0, 1, 1, 2, 2, 2, 5, 7, 7]
    B = [1, 1, 2, 3, 5, 5, 7, 8]
    na, nb = len(A), len(B)
    splits = orc.partition(np.array(A, np.uint32), np.array(B, np.uint32),
                           np.arange(na + nb + 1, dtype=np.int64))
    for d in range(na + nb + 1):
        s = int(splits[d])
        dlo, dhi = max(0, d - nb), min(d, na)
        if where == "lo=hi=split":
            args, fb = (s, 0, 0), False
        elif where == "lo=hi=dlo":
            args, fb = (dlo, 0, 0), s != dlo
        elif where == "hi=dhi":
            args, fb = (s, 0, dhi - s + 5), False
        elif where == "lo=dlo":
            args, fb = (s, dlo - s - 5, 0), False
        elif where == "just_below":
            if s == dlo:
                continue
            args, fb = (s - 1, -3, 0), True
        else:
            if s == dhi:
                continue
            args, fb = (s + 1, 0, 3), True
        assert learned.learned_split(A, B, d, *args) == (s, fb), (d, where)
