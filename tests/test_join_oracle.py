"""Pins of the oracle's inner join (oracle_join_*: a nested loop over A then
B) against a hand-worked fixture, closed forms and the merge's own
quantities, none of which retypes the loop."""
import os

import numpy as np
import pytest

import mp_inputs as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DTYPES = [np.uint32, np.int32, np.uint64, np.float32]


def _golden(name):
    rec = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.split()
    dt = gen.NP_DTYPE[rec["dtype"][0]]
    return (np.array([int(x) for x in rec["A"]], dt), np.array([int(x) for x in rec["B"]], dt),
            np.array([int(x) for x in rec["I"]]), np.array([int(x) for x in rec["J"]]))


def test_hand_worked_fixture(orc):
    A, B, I, J = _golden("join_duplicates.txt")
    gi, gj, k = orc.join(A, B)
    assert k == len(I) and np.array_equal(gi, I) and np.array_equal(gj, J)


def _count_by_values(A, B):
    """Closed form: sum over values of (copies in A) x (copies in B)."""
    va, ca = np.unique(A, return_counts=True)
    vb, cb = np.unique(B, return_counts=True)
    common, ia, ib = np.intersect1d(va, vb, assume_unique=True, return_indices=True)
    return int(np.sum(ca[ia].astype(np.int64) * cb[ib].astype(np.int64)))


@pytest.mark.parametrize("dt", DTYPES)
def test_pairs_are_the_equal_ranges_of_the_merge(orc, dt):
    """For each i the matched j are exactly [lower_bound(B, A[i]),
    upper_bound(B, A[i])): the B positions the merge path visits between
    taking A[i] (ties take A first) and passing the last B copy of A[i];
    and the count is the closed form over values."""
    g = np.random.default_rng(7)
    for hi in (3, 40, 5000):
        A = np.sort(g.integers(0, hi, 1500)).astype(dt)
        B = np.sort(g.integers(0, hi, 1100)).astype(dt)
        I, J, k = orc.join(A, B)
        assert k == len(I) == _count_by_values(A, B)
        lo = np.searchsorted(B, A, side="left")
        up = np.searchsorted(B, A, side="right")
        want_i = np.repeat(np.arange(len(A)), up - lo)
        want_j = np.concatenate([np.arange(a, b) for a, b in zip(lo, up)]) if k else np.empty(0, int)
        assert np.array_equal(I, want_i) and np.array_equal(J, want_j)


def test_all_equal_keys_give_every_pair_in_order(orc):
    A = np.full(37, 9, np.uint32)
    B = np.full(23, 9, np.uint32)
    I, J, k = orc.join(A, B)
    assert k == 37 * 23
    assert np.array_equal(I, np.repeat(np.arange(37), 23))
    assert np.array_equal(J, np.tile(np.arange(23), 37))


def test_disjoint_and_empty_inputs(orc):
    A = np.arange(0, 100, 2, dtype=np.uint32)
    for B in (np.arange(1, 100, 2, dtype=np.uint32), np.empty(0, np.uint32)):
        I, J, k = orc.join(A, B)
        assert k == 0 and len(I) == 0
    I, J, k = orc.join(np.empty(0, np.uint32), A)
    assert k == 0


def test_signed_zeros_are_equal(orc):
    A = np.array([-1.0, -0.0, 0.0, 2.0], np.float32)
    B = np.array([0.0, 0.0, 2.0], np.float32)
    I, J, k = orc.join(A, B)
    assert k == 5
    assert list(zip(I, J)) == [(1, 0), (1, 1), (2, 0), (2, 1), (3, 2)]


def test_cap_keeps_the_first_pairs_and_the_full_count(orc):
    A = np.repeat(np.arange(10, dtype=np.uint64), 7)
    B = np.repeat(np.arange(0, 20, 2, dtype=np.uint64), 5)
    I, J, k = orc.join(A, B)
    I2, J2, k2 = orc.join(A, B, cap=40)
    assert k2 == k == 5 * 7 * 5 and np.array_equal(I2, I[:40]) and np.array_equal(J2, J[:40])


def test_pins_reject_a_wrong_equality(orc, tmp_path):
    """An oracle built with <= in place of equality must fail the pins."""
    bad = orc.load(orc.build(str(tmp_path / "bad_join.so"),
                             extra_flags=["-DORACLE_JOIN_EQ(a,b)=((a)<=(b))"]))
    A, B, I, J = _golden("join_duplicates.txt")
    gi, gj, k = orc.join(A, B, lib=bad)
    assert k != len(I)
    g = np.random.default_rng(8)
    A = np.sort(g.integers(0, 40, 300)).astype(np.uint32)
    B = np.sort(g.integers(0, 40, 200)).astype(np.uint32)
    assert orc.join(A, B, lib=bad)[2] != _count_by_values(A, B)
