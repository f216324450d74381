"""Pins of the multiset-operation oracle (no GPU).

A value found m times in A and n times in B must come out min(m, n) times
(intersection), max(m, n) (union), max(m - n, 0) (difference) and |m - n|
(symmetric difference), in sorted order; equal keys pair front to front, so
intersection keeps A's first copies, difference A's last ones, and union and
symmetric difference take a longer run's excess from its end.
"""
from collections import Counter

import numpy as np
import pytest

import oracle

OPS = ["intersection", "union", "difference", "symmetric_difference"]
RULE = {"intersection": lambda m, n: min(m, n), "union": max,
        "difference": lambda m, n: max(m - n, 0), "symmetric_difference": lambda m, n: abs(m - n)}


def _counts(op, A, B):
    ca, cb = Counter(A.tolist()), Counter(B.tolist())
    return {v: RULE[op](ca[v], cb[v]) for v in set(ca) | set(cb) if RULE[op](ca[v], cb[v]) > 0}


@pytest.mark.parametrize("op", OPS)
def test_counts_and_order_by_brute_force(op):
    g = np.random.default_rng(17)
    for _ in range(400):
        A = np.sort(g.integers(0, 5, g.integers(0, 13))).astype(np.int32)
        B = np.sort(g.integers(0, 5, g.integers(0, 13))).astype(np.int32)
        got = oracle.set_op(op, A, B)
        assert np.all(got[1:] >= got[:-1])
        assert dict(Counter(got.tolist())) == _counts(op, A, B), (A, B)


@pytest.mark.parametrize("dt", [np.uint32, np.int32, np.uint64, np.float32])
def test_closed_forms(dt):
    g = np.random.default_rng(3)
    A = np.sort(g.integers(0, 1000, 500)).astype(dt)
    # A with itself: everything matches
    assert np.array_equal(oracle.set_op("intersection", A, A), A)
    assert np.array_equal(oracle.set_op("union", A, A), A)
    assert len(oracle.set_op("difference", A, A)) == 0
    assert len(oracle.set_op("symmetric_difference", A, A)) == 0
    # disjoint ranges: nothing matches
    B = (np.sort(g.integers(0, 1000, 300)) + 2000).astype(dt)
    merged = np.sort(np.concatenate([A, B]), kind="stable")
    assert len(oracle.set_op("intersection", A, B)) == 0
    assert np.array_equal(oracle.set_op("union", A, B), merged)
    assert np.array_equal(oracle.set_op("difference", A, B), A)
    assert np.array_equal(oracle.set_op("symmetric_difference", A, B), merged)
    # one side empty
    E = A[:0]
    assert np.array_equal(oracle.set_op("union", A, E), A)
    assert np.array_equal(oracle.set_op("union", E, A), A)
    assert len(oracle.set_op("intersection", A, E)) == 0


def _bits(x):
    return np.asarray(x, np.float32).view(np.uint32).tolist()


def test_which_copies_signed_zeros():
    """-0.0 and +0.0 are equal keys with different bits: the bits show which
    copies each operation keeps."""
    n0, p0 = -0.0, 0.0
    A = np.array([n0, n0, p0], np.float32)        # m = 3
    B = np.array([p0], np.float32)                # n = 1
    assert _bits(oracle.set_op("intersection", A, B)) == _bits([n0])          # A's first copy
    assert _bits(oracle.set_op("difference", A, B)) == _bits([n0, p0])        # A's last two
    assert _bits(oracle.set_op("union", A, B)) == _bits([n0, n0, p0])         # all of A
    assert _bits(oracle.set_op("symmetric_difference", A, B)) == _bits([n0, p0])
    A = np.array([n0], np.float32)                # m = 1
    B = np.array([p0, n0, n0, p0], np.float32)    # n = 4
    assert _bits(oracle.set_op("union", A, B)) == _bits([n0, n0, n0, p0])     # A's, then B's last 3
    assert _bits(oracle.set_op("symmetric_difference", A, B)) == _bits([n0, n0, p0])
    assert _bits(oracle.set_op("intersection", A, B)) == _bits([n0])
    assert len(oracle.set_op("difference", A, B)) == 0
