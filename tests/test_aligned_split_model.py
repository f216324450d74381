"""A CPU model of the aligned split search (binary lifting from origin 0,
used by the partition kernel on diagonals that are multiples of a power of
two) against the oracle's split on every diagonal of small inputs with
duplicates and one-sided cases."""
import numpy as np

import oracle


def _aligned_split(A, B, d, lo, hi):
    # x counts the positions that fail B[d-1-c] < A[c]; below lo they fail by
    # the grid's bounds and are not read; positions at or past hi are never
    # probed
    x = 0
    if hi <= 0:
        return 0
    bit = 1 << (hi.bit_length() - 1)
    while bit:
        c = x + bit - 1
        if c < hi and (c < lo or not (B[d - 1 - c] < A[c])):
            x += bit
        bit >>= 1
    return x


def test_aligned_split_equals_oracle_on_every_diagonal():
    rng = np.random.default_rng(810)
    for _ in range(150):
        na, nb = int(rng.integers(0, 120)), int(rng.integers(0, 120))
        hi = int(rng.choice([2, 4, 30, 1 << 30]))
        A = np.sort(rng.integers(0, hi, na)).astype(np.uint32)
        B = np.sort(rng.integers(0, hi, nb)).astype(np.uint32)
        d = np.arange(0, na + nb + 1, dtype=np.int64)
        want = oracle.partition(A, B, d)
        for k in range(len(d)):
            dd = int(d[k])
            lo, hi_ = max(0, dd - nb), min(dd, na)
            assert _aligned_split(A, B, dd, lo, hi_) == want[k], (na, nb, dd)
