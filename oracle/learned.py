"""CPU emulation of the learned split search: TEST INFRASTRUCTURE ONLY.

The paper has no learned component.  The project's learned partitioner
predicts a split a_hat for a cross diagonal d, searches only a window around
it, certifies the result with the two conditions of Algorithm 2 and falls
back to the full-range search when the certificate fails.  Its contract is
that the output equals the plain split of Algorithm 2 whatever the
prediction and the window.  This module restates those steps in plain Python
so that a property test can feed them arbitrary predictions and windows and
compare with the oracle's split (Lemma 8: the A count among the first d
merged outputs).  It shares no code with the GPU library.

Steps, for sorted A (length na), B (length nb) and diagonal d:
  1. The candidate splits on d are a in [dlo, dhi] = [max(0, d - nb),
     min(d, na)] (the diagonal's extent inside the grid).
  2. The prediction is clipped into [dlo, dhi]; the window [a_hat + wlo,
     a_hat + whi] (wlo <= whi) is clipped the same way, giving [lo, hi].
  3. A lower-bound search over a in [lo, hi) for the first a with
     B[d - 1 - a] < A[a] (Corollary 12: the predicate is monotone along the
     diagonal, false then true; an index outside B or A counts as true);
     hi if it never holds inside the window.
  4. Certificate: a result strictly inside the window is the split (the
     predicate was seen false just before it and true at it).  At a = hi < dhi
     the predicate at a was never evaluated; at a = lo > dlo its failure at
     a - 1 was never evaluated.  Those two cases evaluate the missing
     condition of Algorithm 2: B[d - 1 - a] < A[a], respectively
     A[a - 1] <= B[d - a].
  5. If the certificate fails, the lower-bound search runs over the whole
     [dlo, dhi] (the plain search, Theorem 14).
"""
from __future__ import annotations


def _pred(A, B, d, a):
    """B[d-1-a] < A[a], with a term outside B or A counting as true."""
    j = d - 1 - a
    if j < 0 or a >= len(A):
        return True
    return B[j] < A[a]


def _lower_bound(A, B, d, lo, hi):
    """First a in [lo, hi) where _pred holds, hi if none (binary search,
    floor midpoints)."""
    while lo < hi:
        mid = lo + (hi - lo) // 2
        if _pred(A, B, d, mid):
            hi = mid
        else:
            lo = mid + 1
    return lo


def learned_split(A, B, d: int, a_hat: int, wlo: int, whi: int):
    """Split on diagonal d from prediction a_hat and window offsets
    [wlo, whi]; returns (split, used_fallback)."""
    na, nb = len(A), len(B)
    assert 0 <= d <= na + nb and wlo <= whi
    dlo, dhi = max(0, d - nb), min(d, na)
    a_hat = min(max(a_hat, dlo), dhi)
    lo = min(max(a_hat + wlo, dlo), dhi)
    hi = min(max(a_hat + whi, dlo), dhi)
    a = _lower_bound(A, B, d, lo, hi)
    ok = True
    if a == hi and hi < dhi:
        ok = _pred(A, B, d, a)
    if ok and a == lo and lo > dlo:
        # A[a-1] <= B[d-a], i.e. the predicate fails at a - 1
        ok = not (B[d - a] < A[a - 1])
    if ok:
        return a, False
    return _lower_bound(A, B, d, dlo, dhi), True
