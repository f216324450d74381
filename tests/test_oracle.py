"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks retypes the oracle's loop: each compares it with a
hand-worked fixture, a library routine the definition reduces to, a closed
form, a brute-force enumeration or an invariant stated in the paper.
"""
import glob
import itertools
import os

import numpy as np
import pytest

import mp_inputs as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DTYPES = [np.uint32, np.int32, np.uint64, np.float32]


def load_golden(path):
    rec = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split(":", 1)
        rec[k.strip()] = v.split()
    dt = gen.NP_DTYPE[rec["dtype"][0]]
    conv = (lambda xs: np.array([float(x) for x in xs], dtype=dt)) if dt == np.float32 else \
        (lambda xs: np.array([int(x) for x in xs], dtype=dt))
    return (conv(rec.get("A", [])), conv(rec.get("B", [])), conv(rec["S"]),
            np.array([int(x) for x in rec["src"]]), np.array([int(x) for x in rec["split"]]))


# ---------------------------------------------------------------- brute force

def certificate(A, B, d, a):
    """Both predicates of the split on diagonal d (out-of-range terms hold)."""
    b = d - a
    p_down = a == 0 or b == len(B) or A[a - 1] <= B[b]
    p_right = b == 0 or a == len(A) or B[b - 1] < A[a]
    return p_down and p_right


def brute_splits(A, B):
    out = []
    for d in range(len(A) + len(B) + 1):
        ok = [a for a in range(max(0, d - len(B)), min(d, len(A)) + 1) if certificate(A, B, d, a)]
        assert len(ok) == 1, (A, B, d, ok)   # the split is unique on every diagonal
        out.append(ok[0])
    return np.array(out)


def stable_reference(A, B):
    """Merge as a stable sort of A ++ B: A's copies of a key precede B's."""
    cat = np.concatenate([A, B])
    order = np.argsort(cat, kind="stable")
    return cat[order], order


# ---------------------------------------------------------------- fixtures

@pytest.mark.parametrize("path", sorted(p for p in glob.glob(os.path.join(GOLDEN, "*.txt"))
                                          if not os.path.basename(p).startswith("join_")))
def test_golden(orc, path):
    A, B, S, src, split = load_golden(path)
    got, got_src = orc.merge(A, B, with_src=True)
    assert got.tobytes() == S.tobytes()
    assert np.array_equal(got_src, src)
    d = np.arange(len(A) + len(B) + 1)
    assert np.array_equal(orc.partition(A, B, d), split)
    assert np.array_equal(brute_splits(A, B), split)


# ---------------------------------------------------------------- library pins

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("case", ["uniform", "dups", "unequal"])
def test_merge_equals_stable_sort(orc, dt, case):
    g = np.random.default_rng(7)
    na, nb = (3000, 5000) if case != "unequal" else (17, 9000)
    if case == "dups":
        A = np.sort(g.integers(0, 20, na)).astype(dt)
        B = np.sort(g.integers(0, 20, nb)).astype(dt)
    else:
        A = np.sort(g.integers(0, 2**31, na)).astype(dt)
        B = np.sort(g.integers(0, 2**31, nb)).astype(dt)
    S, src = orc.merge(A, B, with_src=True)
    ref, order = stable_reference(A, B)
    assert S.tobytes() == ref.tobytes()
    assert np.array_equal(src, order)


@pytest.mark.parametrize("dt", DTYPES)
def test_merge_positions_closed_form(orc, dt):
    """A[i] lands at i + #{B < A[i]}; B[j] lands at j + #{A <= B[j]}."""
    g = np.random.default_rng(3)
    A = np.sort(g.integers(0, 50, 700)).astype(dt)
    B = np.sort(g.integers(0, 50, 400)).astype(dt)
    S, src = orc.merge(A, B, with_src=True)
    pa = np.arange(len(A)) + np.searchsorted(B, A, side="left")
    pb = np.arange(len(B)) + np.searchsorted(A, B, side="right")
    assert np.array_equal(src[pa], np.arange(len(A)))
    assert np.array_equal(src[pb], len(A) + np.arange(len(B)))
    assert S[pa].tobytes() == A.tobytes() and S[pb].tobytes() == B.tobytes()


def test_signed_zero_ties(orc):
    nz, pz = np.float32(-0.0), np.float32(0.0)
    S = orc.merge(np.array([nz], np.float32), np.array([pz], np.float32))
    assert np.signbit(S).tolist() == [True, False]
    S = orc.merge(np.array([pz], np.float32), np.array([nz], np.float32))
    assert np.signbit(S).tolist() == [False, True]


def test_extreme_keys(orc):
    for dt in (np.uint32, np.uint64):
        m = np.iinfo(dt).max
        A = np.array([0, m, m], dt)
        B = np.array([m], dt)
        S, src = orc.merge(A, B, with_src=True)
        assert src.tolist() == [0, 1, 2, 3]
        assert orc.partition(A, B, [0, 1, 2, 3, 4]).tolist() == [0, 1, 2, 3, 3]
    A = np.array([-2**31, 2**31 - 1], np.int32)
    B = np.array([-2**31, 0], np.int32)
    assert orc.merge(A, B, with_src=True)[1].tolist() == [0, 2, 3, 1]
    fmax = np.finfo(np.float32).max
    A = np.array([-fmax, fmax], np.float32)
    B = np.array([-fmax, fmax], np.float32)
    assert orc.merge(A, B, with_src=True)[1].tolist() == [0, 2, 1, 3]


# ---------------------------------------------------------------- brute force

def _sorted_seqs(max_len, alphabet):
    for L in range(max_len + 1):
        for c in itertools.combinations_with_replacement(range(alphabet), L):
            yield np.array(c, dtype=np.uint32)


def test_partition_bruteforce_exhaustive(orc):
    seqs = list(_sorted_seqs(4, 3))
    for A in seqs:
        for B in seqs:
            d = np.arange(len(A) + len(B) + 1)
            assert np.array_equal(orc.partition(A, B, d), brute_splits(A, B))


def test_partition_bruteforce_random(orc):
    g = np.random.default_rng(11)
    for _ in range(300):
        na, nb = g.integers(0, 13, 2)
        alpha = int(g.integers(1, 6))
        dt = DTYPES[int(g.integers(0, 4))]
        A = np.sort(g.integers(0, alpha, na)).astype(dt)
        B = np.sort(g.integers(0, alpha, nb)).astype(dt)
        d = np.arange(na + nb + 1)
        assert np.array_equal(orc.partition(A, B, d), brute_splits(A, B))


def test_partition_any_diagonal_order(orc):
    A, B = gen.uniform_pair(500, 300, 5)
    d = np.random.default_rng(1).integers(0, 801, 200)
    full = orc.partition(A, B, np.arange(801))
    assert np.array_equal(orc.partition(A, B, d), full[d])


# ---------------------------------------------------------------- closed forms

def test_closed_form_all_a_greater(orc):
    """Section 1 counter-example: all of A > all of B, so S = B ++ A."""
    A, B = gen.disjoint_pair(1000, 700, 3)
    S = orc.merge(A, B)
    assert S.tobytes() == np.concatenate([B, A]).tobytes()
    d = np.arange(1701)
    assert np.array_equal(orc.partition(A, B, d), np.maximum(0, d - 700))


def test_closed_form_all_a_not_greater(orc):
    hi, lo = gen.disjoint_pair(900, 600, 4)
    A, B = lo, hi  # now every A key is below every B key
    d = np.arange(1501)
    assert np.array_equal(orc.partition(A, B, d), np.minimum(d, 600))
    eq_a, eq_b = np.full(40, 9, np.uint32), np.full(25, 9, np.uint32)
    d = np.arange(66)
    assert np.array_equal(orc.partition(eq_a, eq_b, d), np.minimum(d, 40))
    S, src = orc.merge(eq_a, eq_b, with_src=True)
    assert np.array_equal(src, np.arange(65))


def test_closed_form_interleaved(orc):
    A = np.arange(0, 2000, 2, dtype=np.uint32)       # evens
    B = np.arange(1, 2001, 2, dtype=np.uint32)       # odds
    d = np.arange(2001)
    assert np.array_equal(orc.partition(A, B, d), (d + 1) // 2)
    assert np.array_equal(orc.partition(B, A, d), d // 2)
    C = np.arange(1000, dtype=np.uint32)             # identical distinct arrays
    assert np.array_equal(orc.partition(C, C.copy(), d), (d + 1) // 2)


# ---------------------------------------------------------------- invariants

def test_lemma8_unit_steps(orc):
    for seed, (na, nb) in enumerate([(1000, 1000), (1, 3000), (2500, 3), (0, 10), (10, 0)]):
        A, B = gen.uniform_pair(na, nb, seed)
        a = orc.partition(A, B, np.arange(na + nb + 1))
        assert a[0] == 0 and a[-1] == na
        assert set(np.diff(a).tolist()) <= {0, 1}


def test_theorem5_independent_pairs_concatenate(orc):
    """Cor. 6: merging the pairs cut at any diagonals and concatenating gives S."""
    A, B = gen.dups_pair(3000, 2000, 9, hi=50)
    N = 5000
    cuts = np.unique(np.concatenate([[0, N], np.random.default_rng(2).integers(0, N, 37)]))
    a = orc.partition(A, B, cuts)
    b = cuts - a
    parts = []
    for k in range(len(cuts) - 1):
        pa, pb = A[a[k]:a[k + 1]], B[b[k]:b[k + 1]]
        assert len(pa) + len(pb) == cuts[k + 1] - cuts[k]        # pair sizes exactly as asked
        parts.append(stable_reference(pa, pb)[0])
    assert np.concatenate(parts).tobytes() == orc.merge(A, B).tobytes()


def test_naive_equal_split_is_wrong(orc):
    """Section 1: cutting both arrays at the same fraction does not merge correctly."""
    A, B = gen.disjoint_pair(64, 64, 1)
    naive = np.concatenate([stable_reference(A[:32], B[:32])[0], stable_reference(A[32:], B[32:])[0]])
    assert naive.tobytes() != orc.merge(A, B).tobytes()
    assert np.any(np.diff(naive.astype(np.int64)) < 0)


# ---------------------------------------------------------------- kv, sort, batched

@pytest.mark.parametrize("dt", DTYPES)
def test_merge_kv(orc, dt):
    g = np.random.default_rng(5)
    A = np.sort(g.integers(0, 30, 900)).astype(dt)
    B = np.sort(g.integers(0, 30, 1300)).astype(dt)
    va, vb = gen.index_payload(900, 1300)
    Sk, Sv = orc.merge_kv(A, va, B, vb)
    ref, order = stable_reference(A, B)
    assert Sk.tobytes() == ref.tobytes()
    assert np.array_equal(Sv, order.astype(np.uint32))


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 1000, 4097])
def test_sort_equals_stable_sort(orc, dt, n):
    g = np.random.default_rng(n)
    keys = g.integers(0, 64, n).astype(dt)
    vals = np.arange(n, dtype=np.uint32)
    k, v = orc.sort(keys, vals)
    order = np.argsort(keys, kind="stable")
    assert k.tobytes() == keys[order].tobytes()
    assert np.array_equal(v, order.astype(np.uint32))
    assert orc.sort(keys).tobytes() == keys[order].tobytes()


def test_sort_zipf(orc):
    keys = gen.zipf_keys(20000, 32)
    assert orc.sort(keys).tobytes() == np.sort(keys, kind="stable").tobytes()


def test_batched(orc):
    A, a_off, B, b_off = gen.batched_pairs(60, 41, median=64)
    S = orc.merge_batched(A, a_off, B, b_off)
    for k in range(60):
        ref = stable_reference(A[a_off[k]:a_off[k + 1]], B[b_off[k]:b_off[k + 1]])[0]
        o = a_off[k] + b_off[k]
        assert S[o:o + len(ref)].tobytes() == ref.tobytes()


# ---------------------------------------------------------------- planted mistake

def test_pins_reject_wrong_tie_rule(orc, tmp_path):
    """An oracle built with ties taking B must fail the pins above."""
    bad = orc.load(orc.build(str(tmp_path / "bad.so"),
                             extra_flags=["-DORACLE_TAKE_B(a,b)=((a)>=(b))"]))
    A, B, S, src, split = load_golden(os.path.join(GOLDEN, "tie_rule_duplicates.txt"))
    _, got_src = orc.merge(A, B, with_src=True, lib=bad)
    assert not np.array_equal(got_src, src)
    d = np.arange(len(A) + len(B) + 1)
    assert not np.array_equal(orc.partition(A, B, d, lib=bad), brute_splits(A, B))
