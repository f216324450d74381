"""A CPU model of the set-operation tile kernel's walk, checked against the
oracle on small inputs with tiny tiles.

The model follows the kernel step by step: each tile's pair sits in one LDS
array (A's 16-byte chunks from position 0, B's after them, whatever the
chunks hold around the windows), every lane finds its split at local
diagonal lane * VT, takes the rank of its first A and B copy from a search
in the window (or from the run start before the window), then walks VT
steps keeping, per side, the position where the current run starts.  A
partner inside the window is one read; one outside takes the exact index
into the input.  The first runs' starts are placed at most SAT back; SAT is
2^30 in the kernel and is lowered here to just past the LDS array, so that
the exact-rank path runs on small inputs too.  Any mistake in the position
arithmetic shows up as a wrong multiset.
"""
import numpy as np
import pytest

import oracle

OPS = {"intersection": 0, "union": 1, "difference": 2, "symmetric_difference": 3}
CH = 4  # keys per 16-byte chunk (4-byte keys)


def _split(A, B, d):
    lo, hi = max(0, d - len(B)), min(d, len(A))
    while lo < hi:
        m = (lo + hi) // 2
        if B[d - 1 - m] < A[m]:
            hi = m
        else:
            lo = m + 1
    return lo


def _run_start(X, p):
    v = X[p]
    while p > 0 and X[p - 1] == v:
        p -= 1
    return p


def _tile(op, A, B, d0, n, NT, VT, SAT, offA, offB, rng):
    na, nb = len(A), len(B)
    a0 = _split(A, B, d0)
    b0 = d0 - a0
    wa = _split(A, B, d0 + n) - a0
    wb = n - wa
    # chunk layout: A[a0] at oa, B[b0] at ob; the array is filled with
    # garbage first, then whole chunks are stored
    sa, sb = (a0 + offA) % CH, (b0 + offB) % CH
    ca, cb = (sa + wa + CH - 1) // CH, (sb + wb + CH - 1) // CH
    oa, ob = sa, ca * CH + sb
    ae, be = oa + wa, ob + wb
    T = NT * VT
    keys = [int(x) for x in rng.integers(0, 1 << 32, T + 4 * CH + VT + 1)]
    for c in range(ca):
        for j in range(CH):
            g = a0 - sa + c * CH + j
            keys[c * CH + j] = int(A[g]) if 0 <= g < na else 0
    for c in range(cb):
        for j in range(CH):
            g = b0 - sb + c * CH + j
            keys[(ca + c) * CH + j] = int(B[g]) if 0 <= g < nb else 0
    lbA = _run_start(A, a0) if wa > 0 and a0 > 0 else a0
    lbB = _run_start(B, b0) if wb > 0 and b0 > 0 else b0
    out = []
    for lane in range(NT):
        dl = min(lane * VT, n)
        lo, hi = max(0, dl - wb), min(dl, wa)
        while lo < hi:
            m = (lo + hi) // 2
            if keys[ob + dl - 1 - m] < keys[oa + m]:
                hi = m
            else:
                lo = m + 1
        ai, bi = oa + lo, ob + dl - lo
        steps = min(n - dl, VT)
        # ranks of the lane's first A and B copies
        kA = kB = 0
        if ai < ae:
            v = keys[ai]
            if ai > oa and keys[ai - 1] == v:
                l = oa
                while keys[l] < v:
                    l += 1
                kA = ai - l if l > oa else (a0 + ai - oa) - lbA
            else:
                kA = 0 if ai > oa else a0 - lbA
        if bi < be:
            v = keys[bi]
            if bi > ob and keys[bi - 1] == v:
                l = ob
                while keys[l] < v:
                    l += 1
                kB = bi - l if l > ob else (b0 + bi - ob) - lbB
            else:
                kB = 0 if bi > ob else b0 - lbB
        kA0, kB0 = min(kA, SAT), min(kB, SAT)
        xA, xB = kA - kA0, kB - kB0
        sA0, sB0 = ai - kA0, bi - kB0
        sA, sB = sA0, sB0
        ka, kb = keys[ai], keys[bi]
        for s in range(VT):
            tb = bi < be and (ai >= ae or kb < ka)
            v = kb if tb else ka
            pos = bi if tb else ai
            st = sB if tb else sA
            r = pos - st
            idx = ai - 1 - r if tb else bi + r
            if oa <= idx < be:
                m = keys[idx] == v
            else:
                r64 = r + ((xB if st == sB0 else 0) if tb else (xA if st == sA0 else 0))
                q = a0 + (ai - oa) - 1 - r64 if tb else b0 + (bi - ob) + r64
                m = (q >= 0 if tb else q < nb) and int((A if tb else B)[q]) == v
            kept = (op in (1, 3) and not m) if tb else (op == 1 or (m if op == 0 else not m))
            if kept and s < steps:
                out.append(v)
            p1 = pos + 1
            nxt = keys[p1]
            st1 = st if nxt == v else p1
            if tb:
                bi, kb, sB = p1, nxt, st1
            else:
                ai, ka, sA = p1, nxt, st1
    return out


def _emulate(op, A, B, NT, VT, SAT, offA, offB, rng):
    T = NT * VT
    N = len(A) + len(B)
    out = []
    for d0 in range(0, N, T):
        out += _tile(OPS[op], A, B, d0, min(T, N - d0), NT, VT, SAT, offA, offB, rng)
    return np.array(out, dtype=A.dtype)


@pytest.mark.parametrize("seed", range(6))
def test_walk_model_matches_oracle(seed):
    rng = np.random.default_rng(700 + seed)
    for _ in range(12):
        na, nb = int(rng.integers(0, 260)), int(rng.integers(0, 260))
        hi = int(rng.choice([2, 3, 7, 40, 1 << 20]))
        A = np.sort(rng.integers(0, hi, na)).astype(np.uint32)
        B = np.sort(rng.integers(0, hi, nb)).astype(np.uint32)
        NT, VT = int(rng.choice([2, 3, 4])), int(rng.choice([1, 2, 3, 5, 7]))
        # lowest saturation that still puts every saturated partner outside
        # the LDS array, or the kernel's own 2^30
        SAT = int(rng.choice([NT * VT + 4 * CH + VT + 1, 1 << 30]))
        offA, offB = int(rng.integers(0, CH)), int(rng.integers(0, CH))
        for op in OPS:
            got = _emulate(op, A, B, NT, VT, SAT, offA, offB, rng)
            want = oracle.set_op(op, A, B)
            assert got.tobytes() == want.tobytes(), (op, na, nb, hi, NT, VT, SAT, offA, offB)


def test_walk_model_long_runs_saturate():
    """Runs far longer than a tile on both sides, so that lanes deep inside
    them start past the lowered saturation point."""
    rng = np.random.default_rng(720)
    for m, k in ((300, 170), (170, 300), (250, 250)):
        A = np.sort(np.concatenate([np.full(m, 5, np.uint32), rng.integers(0, 9, 20).astype(np.uint32)]))
        B = np.sort(np.concatenate([np.full(k, 5, np.uint32), rng.integers(0, 9, 20).astype(np.uint32)]))
        NT, VT = 3, 5
        SAT = NT * VT + 4 * CH + VT + 1
        for op in OPS:
            got = _emulate(op, A, B, NT, VT, SAT, 1, 2, rng)
            assert got.tobytes() == oracle.set_op(op, A, B).tobytes(), (op, m, k)
