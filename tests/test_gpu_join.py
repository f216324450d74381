"""GPU parity of mp_join (inner join through the merge partition) against
the oracle's nested-loop join, pair for pair."""
import numpy as np
import pytest
import torch

import mp_inputs as gen

pytestmark = pytest.mark.gpu

DTYPES = [gen.U32, gen.I32, gen.U64, gen.F32]


@pytest.fixture(scope="module")
def mp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    return mp


def _check(mp, orc, A, B):
    from gpu_util import dev, host
    I, J = mp.join(dev(A), dev(B))
    wi, wj, k = orc.join(A, B)
    assert len(I) == k, (len(A), len(B), len(I), k)
    assert np.array_equal(host(I), wi) and np.array_equal(host(J), wj)
    return k


@pytest.mark.parametrize("dt", DTYPES)
def test_join_uniform_and_duplicates(mp, orc, dt):
    g = np.random.default_rng(301)
    npd = gen.NP_DTYPE[dt]
    _check(mp, orc, *gen.uniform_pair(15_003, 12_001, 302, dt))     # few matches
    for hi in (3, 60, 2000):
        A = np.sort(g.integers(0, hi, 9_001 if hi == 3 else 15_001)).astype(npd)
        B = np.sort(g.integers(0, hi, 700 if hi == 3 else 12_007)).astype(npd)
        assert _check(mp, orc, A, B) > 0


def test_join_runs_longer_than_a_tile(mp, orc):
    """A run of one key far longer than a merge tile on either side, next to
    short runs and keys found on one side only."""
    g = np.random.default_rng(303)
    base = np.sort(g.integers(0, 5000, 8_000)).astype(np.uint32)
    A = np.sort(np.concatenate([base, np.full(20_000, 2500, np.uint32)]))
    B = np.sort(np.concatenate([base[::3], np.full(40, 2500, np.uint32)]))
    _check(mp, orc, A, B)
    A = np.sort(np.concatenate([base[::5], np.full(30, 777, np.uint32)]))
    B = np.sort(np.concatenate([base, np.full(25_000, 777, np.uint32)]))
    _check(mp, orc, A, B)


def test_join_edges(mp, orc):
    A = np.arange(0, 20_000, 2, dtype=np.uint32)
    cases = [(A, A + 1), (A, A.copy()), (A, A[:0]), (A[:0], A), (A[:0], A[:0]), (A[:1], A[:1]),
             (np.full(300, 7, np.uint32), np.full(200, 7, np.uint32)),
             (np.array([0, 0xFFFFFFFF], np.uint32), np.array([0xFFFFFFFF] * 3, np.uint32))]
    for A_, B_ in cases:
        _check(mp, orc, A_, B_)


def test_join_signed_zeros(mp, orc):
    A = np.array([-2.0, -0.0, -0.0, 0.0, 1.5], np.float32)
    B = np.array([-0.0, 0.0, 0.0, 1.5, 1.5], np.float32)
    assert _check(mp, orc, A, B) == 3 * 3 + 2


def test_join_cap_and_guards(mp, orc):
    """With room for fewer pairs than the join has, the first cap pairs are
    written, nothing past them, and count is the total; cap = 0 counts only."""
    from gpu_util import dev, host
    g = np.random.default_rng(304)
    A = np.sort(g.integers(0, 300, 12_000)).astype(np.uint32)
    B = np.sort(g.integers(0, 300, 9_000)).astype(np.uint32)
    wi, wj, k = orc.join(A, B)
    dA, dB = dev(A), dev(B)
    for cap in (0, 1, 1000, k - 1, k, k + 50):
        G = 8192  # guard words (int64) on each side
        Ib = torch.full((cap + 2 * G,), -7, dtype=torch.int64, device="cuda")
        Jb = torch.full((cap + 2 * G,), -9, dtype=torch.int64, device="cuda")
        cnt = torch.full((2 * G + 1,), -5, dtype=torch.int64, device="cuda")
        I, J, count = mp.join(dA, dB, cap=cap, I=Ib[G:G + cap] if cap else Ib[G:G],
                              J=Jb[G:G + cap] if cap else Jb[G:G], count=cnt[G:G + 1], sync=False)
        got_k = int(host(count)[0])
        ib, jb, cb = host(Ib), host(Jb), host(cnt)
        assert got_k == k
        assert (ib[:G] == -7).all() and (ib[G + cap:] == -7).all()
        assert (jb[:G] == -9).all() and (jb[G + cap:] == -9).all()
        assert (cb[:G] == -5).all() and (cb[G + 1:] == -5).all()
        m = min(cap, k)
        assert np.array_equal(ib[G:G + m], wi[:m]) and np.array_equal(jb[G:G + m], wj[:m])


def test_join_unsorted_inputs_stay_in_bounds(mp):
    """Sortedness is a precondition: unsorted inputs give unspecified pairs,
    but every store stays inside I, J (cap) and count."""
    from gpu_util import dev, host
    g = np.random.default_rng(305)
    A = g.integers(0, 40, 20_000).astype(np.uint32)
    B = g.integers(0, 40, 15_000).astype(np.uint32)
    G, cap = 4096, 100_000
    Ib = torch.full((cap + 2 * G,), -7, dtype=torch.int64, device="cuda")
    Jb = torch.full((cap + 2 * G,), -9, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    mp.join(dev(A), dev(B), cap=cap, I=Ib[G:G + cap], J=Jb[G:G + cap], count=cnt, sync=False)
    ib, jb = host(Ib), host(Jb)
    assert (ib[:G] == -7).all() and (ib[G + cap:] == -7).all()
    assert (jb[:G] == -9).all() and (jb[G + cap:] == -9).all()
    assert int(host(cnt)[0]) >= 0


@pytest.mark.parametrize("dt", [gen.U32, gen.U64])
def test_join_unaligned_views(mp, orc, dt):
    """A and B as views at element offsets that leave them off the 16-byte
    grid: the rank tiles read their windows in chunks aligned in memory,
    with element loads at the arrays' ends."""
    from gpu_util import dev, host
    g = np.random.default_rng(306)
    npd = gen.NP_DTYPE[dt]
    A = np.sort(g.integers(0, 30_000, 40_003)).astype(npd)
    B = np.sort(g.integers(0, 30_000, 35_001)).astype(npd)
    wi, wj, k = orc.join(A, B)
    for oa, ob in ((1, 2), (3, 0), (0, 1), (2, 3)):
        dA = dev(np.concatenate([np.zeros(oa, npd), A]))[oa:]
        dB = dev(np.concatenate([np.zeros(ob, npd), B]))[ob:]
        I, J = mp.join(dA, dB)
        assert len(I) == k, (oa, ob, len(I), k)
        assert np.array_equal(host(I), wi) and np.array_equal(host(J), wj), (oa, ob)


def test_join_workspace_alignment(mp, orc):
    """The offsets array sits on 16 bytes inside the workspace whatever the
    caller's 8-byte-aligned workspace and the parity of |A|: both parities,
    with the workspace at a 16-byte and at an 8-byte (not 16-byte) address."""
    from gpu_util import dev, host
    g = np.random.default_rng(307)
    for na in (20_001, 20_002):
        A = np.sort(g.integers(0, 9_000, na)).astype(np.uint32)
        B = np.sort(g.integers(0, 9_000, 17_003)).astype(np.uint32)
        wi, wj, k = orc.join(A, B)
        need = mp.lib().mp_join_workspace_bytes(na, len(B))
        for shift in (0, 8):
            ws = torch.empty(need + 16, dtype=torch.uint8, device="cuda")[shift:shift + need]
            I, J = mp.join(dev(A), dev(B), ws=ws)
            assert len(I) == k, (na, shift)
            assert np.array_equal(host(I), wi) and np.array_equal(host(J), wj), (na, shift)


def test_join_tile_boundaries(mp, orc):
    """Total sizes at and next to whole numbers of 2048-key rank tiles, one
    input empty or tiny, with few and with many distinct keys (runs of one
    value then straddle the rank tiles and the emission tiles)."""
    g = np.random.default_rng(308)
    T = 2048
    for total in (T - 1, T, T + 1, 2 * T, 5 * T - 1, 5 * T + 1):
        for na in (0, 1, total // 3, total // 2, total - 1, total):
            nb = total - na
            for hi in (5, 1 << 20):
                A = np.sort(g.integers(0, hi, na)).astype(np.uint32)
                B = np.sort(g.integers(0, hi, nb)).astype(np.uint32)
                _check(mp, orc, A, B)
