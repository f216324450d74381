"""GPU parity of mp_partition, mp_merge and mp_merge_kv against the oracle (bit-exact)."""
import numpy as np
import pytest

import mp_inputs as gen

pytestmark = pytest.mark.gpu

DTYPES = [gen.U32, gen.I32, gen.U64, gen.F32]


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    return mp


def _cases():
    # (na, nb) spanning several tiles, ragged tails, empties and skewed lengths
    return [(0, 0), (0, 5), (7, 0), (1, 1), (1, 4096), (4096, 1), (4095, 4097),
            (100_003, 77_777), (3, 250_000), (250_000, 3), (1 << 17, 1 << 17)]


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("na,nb", _cases())
def test_merge_uniform(mp, orc, dt, na, nb):
    from gpu_util import dev, host, first_mismatch
    A, B = gen.uniform_pair(na, nb, 1000 + na + 7 * nb, dt)
    got = host(mp.merge(dev(A), dev(B)))
    want = orc.merge(A, B)
    assert first_mismatch(got, want) is None, first_mismatch(got, want)


@pytest.mark.parametrize("kind", ["dups", "disjoint", "disjoint_rev", "all_equal"])
def test_merge_structured(mp, orc, kind):
    from gpu_util import dev, host, first_mismatch
    na, nb = 300_001, 200_017
    if kind == "dups":
        A, B = gen.dups_pair(na, nb, 22)
    elif kind == "disjoint":
        A, B = gen.disjoint_pair(na, nb, 23)
    elif kind == "disjoint_rev":
        B, A = gen.disjoint_pair(nb, na, 23)
    else:
        A, B = np.full(na, 7, np.uint32), np.full(nb, 7, np.uint32)
    got = host(mp.merge(dev(A), dev(B)))
    assert first_mismatch(got, orc.merge(A, B)) is None


def test_merge_config1(mp, orc):
    """|A| = |B| = 2^20 uniform u32 keys (seed 1)."""
    from gpu_util import dev, host, first_mismatch
    A, B = gen.uniform_pair(1 << 20, 1 << 20, 1)
    got = host(mp.merge(dev(A), dev(B)))
    assert first_mismatch(got, orc.merge(A, B)) is None


def test_merge_extreme_keys(mp, orc):
    from gpu_util import dev, host, first_mismatch
    g = np.random.default_rng(5)
    for dt, lo, hi in [(np.uint32, 0, 2**32 - 1), (np.int32, -2**31, 2**31 - 1),
                       (np.uint64, 0, 2**64 - 1)]:
        A = np.sort(g.choice(np.array([lo, hi, lo + 1, hi - 1], dtype=dt), 10_000))
        B = np.sort(g.choice(np.array([lo, hi], dtype=dt), 7_000))
        got = host(mp.merge(dev(A), dev(B)))
        assert first_mismatch(got, orc.merge(A, B)) is None
    f = np.finfo(np.float32).max
    A = np.sort(g.choice(np.array([-f, -0.0, 0.0, f], dtype=np.float32), 10_000))
    B = np.sort(g.choice(np.array([-f, 0.0, -0.0, f], dtype=np.float32), 9_000))
    got = host(mp.merge(dev(A), dev(B)))
    assert first_mismatch(got, orc.merge(A, B)) is None


def test_merge_f32_mixture_signed_zeros(mp, orc):
    from gpu_util import dev, host, first_mismatch
    A, B = gen.f32_mixture_pair(200_000, 150_000, 51)
    assert np.any(np.signbit(A) & (A == 0))
    got = host(mp.merge(dev(A), dev(B)))
    assert first_mismatch(got, orc.merge(A, B)) is None


@pytest.mark.parametrize("dt", DTYPES)
def test_partition(mp, orc, dt):
    from gpu_util import dev, host
    A, B = gen.uniform_pair(50_000, 30_001, 3, dt)
    n = len(A) + len(B)
    g = np.random.default_rng(0)
    diag = np.concatenate([[0, n, 1, n - 1], g.integers(0, n + 1, 5000)]).astype(np.int64)
    got = host(mp.partition(dev(A), dev(B), dev(diag)))
    assert np.array_equal(got, orc.partition(A, B, diag))


def _position_checksum(S):
    """sum of S[i] * (i + 1) modulo 2^64, keys as unsigned bits."""
    bits = S.view(np.uint64) if S.dtype.itemsize == 8 else S.view(np.uint32).astype(np.uint64)
    with np.errstate(over="ignore"):
        return int(np.sum(bits * np.arange(1, len(S) + 1, dtype=np.uint64), dtype=np.uint64))


def _tile_diagonals(n, tile):
    return np.minimum(np.arange((n + tile - 1) // tile + 1, dtype=np.int64) * tile, n)


@pytest.mark.parametrize("tile", [2048, 3840, 4096, 8192, 16384])
def test_merge_split_from_partition(mp, orc, tile):
    """Algorithm 1 in two calls: splits on the tile diagonals, then the tiles
    merged independently, gives the oracle's merge."""
    from gpu_util import dev, host, first_mismatch
    cases = [gen.uniform_pair(100_003, 77_777, 71, dt) for dt in DTYPES]
    cases += [gen.dups_pair(50_001, 60_007, 72, hi=9), gen.disjoint_pair(40_000, 30_001, 73),
              gen.uniform_pair(5, 60_000, 74), gen.uniform_pair(0, 1000, 75),
              gen.uniform_pair(1, 0, 76), gen.uniform_pair(tile, tile, 77)]
    for A, B in cases:
        n = len(A) + len(B)
        d = _tile_diagonals(n, tile)
        dA, dB = dev(A), dev(B)
        sp = mp.partition(dA, dB, dev(d))
        if tile * A.itemsize > 64 * 1024:
            # a tile of 8-byte keys that would need 128 KiB of LDS is not built
            with pytest.raises(mp.MergePathError, match="MP_ERR_UNSUPPORTED"):
                mp.merge_split(dA, dB, sp, tile)
            continue
        got = host(mp.merge_split(dA, dB, sp, tile))
        assert first_mismatch(got, orc.merge(A, B)) is None, (A.dtype, len(A), len(B))


def test_merge_split_keeps_any_splits_in_bounds(mp, orc):
    """Split values that are not the true splits (out of range, decreasing,
    random) give some other output, but every access stays inside the
    arrays: the kernel clamps each split to its diagonal's extent."""
    import torch
    from gpu_util import dev, host
    A, B = gen.uniform_pair(30_001, 20_011, 78)
    n = len(A) + len(B)
    k = (n + 4095) // 4096 + 1
    g = np.random.default_rng(79)
    for sp in (np.full(k, 1 << 62, np.int64), np.full(k, -5, np.int64),
               np.arange(k, dtype=np.int64)[::-1].copy() * 4096, g.integers(-n, 2 * n, k)):
        out = mp.merge_split(dev(A), dev(B), dev(sp), 4096)
        torch.cuda.synchronize()
        assert host(out).shape == (n,)
    # the true splits still give the merge afterwards
    d = _tile_diagonals(n, 4096)
    got = host(mp.merge_split(dev(A), dev(B), mp.partition(dev(A), dev(B), dev(d)), 4096))
    assert np.array_equal(got, orc.merge(A, B))


@pytest.mark.parametrize("cfg", [None, (2, 256, 16, 0, 0), (2, 192, 24, 5, 0), (2, 256, 16, 0, 64)])
def test_merge_checksum_no_store(mp, orc, cfg):
    """The merge kept in registers (nothing stored) accounts for every output
    at its position: its checksum equals the oracle merge's."""
    from gpu_util import dev, host
    if cfg is not None:
        mp.set_config("merge", *cfg)
    try:
        cases = [gen.uniform_pair(300_007, 200_003, 61, dt) for dt in DTYPES]
        cases += [gen.dups_pair(150_001, 90_007, 62, hi=50), gen.disjoint_pair(70_000, 50_001, 63),
                  gen.uniform_pair(0, 5000, 64), gen.uniform_pair(4999, 0, 65), gen.uniform_pair(1, 1, 66)]
        A, B = gen.f32_mixture_pair(100_000, 80_001, 67)
        cases.append((A, B))
        for A, B in cases:
            got = int(host(mp.merge_checksum(dev(A), dev(B)))[0])
            assert got == _position_checksum(orc.merge(A, B)), (A.dtype, len(A), len(B))
    finally:
        mp.set_config("merge", None)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64, 0])
def test_partition_lanes_per_diagonal(mp, orc, lanes):
    """Every group size of the search (forced, and chosen per call for launch
    sizes that pick different groups) gives the oracle's splits."""
    from gpu_util import dev, host
    mp.set_partition_lanes(lanes)
    try:
        for dt in (gen.U32, gen.I32, gen.U64, gen.F32):
            A, B = gen.uniform_pair(70_001, 40_003, 5, dt)
            n = len(A) + len(B)
            for n_diag in (1, 3, 65, 5003, 20_011, 70_001):
                g = np.random.default_rng(n_diag)
                diag = np.concatenate([[0, n, 1, n - 1], g.integers(-5, n + 6, n_diag)]).astype(np.int64)
                got = host(mp.partition(dev(A), dev(B), dev(diag)))
                assert np.array_equal(got, orc.partition(A, B, np.clip(diag, 0, n))), (dt, n_diag)
        for (na, nb) in [(1, 100_000), (100_000, 1), (0, 10), (10, 0), (30_000, 30_000)]:
            A, B = gen.dups_pair(na, nb, 9, hi=7)
            n = na + nb
            diag = np.arange(0, n + 1, max(1, n // 997), dtype=np.int64)
            got = host(mp.partition(dev(A), dev(B), dev(diag)))
            assert np.array_equal(got, orc.partition(A, B, diag)), (na, nb)
    finally:
        mp.set_partition_lanes(0)


def test_partition_dups_and_skew(mp, orc):
    from gpu_util import dev, host
    for (na, nb) in [(1, 100_000), (100_000, 1), (0, 10), (10, 0)]:
        A, B = gen.dups_pair(na, nb, 9, hi=16)
        n = na + nb
        diag = np.arange(0, n + 1, max(1, n // 997), dtype=np.int64)
        got = host(mp.partition(dev(A), dev(B), dev(diag)))
        assert np.array_equal(got, orc.partition(A, B, diag))


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("kind", ["uniform", "dups", "disjoint"])
def test_merge_kv(mp, orc, dt, kind):
    from gpu_util import dev, host, first_mismatch
    na, nb = 123_457, 98_765
    if kind == "uniform":
        A, B = gen.uniform_pair(na, nb, 21, dt)
    elif kind == "dups":
        A, B = gen.dups_pair(na, nb, 22)
        A, B = A.astype(gen.NP_DTYPE[dt]), B.astype(gen.NP_DTYPE[dt])
    else:
        A, B = gen.disjoint_pair(na, nb, 23)
        A, B = A.astype(gen.NP_DTYPE[dt]), B.astype(gen.NP_DTYPE[dt])
    va, vb = gen.index_payload(na, nb)
    gk, gv = mp.merge_kv(dev(A), dev(va), dev(B), dev(vb))
    wk, wv = orc.merge_kv(A, va, B, vb)
    assert first_mismatch(host(gk), wk) is None
    assert first_mismatch(host(gv), wv) is None
