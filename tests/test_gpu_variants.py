"""Every compiled kernel variant (the autotuner's candidates) gives the oracle's bits."""
import numpy as np
import pytest

import mp_inputs as gen

pytestmark = pytest.mark.gpu

MERGE_VARIANTS = [(1, 256, 16, 0), (1, 256, 15, 0), (1, 256, 8, 0), (1, 128, 16, 0),
                  (2, 256, 16, 0), (2, 256, 8, 0), (2, 256, 12, 0), (2, 256, 14, 0),
                  (2, 256, 18, 0), (2, 128, 16, 0), (2, 192, 24, 0),
                  (2, 512, 8, 0), (2, 512, 16, 0), (2, 256, 16, 7), (2, 256, 16, 1)]
FOUR_BYTE_ONLY = {(512, 16)}  # persistent tiles compiled for 4-byte keys only


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    yield mp
    mp.set_config("merge", None)


@pytest.mark.parametrize("variant", MERGE_VARIANTS, ids=lambda v: "m%d_nt%d_vt%d_g%d" % v)
def test_merge_variants(mp, orc, variant):
    from gpu_util import dev, host, first_mismatch
    mode, nt, vt, grid = variant
    mp.set_config("merge", mode, nt, vt, grid)
    try:
        for (na, nb, seed) in [(100_003, 77_777, 1), (5, 60_000, 2), (60_000, 5, 3), (0, 1000, 4)]:
            for dt in (gen.U32, gen.U64):
                A, B = gen.uniform_pair(na, nb, seed, dt)
                if dt == gen.U64 and (nt, vt) in FOUR_BYTE_ONLY and mode == 2 and na + nb > 0:
                    with pytest.raises(mp.MergePathError, match="UNSUPPORTED"):
                        mp.merge(dev(A), dev(B))
                    continue
                got = host(mp.merge(dev(A), dev(B)))
                assert first_mismatch(got, orc.merge(A, B)) is None, (na, nb, dt)
        A, B = gen.dups_pair(50_001, 70_003, 7, hi=100)
        va, vb = gen.index_payload(len(A), len(B))
        gk, gv = mp.merge_kv(dev(A), dev(va), dev(B), dev(vb))
        wk, wv = orc.merge_kv(A, va, B, vb)
        assert first_mismatch(host(gk), wk) is None
        assert first_mismatch(host(gv), wv) is None
    finally:
        mp.set_config("merge", None)


@pytest.mark.parametrize("margin", [-1, 1, 7, 0, 100000])
@pytest.mark.parametrize("vt", [8, 12])
def test_speculative_window_margins(mp, orc, margin, vt):
    """Tiny margins force the exact full-window reload on almost every tile;
    -1 disables speculation.  Every setting must give the oracle's bits.
    The grid is 8 workgroups, so each walks dozens of tiles and every tile
    after its first merges from windows sized (or reloaded) from the tile
    before it."""
    from gpu_util import dev, host, first_mismatch
    grid = 8
    mp.set_config("merge", 2, 256, vt, grid, margin)
    try:
        cases = [gen.uniform_pair(200_003, 150_001, 31), gen.dups_pair(180_001, 170_003, 32, hi=40),
                 gen.disjoint_pair(120_000, 90_001, 33), gen.uniform_pair(7, 300_000, 34),
                 gen.uniform_pair(300_000, 7, 35)]
        for i, (A, B) in enumerate(cases):
            mp.timing_enable(True)
            got = host(mp.merge(dev(A), dev(B)))
            tiles, reloads = mp.stats_query()
            groups = mp.stats_workgroups()
            mp.timing_enable(False)
            assert first_mismatch(got, orc.merge(A, B)) is None, (len(A), len(B), margin)
            assert groups == grid and tiles == -(-(len(A) + len(B)) // (256 * vt)), (tiles, groups)
            assert tiles >= 6 * groups
            if margin < 0:
                assert reloads == 0, reloads          # full windows never miss
            if margin == 1 and i == 0:
                # uniform keys: the A/B mix of a tile wanders by about
                # sqrt(T) keys, so a one-key margin misses on most tiles
                assert reloads > (tiles - groups) // 2, (reloads, tiles)
        A, B = gen.dups_pair(100_001, 90_007, 36, hi=30)
        va, vb = gen.index_payload(len(A), len(B))
        gk, gv = mp.merge_kv(dev(A), dev(va), dev(B), dev(vb))
        wk, wv = orc.merge_kv(A, va, B, vb)
        assert first_mismatch(host(gk), wk) is None
        assert first_mismatch(host(gv), wv) is None
    finally:
        mp.timing_enable(False)
        mp.set_config("merge", None)


def _equal_key_runs(n, seed):
    """Sorted pair made of long runs of few distinct keys: the A/B mix of
    consecutive tiles flips between all-A and all-B."""
    g = np.random.default_rng(seed)
    vals = np.sort(g.choice(1 << 30, 200, replace=False)).astype(np.uint32)
    w = 1.0 / np.arange(1, 201)  # Zipf(1) masses in random key order
    g.shuffle(w)
    p = w / w.sum()
    A = np.sort(g.choice(vals, n, p=p)).astype(np.uint32)
    B = np.sort(g.choice(vals, n + 12_345, p=p)).astype(np.uint32)
    return A, B


@pytest.mark.parametrize("kind", ["merge", "sort"])
def test_lookahead_windows_on_equal_key_runs(mp, orc, kind):
    """The default window sizing switches to lookahead probes once the
    prediction misses: same bits as the oracle, and far fewer window reloads
    than prediction alone (margin > 0)."""
    from gpu_util import dev, host, first_mismatch
    A, B = _equal_key_runs(600_000, 5)
    reloads = {}
    for margin in (0, 64):
        # a small grid: every workgroup walks dozens of tiles
        mp.set_config(kind, 2, 256, 16, 8, margin)
        try:
            mp.timing_enable(True)
            if kind == "merge":
                got = host(mp.merge(dev(A), dev(B)))
                want = orc.merge(A, B)
            else:
                keys = np.concatenate([A, B])
                np.random.default_rng(9).shuffle(keys)
                got = host(mp.sort(dev(keys)))
                want = orc.sort(keys)
            reloads[margin] = mp.stats_query()[1]
            mp.timing_enable(False)
        finally:
            mp.set_config(kind, None)
        assert first_mismatch(got, want) is None, margin
    assert reloads[64] > 50, reloads
    assert reloads[0] * 4 < reloads[64], reloads


def test_unaligned_views(mp, orc):
    """Sub-array views whose base is not 16-byte aligned take the element-wise path."""
    import torch
    from gpu_util import dev, host, first_mismatch
    A, B = gen.uniform_pair(30_001, 20_003, 9)
    dA, dB = dev(A), dev(B)
    out = torch.empty((len(A) - 1) + (len(B) - 3) + 1, dtype=torch.uint32, device="cuda")
    got = host(mp.merge(dA[1:], dB[3:], out=out[1:]))
    assert first_mismatch(got, orc.merge(A[1:], B[3:])) is None


def test_copy_reference(mp):
    import torch
    x = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    mp.copy(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


@pytest.mark.parametrize("dt", [gen.U32, gen.U64])
def test_short_last_tile(mp, orc, dt):
    """Per-tile merges (split kernel, then tiles; 256 x 15 tiles) whose last
    tile is shorter than the 32-byte header that carries a tile's splits:
    that tile steps the path back from the grid's end instead.  Uniform
    keys and heavy duplicates (backwards, ties go to B), keys and
    key-value."""
    from gpu_util import dev, host, first_mismatch
    mp.set_config("merge", 1, 256, 15)
    try:
        for r in (1, 3, 7):
            N = 3 * 3840 + r
            for frac in (0.3, 0.7):
                na = int(N * frac)
                nb = N - na
                for dups in (False, True):
                    if dups:
                        g = np.random.default_rng(600 + r)
                        npd = gen.NP_DTYPE[dt]
                        A = np.sort(g.integers(0, 5, na)).astype(npd)
                        B = np.sort(g.integers(0, 5, nb)).astype(npd)
                    else:
                        A, B = gen.uniform_pair(na, nb, 500 + r, dt)
                    got = host(mp.merge(dev(A), dev(B)))
                    assert first_mismatch(got, orc.merge(A, B)) is None, (r, frac, dups)
                    va, vb = gen.index_payload(na, nb)
                    gk, gv = mp.merge_kv(dev(A), dev(va), dev(B), dev(vb))
                    wk, wv = orc.merge_kv(A, va, B, vb)
                    assert first_mismatch(host(gk), wk) is None and first_mismatch(host(gv), wv) is None
    finally:
        mp.set_config("merge", None)
