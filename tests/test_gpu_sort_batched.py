"""GPU parity of mp_sort (block sort + merge rounds) and mp_merge_batched."""
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
    yield mp
    mp.set_config("sort", None)
    mp.set_config("batched", None)


# ------------------------------------------------------------------ sort

@pytest.mark.parametrize("n", [0, 1, 2, 7, 17, 2047, 2048, 2049, 4095, 4096, 4097, 6145, 8191,
                               8192, 8193, 12_289, 16_383, 16_384, 16_385, 3 * 16_384 + 5,
                               100_003, 1 << 20])
def test_sort_sizes(mp, orc, n):
    from gpu_util import dev, host, first_mismatch
    keys = gen.unsorted_uniform(n, 100 + n)
    got = host(mp.sort(dev(keys)))
    assert first_mismatch(got, orc.sort(keys)) is None, n


@pytest.mark.parametrize("dt", DTYPES)
def test_sort_dtypes(mp, orc, dt):
    from gpu_util import dev, host, first_mismatch
    keys = gen.unsorted_uniform(300_001, 7, dt)
    if dt == gen.F32:
        keys[::97] = np.float32(0.0)
        keys[::89] = np.float32(-0.0)
    got = host(mp.sort(dev(keys)))
    assert first_mismatch(got, orc.sort(keys)) is None


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", [1000, 4097, 5003, 8192 + 777, 16_384 + 1001])
def test_sort_largest_keys_in_partial_blocks(mp, orc, dt, n):
    """The last block pads one lane's registers with the largest key; real
    keys equal to it (and +inf for floats) must still come out in input
    order, with their values."""
    from gpu_util import dev, host, first_mismatch
    g = np.random.default_rng(n)
    top = np.inf if dt == gen.F32 else np.iinfo(gen.NP_DTYPE[dt]).max
    keys = g.integers(0, 50, n).astype(gen.NP_DTYPE[dt])
    keys[g.random(n) < 0.3] = top
    vals = np.arange(n, dtype=np.uint32)
    assert first_mismatch(host(mp.sort(dev(keys))), orc.sort(keys)) is None
    gk, gv = mp.sort(dev(keys), dev(vals))
    wk, wv = orc.sort(keys, vals)
    assert first_mismatch(host(gk), wk) is None
    assert first_mismatch(host(gv), wv) is None


@pytest.mark.parametrize("dt", [gen.U32, gen.I32, gen.F32, gen.U64])
def test_sort_kv_stable(mp, orc, dt):
    """Values follow keys; equal keys keep their input order (stability)."""
    from gpu_util import dev, host, first_mismatch
    g = np.random.default_rng(3)
    n = 250_007
    keys = g.integers(0, 500, n).astype(gen.NP_DTYPE[dt])
    vals = np.arange(n, dtype=np.uint32)
    gk, gv = mp.sort(dev(keys), dev(vals))
    wk, wv = orc.sort(keys, vals)
    assert first_mismatch(host(gk), wk) is None
    assert first_mismatch(host(gv), wv) is None


def test_sort_block_sizes(mp):
    """Blocks are sized per key width (and never too large for the LDS)."""
    import torch
    b4 = mp.sort_block_keys(torch.uint32)
    assert b4 == mp.sort_block_keys(torch.float32, torch.uint32) == mp.sort_block_keys(torch.int32)
    b8 = mp.sort_block_keys(torch.uint64, torch.uint32)
    assert 4096 <= b8 <= 8192 and 4096 <= b4 <= 16384


def test_sort_zipf(mp, orc):
    from gpu_util import dev, host, first_mismatch
    keys = gen.zipf_keys(1 << 20, 32)
    got = host(mp.sort(dev(keys)))
    assert first_mismatch(got, orc.sort(keys)) is None


def test_sort_presorted_and_reversed(mp, orc):
    from gpu_util import dev, host, first_mismatch
    a = np.arange(200_000, dtype=np.uint32)
    for keys in (a, a[::-1].copy(), np.full(70_001, 5, np.uint32)):
        got = host(mp.sort(dev(keys)))
        assert first_mismatch(got, orc.sort(keys)) is None


def test_sort_rejects_tiles_that_do_not_divide_run_pairs(mp):
    with pytest.raises(mp.MergePathError, match="UNSUPPORTED"):
        mp.set_config("sort", 2, 256, 12)
    mp.set_config("sort", None)


@pytest.mark.parametrize("variant", [(2, 256, 8, 0, 0), (2, 512, 8, 0, 0), (2, 128, 16, 0, 0),
                                     (2, 512, 16, 0, 0), (2, 256, 16, 0, -1), (2, 256, 16, 0, 1),
                                     (2, 128, 16, 3, 0)])
def test_sort_round_variants(mp, orc, variant):
    from gpu_util import dev, host, first_mismatch
    mp.set_config("sort", *variant)
    try:
        keys = gen.unsorted_uniform(150_001, 5)
        vals = np.arange(len(keys), dtype=np.uint32)
        gk, gv = mp.sort(dev(keys), dev(vals))
        wk, wv = orc.sort(keys, vals)
        assert first_mismatch(host(gk), wk) is None
        assert first_mismatch(host(gv), wv) is None
    finally:
        mp.set_config("sort", None)


# ------------------------------------------------------------------ batched

def _batched_case(n_pairs, seed, median):
    A, a_off, B, b_off = gen.batched_pairs(n_pairs, seed, median=median)
    return A, a_off, B, b_off


@pytest.mark.parametrize("n_pairs,median", [(1, 5000), (3, 20000), (200, 4096), (2000, 64),
                                            (5000, 3), (300, 30000)])
def test_batched(mp, orc, n_pairs, median):
    from gpu_util import dev, host, first_mismatch
    A, a_off, B, b_off = _batched_case(n_pairs, 41 + n_pairs, median)
    got = host(mp.merge_batched(dev(A), dev(a_off), dev(B), dev(b_off)))
    assert first_mismatch(got, orc.merge_batched(A, a_off, B, b_off)) is None


def test_batched_empty_and_skewed_pairs(mp, orc):
    """Empty pairs, one-sided pairs and runs of many empty pairs."""
    from gpu_util import dev, host, first_mismatch
    g = np.random.default_rng(8)
    na = g.integers(0, 50, 3000)
    nb = g.integers(0, 50, 3000)
    na[100:1500] = 0
    nb[100:1500] = 0          # a long run of empty pairs
    na[2000:2100] = 0         # B-only pairs
    nb[2200:2300] = 0         # A-only pairs
    na[2500] = 70_000         # one large pair
    a_off, b_off = gen.offsets(na), gen.offsets(nb)
    A = np.concatenate([np.sort(g.integers(-2**31, 2**31, k)).astype(np.int32) for k in na])
    B = np.concatenate([np.sort(g.integers(-2**31, 2**31, k)).astype(np.int32) for k in nb])
    got = host(mp.merge_batched(dev(A), dev(a_off), dev(B), dev(b_off)))
    assert first_mismatch(got, orc.merge_batched(A, a_off, B, b_off)) is None


@pytest.mark.parametrize("dt", DTYPES)
def test_batched_dtypes_dups(mp, orc, dt):
    from gpu_util import dev, host, first_mismatch
    g = np.random.default_rng(12)
    na, nb = g.integers(0, 3000, 150), g.integers(0, 3000, 150)
    a_off, b_off = gen.offsets(na), gen.offsets(nb)
    npd = gen.NP_DTYPE[dt]
    A = np.concatenate([np.sort(g.integers(0, 20, k)).astype(npd) for k in na])
    B = np.concatenate([np.sort(g.integers(0, 20, k)).astype(npd) for k in nb])
    got = host(mp.merge_batched(dev(A), dev(a_off), dev(B), dev(b_off)))
    assert first_mismatch(got, orc.merge_batched(A, a_off, B, b_off)) is None


@pytest.mark.parametrize("variant", [(2, 256, 8, 0, 0), (2, 256, 12, 0, 0), (2, 512, 8, 0, 0),
                                     (2, 512, 16, 0, 0), (2, 256, 16, 0, -1), (2, 256, 16, 0, 1),
                                     (2, 128, 16, 5, 0)])
def test_batched_variants(mp, orc, variant):
    from gpu_util import dev, host, first_mismatch
    mp.set_config("batched", *variant)
    try:
        A, a_off, B, b_off = _batched_case(700, 43, 900)
        got = host(mp.merge_batched(dev(A), dev(a_off), dev(B), dev(b_off)))
        assert first_mismatch(got, orc.merge_batched(A, a_off, B, b_off)) is None
    finally:
        mp.set_config("batched", None)
