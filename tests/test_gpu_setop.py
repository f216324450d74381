"""GPU parity of mp_set_op (multiset operations through the partition)
against the oracle, bit for bit."""
import numpy as np
import pytest

import mp_inputs as gen

pytestmark = pytest.mark.gpu

OPS = ["intersection", "union", "difference", "symmetric_difference"]
DTYPES = [gen.U32, gen.I32, gen.U64, gen.F32]


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    return mp


def _check(mp, orc, op, A, B):
    from gpu_util import dev, host
    got = host(mp.set_op(op, dev(A), dev(B)))
    want = orc.set_op(op, A, B)
    assert got.dtype == want.dtype and got.tobytes() == want.tobytes(), (op, len(A), len(B), len(got), len(want))


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dt", DTYPES)
def test_set_op_uniform_and_dups(mp, orc, op, dt):
    # distinct-ish keys, few matches; and heavy duplicates, many matches
    _check(mp, orc, op, *gen.uniform_pair(100_003, 77_777, 81, dt))
    g = np.random.default_rng(82)
    npd = gen.NP_DTYPE[dt]
    for hi in (3, 50, 5000):
        A = np.sort(g.integers(0, hi, 90_001)).astype(npd)
        B = np.sort(g.integers(0, hi, 60_007)).astype(npd)
        _check(mp, orc, op, A, B)


@pytest.mark.parametrize("op", OPS)
def test_set_op_edges(mp, orc, op):
    g = np.random.default_rng(83)
    A = np.sort(g.integers(0, 1 << 20, 50_000)).astype(np.uint32)
    cases = [(A, A.copy()),                                    # identical
             (A, (A + (1 << 21)).astype(np.uint32)),           # disjoint, B above
             ((A + (1 << 21)).astype(np.uint32), A),           # disjoint, A above
             (A, A[:0]), (A[:0], A), (A[:1], A[:1]), (A[:0], A[:0]),
             (np.full(20_000, 7, np.uint32), np.full(30_000, 7, np.uint32)),   # one long run
             (np.full(30_000, 7, np.uint32), np.full(9_000, 7, np.uint32)),
             (np.repeat(np.arange(100, dtype=np.uint32), 97), np.repeat(np.arange(50, 150, dtype=np.uint32), 61)),
             (np.array([0, 0xFFFFFFFF], np.uint32), np.array([0xFFFFFFFF] * 3, np.uint32))]
    for A_, B_ in cases:
        _check(mp, orc, op, A_, B_)


@pytest.mark.parametrize("op", OPS)
def test_set_op_signed_zeros_and_mixture(mp, orc, op):
    """Equal keys with different bits: which copies are kept must match."""
    A, B = gen.f32_mixture_pair(120_000, 90_001, 84)
    _check(mp, orc, op, A, B)
    z = np.array([-0.0, 0.0], np.float32)
    g = np.random.default_rng(85)
    A = np.sort(g.choice(z, 10_000)).astype(np.float32)
    A = np.concatenate([A, np.float32([1.0] * 5)])
    B = np.concatenate([g.choice(z, 17_000).astype(np.float32), np.float32([1.0] * 9)])
    _check(mp, orc, op, A, B)


@pytest.mark.parametrize("op", OPS)
def test_set_op_runs_across_many_tiles(mp, orc, op):
    """Runs of equal keys longer than a tile, starting anywhere: the global
    run-start search of each tile."""
    g = np.random.default_rng(86)
    vals = np.sort(g.choice(1 << 30, 20, replace=False)).astype(np.uint32)
    A = np.sort(g.choice(vals, 400_000)).astype(np.uint32)
    B = np.sort(g.choice(vals, 300_001)).astype(np.uint32)
    _check(mp, orc, op, A, B)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dt", [gen.U32, gen.U64])
def test_set_op_lookback_over_many_tiles(mp, orc, op, dt):
    """Hundreds of tiles, so each output offset adds up more than one round
    of 64 predecessors; the sizes leave a ragged last tile."""
    _check(mp, orc, op, *gen.uniform_pair(1_500_007, 1_300_001, 87, dt))
    g = np.random.default_rng(88)
    npd = gen.NP_DTYPE[dt]
    A = np.sort(g.integers(0, 2_000_000, 1_500_007)).astype(npd)
    B = np.sort(g.integers(0, 2_000_000, 1_300_001)).astype(npd)
    _check(mp, orc, op, A, B)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dt", [gen.U32, gen.U64])
def test_set_op_unaligned_views(mp, orc, op, dt):
    """A, B and S as views at element offsets that leave them off the 16-byte
    grid: the windows are read and the output written in chunks aligned in
    memory, with element accesses at the ends."""
    from gpu_util import dev, host
    g = np.random.default_rng(89)
    npd = gen.NP_DTYPE[dt]
    A = np.sort(g.integers(0, 40_000, 70_001)).astype(npd)
    B = np.sort(g.integers(0, 40_000, 50_003)).astype(npd)
    want = orc.set_op(op, A, B)
    for oa, ob, os_ in ((1, 2, 3), (3, 0, 1), (2, 1, 0), (0, 3, 2)):
        dA = dev(np.concatenate([np.zeros(oa, npd), A]))[oa:]
        dB = dev(np.concatenate([np.zeros(ob, npd), B]))[ob:]
        cap = len(A) + len(B)
        base = dev(np.full(cap + os_ + 8, 0x5A, npd))
        out, count = mp.set_op(op, dA, dB, out=base[os_:os_ + cap], sync=False)
        k = int(host(count)[0])
        full = host(base)
        assert k == len(want), (op, oa, ob, os_, k, len(want))
        assert full[os_:os_ + k].tobytes() == want.tobytes(), (op, oa, ob, os_)
        assert np.all(full[:os_] == 0x5A) and np.all(full[os_ + cap:] == 0x5A), (op, oa, ob, os_)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dt", [gen.U32, gen.U64])
def test_set_op_tile_boundaries(mp, orc, op, dt):
    """Total sizes at and next to whole numbers of tiles (12800 keys for
    4-byte keys, 6656 for 8-byte keys, and small multiples), one input
    empty or tiny, and runs of one value that straddle the tile ends."""
    g = np.random.default_rng(90)
    npd = gen.NP_DTYPE[dt]
    T = 12800 if dt == gen.U32 else 6656
    for total in (T - 1, T, T + 1, 2 * T, 3 * T - 1, 3 * T + 1):
        for na in (0, 1, total // 3, total // 2, total - 1, total):
            nb = total - na
            for hi in (4, 1 << 20):
                A = np.sort(g.integers(0, hi, na)).astype(npd)
                B = np.sort(g.integers(0, hi, nb)).astype(npd)
                _check(mp, orc, op, A, B)
