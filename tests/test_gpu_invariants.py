"""Output-range invariants on the GPU.

Theorem 5 and Corollary 6: every partition pair writes exactly its own
contiguous range of S, and the ranges tile S.  So a call must write every
slot of its output and nothing outside it.  Each output here sits between
64 KiB guards filled with a byte pattern; after the call the guards must be
unchanged, and the output itself (filled with a different pattern before
each of two calls) must equal the oracle's both times, so every slot was
written and the result does not depend on what the buffer held.

The merges run in the shipped default configuration (no set_config) at
sizes where each persistent workgroup walks several tiles, so the
cross-tile window prediction, prefetch, lookahead probes and window reloads
all meet oracle-checked random data.
"""
import numpy as np
import pytest
import torch

import mp_inputs as gen

pytestmark = pytest.mark.gpu

GUARD_BYTES = 64 * 1024
FILLS = (0xA5, 0x3C)


@pytest.fixture(scope="module")
def mp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    for op in ("merge", "batched", "sort"):
        mp.set_config(op, None)
    yield mp
    mp.timing_enable(False)


class Guarded:
    """A device array of n elements with GUARD_BYTES of pattern on each side."""

    def __init__(self, n, dtype, fill):
        es = torch.empty(0, dtype=dtype).element_size()
        self.g = GUARD_BYTES // es
        self.n = n
        self.es = es
        self.buf = torch.empty(n + 2 * self.g, dtype=dtype, device="cuda")
        self.buf.view(torch.uint8).fill_(fill)
        self.fill = fill
        self.view = self.buf[self.g:self.g + n]

    def refill(self, fill):
        self.buf.view(torch.uint8).fill_(fill)
        self.fill = fill

    def guards_intact(self):
        b = self.buf.view(torch.uint8)
        head = b[: self.g * self.es]
        tail = b[(self.g + self.n) * self.es:]
        return bool((head == self.fill).all().item()) and bool((tail == self.fill).all().item())

    def host(self):
        from gpu_util import host
        return host(self.view)


def _torch_dtype(np_dtype):
    from gpu_util import NP_TO_TORCH
    return NP_TO_TORCH[np.dtype(np_dtype)]


# The built-in merge (per tile: split search on the tile diagonals, then one
# workgroup per tile) and the persistent kernel in its own default shapes
# (192 x 24; 256 x 12 for 8-byte keys with values), whose workgroups walk
# runs of tiles.
PATHS = {"per_tile": None, "persistent": (2, 192, 24, 0, 0)}


def _use(mp, path, kv8=False):
    cfg = PATHS[path]
    if cfg is not None and kv8:
        cfg = (2, 256, 12, 0, 0)
    if cfg is None:
        mp.set_config("merge", None)
    else:
        mp.set_config("merge", *cfg)


def _multi_tile_merge(mp, orc, A, B, path, min_tiles_per_group=4):
    """Merge of (A, B) into a guarded output, twice, with different fills;
    asserts everything."""
    from gpu_util import dev, first_mismatch
    want = orc.merge(A, B)
    dA, dB = dev(A), dev(B)
    out = Guarded(len(A) + len(B), _torch_dtype(A.dtype), FILLS[0])
    _use(mp, path)
    try:
        for fill in FILLS:
            out.refill(fill)
            mp.timing_enable(True)
            mp.merge(dA, dB, out=out.view)
            tiles, _ = mp.stats_query()
            groups = mp.stats_workgroups()
            mp.timing_enable(False)
            assert out.guards_intact(), "a store landed outside S"
            assert first_mismatch(out.host(), want) is None, (A.dtype, len(A), len(B), fill)
            if path == "persistent":
                assert groups > 0 and tiles >= min_tiles_per_group * groups, (tiles, groups)
    finally:
        mp.set_config("merge", None)


@pytest.mark.parametrize("path", list(PATHS))
def test_merge_u32_uniform_many_tiles(mp, orc, path):
    A, B = gen.uniform_pair(1 << 24, (1 << 24) + 4321, 101)
    _multi_tile_merge(mp, orc, A, B, path)


@pytest.mark.parametrize("path", list(PATHS))
def test_merge_u32_dups_many_tiles(mp, orc, path):
    A, B = gen.dups_pair(1 << 23, (1 << 23) - 999, 102, hi=1024)
    _multi_tile_merge(mp, orc, A, B, path, min_tiles_per_group=2)


@pytest.mark.parametrize("path", list(PATHS))
def test_merge_f32_mixture_many_tiles(mp, orc, path):
    A, B = gen.f32_mixture_pair(1 << 23, (1 << 23) + 77, 103)
    _multi_tile_merge(mp, orc, A, B, path, min_tiles_per_group=2)


@pytest.mark.parametrize("path", list(PATHS))
def test_merge_u64_many_tiles(mp, orc, path):
    A, B = gen.uniform_pair(1 << 23, (1 << 23) + 5, 104, gen.U64)
    _multi_tile_merge(mp, orc, A, B, path, min_tiles_per_group=2)


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("dt,log2n", [(gen.U32, 23), (gen.U64, 22)])
def test_merge_kv_many_tiles(mp, orc, dt, log2n, path):
    """Key-value merges, values = index in A ++ B, so stability is checked."""
    from gpu_util import dev, first_mismatch
    n = 1 << log2n
    A, B = gen.uniform_pair(n, n + 1234, 105, dt)
    va, vb = gen.index_payload(len(A), len(B))
    wk, wv = orc.merge_kv(A, va, B, vb)
    dA, dB, dva, dvb = dev(A), dev(B), dev(va), dev(vb)
    m = len(A) + len(B)
    ok = Guarded(m, _torch_dtype(A.dtype), FILLS[0])
    ov = Guarded(m, _torch_dtype(np.uint32), FILLS[0])
    _use(mp, path, kv8=dt == gen.U64)
    try:
        for fill in FILLS:
            ok.refill(fill)
            ov.refill(fill)
            mp.timing_enable(True)
            mp.merge_kv(dA, dva, dB, dvb, out_k=ok.view, out_v=ov.view)
            tiles, _ = mp.stats_query()
            groups = mp.stats_workgroups()
            mp.timing_enable(False)
            assert ok.guards_intact() and ov.guards_intact()
            assert first_mismatch(ok.host(), wk) is None
            assert first_mismatch(ov.host(), wv) is None
            if path == "persistent":
                assert groups > 0 and tiles >= 2 * groups, (tiles, groups)
    finally:
        mp.set_config("merge", None)


@pytest.mark.parametrize("shape", [(1024, 16), (1024, 8), (512, 16), (512, 12), (256, 16),
                                   (256, 15), (256, 8), (128, 16)])
def test_per_tile_shapes_guards(mp, orc, shape):
    """Every per-tile shape (mode 1) over many tiles, keys and key-value,
    4- and 8-byte keys; shapes whose LDS is not built for a key type report
    MP_ERR_UNSUPPORTED."""
    from gpu_util import dev, first_mismatch
    nt, vt = shape
    for dt in (gen.U32, gen.U64):
        A, B = gen.uniform_pair(3_000_017, 2_500_001, 106, dt)
        va, vb = gen.index_payload(len(A), len(B))
        wk, wv = orc.merge_kv(A, va, B, vb)
        dA, dB, dva, dvb = dev(A), dev(B), dev(va), dev(vb)
        m = len(A) + len(B)
        mp.set_config("merge", 1, nt, vt)
        try:
            out = Guarded(m, _torch_dtype(A.dtype), FILLS[0])
            ov = Guarded(m, _torch_dtype(np.uint32), FILLS[1])
            try:
                mp.merge(dA, dB, out=out.view)
            except mp.MergePathError as e:
                assert "UNSUPPORTED" in str(e) and dt == gen.U64 and nt * vt > 8192
                continue
            assert out.guards_intact()
            assert first_mismatch(out.host(), wk) is None, (nt, vt, dt)
            out.refill(FILLS[1])
            try:
                mp.merge_kv(dA, dva, dB, dvb, out_k=out.view, out_v=ov.view)
            except mp.MergePathError as e:
                assert "UNSUPPORTED" in str(e) and nt * vt * (A.itemsize + 4) > 64 * 1024
                continue
            assert out.guards_intact() and ov.guards_intact()
            assert first_mismatch(out.host(), wk) is None
            assert first_mismatch(ov.host(), wv) is None
        finally:
            mp.set_config("merge", None)


@pytest.mark.parametrize("dt,kv", [(gen.U32, False), (gen.F32, True), (gen.U64, True)])
def test_sort_guards(mp, orc, dt, kv):
    """Sort in place inside a guarded buffer, with a guarded workspace."""
    from gpu_util import first_mismatch
    n = (1 << 20) + 12_345
    keys = gen.unsorted_uniform(n, 107, dt)
    vals = np.arange(n, dtype=np.uint32)
    kbuf = Guarded(n, _torch_dtype(keys.dtype), FILLS[0])
    vbuf = Guarded(n, torch.uint32, FILLS[0]) if kv else None
    vt = torch.uint32 if kv else None
    ws = Guarded(mp.sort_workspace_bytes(kbuf.view.dtype, vt, n), torch.uint8, FILLS[1])
    kbuf.view.copy_(torch.from_numpy(keys))
    if kv:
        vbuf.view.copy_(torch.from_numpy(vals))
        mp.sort(kbuf.view, vbuf.view, ws=ws.view)
    else:
        mp.sort(kbuf.view, ws=ws.view)
    assert kbuf.guards_intact() and ws.guards_intact()
    if kv:
        assert vbuf.guards_intact()
        wk, wv = orc.sort(keys, vals)
        assert first_mismatch(kbuf.host(), wk) is None
        assert first_mismatch(vbuf.host(), wv) is None
    else:
        assert first_mismatch(kbuf.host(), orc.sort(keys)) is None


@pytest.mark.parametrize("path", ["built_in", "persistent"])
def test_batched_guards(mp, orc, path):
    """Batched merge (built-in batch tiles, and the persistent kernel whose
    workgroups walk several tiles) into a guarded output, two fills."""
    from gpu_util import dev, first_mismatch
    A, a_off, B, b_off = gen.batched_pairs(3000, 108, median=700.0)
    want = orc.merge_batched(A, a_off, B, b_off)
    out = Guarded(len(A) + len(B), _torch_dtype(np.int32), FILLS[0])
    dA, dB, da, db = dev(A), dev(B), dev(a_off), dev(b_off)
    if path == "persistent":
        mp.set_config("batched", 2, 256, 16)
    try:
        for fill in FILLS:
            out.refill(fill)
            mp.timing_enable(True)
            mp.merge_batched(dA, da, dB, db, out=out.view)
            tiles, _ = mp.stats_query()
            groups = mp.stats_workgroups()
            mp.timing_enable(False)
            assert out.guards_intact()
            assert first_mismatch(out.host(), want) is None, fill
            if path == "persistent":
                assert tiles >= groups > 0
    finally:
        mp.set_config("batched", None)


@pytest.mark.parametrize("op", ["intersection", "union", "difference", "symmetric_difference"])
def test_set_op_guards(mp, orc, op):
    """The output holds exactly the capacity the header asks for (|A| for
    intersection and difference, |A| + |B| otherwise)."""
    from gpu_util import dev, host
    g = np.random.default_rng(109)
    A = np.sort(g.integers(0, 1 << 21, 1_000_003)).astype(np.uint32)
    B = np.sort(g.integers(0, 1 << 21, 900_007)).astype(np.uint32)
    want = orc.set_op(op, A, B)
    cap = len(A) if op in ("intersection", "difference") else len(A) + len(B)
    out = Guarded(cap, torch.uint32, FILLS[0])
    cnt = Guarded(1, torch.int64, FILLS[1])
    got, count = mp.set_op(op, dev(A), dev(B), out=out.view, count=cnt.view, sync=False)
    k = int(host(count)[0])
    assert out.guards_intact() and cnt.guards_intact()
    assert k == len(want)
    assert out.host()[:k].tobytes() == want.tobytes()


def test_merge_split_wrong_splits_stay_inside_s(mp, orc):
    """Splits that are not the true ones (huge, negative, decreasing, random)
    give some other output, but never a store outside S."""
    from gpu_util import dev
    A, B = gen.uniform_pair(30_001, 20_011, 110)
    n = len(A) + len(B)
    k = (n + 4095) // 4096 + 1
    g = np.random.default_rng(111)
    dA, dB = dev(A), dev(B)
    for sp in (np.full(k, 1 << 62, np.int64), np.full(k, -5, np.int64),
               np.arange(k, dtype=np.int64)[::-1].copy() * 4096, g.integers(-n, 2 * n, k)):
        out = Guarded(n, torch.uint32, FILLS[0])
        mp.merge_split(dA, dB, dev(sp), 4096, out=out.view)
        assert out.guards_intact()


def test_partition_guards(mp, orc):
    from gpu_util import dev, first_mismatch
    A, B = gen.uniform_pair(500_001, 400_003, 112)
    d = np.sort(np.random.default_rng(113).integers(0, len(A) + len(B) + 1, 70_001)).astype(np.int64)
    out = Guarded(len(d), torch.int64, FILLS[0])
    mp.partition(dev(A), dev(B), dev(d), out=out.view)
    assert out.guards_intact()
    assert first_mismatch(out.host(), orc.partition(A, B, d)) is None


@pytest.mark.parametrize("op", ["intersection", "union", "difference", "symmetric_difference"])
def test_set_op_unsorted_inputs_stay_inside_s(mp, op):
    """Sortedness is a precondition: violating it gives unspecified output,
    but no store past S's room.  The first case makes non-monotone splits,
    so without the room bound the tiles of a difference would together keep
    three times |A| keys: A = [1] * T + [10] * T, B = [5] * T + [0] * T with
    T = 12288 (one 4-byte-key tile)."""
    from gpu_util import dev, host
    T = 12288
    A = np.concatenate([np.full(T, 1, np.uint32), np.full(T, 10, np.uint32)])
    B = np.concatenate([np.full(T, 5, np.uint32), np.full(T, 0, np.uint32)])
    g = np.random.default_rng(114)
    cases = [(A, B), (g.integers(0, 50, 100_003).astype(np.uint32),
                      g.integers(0, 50, 90_001).astype(np.uint32)),
             (np.sort(g.integers(0, 1000, 80_000)).astype(np.uint32)[::-1].copy(),
              np.sort(g.integers(0, 1000, 70_000)).astype(np.uint32))]
    for A_, B_ in cases:
        cap = len(A_) if op in ("intersection", "difference") else len(A_) + len(B_)
        out = Guarded(cap, torch.uint32, FILLS[0])
        cnt = Guarded(1, torch.int64, FILLS[1])
        _, count = mp.set_op(op, dev(A_), dev(B_), out=out.view, count=cnt.view, sync=False)
        k = int(host(count)[0])
        assert out.guards_intact() and cnt.guards_intact(), (op, len(A_), len(B_))
        assert 0 <= k <= cap, (k, cap)


def _batch_edge_pairs(T, seed):
    """Pair sizes that meet every edge of tiles of T outputs: empty pairs
    (runs of them), one-sided pairs, sizes just under, at and just over
    multiples of T, tiny pairs, and lognormal bulk."""
    g = np.random.default_rng(seed)
    sizes = [0, 0, 0, T, T - 1, T + 1, 2 * T, 2 * T + 3, 3 * T + 7, 1, 2, 7, 8, 9, 5 * T + 5]
    sizes += list(np.clip(np.rint(g.lognormal(np.log(0.7 * T), 0.8, 300)), 0, 8 * T).astype(int))
    sizes += [0] * 20 + [17 * T + 6]
    na, nb = [], []
    for i, s in enumerate(sizes):
        if i % 7 == 3:
            a = s          # B empty
        elif i % 7 == 5:
            a = 0          # A empty
        else:
            a = int(g.integers(0, s + 1))
        na.append(a)
        nb.append(s - a)
    na, nb = np.array(na, np.int64), np.array(nb, np.int64)
    A = np.concatenate([np.sort(g.integers(-(2**31), 2**31, k)).astype(np.int32) for k in na])
    B = np.concatenate([np.sort(g.integers(-(2**31), 2**31, k)).astype(np.int32) for k in nb])
    # a few pairs with heavy duplicates
    A[: len(A) // 50] = np.sort(A[: len(A) // 50] % 5)
    return A, gen.offsets(na), B, gen.offsets(nb)


@pytest.mark.parametrize("shape", [(256, 8), (256, 16), (512, 16), (1024, 8), (1024, 16)])
def test_batched_per_pair_tiles(mp, orc, shape):
    """Batches through batch tiles (mode 1), every tile shape, against the
    oracle, with guard canaries and two fills."""
    from gpu_util import dev, first_mismatch
    nt, vt = shape
    A, a_off, B, b_off = _batch_edge_pairs(nt * vt, 120 + nt + vt)
    # re-sort each A pair (the duplicate injection above may have broken order)
    for k in range(len(a_off) - 1):
        A[a_off[k]:a_off[k + 1]] = np.sort(A[a_off[k]:a_off[k + 1]])
    want = orc.merge_batched(A, a_off, B, b_off)
    dA, dB, da, db = dev(A), dev(B), dev(a_off), dev(b_off)
    out = Guarded(len(A) + len(B), torch.int32, FILLS[0])
    need = mp.merge_batched_workspace_bytes(torch.int32, len(a_off) - 1, len(A) + len(B))
    ws = Guarded(need, torch.uint8, FILLS[1])
    mp.set_config("batched", 1, nt, vt)
    try:
        for fill in FILLS:
            out.refill(fill)
            mp.merge_batched(dA, da, dB, db, out=out.view, ws=ws.view)
            assert out.guards_intact() and ws.guards_intact()
            assert first_mismatch(out.host(), want) is None, (shape, fill)
    finally:
        mp.set_config("batched", None)


@pytest.mark.parametrize("shape", [(256, 8), (256, 16), (1024, 16)])
@pytest.mark.parametrize("hi", [6, 40])
def test_batched_tiles_tiny_pairs(mp, orc, shape, hi):
    """Tiles over batches of short pairs (0 to 5 or 0 to 39 keys, runs of
    empty pairs, pairs of exactly one lane's outputs), so that many lanes'
    outputs cross one or more pair ends; tiles spanning fewer or more pairs
    than their LDS pair table holds; against the oracle with guards."""
    from gpu_util import dev, first_mismatch
    nt, vt = shape
    g = np.random.default_rng(130 + vt + hi)
    sizes = list(g.integers(0, hi, 20000)) + [0] * 500 + [vt] * 300 + [2 * vt + 1] * 50
    sizes += list(g.integers(0, 3, 5000)) + [nt * vt + 1, 1, 0, 0, 3]
    na = np.array([int(g.integers(0, s + 1)) for s in sizes], np.int64)
    nb = np.array(sizes, np.int64) - na
    A = np.concatenate([np.sort(g.integers(0, 8, k)).astype(np.int32) for k in na])
    B = np.concatenate([np.sort(g.integers(0, 8, k)).astype(np.int32) for k in nb])
    a_off, b_off = gen.offsets(na), gen.offsets(nb)
    want = orc.merge_batched(A, a_off, B, b_off)
    out = Guarded(len(A) + len(B), torch.int32, FILLS[0])
    need = mp.merge_batched_workspace_bytes(torch.int32, len(sizes), len(A) + len(B))
    ws = Guarded(need, torch.uint8, FILLS[1])
    mp.set_config("batched", 1, nt, vt)
    try:
        for fill in FILLS:
            out.refill(fill)
            mp.merge_batched(dev(A), dev(a_off), dev(B), dev(b_off), out=out.view, ws=ws.view)
            assert out.guards_intact() and ws.guards_intact()
            assert first_mismatch(out.host(), want) is None, (shape, fill)
    finally:
        mp.set_config("batched", None)


def test_batched_built_in_choice(mp, orc):
    """The built-in batch configuration (batch tiles) on a batch of long
    pairs and on one of short pairs; both exact."""
    from gpu_util import dev, first_mismatch
    for median in (6000.0, 40.0):
        A, a_off, B, b_off = gen.batched_pairs(2000, 121, median=median)
        want = orc.merge_batched(A, a_off, B, b_off)
        out = Guarded(len(A) + len(B), torch.int32, FILLS[0])
        mp.merge_batched(dev(A), dev(a_off), dev(B), dev(b_off), out=out.view)
        assert out.guards_intact()
        assert first_mismatch(out.host(), want) is None, median
