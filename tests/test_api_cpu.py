"""Host-side checks of the C ABI that need no GPU.

The library must load and export every entry point declared in
include/*.h, and every argument error must be reported before any device
work (fake device pointers are never dereferenced on these paths).
"""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1406_2628_amd", "libmergepath.so")

MP_NONE, MP_U32, MP_I32, MP_U64, MP_F32 = 0, 1, 2, 3, 4
OK, INVALID, UNSUPPORTED, OVERLAP, WORKSPACE = 0, -1, -2, -3, -4


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(mp_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import paper_1406_2628_amd as mp
    return mp.lib()


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ["mp_partition", "mp_merge", "mp_merge_kv", "mp_sort", "mp_merge_batched"]:
        assert required in names


def test_every_declared_symbol_is_exported(L):
    for name in declared_symbols():
        assert hasattr(L, name), name


def P(x):
    return ctypes.c_void_p(x)


def test_merge_argument_errors(L):
    a, b, s = P(0x10000), P(0x20000), P(0x30000)
    assert L.mp_merge(99, a, 10, b, 10, s, None) == UNSUPPORTED
    assert L.mp_merge(MP_U32, a, -1, b, 10, s, None) == INVALID
    assert L.mp_merge(MP_U32, None, 10, b, 10, s, None) == INVALID
    assert L.mp_merge(MP_U32, a, 10, b, 10, None, None) == INVALID
    assert L.mp_merge(MP_U32, P(0x10001), 10, b, 10, s, None) == INVALID   # misaligned
    assert L.mp_merge(MP_U32, a, 16, b, 16, P(0x10000 + 32), None) == OVERLAP
    assert L.mp_merge(MP_U32, a, 16, b, 16, P(0x20000 - 64), None) == OVERLAP
    assert b"overlap" in L.mp_last_error()
    assert L.mp_merge(MP_U32, None, 0, None, 0, None, None) == OK          # empty no-op
    assert L.mp_merge(MP_U64, a, 1 << 62, b, 1 << 62, s, None) in (INVALID, OVERLAP)


def test_set_op_argument_errors(L):
    a, b, s, c, ws = P(0x10000), P(0x20000), P(0x30000), P(0x40000), P(0x50000)
    need = L.mp_set_op_workspace_bytes(10, 10)
    assert need >= 3 * 2 * 8
    assert L.mp_set_op(4, MP_U32, a, 10, b, 10, s, c, ws, need, None) == INVALID
    assert L.mp_set_op(0, 99, a, 10, b, 10, s, c, ws, need, None) == UNSUPPORTED
    assert L.mp_set_op(0, MP_U32, a, 10, b, 10, s, None, ws, need, None) == INVALID
    assert L.mp_set_op(0, MP_U32, a, 10, b, 10, s, P(0x40004), ws, need, None) == INVALID
    assert L.mp_set_op(0, MP_U32, a, 10, b, 10, s, c, ws, need - 8, None) == WORKSPACE
    assert L.mp_set_op(0, MP_U32, a, 10, b, 10, s, c, None, need, None) == WORKSPACE
    assert L.mp_set_op(1, MP_U32, a, 10, b, 10, P(0x20000 - 40), c, ws, need, None) == OVERLAP
    assert L.mp_set_op(0, MP_U32, a, 10, b, 10, s, P(0x30000 + 8), ws, need, None) == OVERLAP
    assert L.mp_set_op(0, MP_U32, a, 10, b, 10, s, c, P(0x40000), need, None) == OVERLAP


def test_set_op_noalloc_argument_errors(L):
    a, b, s, c = P(0x10000), P(0x20000), P(0x30000), P(0x40000)
    assert L.mp_set_op_noalloc(4, MP_U32, a, 10, b, 10, s, c, None) == INVALID
    assert L.mp_set_op_noalloc(0, 0, a, 10, b, 10, s, c, None) == UNSUPPORTED
    assert L.mp_set_op_noalloc(0, MP_U32, a, 10, b, 10, s, None, None) == INVALID
    assert L.mp_set_op_noalloc(0, MP_U32, a, 10, b, 10, P(0x10000 + 4), c, None) == OVERLAP
    # inputs beyond the fixed scratch are refused before any device access
    big = 1 << 30
    assert L.mp_set_op_noalloc(1, MP_U32, P(0x10000), big, P(0x10000 + 8 * big), big,
                               P(0x10000 + 16 * big), c, None) == UNSUPPORTED
    assert b"scratch" in L.mp_last_error()


def test_join_argument_errors(L):
    a, b, i, j, c, w = P(0x10000), P(0x20000), P(0x30000), P(0x40000), P(0x50000), P(0x60000)
    need = L.mp_join_workspace_bytes(10, 10)
    assert need > 0
    assert L.mp_join(0, a, 10, b, 10, i, j, 5, c, w, need, None) == UNSUPPORTED
    assert L.mp_join(MP_U32, a, 10, b, 10, i, j, -1, c, w, need, None) == INVALID
    assert L.mp_join(MP_U32, a, 10, b, 10, i, j, 5, None, w, need, None) == INVALID
    assert L.mp_join(MP_U32, a, 10, b, 10, None, j, 5, c, w, need, None) == INVALID
    assert L.mp_join(MP_U32, a, 10, b, 10, i, j, 5, c, None, 0, None) == WORKSPACE
    assert L.mp_join(MP_U32, a, 10, b, 10, i, j, 5, c, w, need - 8, None) == WORKSPACE
    assert L.mp_join(MP_U32, a, 10, b, 10, i, j, 5, c, P(0x60004), need, None) == INVALID
    assert L.mp_join(MP_U32, a, 10, b, 10, P(0x10000 + 8), j, 5, c, w, need, None) == OVERLAP
    assert L.mp_join(MP_U32, a, 10, b, 10, i, P(0x30000 + 16), 5, c, w, need, None) == OVERLAP


def test_merge_split_argument_errors(L):
    a, b, sp, s = P(0x10000), P(0x20000), P(0x30000), P(0x40000)
    assert L.mp_merge_split(MP_U32, a, 10, b, 10, sp, 1000, s, None) == UNSUPPORTED
    assert L.mp_merge_split(99, a, 10, b, 10, sp, 4096, s, None) == UNSUPPORTED
    assert L.mp_merge_split(MP_U32, a, 10, b, 10, None, 4096, s, None) == INVALID
    assert L.mp_merge_split(MP_U32, a, 10, b, 10, P(0x30004), 4096, s, None) == INVALID
    assert L.mp_merge_split(MP_U32, a, 10, b, 10, sp, 4096, None, None) == INVALID
    assert L.mp_merge_split(MP_U32, a, 10, b, 10, sp, 4096, P(0x30000 - 16), None) == OVERLAP
    assert L.mp_merge_split(MP_U32, a, 10, b, 10, sp, 4096, P(0x10000 + 4), None) == OVERLAP
    assert L.mp_merge_split(MP_U32, None, 0, None, 0, None, 4096, None, None) == OK


def test_merge_checksum_argument_errors(L):
    a, b, c = P(0x10000), P(0x20000), P(0x30000)
    assert L.mp_merge_checksum(99, a, 10, b, 10, c, None) == UNSUPPORTED
    assert L.mp_merge_checksum(MP_U32, a, 10, b, 10, None, None) == INVALID
    assert L.mp_merge_checksum(MP_U32, a, 10, b, 10, P(0x30004), None) == INVALID   # misaligned
    assert L.mp_merge_checksum(MP_U32, a, 16, b, 16, P(0x10000 + 8), None) == OVERLAP
    assert L.mp_merge_checksum(MP_U32, a, -1, b, 10, c, None) == INVALID
    assert L.mp_merge_checksum(MP_U32, None, 0, None, 0, c, None) == OK          # empty no-op


def test_merge_kv_argument_errors(L):
    ak, av, bk, bv, sk, sv = (P(x) for x in (0x10000, 0x20000, 0x30000, 0x40000, 0x50000, 0x60000))
    assert L.mp_merge_kv(MP_U32, MP_NONE, ak, av, 4, bk, bv, 4, sk, sv, None) == INVALID
    assert L.mp_merge_kv(MP_U32, MP_U64, ak, av, 4, bk, bv, 4, sk, sv, None) == UNSUPPORTED
    assert L.mp_merge_kv(MP_U32, MP_U32, ak, None, 4, bk, bv, 4, sk, sv, None) == INVALID
    assert L.mp_merge_kv(MP_U32, MP_U32, ak, av, 4, bk, bv, 4, sk, P(0x50000 + 16), None) == OVERLAP
    assert L.mp_merge_kv(MP_U32, MP_U32, ak, av, 4, bk, bv, 4, sk, P(0x20000), None) == OVERLAP


def test_learned_argument_errors(L):
    h = ctypes.c_void_p()
    assert L.mp_lp_create(ctypes.byref(h), 0, 5, 1) == INVALID
    assert L.mp_lp_create(ctypes.byref(h), 65, 5, 1) == INVALID
    assert L.mp_lp_create(ctypes.byref(h), 32, 2, 1) == INVALID
    assert L.mp_lp_create(None, 32, 5, 1) == INVALID
    assert L.mp_lp_set_window(None, 5) == INVALID
    assert L.mp_lp_window(None) == -1
    assert L.mp_partition_learned(None, MP_F32, None, 0, None, 0, None, 0, None, None, None) == INVALID
    assert L.mp_lp_load(ctypes.byref(h), b"/nonexistent/model") == INVALID


def test_sort_and_batched_argument_errors(L):
    k, ws = P(0x10000), P(0x80000)
    assert L.mp_sort(MP_U32, MP_NONE, k, None, 100_000, None, 0, None) == WORKSPACE
    need = L.mp_sort_workspace_bytes(MP_U32, MP_U32, 1000)
    assert need >= 1000 * 8
    for kt in (MP_U32, MP_I32, MP_U64, MP_F32):
        for vt in (MP_NONE, MP_U32, MP_I32, MP_F32):
            blk = L.mp_sort_block_keys(kt, vt)
            assert blk >= 4096 and blk & (blk - 1) == 0, (kt, vt)
    assert L.mp_sort_block_keys(99, MP_NONE) == 0
    assert L.mp_sort_block_keys(MP_U32, MP_U64) == 0
    assert L.mp_sort(MP_U32, MP_U32, k, None, 1000, ws, need, None) == INVALID
    assert L.mp_sort(MP_U32, MP_NONE, k, P(0x20000), 1000, ws, need, None) == INVALID
    assert L.mp_sort(MP_U32, MP_NONE, k, None, 1000, P(0x10000 + 64), need, None) == OVERLAP
    assert L.mp_sort(MP_U32, MP_U64, k, P(0x20000), 1000, ws, need, None) == UNSUPPORTED
    assert L.mp_sort(MP_U32, MP_NONE, k, None, 1, None, 0, None) == OK
    a, ao, b, bo, s = (P(x) for x in (0x10000, 0x20000, 0x30000, 0x40000, 0x50000))
    assert L.mp_merge_batched(MP_I32, a, ao, b, bo, -1, 0, 0, s, None, 0, None) == INVALID
    assert L.mp_merge_batched(MP_I32, a, ao, b, bo, 0, 5, 0, s, None, 0, None) == INVALID
    assert L.mp_merge_batched(MP_I32, a, None, b, bo, 3, 5, 5, s, None, 0, None) == INVALID
    assert L.mp_merge_batched(MP_I32, a, ao, b, bo, 3, 5, 5, P(0x10000 + 8), None, 0, None) == OVERLAP
    assert L.mp_merge_batched(MP_I32, None, None, None, None, 0, 0, 0, None, None, 0, None) == OK
    # batch tiles need the workspace
    a2, b2, s2, w2 = P(0x100000), P(0x200000), P(0x300000), P(0x400000)
    need = L.mp_merge_batched_workspace_bytes(MP_I32, 1, 4000)
    assert need > 0
    assert L.mp_merge_batched(MP_I32, a2, ao, b2, bo, 1, 2000, 2000, s2, None, 0, None) == WORKSPACE
    assert L.mp_merge_batched(MP_I32, a2, ao, b2, bo, 1, 2000, 2000, s2, w2, need - 8, None) == WORKSPACE
    assert L.mp_merge_batched(MP_I32, a2, ao, b2, bo, 1, 2000, 2000, s2, P(0x400004), need, None) == INVALID
    assert L.mp_merge_batched(MP_I32, a2, ao, b2, bo, 1, 2000, 2000, s2, P(0x300000 + 64), need,
                              None) == OVERLAP


def test_config_errors(L):
    import paper_1406_2628_amd as mp
    with pytest.raises(mp.MergePathError):
        mp.set_config("nonsense", 2)
    with pytest.raises(mp.MergePathError):
        mp.set_config("merge", 3)
    with pytest.raises(mp.MergePathError):
        mp.set_config("batched", 1, 128, 8)   # per-tile batches need tiles of >= 2048 keys
    mp.set_config("batched", 1, 256, 8)
    mp.set_config("batched", None)
    with pytest.raises(mp.MergePathError):
        mp.set_config("sort", 2, 256, 12)
    with pytest.raises(mp.MergePathError):
        mp.set_config("sort", 1, 512, 12)     # per-tile sort tiles are powers of two
    with pytest.raises(mp.MergePathError):
        mp.set_config("merge", 2, 0, 0)       # only per-tile mode picks its own tile
    mp.set_config("merge", 1, 0, 0)           # per-tile, tile picked per call
    assert mp.get_config("merge")[:3] == (1, 0, 0)
    mp.set_config("merge", None)
    mp.set_config("sort", None)
    assert mp.get_config("merge")[0] == 1 and mp.get_config("sort")[0] == 1
    assert mp.get_config("batched")[:3] == (1, 0, 0)


def test_partition_lanes_argument_errors(L):
    for bad in (-1, 3, 65, 128):
        assert L.mp_partition_lanes(bad) == INVALID
    for ok in (1, 2, 4, 8, 16, 32, 64, 0):
        assert L.mp_partition_lanes(ok) == OK


def test_partition_argument_errors(L):
    a, b, d, o = P(0x10000), P(0x20000), P(0x30000), P(0x40000)
    assert L.mp_partition(0, a, 4, b, 4, d, 4, o, None) == UNSUPPORTED
    assert L.mp_partition(MP_F32, a, 4, b, 4, d, -3, o, None) == INVALID
    assert L.mp_partition(MP_F32, a, 4, b, 4, d, 4, None, None) == INVALID
    assert L.mp_partition(MP_F32, a, 4, b, 4, d, 4, P(0x30000 + 8), None) == OVERLAP
    assert L.mp_partition(MP_F32, a, 4, b, 4, d, 0, o, None) == OK


def test_bw_probe_argument_errors(L):
    s, d = P(0x10000), P(0x20000)
    assert L.mp_bw_probe(3, s, d, 1024, 0, 0, None) == INVALID
    assert L.mp_bw_probe(0, s, d, 1000, 0, 0, None) == INVALID        # not a multiple of 16
    assert L.mp_bw_probe(0, s, d, 1024, 0, -1, None) == INVALID
    assert L.mp_bw_probe(0, None, d, 1024, 0, 0, None) == INVALID
    assert L.mp_bw_probe(1, P(0x10008), d, 1024, 0, 8, None) == INVALID  # misaligned
    assert L.mp_bw_probe(0, s, P(0x10000 + 512), 1024, 0, 0, None) == OVERLAP
    assert L.mp_bw_probe(1, s, P(0x10000 + 512), 1024, 0, 8, None) == OVERLAP  # sink inside src
    assert L.mp_bw_probe(0, s, d, 1024, 3, 8, None) in (UNSUPPORTED, -5)  # unroll 3 not built
    assert L.mp_bw_probe(2, None, d, 0, 0, 0, None) == OK
