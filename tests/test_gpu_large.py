"""Parity at sizes past 2^31 and 2^32 elements (64-bit index paths), checked
on the device against closed forms that hold at any size.

* Merge: A[i] = floor(i / 2) and B[j] = floor(j / 2), |A| = |B| = 3 * 2^30.
  Every value appears twice in each input, and ties take A first, so the
  merge holds each value four times: S[p] = floor(p / 4) over 3 * 2^31
  outputs, and the split on diagonal d = 4v + r is a = 2v + min(r, 2).
* Set operations: A[i] = floor(i / 2), B[j] = floor(j / 3), |A| = |B| =
  3 * 2^30: values below 2^30 appear twice in A and three times in B, the
  values from 2^30 to 1.5 * 2^30 twice in A only, which fixes every output
  (up to 2^32 keys) in closed form.
* Sort: keys k_i = (i * 0x9E3779B1) mod 2^32 for i < 2^31 + 12345 are
  distinct (multiplying by an odd constant is a bijection modulo 2^32), so
  with values v_i = i the sorted keys must increase strictly and every value
  must still map to its key.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CHUNK = 1 << 28


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    return mp


def _need(gib):
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < gib * (1 << 30):
        pytest.skip(f"needs {gib} GiB of free device memory")


def _u32_from(x64):
    """int64 tensor with values in [0, 2^32) -> uint32 tensor (same values)."""
    import torch
    return x64.to(torch.int32).view(torch.uint32)


def _half_index(n):
    """uint32 tensor t[i] = floor(i / 2), built in chunks."""
    import torch
    t = torch.empty(n, dtype=torch.uint32, device="cuda")
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        t[s:e] = _u32_from(torch.arange(s, e, dtype=torch.int64, device="cuda") >> 1)
    return t


def test_merge_and_partition_past_2p32_outputs(mp):
    import torch
    _need(56)
    na = nb = 3 << 30
    A = _half_index(na)
    B = _half_index(nb)
    S = torch.empty(na + nb, dtype=torch.uint32, device="cuda")
    mp.merge(A, B, out=S)
    torch.cuda.synchronize()
    N = na + nb
    assert N > 1 << 32
    for s in range(0, N, CHUNK):
        e = min(N, s + CHUNK)
        want = torch.arange(s, e, dtype=torch.int64, device="cuda") >> 2
        got = S[s:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(got, want), s
    del S
    g = np.random.default_rng(5)
    d = np.concatenate([[0, 1, 2, 3, N - 1, N, (1 << 31) - 1, 1 << 31, (1 << 32) - 1, 1 << 32,
                         (1 << 32) + 1], g.integers(0, N + 1, 20000)]).astype(np.int64)
    got = mp.partition(A, B, torch.from_numpy(d).cuda()).cpu().numpy()
    want = 2 * (d // 4) + np.minimum(d % 4, 2)
    assert np.array_equal(got, want)


def _third_index(n):
    """uint32 tensor t[i] = floor(i / 3), built in chunks."""
    import torch
    t = torch.empty(n, dtype=torch.uint32, device="cuda")
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        t[s:e] = _u32_from(torch.arange(s, e, dtype=torch.int64, device="cuda") // 3)
    return t


def test_set_ops_past_2p32_outputs(mp):
    import torch
    _need(56)
    na = nb = 3 << 30
    A = _half_index(na)
    B = _third_index(nb)
    H = 1 << 30
    out = torch.empty(na + nb, dtype=torch.uint32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(mp.lib().mp_set_op_workspace_bytes(na, nb), dtype=torch.uint8, device="cuda")

    def union_ref(p):
        return torch.where(p < 3 * H, p // 3, H + (p - 3 * H) // 2)

    def symdiff_ref(p):
        return torch.where(p < H, p, H + (p - H) // 2)

    expect = {"intersection": (1 << 31, lambda p: p >> 1),
              "union": (1 << 32, union_ref),
              "difference": (H, lambda p: H + (p >> 1)),
              "symmetric_difference": (1 << 31, symdiff_ref)}
    for op, (length, ref) in expect.items():
        mp.set_op(op, A, B, out=out, count=cnt, ws=ws, sync=False)
        torch.cuda.synchronize()
        assert int(cnt.item()) == length, op
        for s in range(0, length, CHUNK):
            e = min(length, s + CHUNK)
            got = out[s:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
            want = ref(torch.arange(s, e, dtype=torch.int64, device="cuda"))
            assert torch.equal(got, want), (op, s)


@pytest.mark.parametrize("m,k", [((1 << 30) + 12345, (1 << 30) + 54321),
                                 ((1 << 30) + 54321, (1 << 30) + 12345)])
def test_set_ops_runs_longer_than_2p30(mp, m, k):
    """One value repeated more than 2^30 times in each input (m copies in A,
    k in B, between other values).  Lanes deep inside the run hold ranks
    past 2^30, which the walk keeps exact in 64 bits; every output is a
    closed form of m and k (the standard library's multiset counts)."""
    import torch
    _need(40)
    i32 = torch.int32

    def seq(*parts):
        return torch.cat([torch.full((c,), v, dtype=i32, device="cuda") for v, c in parts if c > 0])

    A = seq((7, m), (11, 100))
    B = seq((5, 10), (7, k), (9, 50))
    out = torch.empty(len(A) + len(B), dtype=i32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(mp.lib().mp_set_op_workspace_bytes(len(A), len(B)), dtype=torch.uint8,
                     device="cuda")
    expect = {"intersection": [(7, min(m, k))],
              "union": [(5, 10), (7, max(m, k)), (9, 50), (11, 100)],
              "difference": [(7, max(0, m - k)), (11, 100)],
              "symmetric_difference": [(5, 10), (7, abs(m - k)), (9, 50), (11, 100)]}
    for op, parts in expect.items():
        mp.set_op(op, A, B, out=out, count=cnt, ws=ws, sync=False)
        torch.cuda.synchronize()
        length = sum(c for _, c in parts)
        assert int(cnt.item()) == length, op
        pos = 0
        for v, c in parts:
            assert bool((out[pos:pos + c] == v).all()), (op, v)
            pos += c
    del A, B, out, ws
    torch.cuda.empty_cache()


def test_sort_kv_past_2p31_keys(mp):
    import torch
    _need(40)
    n = (1 << 31) + 12345
    c = 0x9E3779B1
    keys = torch.empty(n, dtype=torch.uint32, device="cuda")
    vals = torch.empty(n, dtype=torch.uint32, device="cuda")
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        i = torch.arange(s, e, dtype=torch.int64, device="cuda")
        keys[s:e] = _u32_from((i * c) & 0xFFFFFFFF)
        vals[s:e] = _u32_from(i)
    mp.sort(keys, vals)
    torch.cuda.synchronize()
    prev = None
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        k = keys[s:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        v = vals[s:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        assert bool(torch.all(k[1:] > k[:-1])), s
        if prev is not None:
            assert int(k[0]) > prev, s
        prev = int(k[-1])
        assert torch.equal((v * c) & 0xFFFFFFFF, k), s
        assert bool(torch.all(v < n)), s
