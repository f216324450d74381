"""The allocation-free set operation (mp_set_op_noalloc) against the
workspace one (mp_set_op) through the C ABI, on two calls in a row, the
second with a smaller input (the fixed scratch keeps the first call's
contents and must be cleared by the second)."""
import ctypes

import numpy as np
import pytest

import mp_inputs as gen

pytestmark = pytest.mark.gpu

OPS = ["intersection", "union", "difference", "symmetric_difference"]


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    return mp


def _run_both(mp, op, A, B):
    import torch
    from gpu_util import dev, host
    dA, dB = dev(A), dev(B)
    cap = len(A) if op in ("intersection", "difference") else len(A) + len(B)
    out_ws = torch.empty(max(cap, 1), dtype=dA.dtype, device="cuda")
    cnt_ws = torch.empty(1, dtype=torch.int64, device="cuda")
    mp.set_op(op, dA, dB, out=out_ws, count=cnt_ws, sync=False)
    out_na = torch.empty(max(cap, 1), dtype=dA.dtype, device="cuda")
    out_na.view(torch.uint8).fill_(0x5A)
    cnt_na = torch.full((1,), -123, dtype=torch.int64, device="cuda")
    L = mp.lib()
    st = L.mp_set_op_noalloc(mp.SET_OPS[op], mp.TORCH_TO_MP[dA.dtype], ctypes.c_void_p(dA.data_ptr()),
                             len(A), ctypes.c_void_p(dB.data_ptr()), len(B),
                             ctypes.c_void_p(out_na.data_ptr()), ctypes.c_void_p(cnt_na.data_ptr()),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, mp.last_error()
    k_ws, k_na = int(host(cnt_ws)[0]), int(host(cnt_na)[0])
    assert k_na == k_ws >= 0
    assert host(out_na)[:k_na].tobytes() == host(out_ws)[:k_ws].tobytes()
    return k_na


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dt", [gen.U32, gen.U64])
def test_noalloc_matches_workspace_entry_point(mp, op, dt):
    g = np.random.default_rng(201)
    npd = gen.NP_DTYPE[dt]
    big = (np.sort(g.integers(0, 3000, 700_003)).astype(npd),
           np.sort(g.integers(0, 3000, 650_001)).astype(npd))
    small = (np.sort(g.integers(0, 50, 13_007)).astype(npd),
             np.sort(g.integers(0, 60, 9_001)).astype(npd))
    k1 = _run_both(mp, op, *big)
    k2 = _run_both(mp, op, *small)       # smaller input right after: stale scratch
    assert k1 > 0 and k2 > 0
