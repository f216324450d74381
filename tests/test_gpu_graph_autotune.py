"""hipGraph replay and the autotuner: both must leave outputs bit-identical."""
import json

import numpy as np
import pytest

import mp_inputs as gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    yield mp
    mp.graph_mode(False)
    mp.graph_clear()
    for op in ("merge", "sort", "batched"):
        mp.set_config(op, None)


def test_graph_sort_replays_match_eager(mp, orc):
    import torch
    from gpu_util import dev, host
    keys = gen.unsorted_uniform(300_001, 77)
    vals = np.arange(len(keys), dtype=np.uint32)
    want_k, want_v = orc.sort(keys, vals)
    d0k, d0v = dev(keys), dev(vals)
    k, v = torch.empty_like(d0k), torch.empty_like(d0v)
    ws = torch.empty(mp.sort_workspace_bytes(torch.uint32, torch.uint32, len(keys)),
                     dtype=torch.uint8, device="cuda")
    other_a, other_b = gen.uniform_pair(50_000, 40_000, 3)
    oa, ob = dev(other_a), dev(other_b)
    mp.graph_clear()
    mp.graph_mode(True)
    try:
        for rep in range(4):
            k.copy_(d0k)
            v.copy_(d0v)
            mp.sort(k, v, ws=ws)
            assert mp.graph_count() == 1
            assert host(k).tobytes() == want_k.tobytes(), rep
            assert host(v).tobytes() == want_v.tobytes(), rep
            # eager work and synchronisation between replays
            m = host(mp.merge(oa, ob))
            assert m.tobytes() == orc.merge(other_a, other_b).tobytes()
        # same buffers, new contents: the replay sorts the new data
        keys2 = gen.unsorted_uniform(len(keys), 78)
        k.copy_(dev(keys2))
        v.copy_(d0v)
        mp.sort(k, v, ws=ws)
        w2k, w2v = orc.sort(keys2, vals)
        assert host(k).tobytes() == w2k.tobytes() and host(v).tobytes() == w2v.tobytes()
        assert mp.graph_count() == 1
    finally:
        mp.graph_mode(False)


def test_graph_batched_replays_match_eager(mp, orc):
    import torch
    from gpu_util import dev, host
    A, a_off, B, b_off = gen.batched_pairs(500, 44, median=700)
    want = orc.merge_batched(A, a_off, B, b_off)
    dA, dB, da, db = dev(A), dev(B), dev(a_off), dev(b_off)
    out = torch.empty(len(A) + len(B), dtype=torch.int32, device="cuda")
    ws = torch.empty(mp.merge_batched_workspace_bytes(torch.int32, len(a_off) - 1, len(out)),
                     dtype=torch.uint8, device="cuda")
    mp.graph_clear()
    mp.graph_mode(True)
    try:
        for rep in range(3):
            out.fill_(0)
            mp.merge_batched(dA, da, dB, db, out=out, ws=ws)
            assert host(out).tobytes() == want.tobytes(), rep
        assert mp.graph_count() == 1
        out2 = torch.empty_like(out)          # new output pointer -> a second graph
        mp.merge_batched(dA, da, dB, db, out=out2, ws=ws)
        assert host(out2).tobytes() == want.tobytes()
        assert mp.graph_count() == 2
    finally:
        mp.graph_mode(False)


def test_autotune_merge_and_cache(mp, orc, tmp_path):
    import torch
    from gpu_util import dev, host
    from paper_1406_2628_amd import autotune
    A, B = gen.uniform_pair(400_000, 300_000, 5)
    dA, dB = dev(A), dev(B)
    out = torch.empty(len(A) + len(B), dtype=torch.uint32, device="cuda")
    cfg = autotune.tune_merge(dA, dB, out, reps=3)
    assert cfg[0] in (1, 2) and cfg[1] > 0 and mp.get_config("merge") == cfg
    got = host(mp.merge(dA, dB))
    assert got.tobytes() == orc.merge(A, B).tobytes()
    path = str(tmp_path / "tuned.json")
    autotune.save(path)
    mp.set_config("merge", None)
    assert autotune.apply(path, "merge", torch.uint32, len(A) + len(B))
    assert mp.get_config("merge") == cfg
    assert any(k.endswith("/merge/uint32/19") for k in json.load(open(path)))
    mp.set_config("merge", None)


def test_autotune_sort_and_batched(mp, orc):
    import torch
    from gpu_util import dev, host
    from paper_1406_2628_amd import autotune
    keys = gen.unsorted_uniform(200_000, 9)
    d_in = dev(keys)
    work = torch.empty_like(d_in)
    cfg = autotune.tune_sort(d_in, work, reps=2)
    assert (cfg[1] * cfg[2]) & (cfg[1] * cfg[2] - 1) == 0
    work.copy_(d_in)
    assert host(mp.sort(work)).tobytes() == orc.sort(keys).tobytes()
    A, a_off, B, b_off = gen.batched_pairs(300, 45, median=900)
    dA, dB, da, db = dev(A), dev(B), dev(a_off), dev(b_off)
    out = torch.empty(len(A) + len(B), dtype=torch.int32, device="cuda")
    autotune.tune_batched(dA, da, dB, db, out, reps=2)
    got = host(mp.merge_batched(dA, da, dB, db))
    assert got.tobytes() == orc.merge_batched(A, a_off, B, b_off).tobytes()
    mp.set_config("sort", None)
    mp.set_config("batched", None)
