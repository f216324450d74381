"""Merge Path benchmark on one MI355X.

Headline: merge of two sorted uint32 arrays, |A| = |B| = 2^28, keys uniform
in [0, 2^32) (seed 11), inputs resident in HBM, output preallocated.  One
step = one mp_merge call (Algorithm 1: the split search on every tile
diagonal, then one workgroup per 16384-key tile: LDS windows, per-lane split
search, serial merge, coalesced stores).

Prints ONE JSON line: throughput (Gkeys/s merged), the roofline of the merge
kernel timed with HIP events that the library records on its launch stream,
the single-core oracle baseline timed on the host, the same merge kept in
registers (nothing stored), and under "extras" the other workloads: a small
cache-resident merge (hot and cold), key-value merges, merge sort, batched
merge, the learned split predictor against the plain split search, the
multiset operations and the inner join.  Every output is checked
(bit-exact against the oracle, or for the 2^28 sort against numpy's sort,
which the oracle's own tests pin).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs a,b,...]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gkeys/s merged & % HBM peak (2^28+2^28 u32); learned vs bsearch split time"
LEGS = ("headline", "small", "kv", "sort", "batched", "learned", "setops", "join")
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "merge_tile_u32_2p28.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1406_2628_amd", "csrc", f)
                  for f in ("mp_tile_impl.h", "mp_device.h")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sync():
    import torch
    torch.cuda.synchronize()


def time_steps(fn, steps, warmup):
    """Mean ms per call over `steps` back-to-back calls after `warmup` calls."""
    import torch
    for _ in range(warmup):
        fn()
    sync()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    sync()
    return start.elapsed_time(stop) / steps


def event_times(fn, steps, warmup):
    """Per-call times (ms) of `steps` calls after `warmup` calls, each call
    bracketed by its own pair of events on the current stream: mean, median
    and min."""
    import numpy as np
    import torch
    for _ in range(warmup):
        fn()
    sync()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for s, e in evs:
        s.record()
        fn()
        e.record()
    sync()
    ts = np.array([s.elapsed_time(e) for s, e in evs])
    return {"mean": float(ts.mean()), "median": float(np.median(ts)), "min": float(ts.min())}


def time_each(fn, setup, reps, warmup=1):
    """Median ms of fn() over reps, each preceded by an untimed setup()."""
    import numpy as np
    import torch
    ts = []
    for r in range(warmup + reps):
        setup()
        sync()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        sync()
        if r >= warmup:
            ts.append(s.elapsed_time(e))
    return float(np.median(ts))


def dev(x):
    import torch
    return torch.from_numpy(x).cuda()


def source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def profiled_traffic():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    try:
        fields = {}
        for line in open(PROFILE_SUMMARY):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
        if fields.get("kernel source sha256") != source_sha():
            return None
        return float(fields["HBM bytes per launch"])
    except (OSError, KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
def leg_headline(args, out):
    import numpy as np
    import torch

    import mp_inputs as gen
    import paper_1406_2628_amd as mp
    na = nb = 1 << args.log2n
    seed = 11
    log(f"bench: headline: generating u32 inputs 2^{args.log2n}+2^{args.log2n} (seed {seed})")
    A, B = gen.uniform_pair(na, nb, seed)
    dA, dB = dev(A), dev(B)
    dS = torch.empty(na + nb, dtype=torch.uint32, device="cuda")
    n_out = na + nb
    alg_bytes = n_out * 4 * 2  # each input key read once, each output key written once

    if args.copy_probe:
        del dA, dB
        src = torch.empty(n_out * 4, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        ms = time_steps(lambda: mp.copy(src, dst), args.steps, args.warmup)
        print(json.dumps({"probe": "copy", "bytes_moved": 2 * src.numel(), "ms": round(ms, 4),
                          "GBs": round(2 * src.numel() / ms / 1e6, 1)}), flush=True)
        sys.exit(0)

    log("bench: headline: timing mp_merge")
    step = lambda: mp.merge(dA, dB, out=dS)  # noqa: E731
    mp.timing_enable(False)
    ms = time_steps(step, args.steps, args.warmup)
    # the same steps one by one, each between its own pair of events
    per = event_times(step, max(20, args.steps), 0)
    # kernel durations over a second timed region: HIP events the library
    # records on the launch stream around each kernel (split search on the
    # tile diagonals, then the tile merge)
    mp.timing_enable(True)
    time_steps(step, args.steps, 0)
    k_ms, k_n = mp.timing_query("tile_merge")
    s_ms, s_n = mp.timing_query("tile_splits")
    mp.timing_enable(False)
    kern_ms = k_ms / max(1, k_n)
    splits_ms = s_ms / max(1, s_n)
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = profiled_traffic()
    # the split search alone on the same diagonals (Algorithm 2 only)
    T = 1 << 14
    tdiag = torch.clamp(torch.arange(n_out // T + 2, device="cuda", dtype=torch.int64) * T,
                        max=n_out)
    sp = torch.empty_like(tdiag)
    part_ms = event_times(lambda: mp.partition(dA, dB, tdiag, out=sp), 20, 3)["median"]
    del tdiag, sp
    # measured copy of the same bytes (2^29 keys read, 2^29 written) with the
    # bandwidth probe's best measured launch shape
    log("bench: headline: copy reference")
    cpy_src = torch.ones(n_out, dtype=torch.int32, device="cuda")
    cpy_dst = torch.empty_like(cpy_src)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    cpy = event_times(lambda: mp.bw_probe("copy", cpy_src, cpy_dst, n_out * 4, 4, 64 * cus),
                      20, 3)
    del cpy_src, cpy_dst
    copy_gbs = alg_bytes / (cpy["median"] * 1e-3) / 1e9
    step_gbs = alg_bytes / (ms * 1e-3) / 1e9

    out.update({
        "metric": METRIC,
        "value": round(n_out / (ms * 1e-3) / 1e9, 2),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded uniform u32 keys, sorted)",
        "config": {"workload": f"merge of sorted u32 arrays, 2^{args.log2n}+2^{args.log2n} "
                               f"uniform keys, seed {seed}", "na": na, "nb": nb},
        "step_ms": {"median": round(per["median"], 4), "min": round(per["min"], 4),
                    "mean": round(per["mean"], 4), "steps": max(20, args.steps)},
        "hbm_frac_step": round(step_gbs / HBM_PEAK_GBS, 4),
        "copy_reference": {"GBs_median": round(copy_gbs, 1),
                           "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
                           "step_frac_of_copy": round(step_gbs / copy_gbs, 4),
                           "kernel_frac_of_copy": round(achieved / copy_gbs, 4)},
        "partition_alone_ms": round(part_ms, 4),
        "roofline": {"bound": "hbm", "kernel": "merge_tile_kernel (1024 x 16, single pair)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / 1e9, 4),
                     "traffic_unit": "GB per launch", "algorithmic_GB": round(alg_bytes / 1e9, 4),
                     "kernel_ms": round(kern_ms, 4), "splits_kernel_ms": round(splits_ms, 4)},
    })
    # The same merge kept in registers (nothing stored; section 6's runs
    # that write to a local register): reading and comparing alone.
    log("bench: headline: timing the no-store merge (mp_merge_checksum)")
    ck = torch.zeros(1, dtype=torch.uint64, device="cuda")
    nw_ms = time_steps(lambda: mp.merge_checksum(dA, dB, out=ck), args.steps, args.warmup)
    ck.zero_()
    mp.merge_checksum(dA, dB, out=ck)
    ck_got = int(ck.cpu().numpy()[0])
    S = dS.cpu().numpy()
    del dA, dB, dS
    if args.no_cpu_baseline:
        import oracle
        ref = oracle.merge(A, B)
    else:
        log("bench: headline: oracle merge on the host (cpu baseline and verification)")
        import oracle
        times = []
        t_all = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            ref = oracle.merge(A, B)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_all > 10.0 or len(times) >= 8:
                break
        times.sort()
        out["cpu_baseline"] = {
            "value": round(n_out / times[len(times) // 2] / 1e9, 4), "unit": "Gkeys/s", "cores": 1,
            "kind": "oracle",
            "sample": f"the full headline workload, median of {len(times)} single-threaded runs "
                      f"(1 of {os.cpu_count()} host threads)"}
    out["bit_exact"] = bool(S.tobytes() == ref.tobytes())
    with np.errstate(over="ignore"):
        ck_want = int(np.sum(ref.astype(np.uint64) * np.arange(1, n_out + 1, dtype=np.uint64),
                             dtype=np.uint64))
    out["no_write"] = {"ms": round(nw_ms, 4), "Gkeys_s": round(n_out / (nw_ms * 1e-3) / 1e9, 2),
                       "read_GBs": round(n_out * 4 / (nw_ms * 1e-3) / 1e9, 1),
                       "read_frac": round(n_out * 4 / (nw_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "store_over_no_store": round(ms / nw_ms, 3),
                       "checksum_matches_oracle": ck_got == ck_want}


def bw_sweep(args):
    """Bandwidth references (mp_bw_probe): copy, read-only and write-only
    passes moving 4.3 GB and 8.6 GB in total, over a sweep of loads or stores
    in flight per lane and workgroups per compute unit.  One JSON line per
    point: median and min of event-timed launches."""
    import torch

    import paper_1406_2628_amd as mp
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for moved in (1 << 32, 1 << 33):
        for kind in ("copy", "read", "write"):
            n = moved // 2 if kind == "copy" else moved
            src = None if kind == "write" else torch.ones(n // 4, dtype=torch.int32, device="cuda")
            for per_cu in (4, 8, 16, 32, 64):
                grid = per_cu * cus
                dst = (torch.empty(grid * 64, dtype=torch.int32, device="cuda") if kind == "read"
                       else torch.empty(n // 4, dtype=torch.int32, device="cuda"))
                for unroll in (1, 2, 4, 8, 16):
                    ts = event_times(lambda: mp.bw_probe(kind, src, dst, n, unroll, grid),
                                     args.steps, args.warmup)
                    print(json.dumps({"probe": kind, "bytes_moved": moved, "per_cu": per_cu,
                                      "grid": grid, "unroll": unroll,
                                      "median_ms": round(ts["median"], 4),
                                      "min_ms": round(ts["min"], 4),
                                      "GBs_median": round(moved / ts["median"] / 1e6, 1),
                                      "GBs_best": round(moved / ts["min"] / 1e6, 1)}), flush=True)
                del dst
            del src
            torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
def leg_small(args, ex):
    """2^20 + 2^20 u32 keys (seed 1): 16 MiB of traffic, which the 256 MB
    last-level cache holds, so the HBM fraction means nothing here.  Hot: the
    same merge repeated; cold: a 512 MiB buffer written between calls."""
    import torch

    import mp_inputs as gen
    import oracle
    import paper_1406_2628_amd as mp
    n = 1 << 20
    log("bench: small 2^20+2^20 u32")
    A, B = gen.uniform_pair(n, n, 1)
    dA, dB = dev(A), dev(B)
    dS = torch.empty(2 * n, dtype=torch.uint32, device="cuda")
    hot = time_each(lambda: mp.merge(dA, dB, out=dS), lambda: None, 50, 5)
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    cold = time_each(lambda: mp.merge(dA, dB, out=dS), lambda: flush.fill_(1), 20, 2)
    ok = bool(dS.cpu().numpy().tobytes() == oracle.merge(A, B).tobytes())
    ex["small"] = {"n": 2 * n, "hot_us": round(hot * 1e3, 2), "cold_us": round(cold * 1e3, 2),
                   "hot_Gkeys_s": round(2 * n / hot / 1e6, 1),
                   "cold_Gkeys_s": round(2 * n / cold / 1e6, 1), "bit_exact": ok}


# ---------------------------------------------------------------------------
def leg_setops(args, ex):
    """Multiset operations on 2^28 + 2^28 sorted u32 keys drawn from [0, 2^29)
    (about 40% of A's keys find a partner in B), seed 91."""
    import numpy as np
    import torch

    import oracle
    import paper_1406_2628_amd as mp
    n = 1 << args.log2n
    log(f"bench: set operations 2^{args.log2n}+2^{args.log2n} u32")
    g = np.random.default_rng(91)
    A = np.sort(g.integers(0, 2 * n, n, dtype=np.uint32))
    B = np.sort(g.integers(0, 2 * n, n, dtype=np.uint32))
    dA, dB = dev(A), dev(B)
    out = torch.empty(2 * n, dtype=torch.uint32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(mp.lib().mp_set_op_workspace_bytes(n, n), dtype=torch.uint8, device="cuda")
    res = {"n_per_input": n}
    for op in ("intersection", "union", "difference", "symmetric_difference"):
        ms = time_steps(lambda: mp.set_op(op, dA, dB, out=out, count=cnt, ws=ws, sync=False),
                        max(3, args.steps // 2), 2)
        k = int(cnt.item())
        got = out[:k].cpu().numpy()
        want = oracle.set_op(op, A, B)
        # fewest bytes: each input key read once, each kept key written once
        bytes_ = (2 * n + k) * 4
        res[op] = {"ms": round(ms, 4), "out": k, "Gkeys_in_s": round(2 * n / ms / 1e6, 1),
                   "hbm_frac_min_bytes": round(bytes_ / ms / 1e6 / HBM_PEAK_GBS, 4),
                   "bit_exact": bool(got.tobytes() == want.tobytes())}
    ex["setops"] = res


# ---------------------------------------------------------------------------
def leg_join(args, ex):
    """Inner join of 2^26 + 2^26 sorted u32 keys drawn from [0, 2^27) (seed
    93): every equal-key pair (i, j).  The count is checked against the
    closed form sum over values of (copies in A) x (copies in B), and 2^20
    sampled pairs for equal keys and (i, j) order."""
    import numpy as np
    import torch

    import paper_1406_2628_amd as mp
    n = 1 << (args.log2n - 2)
    log(f"bench: join 2^{n.bit_length() - 1}+2^{n.bit_length() - 1} u32")
    g = np.random.default_rng(93)
    A = np.sort(g.integers(0, 2 * n, n, dtype=np.uint32))
    B = np.sort(g.integers(0, 2 * n, n, dtype=np.uint32))
    dA, dB = dev(A), dev(B)
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(mp.lib().mp_join_workspace_bytes(n, n), dtype=torch.uint8, device="cuda")
    mp.join(dA, dB, cap=0, count=cnt, ws=ws, sync=False)
    k = int(cnt.item())
    I = torch.empty(max(k, 1), dtype=torch.int64, device="cuda")
    J = torch.empty_like(I)
    ms = time_steps(lambda: mp.join(dA, dB, cap=k, I=I, J=J, count=cnt, ws=ws, sync=False),
                    max(3, args.steps // 2), 2)
    lo, hi = np.searchsorted(B, A, "left"), np.searchsorted(B, A, "right")
    want = int(np.sum(hi - lo))
    idx = np.sort(np.random.default_rng(0).integers(0, max(k, 1), 1 << 20))
    hi_, hj = I.cpu().numpy()[idx], J.cpu().numpy()[idx]
    ordered = bool(np.all((np.diff(hi_) > 0) | ((np.diff(hi_) == 0) & (np.diff(hj) >= 0))))
    # fewest bytes: both inputs once, each pair (two int64) once
    bytes_ = 2 * n * 4 + k * 16
    ex["join"] = {"n_per_input": n, "pairs": k, "ms": round(ms, 4),
                  "Gpairs_s": round(k / ms / 1e6, 2),
                  "hbm_frac_min_bytes": round(bytes_ / ms / 1e6 / HBM_PEAK_GBS, 4),
                  "count_matches_closed_form": k == want,
                  "sampled_pairs_equal_and_ordered": bool(np.all(A[hi_] == B[hj])) and ordered}


# ---------------------------------------------------------------------------
def leg_kv(args, ex):
    import torch

    import mp_inputs as gen
    import oracle
    import paper_1406_2628_amd as mp
    res = {}
    n = 1 << args.log2n
    cases = [("u32_uniform", 21, n), ("u32_dups_1024", 22, n), ("u32_disjoint", 23, n),
             ("u64_uniform", 24, n // 2)]
    for name, seed, m in cases:
        log(f"bench: kv {name} 2^{m.bit_length() - 1}+2^{m.bit_length() - 1}")
        if name == "u32_dups_1024":
            A, B = gen.dups_pair(m, m, seed)
        elif name == "u32_disjoint":
            A, B = gen.disjoint_pair(m, m, seed)
        else:
            A, B = gen.uniform_pair(m, m, seed, gen.U64 if name.startswith("u64") else gen.U32)
        va, vb = gen.index_payload(m, m)
        dA, dB, dva, dvb = dev(A), dev(B), dev(va), dev(vb)
        ok_ = torch.empty(2 * m, dtype=dA.dtype, device="cuda")
        ov = torch.empty(2 * m, dtype=torch.uint32, device="cuda")
        ms = time_steps(lambda: mp.merge_kv(dA, dva, dB, dvb, out_k=ok_, out_v=ov),
                        max(3, args.steps // 2), 2)
        gk, gv = ok_.cpu().numpy(), ov.cpu().numpy()
        del dA, dB, dva, dvb, ok_, ov
        wk, wv = oracle.merge_kv(A, va, B, vb)
        bytes_ = 2 * m * (A.itemsize + 4) * 2
        res[name] = {"n": 2 * m, "ms": round(ms, 4), "Gkeys_s": round(2 * m / ms / 1e6, 2),
                     "hbm_frac": round(bytes_ / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "bit_exact": bool(gk.tobytes() == wk.tobytes() and gv.tobytes() == wv.tobytes())}
    ex["kv"] = res


def leg_sort(args, ex):
    import numpy as np
    import torch

    import mp_inputs as gen
    import paper_1406_2628_amd as mp
    n = 1 << args.log2n
    res = {}
    for name, seed in (("u32_uniform", 31), ("u32_zipf_1.1", 32)):
        log(f"bench: sort {name} 2^{args.log2n}")
        keys = gen.unsorted_uniform(n, seed) if "uniform" in name else gen.zipf_keys(n, seed)
        d0 = dev(keys)
        dk = torch.empty_like(d0)
        ws = torch.empty(mp.sort_workspace_bytes(torch.uint32, None, n), dtype=torch.uint8,
                         device="cuda")
        # per-round kernel times (eager launches after one untimed sort,
        # events around each kernel, summed over 3 sorts)
        dk.copy_(d0)
        mp.sort(dk, ws=ws)
        sync()
        mp.timing_enable(True)
        time_each(lambda: mp.sort(dk, ws=ws), lambda: dk.copy_(d0), 3, warmup=0)
        bs, rd = mp.timing_query("blocksort"), mp.timing_query("sort_round")
        mp.timing_enable(False)
        # the timed sort: autotuned round variant, the whole sequence as one hipGraph
        from paper_1406_2628_amd import autotune
        tuned = autotune.tune_sort(d0, dk, reps=2, ws=ws)
        mp.graph_mode(True)
        ms = time_each(lambda: mp.sort(dk, ws=ws), lambda: dk.copy_(d0), max(3, args.steps // 4))
        mp.graph_mode(False)
        mp.graph_clear()
        mp.set_config("sort", None)
        got = dk.cpu().numpy()
        del d0, dk, ws
        block = mp.sort_block_keys(torch.uint32)
        rounds = int(np.ceil(np.log2(max(1, n / block))))
        bytes_ = (1 + rounds) * n * 8
        # the same sort counted as the 2048-key-block layout does it (one
        # block pass, then a round per doubling from 2048 keys)
        passes_2048 = 1 + int(np.ceil(np.log2(max(1, n / 2048))))
        res[name] = {"n": n, "ms": round(ms, 4), "Gkeys_s": round(n / ms / 1e6, 3),
                     "passes": 1 + rounds, "block_keys": block,
                     "hbm_frac": round(bytes_ / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "passes_with_2048_key_blocks": passes_2048,
                     "hbm_frac_counting_2048_key_block_passes":
                         round(passes_2048 * n * 8 / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "blocksort_ms": round(bs[0] / max(1, bs[1]), 4),
                     "round_ms": round(rd[0] / max(1, rd[1]), 4),
                     "autotuned_config": {"nt": tuned[1], "vt": tuned[2]}, "hip_graph": True,
                     "equals_numpy_sort": bool(np.array_equal(got, np.sort(keys)))}
    ex["sort"] = res


def leg_batched(args, ex):
    import torch

    import mp_inputs as gen
    import oracle
    import paper_1406_2628_amd as mp
    n_pairs = 100_000 if args.log2n == 28 else max(10, 100_000 >> (28 - args.log2n))
    log(f"bench: batched {n_pairs} pairs")
    A, a_off, B, b_off = gen.batched_pairs(n_pairs, 41)
    tot = len(A) + len(B)
    dA, dB, da, db = dev(A), dev(B), dev(a_off), dev(b_off)
    dS = torch.empty(tot, dtype=torch.int32, device="cuda")
    # variant chosen by the autotuner on this workload, launch replayed from a hipGraph
    from paper_1406_2628_amd import autotune
    tuned = autotune.tune_batched(dA, da, dB, db, dS, reps=3)
    mp.graph_mode(True)
    mp.timing_enable(True)
    ms = time_steps(lambda: mp.merge_batched(dA, da, dB, db, out=dS), args.steps, 10)
    tiles, reloads = mp.stats_query()
    mp.timing_enable(False)
    mp.graph_mode(False)
    mp.graph_clear()
    mp.set_config("batched", None)
    got = dS.cpu().numpy()
    del dA, dB, da, db, dS
    ref = oracle.merge_batched(A, a_off, B, b_off)
    ex["batched"] = {"pairs": n_pairs, "n": tot, "ms": round(ms, 4),
                     "Gkeys_s": round(tot / ms / 1e6, 2),
                     "hbm_frac": round(tot * 8 / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "autotuned_config": {"nt": tuned[1], "vt": tuned[2]}, "hip_graph": True,
                     "window_reload_rate": round(reloads / max(1, tiles), 6),
                     "bit_exact": bool(got.tobytes() == ref.tobytes())}


def leg_learned(args, ex):
    import numpy as np
    import torch

    import mp_inputs as gen
    import oracle
    import paper_1406_2628_amd as mp
    n = 1 << (args.log2n + 1)          # |A| = |B| = 2^29 at the default size
    n_train = max(1 << 16, n >> 7)     # training sets of the same family, smaller
    res = {"n_per_array": n, "train_n_per_array": n_train}
    log(f"bench: learned: training on 8 seeds of 2^{n_train.bit_length() - 1}")
    sets = [gen.f32_mixture_pair_torch(n_train, n_train, s) for s in range(51, 59)]
    lp = mp.LearnedPartitioner(32, 5, 7)
    sync()
    t0 = time.perf_counter()
    loss = lp.train(sets, k_diag=1 << 14, epochs=4000, lr=1e-2)
    res["train_s"] = round(time.perf_counter() - t0, 3)
    res["train_loss"] = loss
    del sets
    log("bench: learned: calibrating on a held-out full-size pair (seed 59)")
    A, B = gen.f32_mixture_pair_torch(n, n, 59)
    res["max_val_err"] = lp.calibrate(A, B, 1 << 20)
    w = lp.windows()
    span = (w[:, 1] - w[:, 0]) if len(w) else np.array([2 * lp.window])
    res["window_buckets"] = int(len(w))
    res["window_span_median"] = int(np.median(span))
    res["window_span_max"] = int(span.max())
    # probes of a lower-bound search over a window, averaged over buckets
    res["mean_window_probes"] = round(float(np.mean(np.ceil(np.log2(span + 1.0)))), 2)
    res["plain_probes"] = int(np.ceil(np.log2(n + 1.0)))
    # The same method without the network: a zero-weight model (the
    # proportional prior d * na / N alone) calibrated on the same pair and
    # diagonals, so it gets its own per-bucket window table.
    zero = mp.LearnedPartitioner(32, 5, 7)
    zero.set_params(np.zeros(zero.num_params, np.float32))
    zero_err = zero.calibrate(A, B, 1 << 20)
    wz = zero.windows()
    zspan = wz[:, 1] - wz[:, 0]
    res["no_network"] = {
        "max_val_err": int(zero_err),
        "window_span_median": int(np.median(zspan)), "window_span_max": int(zspan.max()),
        "mean_window_probes": round(float(np.mean(np.ceil(np.log2(zspan + 1.0)))), 2),
        # one symmetric window from the largest error, no per-bucket table:
        # probes of a search over 2 * err + 1 candidates, network vs prior
        "symmetric_window_probes": int(np.ceil(np.log2(2 * zero_err + 1.0))),
        "symmetric_window_probes_trained": int(np.ceil(np.log2(2 * res["max_val_err"] + 1.0)))}
    del A, B
    torch.cuda.empty_cache()
    log("bench: learned: timing on the evaluation pair (seed 60)")
    A, B = gen.f32_mixture_pair_torch(n, n, 60)
    N = 2 * n
    sweep = {}
    for logp in (12, 16, 18, 20):
        P = 1 << logp
        diag = (torch.arange(P + 1, device="cuda", dtype=torch.int64) * N) // P
        out_p = torch.empty(P + 1, dtype=torch.int64, device="cuda")
        out_l = torch.empty(P + 1, dtype=torch.int64, device="cuda")
        fb = torch.zeros(1, dtype=torch.uint64, device="cuda")
        out_z = torch.empty(P + 1, dtype=torch.int64, device="cuda")
        t_plain = time_steps(lambda: mp.partition(A, B, diag, out=out_p), 10, 3)
        t_learn = time_steps(lambda: lp.partition(A, B, diag, out=out_l), 10, 3)
        t_zero = time_steps(lambda: zero.partition(A, B, diag, out=out_z), 10, 3)
        fb.zero_()
        lp.partition(A, B, diag, out=out_l, fallbacks=fb)
        fbz = torch.zeros(1, dtype=torch.uint64, device="cuda")
        zero.partition(A, B, diag, out=out_z, fallbacks=fbz)
        same = bool(torch.equal(out_p, out_l))
        sweep[f"P=2^{logp}"] = {"plain_ms": round(t_plain, 4), "learned_ms": round(t_learn, 4),
                                "speedup": round(t_plain / t_learn, 3), "identical": same,
                                "fallbacks": int(fb.cpu().numpy()[0]),
                                "no_network_ms": round(t_zero, 4),
                                "no_network_identical": bool(torch.equal(out_p, out_z)),
                                "no_network_fallbacks": int(fbz.cpu().numpy()[0])}
    res["sweep"] = sweep
    # training break-even: P = 2^18 partition calls whose saving repays the
    # training time
    s18 = sweep["P=2^18"]
    gain_ms = s18["plain_ms"] - s18["learned_ms"]
    res["training_break_even_calls_2p18"] = (round(res["train_s"] * 1e3 / gain_ms)
                                             if gain_ms > 0 else None)
    # spot-check against the oracle on sampled diagonals (one sequential walk)
    Ah, Bh = A.cpu().numpy(), B.cpu().numpy()
    ds = np.sort(np.random.default_rng(0).integers(0, N + 1, 256)).astype(np.int64)
    got = lp.partition(A, B, dev(ds)).cpu().numpy()
    res["oracle_spot_check_256"] = bool(np.array_equal(got, oracle.partition(Ah, Bh, ds)))
    # the full f32 merge (Algorithm 1 in two calls) on learned splits of the
    # diagonals of the built-in merge's 16384-key tiles, against the same on
    # plain splits and against the built-in merge (its own tile splits, then
    # the same tile kernel)
    log("bench: learned: full f32 merge on learned splits")
    T = 16384
    tdiag = torch.clamp(torch.arange((N + T - 1) // T + 1, device="cuda", dtype=torch.int64) * T,
                        max=N)
    sp_l = torch.empty_like(tdiag)
    sp_p = torch.empty_like(tdiag)
    S = torch.empty(N, dtype=torch.float32, device="cuda")
    t_pl = time_steps(lambda: lp.partition(A, B, tdiag, out=sp_l), 10, 3)
    t_pp = time_steps(lambda: mp.partition(A, B, tdiag, out=sp_p), 10, 3)
    t_mt = time_steps(lambda: mp.merge_split(A, B, sp_l, T, out=S), 10, 3)
    got = S.cpu().numpy()
    t_ps = time_steps(lambda: mp.merge(A, B, out=S), 10, 3)
    ref = oracle.merge(Ah, Bh)
    res["f32_merge_on_learned_splits"] = {
        "n": N, "tile": T, "tiles": int(tdiag.numel() - 1),
        "learned_split_ms": round(t_pl, 4), "plain_split_ms": round(t_pp, 4),
        "tile_merge_ms": round(t_mt, 4), "total_learned_ms": round(t_pl + t_mt, 4),
        "total_plain_ms": round(t_pp + t_mt, 4), "builtin_merge_ms": round(t_ps, 4),
        "splits_identical": bool(torch.equal(sp_l, sp_p)),
        "bit_exact": bool(got.tobytes() == ref.tobytes())}
    ex["learned"] = res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--log2n", type=int, default=28, help="log2 of |A| = |B| for the headline")
    ap.add_argument("--legs", default=",".join(LEGS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time only the reference copy of the headline's byte count")
    ap.add_argument("--bw-sweep", action="store_true",
                    help="only the bandwidth references: copy / read / write sweeps")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU only; a merge would shard by "
              "splitting the output at G-1 diagonals, but no multi-GPU path exists. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.bw_sweep:
        bw_sweep(args)
        return
    legs = [x for x in args.legs.split(",") if x]
    out = {}
    if "headline" in legs:
        leg_headline(args, out)
    ex = {}
    for name, fn in (("small", leg_small), ("kv", leg_kv), ("sort", leg_sort),
                     ("batched", leg_batched), ("learned", leg_learned), ("setops", leg_setops),
                     ("join", leg_join)):
        if name in legs:
            fn(args, ex)
            torch.cuda.empty_cache()
    if ex:
        out["extras"] = ex
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
