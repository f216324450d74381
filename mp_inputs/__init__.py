"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and prepares sorted input arrays with
library sorts (numpy).  It holds none of the merge method's arithmetic: no
merge, no split search, no merge sort.  Every generator is a pure function of
its arguments (numpy ``Generator(PCG64(seed))``).

Workload recipes (sizes are the full benchmark sizes; tests call the same
functions at smaller ``n``):

* uniform keys: ``U[0, 2^32)`` (u32), ``U[0, 2^64)`` (u64), ``U[-2^31, 2^31)``
  (i32), drawn then sorted.
* duplicates: keys ``U[0, 1024)`` sorted.
* disjoint: every A key in ``[2^31, 2^32)``, every B key in ``[0, 2^31)``
  (the case where all of A exceeds all of B, the paper's counter-example to
  splitting both inputs at equal lengths, section 1).
* Zipf: rank ``r`` in ``1..2^20`` with probability proportional to
  ``r^-1.1`` (inverse-CDF table), key = a bijective 32-bit mixer of ``r``.
* batched pairs: total pair size ``s = round(LogNormal(ln 4096, 0.7356))``
  clamped to ``[0, 2^22]``; ``|A_k| = floor(s * U(0,1))``, ``|B_k| = s - |A_k|``;
  int32 keys uniform within each array, sorted per array.
* float32 mixtures: uniform ``U[-1e6, 1e6)``, normal ``N(0, 1e3^2)``, Zipf
  rank as float, and 64 Gaussian clusters; each array mixes these with fixed
  weights; 0.1% of keys are replaced by +0.0 or -0.0.
"""
from __future__ import annotations

import numpy as np

U32, I32, U64, F32 = "u32", "i32", "u64", "f32"
NP_DTYPE = {U32: np.uint32, I32: np.int32, U64: np.uint64, F32: np.float32}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _uniform(g: np.random.Generator, n: int, dtype: str) -> np.ndarray:
    if dtype == U32:
        return g.integers(0, 2**32, size=n, dtype=np.uint32)
    if dtype == I32:
        return g.integers(-(2**31), 2**31, size=n, dtype=np.int32)
    if dtype == U64:
        return g.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    if dtype == F32:
        return g.uniform(-1e6, 1e6, size=n).astype(np.float32)
    raise ValueError(dtype)


def sorted_uniform(n: int, seed: int, dtype: str = U32) -> np.ndarray:
    a = _uniform(rng(seed), n, dtype)
    a.sort()
    return a


def uniform_pair(na: int, nb: int, seed: int, dtype: str = U32):
    """Two sorted arrays drawn from one seeded stream (A first, then B)."""
    g = rng(seed)
    a = _uniform(g, na, dtype)
    b = _uniform(g, nb, dtype)
    a.sort()
    b.sort()
    return a, b


def dups_pair(na: int, nb: int, seed: int, hi: int = 1024):
    g = rng(seed)
    a = g.integers(0, hi, size=na, dtype=np.uint32)
    b = g.integers(0, hi, size=nb, dtype=np.uint32)
    a.sort()
    b.sort()
    return a, b


def disjoint_pair(na: int, nb: int, seed: int):
    """All of A in [2^31, 2^32), all of B in [0, 2^31): every A key exceeds every B key."""
    g = rng(seed)
    a = g.integers(2**31, 2**32, size=na, dtype=np.uint32)
    b = g.integers(0, 2**31, size=nb, dtype=np.uint32)
    a.sort()
    b.sort()
    return a, b


def index_payload(na: int, nb: int):
    """Payload = position of the element in the concatenation A ++ B."""
    va = np.arange(na, dtype=np.uint32)
    vb = np.arange(na, na + nb, dtype=np.uint32)
    return va, vb


def fmix32(x: np.ndarray) -> np.ndarray:
    """MurmurHash3's 32-bit finaliser: a bijection on 32-bit words (spreads hot keys)."""
    h = x.astype(np.uint32).copy()
    h ^= h >> np.uint32(16)
    h *= np.uint32(0x85EBCA6B)
    h ^= h >> np.uint32(13)
    h *= np.uint32(0xC2B2AE35)
    h ^= h >> np.uint32(16)
    return h


def zipf_ranks(g: np.random.Generator, n: int, s: float = 1.1, n_values: int = 2**20) -> np.ndarray:
    w = np.arange(1, n_values + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = g.random(n)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, n_values).astype(np.uint32)


def zipf_keys(n: int, seed: int, s: float = 1.1, n_values: int = 2**20) -> np.ndarray:
    """Unsorted u32 keys, Zipf(s) over n_values distinct values (input for sort)."""
    return fmix32(zipf_ranks(rng(seed), n, s, n_values))


def unsorted_uniform(n: int, seed: int, dtype: str = U32) -> np.ndarray:
    return _uniform(rng(seed), n, dtype)


# --- batched (segmented) pairs -------------------------------------------------

LOGNORMAL_SIGMA = 0.7356  # E[s] = 4096 * exp(sigma^2 / 2) = 2^29 / 1e5


def batched_sizes(n_pairs: int, seed: int, median: float = 4096.0,
                  sigma: float = LOGNORMAL_SIGMA, cap: int = 2**22):
    g = rng(seed)
    s = np.rint(g.lognormal(np.log(median), sigma, size=n_pairs))
    s = np.clip(s, 0, cap).astype(np.int64)
    na = np.floor(s * g.random(n_pairs)).astype(np.int64)
    nb = s - na
    return na, nb


def offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def _segment_sorted_i32(g: np.random.Generator, sizes: np.ndarray) -> np.ndarray:
    total = int(sizes.sum())
    keys = g.integers(-(2**31), 2**31, size=total, dtype=np.int64)
    seg = np.repeat(np.arange(len(sizes), dtype=np.int64), sizes)
    # (segment, key) packed in one int64 so that one library sort orders by
    # segment first and by key inside each segment.
    packed = (seg << 32) | (keys + 2**31)
    packed.sort()
    return ((packed & 0xFFFFFFFF) - 2**31).astype(np.int32)


def batched_pairs(n_pairs: int, seed: int, median: float = 4096.0,
                  sigma: float = LOGNORMAL_SIGMA, cap: int = 2**22):
    """Returns (A, a_off, B, b_off): CSR-concatenated independent sorted pairs."""
    na, nb = batched_sizes(n_pairs, seed, median, sigma, cap)
    g = rng(seed + 1_000_003)
    a = _segment_sorted_i32(g, na)
    b = _segment_sorted_i32(g, nb)
    return a, offsets(na), b, offsets(nb)


# --- float32 mixtures ------------------------------------------------------------

FAMILY_SEED = 5000  # fixes the cluster geometry shared by every seed of a family

# mixture weights over (uniform, normal, zipf, clustered), one row per array role
MIX_A = np.array([0.40, 0.30, 0.10, 0.20])
MIX_B = np.array([0.15, 0.25, 0.20, 0.40])


def _clusters(n_clusters: int = 64):
    g = rng(FAMILY_SEED)
    centres = g.uniform(-1e6, 1e6, size=n_clusters)
    sig = np.exp(g.uniform(np.log(1.0), np.log(1e3), size=n_clusters))
    w = g.dirichlet(np.ones(n_clusters))
    return centres, sig, w


def f32_mixture(n: int, g: np.random.Generator, mix: np.ndarray) -> np.ndarray:
    counts = g.multinomial(n, mix)
    parts = [
        g.uniform(-1e6, 1e6, size=counts[0]),
        g.normal(0.0, 1e3, size=counts[1]),
        zipf_ranks(g, counts[2]).astype(np.float64),
    ]
    centres, sig, w = _clusters()
    cid = g.choice(len(centres), size=counts[3], p=w)
    parts.append(centres[cid] + sig[cid] * g.standard_normal(counts[3]))
    x = np.concatenate(parts).astype(np.float32)
    # signed zeros: both compare equal, their bit patterns tell which input won a tie
    nz = max(1, n // 1000) if n >= 1000 else 0
    if nz:
        idx = g.choice(n, size=nz, replace=False)
        x[idx] = np.where(g.random(nz) < 0.5, np.float32(0.0), np.float32(-0.0))
    x.sort()
    return x


def f32_mixture_pair(na: int, nb: int, seed: int):
    g = rng(seed)
    return f32_mixture(na, g, MIX_A), f32_mixture(nb, g, MIX_B)


def f32_mixture_torch(n: int, seed: int, mix: np.ndarray, device="cuda"):
    """The f32 mixture recipe drawn with torch's generator on `device` (for
    sizes where host generation is slow).  Same family as f32_mixture (same
    weights, cluster geometry and signed-zero rate), different random stream."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def categorical(weights, count):
        # inverse-CDF draw of `count` category indices
        cdf = torch.cumsum(torch.as_tensor(weights, dtype=torch.float64, device=device), 0)
        cdf = cdf / cdf[-1]
        u = torch.rand(count, generator=g, device=device, dtype=torch.float64)
        return torch.searchsorted(cdf, u, right=True).clamp(max=len(weights) - 1)

    comp = categorical(mix, n)
    x = torch.empty(n, dtype=torch.float64, device=device)
    m = comp == 0
    x[m] = torch.rand(int(m.sum()), generator=g, device=device, dtype=torch.float64) * 2e6 - 1e6
    m = comp == 1
    x[m] = torch.randn(int(m.sum()), generator=g, device=device, dtype=torch.float64) * 1e3
    m = comp == 2
    w = torch.arange(1, 2**20 + 1, dtype=torch.float64, device=device) ** (-1.1)
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    u = torch.rand(int(m.sum()), generator=g, device=device, dtype=torch.float64)
    x[m] = (torch.searchsorted(cdf, u, right=True) + 1).clamp(max=2**20).to(torch.float64)
    m = comp == 3
    centres, sig, wts = (torch.tensor(a, device=device) for a in _clusters())
    cid = categorical(wts, int(m.sum()))
    x[m] = centres[cid] + sig[cid] * torch.randn(int(m.sum()), generator=g, device=device,
                                                  dtype=torch.float64)
    x = x.to(torch.float32)
    nz = n // 1000
    if nz:
        idx = torch.randint(0, n, (nz,), generator=g, device=device)
        signs = torch.rand(nz, generator=g, device=device) < 0.5
        x[idx] = torch.where(signs, torch.tensor(0.0, device=device), torch.tensor(-0.0, device=device))
    return torch.sort(x).values


def f32_mixture_pair_torch(na: int, nb: int, seed: int, device="cuda"):
    return (f32_mixture_torch(na, 2 * seed, MIX_A, device),
            f32_mixture_torch(nb, 2 * seed + 1, MIX_B, device))
