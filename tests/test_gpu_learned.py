"""GPU tests of the learned split predictor: network kernels against the
float64 oracle, and split output identical to the plain search."""
import os

import numpy as np
import pytest

import mp_inputs as gen
from oracle import mlp

pytestmark = pytest.mark.gpu

F, H = 5, 32


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_2628_amd as mp
    mp.lib()
    return mp


def _rand_model(mp, seed):
    g = np.random.default_rng(seed)
    lp = mp.LearnedPartitioner(H, F, seed)
    p = (g.normal(size=lp.num_params) * 0.8).astype(np.float32)
    lp.set_params(p)
    return lp, p.astype(np.float64)


def _features_np(d, na, nb):
    t = d / (na + nb)
    return np.stack([t, np.sin(2 * np.pi * t), np.cos(2 * np.pi * t),
                     np.sin(4 * np.pi * t), np.cos(4 * np.pi * t)], 1)


def _prior_np(d, na, nb):
    a = np.rint(d * na / (na + nb)).astype(np.int64)
    return np.clip(a, np.maximum(0, d - nb), np.minimum(d, na))


def test_forward_matches_oracle(mp):
    import torch
    from gpu_util import dev, host
    lp, p = _rand_model(mp, 1)
    X = np.random.default_rng(2).uniform(-1, 1, (3000, F)).astype(np.float32)
    got = host(lp.forward(dev(X)))
    want = mlp.forward(p, X.astype(np.float64), H)
    assert np.max(np.abs(got - want)) < 1e-4 * (1 + np.max(np.abs(want)))


def test_grad_matches_oracle_and_is_deterministic(mp):
    from gpu_util import dev, host
    lp, p = _rand_model(mp, 3)
    g = np.random.default_rng(4)
    X = g.uniform(-1, 1, (5000, F)).astype(np.float32)
    r = g.normal(size=5000).astype(np.float32)
    dX, dr = dev(X), dev(r)
    g1, l1 = lp.grad(dX, dr)
    g2, l2 = lp.grad(dX, dr)
    g1, l1, g2 = host(g1), host(l1), host(g2)
    assert g1.tobytes() == g2.tobytes()          # fixed-order reduction
    loss, want = mlp.loss_and_grad(p, X.astype(np.float64), r.astype(np.float64), H)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(g1 - want)) < 1e-4 * scale
    assert abs(l1[0] - loss) < 1e-4 * loss


def test_adam_step_matches_oracle(mp):
    from gpu_util import dev, host
    lp, p = _rand_model(mp, 5)
    g = np.random.default_rng(6)
    X = g.uniform(-1, 1, (2000, F)).astype(np.float32)
    r = g.normal(size=2000).astype(np.float32)
    _, grad = mlp.loss_and_grad(p, X.astype(np.float64), r.astype(np.float64), H)
    want, m, v = mlp.adam_step(p, grad, np.zeros_like(p), np.zeros_like(p), t=1, lr=1e-3)
    lp.adam_step(dev(X), dev(r), 1e-3)
    got = lp.get_params()
    assert np.max(np.abs(got - want)) < 2e-5


def test_examples_match_oracle(mp, orc):
    from gpu_util import dev, host
    A, B = gen.f32_mixture_pair(300_000, 200_000, 51)
    lp = mp.LearnedPartitioner(H, F, 7)
    X, r, d, s = lp.examples(dev(A), dev(B), 4096, seed=9)
    d, s, X, r = host(d), host(s), host(X), host(r)
    assert np.all((d >= 0) & (d <= len(A) + len(B)))
    assert np.array_equal(s, orc.partition(A, B, d))
    assert np.max(np.abs(X - _features_np(d, len(A), len(B)))) < 2e-6
    want_r = (s - _prior_np(d, len(A), len(B))) / len(A)
    assert np.max(np.abs(r - want_r)) < 1e-6


@pytest.fixture(scope="module")
def trained(mp):
    """A model trained on four seeds and calibrated on a fifth (small arrays)."""
    from gpu_util import dev
    n = 1 << 18
    sets = [tuple(map(dev, gen.f32_mixture_pair(n, n, s))) for s in (51, 52, 53, 54)]
    lp = mp.LearnedPartitioner(H, F, 11)
    loss0 = None
    X, r, _, _ = lp.examples(*sets[0], 2048)
    _, l = lp.grad(X, r)
    loss0 = float(l.cpu()[0])
    loss = lp.train(sets, k_diag=4096, epochs=600, lr=1e-2)
    A, B = map(dev, gen.f32_mixture_pair(n, n, 59))
    err = lp.calibrate(A, B, 1 << 14)
    return lp, loss0, loss, err, n


BUCKETS = 16384
CAL_SEED, CAL_DIAG = 11 ^ 0xC0FFEE, 1 << 14   # the fixture's calibration diagonals


def test_training_reduces_loss(trained):
    lp, loss0, loss, err, n = trained
    assert loss < 0.2 * loss0
    assert err < n // 4
    # one (lo, hi) window per bucket of t; lp.window is the largest |offset|
    w = lp.windows()
    assert w.shape == (BUCKETS, 2) and np.all(w[:, 0] < w[:, 1])
    assert lp.window == np.abs(w).max() and lp.window >= err


def _mean_window_probes(lp):
    w = lp.windows()
    return float(np.mean(np.ceil(np.log2(w[:, 1] - w[:, 0] + 1.0))))


def test_network_gain_attribution(mp, orc, trained):
    """What the trained network adds, measured against the same method
    without it: a zero-weight model (the proportional prior d * na / N
    alone) calibrated on the same held-out pair and diagonals.

    - One symmetric window (the largest calibration error on either side,
      no per-bucket table): the network shrinks the largest error, so the
      window search needs fewer probes than with the prior alone, and both
      need fewer than the plain search.
    - Per-bucket windows (the shipped calibration): the 16384-entry window
      table already follows the split curve piecewise, and the network
      adds no more than about one probe either way; both beat the plain
      search by several probes.
    Every variant gives the plain search's splits."""
    lp, _, _, err, n = trained
    from gpu_util import dev
    A, B = map(dev, gen.f32_mixture_pair(n, n, 59))
    z = mp.LearnedPartitioner(H, F, 11)           # same seed: same calibration diagonals
    z.set_params(np.zeros(z.num_params, np.float32))
    err_z = z.calibrate(A, B, CAL_DIAG)
    plain = int(np.ceil(np.log2(n + 1)))
    t_tab, z_tab = _mean_window_probes(lp), _mean_window_probes(z)
    assert t_tab < plain - 4 and z_tab < plain - 4, (t_tab, z_tab, plain)
    assert t_tab <= z_tab + 1.0, (t_tab, z_tab)
    # symmetric windows: probes of a search over 2 * err + 1 candidates
    assert err < err_z, (err, err_z)
    assert np.ceil(np.log2(2 * err + 1)) < np.ceil(np.log2(2 * err_z + 1)) <= plain
    E, Bv = gen.f32_mixture_pair(n, n, 60)
    diag = np.random.default_rng(4).integers(0, 2 * n + 1, 20000).astype(np.int64)
    _check_identical(mp, orc, z, E, Bv, diag)
    saved = lp.windows()
    lp.window = err + 1
    z.window = err_z + 1
    try:
        _check_identical(mp, orc, lp, E, Bv, diag)
        _check_identical(mp, orc, z, E, Bv, diag)
    finally:
        lp.calibrate(A, B, CAL_DIAG)                # restore the shipped windows
    assert np.array_equal(lp.windows(), saved)


def _calibration_windows_np(e, d, na, nb, n_diag):
    """The documented calibration rule, written out with a brute-force
    neighbourhood (the library uses running extremes)."""
    N = na + nb
    b = np.minimum(d * BUCKETS // (N + 1), BUCKETS - 1)
    r = max(1, -(-16 * BUCKETS // n_diag))
    noise = int(np.ceil(3.0 * np.sqrt(float(na) * float(nb) / (4.0 * float(N))))) + 1
    w = np.empty((BUCKETS, 2), np.int64)
    for k in range(BUCKETS):
        m = (b >= k - r) & (b <= k + r)
        lo, hi = (e[m].min(), e[m].max()) if m.any() else (e.min(), e.max())
        pad = (hi - lo) // 8 + noise
        w[k] = (lo - pad, hi + pad)
    return w


def test_calibration_windows_follow_the_rule(mp, trained):
    """Rebuild the calibration sample (same diagonals, exact splits, model
    outputs), apply the documented rule on the host, and compare bit for
    bit; then every calibration diagonal must be found inside its window."""
    import torch
    from gpu_util import dev, host
    lp, _, _, _, n = trained
    A, B = gen.f32_mixture_pair(n, n, 59)
    dA, dB = dev(A), dev(B)
    X, _, d, s = lp.examples(dA, dB, CAL_DIAG, seed=CAL_SEED)
    y = host(lp.forward(X))
    d, s = host(d), host(s)
    na = nb = n
    ys = y.astype(np.float32) * np.float32(na)
    ok = np.isfinite(ys) & (np.abs(ys) < np.float32(4e18))
    ahat = _prior_np(d, na, nb) + np.where(ok, np.rint(np.where(ok, ys, 0)), 0).astype(np.int64)
    ahat = np.clip(ahat, np.maximum(0, d - nb), np.minimum(d, na))
    e = s - ahat
    assert np.array_equal(lp.windows(), _calibration_windows_np(e, d, na, nb, CAL_DIAG))
    fb = torch.zeros(1, dtype=torch.uint64, device="cuda")
    got = host(lp.partition(dA, dB, dev(d), fallbacks=fb))
    assert np.array_equal(got, s)
    assert int(fb.cpu().numpy()[0]) == 0


def _check_identical(mp, orc, lp, A, B, diag, expect_fallback=None):
    import torch
    from gpu_util import dev, host
    dA, dB, dd = dev(A), dev(B), dev(diag)
    fb = torch.zeros(1, dtype=torch.uint64, device="cuda")
    got = host(lp.partition(dA, dB, dd, fallbacks=fb))
    plain = host(mp.partition(dA, dB, dd))
    assert np.array_equal(got, plain)
    assert np.array_equal(got, orc.partition(A, B, diag))
    n_fb = int(fb.cpu().numpy()[0])
    if expect_fallback is True:
        assert n_fb > 0
    elif expect_fallback is False:
        assert n_fb == 0
    return n_fb


def test_learned_partition_identical(mp, orc, trained):
    lp, _, _, _, n = trained
    A, B = gen.f32_mixture_pair(n, n, 60)
    diag = np.concatenate([[0, 1, 2 * n - 1, 2 * n],
                           np.random.default_rng(3).integers(0, 2 * n + 1, 20000)]).astype(np.int64)
    _check_identical(mp, orc, lp, A, B, diag)


def test_merge_from_learned_splits(mp, orc, trained):
    """The learned splits on the tile diagonals drive a full merge
    (mp_merge_split) to the oracle's bits."""
    from gpu_util import dev, host, first_mismatch
    lp, _, _, _, n = trained
    A, B = gen.f32_mixture_pair(n, n, 60)
    dA, dB = dev(A), dev(B)
    N = len(A) + len(B)
    d = np.minimum(np.arange((N + 4095) // 4096 + 1, dtype=np.int64) * 4096, N)
    sp = lp.partition(dA, dB, dev(d))
    got = host(mp.merge_split(dA, dB, sp, 4096))
    assert first_mismatch(got, orc.merge(A, B)) is None


def test_forced_fallback_zero_window(mp, orc, trained, tmp_path):
    lp, _, _, _, n = trained
    path = str(tmp_path / "copy.mplp")
    lp.save(path)
    lp0 = mp.LearnedPartitioner.load(path)
    lp0.window = 0  # one zero-width window everywhere
    assert len(lp0.windows()) == 0 and lp0.window == 0
    A, B = gen.f32_mixture_pair(n, n, 60)
    diag = np.random.default_rng(4).integers(0, 2 * n + 1, 5000).astype(np.int64)
    _check_identical(mp, orc, lp0, A, B, diag, expect_fallback=True)


def test_unbounded_window_is_the_full_search(mp, orc, trained, tmp_path):
    """The largest window offset clips to the diagonal without overflow."""
    lp, _, _, _, n = trained
    path = str(tmp_path / "copy.mplp")
    lp.save(path)
    big = mp.LearnedPartitioner.load(path)
    big.window = (1 << 63) - 1
    A, B = gen.f32_mixture_pair(n, n, 60)
    diag = np.concatenate([[0, 1, n, 2 * n - 1, 2 * n],
                           np.random.default_rng(9).integers(0, 2 * n + 1, 4000)]).astype(np.int64)
    _check_identical(mp, orc, big, A, B, diag, expect_fallback=False)


@pytest.mark.parametrize("lanes", [1, 4, 16, 64])
def test_learned_lanes_per_diagonal(mp, orc, trained, lanes):
    """The group searches of the learned partition (window, certificate and
    fallback) give the plain search's splits for every group size."""
    import torch
    from gpu_util import dev, host
    lp, _, _, _, n = trained
    A, B = gen.f32_mixture_pair(n, n, 60)
    diag = np.concatenate([[0, 1, n, 2 * n - 1, 2 * n],
                           np.random.default_rng(lanes).integers(0, 2 * n + 1, 3001)]).astype(np.int64)
    mp.set_partition_lanes(lanes)
    try:
        _check_identical(mp, orc, lp, A, B, diag)
        # a zero window sends every diagonal off its window edge to the fallback
        narrow = mp.LearnedPartitioner(H, F, 3)
        narrow.set_params(lp.get_params())
        narrow.window = 0
        _check_identical(mp, orc, narrow, A, B, diag, expect_fallback=True)
        # a model of another shape runs the kernel whose shape is not compiled in
        other = mp.LearnedPartitioner(7, 3, 4)
        other.window = 1000
        _check_identical(mp, orc, other, A, B, diag)
    finally:
        mp.set_partition_lanes(0)


def test_garbage_model_still_exact(mp, orc):
    lp = mp.LearnedPartitioner(H, F, 1)
    p = np.full(lp.num_params, 1e30, np.float32)
    p[::7] = np.nan
    lp.set_params(p)
    lp.window = 3
    for dt in (gen.U32, gen.I32, gen.U64, gen.F32):
        A, B = gen.uniform_pair(40_000, 70_001, 8, dt)
        diag = np.random.default_rng(5).integers(0, len(A) + len(B) + 1, 3000).astype(np.int64)
        _check_identical(mp, orc, lp, A, B, diag, expect_fallback=True)


def test_other_distribution_and_skew(mp, orc, trained):
    """A model trained on one distribution, used on another: still exact."""
    lp, _, _, _, n = trained
    for A, B in (gen.disjoint_pair(50_000, 80_000, 3), gen.dups_pair(70_000, 10, 4, hi=9)):
        A, B = A.astype(np.float32), B.astype(np.float32)
        diag = np.arange(0, len(A) + len(B) + 1, 37, dtype=np.int64)
        _check_identical(mp, orc, lp, A, B, diag)


def test_save_load_roundtrip(mp, orc, trained, tmp_path):
    import struct
    lp, _, _, _, n = trained
    path = str(tmp_path / "model.mplp")
    lp.save(path)
    lp2 = mp.LearnedPartitioner.load(path)
    assert lp2.shape == lp.shape and lp2.window == lp.window
    assert lp2.get_params().tobytes() == lp.get_params().tobytes()
    assert np.array_equal(lp2.windows(), lp.windows())
    # a file of the first format (one window, no table) still loads
    F_, H_ = lp.shape
    old = str(tmp_path / "v1.mplp")
    with open(old, "wb") as f:
        f.write(b"MPLP" + struct.pack("<Iiiq", 1, F_, H_, 12345) + struct.pack("<Q", 11))
        f.write(lp.get_params().astype("<f4").tobytes())
    lp1 = mp.LearnedPartitioner.load(old)
    assert lp1.window == 12345 and len(lp1.windows()) == 0
    # the second format: 1024 symmetric per-bucket windows, each covering 16
    # of today's buckets
    sym = np.random.default_rng(12).integers(0, 5000, 1024).astype("<i8")
    v2 = str(tmp_path / "v2.mplp")
    with open(v2, "wb") as f:
        f.write(b"MPLP" + struct.pack("<Iiiq", 2, F_, H_, int(sym.max())) + struct.pack("<Q", 11))
        f.write(lp.get_params().astype("<f4").tobytes())
        f.write(struct.pack("<i", 1024) + sym.tobytes())
    lp2w = mp.LearnedPartitioner.load(v2)
    rep = np.repeat(sym, BUCKETS // 1024)
    assert np.array_equal(lp2w.windows(), np.stack([-rep, rep], 1))
    assert lp2w.window == sym.max()
    A, B = gen.f32_mixture_pair(n, n, 61)
    diag = np.random.default_rng(6).integers(0, 2 * n + 1, 3000).astype(np.int64)
    _check_identical(mp, orc, lp1, A, B, diag)
    _check_identical(mp, orc, lp2w, A, B, diag)
    with open(path, "r+b") as f:
        f.write(b"XXXX")
    with pytest.raises(mp.MergePathError, match="STATE"):
        mp.LearnedPartitioner.load(path)


def test_uncalibrated_raises(mp):
    from gpu_util import dev
    lp = mp.LearnedPartitioner(H, F, 2)
    A, B = gen.uniform_pair(100, 100, 1)
    with pytest.raises(mp.MergePathError, match="STATE"):
        lp.partition(dev(A), dev(B), dev(np.arange(10, dtype=np.int64)))
