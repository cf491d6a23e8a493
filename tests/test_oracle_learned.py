"""Pins of the learned-path oracle: the counter-based generator against its
published known answers, the Poisson inversion table against scipy's Poisson
CDF, the generated stacks against Poisson additivity and the closed-form mean
of the lock-in sums, the clean target against its closed form, the denoiser's
forward pass against scipy's correlation and its backward pass against
central finite differences, and Adam's first step against its closed form."""
import math

import numpy as np
import pytest
from scipy import signal, stats

import oracle
import scenes
from oracle import learned as L
from tests.golden.fixtures import read_rows


def test_philox_known_answers():
    rows = read_rows("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        assert L.philox4x32_10(r[0:4], r[4:6]) == r[6:10]


@pytest.mark.parametrize("lam", [1.5, 7.0, 100.0, 2000.0, 2001.2345])
def test_poisson_table_matches_scipy_cdf(lam):
    lo, thr = L.poisson_table(lam)
    k = lo + np.arange(len(thr))
    cdf = stats.poisson.cdf(k, lam)
    assert np.all(np.abs(thr / 2.0 ** 32 - cdf) <= 2.0 ** -31 + 1e-12)
    assert np.all(np.diff(thr.astype(np.int64)) >= 0)
    # Mass outside [lo, hi] is negligible.
    assert stats.poisson.cdf(lo - 1, lam) < 1e-20 and stats.poisson.sf(lo + len(thr), lam) < 1e-20


def test_inversion_is_the_smallest_k_above_u():
    lam = 3.7
    lo, thr = L.poisson_table(lam)
    u = np.linspace(1, 2 ** 32 - 1, 20001).astype(np.uint64)      # scipy's ppf(0) is -1 by convention
    x = L.poisson_invert(lo, thr, u)
    ppf = stats.poisson.ppf(u / 2.0 ** 32, lam)           # smallest k with cdf(k) >= q
    near = np.min(np.abs(u[:, None] / 2.0 ** 32 - stats.poisson.cdf(np.arange(30), lam)[None, :]), axis=1) < 1e-9
    assert np.all((x == ppf) | near)


def test_poisson_draws_statistics():
    lam = 2000.0
    lo, thr = L.poisson_table(lam)
    u = np.array([w for c in range(20000) for w in L.philox4x32_10([c, 7, 3, 0], [11, 22])], dtype=np.uint64)
    x = L.poisson_invert(lo, thr, u).astype(np.float64)
    n = len(x)
    assert abs(x.mean() - lam) < 5 * math.sqrt(lam / n)
    assert abs(x.var() - lam) < 5 * lam * math.sqrt(2.0 / n)
    # Chi-square against the Poisson pmf on 8 equiprobable-ish bins.
    edges = stats.poisson.ppf(np.linspace(0, 1, 9)[1:-1], lam)
    obs = np.bincount(np.searchsorted(edges, x, side="left"), minlength=8)
    cdf = np.concatenate([[0.0], stats.poisson.cdf(edges, lam), [1.0]])     # bin b: edges[b-1] < x <= edges[b]
    exp = np.diff(cdf) * n
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert chi2 < stats.chi2.ppf(0.9999, 7)


def small_tiles(n=2, H=10, W=12, seed=5):
    p = scenes.tile_params(seed, n, H=H, W=W, smin=3, smax=6)
    return p["mask"], p["rates"], p


def test_generated_stacks_poisson_additivity_and_lockin_mean():
    mask, rates, p = small_tiles(n=1, H=16, W=16)
    M = 64
    fr = L.gen_frames(mask, rates, M, tile0=3, seed=99).astype(np.float64)[0]     # [4M][H][W]
    for j in range(4):
        s = fr[j::4].sum(axis=0)                              # per-phase sums ~ Poisson(M lam_j)
        lam = np.where(mask[0] > 0, rates[0, 1, j], rates[0, 0, j]) * M
        z = (s - lam) / np.sqrt(lam)
        assert abs(z.mean()) < 5 / math.sqrt(z.size) and abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    # Same seed and tile -> same frames; another tile index -> different ones.
    a = L.gen_frames(mask, rates, 2, tile0=3, seed=99)
    b = L.gen_frames(mask, rates, 2, tile0=3, seed=99)
    c = L.gen_frames(mask, rates, 2, tile0=4, seed=99)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_pairs_short_window_is_prefix_and_mean_matches():
    mask, rates, p = small_tiles(n=3)
    d = L.gen_pairs(mask, rates, M_S=2, M_L=16, tile0=0, seed=1)
    fr = L.gen_frames(mask, rates, 16, tile0=0, seed=1)
    for i in range(3):
        I, Q = oracle.qld(fr[i, :8])
        assert np.array_equal(d["I_S"][i], I) and np.array_equal(d["Q_S"][i], Q)
        assert d["sum_L"][i] == fr[i].astype(np.int64).sum()
    # Noise-free lock-in of the rates: 2 A inside the mask, 0 outside (A = ballistic * background).
    a = L.a_star(mask, rates)
    A = p["ballistic"] * p["background"]
    assert np.allclose(a[mask > 0], 2 * A, rtol=1e-12) and np.allclose(a[mask == 0], 0.0, atol=1e-9)


def test_pairs_pixel_sums():
    mask, rates, p = small_tiles(n=2)
    d = L.gen_pairs(mask, rates, M_S=2, M_L=8, tile0=0, seed=5)
    fr = L.gen_frames(mask, rates, 8, tile0=0, seed=5)
    for i in range(2):
        assert np.array_equal(d["psum_S"][i], fr[i, :8].astype(np.int64).sum(axis=0))
        assert np.array_equal(d["psum_L"][i], fr[i].astype(np.int64).sum(axis=0))
        assert d["sum_S"][i] == d["psum_S"][i].sum() and d["sum_L"][i] == d["psum_L"][i].sum()


def test_target_bias_reduction_closed_form():
    # Without signal, E[I^2 + Q^2] = 4 M lam = the pixel's expected sample sum:
    # the bias-reduced target is ~0 on average.
    M, lam, H, W = 64, 2000.0, 64, 64
    rng = np.random.default_rng(3)
    I = rng.normal(0, math.sqrt(2 * M * lam), (1, H, W))
    Q = rng.normal(0, math.sqrt(2 * M * lam), (1, H, W))
    t = L.target(I, Q, np.full((1, H, W), 4 * M * lam), M, np.array([1.0]))
    plain = np.sqrt(I ** 2 + Q ** 2) / M
    assert t.mean() < 0.45 * plain.mean()


def test_normalise_hand_built():
    # Reading L17: x = (I, Q) / sqrt(P / 2) with P the pixel's sample sum;
    # scale = sigma / sqrt(M_S), sigma^2 = 2 b, b the tile's mean sample level.
    # P = 128, 32, 72, 280 give divisors 8, 4, 6, sqrt(140); H = W = 2, M_S = 4:
    # the tile's 64 samples summing to 512 give b = 8, sigma = 4, scale 4 / 2 = 2.
    I = np.array([[[8, -16], [24, 0]]])
    Q = np.array([[[0, 4], [-12, 0]]])
    P = np.array([[[128, 32], [72, 280]]])
    x, scale = L.normalise(I, Q, P, np.array([512]), 4, 2, 2)
    assert x.shape == (1, 2, 2, 2)
    assert np.array_equal(x[0, :, :, 0], [[1.0, -4.0], [4.0, 0.0]])
    assert np.array_equal(x[0, :, :, 1], [[0.0, 1.0], [-2.0, 0.0]])
    assert np.array_equal(scale, [2.0])
    # A pixel with no light (P = 0) gives x = 0.
    x0, _ = L.normalise(np.zeros((1, 1, 1)), np.zeros((1, 1, 1)), np.zeros((1, 1, 1)), np.array([8]), 1, 1, 1)
    assert np.array_equal(x0, np.zeros((1, 1, 1, 2)))


def test_normalise_unit_variance_on_signal_free_poisson():
    # Unmodulated Poisson light of rate lam: each cycle adds S0 - S2 of variance
    # 2 lam to I (and S1 - S3 to Q), so Var(I) = 2 M lam while the pixel's
    # sample sum estimates 4 M lam: x has unit variance per channel and zero
    # mean, in each half of a tile whose halves differ tenfold in rate (a
    # tile-wide level would give variances 2 lam_half / (lam_1 + lam_2)).
    rng = np.random.default_rng(11)
    M, H, W = 16, 128, 128
    lam = np.where(np.arange(W)[None, :] < W // 2, 300.0, 3000.0) * np.ones((H, 1))
    fr = rng.poisson(lam, size=(4 * M, H, W)).astype(np.uint16)
    I, Q = oracle.qld(fr)
    P = fr.astype(np.int64).sum(axis=0)
    x, scale = L.normalise(I[None], Q[None], P[None], np.array([int(P.sum())]), M, H, W)
    for half in (slice(0, W // 2), slice(W // 2, W)):
        for ch in range(2):
            v = x[0, :, half, ch]
            assert abs(v.var() - 1.0) < 0.04, (half, ch, v.var())
            assert abs(v.mean()) < 0.03, (half, ch)
    # The scale is the tile's: the standard deviation of I / M at the mean rate.
    assert abs(scale[0] - math.sqrt(2 * 1650.0 / M)) / scale[0] < 0.01


def test_target_hand_built():
    # t = sqrt(max(I^2 + Q^2 - P, 0)) / M_L / scale, P the pixel's sample sum.
    # M_L = 5, scale 0.5: (30, 40) with P = 2000: sqrt(500) / 5 / 0.5 = sqrt(80);
    # (10, 0) with P = 2000: 100 < 2000, clipped to 0; (30, 40) with P = 100:
    # sqrt(2400) / 2.5.
    t = L.target(np.array([[[30, 10, 30]]]), np.array([[[40, 0, 40]]]), np.array([[[2000, 2000, 100]]]), 5,
                 np.array([0.5]))
    assert t.shape == (1, 1, 3)
    assert abs(t[0, 0, 0] - math.sqrt(80.0)) < 1e-12 and t[0, 0, 1] == 0.0
    assert abs(t[0, 0, 2] - math.sqrt(2400.0) / 2.5) < 1e-12


def test_target_signal_free_closed_form():
    # Without signal, I and Q are (to a very good approximation) independent
    # Gaussians of variance 2 M lam, so r^2 = I^2 + Q^2 is 4 M lam times a unit
    # exponential E, and M^2 t^2 = 4 M lam max(E - 1, 0) with E[max(E - 1, 0)]
    # = 1/e: mean(t^2) = (4 lam / M) / e in each half of a tile whose halves
    # differ tenfold in rate.  (Removing 2 M lam instead would give e^-1/2,
    # i.e. 65% more; 8 M lam, e^-2; the tile's mean level, 1.6x or 0.2x.)
    rng = np.random.default_rng(12)
    M, H, W = 32, 256, 256
    lam = np.where(np.arange(W)[None, :] < W // 2, 300.0, 3000.0) * np.ones((H, 1))
    fr = rng.poisson(lam, size=(4 * M, H, W)).astype(np.uint16)
    I, Q = oracle.qld(fr)
    P = fr.astype(np.int64).sum(axis=0)
    t = L.target(I[None], Q[None], P[None], M, np.array([1.0]))
    for half, lh in ((slice(0, W // 2), 300.0), (slice(W // 2, W), 3000.0)):
        ratio = float((t[0, :, half] ** 2).mean()) / (4 * lh / M / math.e)
        assert abs(ratio - 1.0) < 0.04, (lh, ratio)


def test_bf16_rounding():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.0e38 * 0 + 65504.0])
    r = L.bf16(v)
    assert list(r[:4]) == [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7]      # ties to even
    assert r[4] == -2.5 and r[5] == 65536.0


def test_param_count():
    p = L.init_params(0)
    assert sum(p[k].size for k in p if not k.endswith("g")) == L.N_PARAMS == 19393


def test_conv_forward_against_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 9, 3))
    w = rng.normal(size=(3, 3, 3, 4))
    out = L.conv(x, w)
    for b in range(2):
        for co in range(4):
            ref = sum(signal.correlate2d(x[b, :, :, ci], w[:, :, ci, co], mode="same", boundary="fill")
                      for ci in range(3))
            assert np.allclose(out[b, :, :, co], ref, atol=1e-12)


def test_backward_against_finite_differences():
    rng = np.random.default_rng(2)
    p = L.init_params(4)
    for k in p:
        p[k] = p[k] + rng.normal(0, 0.05, size=p[k].shape)     # nonzero biases and gate
    x = rng.normal(size=(2, 6, 5, 2))
    t = rng.normal(size=(2, 6, 5))
    e = rng.normal(size=2)
    _, _, g, _ = L.loss_and_grads(p, x, t, e, emulate=False)
    h = 1e-6
    for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "Wg", "bg"):
        which = 1 if k in ("Wg", "bg") else 0      # the gate has its own loss
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = L.loss_and_grads(p, x, t, e, emulate=False)[which]
            flat[idx] = old - h
            lm = L.loss_and_grads(p, x, t, e, emulate=False)[which]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, an)


def test_adam_first_step_closed_form():
    p = {"w": np.array([0.5, -1.0, 2.0])}
    g = {"w": np.array([0.3, -0.02, 0.0])}
    st = {}
    L.adam(p, g, st, lr=0.01)
    expect = np.array([0.5, -1.0, 2.0]) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], expect, rtol=0, atol=1e-15)
