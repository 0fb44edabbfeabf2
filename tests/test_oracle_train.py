"""Pins for the oracle's HashSIFT training pieces (Sec. III-B): the data
augmentation by special cases that reduce to exact operations, Adam by its
closed-form first step and a hand-computed second step, and the gradient of
one training step by finite differences of its own forward loss."""
import math

import numpy as np
import pytest

from paper_2108_08380_amd import synth

IDENT = (0.0, 1.0, 1.0, 0.0, 0.0)


def patches(n=3, seed=100):
    return np.random.default_rng(seed).uniform(0.05, 0.95, (n, 32, 32)).astype(np.float32)


def aug(ref, src, params, noise=None):
    n = len(src)
    return ref.augment_patches(src, np.asarray(params, dtype=np.float64).reshape(n, 5),
                               np.zeros((n, 32, 32), np.float32) if noise is None else noise)


def test_identity_is_exact(ref):
    p = patches()
    np.testing.assert_array_equal(aug(ref, p, [IDENT] * 3), p)


def test_quarter_and_half_turns(ref):
    p = patches(1)
    q = aug(ref, p, [(math.pi / 2, 1.0, 1.0, 0.0, 0.0)])[0]
    # output (i, j) samples x = 15.5 - (i - 15.5) = 31 - i, y = j: src[j, 31 - i]
    np.testing.assert_allclose(q, p[0].T[::-1, :], atol=1e-6)
    h = aug(ref, p, [(math.pi, 1.0, 1.0, 0.0, 0.0)])[0]
    np.testing.assert_allclose(h, p[0][::-1, ::-1], atol=1e-6)


def test_scale_two_averages_neighbours(ref):
    p = patches(1)
    s = aug(ref, p, [(0.0, 2.0, 1.0, 0.0, 0.0)])[0]
    # (i, j) samples (2j - 15.5, 2i - 15.5): the mean of four pixels, inside for 8 <= i, j <= 23
    for i in range(8, 24):
        for j in range(8, 24):
            x0, y0 = 2 * j - 16, 2 * i - 16
            exp = p[0][y0:y0 + 2, x0:x0 + 2].astype(np.float64).mean()
            assert abs(s[i, j] - exp) < 1e-6


def test_illumination_noise_and_clipping(ref):
    p = patches(2)
    noise = np.random.default_rng(3).normal(0, 0.3, (2, 32, 32)).astype(np.float32)
    out = aug(ref, p, [(0.0, 1.0, 1.3, -0.1, 0.0), (0.0, 1.0, 0.7, 0.2, 0.0)], noise)
    for k, (g, b) in enumerate(((1.3, -0.1), (0.7, 0.2))):
        exp = np.clip(g * p[k].astype(np.float64) + b + noise[k], 0.0, 1.0).astype(np.float32)
        np.testing.assert_allclose(out[k], exp, atol=1e-7)
    assert (out == 0.0).any() and (out == 1.0).any()


def test_blur_special_cases(ref):
    const = np.full((1, 32, 32), 0.37, np.float32)
    np.testing.assert_allclose(aug(ref, const, [(0.0, 1.0, 1.0, 0.0, 1.3)]), const, atol=1e-7)
    ramp = np.tile((np.arange(32) / 40.0).astype(np.float32), (32, 1))[None]
    out = aug(ref, ramp, [(0.0, 1.0, 1.0, 0.0, 1.0)])[0]
    np.testing.assert_allclose(out[:, 3:29], ramp[0][:, 3:29], atol=1e-7)  # symmetric kernel keeps a ramp
    imp = np.zeros((1, 32, 32), np.float32)
    imp[0, 16, 16] = 1.0
    sigma = 1.5
    out = aug(ref, imp, [(0.0, 1.0, 1.0, 0.0, sigma)])[0]
    d = np.arange(-5, 6)
    w = np.exp(-d * d / (2 * sigma * sigma))
    w /= w.sum()
    np.testing.assert_allclose(out[11:22, 11:22], np.outer(w, w), atol=1e-7)
    assert abs(out.sum() - 1.0) < 1e-6


def test_adam_first_step_and_hand_example(ref):
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    ref.adam_step(p, g, m, v, 1, 0.1)
    np.testing.assert_allclose(p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # scalar, two steps: p0 = 1, g = 0.5 then -0.25, lr = 0.1
    p, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    ref.adam_step(p, np.array([0.5]), m, v, 1, 0.1)
    ref.adam_step(p, np.array([-0.25]), m, v, 2, 0.1)
    m2 = 0.9 * 0.05 + 0.1 * -0.25                      # = 0.02
    v2 = 0.999 * 0.00025 + 0.001 * 0.0625              # = 0.00031225
    p1 = 1.0 - 0.1 * 0.5 / (0.5 + 1e-8)               # m1_hat = 0.5, sqrt(v1_hat) = 0.5
    p2 = p1 - 0.1 * (m2 / (1 - 0.81)) / (math.sqrt(v2 / (1 - 0.998001)) + 1e-8)
    assert abs(p[0] - p2) < 1e-12


def step_inputs(n=6, P=10, K=64, seed=101):
    rng = np.random.default_rng(seed)
    b = synth.triplets(synth.SEED_BASE + seed, n=P)
    pool = np.empty((2 * P, 32, 32), np.float32)
    pool[0::2], pool[1::2] = b.anchor, b.positive
    batch = rng.permutation(P)[:n]
    params = np.stack([rng.uniform(-0.17, 0.17, 2 * n), rng.uniform(0.9, 1.1, 2 * n), rng.uniform(0.8, 1.2, 2 * n),
                       rng.uniform(-0.1, 0.1, 2 * n), rng.uniform(0.0, 1.0, 2 * n)], axis=1)
    noise = rng.normal(0, 0.02, (2 * n, 32, 32)).astype(np.float32)
    B = rng.normal(0, 0.5, (K, 128))
    t = rng.normal(0, 0.1, K)
    return pool, batch, params, noise, B, t


def forward_loss(ref, pool, batch, params, noise, B, t, tau=0.5, beta=1.0):
    src = np.empty((2 * len(batch), 32, 32), np.float32)
    src[0::2], src[1::2] = pool[2 * batch], pool[2 * batch + 1]
    a = ref.augment_patches(src, params, noise)
    fa, fp = ref.hashsift_patch_features(a[0::2]), ref.hashsift_patch_features(a[1::2])
    _, Da = ref.relaxed_hashsift(fa, B, t, beta)
    _, Dp = ref.relaxed_hashsift(fp, B, t, beta)
    loss, neg, _, _ = ref.trl_hnm(Da, Dp, tau, grads=False)
    return loss, neg


def test_training_step_gradient_by_finite_differences(ref):
    pool, batch, params, noise, B, t = step_inputs()
    K = B.shape[0]
    state = {"mB": np.zeros_like(B), "vB": np.zeros_like(B), "mt": np.zeros(K), "vt": np.zeros(K), "step": 0}
    B1, t1 = B.copy(), t.copy()
    loss, gB, gt = ref.hashsift_train_step(pool, batch, params, noise, B1, t1, state)
    l0, neg0 = forward_loss(ref, pool, batch, params, noise, B, t)
    assert loss == l0 and loss > 0
    rng = np.random.default_rng(5)
    h = 1e-6
    checked = 0
    for c in rng.choice(B.size, 40, replace=False):
        Bp, Bm = B.copy(), B.copy()
        Bp.flat[c] += h
        Bm.flat[c] -= h
        lp, np_ = forward_loss(ref, pool, batch, params, noise, Bp, t)
        lm, nm = forward_loss(ref, pool, batch, params, noise, Bm, t)
        if not (np.array_equal(np_, neg0) and np.array_equal(nm, neg0)):
            continue
        assert abs((lp - lm) / (2 * h) - gB.flat[c]) <= 1e-6 + 1e-4 * abs(gB.flat[c])
        checked += 1
    assert checked >= 30
    # the Adam step moved every coordinate with a non-zero gradient by about lr
    moved = np.abs(B1 - B)[np.abs(gB) > 1e-4]
    assert np.allclose(moved, 2e-4, rtol=1e-3) and state["step"] == 1
