"""Differentiation extension on the GPU against the FP64 oracle: relaxed BAD
and HashSIFT descriptors, the hardest-negative triplet loss, the hand-written
backward kernels and the autograd chain.  Tolerances follow from FP32
arithmetic: descriptor values to ~1e-6 (times beta = 10 through tanh),
similarities of unit-range codes to ~1e-6, gradients to 1e-4 relative."""
import numpy as np
import pytest
import torch

import paper_2108_08380_amd as bd
from paper_2108_08380_amd import autograd as ag
from paper_2108_08380_amd import synth
from conftest import to_np

pytestmark = pytest.mark.gpu

BETA, TAU = 10.0, 0.5


def dev_t(a, dev, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype)


def test_patch_features(ref, dev):
    b = synth.triplets(synth.SEED_BASE + 50, n=300)
    got = to_np(bd.hashsift_patch_features(dev_t(b.anchor, dev)))
    np.testing.assert_allclose(got, ref.hashsift_patch_features(b.anchor), atol=1e-5)


@pytest.mark.parametrize("n_bits", [256, 512])
def test_relaxed_bad_forward(ref, dev, n_bits):
    rng = np.random.default_rng(51)
    b = synth.triplets(synth.SEED_BASE + 51, n=257)
    pairs = synth.box_pairs(rng, n_bits)
    w1, w2, th = rng.uniform(0.8, 1.2, n_bits), rng.uniform(0.8, 1.2, n_bits), rng.normal(0, 0.05, n_bits)
    D, m1, m2 = bd.relaxed_bad_fwd(dev_t(b.anchor, dev), bd.pairs_tensor(pairs, dev), dev_t(w1, dev), dev_t(w2, dev),
                                   dev_t(th, dev), BETA)
    w1f, w2f, thf = (np.float32(x).astype(np.float64) for x in (w1, w2, th))
    rho, Dr, m1r, m2r = ref.relaxed_bad(b.anchor, pairs, w1f, w2f, thf, BETA)
    np.testing.assert_allclose(to_np(m1), m1r, atol=2e-7)
    np.testing.assert_allclose(to_np(m2), m2r, atol=2e-7)
    np.testing.assert_allclose(to_np(D), Dr, atol=5e-6)


def test_relaxed_hashsift_forward(ref, dev):
    rng = np.random.default_rng(52)
    b = synth.triplets(synth.SEED_BASE + 52, n=300)
    f = bd.hashsift_patch_features(dev_t(b.anchor, dev))
    B, t = synth.projection(rng, 512)
    rho, D = bd.relaxed_hashsift_fwd(f, dev_t(B, dev), dev_t(t, dev), BETA)
    rr, Dr = ref.relaxed_hashsift(to_np(f).astype(np.float64), B.astype(np.float64), t.astype(np.float64), BETA)
    np.testing.assert_allclose(to_np(rho), rr, atol=1e-6)
    np.testing.assert_allclose(to_np(D), Dr, atol=2e-5)


def codes_pair(rng, n, K):
    A = np.tanh(rng.normal(0, 1, (n, K))).astype(np.float32)
    P = np.tanh(np.arctanh(A) + rng.normal(0, 0.7, A.shape)).astype(np.float32)
    return A, P


@pytest.mark.parametrize("n,K", [(2, 64), (5, 64), (100, 256), (257, 512), (1000, 512)])
def test_triplet_loss_forward_backward(ref, dev, n, K):
    rng = np.random.default_rng(n * 7 + K)
    A, P = codes_pair(rng, n, K)
    loss, neg, hinge = bd.trl_hnm_fwd(dev_t(A, dev), dev_t(P, dev), TAU)
    g = torch.ones(1, dtype=torch.float32, device=dev)
    gA, gP = bd.trl_hnm_bwd(dev_t(A, dev), dev_t(P, dev), neg, hinge, g)
    l64, n64, gA64, gP64 = ref.trl_hnm(A.astype(np.float64), P.astype(np.float64), TAU)
    assert abs(float(to_np(loss)[0]) - l64) <= 1e-6 + 1e-5 * abs(l64)
    neg = to_np(neg)
    same = neg == n64
    print(f"n={n} K={K} loss {l64:.6f} hardest-negative agreement {same.mean():.4f}")
    # the inputs are seeded, so every choice must agree; the message gives the
    # FP64 similarity gap of any that does not
    S = A.astype(np.float64) @ P.astype(np.float64).T / K
    val = lambda i, c: S[i, c] if c >= 0 else S[-1 - c, i]
    gaps = [(int(i), abs(val(i, neg[i]) - val(i, n64[i]))) for i in np.nonzero(~same)[0]]
    assert same.all(), f"hardest negatives differ from the oracle at (triplet, FP64 gap) {gaps[:8]}"
    scale = max(np.abs(gA64).max(), np.abs(gP64).max())
    np.testing.assert_allclose(to_np(gA), gA64, atol=1e-5 * scale)
    np.testing.assert_allclose(to_np(gP), gP64, atol=1e-5 * scale)


def test_hub_negative_gathers_many_sources(ref, dev):
    """One positive is every anchor's hardest negative: its gradient gathers
    contributions from all samples (the stable counting-sort path)."""
    rng = np.random.default_rng(53)
    n, K = 64, 128
    base = np.sign(rng.normal(size=K))
    flip = lambda x, p: x * np.where(rng.random(x.shape) < p, -1.0, 1.0)
    A = flip(np.tile(base, (n, 1)), 0.25).astype(np.float32)  # s(a_i, base) ~ 0.5
    P = flip(A, 0.10).astype(np.float32)                      # s(a_i, p_j) ~ 0.2 for j != i
    P[7] = base                                               # the hub
    loss, neg, hinge = bd.trl_hnm_fwd(dev_t(A, dev), dev_t(P, dev), 2.0)
    gA, gP = bd.trl_hnm_bwd(dev_t(A, dev), dev_t(P, dev), neg, hinge, torch.ones(1, device=dev))
    l64, n64, gA64, gP64 = ref.trl_hnm(A.astype(np.float64), P.astype(np.float64), 2.0)
    np.testing.assert_array_equal(to_np(neg), n64)
    assert (n64 == 7).sum() > 40
    np.testing.assert_allclose(to_np(gA), gA64, atol=1e-7)
    np.testing.assert_allclose(to_np(gP), gP64, atol=1e-7)


def test_relaxed_backward_kernels(ref, dev):
    rng = np.random.default_rng(54)
    n, K = 300, 512
    b = synth.triplets(synth.SEED_BASE + 54, n=n)
    pairs = synth.box_pairs(rng, K)
    w1, w2, th = (np.float32(x) for x in (rng.uniform(0.8, 1.2, K), rng.uniform(0.8, 1.2, K), rng.normal(0, 0.05, K)))
    D, m1, m2 = bd.relaxed_bad_fwd(dev_t(b.anchor, dev), bd.pairs_tensor(pairs, dev), dev_t(w1, dev), dev_t(w2, dev),
                                   dev_t(th, dev), BETA)
    gD = rng.normal(0, 1e-3, (n, K)).astype(np.float32)
    g1, g2, gt = bd.relaxed_bad_bwd(dev_t(gD, dev), D, m1, m2, BETA)
    e1, e2, et = ref.relaxed_bad_grad(gD, to_np(D), to_np(m1), to_np(m2), BETA)
    for got, exp in ((g1, e1), (g2, e2), (gt, et)):
        np.testing.assert_allclose(to_np(got), exp, rtol=1e-4, atol=1e-7)
    f = bd.hashsift_patch_features(dev_t(b.anchor, dev))
    B, t = synth.projection(rng, K)
    _, Dh = bd.relaxed_hashsift_fwd(f, dev_t(B, dev), dev_t(t, dev), BETA)
    gB, gtt = bd.relaxed_hashsift_bwd(dev_t(gD, dev), Dh, f, BETA)
    eB, egt = ref.relaxed_hashsift_grad(gD, to_np(Dh), to_np(f), BETA)
    np.testing.assert_allclose(to_np(gB), eB, rtol=1e-4, atol=1e-7)
    np.testing.assert_allclose(to_np(gtt), egt, rtol=1e-4, atol=1e-7)


def chain_reference_bad(ref, b, pairs, w1, w2, th):
    _, Da, m1a, m2a = ref.relaxed_bad(b.anchor, pairs, w1, w2, th, BETA)
    _, Dp, m1p, m2p = ref.relaxed_bad(b.positive, pairs, w1, w2, th, BETA)
    loss, neg, gA, gP = ref.trl_hnm(Da, Dp, TAU)
    a = ref.relaxed_bad_grad(gA, Da, m1a, m2a, BETA)
    p = ref.relaxed_bad_grad(gP, Dp, m1p, m2p, BETA)
    return loss, neg, [x + y for x, y in zip(a, p)]


def test_autograd_bad_chain(ref, dev):
    rng = np.random.default_rng(55)
    n, K = 128, 512
    b = synth.triplets(synth.SEED_BASE + 55, n=n)
    pairs = synth.box_pairs(rng, K)
    w1 = np.float32(rng.uniform(0.9, 1.1, K)); w2 = np.float32(rng.uniform(0.9, 1.1, K))
    th = np.float32(rng.normal(0, 0.05, K))
    P = [dev_t(x, dev).requires_grad_() for x in (w1, w2, th)]
    loss = ag.bad_triplet_loss(dev_t(b.anchor, dev), dev_t(b.positive, dev), *P, bd.pairs_tensor(pairs, dev), BETA, TAU)
    loss.backward()
    l64, neg, (e1, e2, et) = chain_reference_bad(ref, b, pairs, *(x.astype(np.float64) for x in (w1, w2, th)))
    assert abs(float(loss.detach()) - l64) < 1e-5
    scale = max(np.abs(e1).max(), np.abs(et).max())
    for p, e in zip(P, (e1, e2, et)):
        np.testing.assert_allclose(to_np(p.grad), e, atol=2e-4 * scale)


def test_autograd_hashsift_chain(ref, dev):
    rng = np.random.default_rng(56)
    n, K = 128, 512
    b = synth.triplets(synth.SEED_BASE + 56, n=n)
    fa = bd.hashsift_patch_features(dev_t(b.anchor, dev))
    fp = bd.hashsift_patch_features(dev_t(b.positive, dev))
    B, t = synth.projection(rng, K)
    Bt, tt = dev_t(B, dev).requires_grad_(), dev_t(t, dev).requires_grad_()
    loss = ag.hashsift_triplet_loss(fa, fp, Bt, tt, BETA, TAU)
    loss.backward()
    fa64, fp64 = to_np(fa).astype(np.float64), to_np(fp).astype(np.float64)
    _, Da = ref.relaxed_hashsift(fa64, B, t, BETA)
    _, Dp = ref.relaxed_hashsift(fp64, B, t, BETA)
    l64, neg, gA, gP = ref.trl_hnm(Da, Dp, TAU)
    eBa, eta = ref.relaxed_hashsift_grad(gA, Da, fa64, BETA)
    eBp, etp = ref.relaxed_hashsift_grad(gP, Dp, fp64, BETA)
    assert abs(float(loss.detach()) - l64) < 1e-5
    scale = np.abs(eBa + eBp).max()
    np.testing.assert_allclose(to_np(Bt.grad), eBa + eBp, atol=2e-4 * scale)
    np.testing.assert_allclose(to_np(tt.grad), eta + etp, atol=2e-4 * np.abs(eta + etp).max())


def test_full_batch_8192_triplets(dev):
    """8192 triplets, BAD-512 and HashSIFT-512: forward + backward are
    deterministic, and sampled hardest negatives match FP64 similarities."""
    rng = np.random.default_rng(57)
    b = synth.triplets(synth.SEED_BASE + 4, n=8192)
    pairs = bd.pairs_tensor(synth.box_pairs(rng, 512), dev)
    w1 = torch.ones(512, device=dev, requires_grad=True)
    w2 = torch.ones(512, device=dev, requires_grad=True)
    th = torch.zeros(512, device=dev, requires_grad=True)
    an, po = dev_t(b.anchor, dev), dev_t(b.positive, dev)
    grads = []
    for _ in range(2):
        for p in (w1, w2, th):
            p.grad = None
        loss = ag.bad_triplet_loss(an, po, w1, w2, th, pairs, BETA, TAU)
        loss.backward()
        grads.append([to_np(p.grad) for p in (w1, w2, th)] + [float(loss.detach())])
    for a, c in zip(grads[0], grads[1]):
        np.testing.assert_array_equal(a, c)
    # sampled check of the hardest negatives against FP64 similarities
    D_a = bd.relaxed_bad_fwd(an, pairs, w1.detach(), w2.detach(), th.detach(), BETA)[0]
    D_p = bd.relaxed_bad_fwd(po, pairs, w1.detach(), w2.detach(), th.detach(), BETA)[0]
    _, neg, hinge = bd.trl_hnm_fwd(D_a, D_p, TAU)
    A64, P64, neg = to_np(D_a).astype(np.float64), to_np(D_p).astype(np.float64), to_np(neg)
    for i in rng.choice(8192, 64, replace=False):
        row = A64[i] @ P64.T / 512
        col = A64 @ P64[i] / 512
        row[i] = col[i] = -np.inf
        best = max(row.max(), col.max())
        c = neg[i]
        got = row[c] if c >= 0 else col[-1 - c]
        assert abs(got - best) < 1e-5
        assert abs(float(to_np(hinge)[i]) - (TAU - A64[i] @ P64[i] / 512 + best)) < 1e-5
