"""Pins for the oracle's relaxed descriptors and triplet ranking loss (the
differentiation extension; the loss is Eq. 1 of Sec. III-A / Eq. 3 of
Sec. III-B with in-batch hardest negatives and anchor swap).

The analytic FP64 gradients are checked against finite differences (epsilon
1e-3, fourth-order central stencil) of the oracle's own forward loss,
skipping coordinates where the hardest-negative choice or the hinge activity
changes within +-epsilon.
The loss is pinned by a closed form on orthogonal codes and by the anchor
swap symmetry; the relaxed codes by the exact BAD and HashSIFT bits."""
import numpy as np
import pytest

from paper_2108_08380_amd import synth

BETA, TAU, EPS = 10.0, 0.5, 1e-3


def small_batch(seed, n, K):
    rng = np.random.default_rng(seed)
    b = synth.triplets(seed, n=n)
    pairs = synth.box_pairs(rng, K, radius_range=(1, 5))
    return rng, b, pairs


def bad_loss(ref, b, pairs, w1, w2, th):
    _, Da, m1a, m2a = ref.relaxed_bad(b.anchor, pairs, w1, w2, th, BETA)
    _, Dp, m1p, m2p = ref.relaxed_bad(b.positive, pairs, w1, w2, th, BETA)
    loss, neg, gA, gP = ref.trl_hnm(Da, Dp, TAU)
    return loss, neg, (Da, m1a, m2a, gA), (Dp, m1p, m2p, gP)


def check_fd(f, x0, grad, coords, state):
    """Finite differences of f at x0 along `coords` with the fourth-order
    central stencil on +-EPS and +-EPS/2 (truncation error O(EPS^4), which the
    strong curvature of tanh(beta rho) with beta = 10 needs at EPS = 1e-3).
    Coordinates whose discrete state (hardest negatives, active hinges)
    changes anywhere on the stencil are skipped."""
    checked = 0
    for c in coords:
        vals = []
        ok = True
        for d in (2.0, 1.0, -1.0, -2.0):
            x = x0.copy()
            x.flat[c] += d * EPS / 2
            v, st = f(x)
            ok &= np.array_equal(st, state)
            vals.append(v)
        if not ok:
            continue
        h = EPS / 2
        fd = (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)
        assert abs(fd - grad.flat[c]) <= 1e-8 + 1e-5 * abs(grad.flat[c]), (c, fd, grad.flat[c])
        checked += 1
    return checked


def test_bad_parameter_gradients_match_finite_differences(ref):
    rng, b, pairs = small_batch(synth.SEED_BASE + 40, 12, 64)
    K = 64
    w1 = rng.uniform(0.8, 1.2, K)
    w2 = rng.uniform(0.8, 1.2, K)
    th = rng.normal(0, 0.03, K)
    loss, neg, (Da, m1a, m2a, gA), (Dp, m1p, m2p, gP) = bad_loss(ref, b, pairs, w1, w2, th)
    assert loss > 0
    g1a, g2a, gta = ref.relaxed_bad_grad(gA, Da, m1a, m2a, BETA)
    g1p, g2p, gtp = ref.relaxed_bad_grad(gP, Dp, m1p, m2p, BETA)
    grads = {"w1": g1a + g1p, "w2": g2a + g2p, "theta": gta + gtp}
    state = np.concatenate([neg, [0]])

    def f_of(name):
        def f(x):
            args = {"w1": w1, "w2": w2, "theta": th}
            args[name] = x
            l, ng, A, P = bad_loss(ref, b, pairs, args["w1"], args["w2"], args["theta"])
            return l, np.concatenate([ng, [0]])
        return f

    total = 0
    for name, x0 in (("w1", w1), ("w2", w2), ("theta", th)):
        total += check_fd(f_of(name), x0, grads[name], range(K), state)
    assert total >= 2 * K  # most coordinates are away from a kink


def test_hashsift_parameter_gradients_match_finite_differences(ref):
    rng, b, _ = small_batch(synth.SEED_BASE + 41, 10, 64)
    K = 64
    fa = ref.hashsift_patch_features(b.anchor)
    fp = ref.hashsift_patch_features(b.positive)
    B, t = synth.projection(rng, K)
    B, t = B.astype(np.float64), t.astype(np.float64)

    def loss_of(Bx, tx):
        _, Da = ref.relaxed_hashsift(fa, Bx, tx, BETA)
        _, Dp = ref.relaxed_hashsift(fp, Bx, tx, BETA)
        return ref.trl_hnm(Da, Dp, TAU), Da, Dp

    (loss, neg, gA, gP), Da, Dp = loss_of(B, t)
    gBa, gta = ref.relaxed_hashsift_grad(gA, Da, fa, BETA)
    gBp, gtp = ref.relaxed_hashsift_grad(gP, Dp, fp, BETA)
    gB, gt = gBa + gBp, gta + gtp
    coords = rng.choice(B.size, 150, replace=False)
    nB = check_fd(lambda x: (lambda r: (r[0][0], r[0][1]))(loss_of(x, t)), B, gB, coords, neg)
    nt = check_fd(lambda x: (lambda r: (r[0][0], r[0][1]))(loss_of(B, x)), t, gt, range(K), neg)
    assert nB >= 100 and nt >= K // 2


def test_loss_gradients_wrt_codes_match_finite_differences(ref):
    rng = np.random.default_rng(42)
    A = np.tanh(rng.normal(0, 1, (14, 64)))
    P = np.tanh(A + rng.normal(0, 0.6, A.shape))
    loss, neg, gA, gP = ref.trl_hnm(A, P, TAU)
    assert loss > 0
    f = lambda X: (lambda r: (r[0], r[1]))(ref.trl_hnm(X, P, TAU, grads=False))
    g = lambda X: (lambda r: (r[0], r[1]))(ref.trl_hnm(A, X, TAU, grads=False))
    coords = rng.choice(A.size, 200, replace=False)
    assert check_fd(f, A, gA, coords, neg) >= 150
    assert check_fd(g, P, gP, coords, neg) >= 150


def test_anchor_swap_symmetry(ref):
    rng = np.random.default_rng(43)
    A = np.tanh(rng.normal(0, 1, (20, 128)))
    P = np.tanh(A + rng.normal(0, 0.5, A.shape))
    l1, _, gA1, gP1 = ref.trl_hnm(A, P, TAU)
    l2, _, gA2, gP2 = ref.trl_hnm(P, A, TAU)
    assert abs(l1 - l2) < 1e-12
    np.testing.assert_allclose(gA1, gP2, atol=1e-12)
    np.testing.assert_allclose(gP1, gA2, atol=1e-12)


def test_orthogonal_codes_closed_form(ref):
    """Rows of a Hadamard matrix: s(a_i, p_i) = 1 and every other similarity is 0,
    so each hinge is tau - 1: the loss is max(0, tau - 1)."""
    H = np.array([[1.0]])
    while H.shape[0] < 64:
        H = np.block([[H, H], [H, -H]])
    for tau, expect in ((0.5, 0.0), (1.5, 0.5), (3.0, 2.0)):
        loss, _, _, _ = ref.trl_hnm(H[:16], H[:16], tau)
        assert abs(loss - expect) < 1e-12


def test_hardest_negative_choice(ref):
    """A planted near-duplicate of p_0 among the positives is the hardest
    negative of a_0 (row candidate); a planted near-duplicate of a_3 among the
    anchors is the hardest negative of p_3 (column candidate)."""
    rng = np.random.default_rng(44)
    A = np.sign(rng.normal(size=(8, 64)))
    P = A.copy()
    P[5] = A[0]
    P[5, :4] *= -1  # s(a_0, p_5) = 56/64, the largest off-diagonal entry of row 0
    A[6] = P[3]
    A[6, :2] *= -1  # s(a_6, p_3) = 60/64
    _, neg, _, _ = ref.trl_hnm(A, P, TAU, grads=False)
    assert neg[0] == 5
    assert neg[3] == -1 - 6


def test_relaxed_bad_signs_are_the_bad_bits(ref):
    """With w1 = w2 = 1 the sign of rho is the BAD stump on the patch, computed
    by the exact integral-image path with the keypoint at the patch centre."""
    rng = np.random.default_rng(45)
    b = synth.triplets(synth.SEED_BASE + 45, n=12)
    patches = np.round(b.anchor * 255.0).astype(np.float32)  # integer grey levels
    pairs = synth.box_pairs(rng, 256, threshold_range=(-20, 20))
    th = pairs["threshold"].astype(np.float64) + 0.5  # off the integer ties
    rho, D, _, _ = ref.relaxed_bad(patches, pairs, np.ones(256), np.ones(256), th, BETA)
    p2 = pairs.copy()
    p2["threshold"] = th.astype(np.float32)
    kp = np.zeros(1, dtype=synth.KEYPOINT_DTYPE)
    kp[0] = (15.5, 15.5, 1.0, 0.0)
    for i in range(len(patches)):
        codes, _ = ref.describe_bad(ref.build_integral(patches[i].astype(np.uint8)), kp, p2)
        bits = np.unpackbits(codes.view(np.uint8), bitorder="little")
        np.testing.assert_array_equal(bits, (rho[i] >= 0).astype(np.uint8))
        np.testing.assert_array_equal(np.sign(D[i]), 2.0 * bits - 1)


def test_relaxed_hashsift_signs_are_the_hashsift_bits(ref):
    rng = np.random.default_rng(46)
    b = synth.triplets(synth.SEED_BASE + 46, n=10)
    B, t = synth.projection(rng, 256)
    f = ref.hashsift_patch_features(b.anchor)
    rho, D = ref.relaxed_hashsift(f, B, t, BETA)
    kp = np.zeros(1, dtype=synth.KEYPOINT_DTYPE)
    kp[0] = (15.5, 15.5, 1.0, 0.0)
    for i in range(len(f)):
        _, resp, codes = ref.describe_hashsift(b.anchor[i], kp, B, t)
        np.testing.assert_allclose(resp[0], rho[i], atol=1e-12)
        bits = np.unpackbits(codes.view(np.uint8), bitorder="little")
        np.testing.assert_array_equal(bits, (rho[i] > 0).astype(np.uint8))


def test_tanh_slope_at_zero_is_beta(ref):
    """d tanh(beta rho)/d theta at rho = 0 equals beta."""
    b = synth.triplets(synth.SEED_BASE + 47, n=1)
    pairs = synth.box_pairs(np.random.default_rng(47), 64)
    rho, _, m1, m2 = ref.relaxed_bad(b.anchor, pairs, np.ones(64), np.ones(64), np.zeros(64), BETA)
    th0 = m1[0] - m2[0]  # rho = 0 for every pair
    h = 1e-6
    _, Dp, _, _ = ref.relaxed_bad(b.anchor, pairs, np.ones(64), np.ones(64), th0 + h, BETA)
    _, Dm, _, _ = ref.relaxed_bad(b.anchor, pairs, np.ones(64), np.ones(64), th0 - h, BETA)
    np.testing.assert_allclose((Dp[0] - Dm[0]) / (2 * h), BETA, rtol=1e-6)


def _hnm_by_matrix(A, P, tau):
    """Hardest negatives and loss from the full similarity matrix S = A P^T / K
    (numpy's product): row candidates S[i, j], column candidates S[j, i],
    j != i, each taking its first maximum; the row candidate is kept when the
    two maxima are equal."""
    n, K = A.shape
    S = (A @ P.T) / K
    neg = np.zeros(n, dtype=np.int64)
    loss = 0.0
    for i in range(n):
        others = [j for j in range(n) if j != i]
        row = S[i, others]
        col = S[others, i]
        jr, jc = others[int(np.argmax(row))], others[int(np.argmax(col))]
        if row.max() >= col.max():
            neg[i], best = jr, row.max()
        else:
            neg[i], best = -1 - jc, col.max()
        loss += max(0.0, tau - S[i, i] + best) / n
    return neg, loss


def test_hardest_negative_ties_keep_first_row_candidate(ref):
    """With +-1 codes of 4 bits every similarity is a multiple of 1/4, so equal
    row and column maxima and equal candidates inside a row or a column are
    common.  The reading: the first maximum in index order, and the row
    candidate (a positive p_j) when its similarity equals the column
    candidate's (an anchor a_j)."""
    rng = np.random.default_rng(45)
    n_row_col_ties = 0
    for trial in range(20):
        A = np.sign(rng.normal(size=(12, 4)))
        P = np.sign(rng.normal(size=(12, 4)))
        loss, neg, _, _ = ref.trl_hnm(A, P, TAU, grads=False)
        expect, expect_loss = _hnm_by_matrix(A, P, TAU)
        np.testing.assert_array_equal(neg, expect)
        assert abs(loss - expect_loss) < 1e-12
        S = A @ P.T
        for i in range(12):
            others = [j for j in range(12) if j != i]
            n_row_col_ties += S[i, others].max() == S[others, i].max()
    assert n_row_col_ties > 50


def test_planted_row_column_tie(ref):
    """For triplet 0 the best row candidate s(a_0, p_5) and the best column
    candidate s(a_6, p_0) are both 60/64; the row candidate p_5 is the hardest
    negative."""
    rng = np.random.default_rng(46)
    A = np.sign(rng.normal(size=(8, 64)))
    P = A.copy()
    P[5] = A[0]
    P[5, :2] *= -1  # s(a_0, p_5) = 60/64
    A[6] = P[0]
    A[6, 10:12] *= -1  # s(a_6, p_0) = 60/64
    S = A @ P.T / 64
    assert S[0, 5] == S[6, 0] == 60 / 64
    assert S[0, [1, 2, 3, 4, 5, 6, 7]].max() == S[[1, 2, 3, 4, 5, 6, 7], 0].max()
    _, neg, _, _ = ref.trl_hnm(A, P, TAU, grads=False)
    assert neg[0] == 5
