"""Pins for the oracle's threshold search (Sec. III-A, Alg. 2 with integer
sorting into m bins).

* The bin count is the paper's m = 5110 (tests/golden/threshold_search.txt).
* Bins are pinned by exact rational arithmetic on box sums computed with
  numpy slicing, including clamped boxes and the extreme features +-255.
* The whole search is pinned by brute force: the loss of Eq. 2 evaluated
  directly at every one of the 5110 thresholds (the O(P^2)-type search the
  paper contrasts with), on sets with tied feature values inside triplets.
* A one-triplet closed form: the best stump separates the negative from the
  identical anchor and positive, loss 0."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2108_08380_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "threshold_search.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def cand(x1, y1, x2, y2, r):
    c = np.zeros(1, dtype=synth.BOX_PAIR_DTYPE)
    c[0]["x1"], c[0]["y1"], c[0]["x2"], c[0]["y2"], c[0]["radius"] = x1, y1, x2, y2, r
    return c


def box_sum(patch, ux, uy, r):
    r = min(int(r), 15)
    cx = min(max(16 + int(ux), r), 31 - r)
    cy = min(max(16 + int(uy), r), 31 - r)
    return int(patch[cy - r:cy + r + 1, cx - r:cx + r + 1].astype(np.int64).sum()), (2 * r + 1) ** 2


def bin_exact(patch, c):
    s1, a = box_sum(patch, c["x1"], c["y1"], c["radius"])
    s2, _ = box_sum(patch, c["x2"], c["y2"], c["radius"])
    return math.floor((Fraction(s1 - s2, a) + 255) * 10)


def test_bin_count_is_the_papers_m(ref):
    g = golden()
    assert ref.THRESHOLD_BINS == int(g["m"]) == round((g["search_max"] - g["search_min"] + 1) / g["precision"])


def test_bins_by_exact_rationals(ref):
    rng = np.random.default_rng(80)
    patches = rng.integers(0, 256, (40, 32, 32), dtype=np.uint8)
    cands = synth.box_pairs(rng, 60, max_offset=16, radius_range=(0, 15))
    for p in patches[:10]:
        for c in cands:
            assert ref.threshold_bin(p, c) == bin_exact(p, c)
    # extremes: +-255 and 0
    p = np.zeros((32, 32), dtype=np.uint8)
    p[:, :16] = 255
    assert ref.threshold_bin(p, cand(-8, 0, 8, 0, 3)) == 5100
    assert ref.threshold_bin(p, cand(8, 0, -8, 0, 3)) == 0
    assert ref.threshold_bin(p, cand(-8, 0, -8, 5, 3)) == 2550
    # fractional features: six ones in a 3x3 box give f = 2/3, bin floor(2556.67) = 2556;
    # the reverse gives f = -2/3, bin floor(2543.33) = 2543
    q = np.zeros((32, 32), dtype=np.uint8)
    q[14:17, 2:4] = 1  # columns 2, 3 of the box centred at (3, 15)
    assert ref.threshold_bin(q, cand(-13, -1, 10, 10, 1)) == 2556
    assert ref.threshold_bin(q, cand(10, 10, -13, -1, 1)) == 2543


def brute_force(patches, s_ap, s_an, tau, cands):
    n = len(s_ap)
    best_bin, best_loss = [], []
    for c in cands:
        q = np.array([bin_exact(patches[k], c) for k in range(3 * n)]).reshape(n, 3)
        b = np.arange(5110)[:, None]
        h = np.where(q[None, :, :] <= b[:, :, None], 1, -1)  # (bins, n, 3)
        terms = tau - s_ap[None] - h[:, :, 0] * h[:, :, 1] + s_an[None] + h[:, :, 0] * h[:, :, 2]
        L = np.maximum(terms, 0).sum(axis=1)
        bb = int(np.argmin(L))  # first minimum
        best_bin.append(bb)
        best_loss.append(float(L[bb]))
    return np.array(best_bin), np.array(best_loss)


@pytest.mark.parametrize("tau", [0.5, 1.0, 2.5])
def test_search_equals_brute_force(ref, tau):
    rng = np.random.default_rng(81 + int(tau * 2))
    n = 40
    base = rng.integers(0, 256, (n, 32, 32), dtype=np.uint8)
    patches = np.empty((3 * n, 32, 32), dtype=np.uint8)
    patches[0::3] = base
    patches[1::3] = np.clip(base.astype(int) + rng.integers(-30, 31, base.shape), 0, 255)
    patches[2::3] = rng.integers(0, 256, (n, 32, 32), dtype=np.uint8)
    patches[3] = patches[4]            # tied anchor/positive values
    patches[7] = patches[8]            # tied positive/negative values
    patches[9:12] = 100                # a constant triplet: every feature 0
    s_ap = rng.integers(-8, 9, n).astype(np.int32)
    s_an = rng.integers(-8, 9, n).astype(np.int32)
    cands = synth.box_pairs(rng, 12, radius_range=(0, 6))
    got_bin, got_loss = ref.find_threshold(patches, s_ap, s_an, tau, cands)
    exp_bin, exp_loss = brute_force(patches, s_ap, s_an, tau, cands)
    np.testing.assert_array_equal(got_bin, exp_bin)
    np.testing.assert_array_equal(got_loss, exp_loss)


def test_one_triplet_closed_form(ref):
    """Anchor = positive, negative brighter in box 1: tau = 1, s = 0.  At the
    lowest threshold every stump is -1 and the loss is [1 - 1 + 1]_+ = 1; the
    best stump puts anchor and positive on one side and the negative on the
    other, loss [1 - 1 - 1]_+ = 0, first reached at the anchor's bin."""
    a = np.full((32, 32), 50, dtype=np.uint8)
    n_ = a.copy()
    n_[:, :16] = 200
    patches = np.stack([a, a, n_])
    c = cand(-8, 0, 8, 0, 2)
    qa, qn = bin_exact(a, c[0]), bin_exact(n_, c[0])
    assert qa < qn
    b, loss = ref.find_threshold(patches, np.zeros(1, np.int32), np.zeros(1, np.int32), 1.0, c)
    assert b[0] == qa and loss[0] == 0.0
    # with the negative darker the stump flips it alone first
    b, loss = ref.find_threshold(np.stack([n_, n_, a]), np.zeros(1, np.int32), np.zeros(1, np.int32), 1.0, c)
    assert b[0] == qa and loss[0] == 0.0


# ---------------------------------------------------------------- Alg. 1: greedy selection


def hamming_matrix(x, y):
    xb = np.unpackbits(x.view(np.uint8), axis=1).astype(np.int32)
    yb = np.unpackbits(y.view(np.uint8), axis=1).astype(np.int32)
    return (xb[:, None, :] != yb[None, :, :]).sum(axis=2)


def hnm_by_matrix(a, p):
    n = len(a)
    Dap = hamming_matrix(a, p)  # row candidates: d(a_s, p_j)
    Dpa = hamming_matrix(p, a)  # column candidates: d(p_s, a_j)
    neg, dn = [], []
    for s in range(n):
        order = (s + 1 + np.arange(n - 1)) % n  # cyclic from s + 1: argmin keeps the first
        r, c = Dap[s][order], Dpa[s][order]
        jr, jc = int(order[np.argmin(r)]), int(order[np.argmin(c)])
        r, c = Dap[s], Dpa[s]
        if r[jr] <= c[jc]:
            neg.append(jr)
            dn.append(r[jr])
        else:
            neg.append(-1 - jc)
            dn.append(c[jc])
    return np.array(neg), np.array(dn), np.diag(Dap)


def test_hardest_negatives_by_distance_matrix(ref):
    rng = np.random.default_rng(90)
    for n, w in ((2, 1), (9, 1), (33, 2), (40, 4)):
        a = rng.integers(0, 2**63, (n, w), dtype=np.uint64)
        p = a ^ (rng.random((n, w)) < 0.3).astype(np.uint64) * rng.integers(0, 2**63, (n, w), dtype=np.uint64)
        if n > 4:
            p[2] = a[0]  # ties and exact duplicates
            a[3] = p[1]
        neg, dn, dp = ref.hnm_codes(a, p)
        en, ed, ep = hnm_by_matrix(a, p)
        np.testing.assert_array_equal(neg, en)
        np.testing.assert_array_equal(dn, ed)
        np.testing.assert_array_equal(dp, ep)
    # all codes equal (the first round: no bits yet): the next pair's positive
    z = np.zeros((5, 1), dtype=np.uint64)
    neg, dn, _ = ref.hnm_codes(z, z)
    np.testing.assert_array_equal(neg, [1, 2, 3, 4, 0])
    assert (dn == 0).all()


def select_by_brute_force(pool, samples, cands, tau):
    """Alg. 1 written out with numpy: exact bins, HNM by distance matrices and the
    loss of Eq. 2 at all 5110 thresholds."""
    K, N = samples.shape
    P2 = len(pool)
    bits = np.zeros((P2, K), dtype=np.int64)  # 1 where the stump is +1
    out = []
    for k in range(K):
        sm = samples[k]
        def codes_of(rows):
            b = np.zeros((len(rows), 64), dtype=np.uint8)
            b[:, :k] = bits[rows][:, :k]
            return np.packbits(b, axis=1, bitorder="little").view(np.uint64)
        a, p = codes_of(2 * sm), codes_of(2 * sm + 1)
        neg, dn, dp = hnm_by_matrix(a, p)
        trip = []
        for s in range(N):
            if neg[s] >= 0:
                trip += [2 * sm[s], 2 * sm[s] + 1, 2 * sm[neg[s]] + 1]
            else:
                trip += [2 * sm[s] + 1, 2 * sm[s], 2 * sm[-1 - neg[s]]]
        s_ap = k - 2 * dp
        s_an = k - 2 * dn
        bb, bl = brute_force(pool[trip], s_ap, s_an, tau, cands[k])
        c = int(np.argmin(bl))
        out.append((c, int(bb[c]), float(bl[c])))
        for x in range(P2):
            bits[x, k] = int(bin_exact(pool[x], cands[k][c]) <= bb[c])
    return out, bits


def test_greedy_selection_by_brute_force(ref):
    rng = np.random.default_rng(91)
    P, N, J, K = 14, 9, 5, 4
    b = synth.triplets(synth.SEED_BASE + 91, n=P)
    pool = np.empty((2 * P, 32, 32), dtype=np.uint8)
    pool[0::2] = np.clip(np.rint(b.anchor * 255), 0, 255)
    pool[1::2] = np.clip(np.rint(b.positive * 255), 0, 255)
    samples = np.stack([rng.permutation(P)[:N] for _ in range(K)]).astype(np.int32)
    cands = np.stack([synth.box_pairs(rng, J, radius_range=(0, 5)) for _ in range(K)])
    table, chosen, cbin, loss, codes = ref.select_features(pool, samples, cands, 1.0)
    exp, bits = select_by_brute_force(pool, samples, cands, 1.0)
    assert [(int(c), int(q), float(l)) for c, q, l in zip(chosen, cbin, loss)] == exp
    got_bits = np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little")[:, :K]
    np.testing.assert_array_equal(got_bits, bits)
    # the table's thresholds reproduce the stumps with the BAD convention f <= theta
    for k in range(K):
        c = table[k]
        for x in range(2 * P):
            s1, a = box_sum(pool[x], c["x1"], c["y1"], c["radius"])
            s2, _ = box_sum(pool[x], c["x2"], c["y2"], c["radius"])
            assert (Fraction(s1 - s2, a) <= Fraction(float(c["threshold"]))) == bool(bits[x, k])
